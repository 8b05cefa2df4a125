"""Host-side accounting of bench.py (no GPU)."""
import bench


def test_paper_flop_count_matches_its_sustained_rate():
    # Eq. 9 at N = 50 over the paper's 128-bit run time of 73,773 s gives
    # 2.73 PFLOP/s, within 2% of the sustained 2.78 PFLOP/s it reports at N = 45
    rate = bench.paper_eq9_flops(50) / 73773.0 / 1e15
    assert abs(rate - 2.73) < 0.01
    assert abs(rate / 2.78 - 1) < 0.02


def test_paper_flop_count_small_cases():
    # one mode: one 2x2 solve, 4/3*8 + 4 - 8/3 = 12 flops (Eq. 8 at matrix size 2)
    assert abs(bench.paper_eq9_flops(1) - 12.0) < 1e-12
    # two modes: two 2x2 solves and one 4x4 solve
    assert abs(bench.paper_eq9_flops(2) - (2 * 12.0 + (4 / 3 * 64 + 16 - 16 / 3))) < 1e-9


def test_kernel_code_hash_ignores_comments_and_blank_lines():
    names = bench.KERNEL_SOURCES

    def texts(body):
        return {k: (body if k == names[0] else "") for k in names}

    a = "int x;  // note\n\n  y = 1;\n"
    b = "int x;\n  y = 1;   // other\n"
    assert bench.kernel_code_hash(texts(a)) == bench.kernel_code_hash(texts(b))
    assert bench.kernel_code_hash(texts(a)) != bench.kernel_code_hash(texts("int x;\n  y = 2;\n"))
