// tor_schur.hip -- right-looking Schur-complement subset-tree kernels in the
// real quadrature basis, for gfx950.
//
// Real form.  In the (a, a^dagger) basis I - O = [[X, Y], [conj(Y), conj(X)]]
// with X Hermitian and Y symmetric (the block symmetries of Eq. 3).  The
// per-mode unitary that maps each mode's pair (a, a^dagger) to its
// quadratures (q, p) turns it into the real symmetric matrix
//     R = [[Re(X+Y), -Im(X-Y)], [Im(X+Y), Re(X-Y)]],
// and because that unitary is block-diagonal over modes, every principal
// minor keeps its value: det(I - O_Z) = det(R_Z).  All arithmetic below is
// real, a quarter of the complex work.
//
// Right-looking recursion.  Decide the modes in order 0..n-1.  The state
// after deciding modes 0..k-1 (chosen subset Z) is the Schur complement of
// the undecided modes {k..n-1}:  T = R[U,U] - R[U,Z] R_Z^{-1} R[Z,U], plus
// g = det(R_Z)^(-1/2).  Leaving mode k out keeps T without its first 2x2
// block row/column; taking it in is a rank-2 update
//     P = T[k,k] = L L^T,  u = T[U',k] L^{-T},  T' = T[U',U'] - u u^T,
//     det(R_{Z+k}) = det(R_Z) det(P),
// (the quotient property of Schur complements).  So each subset costs, in
// amortised terms, about twelve rank-2 updates of the small trailing
// matrices, in place of the paper's per-subset elimination (Alg. 1, Sec.
// 4.2) or even the bordered update of the factor.  g of a child is g times
// det(P)^(-1/2).
//
// Three levels, one per memory:
//   top    (HBM)  breadth-first expansion, one launch per decided mode, of
//                 every state down to depth n - s_m; each state stores its
//                 packed s_m-mode matrix, g and |Z|.
//   middle (LDS)  one wavefront per depth-(n - s_m) state expands the next
//                 s_m - s_b <= 6 modes breadth-first, the updates of a whole
//                 level spread over the lanes as 2x2 mode blocks; the last of
//                 these expansions gives each lane one state at depth n - s_b.
//   bottom (VGPR) each lane finishes its own state: all 2^s_b subsets of the
//                 last s_b modes, fully unrolled at compile time with the
//                 matrices in registers.
// Two wavefronts share a workgroup's LDS and take turns: while one expands a
// state's middle levels, the other runs the register-only bottom of the
// state it expanded before.  Every wavefront writes one partial (signed sum,
// sum of magnitudes) per middle state; the reductions run in a fixed order,
// so results do not depend on scheduling or on the grid.
#include <hip/hip_runtime.h>

#include "tiers.hpp"
#include "tor_internal.hpp"

namespace tor {

// Packed lower triangle, row-major: entry (a, b), a >= b.
__host__ __device__ constexpr int pk(int a, int b) { return a * (a + 1) / 2 + b; }
// Entries of the packed 2s x 2s symmetric matrix of s modes.
__host__ __device__ constexpr int psize(int s) { return s * (2 * s + 1); }
// Distance between consecutive states (or pivot columns) in LDS: rounded up
// to an odd number of values, so that lanes reading the same entry of
// different states hit different banks.
__host__ __device__ constexpr int odd_up(int v) { return v | 1; }

// Per-phase clocks of the middle + bottom kernel (a build with
// TOR_PHASE_CLOCKS defined; otherwise PhaseClock is empty and every mark
// compiles to nothing).  Each wavefront adds the shader-clock cycles between
// consecutive marks to the phase the interval belongs to, and at its end
// adds its totals into tor_phase_clk, one atomic per phase.
enum LeafPhase : int {
  PH_EXPAND = 0,  // store, prefetch and the middle levels in LDS
  PH_LAST = 1,    // each lane's own last middle level, in registers
  PH_WAIT_A = 2,  // the barrier after the expansion
  PH_BOTTOM = 3,  // the bottom level, in registers
  PH_TOTALS = 4,  // the wave's fixed-order totals and the partial's store
  PH_WAIT_B = 5,  // the barrier after the bottom
  PH_OTHER = 6,   // set-up and the tail
  PH_COUNT = 7
};
#ifdef TOR_PHASE_CLOCKS
__device__ unsigned long long tor_phase_clk[PH_COUNT];
struct PhaseClock {
  unsigned long long acc[PH_COUNT];
  unsigned long long t;
  __device__ PhaseClock() : t(clock64()) {
    for (int k = 0; k < PH_COUNT; ++k) acc[k] = 0;
  }
  __device__ __forceinline__ void mark(int k) {
    const unsigned long long u = clock64();
    acc[k] += u - t;
    t = u;
  }
  __device__ void flush(int lane) {
    if (lane == 0)
      for (int k = 0; k < PH_COUNT; ++k) atomicAdd(&tor_phase_clk[k], acc[k]);
  }
};
#else
struct PhaseClock {
  __device__ __forceinline__ void mark(int) {}
  __device__ __forceinline__ void flush(int) {}
};
#endif

// --------------------------------------------------------------------------
// Real-tier arithmetic helpers
// --------------------------------------------------------------------------

template <class R>
__device__ __forceinline__ R r_from_sum(double a, double b, double c);
// a + b + c with the tier's precision (exact in QD)
template <>
__device__ __forceinline__ double r_from_sum<double>(double a, double b, double c) { return (a + b) + c; }
template <>
__device__ __forceinline__ dd r_from_sum<dd>(double a, double b, double c) {
  dd s;
  prec::two_sum(a, b, s.hi, s.lo);
  return prec::dd_add_d(s, c);
}
template <>
__device__ __forceinline__ qd r_from_sum<qd>(double a, double b, double c) {
  double s, e;
  prec::two_sum(a, b, s, e);
  return prec::qd_add_d(qd{{s, e, 0.0, 0.0}}, c);
}

// Accumulators of one lane, by the parity of the term's subset size
// relative to the lane's state (p[0]: even, p[1]: odd).  Every term g =
// det^(-1/2) is positive, so one run per parity gives both the signed sum
// (the difference of the two, its sign set by (-1)^(n-|Z|)) and the sum of
// magnitudes (their sum) with one accumulation per term.  NL > 0 (the
// level-sum debug mode) adds one run per relative subset size 0..NL-1.
template <class TT, int NL = 0>
struct LaneAcc {
  typename TT::Acc p[2];
  typename TT::Acc lv[NL > 0 ? NL : 1];
};

// Emit the term g of a completed subset whose size exceeds the lane state's
// by D.
template <class TT, int D, int NL>
__device__ __forceinline__ void emit_term(LaneAcc<TT, NL>& acc, const typename TT::R& g) {
  acc.p[D & 1] = TT::acc_run(acc.p[D & 1], g);
  if constexpr (NL > 0) acc.lv[D] = TT::acc_run(acc.lv[D], g);
}

// Pivot of the 2x2 block at rows (2i, 2i+1): reciprocal square roots of the
// two Cholesky pivots and the sub-diagonal factor entry.
template <class R>
struct Pivot {
  R rl0, l10, rl1;
  bool ok;
};

template <class R>
__device__ __forceinline__ Pivot<R> make_pivot(const R& p00, const R& p10, const R& p11) {
  Pivot<R> p;
  p.ok = r_lead(p00) > 0.0;
  p.rl0 = r_rsqrt(p00);
  p.l10 = r_mul(p10, p.rl0);
  const R d2 = r_fms(p11, p.l10, p.l10);
  p.ok = p.ok && (r_lead(d2) > 0.0);
  p.rl1 = r_rsqrt(d2);
  return p;
}

// det of the 2x2 pivot block, p00 p11 - p10^2 (one rounding in F64; the
// fused form in DD).  Its relative error is of the order of the block's
// condition times u, the same as that of the Cholesky pivot p11 - l10^2.
__device__ __forceinline__ double r_det2(double p00, double p10, double p11) {
  return fma(p00, p11, -(p10 * p10));
}
__device__ __forceinline__ dd r_det2(const dd& p00, const dd& p10, const dd& p11) {
  return prec::dd_fms2(dd{0.0, 0.0}, prec::dd_neg(p00), p11, p10, p10);
}
__device__ __forceinline__ qd r_det2(const qd& p00, const qd& p10, const qd& p11) {
  return r_fms(r_mul(p00, p11), p10, p10);
}

// The same pivot from det(P) = p00 p11 - p10^2: rl1 = p00 rl0 rd with
// rd = det(P)^(-1/2), so the two reciprocal square roots are independent;
// the child's g is g rd.
template <class R>
__device__ __forceinline__ Pivot<R> make_pivot_det(const R& p00, const R& p10, const R& p11, R& rd) {
  Pivot<R> p;
  const R det = r_det2(p00, p10, p11);
  p.ok = r_lead(p00) > 0.0 && r_lead(det) > 0.0;
  p.rl0 = r_rsqrt(p00);
  rd = r_rsqrt(det);
  p.l10 = r_mul(p10, p.rl0);
  p.rl1 = r_mul(r_mul(p00, p.rl0), rd);
  return p;
}

// --------------------------------------------------------------------------
// Bottom level: one lane, all subsets of S modes, registers only.
// T is the packed 2S x 2S matrix of the lane's state, g its det^(-1/2),
// m its subset size.  Children are taken largest index first so the parent
// matrix dies before the largest child (index 0) is formed.
// --------------------------------------------------------------------------

template <class TT, int S>
struct Bottom {
  using R = typename TT::R;

  // PAR: parity of the state's subset size relative to the lane's state
  template <int I, int D, int NL>
  __device__ __forceinline__ static void child(const R (&T)[psize(S)], const R& g, LaneAcc<TT, NL>& acc,
                                               bool& bad) {
    constexpr int SC = S - 1 - I;
    constexpr int O = 2 * I + 2;
    if constexpr (SC == 0) {
      // the last mode: only the term is needed, g det(P)^(-1/2)
      const R& p00 = T[pk(2 * I, 2 * I)];
      const R det = r_det2(p00, T[pk(2 * I + 1, 2 * I)], T[pk(2 * I + 1, 2 * I + 1)]);
      if (!(r_lead(p00) > 0.0 && r_lead(det) > 0.0)) bad = true;
      emit_term<TT, D + 1>(acc, r_mul(g, r_rsqrt(det)));
    } else {
      const Pivot<R> pv = make_pivot(T[pk(2 * I, 2 * I)], T[pk(2 * I + 1, 2 * I)], T[pk(2 * I + 1, 2 * I + 1)]);
      if (!pv.ok) bad = true;
      const R gc = r_mul(r_mul(g, pv.rl0), pv.rl1);
      R u0[2 * SC], u1[2 * SC];
#pragma unroll
      for (int a = 0; a < 2 * SC; ++a) {
        u0[a] = r_mul(T[pk(a + O, 2 * I)], pv.rl0);
        u1[a] = r_mul(r_fms(T[pk(a + O, 2 * I + 1)], u0[a], pv.l10), pv.rl1);
      }
      R C[psize(SC)];
#pragma unroll
      for (int a = 0; a < 2 * SC; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          C[pk(a, b)] = r_fms2(T[pk(a + O, b + O)], u0[a], u0[b], u1[a], u1[b]);
        }
      }
      Bottom<TT, SC>::template run<D + 1>(C, gc, acc, bad);
    }
  }

  template <int I, int D, int NL>
  __device__ __forceinline__ static void children(const R (&T)[psize(S)], const R& g, LaneAcc<TT, NL>& acc,
                                                  bool& bad) {
    child<I, D>(T, g, acc, bad);
    if constexpr (I > 0) children<I - 1, D>(T, g, acc, bad);
  }

  // D: the state's subset size over the lane state's
  template <int D, int NL>
  __device__ __forceinline__ static void run(const R (&T)[psize(S)], const R& g, LaneAcc<TT, NL>& acc, bool& bad) {
    emit_term<TT, D>(acc, g);
    children<S - 1, D>(T, g, acc, bad);
  }
};

// --------------------------------------------------------------------------
// Root staging: the real matrix R of all n modes (packed), g = 1, |Z| = 0.
// Row 2k is mode k's q quadrature, row 2k+1 its p quadrature.
// --------------------------------------------------------------------------

template <class TT>
__global__ void real_root_kernel(const double2* __restrict__ O, const int64_t* __restrict__ offs,
                                 int n, int64_t ld, typename TT::R* __restrict__ mat,
                                 typename TT::R* __restrict__ g, int32_t* __restrict__ msz) {
  using R = typename TT::R;
  const int inst = blockIdx.y;  // instance within the group
  const double2* Oi = O + (offs ? offs[inst] : 0);
  R* out = mat + (size_t)inst * psize(n);
  const int total = psize(n);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    // e -> (r, c), r >= c
    int r = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (pk(r + 1, 0) <= e) ++r;
    while (pk(r, 0) > e) --r;
    const int c = e - pk(r, 0);
    const int i = r >> 1, j = c >> 1;  // modes
    const int qi = r & 1, qj = c & 1;  // 0: q, 1: p
    // O00_ij and O01_ij from the lower triangle of O (block order)
    double2 x;  // O00_ij
    if (i >= j) {
      x = Oi[(int64_t)i * ld + j];
    } else {
      const double2 w = Oi[(int64_t)j * ld + i];
      x = make_double2(w.x, -w.y);
    }
    const double2 w1 = Oi[(int64_t)(j + n) * ld + i];  // O10_ji = conj(O01_ij)
    const double2 y = make_double2(w1.x, -w1.y);       // O01_ij
    const double dlt = (i == j && qi == qj) ? 1.0 : 0.0;
    R v;
    if (qi == 0 && qj == 0) v = r_from_sum<R>(dlt, -x.x, -y.x);       // delta - Re(O00 + O01)
    else if (qi == 0 && qj == 1) v = r_from_sum<R>(0.0, x.y, -y.y);   // Im(O00 - O01)
    else if (qi == 1 && qj == 0) v = r_from_sum<R>(0.0, -x.y, -y.y);  // -Im(O00 + O01)
    else v = r_from_sum<R>(dlt, -x.x, y.x);                           // delta - Re(O00 - O01)
    out[e] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g[inst] = r_of<R>(1.0);
    msz[inst] = 0;
  }
}

// --------------------------------------------------------------------------
// Top level: expand every state of a frontier by one mode.
// in: nst states of s modes; out: 2*nst states of s-1 modes,
// child 2z leaves the mode out, child 2z+1 takes it in.
// G states per 256-thread workgroup, 256/G threads each: every thread forms
// its state's pivot itself (the same operations, so the same values), the
// pivot column goes through LDS, and one barrier separates it from the
// entry updates.  Many small states (the deep levels) take G = 4; the few
// large ones near the root take G = 1.
// --------------------------------------------------------------------------

template <class TT, int G>
__global__ __launch_bounds__(256) void expand_kernel(const typename TT::R* __restrict__ in_mat,
                                                     const typename TT::R* __restrict__ in_g,
                                                     const int32_t* __restrict__ in_m, int s, int nst,
                                                     typename TT::R* __restrict__ out_mat,
                                                     typename TT::R* __restrict__ out_g,
                                                     int32_t* __restrict__ out_m,
                                                     int32_t* __restrict__ status) {
  using R = typename TT::R;
  constexpr int TPS = 256 / G;  // threads per state
  __shared__ R su0[G][128], su1[G][128];
  const int grp = (int)threadIdx.x / TPS, t = (int)threadIdx.x % TPS;
  const int z = (int)blockIdx.x * G + grp;
  const bool live = z < nst;
  const int zc = live ? z : nst - 1;  // a group past the end works on the last state, stores nothing
  const R* T = in_mat + (size_t)zc * psize(s);
  const int sc = s - 1;
  const int nr = 2 * sc;  // rows of a child
  const Pivot<R> pv = make_pivot(T[pk(0, 0)], T[pk(1, 0)], T[pk(1, 1)]);
  if (live && t == 0) {
    if (!pv.ok) atomicOr(status, 1);
    const R g = in_g[z];
    out_g[2 * z] = g;
    out_m[2 * z] = in_m[z];
    out_g[2 * z + 1] = r_mul(r_mul(g, pv.rl0), pv.rl1);
    out_m[2 * z + 1] = in_m[z] + 1;
  }
  for (int a = t; a < nr; a += TPS) {
    const R u0 = r_mul(T[pk(a + 2, 0)], pv.rl0);
    su0[grp][a] = u0;
    su1[grp][a] = r_mul(r_fms(T[pk(a + 2, 1)], u0, pv.l10), pv.rl1);
  }
  __syncthreads();
  if (!live) return;
  R* ex = out_mat + (size_t)(2 * z) * psize(sc);
  R* in = out_mat + (size_t)(2 * z + 1) * psize(sc);
  const int ne = psize(sc);
  for (int e = t; e < ne; e += TPS) {
    int a = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (pk(a + 1, 0) <= e) ++a;
    while (pk(a, 0) > e) --a;
    const int b = e - pk(a, 0);
    const R tv = T[pk(a + 2, b + 2)];
    ex[e] = tv;
    in[e] = r_fms2(tv, su0[grp][a], su0[grp][b], su1[grp][a], su1[grp][b]);
  }
}

// Several top levels in one launch: one workgroup takes a state of s modes
// K levels down, the levels in between in LDS, and writes its 2^K
// descendants (descendant w = the decisions c1 .. cK as bits, c1 the most
// significant, as K single-level expansions would number them).  The
// operations and their operands are those of expand_kernel, so the
// descendants are bit-for-bit the same; only the intermediate states stay
// out of HBM.  LDS (dynamic, expand_multi_lds_bytes): with `stage`, first
// a copy of the input state (read from HBM once, coalesced, instead of by
// the scattered reads of level 0); then the states of levels 1 .. K-1, the
// pivot column of the widest level, pivots, g and |Z|.
__host__ __device__ inline size_t expand_multi_vals(int s, int K) {
  size_t v = 0;
  for (int j = 1; j < K; ++j) v += ((size_t)1 << j) * psize(s - j);
  size_t u = 0;
  for (int j = 0; j < K; ++j) {
    const size_t w = ((size_t)1 << j) * 2 * (s - j - 1);
    u = u > w ? u : w;
  }
  return v + 2 * u + 3 * ((size_t)1 << (K - 1)) + 2 * ((size_t)1 << K);
}

template <class TT>
__global__ __launch_bounds__(256) void expand_multi_kernel(const typename TT::R* __restrict__ in_mat,
                                                           const typename TT::R* __restrict__ in_g,
                                                           const int32_t* __restrict__ in_m, int s, int K,
                                                           typename TT::R* __restrict__ out_mat,
                                                           typename TT::R* __restrict__ out_g,
                                                           int32_t* __restrict__ out_m,
                                                           int32_t* __restrict__ status, int stage) {
  using R = typename TT::R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int z = blockIdx.x;
  const int tid = (int)threadIdx.x;
  // carve: [input state], level states (1 .. K-1), u0 | u1, pivots, g; then
  // |Z| as int32
  const R* T0 = in_mat + (size_t)z * psize(s);
  size_t off = 0;
  if (stage) {
    for (int e = tid; e < psize(s); e += 256) lds[e] = T0[e];
    T0 = lds;
    off = psize(s);
    __syncthreads();
  }
  R* lvl[3] = {nullptr, nullptr, nullptr};
  for (int j = 1; j < K; ++j) {
    lvl[j] = lds + off;
    off += ((size_t)1 << j) * psize(s - j);
  }
  size_t umax = 0;
  for (int j = 0; j < K; ++j) {
    const size_t w = ((size_t)1 << j) * 2 * (s - j - 1);
    umax = umax > w ? umax : w;
  }
  R* su0 = lds + off;
  R* su1 = su0 + umax;
  R* spv = su1 + umax;                  // 3 per state of the widest level
  R* sg = spv + 3 * (1 << (K - 1));     // g of two consecutive levels, 2^K entries each
  int32_t* sm = reinterpret_cast<int32_t*>(sg + 2 * (1 << K));  // |Z|, likewise
  for (int j = 0; j < K; ++j) {
    const int sj = s - j;                // modes of the states of level j
    const int nsj = 1 << j;
    const int nr = 2 * (sj - 1);
    const int ne = psize(sj - 1);
    const bool last = (j == K - 1);
    const R* src = j == 0 ? T0 : lvl[j];
    const int ps = psize(sj);
    // pivots and the children's g and |Z|
    if (tid < nsj) {
      const R* T = src + (size_t)tid * ps;
      const Pivot<R> pv = make_pivot(T[pk(0, 0)], T[pk(1, 0)], T[pk(1, 1)]);
      if (!pv.ok) atomicOr(status, 1);
      spv[3 * tid] = pv.rl0;
      spv[3 * tid + 1] = pv.l10;
      spv[3 * tid + 2] = pv.rl1;
      const int cur = (j & 1) << K, nxt = ((j + 1) & 1) << K;
      const R g = j == 0 ? in_g[z] : sg[cur + tid];
      const int32_t m = j == 0 ? in_m[z] : sm[cur + tid];
      const R gi = r_mul(r_mul(g, pv.rl0), pv.rl1);
      if (last) {
        const size_t w = ((size_t)z << K) + 2 * tid;
        out_g[w] = g;
        out_m[w] = m;
        out_g[w + 1] = gi;
        out_m[w + 1] = m + 1;
      } else {
        sg[nxt + 2 * tid] = g;
        sm[nxt + 2 * tid] = m;
        sg[nxt + 2 * tid + 1] = gi;
        sm[nxt + 2 * tid + 1] = m + 1;
      }
    }
    __syncthreads();
    // pivot columns
    for (int idx = tid; idx < nsj * nr; idx += 256) {
      const int st = idx / nr, a = idx - st * nr;
      const R* T = src + (size_t)st * ps;
      const R u0 = r_mul(T[pk(a + 2, 0)], spv[3 * st]);
      su0[idx] = u0;
      su1[idx] = r_mul(r_fms(T[pk(a + 2, 1)], u0, spv[3 * st + 1]), spv[3 * st + 2]);
    }
    __syncthreads();
    // entries of both children of every state
    R* dst = last ? out_mat + ((size_t)z << K) * ne : lvl[j + 1];
    for (int idx = tid; idx < nsj * ne; idx += 256) {
      const int st = idx / ne, e = idx - st * ne;
      int a = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while (pk(a + 1, 0) <= e) ++a;
      while (pk(a, 0) > e) --a;
      const int b = e - pk(a, 0);
      const R* T = src + (size_t)st * ps;
      const R* u0 = su0 + st * nr;
      const R* u1 = su1 + st * nr;
      const R tv = T[pk(a + 2, b + 2)];
      dst[(size_t)(2 * st) * ne + e] = tv;
      dst[(size_t)(2 * st + 1) * ne + e] = r_fms2(tv, u0[a], u0[b], u1[a], u1[b]);
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// Middle + bottom: one wavefront per middle state of s_m undecided modes.
//
// The middle level expands the state breadth-first in LDS: level j holds
// 2^j states of s_m - j modes (child 2z leaves the next mode out, 2z+1 takes
// it in), so every barrier-separated phase has up to hundreds of
// independent entry updates for the 64 lanes.  The last expansion is done by
// each lane for its own state, straight into registers, and the bottom level
// follows.  L = s_m - s_b <= 6 middle levels give up to 64 bottom states.
// --------------------------------------------------------------------------

// Work item idx of a phase with d items per state -> state idx / d, by a
// multiply and shift: q = (idx * ceil(2^20 / d)) >> 20 is exact while
// idx * d < 2^20 (the rounding excess of the multiplier is below d).
struct DivBy {
  uint32_t m;
  int d;
  __device__ explicit DivBy(int d_) : m(((1u << 20) + (uint32_t)d_ - 1u) / (uint32_t)d_), d(d_) {}
  __device__ int q(int idx) const { return (int)(((uint32_t)idx * m) >> 20); }
};

// One pass of a middle-level expansion over KK * 64 work items starting at
// base: item (state z, child mode block (bi, bj)) computes rows 2bi, 2bi+1
// and columns 2bj, 2bj+1 of both children of z, every load issued before
// the math.  Items past tot repeat the last valid one and are not stored;
// the upper entry of a diagonal block is computed from its mirror and not
// stored.
template <class R, int KK>
__device__ __forceinline__ void entry_pass(int base, int lane, int tot, const DivBy& db,
                                           const uint16_t* blocks, const R* cur, int ps,
                                           const R* u, int urs, R* nxt, int pcs) {
  int zk[KK], rk[KK], ck[KK];
  bool dg[KK];
  R t00[KK], t01[KK], t10[KK], t11[KK], ua[KK][4], ub[KK][4];
#pragma unroll
  for (int k = 0; k < KK; ++k) {
    const int i = min(base + lane + 64 * k, tot - 1);
    zk[k] = db.q(i);
    const uint32_t bp = blocks[i - zk[k] * db.d];
    rk[k] = 2 * (int)(bp & 255u);
    ck[k] = 2 * (int)(bp >> 8);
    dg[k] = rk[k] == ck[k];
  }
#pragma unroll
  for (int k = 0; k < KK; ++k) {
    const R* T = cur + zk[k] * ps;
    const int p0 = pk(rk[k] + 2, ck[k] + 2), p1 = pk(rk[k] + 3, ck[k] + 2);
    t00[k] = T[p0];
    t01[k] = T[dg[k] ? p1 : p0 + 1];
    t10[k] = T[p1];
    t11[k] = T[p1 + 1];
    const R* U = u + zk[k] * urs;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ua[k][v] = U[2 * rk[k] + v];
      ub[k][v] = U[2 * ck[k] + v];
    }
  }
#pragma unroll
  for (int k = 0; k < KK; ++k) {
    const R c00 = r_fms2(t00[k], ua[k][0], ub[k][0], ua[k][1], ub[k][1]);
    const R c01 = r_fms2(t01[k], ua[k][0], ub[k][2], ua[k][1], ub[k][3]);
    const R c10 = r_fms2(t10[k], ua[k][2], ub[k][0], ua[k][3], ub[k][1]);
    const R c11 = r_fms2(t11[k], ua[k][2], ub[k][2], ua[k][3], ub[k][3]);
    if (base + lane + 64 * k < tot) {
      R* X = nxt + (2 * zk[k]) * pcs;  // leaves the mode out
      R* Y = X + pcs;                   // takes it in
      const int q0 = pk(rk[k], ck[k]), q1 = pk(rk[k] + 1, ck[k]);
      X[q0] = t00[k];
      Y[q0] = c00;
      X[q1] = t10[k];
      Y[q1] = c10;
      X[q1 + 1] = t11[k];
      Y[q1 + 1] = c11;
      if (!dg[k]) {
        X[q0 + 1] = t01[k];
        Y[q0 + 1] = c01;
      }
    }
  }
}

template <class TT, int SB>
struct MidSmem {
  using R = typename TT::R;
  static constexpr int L = 6;
  static constexpr int SM = SB + L;
  // level j (s = SM - j modes, 2^j states): even levels in A, odd in B
  static constexpr int level_vals(int j) { return (1 << j) * odd_up(psize(SM - j)); }
  static constexpr int a_vals() {
    int v = 0;
    for (int j = 0; j < L; j += 2) v = v > level_vals(j) ? v : level_vals(j);
    return v;
  }
  static constexpr int b_vals() {
    int v = 0;
    for (int j = 1; j < L; j += 2) v = v > level_vals(j) ? v : level_vals(j);
    return v;
  }
  // pivot columns of the LDS expansions (levels 0 .. L-2): per state, the
  // pair (u0, u1) of every row below the pivot block
  static constexpr int u_vals() {
    int v = 0;
    for (int j = 0; j + 1 < L; ++j) {
      const int w = (1 << j) * odd_up(4 * (SM - j - 1));
      v = v > w ? v : w;
    }
    return v;
  }
  // largest work-item count of an LDS phase (entries of all include
  // children of a level, or their pivot columns)
  static constexpr int max_items() {
    int v = 0;
    for (int j = 0; j + 1 < L; ++j) {
      const int w = (1 << j) * psize(SM - j - 1);
      v = v > w ? v : w;
    }
    return v;
  }
  R A[a_vals()];
  R B[b_vals()];
  R gA[32], gB[32];
  R u[u_vals()];
  int32_t mA[32], mB[32];
  // mode block index q of a child -> (i, j), i >= j, as i | j << 8
  uint16_t blocks[(SM - 1) * SM / 2];
};

// Orders one wavefront's LDS accesses across its lanes: the compiler keeps
// memory accesses on their side, and the wave waits for its outstanding LDS
// operations.  (A wavefront's LDS operations complete in issue order.)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The pieces of the middle + bottom kernel, for one wavefront.
template <class TT, int SB>
struct Leaf {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  using SMEM = MidSmem<TT, SB>;
  static constexpr int NP = psize(SB + 1);
  // The next state's matrix is fetched into registers while the current one
  // is expanded: lane k holds entries k, k + 64, ... (indexes past the
  // matrix are clamped to its last entry and not stored).
  static constexpr int PF = (psize(SMEM::SM) + 63) / 64;
  static_assert(PF <= 6, "prefetch holds at most six entries per lane");

  __device__ __forceinline__ static void fetch(const R* mat, const R* gin, const int32_t* min_, int z,
                                               int ps0, int lane, R& v0, R& v1, R& v2, R& v3, R& v4, R& v5, R& g,
                                               int32_t& m) {
    const R* src = mat + (size_t)z * ps0;
    v0 = src[min(lane, ps0 - 1)];
    if constexpr (PF > 1) v1 = src[min(lane + 64, ps0 - 1)];
    if constexpr (PF > 2) v2 = src[min(lane + 128, ps0 - 1)];
    if constexpr (PF > 3) v3 = src[min(lane + 192, ps0 - 1)];
    if constexpr (PF > 4) v4 = src[min(lane + 256, ps0 - 1)];
    if constexpr (PF > 5) v5 = src[min(lane + 320, ps0 - 1)];
    g = gin[z];
    m = min_[z];
  }

  __device__ __forceinline__ static void store(SMEM& sm, int ps0, int lane, const R& v0, const R& v1,
                                               const R& v2, const R& v3, const R& v4, const R& v5, const R& g,
                                               int32_t m) {
    if (lane < ps0) sm.A[lane] = v0;
    if constexpr (PF > 1) if (lane + 64 < ps0) sm.A[lane + 64] = v1;
    if constexpr (PF > 2) if (lane + 128 < ps0) sm.A[lane + 128] = v2;
    if constexpr (PF > 3) if (lane + 192 < ps0) sm.A[lane + 192] = v3;
    if constexpr (PF > 4) if (lane + 256 < ps0) sm.A[lane + 256] = v4;
    if constexpr (PF > 5) if (lane + 320 < ps0) sm.A[lane + 320] = v5;
    if (lane == 0) {
      sm.gA[0] = g;
      sm.mA[0] = m;
    }
  }

  // Levels 0 .. L-2 of the state in sm.A, breadth-first in LDS; on return
  // cur, cg, cm hold level L-1.
  __device__ __forceinline__ static void middle(SMEM& sm, int s_m, int L, int lane, bool& bad, R*& cur,
                                                R*& cg, int32_t*& cm) {
    cur = sm.A;
    R* nxt = sm.B;
    cg = sm.gA;
    R* ng = sm.gB;
    cm = sm.mA;
    int32_t* nm = sm.mB;
    for (int j = 0; j + 1 < L; ++j) {
      const int S = s_m - j;  // modes of level j
      const int ns = 1 << j;
      const int ps = odd_up(psize(S));      // state stride of level j
      const int pcs = odd_up(psize(S - 1)); // state stride of level j + 1
      const int urs = odd_up(4 * (S - 1));  // pivot-column stride
      {
        // pivot columns, one mode (two rows) per item; every item forms its
        // state's pivot itself (in the determinant form, whose chain of
        // dependent operations is about half that of rsqrt(p00) -> l10 ->
        // p11 - l10^2 -> rsqrt), and the first item of a state also the
        // children's g and |Z|
        const int nmo = S - 1;
        const DivBy dm(nmo);
        if (ns * nmo > 64) {
          // more than one pass's worth: two items per lane per pass, their
          // pivot chains side by side (an item past the end repeats the last
          // one and is not stored)
          const int totu = ns * nmo;
          for (int i0 = lane; i0 < totu; i0 += 128) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const int idx = min(i0 + 64 * k, totu - 1);
              const int zz = dm.q(idx), i = idx - zz * nmo;
              const R* T = cur + zz * ps;
              const int r = 2 * i + 2;
              const R a0 = T[pk(r, 0)], a1 = T[pk(r, 1)];
              const R b0 = T[pk(r + 1, 0)], b1 = T[pk(r + 1, 1)];
              R rd;
              const Pivot<R> pv = make_pivot_det(T[pk(0, 0)], T[pk(1, 0)], T[pk(1, 1)], rd);
              if (!pv.ok) bad = true;
              const R u0a = r_mul(a0, pv.rl0), u0b = r_mul(b0, pv.rl0);
              const R u1a = r_mul(r_fms(a1, u0a, pv.l10), pv.rl1);
              const R u1b = r_mul(r_fms(b1, u0b, pv.l10), pv.rl1);
              if (i0 + 64 * k < totu) {
                R* U = sm.u + zz * urs + 4 * i;
                U[0] = u0a;
                U[1] = u1a;
                U[2] = u0b;
                U[3] = u1b;
                if (i == 0) {
                  ng[2 * zz] = cg[zz];
                  nm[2 * zz] = cm[zz];
                  ng[2 * zz + 1] = r_mul(cg[zz], rd);
                  nm[2 * zz + 1] = cm[zz] + 1;
                }
              }
            }
          }
        } else {
          for (int idx = lane; idx < ns * nmo; idx += 64) {
            const int zz = dm.q(idx), i = idx - zz * nmo;
            const R* T = cur + zz * ps;
            const int r = 2 * i + 2;
            const R a0 = T[pk(r, 0)], a1 = T[pk(r, 1)];
            const R b0 = T[pk(r + 1, 0)], b1 = T[pk(r + 1, 1)];
            R rd;
            const Pivot<R> pv = make_pivot_det(T[pk(0, 0)], T[pk(1, 0)], T[pk(1, 1)], rd);
            if (!pv.ok) bad = true;
            const R u0a = r_mul(a0, pv.rl0), u0b = r_mul(b0, pv.rl0);
            R* U = sm.u + zz * urs + 4 * i;
            U[0] = u0a;
            U[1] = r_mul(r_fms(a1, u0a, pv.l10), pv.rl1);
            U[2] = u0b;
            U[3] = r_mul(r_fms(b1, u0b, pv.l10), pv.rl1);
            if (i == 0) {
              ng[2 * zz] = cg[zz];
              nm[2 * zz] = cm[zz];
              ng[2 * zz + 1] = r_mul(cg[zz], rd);
              nm[2 * zz + 1] = cm[zz] + 1;
            }
          }
        }
      }
      wave_sync();
      {
        // children, in passes of K * 64 mode blocks; the last, partial pass
        // uses only as many 64-item slices as it needs.  K items per lane
        // in flight: four in binary64, three in double- and quad-double (the
        // fastest measured at n = 30: against two, DD 2.5% and QD 6.6%
        // faster; four in QD, or in binary64 eight, are slower)
        constexpr int K = sizeof(R) == sizeof(double) ? 4 : 3;
        const int S1 = S - 1;
        const DivBy db(S1 * (S1 + 1) / 2);
        const int tot = ns * db.d;
        int base = 0;
        for (; base + 64 * K <= tot; base += 64 * K)
          entry_pass<R, K>(base, lane, tot, db, sm.blocks, cur, ps, sm.u, urs, nxt, pcs);
        for (; tot - base > 64; base += 128)
          entry_pass<R, 2>(base, lane, tot, db, sm.blocks, cur, ps, sm.u, urs, nxt, pcs);
        if (tot - base > 0) entry_pass<R, 1>(base, lane, tot, db, sm.blocks, cur, ps, sm.u, urs, nxt, pcs);
      }
      wave_sync();
      R* t0 = cur; cur = nxt; nxt = t0;
      R* t1 = cg; cg = ng; ng = t1;
      int32_t* t2 = cm; cm = nm; nm = t2;
    }
  }

  // Expand state z (its matrix prefetched in v0..v5, g, m) through the
  // middle levels; each lane then forms its own bottom state (leaf, lg,
  // lm) from its pair of the last middle level, in registers: both children
  // run the same code, the excluded one with zero pivot multipliers, whose
  // update leaves every entry unchanged (lane 0 takes the whole state when
  // L == 0; lanes without a state compute on state 0 and are not used).
  // Then fetch the wave's next state zn.
  __device__ __forceinline__ static void expand(SMEM& sm, const R* mat, const R* gin, const int32_t* min_,
                                                int zn, int nstates, int s_m, int L, int ps0, int lane,
                                                bool& bad, R& v0, R& v1, R& v2, R& v3, R& v4, R& v5, R& g, int32_t& m,
                                                R (&leaf)[psize(SB)], R& lg, int32_t& lm, PhaseClock& pc) {
    store(sm, ps0, lane, v0, v1, v2, v3, v4, v5, g, m);
    if (zn < nstates) fetch(mat, gin, min_, zn, ps0, lane, v0, v1, v2, v3, v4, v5, g, m);
    wave_sync();
    R* cur;
    R* cg;
    int32_t* cm;
    middle(sm, s_m, L, lane, bad, cur, cg, cm);
    pc.mark(PH_EXPAND);
    if (L == 0) {
#pragma unroll
      for (int e = 0; e < psize(SB); ++e) leaf[e] = cur[e];
      lg = cg[0];
      lm = cm[0];
      pc.mark(PH_LAST);
      return;
    }
    const int zz = lane < (1 << L) ? lane >> 1 : 0;
    last_level(cur + zz * odd_up(psize(SB + 1)), cg[zz], cm[zz], L, lane, bad, leaf, lg, lm);
    pc.mark(PH_LAST);
  }

  // The same, but the lane's pair state (all of it: lane 0 takes the whole
  // state when L == 0) is only copied into registers P, pg, pm; the last
  // level is then formed by last_level() outside the expansion.
  __device__ __forceinline__ static void expand_pair(SMEM& sm, const R* mat, const R* gin,
                                                     const int32_t* min_, int zn, int nstates, int s_m,
                                                     int L, int ps0, int lane, bool& bad, R& v0, R& v1,
                                                     R& v2, R& v3, R& v4, R& v5, R& g, int32_t& m, R (&P)[NP], R& pg,
                                                     int32_t& pm) {
    store(sm, ps0, lane, v0, v1, v2, v3, v4, v5, g, m);
    if (zn < nstates) fetch(mat, gin, min_, zn, ps0, lane, v0, v1, v2, v3, v4, v5, g, m);
    wave_sync();
    R* cur;
    R* cg;
    int32_t* cm;
    middle(sm, s_m, L, lane, bad, cur, cg, cm);
    const int zz = (L == 0 || lane >= (1 << L)) ? 0 : lane >> 1;
    const R* T = cur + zz * odd_up(psize(SB + 1));
#pragma unroll
    for (int e = 0; e < NP; ++e) P[e] = T[e];
    pg = cg[zz];
    pm = cm[zz];
  }

  // The lane's bottom state from its pair state T (registers or LDS) of the
  // last middle level: both children run the same code, the excluded one
  // with zero pivot multipliers, whose update leaves every entry unchanged.
  // With L == 0 the state is the bottom state itself.
  template <class Src>
  __device__ __forceinline__ static void last_level(const Src& T, const R& tg, int32_t tm, int L, int lane,
                                                    bool& bad, R (&leaf)[psize(SB)], R& lg, int32_t& lm) {
    if (L == 0) {
#pragma unroll
      for (int e = 0; e < psize(SB); ++e) leaf[e] = T[e];
      lg = tg;
      lm = tm;
      return;
    }
    const bool inc = (lane & 1) != 0;
    const Pivot<R> pv = make_pivot(T[pk(0, 0)], T[pk(1, 0)], T[pk(1, 1)]);
    if (inc && lane < (1 << L) && !pv.ok) bad = true;
    const R zero = r_zero<R>();
    const R m0 = inc ? pv.rl0 : zero;
    const R m1 = inc ? pv.rl1 : zero;
    R u0[2 * SB], u1[2 * SB];
#pragma unroll
    for (int a = 0; a < 2 * SB; ++a) {
      u0[a] = r_mul(T[pk(a + 2, 0)], m0);
      u1[a] = r_mul(r_fms(T[pk(a + 2, 1)], u0[a], pv.l10), m1);
    }
#pragma unroll
    for (int a = 0; a < 2 * SB; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) leaf[pk(a, b)] = r_fms2(T[pk(a + 2, b + 2)], u0[a], u0[b], u1[a], u1[b]);
    lg = inc ? r_mul(r_mul(tg, pv.rl0), pv.rl1) : tg;
    lm = tm + (inc ? 1 : 0);
  }

  // The bottom of the lane's state and the wave's fixed-order totals,
  // stored as state z's partial.  LV (the level-sum debug mode): every
  // lane also keeps one run per relative subset size, and the wave adds
  // them into its level sums lvs[0..n] (LDS) lane by lane in lane order.
  template <bool LV = false>
  __device__ __forceinline__ static void finish(const R (&leaf)[psize(SB)], const R& lg, int32_t lm, int L,
                                                int lane, int n, int z, Acc* partials, bool& bad, PhaseClock& pc,
                                                Acc* lvs = nullptr) {
    LaneAcc<TT, LV ? SB + 1 : 0> acc;
    acc.p[0] = TT::acc_zero();
    acc.p[1] = TT::acc_zero();
    if constexpr (LV) {
#pragma unroll
      for (int d = 0; d <= SB; ++d) acc.lv[d] = TT::acc_zero();
    }
    if (lane < (1 << L)) Bottom<TT, SB>::template run<0>(leaf, lg, acc, bad);
    pc.mark(PH_BOTTOM);
    if constexpr (LV) {
      for (int l = 0; l < (1 << L); ++l) {
        const int ml = __builtin_amdgcn_readlane(lm, l);
#pragma unroll
        for (int d = 0; d <= SB; ++d) {
          const Acc x = lane_bcast(TT::acc_fix(acc.lv[d]), l);
          if (lane == 0) lvs[ml + d] = TT::acc_merge(lvs[ml + d], x);
        }
      }
    }
    // the lane's state has |Z| = lm: its own term has sign (-1)^(n - lm)
    const Acc pe = TT::acc_fix(acc.p[0]), po = TT::acc_fix(acc.p[1]);
    const bool odd = ((n - lm) & 1) != 0;
    const Acc lt = odd ? TT::acc_merge(po, r_neg(pe)) : TT::acc_merge(pe, r_neg(po));
    const Acc tt = wave_total<TT>(lt);
    const Acc ta = wave_total<TT>(TT::acc_merge(pe, po));
    if (lane == 0) {
      partials[(size_t)z * 2] = tt;
      partials[(size_t)z * 2 + 1] = ta;
    }
    pc.mark(PH_TOTALS);
  }
};

// Middle + bottom kernel.  W = 1: one wavefront per workgroup expands its
// states one after another.  W = 2: the two wavefronts of a workgroup take
// turns with the workgroup's LDS: while one expands a state's middle levels
// (bound by LDS and dependency latency) down to its lanes' bottom states in
// registers, the other runs the bottom of the state it expanded before
// (register arithmetic only).  Wavefront w takes states W * blockIdx.x + w + t * W *
// gridDim.x, t = 0, 1, ...
// Wavefronts per SIMD the register allocation aims at: two for the
// two-wavefront kernel where its registers allow (not quad-double, not
// double-double with a bottom of four or more modes, nor binary64 with six),
// else one.
template <class TT, int SB, int W>
constexpr int leaf_waves_per_simd() {
  return (W == 2 && TT::id != TOR_QD && !(TT::id == TOR_DD && SB >= 4) && !(TT::id == TOR_FP64 && SB >= 6))
             ? 2
             : 1;
}

// Whether the expanding wavefront hands its lanes' pair states over in
// registers, so that the last middle level runs beside the bottom instead
// of inside the expansion (which the other wavefront waits for): where the
// registers allow it at one wavefront per SIMD (double-double with a
// four-mode bottom, binary64 with a six-mode one; the five-mode
// double-double pair state would need 312 more registers).
template <class TT, int SB, int W>
constexpr bool leaf_pair_in_registers() {
  return W == 2 && ((TT::id == TOR_DD && SB == 4) || (TT::id == TOR_FP64 && SB == 6));
}

template <class TT, int SB, int W, bool LV = false>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(leaf_waves_per_simd<TT, SB, W>()))) void leaf_kernel(const typename TT::R* __restrict__ mat,
                                                      const typename TT::R* __restrict__ gin,
                                                      const int32_t* __restrict__ min_, int s_m,
                                                      int nstates, int n,
                                                      typename TT::Acc* __restrict__ partials,
                                                      int32_t* __restrict__ status,
                                                      typename TT::Acc* __restrict__ lvpart = nullptr) {
  using R = typename TT::R;
  using LF = Leaf<TT, SB>;
  using SMEM = typename LF::SMEM;
  static_assert(SMEM::max_items() * psize(SMEM::SM) < (1 << 20), "DivBy range");
  static_assert(W == 1 || W == 2, "one or two wavefronts");
  static_assert(!LV || W == 1, "the level-sum mode runs one wavefront per workgroup");
  __shared__ SMEM sm;
  // level sums of the wavefront (level-sum mode only)
  __shared__ typename TT::Acc lvs[LV ? TOR_NMAX + 1 : 1];
  const int wv = (int)threadIdx.x >> 6;
  const int lane = (int)threadIdx.x & 63;
  if constexpr (LV) {
    for (int m = lane; m <= n; m += 64) lvs[m] = TT::acc_zero();
  }
  for (int q = (int)threadIdx.x; q < (SMEM::SM - 1) * SMEM::SM / 2; q += 64 * W) {
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    sm.blocks[q] = (uint16_t)(i | ((q - i * (i + 1) / 2) << 8));
  }
  __syncthreads();
  const int L = s_m - SB;  // middle levels, 0..6
  const int ps0 = psize(s_m);
  const int zstride = W * (int)gridDim.x;
  bool bad = false;
  constexpr bool PR = leaf_pair_in_registers<TT, SB, W>();
  R v0 = r_zero<R>(), v1 = v0, v2 = v0, v3 = v0, v4 = v0, v5 = v0, g = v0, lg = v0, pg = v0;
  int32_t m = 0, lm = 0, pm = 0;
  R leaf[psize(SB)];
  R P[LF::NP];

  PhaseClock pc;
  const int zb = W * (int)blockIdx.x;
  if (zb + wv < nstates) LF::fetch(mat, gin, min_, zb + wv, ps0, lane, v0, v1, v2, v3, v4, v5, g, m);
  // W = 2: both wavefronts run the same loop, expand | barrier | bottom |
  // barrier, with wavefront 1 one barrier behind: barrier k of one pairs
  // with barrier k of the other, so each expansion starts after the other
  // wavefront's expansion has ended and its bottom overlaps the other's
  // expansion.  Both run 2 * rounds + 1 barriers.
  const int rounds = zb < nstates ? (nstates - zb + zstride - 1) / zstride : 0;
  if (W == 2 && wv == 1) __syncthreads();
  pc.mark(PH_OTHER);
  for (int t = 0; t < rounds; ++t) {
    const int z = zb + wv + t * zstride;
    if (z < nstates) {
      if constexpr (PR) {
        LF::expand_pair(sm, mat, gin, min_, z + zstride, nstates, s_m, L, ps0, lane, bad, v0, v1, v2, v3, v4, v5, g,
                        m, P, pg, pm);
        pc.mark(PH_EXPAND);
      } else {
        LF::expand(sm, mat, gin, min_, z + zstride, nstates, s_m, L, ps0, lane, bad, v0, v1, v2, v3, v4, v5, g, m,
                   leaf, lg, lm, pc);
      }
    }
    if (W == 2) __syncthreads(); else wave_sync();
    pc.mark(PH_WAIT_A);
    if (z < nstates) {
      if constexpr (PR) {
        LF::last_level(P, pg, pm, L, lane, bad, leaf, lg, lm);
        pc.mark(PH_LAST);
      }
      LF::template finish<LV>(leaf, lg, lm, L, lane, n, z, partials, bad, pc, lvs);
    }
    if (W == 2) __syncthreads();
    pc.mark(PH_WAIT_B);
  }
  if (W == 2 && wv == 0) __syncthreads();
  if constexpr (LV) {
    wave_sync();
    for (int m = lane; m <= n; m += 64) lvpart[(size_t)blockIdx.x * (n + 1) + m] = lvs[m];
  }
  pc.mark(PH_OTHER);
  pc.flush(lane);
  if (bad) atomicOr(status, 1);
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------

template <class TT>
static size_t rbytes() {
  return sizeof(typename TT::R);
}

size_t schur_value_bytes(int tier) {
  return tier == TOR_FP64 ? sizeof(double) : (tier == TOR_DD ? sizeof(dd) : sizeof(qd));
}

void schur_levels(int tier, int n, int sb_req, int* s_m, int* s_b) {
  // bottom size: the largest whose registers fit one wavefront per SIMD and
  // whose middle levels leave two workgroups' LDS per CU (the fastest
  // measured); six middle levels (64 bottom states)
  const int sb_max = tier == TOR_FP64 ? 6 : (tier == TOR_DD ? 5 : 3);
  int sb = sb_max;
  if (sb_req > 0) sb = sb_req < sb_max ? sb_req : sb_max;
  if (sb > n) sb = n;
  int sm = sb + 6;
  if (sm > n) sm = n;
  *s_m = sm;
  *s_b = sb;
}

hipError_t launch_real_root(int tier, const double2* O, const int64_t* offs, int ninst, int n,
                            int64_t ld, void* mat, void* g, int32_t* m, hipStream_t s) {
  const int total = psize(n);
  const dim3 grid((total + 255) / 256, ninst), block(256);
  switch (tier) {
    case TOR_FP64:
      hipLaunchKernelGGL(real_root_kernel<TierF64>, grid, block, 0, s, O, offs, n, ld, (double*)mat,
                         (double*)g, m);
      break;
    case TOR_DD:
      hipLaunchKernelGGL(real_root_kernel<TierDD>, grid, block, 0, s, O, offs, n, ld, (dd*)mat,
                         (dd*)g, m);
      break;
    default:
      hipLaunchKernelGGL(real_root_kernel<TierQD>, grid, block, 0, s, O, offs, n, ld, (qd*)mat,
                         (qd*)g, m);
  }
  return hipGetLastError();
}

// Frontier sizes from which the expansion packs two or four states into a
// workgroup.
constexpr int EXPAND_G2_MIN = 512;
constexpr int EXPAND_G4_MIN = 2048;

hipError_t launch_expand(int tier, const void* in_mat, const void* in_g, const int32_t* in_m,
                         int s, int nst, void* out_mat, void* out_g, int32_t* out_m,
                         int32_t* status, hipStream_t st) {
  if (nst <= 0) return hipSuccess;
  // states per workgroup: enough workgroups to fill the chip several times
  // over with the fewest threads idle on small states
  const int G = nst >= EXPAND_G4_MIN ? 4 : (nst >= EXPAND_G2_MIN ? 2 : 1);
  const dim3 grid((nst + G - 1) / G), block(256);
  switch (tier * 4 + G) {
#define TOR_EXPAND_CASE(TID, TT, RT, GG)                                                                \
  case TID * 4 + GG:                                                                                   \
    hipLaunchKernelGGL((expand_kernel<TT, GG>), grid, block, 0, st, (const RT*)in_mat, (const RT*)in_g, \
                       in_m, s, nst, (RT*)out_mat, (RT*)out_g, out_m, status);                         \
    break;
    TOR_EXPAND_CASE(TOR_FP64, TierF64, double, 1)
    TOR_EXPAND_CASE(TOR_FP64, TierF64, double, 2)
    TOR_EXPAND_CASE(TOR_FP64, TierF64, double, 4)
    TOR_EXPAND_CASE(TOR_DD, TierDD, dd, 1)
    TOR_EXPAND_CASE(TOR_DD, TierDD, dd, 2)
    TOR_EXPAND_CASE(TOR_DD, TierDD, dd, 4)
    TOR_EXPAND_CASE(TOR_QD, TierQD, qd, 1)
    TOR_EXPAND_CASE(TOR_QD, TierQD, qd, 2)
    TOR_EXPAND_CASE(TOR_QD, TierQD, qd, 4)
#undef TOR_EXPAND_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t expand_multi_lds_bytes(int tier, int s, int K) {
  if (K < 2 || K > 3 || s - K < 1) return 0;
  return expand_multi_vals(s, K) * schur_value_bytes(tier) + 2 * ((size_t)1 << K) * sizeof(int32_t);
}

// Whether a launch stages its input state in LDS: where the copy still
// leaves three workgroups room on a CU.
static bool expand_multi_stage(int tier, int s, int K) {
  return expand_multi_lds_bytes(tier, s, K) + (size_t)psize(s) * schur_value_bytes(tier) <=
         EXPAND_MULTI_STAGE_LDS_MAX;
}

hipError_t launch_expand_multi(int tier, const void* in_mat, const void* in_g, const int32_t* in_m,
                               int s, int K, int nst, void* out_mat, void* out_g, int32_t* out_m,
                               int32_t* status, hipStream_t st) {
  if (nst <= 0) return hipSuccess;
  size_t lds = expand_multi_lds_bytes(tier, s, K);
  if (lds == 0 || lds > EXPAND_MULTI_LDS_MAX) return hipErrorInvalidValue;
  const int stage = expand_multi_stage(tier, s, K) ? 1 : 0;
  if (stage) lds += (size_t)psize(s) * schur_value_bytes(tier);
  const dim3 grid(nst), block(256);
  switch (tier) {
    case TOR_FP64:
      hipLaunchKernelGGL(expand_multi_kernel<TierF64>, grid, block, lds, st, (const double*)in_mat,
                         (const double*)in_g, in_m, s, K, (double*)out_mat, (double*)out_g, out_m, status, stage);
      break;
    case TOR_DD:
      hipLaunchKernelGGL(expand_multi_kernel<TierDD>, grid, block, lds, st, (const dd*)in_mat,
                         (const dd*)in_g, in_m, s, K, (dd*)out_mat, (dd*)out_g, out_m, status, stage);
      break;
    default:
      hipLaunchKernelGGL(expand_multi_kernel<TierQD>, grid, block, lds, st, (const qd*)in_mat,
                         (const qd*)in_g, in_m, s, K, (qd*)out_mat, (qd*)out_g, out_m, status, stage);
  }
  return hipGetLastError();
}

// Wavefronts per workgroup of the middle + bottom kernel: two (taking turns
// with the LDS), except quad-double with a bottom of one or two modes, whose
// expansions outweigh its bottoms (measured slower with two).
template <class TT, int SB>
constexpr int leaf_waves() {
  return (TT::id == TOR_QD && SB <= 2) ? 1 : 2;
}

template <class TT, int SB>
static hipError_t launch_leaf_t(const void* mat, const void* g, const int32_t* m, int s_m, int nst,
                                int n, void* partials, int32_t* status, int grid, hipStream_t st) {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  constexpr int W = leaf_waves<TT, SB>();
  const int blocks = grid < (nst + W - 1) / W ? grid : (nst + W - 1) / W;
  hipLaunchKernelGGL((leaf_kernel<TT, SB, W>), dim3(blocks), dim3(64 * W), 0, st, (const R*)mat,
                     (const R*)g, m, s_m, nst, n, (Acc*)partials, status);
  return hipGetLastError();
}

template <class TT, int SB>
static const void* leaf_fn() {
  return reinterpret_cast<const void*>(&leaf_kernel<TT, SB, leaf_waves<TT, SB>()>);
}

// Compiled (tier, s_b) combinations: s_b is the tier's register budget, or n
// when n is smaller.
#define TOR_LEAF_DISPATCH(CALL)                                   \
  if (tier == TOR_FP64) {                                         \
    switch (s_b) {                                                \
      case 1: return CALL(TierF64, 1);                            \
      case 2: return CALL(TierF64, 2);                            \
      case 3: return CALL(TierF64, 3);                            \
      case 4: return CALL(TierF64, 4);                            \
      case 5: return CALL(TierF64, 5);                            \
      case 6: return CALL(TierF64, 6);                            \
      default: break;                                             \
    }                                                             \
  } else if (tier == TOR_DD) {                                    \
    switch (s_b) {                                                \
      case 1: return CALL(TierDD, 1);                             \
      case 2: return CALL(TierDD, 2);                             \
      case 3: return CALL(TierDD, 3);                             \
      case 4: return CALL(TierDD, 4);                             \
      case 5: return CALL(TierDD, 5);                             \
      default: break;                                             \
    }                                                             \
  } else {                                                        \
    switch (s_b) {                                                \
      case 1: return CALL(TierQD, 1);                             \
      case 2: return CALL(TierQD, 2);                             \
      case 3: return CALL(TierQD, 3);                             \
      default: break;                                             \
    }                                                             \
  }                                                               \
  return hipErrorInvalidValue;

hipError_t launch_leaf(int tier, int s_m, int s_b, const void* mat, const void* g, const int32_t* m,
                       int nst, int n, void* partials, int32_t* status, int grid, hipStream_t st) {
  if (s_m < s_b || s_m - s_b > 6) return hipErrorInvalidValue;
#define CALL(TT, SBV) launch_leaf_t<TT, SBV>(mat, g, m, s_m, nst, n, partials, status, grid, st)
  TOR_LEAF_DISPATCH(CALL)
#undef CALL
}

// Level-sum debug mode: one wavefront per workgroup, bottoms of at most
// LEVEL_SB_MAX(tier) modes (their level runs need registers).
template <class TT, int SB>
static hipError_t launch_leaf_levels_t(const void* mat, const void* g, const int32_t* m, int s_m, int nst, int n,
                                       void* partials, int32_t* status, int grid, void* lvpart, hipStream_t st) {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  const int blocks = grid < nst ? grid : nst;
  hipLaunchKernelGGL((leaf_kernel<TT, SB, 1, true>), dim3(blocks), dim3(64), 0, st, (const R*)mat, (const R*)g, m,
                     s_m, nst, n, (Acc*)partials, status, (Acc*)lvpart);
  return hipGetLastError();
}

int level_sb_max(int tier) { return tier == TOR_FP64 ? 4 : (tier == TOR_DD ? 3 : 2); }

hipError_t launch_leaf_levels(int tier, int s_m, int s_b, const void* mat, const void* g, const int32_t* m,
                              int nst, int n, void* partials, int32_t* status, int grid, void* lvpart,
                              hipStream_t st) {
  if (s_m < s_b || s_m - s_b > 6) return hipErrorInvalidValue;
#define LV_CASE(TID, TT, SBV)                                                                                 \
  if (tier == TID && s_b == SBV)                                                                             \
    return launch_leaf_levels_t<TT, SBV>(mat, g, m, s_m, nst, n, partials, status, grid, lvpart, st);
  LV_CASE(TOR_FP64, TierF64, 1) LV_CASE(TOR_FP64, TierF64, 2) LV_CASE(TOR_FP64, TierF64, 3)
  LV_CASE(TOR_FP64, TierF64, 4) LV_CASE(TOR_DD, TierDD, 1) LV_CASE(TOR_DD, TierDD, 2) LV_CASE(TOR_DD, TierDD, 3)
  LV_CASE(TOR_QD, TierQD, 1) LV_CASE(TOR_QD, TierQD, 2)
#undef LV_CASE
  return hipErrorInvalidValue;
}

hipError_t leaf_levels_occupancy(int tier, int s_b, int* blocks_per_cu) {
#define LV_OCC(TID, TT, SBV)                                                                                   \
  if (tier == TID && s_b == SBV)                                                                              \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                      \
        blocks_per_cu, reinterpret_cast<const void*>(&leaf_kernel<TT, SBV, 1, true>), 64, 0);
  LV_OCC(TOR_FP64, TierF64, 1) LV_OCC(TOR_FP64, TierF64, 2) LV_OCC(TOR_FP64, TierF64, 3)
  LV_OCC(TOR_FP64, TierF64, 4) LV_OCC(TOR_DD, TierDD, 1) LV_OCC(TOR_DD, TierDD, 2) LV_OCC(TOR_DD, TierDD, 3)
  LV_OCC(TOR_QD, TierQD, 1) LV_OCC(TOR_QD, TierQD, 2)
#undef LV_OCC
  return hipErrorInvalidValue;
}

hipError_t leaf_occupancy(int tier, int s_b, int* blocks_per_cu) {
#define CALL(TT, SBV) \
  hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, leaf_fn<TT, SBV>(), 64 * leaf_waves<TT, SBV>(), 0)
  TOR_LEAF_DISPATCH(CALL)
#undef CALL
}
#undef TOR_LEAF_DISPATCH

hipError_t phase_clocks(bool reset, uint64_t* out) {
#ifdef TOR_PHASE_CLOCKS
  static_assert(PH_COUNT == TOR_NPHASE, "phase count");
  unsigned long long h[PH_COUNT];
  hipError_t e = hipMemcpyFromSymbol(h, HIP_SYMBOL(tor_phase_clk), sizeof(h), 0, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  for (int k = 0; k < PH_COUNT; ++k) out[k] = h[k];
  if (reset) {
    const unsigned long long zero[PH_COUNT] = {};
    e = hipMemcpyToSymbol(HIP_SYMBOL(tor_phase_clk), zero, sizeof(zero), 0, hipMemcpyHostToDevice);
  }
  return e;
#else
  (void)reset;
  (void)out;
  return hipErrorNotSupported;
#endif
}

}  // namespace tor
