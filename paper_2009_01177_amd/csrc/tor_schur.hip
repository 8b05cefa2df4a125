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
// the reciprocal square roots of the two pivots.
//
// Three levels, one per memory:
//   top    (HBM)  breadth-first expansion, one launch per decided mode, of
//                 every state down to depth n - s_m; each state stores its
//                 packed s_m-mode matrix, g and |Z|.
//   middle (LDS)  one wavefront per depth-(n - s_m) state walks the subsets
//                 of the next s_m - s_b modes depth-first; the updates are
//                 spread over the lanes; each state reached at depth n - s_b
//                 is handed to one lane.
//   bottom (VGPR) each lane finishes its own state: all 2^s_b subsets of the
//                 last s_b modes, fully unrolled at compile time with the
//                 matrices in registers.
// Every wavefront writes one partial (signed sum, sum of magnitudes) per
// middle state; the reductions run in a fixed order, so results do not
// depend on scheduling.
#include <hip/hip_runtime.h>

#include "tiers.hpp"
#include "tor_internal.hpp"

namespace tor {

// Packed lower triangle, row-major: entry (a, b), a >= b.
__host__ __device__ constexpr int pk(int a, int b) { return a * (a + 1) / 2 + b; }
// Entries of the packed 2s x 2s symmetric matrix of s modes.
__host__ __device__ constexpr int psize(int s) { return s * (2 * s + 1); }

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

// Accumulators of one lane: signed sum and sum of magnitudes.
template <class TT>
struct LaneAcc {
  typename TT::Acc t, a;
};

// Emit the term of a completed subset: (-1)^(n-m) g.
template <class TT>
__device__ __forceinline__ void emit_term(LaneAcc<TT>& acc, const typename TT::R& g, int m, int n) {
  acc.t = TT::acc_add(acc.t, ((n - m) & 1) ? r_neg(g) : g);
  acc.a = TT::acc_add(acc.a, g);
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

// --------------------------------------------------------------------------
// Bottom level: one lane, all subsets of S modes, registers only.
// T is the packed 2S x 2S matrix of the lane's state, g its det^(-1/2),
// m its subset size.  Children are taken largest index first so the parent
// matrix dies before the largest child (index 0) is formed.
// --------------------------------------------------------------------------

template <class TT, int S>
struct Bottom {
  using R = typename TT::R;

  template <int I>
  __device__ __forceinline__ static void child(const R (&T)[psize(S)], const R& g, int m, int n,
                                               LaneAcc<TT>& acc, bool& bad) {
    constexpr int SC = S - 1 - I;
    constexpr int O = 2 * I + 2;
    const Pivot<R> pv = make_pivot(T[pk(2 * I, 2 * I)], T[pk(2 * I + 1, 2 * I)], T[pk(2 * I + 1, 2 * I + 1)]);
    if (!pv.ok) bad = true;
    const R gc = r_mul(r_mul(g, pv.rl0), pv.rl1);
    if constexpr (SC == 0) {
      emit_term(acc, gc, m + 1, n);
    } else {
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
          C[pk(a, b)] = r_fms(r_fms(T[pk(a + O, b + O)], u0[a], u0[b]), u1[a], u1[b]);
        }
      }
      Bottom<TT, SC>::run(C, gc, m + 1, n, acc, bad);
    }
  }

  template <int I>
  __device__ __forceinline__ static void children(const R (&T)[psize(S)], const R& g, int m, int n,
                                                  LaneAcc<TT>& acc, bool& bad) {
    child<I>(T, g, m, n, acc, bad);
    if constexpr (I > 0) children<I - 1>(T, g, m, n, acc, bad);
  }

  __device__ __forceinline__ static void run(const R (&T)[psize(S)], const R& g, int m, int n,
                                             LaneAcc<TT>& acc, bool& bad) {
    emit_term(acc, g, m, n);
    children<S - 1>(T, g, m, n, acc, bad);
  }
};

// --------------------------------------------------------------------------
// Root staging: the real matrix R of all n modes (packed), g = 1, |Z| = 0.
// Row 2k is mode k's q quadrature, row 2k+1 its p quadrature.
// --------------------------------------------------------------------------

template <class TT>
__global__ void real_root_kernel(const double2* __restrict__ O, int n, int64_t ld,
                                 typename TT::R* __restrict__ mat, typename TT::R* __restrict__ g,
                                 int32_t* __restrict__ msz) {
  using R = typename TT::R;
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
      x = O[(int64_t)i * ld + j];
    } else {
      const double2 w = O[(int64_t)j * ld + i];
      x = make_double2(w.x, -w.y);
    }
    const double2 w1 = O[(int64_t)(j + n) * ld + i];  // O10_ji = conj(O01_ij)
    const double2 y = make_double2(w1.x, -w1.y);      // O01_ij
    const double dlt = (i == j && qi == qj) ? 1.0 : 0.0;
    R v;
    if (qi == 0 && qj == 0) v = r_from_sum<R>(dlt, -x.x, -y.x);       // delta - Re(O00 + O01)
    else if (qi == 0 && qj == 1) v = r_from_sum<R>(0.0, x.y, -y.y);   // Im(O00 - O01)
    else if (qi == 1 && qj == 0) v = r_from_sum<R>(0.0, -x.y, -y.y);  // -Im(O00 + O01)
    else v = r_from_sum<R>(dlt, -x.x, y.x);                           // delta - Re(O00 - O01)
    mat[e] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g[0] = r_of<R>(1.0);
    msz[0] = 0;
  }
}

// --------------------------------------------------------------------------
// Top level: expand every state of a frontier by one mode.
// in: nst states of s modes; out: 2*nst states of s-1 modes,
// child 2z leaves the mode out, child 2z+1 takes it in.
// --------------------------------------------------------------------------

template <class TT>
__global__ __launch_bounds__(256) void expand_kernel(const typename TT::R* __restrict__ in_mat,
                                                     const typename TT::R* __restrict__ in_g,
                                                     const int32_t* __restrict__ in_m, int s,
                                                     typename TT::R* __restrict__ out_mat,
                                                     typename TT::R* __restrict__ out_g,
                                                     int32_t* __restrict__ out_m,
                                                     int32_t* __restrict__ status) {
  using R = typename TT::R;
  __shared__ R su0[128], su1[128];
  __shared__ R spv[3];
  const int z = blockIdx.x;
  const R* T = in_mat + (size_t)z * psize(s);
  const int sc = s - 1;
  const int nr = 2 * sc;  // rows of a child
  if (threadIdx.x == 0) {
    const Pivot<R> pv = make_pivot(T[pk(0, 0)], T[pk(1, 0)], T[pk(1, 1)]);
    if (!pv.ok) atomicOr(status, 1);
    spv[0] = pv.rl0;
    spv[1] = pv.l10;
    spv[2] = pv.rl1;
    out_g[2 * z] = in_g[z];
    out_m[2 * z] = in_m[z];
    out_g[2 * z + 1] = r_mul(r_mul(in_g[z], pv.rl0), pv.rl1);
    out_m[2 * z + 1] = in_m[z] + 1;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < nr; a += blockDim.x) {
    const R u0 = r_mul(T[pk(a + 2, 0)], spv[0]);
    su0[a] = u0;
    su1[a] = r_mul(r_fms(T[pk(a + 2, 1)], u0, spv[1]), spv[2]);
  }
  __syncthreads();
  R* ex = out_mat + (size_t)(2 * z) * psize(sc);
  R* in = out_mat + (size_t)(2 * z + 1) * psize(sc);
  const int ne = psize(sc);
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    int a = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (pk(a + 1, 0) <= e) ++a;
    while (pk(a, 0) > e) --a;
    const int b = e - pk(a, 0);
    const R t = T[pk(a + 2, b + 2)];
    ex[e] = t;
    in[e] = r_fms(r_fms(t, su0[a], su0[b]), su1[a], su1[b]);
  }
}

// --------------------------------------------------------------------------
// Middle + bottom: one wavefront per middle state (s_m undecided modes).
// --------------------------------------------------------------------------

template <class TT>
struct MidFrame {
  int base, s, m, i;
  typename TT::R g;
};

// LDS layout of one wavefront (WG = 1 wavefront).
template <class TT, int SM, int SB>
struct MidSmem {
  using R = typename TT::R;
  static constexpr int stack_vals() {
    int v = 0;
    for (int s = SM; s >= SB; s -= 2) v += psize(s);
    return v;
  }
  static constexpr int max_frames = (SM - SB) + 2;
  R stack[stack_vals()];
  R u0[2 * SM], u1[2 * SM];
  MidFrame<TT> frames[max_frames];
  uint16_t pairs[psize(SM)];  // packed index -> (row << 8) | col
};

template <class TT, int SM, int SB>
__global__ __launch_bounds__(64) void leaf_kernel(const typename TT::R* __restrict__ mat,
                                                  const typename TT::R* __restrict__ gin,
                                                  const int32_t* __restrict__ min_, int s_m,
                                                  int nstates, int n,
                                                  typename TT::Acc* __restrict__ partials,
                                                  int32_t* __restrict__ status) {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  __shared__ MidSmem<TT, SM, SB> sm;
  const int lane = threadIdx.x;
  for (int e = lane; e < psize(SM); e += 64) {
    int r = 0;
    while (pk(r + 1, 0) <= e) ++r;
    sm.pairs[e] = (uint16_t)((r << 8) | (e - pk(r, 0)));
  }
  bool bad = false;

  for (int z = blockIdx.x; z < nstates; z += gridDim.x) {
    __syncthreads();
    const R* src = mat + (size_t)z * psize(s_m);
    for (int e = lane; e < psize(s_m); e += 64) sm.stack[e] = src[e];
    LaneAcc<TT> acc;
    acc.t = TT::acc_zero();
    acc.a = TT::acc_zero();
    R leaf[psize(SB)];  // this lane's bottom-level state
#pragma unroll
    for (int e = 0; e < psize(SB); ++e) leaf[e] = r_zero<R>();
    R leaf_g = r_zero<R>();
    int leaf_m = 0;
    int nleaf = 0;
    int sp = 0;
    if (lane == 0 && s_m > SB) {
      MidFrame<TT> f;
      f.base = 0;
      f.s = s_m;
      f.m = min_[z];
      f.i = s_m - SB - 1;
      f.g = gin[z];
      sm.frames[0] = f;
    }
    __syncthreads();
    // the pending state to hand to a lane: trailing SB modes of (base, s)
    bool have = true, finished = (s_m == SB);
    int p_base = 0, p_s = s_m, p_m = min_[z];
    R p_g = gin[z];

    for (;;) {
      if (have) {
        const int o = 2 * (p_s - SB);
#pragma unroll
        for (int a = 0; a < 2 * SB; ++a) {
#pragma unroll
          for (int b = 0; b <= a; ++b) {
            const R v = sm.stack[p_base + pk(a + o, b + o)];
            if (lane == nleaf) leaf[pk(a, b)] = v;
          }
        }
        if (lane == nleaf) {
          leaf_g = p_g;
          leaf_m = p_m;
        }
        ++nleaf;
        have = false;
      }
      if (nleaf == 64 || (finished && nleaf > 0)) {
        if (lane < nleaf) Bottom<TT, SB>::run(leaf, leaf_g, leaf_m, n, acc, bad);
        nleaf = 0;
      }
      if (finished) break;

      // one step of the middle-level depth-first walk
      const MidFrame<TT> f = sm.frames[sp];
      if (f.i < 0) {
        --sp;
        if (sp < 0) finished = true;
        continue;
      }
      const int i = f.i;
      const int sc = f.s - 1 - i;  // undecided modes of the child
      const int dst = (i > 0) ? f.base + psize(f.s) : f.base;
      const int o = 2 * i + 2;
      const R* T = sm.stack + f.base;
      const Pivot<R> pv = make_pivot(T[pk(2 * i, 2 * i)], T[pk(2 * i + 1, 2 * i)],
                                     T[pk(2 * i + 1, 2 * i + 1)]);
      if (!pv.ok) bad = true;
      const R gc = r_mul(r_mul(f.g, pv.rl0), pv.rl1);
      if (lane < 2 * sc) {
        const R u0 = r_mul(T[pk(lane + o, 2 * i)], pv.rl0);
        sm.u0[lane] = u0;
        sm.u1[lane] = r_mul(r_fms(T[pk(lane + o, 2 * i + 1)], u0, pv.l10), pv.rl1);
      }
      __syncthreads();
      // child entries; in place (i == 0) is safe: entry e reads index > e
      R* C = sm.stack + dst;
      const int ne = psize(sc);
      for (int e0 = 0; e0 < ne; e0 += 64) {
        const int e = e0 + lane;
        R v = r_zero<R>();
        if (e < ne) {
          const int pr = sm.pairs[e];
          const int a = pr >> 8, b = pr & 255;
          v = r_fms(r_fms(T[pk(a + o, b + o)], sm.u0[a], sm.u0[b]), sm.u1[a], sm.u1[b]);
        }
        __syncthreads();
        if (e < ne) C[e] = v;
      }
      if (lane == 0) {
        if (sc == SB) {
          sm.frames[sp].i = i - 1;
        } else {
          MidFrame<TT> cf;
          cf.base = dst;
          cf.s = sc;
          cf.m = f.m + 1;
          cf.i = sc - SB - 1;
          cf.g = gc;
          if (i > 0) {
            sm.frames[sp].i = i - 1;
            sm.frames[sp + 1] = cf;
          } else {
            sm.frames[sp] = cf;
          }
        }
      }
      if (sc != SB && i > 0) ++sp;
      if (sc == SB && i == 0) {
        // the frame's last child was a leaf: the frame is done
        --sp;
      }
      __syncthreads();
      have = true;
      p_base = dst;
      p_s = sc;
      p_m = f.m + 1;
      p_g = gc;
      if (sp < 0) finished = true;
    }
    // fixed-order butterfly over the wave, then one partial per state
    Acc t = acc.t, a = acc.a;
#pragma unroll
    for (int msk = 32; msk >= 1; msk >>= 1) {
      t = TT::acc_merge(t, lane_xor(t, msk));
      a = TT::acc_merge(a, lane_xor(a, msk));
    }
    if (lane == 0) {
      partials[(size_t)z * 2] = t;
      partials[(size_t)z * 2 + 1] = a;
    }
  }
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

void schur_levels(int tier, int n, int* s_m, int* s_b) {
  // bottom size by register budget; middle size by LDS budget
  int sb = tier == TOR_FP64 ? 5 : (tier == TOR_DD ? 4 : 2);
  int smx = tier == TOR_QD ? 10 : 12;
  if (sb > n) sb = n;
  int sm = smx < n ? smx : n;
  if (sm < sb) sm = sb;
  *s_m = sm;
  *s_b = sb;
}

hipError_t launch_real_root(int tier, const double2* O, int n, int64_t ld, void* mat, void* g,
                            int32_t* m, hipStream_t s) {
  const int total = psize(n);
  const dim3 grid((total + 255) / 256), block(256);
  switch (tier) {
    case TOR_FP64:
      hipLaunchKernelGGL(real_root_kernel<TierF64>, grid, block, 0, s, O, n, ld, (double*)mat,
                         (double*)g, m);
      break;
    case TOR_DD:
      hipLaunchKernelGGL(real_root_kernel<TierDD>, grid, block, 0, s, O, n, ld, (dd*)mat, (dd*)g, m);
      break;
    default:
      hipLaunchKernelGGL(real_root_kernel<TierQD>, grid, block, 0, s, O, n, ld, (qd*)mat, (qd*)g, m);
  }
  return hipGetLastError();
}

hipError_t launch_expand(int tier, const void* in_mat, const void* in_g, const int32_t* in_m,
                         int s, int nst, void* out_mat, void* out_g, int32_t* out_m,
                         int32_t* status, hipStream_t st) {
  if (nst <= 0) return hipSuccess;
  const dim3 grid(nst), block(256);
  switch (tier) {
    case TOR_FP64:
      hipLaunchKernelGGL(expand_kernel<TierF64>, grid, block, 0, st, (const double*)in_mat,
                         (const double*)in_g, in_m, s, (double*)out_mat, (double*)out_g, out_m, status);
      break;
    case TOR_DD:
      hipLaunchKernelGGL(expand_kernel<TierDD>, grid, block, 0, st, (const dd*)in_mat,
                         (const dd*)in_g, in_m, s, (dd*)out_mat, (dd*)out_g, out_m, status);
      break;
    default:
      hipLaunchKernelGGL(expand_kernel<TierQD>, grid, block, 0, st, (const qd*)in_mat,
                         (const qd*)in_g, in_m, s, (qd*)out_mat, (qd*)out_g, out_m, status);
  }
  return hipGetLastError();
}

template <class TT, int SM, int SB>
static hipError_t launch_leaf_t(const void* mat, const void* g, const int32_t* m, int s_m, int nst,
                                int n, void* partials, int32_t* status, int grid, hipStream_t st) {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  hipLaunchKernelGGL((leaf_kernel<TT, SM, SB>), dim3(grid), dim3(64), 0, st, (const R*)mat,
                     (const R*)g, m, s_m, nst, n, (Acc*)partials, status);
  return hipGetLastError();
}

template <class TT, int SM, int SB>
static const void* leaf_fn() {
  return reinterpret_cast<const void*>(&leaf_kernel<TT, SM, SB>);
}

// Dispatch over the compiled (tier, s_b) combinations; s_m is the LDS
// capacity of the middle level (a runtime s_m <= SM is allowed).
#define TOR_LEAF_CASES(TT, SMX)                                                        \
  switch (s_b) {                                                                       \
    case 1: return CALL(TT, SMX, 1);                                                   \
    case 2: return CALL(TT, SMX, 2);                                                   \
    case 3: return CALL(TT, SMX, 3);                                                   \
    case 4: return CALL(TT, SMX, 4);                                                   \
    case 5: return CALL(TT, SMX, 5);                                                   \
    default: break;                                                                    \
  }

hipError_t launch_leaf(int tier, int s_m, int s_b, const void* mat, const void* g, const int32_t* m,
                       int nst, int n, void* partials, int32_t* status, int grid, hipStream_t st) {
#define CALL(TT, SMX, SBV) launch_leaf_t<TT, SMX, SBV>(mat, g, m, s_m, nst, n, partials, status, grid, st)
  if (tier == TOR_FP64) {
    TOR_LEAF_CASES(TierF64, 12)
  } else if (tier == TOR_DD) {
    switch (s_b) {
      case 1: return CALL(TierDD, 12, 1);
      case 2: return CALL(TierDD, 12, 2);
      case 3: return CALL(TierDD, 12, 3);
      case 4: return CALL(TierDD, 12, 4);
      default: break;
    }
  } else {
    switch (s_b) {
      case 1: return CALL(TierQD, 10, 1);
      case 2: return CALL(TierQD, 10, 2);
      default: break;
    }
  }
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t leaf_occupancy(int tier, int s_b, int* blocks_per_cu) {
#define CALL(TT, SMX, SBV) hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, leaf_fn<TT, SMX, SBV>(), 64, 0)
  if (tier == TOR_FP64) {
    TOR_LEAF_CASES(TierF64, 12)
  } else if (tier == TOR_DD) {
    switch (s_b) {
      case 1: return CALL(TierDD, 12, 1);
      case 2: return CALL(TierDD, 12, 2);
      case 3: return CALL(TierDD, 12, 3);
      case 4: return CALL(TierDD, 12, 4);
      default: break;
    }
  } else {
    switch (s_b) {
      case 1: return CALL(TierQD, 10, 1);
      case 2: return CALL(TierQD, 10, 2);
      default: break;
    }
  }
#undef CALL
  return hipErrorInvalidValue;
}
#undef TOR_LEAF_CASES

}  // namespace tor
