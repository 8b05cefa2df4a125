// tor_border.hip -- bordered-Cholesky subset-tree kernel for gfx950.
//
// Method (Sec. 3.1, Eq. 2; Alg. 1 made incremental).  With the rows of
// I - O reordered so that each mode's a and a^dagger rows are adjacent
// (a symmetric permutation: every principal minor keeps its determinant),
// appending a mode k to a subset Z appends two rows and columns to
// M_Z = (I - O)_Z:
//
//     M_{Z+k} = [[M_Z, C], [C^H, D]],   M_Z = L L^H,
//     L W = C  (forward substitution, two right-hand sides),
//     S = D - W^H W  (2 x 2),   L_{Z+k} = [[L, 0], [W^H, chol(S)]],
//     det M_{Z+k} = det M_Z * det S.
//
// So a depth-first walk that appends modes in increasing order reuses the
// factor of every ancestor and pays O(|Z|^2) per subset instead of the
// O(|Z|^3) per-subset elimination of Alg. 1.  det^(-1/2) is carried as a
// running product of the two pivots' reciprocal square roots, so each
// subset's signed term costs two multiplies.
//
// Work split (Sec. 4.1's goal, a different cut): the subsets of the first d
// modes are the work items; item p owns every Z with Z intersect [0, d) = p,
// i.e. the depth-first subtree over modes [d, n) hanging off p.  Items are
// handed out by a persistent queue in decreasing cost (larger |p| first).
//
// GPU mapping: one wavefront per item.  Lane i owns factor row i (and row
// i+64 when 2n > 64); the substitution runs column by column, broadcasting
// each solved entry with a lane read, and every lane below it applies one
// complex multiply-subtract per right-hand side.  The factor lives in LDS as
// a packed lower triangle, column-major, so lanes read consecutive words.
// W^H W is a fixed-order butterfly over the wave.  No matrix cores: the
// updates are ragged triangular solves, not a dense contraction.
//
// Every item writes its own partial sums; a separate fixed-order reduction
// makes the result independent of scheduling.
#include <hip/hip_runtime.h>

#include "tiers.hpp"
#include "tor_internal.hpp"

namespace tor {

// Packed lower triangle, column-major: column r holds rows r..Rmax-1.
__device__ __forceinline__ int col_off(int r, int Rmax) { return r * Rmax - ((r * (r - 1)) >> 1); }

template <class TT>
struct BorderSmem {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  using C = cx<R>;
  C* L;       // Rmax(Rmax+1)/2
  R* rinv;    // Rmax: 1 / L_rr
  R* g;       // n+1: det^(-1/2) after each level
  Acc* lev;   // n+1 (levels mode)
  int* modes; // n+1

  static __host__ __device__ size_t bytes(int n, int mode) {
    const int Rmax = 2 * n;
    size_t b = sizeof(C) * (size_t)(Rmax * (Rmax + 1) / 2);
    b += sizeof(R) * (size_t)Rmax;
    b += sizeof(R) * (size_t)(n + 1);
    if (mode == MODE_LEVELS) b += sizeof(Acc) * (size_t)(n + 1);
    b += sizeof(int) * (size_t)(n + 1);
    return b;
  }
  __device__ void carve(char* base, int n, int mode) {
    const int Rmax = 2 * n;
    L = reinterpret_cast<C*>(base);
    rinv = reinterpret_cast<R*>(L + Rmax * (Rmax + 1) / 2);
    g = rinv + Rmax;
    lev = reinterpret_cast<Acc*>(g + n + 1);
    modes = reinterpret_cast<int*>(lev + (mode == MODE_LEVELS ? n + 1 : 0));
  }
};

template <class TT, int RPL, int MODE>
__global__ __launch_bounds__(64) void border_kernel(const double2* __restrict__ Oi, int n, int d,
                                                    const uint64_t* __restrict__ items, int nitems,
                                                    uint32_t* __restrict__ queue,
                                                    typename TT::Acc* __restrict__ partials,
                                                    int32_t* __restrict__ status) {
  using R = typename TT::R;
  using Acc = typename TT::Acc;
  using C = cx<R>;
  extern __shared__ __align__(16) char smem_raw[];
  BorderSmem<TT> sm;
  sm.carve(smem_raw, n, MODE);

  const int lane = threadIdx.x;
  const int Rmax = 2 * n;
  const int ncols = (MODE == MODE_LEVELS) ? 2 + n + 1 : 2;
  const int64_t ld = Rmax;  // Oi is 2n x 2n

  int myrow[RPL];  // interleaved row of I - O that factor row (lane + 64k) stands for
#pragma unroll
  for (int k = 0; k < RPL; ++k) myrow[k] = 0;

  int bad = 0;

  for (;;) {
    uint32_t it = 0;
    if (lane == 0) it = atomicAdd(queue, 1u);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= (uint32_t)nitems) break;
    const uint64_t pmask = items[it];

    Acc accT = TT::acc_zero();
    Acc accA = TT::acc_zero();
    if (MODE == MODE_LEVELS) {
      for (int m = lane; m <= n; m += 64) sm.lev[m] = TT::acc_zero();
    }
    if (lane == 0) sm.g[0] = r_of<R>(1.0);
    __syncthreads();

    int t = 0;  // number of modes on the stack; factor has 2t rows

    // Border the current factor (2t rows) by mode j.  Leaves W in c0/c1
    // (lane-distributed), returns pivots and the new det^(-1/2).
    C c0[RPL], c1[RPL];
    R rinv0, rinv1, gnew;
    C l10;
    auto border = [&](int j) {
      const int Rc = 2 * t;
      // C = (I - O)[rows of Z, (2j, 2j+1)] = conj((I - O)[(2j, 2j+1), rows]) = -conj(Oi[...])
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int i = lane + 64 * k;
        if (i < Rc) {
          const double2 a = Oi[(int64_t)(2 * j) * ld + myrow[k]];
          const double2 b = Oi[(int64_t)(2 * j + 1) * ld + myrow[k]];
          c0[k] = c_of<R>(-a.x, a.y);
          c1[k] = c_of<R>(-b.x, b.y);
        } else {
          c0[k] = c_of<R>(0.0, 0.0);
          c1[k] = c_of<R>(0.0, 0.0);
        }
      }
      // Forward substitution L W = C, column by column.
      for (int r = 0; r < Rc; ++r) {
        C cr0, cr1;
        if constexpr (RPL == 1) {
          cr0 = lane_bcast(c0[0], r);
          cr1 = lane_bcast(c1[0], r);
        } else {
          if (r < 64) {
            cr0 = lane_bcast(c0[0], r);
            cr1 = lane_bcast(c1[0], r);
          } else {
            cr0 = lane_bcast(c0[1], r - 64);
            cr1 = lane_bcast(c1[1], r - 64);
          }
        }
        const R ri = sm.rinv[r];
        const C w0 = c_scale(cr0, ri);
        const C w1 = c_scale(cr1, ri);
        const int coff = col_off(r, Rmax) - r;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = lane + 64 * k;
          if (i == r) {
            c0[k] = w0;
            c1[k] = w1;
          } else if (i > r && i < Rc) {
            const C l = sm.L[coff + i];
            c0[k] = c_fms(c0[k], l, w0);
            c1[k] = c_fms(c1[k], l, w1);
          }
        }
      }
      // S = D - W^H W
      R s00 = r_zero<R>(), s11 = r_zero<R>();
      C s10 = c_of<R>(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        s00 = r_add(s00, c_abs2(c0[k]));
        s11 = r_add(s11, c_abs2(c1[k]));
        const C p = c_conj_mul(c1[k], c0[k]);
        s10.re = r_add(s10.re, p.re);
        s10.im = r_add(s10.im, p.im);
      }
      s00 = wave_sum(s00);
      s11 = wave_sum(s11);
      s10.re = wave_sum(s10.re);
      s10.im = wave_sum(s10.im);
      const double2 o00 = Oi[(int64_t)(2 * j) * ld + 2 * j];
      const double2 o11 = Oi[(int64_t)(2 * j + 1) * ld + 2 * j + 1];
      const double2 o10 = Oi[(int64_t)(2 * j + 1) * ld + 2 * j];
      const R S00 = r_sub(r_one_minus_t<R>(o00.x), s00);
      const R S11 = r_sub(r_one_minus_t<R>(o11.x), s11);
      C S10;
      S10.re = r_sub(r_of<R>(-o10.x), s10.re);
      S10.im = r_sub(r_of<R>(-o10.y), s10.im);
      // chol(S) through reciprocal square roots of the two pivots
      if (!(r_lead(S00) > 0.0)) bad = 1;
      rinv0 = r_rsqrt(S00);
      l10 = c_scale(S10, rinv0);
      const R d2 = r_sub(S11, c_abs2(l10));
      if (!(r_lead(d2) > 0.0)) bad = 1;
      rinv1 = r_rsqrt(d2);
      gnew = r_mul(r_mul(sm.g[t], rinv0), rinv1);
    };

    // Append the bordered rows of mode j (after border(j)).
    auto push = [&](int j) {
      const int Rc = 2 * t;
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int i = lane + 64 * k;
        if (i < Rc) {
          const int o = col_off(i, Rmax) - i;
          sm.L[o + Rc] = c_conj(c0[k]);
          sm.L[o + Rc + 1] = c_conj(c1[k]);
        }
        if (i == Rc) myrow[k] = 2 * j;
        if (i == Rc + 1) myrow[k] = 2 * j + 1;
      }
      if (lane == 0) {
        sm.L[col_off(Rc, Rmax) + 1] = l10;
        sm.rinv[Rc] = rinv0;
        sm.rinv[Rc + 1] = rinv1;
        sm.g[t + 1] = gnew;
        sm.modes[t] = j;
      }
      ++t;
      __syncthreads();
    };

    auto emit = [&](int m, const R& gval) {
      // term (-1)^(n-m) det^(-1/2)
      const R term = ((n - m) & 1) ? r_neg(gval) : gval;
      accT = TT::acc_add(accT, term);
      accA = TT::acc_add(accA, gval);
      if (MODE == MODE_LEVELS && lane == 0) sm.lev[m] = TT::acc_add(sm.lev[m], gval);
    };

    // Prefix factor: border by each prefix mode in increasing order.
    for (int j = 0; j < n; ++j) {
      if ((pmask >> j) & 1ull) {
        border(j);
        push(j);
      }
    }
    emit(t, sm.g[t]);

    if (MODE != MODE_MASKS) {
      // Depth-first walk over the modes [d, n).
      const int t0 = t;
      int j = d;
      for (;;) {
        if (j < n) {
          border(j);
          emit(t + 1, gnew);
          if (j < n - 1) {
            push(j);
            j = j + 1;
          } else {
            j = n;
          }
        } else {
          if (t == t0) break;
          --t;
          j = sm.modes[t] + 1;
        }
      }
    }

    if (lane == 0) {
      Acc* out = partials + (size_t)it * ncols;
      out[0] = accT;
      out[1] = accA;
    }
    if (MODE == MODE_LEVELS) {
      __syncthreads();
      for (int m = lane; m <= n; m += 64) partials[(size_t)it * ncols + 2 + m] = sm.lev[m];
    }
    __syncthreads();
  }
  if (bad) atomicOr(status, 1);
}

// ---------------------------------------------------------------------------
// Staging, zeroing, reduction
// ---------------------------------------------------------------------------

__global__ void stage_kernel(const double2* __restrict__ O, int n, int64_t ld,
                             double2* __restrict__ Oi) {
  const int N2 = 2 * n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N2 * N2) return;
  const int r = idx / N2, c = idx % N2;
  // interleaved r = 2a+u <-> block row a + u n
  const int br = (r >> 1) + (r & 1) * n;
  const int bc = (c >> 1) + (c & 1) * n;
  double2 v;
  if (br >= bc) {
    v = O[(int64_t)br * ld + bc];
  } else {
    const double2 w = O[(int64_t)bc * ld + br];
    v = make_double2(w.x, -w.y);
  }
  Oi[idx] = v;
}

__global__ void zero_kernel(uint32_t* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

// Fixed-order reduction of part[nitems][ncols]: block (k, col) sums the
// items of segment k = [k*SEG, (k+1)*SEG) -- thread t takes every 256th item
// from k*SEG + t, then a tree over the 256 threads -- into red[k][col].  The
// order depends only on SEG and the block size, never on the launch.
constexpr int RED_SEG = 4096;

template <class TT>
__global__ __launch_bounds__(256) void reduce_cols_kernel(const typename TT::Acc* __restrict__ part,
                                                          int nitems, int ncols,
                                                          typename TT::Acc* __restrict__ red) {
  using Acc = typename TT::Acc;
  __shared__ Acc buf[256];
  const int seg = blockIdx.x;
  const int col = blockIdx.y;
  const int tid = threadIdx.x;
  const int lo = seg * RED_SEG;
  const int hi = min(nitems, lo + RED_SEG);
  Acc a = TT::acc_zero();
  for (int i = lo + tid; i < hi; i += 256) a = TT::acc_merge(a, part[(size_t)i * ncols + col]);
  buf[tid] = a;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (tid < s) buf[tid] = TT::acc_merge(buf[tid], buf[tid + s]);
    __syncthreads();
  }
  if (tid == 0) red[(size_t)seg * ncols + col] = buf[0];
}

__device__ inline void acc_store(const dd& a, double* out4) {
  out4[0] = a.hi;
  out4[1] = a.lo;
  out4[2] = 0.0;
  out4[3] = 0.0;
}
__device__ inline void acc_store(const qd& a, double* out4) {
  const qd z = prec::qd_nonoverlapping(a);
  for (int i = 0; i < 4; ++i) out4[i] = z.x[i];
}
__device__ inline void acc_store2(const dd& a, double* out2) {
  out2[0] = a.hi;
  out2[1] = a.lo;
}
__device__ inline void acc_store2(const qd& a, double* out2) {
  const qd z = prec::qd_nonoverlapping(a);
  double s, e;
  prec::fast_two_sum(z.x[0], z.x[1] + (z.x[2] + z.x[3]), s, e);
  out2[0] = s;
  out2[1] = e;
}

template <class TT>
__global__ void finalize_kernel(const typename TT::Acc* __restrict__ red,
                                const int32_t* __restrict__ status, double err_rel,
                                tor_result_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tor_result_t r;
  acc_store(red[0], r.tor);
  acc_store2(red[1], r.abs_sum);
  r.err_bound = err_rel * r.abs_sum[0];
  r.tier_used = TT::id;
  r.status = (status && status[0]) ? TOR_ENOTPD : TOR_OK;
  *out = r;
}

template <class TT>
__global__ __launch_bounds__(256) void seg_reduce_kernel(const typename TT::Acc* __restrict__ part,
                                                         int seg_len,
                                                         typename TT::Acc* __restrict__ out) {
  using Acc = typename TT::Acc;
  __shared__ Acc bt[256], ba[256];
  const int sg = blockIdx.x, tid = threadIdx.x;
  const size_t lo = (size_t)sg * seg_len;
  Acc t = TT::acc_zero(), a = TT::acc_zero();
  for (int i = tid; i < seg_len; i += 256) {
    t = TT::acc_merge(t, part[(lo + i) * 2]);
    a = TT::acc_merge(a, part[(lo + i) * 2 + 1]);
  }
  bt[tid] = t;
  ba[tid] = a;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (tid < s) {
      bt[tid] = TT::acc_merge(bt[tid], bt[tid + s]);
      ba[tid] = TT::acc_merge(ba[tid], ba[tid + s]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[(size_t)sg * 2] = bt[0];
    out[(size_t)sg * 2 + 1] = ba[0];
  }
}

__device__ inline bool acc_finite(const dd& a) { return isfinite(a.hi) && isfinite(a.lo); }
__device__ inline bool acc_finite(const qd& a) {
  return isfinite(a.x[0]) && isfinite(a.x[1]) && isfinite(a.x[2]) && isfinite(a.x[3]);
}

template <class TT>
__global__ void finalize_batch_kernel(const typename TT::Acc* __restrict__ red, int ninst,
                                      const int32_t* __restrict__ out_index, double err_rel,
                                      tor_result_t* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ninst) return;
  tor_result_t r;
  acc_store(red[2 * k], r.tor);
  acc_store2(red[2 * k + 1], r.abs_sum);
  r.err_bound = err_rel * r.abs_sum[0];
  r.tier_used = TT::id;
  r.status = (acc_finite(red[2 * k]) && acc_finite(red[2 * k + 1])) ? TOR_OK : TOR_ENOTPD;
  out[out_index ? out_index[k] : k] = r;
}

__global__ void fill_trivial_kernel(tor_result_t* __restrict__ out,
                                    const int32_t* __restrict__ idx,
                                    const int32_t* __restrict__ tiers, int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  tor_result_t r;
  for (int i = 0; i < 4; ++i) r.tor[i] = 0.0;
  r.tor[0] = 1.0;
  r.abs_sum[0] = 1.0;
  r.abs_sum[1] = 0.0;
  r.err_bound = 0.0;
  r.tier_used = tiers[k];
  r.status = TOR_OK;
  out[idx[k]] = r;
}

template <class Acc>
__global__ void expand_terms_kernel(const Acc* __restrict__ part, int nitems, double* __restrict__ out4) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nitems) acc_store(part[(size_t)i * 2], out4 + 4 * (size_t)i);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

size_t acc_bytes(int tier) { return tier == TOR_QD ? sizeof(qd) : sizeof(dd); }

hipError_t launch_stage(const double2* O, int n, int64_t ld, double2* Oi, hipStream_t s) {
  const int total = 4 * n * n;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(stage_kernel, dim3((total + 255) / 256), dim3(256), 0, s, O, n, ld, Oi);
  return hipGetLastError();
}

// The input conventions the kernels rely on, checked on the device: every
// entry finite, O Hermitian, and the block structure of Eq. 3 (O11 = conj
// O00, O10 = conj O01).  One workgroup per instance; bad[inst] is set to 1
// on any violation (it must be zero on entry).  offs == nullptr: a single
// instance at O with leading dimension ld; else instance k at O + offs[k]
// with leading dimension 2 ns[k].
__global__ __launch_bounds__(256) void check_input_kernel(const double2* __restrict__ O,
                                                          const int64_t* __restrict__ offs,
                                                          const int32_t* __restrict__ ns, int n1, int64_t ld1,
                                                          int32_t* __restrict__ bad) {
  const int inst = blockIdx.x;
  const int n = offs ? ns[inst] : n1;
  const int64_t ld = offs ? 2 * (int64_t)n : ld1;
  const double2* A = offs ? O + offs[inst] : O;
  const int N2 = 2 * n;
  bool ok = true;
  for (int e = threadIdx.x; e < N2 * N2; e += 256) {
    const int i = e / N2, j = e - (e / N2) * N2;
    const double2 a = A[(int64_t)i * ld + j], t = A[(int64_t)j * ld + i];
    ok = ok && isfinite(a.x) && isfinite(a.y) && a.x == t.x && a.y == -t.y;
    if (i < n && j < n) {
      const double2 d = A[(int64_t)(i + n) * ld + (j + n)];  // O11 = conj(O00)
      const double2 c = A[(int64_t)(i + n) * ld + j];        // O10 = conj(O01)
      const double2 b = A[(int64_t)i * ld + (j + n)];
      ok = ok && d.x == a.x && d.y == -a.y && c.x == b.x && c.y == -b.y;
    }
  }
  if (!ok) atomicOr(&bad[inst], 1);
}

hipError_t launch_check_input(const double2* O, const int64_t* offs, const int32_t* ns, int ninst, int n1, int64_t ld1,
                              int32_t* bad, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_input_kernel, dim3(ninst), dim3(256), 0, s, O, offs, ns, n1, ld1, bad);
  return hipGetLastError();
}

hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

size_t border_lds_bytes(int tier, int mode, int n) {
  switch (tier) {
    case TOR_FP64: return BorderSmem<TierF64>::bytes(n, mode);
    case TOR_DD: return BorderSmem<TierDD>::bytes(n, mode);
    default: return BorderSmem<TierQD>::bytes(n, mode);
  }
}

template <class TT, int RPL, int MODE>
static const void* border_fn() {
  return reinterpret_cast<const void*>(&border_kernel<TT, RPL, MODE>);
}

template <class TT>
static const void* border_pick(int n, int mode) {
  const bool two = (2 * n > 64);
  if (mode == MODE_SUM) return two ? border_fn<TT, 2, MODE_SUM>() : border_fn<TT, 1, MODE_SUM>();
  if (mode == MODE_LEVELS)
    return two ? border_fn<TT, 2, MODE_LEVELS>() : border_fn<TT, 1, MODE_LEVELS>();
  return two ? border_fn<TT, 2, MODE_MASKS>() : border_fn<TT, 1, MODE_MASKS>();
}

static const void* border_select(int tier, int n, int mode) {
  switch (tier) {
    case TOR_FP64: return border_pick<TierF64>(n, mode);
    case TOR_DD: return border_pick<TierDD>(n, mode);
    default: return border_pick<TierQD>(n, mode);
  }
}

hipError_t border_occupancy(int tier, int mode, int n, int* blocks_per_cu) {
  const void* fn = border_select(tier, n, mode);
  const size_t lds = border_lds_bytes(tier, mode, n);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, 64, lds);
}

hipError_t launch_border(const BorderLaunch& a, hipStream_t s) {
  const void* fn = border_select(a.tier, a.n, a.mode);
  const size_t lds = border_lds_bytes(a.tier, a.mode, a.n);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const double2* Oi = a.Oi;
  int n = a.n, d = a.d, nitems = a.nitems;
  const uint64_t* items = a.items;
  uint32_t* queue = a.queue;
  void* part = a.partials;
  int32_t* status = a.status;
  void* args[] = {(void*)&Oi, (void*)&n, (void*)&d, (void*)&items, (void*)&nitems,
                  (void*)&queue, (void*)&part, (void*)&status};
  return hipLaunchKernel(fn, dim3(a.grid), dim3(64), args, lds, s);
}

template <class TT>
static void reduce_stage(const void* part, int nitems, int ncols, void* out, hipStream_t s) {
  using Acc = typename TT::Acc;
  const int nseg = (nitems + RED_SEG - 1) / RED_SEG;
  hipLaunchKernelGGL(reduce_cols_kernel<TT>, dim3(nseg > 0 ? nseg : 1, ncols), dim3(256), 0, s,
                     (const Acc*)part, nitems, ncols, (Acc*)out);
}

size_t reduce_scratch_bytes(int tier, int nitems, int ncols) {
  const size_t nseg = (size_t)(nitems + RED_SEG - 1) / RED_SEG;
  return acc_bytes(tier) * (nseg > 1 ? nseg : 1) * ncols;
}

hipError_t launch_reduce_cols(int tier, const void* partials, int nitems, int ncols, void* red,
                              void* scratch, hipStream_t s) {
  const bool two = nitems > RED_SEG;
  const int nseg = (nitems + RED_SEG - 1) / RED_SEG;
  if (tier == TOR_QD) {
    reduce_stage<TierQD>(partials, nitems, ncols, two ? scratch : red, s);
    if (two) reduce_stage<TierQD>(scratch, nseg, ncols, red, s);
  } else {
    reduce_stage<TierDD>(partials, nitems, ncols, two ? scratch : red, s);
    if (two) reduce_stage<TierDD>(scratch, nseg, ncols, red, s);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(int tier, const void* red, const int32_t* status, double err_rel,
                           tor_result_t* out, hipStream_t s) {
  switch (tier) {
    case TOR_FP64:
      hipLaunchKernelGGL(finalize_kernel<TierF64>, dim3(1), dim3(64), 0, s, (const dd*)red, status,
                         err_rel, out);
      break;
    case TOR_DD:
      hipLaunchKernelGGL(finalize_kernel<TierDD>, dim3(1), dim3(64), 0, s, (const dd*)red, status,
                         err_rel, out);
      break;
    default:
      hipLaunchKernelGGL(finalize_kernel<TierQD>, dim3(1), dim3(64), 0, s, (const qd*)red, status,
                         err_rel, out);
  }
  return hipGetLastError();
}

hipError_t launch_seg_reduce(int tier, const void* part, int nseg, int seg_len, void* out,
                             hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  if (tier == TOR_QD)
    hipLaunchKernelGGL(seg_reduce_kernel<TierQD>, dim3(nseg), dim3(256), 0, s, (const qd*)part,
                       seg_len, (qd*)out);
  else
    hipLaunchKernelGGL(seg_reduce_kernel<TierDD>, dim3(nseg), dim3(256), 0, s, (const dd*)part,
                       seg_len, (dd*)out);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(int tier, const void* red, int ninst, const int32_t* out_index,
                                 int n, double err_rel, tor_result_t* out, hipStream_t s) {
  (void)n;
  if (ninst <= 0) return hipSuccess;
  const dim3 g((ninst + 63) / 64), b(64);
  switch (tier) {
    case TOR_FP64:
      hipLaunchKernelGGL(finalize_batch_kernel<TierF64>, g, b, 0, s, (const dd*)red, ninst,
                         out_index, err_rel, out);
      break;
    case TOR_DD:
      hipLaunchKernelGGL(finalize_batch_kernel<TierDD>, g, b, 0, s, (const dd*)red, ninst,
                         out_index, err_rel, out);
      break;
    default:
      hipLaunchKernelGGL(finalize_batch_kernel<TierQD>, g, b, 0, s, (const qd*)red, ninst,
                         out_index, err_rel, out);
  }
  return hipGetLastError();
}

hipError_t launch_fill_trivial(tor_result_t* out, const int32_t* idx, const int32_t* tiers,
                               int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_trivial_kernel, dim3((count + 63) / 64), dim3(64), 0, s, out, idx, tiers,
                     count);
  return hipGetLastError();
}

hipError_t launch_expand_terms(int tier, const void* partials, int nitems, double* out4,
                               hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g((nitems + 255) / 256), b(256);
  if (tier == TOR_QD)
    hipLaunchKernelGGL(expand_terms_kernel<qd>, g, b, 0, s, (const qd*)partials, nitems, out4);
  else
    hipLaunchKernelGGL(expand_terms_kernel<dd>, g, b, 0, s, (const dd*)partials, nitems, out4);
  return hipGetLastError();
}

}  // namespace tor
