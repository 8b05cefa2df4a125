/*
 * tor_oracle.c -- float128 CPU oracle for the Torontonian.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the library's product path never
 * does, and the two share no code, headers or tables.
 *
 * What it computes is the plain definition (Sec. 3.1, Eq. 2):
 *
 *     Tor(O) = sum over Z subset of {0..n-1} of (-1)^(n-|Z|) / sqrt(det(I - O_Z))
 *
 * where O_Z keeps rows/columns i and i+n for every i in Z, in block order
 * (the rule Eq. 1 uses for A_{S}).  Per subset the oracle follows the
 * per-mask steps of Alg. 1 in the paper's order: build the submatrix,
 * factor it, take 1/sqrt(det), add the signed term -- with no partitioning,
 * no reuse between subsets and no reordering of the matrix.
 *
 * Readings of the paper taken here:
 *   - The empty set is a term: det of an empty matrix is 1, so it adds
 *     (-1)^n.  (Eq. 2 sums over the whole power set.)
 *   - det(I - O_Z) > 0 for a valid input (I - O = sigma_Q^{-1} is Hermitian
 *     positive definite, hence every principal submatrix is), so |det| is det;
 *     a non-positive or NaN pivot is reported as an error, never abs()'d.
 *   - The lower triangle of the block-ordered submatrix is read; the input
 *     must be exactly Hermitian.
 *
 * Arithmetic: every entry is widened exactly from binary64 to binary128
 * (__float128, 113-bit significand); the Hermitian Cholesky factorisation
 * (lower, no pivoting) runs in binary128; det is the product of the squared
 * pivots; the signed terms, their absolute values and the per-level sums are
 * accumulated with Neumaier's compensated summation in binary128.  Threads
 * take static contiguous mask ranges and their partial sums are combined in
 * thread-index order.
 *
 * Outputs are returned as non-overlapping 3-term binary64 expansions
 * (hi, mid, lo), which represent a binary128 value exactly.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 q_t;

#define TORO_OK 0
#define TORO_EINVAL (-1)
#define TORO_ENOTPD (-2)
#define TORO_ENOMEM (-4)

#define TORO_NMAX_FULL 26
#define TORO_NMAX 60

typedef struct {
  double tor[3];      /* Tor as a 3-term expansion of the binary128 result */
  double abs_sum[3];  /* sum of |term| */
  double min_det[3];  /* smallest det(I - O_Z) met */
  double max_term[3]; /* largest |term| met */
  int64_t bad_mask;   /* first mask (lowest) with a non-positive pivot, or -1 */
  int32_t status;     /* TORO_OK or TORO_ENOTPD */
  int32_t threads;    /* threads used */
} toro_result_t;

/* ---- binary128 helpers ------------------------------------------------- */

static void q_split3(q_t x, double out[3]) {
  double h = (double)x;
  q_t r = x - (q_t)h;
  double m = (double)r;
  double l = (double)(r - (q_t)m);
  out[0] = h;
  out[1] = m;
  out[2] = l;
}

/* Neumaier's improvement of Kahan summation: carries the rounding error of
 * every addition in a separate compensation term. */
typedef struct {
  q_t s, c;
} neum_t;

static inline void neum_add(neum_t* a, q_t x) {
  q_t t = a->s + x;
  if (fabsq(a->s) >= fabsq(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static inline q_t neum_val(const neum_t* a) { return a->s + a->c; }

static inline void neum_merge(neum_t* a, const neum_t* b) {
  neum_add(a, b->s);
  neum_add(a, b->c);
}

/* ---- one subset --------------------------------------------------------- */

/* det(I - O_Z) for the subset z, in binary128.
 * O: 2n x 2n complex128 (interleaved re, im), row-major, leading dimension
 * ld (in complex elements), block order.  Scratch: ar/ai of (2n)^2, idx of 2n.
 * Returns TORO_OK, or TORO_ENOTPD when a pivot is not > 0. */
static int subset_det(const double* O, int n, int64_t ld, uint64_t z, q_t* ar, q_t* ai,
                      int* idx, q_t* det_out) {
  int m = 0;
  for (int i = 0; i < n; ++i)
    if ((z >> i) & 1u) idx[m++] = i;
  for (int a = 0; a < m; ++a) idx[m + a] = idx[a] + n;
  const int s = 2 * m;

  /* A = I - O[idx, idx], lower triangle. */
  for (int i = 0; i < s; ++i) {
    for (int j = 0; j <= i; ++j) {
      const double* e = O + 2 * ((int64_t)idx[i] * ld + idx[j]);
      ar[i * s + j] = (i == j ? (q_t)1 : (q_t)0) - (q_t)e[0];
      ai[i * s + j] = -(q_t)e[1];
    }
  }

  /* Hermitian Cholesky A = L L^H, lower, column by column. */
  q_t det = 1;
  for (int j = 0; j < s; ++j) {
    q_t d = ar[j * s + j];
    for (int k = 0; k < j; ++k) d -= ar[j * s + k] * ar[j * s + k] + ai[j * s + k] * ai[j * s + k];
    if (!(d > 0)) return TORO_ENOTPD;
    det *= d;
    q_t ljj = sqrtq(d);
    ar[j * s + j] = ljj;
    ai[j * s + j] = 0;
    for (int i = j + 1; i < s; ++i) {
      /* L_ij = (A_ij - sum_k L_ik conj(L_jk)) / L_jj */
      q_t re = ar[i * s + j], im = ai[i * s + j];
      for (int k = 0; k < j; ++k) {
        q_t xr = ar[i * s + k], xi = ai[i * s + k];
        q_t yr = ar[j * s + k], yi = ai[j * s + k];
        re -= xr * yr + xi * yi;
        im -= xi * yr - xr * yi;
      }
      ar[i * s + j] = re / ljj;
      ai[i * s + j] = im / ljj;
    }
  }
  *det_out = det;
  return TORO_OK;
}

static inline int popcount64(uint64_t x) { return __builtin_popcountll(x); }

/* The signed term (-1)^(n-|Z|) det^(-1/2). */
static inline q_t signed_term(int n, uint64_t z, q_t det) {
  q_t t = (q_t)1 / sqrtq(det);
  return ((n - popcount64(z)) & 1) ? -t : t;
}

static int valid_input(const double* O, int n, int64_t ld) {
  if (n < 0 || n > TORO_NMAX) return 0;
  if (n > 0 && (O == NULL || ld < 2 * n)) return 0;
  for (int i = 0; i < 2 * n; ++i)
    for (int j = 0; j < 2 * n; ++j) {
      const double* e = O + 2 * ((int64_t)i * ld + j);
      if (!isfinite(e[0]) || !isfinite(e[1])) return 0;
    }
  return 1;
}

/* ---- full sum ----------------------------------------------------------- */

/* Tor(O) over all 2^n subsets (n <= 26).  level_sums, if not NULL, receives
 * 3*(n+1) doubles: L_m = sum over |Z| = m of det^(-1/2) (unsigned). */
int toro_tor(const double* O, int n, int64_t ld, int threads, double* level_sums,
             toro_result_t* out) {
  if (out == NULL) return TORO_EINVAL;
  memset(out, 0, sizeof(*out));
  out->bad_mask = -1;
  if (!valid_input(O, n, ld) || n > TORO_NMAX_FULL) return TORO_EINVAL;
  if (threads <= 0) threads = omp_get_max_threads();
  const uint64_t total = (uint64_t)1 << n;
  if ((uint64_t)threads > total) threads = (int)total;

  neum_t* sums = (neum_t*)calloc((size_t)threads * (n + 3), sizeof(neum_t));
  q_t* mins = (q_t*)malloc(sizeof(q_t) * threads);
  q_t* maxs = (q_t*)malloc(sizeof(q_t) * threads);
  int64_t* bad = (int64_t*)malloc(sizeof(int64_t) * threads);
  if (!sums || !mins || !maxs || !bad) {
    free(sums); free(mins); free(maxs); free(bad);
    return TORO_ENOMEM;
  }

#pragma omp parallel num_threads(threads)
  {
    const int tid = omp_get_thread_num();
    const int nt = omp_get_num_threads();
    neum_t* my = sums + (size_t)tid * (n + 3); /* [0]=signed, [1]=abs, [2..]=levels */
    q_t mn = 1, mx = 0;
    int64_t my_bad = -1;
    const int s = 2 * (n > 0 ? n : 1);
    q_t* ar = (q_t*)malloc(sizeof(q_t) * s * s);
    q_t* ai = (q_t*)malloc(sizeof(q_t) * s * s);
    int* idx = (int*)malloc(sizeof(int) * s);
    const uint64_t lo = total * (uint64_t)tid / (uint64_t)nt;
    const uint64_t hi = total * (uint64_t)(tid + 1) / (uint64_t)nt;
    for (uint64_t z = lo; z < hi && ar && ai && idx; ++z) {
      q_t det;
      if (subset_det(O, n, ld, z, ar, ai, idx, &det) != TORO_OK) {
        if (my_bad < 0) my_bad = (int64_t)z;
        continue;
      }
      q_t t = signed_term(n, z, det);
      q_t at = fabsq(t);
      neum_add(&my[0], t);
      neum_add(&my[1], at);
      neum_add(&my[2 + popcount64(z)], at);
      if (det < mn) mn = det;
      if (at > mx) mx = at;
    }
    if (!ar || !ai || !idx) my_bad = -2;
    free(ar); free(ai); free(idx);
    mins[tid] = mn;
    maxs[tid] = mx;
    bad[tid] = my_bad;
  }

  neum_t tot[2 + TORO_NMAX_FULL + 1];
  memset(tot, 0, sizeof(tot));
  q_t mn = 1, mx = 0;
  int64_t first_bad = -1;
  int nomem = 0;
  for (int t = 0; t < threads; ++t) {
    for (int k = 0; k < n + 3; ++k) neum_merge(&tot[k], &sums[(size_t)t * (n + 3) + k]);
    if (mins[t] < mn) mn = mins[t];
    if (maxs[t] > mx) mx = maxs[t];
    if (bad[t] == -2) nomem = 1;
    else if (bad[t] >= 0 && first_bad < 0) first_bad = bad[t];
  }
  free(sums); free(mins); free(maxs); free(bad);
  if (nomem) return TORO_ENOMEM;

  q_split3(neum_val(&tot[0]), out->tor);
  q_split3(neum_val(&tot[1]), out->abs_sum);
  q_split3(mn, out->min_det);
  q_split3(mx, out->max_term);
  out->threads = threads;
  if (level_sums)
    for (int m = 0; m <= n; ++m) q_split3(neum_val(&tot[2 + m]), level_sums + 3 * m);
  out->bad_mask = first_bad;
  out->status = first_bad >= 0 ? TORO_ENOTPD : TORO_OK;
  return out->status;
}

/* ---- selected subsets --------------------------------------------------- */

/* det(I - O_Z) and the signed term for each of k caller-given masks, any
 * n <= 60.  det3/term3: 3*k doubles each (either may be NULL).  status, if
 * not NULL, receives k codes (TORO_OK / TORO_ENOTPD); a failed mask gets
 * det = term = 0.  Returns TORO_ENOTPD if any mask failed. */
int toro_terms(const double* O, int n, int64_t ld, const uint64_t* masks, int64_t k,
               int threads, double* det3, double* term3, int32_t* status) {
  if (!valid_input(O, n, ld) || (k > 0 && masks == NULL) || k < 0) return TORO_EINVAL;
  if (n < 64)
    for (int64_t i = 0; i < k; ++i)
      if (masks[i] >> n) return TORO_EINVAL;
  if (threads <= 0) threads = omp_get_max_threads();
  int any_bad = 0, nomem = 0;
#pragma omp parallel num_threads(threads) reduction(| : any_bad, nomem)
  {
    const int s = 2 * (n > 0 ? n : 1);
    q_t* ar = (q_t*)malloc(sizeof(q_t) * s * s);
    q_t* ai = (q_t*)malloc(sizeof(q_t) * s * s);
    int* idx = (int*)malloc(sizeof(int) * s);
    if (!ar || !ai || !idx) nomem = 1;
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < k; ++i) {
      if (nomem) continue;
      q_t det = 0, t = 0;
      int st = subset_det(O, n, ld, masks[i], ar, ai, idx, &det);
      if (st == TORO_OK) t = signed_term(n, masks[i], det);
      else { det = 0; any_bad = 1; }
      if (det3) q_split3(det, det3 + 3 * i);
      if (term3) q_split3(t, term3 + 3 * i);
      if (status) status[i] = st;
    }
    free(ar); free(ai); free(idx);
  }
  if (nomem) return TORO_ENOMEM;
  return any_bad ? TORO_ENOTPD : TORO_OK;
}

/* ---- sums over whole levels -------------------------------------------- */

/* L_m = sum over |Z| = m of det^(-1/2) (unsigned), for each requested level
 * m, any n <= 60 (the caller bounds the cost: C(n, m) subsets of size 2m).
 * out3: 3*nlev doubles. */
int toro_level_sums(const double* O, int n, int64_t ld, const int32_t* levels, int nlev,
                    int threads, double* out3) {
  if (!valid_input(O, n, ld) || nlev < 0 || (nlev > 0 && (!levels || !out3))) return TORO_EINVAL;
  if (threads <= 0) threads = omp_get_max_threads();
  for (int li = 0; li < nlev; ++li) {
    const int m = levels[li];
    if (m < 0 || m > n) return TORO_EINVAL;
    /* Count and list the masks of popcount m in increasing order
     * (next combination: lowest set bit moved up, the rest packed low). */
    double cnt_d = 1;
    for (int i = 0; i < m; ++i) cnt_d = cnt_d * (n - i) / (i + 1);
    if (cnt_d > 5e7) return TORO_EINVAL;
    const int64_t cnt = (int64_t)(cnt_d + 0.5);
    uint64_t* masks = (uint64_t*)malloc(sizeof(uint64_t) * (cnt > 0 ? cnt : 1));
    if (!masks) return TORO_ENOMEM;
    uint64_t z = (m == 0) ? 0 : (((uint64_t)1 << m) - 1);
    for (int64_t c = 0; c < cnt; ++c) {
      masks[c] = z;
      if (z == 0) break;
      uint64_t low = z & (~z + 1);
      uint64_t rip = z + low;
      z = rip | (((z ^ rip) >> 2) / low);
    }
    neum_t* part = (neum_t*)calloc((size_t)threads, sizeof(neum_t));
    int bad = 0, nomem = 0;
    if (!part) { free(masks); return TORO_ENOMEM; }
#pragma omp parallel num_threads(threads) reduction(| : bad, nomem)
    {
      const int tid = omp_get_thread_num();
      const int nt = omp_get_num_threads();
      const int s = 2 * (n > 0 ? n : 1);
      q_t* ar = (q_t*)malloc(sizeof(q_t) * s * s);
      q_t* ai = (q_t*)malloc(sizeof(q_t) * s * s);
      int* idx = (int*)malloc(sizeof(int) * s);
      if (!ar || !ai || !idx) nomem = 1;
      const int64_t lo = cnt * tid / nt, hi = cnt * (tid + 1) / nt;
      for (int64_t c = lo; c < hi && !nomem; ++c) {
        q_t det;
        if (subset_det(O, n, ld, masks[c], ar, ai, idx, &det) != TORO_OK) { bad = 1; continue; }
        neum_add(&part[tid], (q_t)1 / sqrtq(det));
      }
      free(ar); free(ai); free(idx);
    }
    neum_t tot = {0, 0};
    for (int t = 0; t < threads; ++t) neum_merge(&tot, &part[t]);
    free(part);
    free(masks);
    if (nomem) return TORO_ENOMEM;
    if (bad) return TORO_ENOTPD;
    q_split3(neum_val(&tot), out3 + 3 * li);
  }
  return TORO_OK;
}

int toro_max_threads(void) { return omp_get_max_threads(); }
