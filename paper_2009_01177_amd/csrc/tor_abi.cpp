// tor_abi.cpp -- the C ABI (include/tor.h): argument checks, per-device
// workspace, work-item planning and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/tor.h"
#include "tor_host.h"
#include "tor_internal.hpp"

namespace tor {
namespace {

struct ItemTable {
  uint64_t* dev = nullptr;
  int count = 0;
};

struct Workspace {
  int device = -1;
  int cus = 0;
  size_t lds_per_block = 0;
  char* buf = nullptr;
  size_t cap = 0;
  tor_result_t* host_res = nullptr;  // pinned
  double* host_lev = nullptr;        // pinned, 4*(TOR_NMAX+1)
  std::map<std::pair<int, int>, ItemTable> tables;  // (n, d) -> prefix items
  std::vector<hipEvent_t> evs;  // kernel timing (TOR_FLAG_TIME_KERNEL): start/stop pairs
  int ev_pairs = 0;             // pairs recorded by the last evaluation
  double last_ms = -1.0;
  int last_d = -1, last_grid = -1, last_launches = 0;
};

std::mutex g_mu;
std::map<int, Workspace*> g_ws;

inline int hip_err(hipError_t e) { return e == hipSuccess ? TOR_OK : (e == hipErrorOutOfMemory ? TOR_ENOMEM : TOR_EHIP); }

#define TOR_TRY(expr)                   \
  do {                                  \
    int rc__ = (expr);                  \
    if (rc__ != TOR_OK) return rc__;    \
  } while (0)
#define TOR_HIP(expr) TOR_TRY(hip_err(expr))

// Record the start (k even) or stop (k odd) event of timed launch k/2.
int record_ev(Workspace* w, int k, hipStream_t s) {
  while ((int)w->evs.size() <= k) {
    hipEvent_t e;
    TOR_HIP(hipEventCreate(&e));
    w->evs.push_back(e);
  }
  TOR_HIP(hipEventRecord(w->evs[k], s));
  return TOR_OK;
}

// Sum the recorded launch durations (after the stream has synchronised).
int collect_ev(Workspace* w) {
  double tot = 0.0;
  for (int p = 0; p < w->ev_pairs; ++p) {
    float ms = 0.0f;
    TOR_HIP(hipEventElapsedTime(&ms, w->evs[2 * p], w->evs[2 * p + 1]));
    tot += ms;
  }
  w->last_ms = w->ev_pairs > 0 ? tot : -1.0;
  w->last_launches = w->ev_pairs;
  w->ev_pairs = 0;
  return TOR_OK;
}


int get_ws(Workspace** out) {
  int dev = 0;
  TOR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) {
    *out = it->second;
    return TOR_OK;
  }
  Workspace* w = new Workspace();
  w->device = dev;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    delete w;
    return hip_err(e);
  }
  w->cus = prop.multiProcessorCount;
  w->lds_per_block = prop.sharedMemPerBlock;
  e = hipHostMalloc((void**)&w->host_res, sizeof(tor_result_t), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&w->host_lev, sizeof(double) * 4 * (TOR_NMAX + 1) * 2, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (w->host_res) (void)hipHostFree(w->host_res);
    delete w;
    return hip_err(e);
  }
  g_ws[dev] = w;
  *out = w;
  return TOR_OK;
}

int ensure_cap(Workspace* w, size_t bytes) {
  if (bytes <= w->cap) return TOR_OK;
  size_t ncap = w->cap ? w->cap : (size_t)1 << 20;
  while (ncap < bytes) ncap *= 2;
  if (w->buf) {
    // the old buffer may still be in use by enqueued work
    TOR_HIP(hipDeviceSynchronize());
    TOR_HIP(hipFree(w->buf));
    w->buf = nullptr;
    w->cap = 0;
  }
  TOR_HIP(hipMalloc((void**)&w->buf, ncap));
  w->cap = ncap;
  return TOR_OK;
}

// Carve aligned slices out of the workspace buffer.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    size_t o = off;
    off += bytes;
    return o;
  }
};

int get_items(Workspace* w, int n, int d, ItemTable** out) {
  auto key = std::make_pair(n, d);
  auto it = w->tables.find(key);
  if (it != w->tables.end()) {
    *out = &it->second;
    return TOR_OK;
  }
  std::vector<uint64_t> items((size_t)1 << d);
  if (tor_plan_items(n, d, items.data()) != TOR_OK) return TOR_EINVAL;
  ItemTable t;
  t.count = (int)items.size();
  TOR_HIP(hipMalloc((void**)&t.dev, sizeof(uint64_t) * items.size()));
  TOR_HIP(hipMemcpy(t.dev, items.data(), sizeof(uint64_t) * items.size(), hipMemcpyHostToDevice));
  auto res = w->tables.emplace(key, t);
  *out = &res.first->second;
  return TOR_OK;
}

double unit_roundoff(int tier) {
  if (tier == TOR_FP64) return ldexp(1.0, -53);
  if (tier == TOR_DD) return ldexp(1.0, -104);
  return ldexp(1.0, -208);
}

int check_common(const void* O, int32_t n, int64_t ld, int32_t tier) {
  if (n < 0 || n > TOR_NMAX) return TOR_EINVAL;
  if (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD) return TOR_EINVAL;
  if (n > 0 && (O == nullptr || ld < 2 * (int64_t)n)) return TOR_EINVAL;
  return TOR_OK;
}

int fits_border(Workspace* w, int tier, int mode, int n) {
  const size_t lds = border_lds_bytes(tier, mode, n);
  if (lds > w->lds_per_block) return TOR_EUNSUPPORTED;
  return TOR_OK;
}

// Split depth: enough items to keep every resident wave busy with a
// largest-first queue, but subtrees of at least 8 subsets so the prefix
// factor is amortised.
int auto_split(int n, int resident) {
  const int target = resident * 8;
  int d = 0;
  while ((1 << d) < target && d < 24) ++d;
  int dmax = n > 3 ? n - 3 : 0;
  if (d > dmax) d = dmax;
  return d;
}

void fill_trivial(tor_result_t* out, int tier) {
  memset(out, 0, sizeof(*out));
  out->tor[0] = 1.0;
  out->abs_sum[0] = 1.0;
  out->tier_used = tier;
  out->status = TOR_OK;
}

struct RunOut {
  tor_result_t* dres;
  void* red;
  int ncols;
};

// Enqueue one subset-tree evaluation: stage, zero counters, kernel,
// reduction, finalize.  Device result in *ro.
int enqueue_tree(Workspace* w, const void* O, int n, int64_t ld, int tier, int mode,
                 const tor_options_t* opt, hipStream_t s, RunOut* ro) {
  TOR_TRY(fits_border(w, tier, mode, n));
  int occ = 0;
  TOR_HIP(border_occupancy(tier, mode, n, &occ));
  if (occ < 1) return TOR_EUNSUPPORTED;
  const int resident = occ * w->cus;
  int d = (opt && opt->split_depth >= 0) ? opt->split_depth : auto_split(n, resident);
  if (d > n) d = n;
  if (d > 30) return TOR_EINVAL;
  ItemTable* items = nullptr;
  TOR_TRY(get_items(w, n, d, &items));
  const int nitems = items->count;
  const int ncols = (mode == MODE_LEVELS) ? 2 + n + 1 : 2;
  const size_t ab = acc_bytes(tier);

  Carver c;
  const size_t o_oi = c.take(sizeof(double2) * 4 * (size_t)n * n);
  const size_t o_part = c.take(ab * (size_t)nitems * ncols);
  const size_t o_red = c.take(ab * (size_t)ncols);
  const size_t o_rsc = c.take(reduce_scratch_bytes(tier, nitems, ncols));
  const size_t o_cnt = c.take(sizeof(uint32_t) * 64);
  const size_t o_res = c.take(sizeof(tor_result_t));
  TOR_TRY(ensure_cap(w, c.off));

  double2* Oi = (double2*)(w->buf + o_oi);
  uint32_t* cnt = (uint32_t*)(w->buf + o_cnt);  // [0] queue, [1] status
  TOR_HIP(launch_stage((const double2*)O, n, ld, Oi, s));
  TOR_HIP(launch_zero_words(cnt, 64, s));
  BorderLaunch bl;
  bl.tier = tier;
  bl.mode = mode;
  bl.n = n;
  bl.d = d;
  bl.nitems = nitems;
  int grid = (opt && opt->grid > 0) ? opt->grid : resident;
  if (grid > nitems) grid = nitems;
  bl.grid = grid;
  bl.Oi = Oi;
  bl.items = items->dev;
  bl.queue = cnt;
  bl.partials = w->buf + o_part;
  bl.status = (int32_t*)(cnt + 1);
  const bool timed = opt && (opt->flags & TOR_FLAG_TIME_KERNEL);
  w->ev_pairs = 0;
  if (timed) TOR_TRY(record_ev(w, 0, s));
  TOR_HIP(launch_border(bl, s));
  if (timed) {
    TOR_TRY(record_ev(w, 1, s));
    w->ev_pairs = 1;
  }
  w->last_d = d;
  w->last_grid = grid;
  TOR_HIP(launch_reduce_cols(tier, w->buf + o_part, nitems, ncols, w->buf + o_red, w->buf + o_rsc, s));
  const double err_rel = (double)(4 * n * n + d + 8) * unit_roundoff(tier);
  TOR_HIP(launch_finalize(tier, w->buf + o_red, (const int32_t*)(cnt + 1), err_rel,
                          (tor_result_t*)(w->buf + o_res), s));
  ro->dres = (tor_result_t*)(w->buf + o_res);
  ro->red = w->buf + o_red;
  ro->ncols = ncols;
  return TOR_OK;
}


// Right-looking Schur-complement evaluation (MODE_SUM only).
//   depth 0 -> D_s : breadth-first in HBM, all states kept ("roots")
//   per chunk      : Cr consecutive roots expanded breadth-first to depth
//                    D_m = n - s_m, then the middle + bottom kernel over the
//                    Cr 2^(D_m - D_s) middle states
// A chunk's last top level is kept near 1.5 GB.
int enqueue_schur(Workspace* w, const void* O, int n, int64_t ld, int tier,
                  const tor_options_t* opt, hipStream_t s, RunOut* ro) {
  int s_m = 0, s_b = 0;
  schur_levels(tier, n, opt ? opt->bottom_modes : 0, &s_m, &s_b);
  const int D_m = n - s_m;
  const size_t rb = schur_value_bytes(tier);
  const size_t ab = acc_bytes(tier);
  auto ps = [](int k) { return (size_t)k * (2 * k + 1); };
  // middle states per chunk: about 1.5 GB of them at the last top level
  int LT = 0;
  while (LT < 22 && ((size_t)2 << LT) * ps(s_m) * rb <= ((size_t)3 << 29)) ++LT;
  // stage 0 keeps every state of depth D_s; a chunk expands Cr of them
  int D_s = D_m < 10 ? D_m : 10;
  if (D_m - D_s > LT) D_s = D_m - LT;
  const int Dl = D_m - D_s;  // levels expanded per chunk
  const int lcr = std::min(D_s, LT - Dl);
  const int Cr = 1 << lcr;             // roots per chunk
  const int nchunks = 1 << (D_s - lcr);
  const int D_c = D_s;

  size_t lvl_vals = ps(n);
  for (int j = 1; j <= D_s; ++j) lvl_vals = std::max(lvl_vals, ((size_t)1 << j) * ps(n - j));
  for (int j = 1; j <= Dl; ++j) lvl_vals = std::max(lvl_vals, ((size_t)Cr << j) * ps(n - D_s - j));
  const size_t lvl_states = std::max((size_t)1 << D_s, (size_t)Cr << Dl);
  const size_t mids = (size_t)Cr << Dl;

  Carver c;
  const size_t o_rm = c.take(rb * (((size_t)1 << D_s) * ps(n - D_s)));
  const size_t o_rg = c.take(rb * ((size_t)1 << D_s));
  const size_t o_rn = c.take(sizeof(int32_t) * ((size_t)1 << D_s));
  size_t o_m[2], o_g[2], o_n[2];
  for (int k = 0; k < 2; ++k) {
    o_m[k] = c.take(rb * lvl_vals);
    o_g[k] = c.take(rb * lvl_states);
    o_n[k] = c.take(sizeof(int32_t) * lvl_states);
  }
  const size_t o_part = c.take(ab * 2 * mids);
  const size_t o_chunk = c.take(ab * 2 * (size_t)nchunks);
  const size_t o_red = c.take(ab * 2);
  const size_t o_rsc = c.take(std::max(reduce_scratch_bytes(tier, (int)mids, 2),
                                       reduce_scratch_bytes(tier, nchunks, 2)));
  const size_t o_cnt = c.take(sizeof(uint32_t) * 64);
  const size_t o_res = c.take(sizeof(tor_result_t));
  TOR_TRY(ensure_cap(w, c.off));
  char* B = w->buf;
  uint32_t* cnt = (uint32_t*)(B + o_cnt);
  int32_t* status = (int32_t*)(cnt + 1);

  int occ = 0;
  TOR_HIP(leaf_occupancy(tier, s_b, &occ));
  if (occ < 1) return TOR_EUNSUPPORTED;
  int grid = (opt && opt->grid > 0) ? opt->grid : occ * w->cus;
  if ((size_t)grid > mids) grid = (int)mids;

  TOR_HIP(launch_zero_words(cnt, 64, s));
  const bool timed = opt && (opt->flags & TOR_FLAG_TIME_KERNEL);
  w->ev_pairs = 0;
  // stage 0: root, then breadth-first to depth D_c into the roots buffer
  {
    int cur = 0;
    void* dm = D_c == 0 ? (void*)(B + o_rm) : (void*)(B + o_m[0]);
    void* dg = D_c == 0 ? (void*)(B + o_rg) : (void*)(B + o_g[0]);
    int32_t* dn = D_c == 0 ? (int32_t*)(B + o_rn) : (int32_t*)(B + o_n[0]);
    TOR_HIP(launch_real_root(tier, (const double2*)O, n, ld, dm, dg, dn, s));
    for (int j = 0; j < D_c; ++j) {
      const bool last = (j == D_c - 1);
      void* om = last ? (void*)(B + o_rm) : (void*)(B + o_m[1 - cur]);
      void* og = last ? (void*)(B + o_rg) : (void*)(B + o_g[1 - cur]);
      int32_t* on = last ? (int32_t*)(B + o_rn) : (int32_t*)(B + o_n[1 - cur]);
      TOR_HIP(launch_expand(tier, B + o_m[cur], B + o_g[cur], (const int32_t*)(B + o_n[cur]), n - j,
                            1 << j, om, og, on, status, s));
      cur = 1 - cur;
    }
  }
  // per chunk of Cr roots: expand Dl levels, then the middle + bottom kernel
  for (int ch = 0; ch < nchunks; ++ch) {
    const char* im = B + o_rm + rb * ((size_t)ch * Cr * ps(n - D_c));
    const char* ig = B + o_rg + rb * ((size_t)ch * Cr);
    const int32_t* in_ = (const int32_t*)(B + o_rn) + (size_t)ch * Cr;
    int cur = -1;  // -1: the chunk's roots themselves
    for (int j = 0; j < Dl; ++j) {
      const int nx = (cur == 0) ? 1 : 0;
      TOR_HIP(launch_expand(tier, cur < 0 ? (const void*)im : (const void*)(B + o_m[cur]),
                            cur < 0 ? (const void*)ig : (const void*)(B + o_g[cur]),
                            cur < 0 ? in_ : (const int32_t*)(B + o_n[cur]), n - D_c - j, Cr << j,
                            B + o_m[nx], B + o_g[nx], (int32_t*)(B + o_n[nx]), status, s));
      cur = nx;
    }
    const void* lm = cur < 0 ? (const void*)im : (const void*)(B + o_m[cur]);
    const void* lg = cur < 0 ? (const void*)ig : (const void*)(B + o_g[cur]);
    const int32_t* ln = cur < 0 ? in_ : (const int32_t*)(B + o_n[cur]);
    if (timed) TOR_TRY(record_ev(w, 2 * ch, s));
    TOR_HIP(launch_leaf(tier, s_m, s_b, lm, lg, ln, (int)mids, n, B + o_part, status, grid, s));
    if (timed) {
      TOR_TRY(record_ev(w, 2 * ch + 1, s));
      w->ev_pairs = ch + 1;
    }
    TOR_HIP(launch_reduce_cols(tier, B + o_part, (int)mids, 2, B + o_chunk + ab * 2 * ch, B + o_rsc, s));
  }
  w->last_d = D_m;
  w->last_grid = grid;
  TOR_HIP(launch_reduce_cols(tier, B + o_chunk, nchunks, 2, B + o_red, B + o_rsc, s));
  const double err_rel = (double)(4 * n * n + n + 8) * unit_roundoff(tier);
  TOR_HIP(launch_finalize(tier, B + o_red, status, err_rel, (tor_result_t*)(B + o_res), s));
  ro->dres = (tor_result_t*)(B + o_res);
  ro->red = B + o_red;
  ro->ncols = 2;
  return TOR_OK;
}

}  // namespace
}  // namespace tor

using namespace tor;

extern "C" {

const char* tor_version(void) { return "tor-mi355x 0.1 (gfx950)"; }

const char* tor_strerror(int code) {
  switch (code) {
    case TOR_OK: return "ok";
    case TOR_EINVAL: return "invalid argument";
    case TOR_ENOTPD: return "I - O is not positive definite (a pivot was not > 0)";
    case TOR_EHIP: return "HIP runtime error";
    case TOR_ENOMEM: return "device allocation failed";
    case TOR_EUNSUPPORTED: return "tier and n do not fit the kernel's storage plan";
    default: return "unknown error";
  }
}

int tor_init(void) {
  Workspace* w = nullptr;
  return get_ws(&w);
}

int tor_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = TOR_OK;
  for (auto& kv : g_ws) {
    Workspace* w = kv.second;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(w->device) == hipSuccess) {
      if (hipDeviceSynchronize() != hipSuccess) rc = TOR_EHIP;
      for (auto& t : w->tables) (void)hipFree(t.second.dev);
      if (w->buf) (void)hipFree(w->buf);
      if (w->host_res) (void)hipHostFree(w->host_res);
      if (w->host_lev) (void)hipHostFree(w->host_lev);
      for (hipEvent_t e : w->evs) (void)hipEventDestroy(e);
      (void)hipSetDevice(cur);
    }
    delete w;
  }
  g_ws.clear();
  return rc;
}

int tor_eval(const void* O, int32_t n, int64_t ld, int32_t tier, const tor_options_t* opt,
             void* stream, tor_result_t* out) {
  if (out == nullptr) return TOR_EINVAL;
  TOR_TRY(check_common(O, n, ld, tier));
  if (n == 0) {
    fill_trivial(out, tier);
    return TOR_OK;
  }
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  RunOut ro;
  const int algo = opt ? opt->algo : TOR_ALGO_AUTO;
  if (algo != TOR_ALGO_AUTO && algo != TOR_ALGO_BORDER && algo != TOR_ALGO_SCHUR) return TOR_EINVAL;
  if (algo == TOR_ALGO_BORDER)
    TOR_TRY(enqueue_tree(w, O, n, ld, tier, MODE_SUM, opt, s, &ro));
  else
    TOR_TRY(enqueue_schur(w, O, n, ld, tier, opt, s, &ro));
  TOR_HIP(hipMemcpyAsync(w->host_res, ro.dres, sizeof(tor_result_t), hipMemcpyDeviceToHost, s));
  TOR_HIP(hipStreamSynchronize(s));
  if (w->ev_pairs > 0) TOR_TRY(collect_ev(w));
  *out = *w->host_res;
  return out->status;
}

double tor_last_kernel_ms(int32_t* split_depth, int32_t* grid, int32_t* launches) {
  Workspace* w = nullptr;
  if (get_ws(&w) != TOR_OK) return -1.0;
  if (split_depth) *split_depth = w->last_d;
  if (grid) *grid = w->last_grid;
  if (launches) *launches = w->last_launches;
  return w->last_ms;
}

int tor_debug_level_sums(const void* O, int32_t n, int64_t ld, int32_t tier, void* stream,
                         double* out_levels, tor_result_t* out) {
  if (out == nullptr || out_levels == nullptr) return TOR_EINVAL;
  TOR_TRY(check_common(O, n, ld, tier));
  if (n == 0) {
    fill_trivial(out, tier);
    out_levels[0] = 1.0;
    out_levels[1] = out_levels[2] = out_levels[3] = 0.0;
    return TOR_OK;
  }
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  RunOut ro;
  TOR_TRY(enqueue_tree(w, O, n, ld, tier, MODE_LEVELS, nullptr, s, &ro));
  const size_t ab = acc_bytes(tier);
  TOR_HIP(hipMemcpyAsync(w->host_res, ro.dres, sizeof(tor_result_t), hipMemcpyDeviceToHost, s));
  TOR_HIP(hipMemcpyAsync(w->host_lev, (char*)ro.red + 2 * ab, ab * (n + 1), hipMemcpyDeviceToHost, s));
  TOR_HIP(hipStreamSynchronize(s));
  *out = *w->host_res;
  const int per = (int)(ab / sizeof(double));
  for (int m = 0; m <= n; ++m)
    for (int k = 0; k < 4; ++k) out_levels[4 * m + k] = k < per ? w->host_lev[per * m + k] : 0.0;
  return out->status;
}

int tor_debug_sampled_terms(const void* O, int32_t n, int64_t ld, int32_t tier,
                            const uint64_t* masks, int64_t k, void* stream, double* out_terms) {
  TOR_TRY(check_common(O, n, ld, tier));
  if (k < 0 || k > (int64_t)1 << 30) return TOR_EINVAL;
  if (k == 0) return TOR_OK;
  if (masks == nullptr || out_terms == nullptr) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  const int mode = MODE_MASKS;
  const int nn = n > 0 ? n : 1;
  TOR_TRY(fits_border(w, tier, mode, nn));
  int occ = 0;
  TOR_HIP(border_occupancy(tier, mode, nn, &occ));
  if (occ < 1) return TOR_EUNSUPPORTED;
  const size_t ab = acc_bytes(tier);
  Carver c;
  const size_t o_oi = c.take(sizeof(double2) * 4 * (size_t)nn * nn);
  const size_t o_part = c.take(ab * (size_t)k * 2);
  const size_t o_cnt = c.take(sizeof(uint32_t) * 64);
  TOR_TRY(ensure_cap(w, c.off));
  double2* Oi = (double2*)(w->buf + o_oi);
  uint32_t* cnt = (uint32_t*)(w->buf + o_cnt);
  if (n == 0) {
    // the only subset is the empty one: term 1
    std::vector<double> one((size_t)4 * k, 0.0);
    for (int64_t i = 0; i < k; ++i) one[4 * i] = 1.0;
    TOR_HIP(hipMemcpyAsync(out_terms, one.data(), sizeof(double) * one.size(), hipMemcpyHostToDevice, s));
    TOR_HIP(hipStreamSynchronize(s));
    return TOR_OK;
  }
  TOR_HIP(launch_stage((const double2*)O, n, ld, Oi, s));
  TOR_HIP(launch_zero_words(cnt, 64, s));
  BorderLaunch bl;
  bl.tier = tier;
  bl.mode = mode;
  bl.n = n;
  bl.d = n;
  bl.nitems = (int)k;
  int grid = occ * w->cus;
  if (grid > k) grid = (int)k;
  bl.grid = grid;
  bl.Oi = Oi;
  bl.items = masks;
  bl.queue = cnt;
  bl.partials = w->buf + o_part;
  bl.status = (int32_t*)(cnt + 1);
  TOR_HIP(launch_border(bl, s));
  TOR_HIP(launch_expand_terms(tier, w->buf + o_part, (int)k, out_terms, s));
  return TOR_OK;
}

}  // extern "C"
