// tor_abi.cpp -- the C ABI (include/tor.h): argument checks, per-device
// workspace, work-item planning and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
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
  char* meta = nullptr;         // device copy of the batch plan (offsets, indices, tiers)
  size_t meta_cap = 0;
  std::map<std::string, hipGraphExec_t> graphs;  // captured batches (TOR_FLAG_GRAPH)
  hipStream_t cap_stream = nullptr;              // private stream graphs are captured on
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
  // captured graphs point into the old buffer
  for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
  w->graphs.clear();
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


// ---------------------------------------------------------------------------
// Right-looking Schur-complement evaluation of a group of R instances that
// share n and the tier (MODE_SUM only).
//   depth 0 -> D_s : breadth-first in HBM over all R roots, every state kept
//   per chunk      : Cr consecutive depth-D_s states expanded breadth-first to
//                    depth D_m = n - s_m, then the middle + bottom kernel over
//                    Cr 2^(D_m - D_s) middle states, their partial sums folded
//                    per depth-D_s state
//   end            : partial sums folded per instance; one result each
// Every fold has a fixed order, so results do not depend on launch shapes.
// ---------------------------------------------------------------------------
struct SchurPlan {
  int tier, n, R, s_m, s_b, D_m, D_s, Dl, Cr, nchunks;
  size_t Ns, mids, rb, ab;
  size_t o_rm, o_rg, o_rn, o_m[2], o_g[2], o_n[2], o_part, o_ds, o_inst, o_rsc, o_cnt, o_res;
  size_t bytes;
};

size_t psz(int k) { return (size_t)k * (2 * k + 1); }

void plan_schur(int tier, int n, int R, int sb_req, SchurPlan* p) {
  p->tier = tier;
  p->n = n;
  p->R = R;
  schur_levels(tier, n, sb_req, &p->s_m, &p->s_b);
  p->D_m = n - p->s_m;
  p->rb = schur_value_bytes(tier);
  p->ab = acc_bytes(tier);
  // middle states per chunk: about 1.5 GB of them at the last top level
  int LT = 0;
  while (LT < 22 && ((size_t)2 << LT) * psz(p->s_m) * p->rb <= ((size_t)3 << 29)) ++LT;
  // keep depth D_s (at most 10, at most ~1 GB of states, at least D_m - LT)
  int D_s = p->D_m < 10 ? p->D_m : 10;
  while (D_s > 0 && ((size_t)R << D_s) * psz(n - D_s) * p->rb > ((size_t)1 << 30)) --D_s;
  if (p->D_m - D_s > LT) D_s = p->D_m - LT;
  p->D_s = D_s;
  p->Dl = p->D_m - D_s;
  p->Ns = (size_t)R << D_s;
  size_t cr = p->Dl >= LT ? 1 : ((size_t)1 << (LT - p->Dl));
  if (cr > p->Ns) cr = p->Ns;
  p->Cr = (int)cr;
  p->nchunks = (int)((p->Ns + cr - 1) / cr);
  p->mids = cr << p->Dl;

  size_t lvl_vals = (size_t)R * psz(n);
  for (int j = 1; j <= D_s; ++j) lvl_vals = std::max(lvl_vals, ((size_t)R << j) * psz(n - j));
  for (int j = 1; j <= p->Dl; ++j) lvl_vals = std::max(lvl_vals, (cr << j) * psz(n - D_s - j));
  const size_t lvl_states = std::max(p->Ns, p->mids);

  Carver c;
  p->o_rm = c.take(p->rb * (p->Ns * psz(n - D_s)));
  p->o_rg = c.take(p->rb * p->Ns);
  p->o_rn = c.take(sizeof(int32_t) * p->Ns);
  for (int k = 0; k < 2; ++k) {
    p->o_m[k] = c.take(p->rb * lvl_vals);
    p->o_g[k] = c.take(p->rb * lvl_states);
    p->o_n[k] = c.take(sizeof(int32_t) * lvl_states);
  }
  p->o_part = c.take(p->ab * 2 * p->mids);
  p->o_ds = c.take(p->ab * 2 * p->Ns);
  p->o_inst = c.take(p->ab * 2 * (size_t)R);
  p->o_rsc = c.take(reduce_scratch_bytes(tier, (int)std::max(p->mids, p->Ns), 2));
  p->o_cnt = c.take(sizeof(uint32_t) * 64);
  p->o_res = c.take(sizeof(tor_result_t));
  p->bytes = c.off;
}

// Fold nseg segments of seg_len partials each (a two-stage reduction when one
// long segment is all there is).
int fold(int tier, const void* part, int nseg, size_t seg_len, void* out, void* scratch, hipStream_t s) {
  if (nseg == 1 && seg_len > 4096)
    return hip_err(launch_reduce_cols(tier, part, (int)seg_len, 2, out, scratch, s));
  return hip_err(launch_seg_reduce(tier, part, nseg, (int)seg_len, out, s));
}

// Enqueue a planned group.  O + offs_dev[k] (offs_dev NULL: O itself) is
// instance k; results go to out[out_index ? out_index[k] : k] (device).
int enqueue_schur_group(Workspace* w, const SchurPlan& p, const void* O, const int64_t* offs_dev,
                        int64_t ld, const tor_options_t* opt, const int32_t* out_index,
                        tor_result_t* out, bool timed, hipStream_t s) {
  const int tier = p.tier, n = p.n;
  char* B = w->buf;
  uint32_t* cnt = (uint32_t*)(B + p.o_cnt);
  int32_t* status = (int32_t*)(cnt + 1);
  int occ = 0;
  TOR_HIP(leaf_occupancy(tier, p.s_b, &occ));
  if (occ < 1) return TOR_EUNSUPPORTED;
  int grid = (opt && opt->grid > 0) ? opt->grid : occ * w->cus;
  if ((size_t)grid > p.mids) grid = (int)p.mids;

  TOR_HIP(launch_zero_words(cnt, 64, s));
  // stage 0: roots, then breadth-first to depth D_s into the kept buffer
  {
    int cur = 0;
    const bool direct = (p.D_s == 0);
    void* dm = direct ? (void*)(B + p.o_rm) : (void*)(B + p.o_m[0]);
    void* dg = direct ? (void*)(B + p.o_rg) : (void*)(B + p.o_g[0]);
    int32_t* dn = direct ? (int32_t*)(B + p.o_rn) : (int32_t*)(B + p.o_n[0]);
    TOR_HIP(launch_real_root(tier, (const double2*)O, offs_dev, p.R, n, ld, dm, dg, dn, s));
    for (int j = 0; j < p.D_s; ++j) {
      const bool last = (j == p.D_s - 1);
      void* om = last ? (void*)(B + p.o_rm) : (void*)(B + p.o_m[1 - cur]);
      void* og = last ? (void*)(B + p.o_rg) : (void*)(B + p.o_g[1 - cur]);
      int32_t* on = last ? (int32_t*)(B + p.o_rn) : (int32_t*)(B + p.o_n[1 - cur]);
      TOR_HIP(launch_expand(tier, B + p.o_m[cur], B + p.o_g[cur], (const int32_t*)(B + p.o_n[cur]),
                            n - j, p.R << j, om, og, on, status, s));
      cur = 1 - cur;
    }
  }
  const size_t rb = p.rb, ab = p.ab;
  for (int ch = 0; ch < p.nchunks; ++ch) {
    const size_t first = (size_t)ch * p.Cr;
    const int cr = (int)std::min<size_t>(p.Cr, p.Ns - first);
    const char* im = B + p.o_rm + rb * (first * psz(n - p.D_s));
    const char* ig = B + p.o_rg + rb * first;
    const int32_t* in_ = (const int32_t*)(B + p.o_rn) + first;
    int cur = -1;  // -1: the chunk's depth-D_s states themselves
    for (int j = 0; j < p.Dl; ++j) {
      const int nx = (cur == 0) ? 1 : 0;
      TOR_HIP(launch_expand(tier, cur < 0 ? (const void*)im : (const void*)(B + p.o_m[cur]),
                            cur < 0 ? (const void*)ig : (const void*)(B + p.o_g[cur]),
                            cur < 0 ? in_ : (const int32_t*)(B + p.o_n[cur]), n - p.D_s - j, cr << j,
                            B + p.o_m[nx], B + p.o_g[nx], (int32_t*)(B + p.o_n[nx]), status, s));
      cur = nx;
    }
    const void* lm = cur < 0 ? (const void*)im : (const void*)(B + p.o_m[cur]);
    const void* lg = cur < 0 ? (const void*)ig : (const void*)(B + p.o_g[cur]);
    const int32_t* ln = cur < 0 ? in_ : (const int32_t*)(B + p.o_n[cur]);
    const int nm = cr << p.Dl;
    if (timed) TOR_TRY(record_ev(w, 2 * w->ev_pairs, s));
    TOR_HIP(launch_leaf(tier, p.s_m, p.s_b, lm, lg, ln, nm, n, B + p.o_part, status,
                        std::min(grid, nm), s));
    if (timed) {
      TOR_TRY(record_ev(w, 2 * w->ev_pairs + 1, s));
      w->ev_pairs += 1;
    }
    TOR_TRY(fold(tier, B + p.o_part, cr, (size_t)1 << p.Dl, B + p.o_ds + ab * 2 * first, B + p.o_rsc, s));
  }
  TOR_TRY(fold(tier, B + p.o_ds, p.R, (size_t)1 << p.D_s, B + p.o_inst, B + p.o_rsc, s));
  const double err_rel = (double)(4 * n * n + n + 8) * unit_roundoff(tier);
  TOR_HIP(launch_finalize_batch(tier, B + p.o_inst, p.R, out_index, n, err_rel, out, s));
  w->last_d = p.D_m;
  w->last_grid = grid;
  return TOR_OK;
}

// Precision selector: fills tier_of[k] for every TOR_AUTO instance with n > 0.
int select_tiers(Workspace* w, const void* O_packed, const int64_t* offsets, const int32_t* n,
                 int batch, double tau, int32_t* tier_of, hipStream_t s) {
  (void)w; (void)O_packed; (void)offsets; (void)n; (void)batch; (void)tau; (void)tier_of; (void)s;
  return TOR_EUNSUPPORTED;
}

// A batch grouped by (n, tier).
struct BatchGroup {
  int n, tier;
  std::vector<int32_t> idx;  // instance indices
};

int upload_meta(Workspace* w, const void* src, size_t bytes) {
  if (bytes > w->meta_cap) {
    if (w->meta) TOR_HIP(hipFree(w->meta));
    w->meta = nullptr;
    w->meta_cap = 0;
    size_t cap = 4096;
    while (cap < bytes) cap *= 2;
    TOR_HIP(hipMalloc((void**)&w->meta, cap));
    w->meta_cap = cap;
    for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    w->graphs.clear();
  }
  TOR_HIP(hipMemcpy(w->meta, src, bytes, hipMemcpyHostToDevice));
  return TOR_OK;
}

// Enqueue every group of a batch (plan already uploaded to w->meta).
int enqueue_batch(Workspace* w, const std::vector<BatchGroup>& groups,
                  const std::vector<SchurPlan>& plans, const std::vector<size_t>& meta_off,
                  size_t triv_off, int ntriv, const void* O_packed, const tor_options_t* opt,
                  tor_result_t* out, hipStream_t s) {
  if (ntriv > 0)
    TOR_HIP(launch_fill_trivial(out, (const int32_t*)(w->meta + triv_off),
                                (const int32_t*)(w->meta + triv_off) + ntriv, ntriv, s));
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const BatchGroup& g = groups[gi];
    const int64_t* offs = (const int64_t*)(w->meta + meta_off[gi]);
    const int32_t* oidx = (const int32_t*)(offs + g.idx.size());
    TOR_TRY(enqueue_schur_group(w, plans[gi], O_packed, offs, 2 * (int64_t)g.n, opt, oidx, out, false, s));
  }
  return TOR_OK;
}

// Single instance through the Schur path.
int enqueue_schur(Workspace* w, const void* O, int n, int64_t ld, int tier,
                  const tor_options_t* opt, hipStream_t s, RunOut* ro) {
  SchurPlan p;
  plan_schur(tier, n, 1, opt ? opt->bottom_modes : 0, &p);
  TOR_TRY(ensure_cap(w, p.bytes));
  const bool timed = opt && (opt->flags & TOR_FLAG_TIME_KERNEL);
  w->ev_pairs = 0;
  tor_result_t* dres = (tor_result_t*)(w->buf + p.o_res);
  TOR_TRY(enqueue_schur_group(w, p, O, nullptr, ld, opt, nullptr, dres, timed, s));
  ro->dres = dres;
  ro->red = w->buf + p.o_inst;
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
      for (auto& kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
      if (w->meta) (void)hipFree(w->meta);
      if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
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

int tor_eval_batched(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                     const int32_t* tiers, double tau, const tor_options_t* opt, void* stream,
                     tor_result_t* out) {
  if (batch < 0) return TOR_EINVAL;
  if (batch == 0) return TOR_OK;
  if (!offsets || !n || !out) return TOR_EINVAL;
  if (opt && opt->algo != TOR_ALGO_AUTO && opt->algo != TOR_ALGO_SCHUR) return TOR_EINVAL;
  bool any_work = false;
  for (int k = 0; k < batch; ++k) {
    if (n[k] < 0 || n[k] > TOR_NMAX || offsets[k] < 0) return TOR_EINVAL;
    const int t = tiers ? tiers[k] : TOR_AUTO;
    if (t != TOR_FP64 && t != TOR_DD && t != TOR_QD && t != TOR_AUTO) return TOR_EINVAL;
    if (n[k] > 0) any_work = true;
  }
  if (any_work && !O_packed) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  // the previous call on this stream may still read the plan buffer
  TOR_HIP(hipStreamSynchronize(s));

  std::vector<int32_t> tier_of(batch);
  for (int k = 0; k < batch; ++k) tier_of[k] = tiers ? tiers[k] : TOR_AUTO;
  bool any_auto = false;
  for (int k = 0; k < batch; ++k) any_auto = any_auto || (tier_of[k] == TOR_AUTO && n[k] > 0);
  if (any_auto) TOR_TRY(select_tiers(w, O_packed, offsets, n, batch, tau, tier_of.data(), s));

  const bool use_graph = opt && (opt->flags & TOR_FLAG_GRAPH);
  std::string key;
  if (use_graph) {
    auto put = [&](const void* p, size_t b) { key.append((const char*)p, b); };
    put(&O_packed, sizeof(O_packed));
    put(&out, sizeof(out));
    put(&s, sizeof(s));
    put(&batch, sizeof(batch));
    put(offsets, sizeof(int64_t) * batch);
    put(n, sizeof(int32_t) * batch);
    put(tier_of.data(), sizeof(int32_t) * batch);
    if (opt) put(opt, sizeof(*opt));
    auto it = w->graphs.find(key);
    if (it != w->graphs.end()) {
      TOR_HIP(hipGraphLaunch(it->second, s));
      return TOR_OK;
    }
  }

  // group by (n, tier); n = 0 instances are filled directly
  std::map<std::pair<int, int>, size_t> gmap;
  std::vector<BatchGroup> groups;
  std::vector<int32_t> triv_idx, triv_tier;
  for (int k = 0; k < batch; ++k) {
    const int t = tier_of[k] == TOR_AUTO ? TOR_DD : tier_of[k];
    if (n[k] == 0) {
      triv_idx.push_back(k);
      triv_tier.push_back(t);
      continue;
    }
    auto key2 = std::make_pair(n[k], t);
    auto it = gmap.find(key2);
    if (it == gmap.end()) {
      gmap[key2] = groups.size();
      groups.push_back(BatchGroup{n[k], t, {}});
      it = gmap.find(key2);
    }
    groups[it->second].idx.push_back(k);
  }
  // plans, one workspace size for all groups (they run one after another)
  std::vector<SchurPlan> plans(groups.size());
  size_t need = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    plan_schur(groups[gi].tier, groups[gi].n, (int)groups[gi].idx.size(), opt ? opt->bottom_modes : 0,
               &plans[gi]);
    need = std::max(need, plans[gi].bytes);
  }
  TOR_TRY(ensure_cap(w, need));
  // plan buffer: per group offsets (int64) then output indices (int32); trivial list
  std::vector<char> meta;
  std::vector<size_t> meta_off(groups.size());
  auto align8 = [&]() { while (meta.size() % 8) meta.push_back(0); };
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    align8();
    meta_off[gi] = meta.size();
    for (int32_t k : groups[gi].idx) {
      const int64_t o = offsets[k];
      meta.insert(meta.end(), (const char*)&o, (const char*)&o + 8);
    }
    for (int32_t k : groups[gi].idx) meta.insert(meta.end(), (const char*)&k, (const char*)&k + 4);
  }
  align8();
  const size_t triv_off = meta.size();
  for (int32_t k : triv_idx) meta.insert(meta.end(), (const char*)&k, (const char*)&k + 4);
  for (int32_t t : triv_tier) meta.insert(meta.end(), (const char*)&t, (const char*)&t + 4);
  if (!meta.empty()) TOR_TRY(upload_meta(w, meta.data(), meta.size()));
  // the buffer may have moved: nothing captured before this point survives
  if (use_graph) {
    // capture on a private stream (the caller's may be the null stream, which
    // cannot be captured), replay on the caller's
    if (!w->cap_stream) TOR_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = w->cap_stream;
    hipGraph_t graph = nullptr;
    TOR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch(w, groups, plans, meta_off, triv_off, (int)triv_idx.size(), O_packed,
                                 opt, out, cs);
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc != TOR_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    TOR_HIP(e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    TOR_HIP(e);
    w->graphs[key] = exec;
    TOR_HIP(hipGraphLaunch(exec, s));
    return TOR_OK;
  }
  return enqueue_batch(w, groups, plans, meta_off, triv_off, (int)triv_idx.size(), O_packed, opt,
                       out, s);
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
