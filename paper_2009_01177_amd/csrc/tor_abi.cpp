// tor_abi.cpp -- the C ABI (include/tor.h): argument checks, per-device
// workspace, work-item planning and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <dlfcn.h>

#include <algorithm>
#include <map>
#include <string>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/tor.h"
#include "prec.hpp"
#include "tor_host.h"
#include "tor_internal.hpp"
#include "tor_mcmc.hpp"

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
  char* meta = nullptr;         // device copy of the selector's plan (synchronous uploads)
  size_t meta_cap = 0;
  // ring of batch-plan slots for stream-ordered batches: a slot is reused
  // only after the event recorded behind its last batch has completed
  struct PlanSlot {
    char* dev = nullptr;
    char* host = nullptr;  // pinned staging of the upload
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
  };
  static constexpr int NSLOT = 4;
  PlanSlot slots[NSLOT];
  int slot_next = 0;
  // captured batches (TOR_FLAG_GRAPH); each owns a private device copy of its
  // plan, since the shared plan buffer is rewritten by every later call
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    char* plan = nullptr;
  };
  std::map<std::string, GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;              // private stream graphs are captured on
  char* aux = nullptr;                           // selector scratch
  size_t aux_cap = 0;
  std::vector<hipEvent_t> evs;  // kernel timing (TOR_FLAG_TIME_KERNEL): start/stop pairs
  int ev_pairs = 0;             // pairs recorded by the last evaluation
  double last_ms = -1.0;
  int last_d = -1, last_grid = -1, last_launches = 0;
};

std::mutex g_mu;
std::map<int, Workspace*> g_ws;

std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tuned;  // (n, tier) -> s_b
// tor_autotune times n <= AUTOTUNE_GROUP_NMAX as batch groups of this many
// instances (the batched workloads' shape), larger n as single instances
constexpr int AUTOTUNE_GROUP = 256;
constexpr int AUTOTUNE_GROUP_NMAX = 24;

int load_tune_table(const char* path);

// The tuned table shipped beside the library (data/autotune_default.txt in
// the library's directory), or the file TOR_AUTOTUNE_TABLE names (empty:
// none), read once per process before the first plan.
void load_default_tune_table() {
  static std::once_flag once;
  std::call_once(once, []() {
    std::string path;
    if (const char* e = getenv("TOR_AUTOTUNE_TABLE")) {
      path = e;
    } else {
      Dl_info info;
      if (dladdr(reinterpret_cast<const void*>(&load_default_tune_table), &info) && info.dli_fname) {
        path = info.dli_fname;
        const size_t slash = path.find_last_of('/');
        path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/data/autotune_default.txt";
      }
    }
    if (!path.empty()) (void)load_tune_table(path.c_str());
  });
}

int tuned_bottom(int n, int tier) {
  load_default_tune_table();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_pair(n, tier));
  return it == g_tuned.end() ? 0 : it->second;
}

std::mutex g_sel_mu;
tor_selector_t g_sel;  // zero-initialised: no network
int g_sel_version = 0;
tor_select_stats_t g_stats;

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

// Device bytes the workspace allocates for a plan of `bytes`: the plan
// rounded up to 2 MiB (the workspace grows to the largest plan seen).
size_t workspace_capacity(size_t bytes) {
  const size_t g = (size_t)2 << 20;
  return (bytes + g - 1) / g * g;
}

// Release every captured graph and its plan copy (after the device has
// finished with them).
void drop_graphs(Workspace* w) {
  for (auto& kv : w->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.plan) (void)hipFree(kv.second.plan);
  }
  w->graphs.clear();
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
  const size_t ncap = workspace_capacity(bytes);
  if (w->buf) {
    // the old buffer may still be in use by enqueued work
    TOR_HIP(hipDeviceSynchronize());
    TOR_HIP(hipFree(w->buf));
    w->buf = nullptr;
    w->cap = 0;
  }
  // captured graphs point into the old buffer
  drop_graphs(w);
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

// Lay out a plan whose chunks end in 2^LT middle states and whose kept
// frontier is at depth D_s (D_m - LT <= D_s <= D_m).
void plan_layout(int tier, int n, int R, int s_m, int s_b, int LT, int D_s, SchurPlan* p) {
  p->tier = tier;
  p->n = n;
  p->R = R;
  p->s_m = s_m;
  p->s_b = s_b;
  p->D_m = n - s_m;
  p->rb = schur_value_bytes(tier);
  p->ab = acc_bytes(tier);
  p->D_s = D_s;
  p->Dl = p->D_m - D_s;
  p->Ns = (size_t)R << D_s;
  size_t cr = p->Dl >= LT ? 1 : ((size_t)1 << (LT - p->Dl));
  if (cr > p->Ns) cr = p->Ns;
  p->Cr = (int)cr;
  p->nchunks = (int)((p->Ns + cr - 1) / cr);
  p->mids = cr << p->Dl;

  // levels in the ping-pong buffers: the root, the top levels above D_s
  // (depth D_s itself goes to the kept frontier) and a chunk's levels
  size_t lvl_vals = (size_t)R * psz(n);
  for (int j = 1; j < D_s; ++j) lvl_vals = std::max(lvl_vals, ((size_t)R << j) * psz(n - j));
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

// The library's plan for R instances of n modes: chunks of about 1.5 GB of
// middle states, the frontier kept at depth 10 where it fits in about 1 GB.
void plan_schur(int tier, int n, int R, int sb_req, SchurPlan* p) {
  if (sb_req <= 0) sb_req = tuned_bottom(n, tier);
  int s_m = 0, s_b = 0;
  schur_levels(tier, n, sb_req, &s_m, &s_b);
  const int D_m = n - s_m;
  const size_t rb = schur_value_bytes(tier);
  // middle states per chunk: about 1.5 GB of them at the last top level
  int LT = 0;
  while (LT < 22 && ((size_t)2 << LT) * psz(s_m) * rb <= ((size_t)3 << 29)) ++LT;
  // keep depth D_s (at most 10, at most ~1 GB of states, at least D_m - LT)
  int D_s = D_m < 10 ? D_m : 10;
  while (D_s > 0 && ((size_t)R << D_s) * psz(n - D_s) * rb > ((size_t)1 << 30)) --D_s;
  if (D_m - D_s > LT) D_s = D_m - LT;
  // large n: the kept frontier doubles with every mode while the chunk
  // stays put, so trade frontier for chunk (up to 2^22 middle states) while
  // the frontier is the larger of the two
  auto frontier_bytes = [&](int d) { return ((size_t)R << d) * psz(n - d) * rb; };
  while (D_s > 10 && LT < 22 && frontier_bytes(D_s) > ((size_t)2 << LT) * psz(s_m) * rb) {
    ++LT;
    D_s = D_m - LT;
  }
  plan_layout(tier, n, R, s_m, s_b, LT, D_s, p);
}

// A plan within max_bytes: the library's plan when it fits, else the one
// with the largest chunks that fits (frontier at the least depth they
// allow).  false when none does.
bool plan_schur_fit(int tier, int n, int R, int sb_req, size_t max_bytes, SchurPlan* p) {
  plan_schur(tier, n, R, sb_req, p);
  if (p->bytes <= max_bytes) return true;
  const int s_m = p->s_m, s_b = p->s_b, D_m = p->D_m;
  for (int LT = 22; LT >= 0; --LT) {
    SchurPlan q;
    plan_layout(tier, n, R, s_m, s_b, LT, std::max(0, D_m - LT), &q);
    if (q.bytes <= max_bytes) {
      *p = q;
      return true;
    }
  }
  return false;
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
// With one instance, only the depth-D_s states [z_lo, z_hi) are expanded and
// summed (a share of the evaluation; the whole of it by default).
// Level-sum debug mode: device buffers of the per-workgroup level sums of
// one chunk (grid x (n+1)), the per-chunk sums (nchunks x (n+1)), the
// result (n+1) and the reductions' scratch.
struct LevelOut {
  char* part;
  char* chunks;
  char* out;
  char* scratch;
};

// B is the plan's base (p.bytes of device memory), cus the device's compute
// units; w (may be NULL) receives the kernel timing events and launch shape.
// lv (single instance, whole evaluation) also runs the level-sum mode.
int enqueue_schur_group(Workspace* w, char* B, int cus, const SchurPlan& p, const void* O,
                        const int64_t* offs_dev, int64_t ld, const tor_options_t* opt,
                        const int32_t* out_index, tor_result_t* out, bool timed, hipStream_t s,
                        size_t z_lo = 0, size_t z_hi = SIZE_MAX, const LevelOut* lv = nullptr) {
  const int tier = p.tier, n = p.n;
  const bool whole = z_lo == 0 && z_hi >= p.Ns;
  if (!whole && (p.R != 1 || z_lo >= z_hi || z_hi > p.Ns)) return TOR_EINVAL;
  if (whole) z_hi = p.Ns;
  if (timed && !w) return TOR_EINVAL;
  uint32_t* cnt = (uint32_t*)(B + p.o_cnt);
  int32_t* status = (int32_t*)(cnt + 1);
  if (lv && (p.R != 1 || !whole)) return TOR_EINVAL;
  int occ = 0;
  if (lv) TOR_HIP(leaf_levels_occupancy(tier, p.s_b, &occ));
  else TOR_HIP(leaf_occupancy(tier, p.s_b, &occ));
  if (occ < 1) return TOR_EUNSUPPORTED;
  int grid = (opt && opt->grid > 0) ? opt->grid : occ * cus;
  if ((size_t)grid > p.mids) grid = (int)p.mids;

  TOR_HIP(launch_zero_words(cnt, 64, s));
  // levels a launch takes from states of `modes` modes, at most `left`:
  // up to three at once where their intermediate states fit in LDS
  auto levels_at = [&](int modes, int left) {
    for (int k = std::min(3, left); k >= 2; --k) {
      const size_t b = expand_multi_lds_bytes(tier, modes, k);
      if (b > 0 && b <= EXPAND_MULTI_LDS_MAX) return k;
    }
    return 1;
  };
  auto expand_levels = [&](const void* im, const void* ig, const int32_t* in_, int modes, int K, int nst,
                           void* om, void* og, int32_t* on) {
    if (K == 1) return launch_expand(tier, im, ig, in_, modes, nst, om, og, on, status, s);
    return launch_expand_multi(tier, im, ig, in_, modes, K, nst, om, og, on, status, s);
  };
  // stage 0: roots, then breadth-first to depth D_s into the kept buffer
  {
    int cur = 0;
    const bool direct = (p.D_s == 0);
    void* dm = direct ? (void*)(B + p.o_rm) : (void*)(B + p.o_m[0]);
    void* dg = direct ? (void*)(B + p.o_rg) : (void*)(B + p.o_g[0]);
    int32_t* dn = direct ? (int32_t*)(B + p.o_rn) : (int32_t*)(B + p.o_n[0]);
    TOR_HIP(launch_real_root(tier, (const double2*)O, offs_dev, p.R, n, ld, dm, dg, dn, s));
    for (int j = 0; j < p.D_s;) {
      const int K = levels_at(n - j, p.D_s - j);
      const bool last = (j + K == p.D_s);
      void* om = last ? (void*)(B + p.o_rm) : (void*)(B + p.o_m[1 - cur]);
      void* og = last ? (void*)(B + p.o_rg) : (void*)(B + p.o_g[1 - cur]);
      int32_t* on = last ? (int32_t*)(B + p.o_rn) : (int32_t*)(B + p.o_n[1 - cur]);
      TOR_HIP(expand_levels(B + p.o_m[cur], B + p.o_g[cur], (const int32_t*)(B + p.o_n[cur]), n - j, K,
                            p.R << j, om, og, on));
      cur = 1 - cur;
      j += K;
    }
  }
  const size_t rb = p.rb, ab = p.ab;
  for (size_t first = z_lo; first < z_hi; first += p.Cr) {
    const int cr = (int)std::min<size_t>(p.Cr, z_hi - first);
    const char* im = B + p.o_rm + rb * (first * psz(n - p.D_s));
    const char* ig = B + p.o_rg + rb * first;
    const int32_t* in_ = (const int32_t*)(B + p.o_rn) + first;
    int cur = -1;  // -1: the chunk's depth-D_s states themselves
    for (int j = 0; j < p.Dl;) {
      const int nx = (cur == 0) ? 1 : 0;
      const int K = levels_at(n - p.D_s - j, p.Dl - j);
      TOR_HIP(expand_levels(cur < 0 ? (const void*)im : (const void*)(B + p.o_m[cur]),
                            cur < 0 ? (const void*)ig : (const void*)(B + p.o_g[cur]),
                            cur < 0 ? in_ : (const int32_t*)(B + p.o_n[cur]), n - p.D_s - j, K, cr << j,
                            B + p.o_m[nx], B + p.o_g[nx], (int32_t*)(B + p.o_n[nx])));
      cur = nx;
      j += K;
    }
    const void* lm = cur < 0 ? (const void*)im : (const void*)(B + p.o_m[cur]);
    const void* lg = cur < 0 ? (const void*)ig : (const void*)(B + p.o_g[cur]);
    const int32_t* ln = cur < 0 ? in_ : (const int32_t*)(B + p.o_n[cur]);
    const int nm = cr << p.Dl;
    if (timed) TOR_TRY(record_ev(w, 2 * w->ev_pairs, s));
    if (lv) {
      const int blocks = std::min(grid, nm);
      TOR_HIP(launch_leaf_levels(tier, p.s_m, p.s_b, lm, lg, ln, nm, n, B + p.o_part, status, blocks, lv->part, s));
      TOR_HIP(launch_reduce_cols(tier, lv->part, blocks, n + 1, lv->chunks + ab * (n + 1) * (first / p.Cr),
                                 lv->scratch, s));
    } else {
      TOR_HIP(launch_leaf(tier, p.s_m, p.s_b, lm, lg, ln, nm, n, B + p.o_part, status, std::min(grid, nm), s));
    }
    if (timed) {
      TOR_TRY(record_ev(w, 2 * w->ev_pairs + 1, s));
      w->ev_pairs += 1;
    }
    TOR_TRY(fold(tier, B + p.o_part, cr, (size_t)1 << p.Dl, B + p.o_ds + ab * 2 * first, B + p.o_rsc, s));
  }
  if (lv) TOR_HIP(launch_reduce_cols(tier, lv->chunks, p.nchunks, n + 1, lv->out, lv->scratch, s));
  if (whole)
    TOR_TRY(fold(tier, B + p.o_ds, p.R, (size_t)1 << p.D_s, B + p.o_inst, B + p.o_rsc, s));
  else
    TOR_TRY(fold(tier, B + p.o_ds + ab * 2 * z_lo, 1, z_hi - z_lo, B + p.o_inst, B + p.o_rsc, s));
  const double err_rel = (double)(4 * n * n + n + 8) * unit_roundoff(tier);
  TOR_HIP(launch_finalize_batch(tier, B + p.o_inst, p.R, out_index, n, err_rel, out, s));
  if (w) {
    w->last_d = p.D_m;
    w->last_grid = grid;
  }
  return TOR_OK;
}

// Largest plan a batch group may take before it is split; a single
// instance takes what its own plan needs.
constexpr size_t GROUP_BUDGET = (size_t)4 << 30;

// Instances per sub-group for a group of R instances of n modes: the most
// whose plan stays within GROUP_BUDGET (at least one).
int group_share(int tier, int n, int R, int sb) {
  SchurPlan p;
  plan_schur(tier, n, R, sb, &p);
  if (p.bytes <= GROUP_BUDGET || R <= 1) return std::max(R, 1);
  int lo = 1, hi = R - 1;  // plan(lo) fits or lo == 1; plan(R) does not
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    plan_schur(tier, n, mid, sb, &p);
    if (p.bytes <= GROUP_BUDGET) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A batch grouped by (n, tier).
struct BatchGroup {
  int n, tier;
  std::vector<int32_t> idx;   // instance indices
  std::vector<int32_t> slot;  // their result slots in the output array
};

// One evaluation of a batch call: instance k at `tier`, its result into
// out[slot].  An instance may appear more than once (at different tiers).
struct BatchItem {
  int32_t k, tier, slot;
};

// Copy a plan into the shared plan buffer.  Earlier work on stream s may still
// read the buffer, so wait for it first.
int upload_meta(Workspace* w, const void* src, size_t bytes, hipStream_t s) {
  TOR_HIP(hipStreamSynchronize(s));
  if (bytes > w->meta_cap) {
    if (w->meta) TOR_HIP(hipFree(w->meta));
    w->meta = nullptr;
    w->meta_cap = 0;
    size_t cap = 4096;
    while (cap < bytes) cap *= 2;
    TOR_HIP(hipMalloc((void**)&w->meta, cap));
    w->meta_cap = cap;
  }
  TOR_HIP(hipMemcpy(w->meta, src, bytes, hipMemcpyHostToDevice));
  return TOR_OK;
}

// Stage a batch plan in the next slot of the ring: wait for the slot's
// previous batch only (its event), copy the plan to pinned memory and enqueue
// its upload on s.  The caller records the slot's event behind the batch.
int stage_plan(Workspace* w, const void* src, size_t bytes, hipStream_t s, Workspace::PlanSlot** out) {
  Workspace::PlanSlot& sl = w->slots[w->slot_next];
  w->slot_next = (w->slot_next + 1) % Workspace::NSLOT;
  if (!sl.ev) TOR_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  if (sl.used) {
    TOR_HIP(hipEventSynchronize(sl.ev));
    sl.used = false;
  }
  if (bytes > sl.cap) {
    if (sl.dev) TOR_HIP(hipFree(sl.dev));
    if (sl.host) TOR_HIP(hipHostFree(sl.host));
    sl.dev = nullptr;
    sl.host = nullptr;
    sl.cap = 0;
    size_t cap = 4096;
    while (cap < bytes) cap *= 2;
    TOR_HIP(hipMalloc((void**)&sl.dev, cap));
    TOR_HIP(hipHostMalloc((void**)&sl.host, cap, hipHostMallocDefault));
    sl.cap = cap;
  }
  memcpy(sl.host, src, bytes);
  TOR_HIP(hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, s));
  *out = &sl;
  return TOR_OK;
}

// Enqueue every group of a batch whose plan is at `plan` (device).
int enqueue_batch(Workspace* w, const char* plan, const std::vector<BatchGroup>& groups,
                  const std::vector<SchurPlan>& plans, const std::vector<size_t>& meta_off,
                  size_t triv_off, int ntriv, const void* O_packed, const tor_options_t* opt,
                  tor_result_t* out, hipStream_t s) {
  if (ntriv > 0)
    TOR_HIP(launch_fill_trivial(out, (const int32_t*)(plan + triv_off),
                                (const int32_t*)(plan + triv_off) + ntriv, ntriv, s));
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const BatchGroup& g = groups[gi];
    const int64_t* offs = (const int64_t*)(plan + meta_off[gi]);
    const int32_t* oidx = (const int32_t*)(offs + g.idx.size());
    TOR_TRY(enqueue_schur_group(w, w->buf, w->cus, plans[gi], O_packed, offs, 2 * (int64_t)g.n, opt, oidx, out,
                                false, s));
  }
  return TOR_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

// Scratch device memory for the selector (features, predictions, gradients),
// separate from the evaluation workspace so either may grow independently.
int ensure_aux(Workspace* w, size_t bytes, hipStream_t s) {
  if (bytes <= w->aux_cap) return TOR_OK;
  TOR_HIP(hipStreamSynchronize(s));
  TOR_HIP(hipDeviceSynchronize());
  if (w->aux) TOR_HIP(hipFree(w->aux));
  w->aux = nullptr;
  w->aux_cap = 0;
  // captured graphs may write their results into the old buffer
  drop_graphs(w);
  size_t cap = 1 << 20;
  while (cap < bytes) cap *= 2;
  TOR_HIP(hipMalloc((void**)&w->aux, cap));
  w->aux_cap = cap;
  return TOR_OK;
}

// TOR_FLAG_CHECK_INPUT: the input conventions of the instances with n > 0,
// checked on the device (one flag per instance, copied back); TOR_EINPUT if
// any is violated.  offsets == nullptr: the single instance O (n, ld).
int check_input(Workspace* w, const void* O, const int64_t* offsets, const int32_t* n, int count, int32_t n1,
                int64_t ld1, hipStream_t s) {
  std::vector<int64_t> off;
  std::vector<int32_t> nn;
  if (offsets) {
    for (int k = 0; k < count; ++k)
      if (n[k] > 0) {
        off.push_back(offsets[k]);
        nn.push_back(n[k]);
      }
  }
  const int m = offsets ? (int)off.size() : (n1 > 0 ? 1 : 0);
  if (m == 0) return TOR_OK;
  const size_t o_off = ((size_t)4 * m + 7) & ~(size_t)7, o_n = o_off + (size_t)8 * m;
  TOR_TRY(ensure_aux(w, o_n + (size_t)4 * m, s));
  int32_t* bad = (int32_t*)w->aux;
  const int64_t* d_off = nullptr;
  const int32_t* d_n = nullptr;
  if (offsets) {
    TOR_HIP(hipMemcpyAsync(w->aux + o_off, off.data(), (size_t)8 * m, hipMemcpyHostToDevice, s));
    TOR_HIP(hipMemcpyAsync(w->aux + o_n, nn.data(), (size_t)4 * m, hipMemcpyHostToDevice, s));
    d_off = (const int64_t*)(w->aux + o_off);
    d_n = (const int32_t*)(w->aux + o_n);
  }
  TOR_HIP(launch_zero_words((uint32_t*)bad, m, s));
  TOR_HIP(launch_check_input((const double2*)O, d_off, d_n, m, n1, ld1, bad, s));
  std::vector<int32_t> h(m);
  TOR_HIP(hipMemcpyAsync(h.data(), bad, (size_t)4 * m, hipMemcpyDeviceToHost, s));
  TOR_HIP(hipStreamSynchronize(s));
  for (int32_t v : h)
    if (v) return TOR_EINPUT;
  return TOR_OK;
}

bool wants_check(const tor_options_t* opt) { return opt && (opt->flags & TOR_FLAG_CHECK_INPUT); }

// Evaluate the items (instance indices into the batch arrays, tiers with no
// TOR_AUTO left, result slots), results to out[slot].
int batch_core(Workspace* w, const void* O_packed, const int64_t* offsets, const int32_t* n,
               const std::vector<BatchItem>& items, const tor_options_t* opt, tor_result_t* out,
               bool use_graph, hipStream_t s) {
  std::string key;
  if (use_graph) {
    auto put = [&](const void* p, size_t b) { key.append((const char*)p, b); };
    put(&O_packed, sizeof(O_packed));
    put(&out, sizeof(out));
    put(&s, sizeof(s));
    for (const BatchItem& it : items) {
      put(&it, sizeof(it));
      put(offsets + it.k, 8);
      put(n + it.k, 4);
    }
    if (opt) put(opt, sizeof(*opt));
    auto it = w->graphs.find(key);
    if (it != w->graphs.end()) {
      TOR_HIP(hipGraphLaunch(it->second.exec, s));
      return TOR_OK;
    }
  }
  // group by (n, tier); n = 0 instances are filled directly
  std::map<std::pair<int, int>, size_t> gmap;
  std::vector<BatchGroup> groups;
  std::vector<int32_t> triv_idx, triv_tier;
  for (const BatchItem& item : items) {
    const int k = item.k, t = item.tier;
    if (n[k] == 0) {
      triv_idx.push_back(item.slot);
      triv_tier.push_back(t == TOR_AUTO ? TOR_FP64 : t);
      continue;
    }
    if (t != TOR_FP64 && t != TOR_DD && t != TOR_QD) return TOR_EINVAL;
    auto key2 = std::make_pair((int)n[k], t);
    auto it = gmap.find(key2);
    if (it == gmap.end()) {
      gmap[key2] = groups.size();
      groups.push_back(BatchGroup{n[k], t, {}, {}});
      it = gmap.find(key2);
    }
    groups[it->second].idx.push_back(k);
    groups[it->second].slot.push_back(item.slot);
  }
  // groups whose plan would outgrow the group budget run as several
  // sub-groups of equal size
  const int sb_opt = opt ? opt->bottom_modes : 0;
  {
    std::vector<BatchGroup> split;
    for (BatchGroup& g : groups) {
      const int R = (int)g.idx.size();
      const int per = group_share(g.tier, g.n, R, sb_opt);
      for (int a = 0; a < R; a += per) {
        BatchGroup h{g.n, g.tier, {}, {}};
        h.idx.assign(g.idx.begin() + a, g.idx.begin() + std::min(R, a + per));
        h.slot.assign(g.slot.begin() + a, g.slot.begin() + std::min(R, a + per));
        split.push_back(std::move(h));
      }
    }
    groups.swap(split);
  }
  // plans, one workspace size for all groups (they run one after another)
  std::vector<SchurPlan> plans(groups.size());
  size_t need = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    plan_schur(groups[gi].tier, groups[gi].n, (int)groups[gi].idx.size(), sb_opt, &plans[gi]);
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
    for (int32_t k : groups[gi].slot) meta.insert(meta.end(), (const char*)&k, (const char*)&k + 4);
  }
  align8();
  const size_t triv_off = meta.size();
  for (int32_t k : triv_idx) meta.insert(meta.end(), (const char*)&k, (const char*)&k + 4);
  for (int32_t t : triv_tier) meta.insert(meta.end(), (const char*)&t, (const char*)&t + 4);
  if (use_graph) {
    if (w->graphs.size() >= 64) {  // bound the cache
      TOR_HIP(hipDeviceSynchronize());
      drop_graphs(w);
    }
    // the graph keeps its own copy of the plan
    Workspace::GraphEntry ge;
    if (!meta.empty()) {
      TOR_HIP(hipMalloc((void**)&ge.plan, meta.size()));
      hipError_t e0 = hipMemcpy(ge.plan, meta.data(), meta.size(), hipMemcpyHostToDevice);
      if (e0 != hipSuccess) {
        (void)hipFree(ge.plan);
        return hip_err(e0);
      }
    }
    // capture on a private stream (the caller's may be the null stream, which
    // cannot be captured), replay on the caller's
    if (!w->cap_stream) TOR_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = w->cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = hip_err(e);
    if (rc == TOR_OK) {
      rc = enqueue_batch(w, ge.plan, groups, plans, meta_off, triv_off, (int)triv_idx.size(), O_packed,
                         opt, out, cs);
      e = hipStreamEndCapture(cs, &graph);
      if (rc == TOR_OK) rc = hip_err(e);
    }
    if (rc == TOR_OK) {
      e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
      rc = hip_err(e);
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != TOR_OK) {
      if (ge.plan) (void)hipFree(ge.plan);
      return rc;
    }
    w->graphs[key] = ge;
    TOR_HIP(hipGraphLaunch(ge.exec, s));
    return TOR_OK;
  }
  // eager: the plan goes into the next ring slot with an asynchronous copy;
  // nothing waits for the stream unless that slot's previous batch is
  // still running
  Workspace::PlanSlot* sl = nullptr;
  if (!meta.empty()) TOR_TRY(stage_plan(w, meta.data(), meta.size(), s, &sl));
  TOR_TRY(enqueue_batch(w, sl ? sl->dev : nullptr, groups, plans, meta_off, triv_off, (int)triv_idx.size(),
                        O_packed, opt, out, s));
  if (sl) {
    TOR_HIP(hipEventRecord(sl->ev, s));
    sl->used = true;
  }
  return TOR_OK;
}

// The instances idx at the tiers tier_of[k], results to out[k].
int batch_core(Workspace* w, const void* O_packed, const int64_t* offsets, const int32_t* n,
               const std::vector<int32_t>& idx, const std::vector<int32_t>& tier_of,
               const tor_options_t* opt, tor_result_t* out, bool use_graph, hipStream_t s) {
  std::vector<BatchItem> items;
  items.reserve(idx.size());
  for (int32_t k : idx) items.push_back(BatchItem{k, tier_of[k], k});
  return batch_core(w, O_packed, offsets, n, items, opt, out, use_graph, s);
}

// ---------------------------------------------------------------------------
// Precision selector
// ---------------------------------------------------------------------------

double tier_unit_log10(int t) {
  return t == TOR_FP64 ? -53.0 * 0.30102999566398120 : (t == TOR_DD ? -104.0 * 0.30102999566398120
                                                                    : -208.0 * 0.30102999566398120);
}

// Bound estimate of the significand bits an instance needs (Eq. 7 for
// floating tiers; see the declaration in tor.h).  feats as tor_features.
// log10 of the relative forward error the selector expects of tier t for
// an instance whose network output is y.
double predicted_log10_err(const tor_selector_t& sel, int t, double y) {
  if (sel.target == TOR_TARGET_ERR64) return y + sel.margin + sel.log10_c[t];
  return sel.log10_c[t] + sel.slope[t] * (y + sel.margin) + tier_unit_log10(t);
}

double fallback_bits(const double* f, double tau) {
  const double n = f[0];
  const double logdet = -2.0 * f[1];
  const double a = f[4], k = f[5];
  const double ln2 = 0.69314718055994531;
  const double base = 1.0 / ((1.0 - a) - k * n / (1.0 - a)) - 1.0;
  if (!(base > 0.0)) return 1e300;  // no usable lower bound: take the widest tier
  const double log2_tor_lower = n * log2(base);
  const double log2_sabs_upper = n - 0.5 * logdet / ln2;
  const double b_cancel = std::max(0.0, log2_sabs_upper - log2_tor_lower);
  const double b_sgn = log2(1.0 / tau);
  const double b_accum = log2(0.5) + n + 2.0 * log2(n);
  return b_cancel + b_sgn + b_accum;
}

// Tiers for the TOR_AUTO instances of a batch; pred/src receive, per
// instance, the predicted log10 kappa (or the bound's bits in log10 units)
// and 0 (network) / 1 (bound estimate).
int select_tiers(Workspace* w, const void* O_packed, const int64_t* offsets, const int32_t* n,
                 int batch, double tau, int32_t* tier_of, std::vector<double>* pred,
                 std::vector<int32_t>* src, hipStream_t s) {
  pred->assign(batch, 0.0);
  src->assign(batch, 0);
  std::vector<int32_t> idx;
  int nmax = 1;
  for (int k = 0; k < batch; ++k)
    if (tier_of[k] == TOR_AUTO && n[k] > 0) {
      idx.push_back(k);
      nmax = std::max(nmax, (int)n[k]);
    }
  tor_select_stats_t st;
  memset(&st, 0, sizeof(st));
  const int m = (int)idx.size();
  if (m > 0) {
    tor_selector_t sel;
    int version;
    {
      std::lock_guard<std::mutex> lk(g_sel_mu);
      sel = g_sel;
      version = g_sel_version;
    }
    // device: offsets, n | feats (m x F) | preds (m) | selector (theta, mean, std)
    const size_t nsel = TOR_MLP_PARAMS + 2 * TOR_NFEAT;
    std::vector<char> meta(sizeof(int64_t) * m + sizeof(int32_t) * m);
    for (int i = 0; i < m; ++i) {
      memcpy(meta.data() + 8 * i, &offsets[idx[i]], 8);
      memcpy(meta.data() + 8 * m + 4 * i, &n[idx[i]], 4);
    }
    TOR_TRY(upload_meta(w, meta.data(), meta.size(), s));
    const size_t o_feat = 0, o_pred = o_feat + sizeof(double) * m * TOR_NFEAT;
    const size_t o_sel = o_pred + sizeof(double) * m;
    TOR_TRY(ensure_aux(w, o_sel + sizeof(double) * nsel, s));
    double* feats = (double*)(w->aux + o_feat);
    double* preds = (double*)(w->aux + o_pred);
    double* dsel = (double*)(w->aux + o_sel);
    TOR_HIP(launch_features((const double2*)O_packed, (const int64_t*)w->meta,
                            (const int32_t*)(w->meta + 8 * m), m, nmax, feats, s));
    if (sel.trained) {
      std::vector<double> hs(nsel);
      memcpy(hs.data(), sel.theta, sizeof(double) * TOR_MLP_PARAMS);
      memcpy(hs.data() + TOR_MLP_PARAMS, sel.mean, sizeof(double) * TOR_NFEAT);
      memcpy(hs.data() + TOR_MLP_PARAMS + TOR_NFEAT, sel.std, sizeof(double) * TOR_NFEAT);
      TOR_HIP(hipMemcpyAsync(dsel, hs.data(), sizeof(double) * nsel, hipMemcpyHostToDevice, s));
      TOR_HIP(launch_mlp_forward(dsel, dsel + TOR_MLP_PARAMS, dsel + TOR_MLP_PARAMS + TOR_NFEAT, feats, m,
                                 preds, s));
      TOR_HIP(hipStreamSynchronize(s));  // hs must outlive the copy
    }
    (void)version;
    std::vector<double> hf((size_t)m * TOR_NFEAT), hp(m, 0.0);
    TOR_HIP(hipMemcpyAsync(hf.data(), feats, sizeof(double) * hf.size(), hipMemcpyDeviceToHost, s));
    if (sel.trained)
      TOR_HIP(hipMemcpyAsync(hp.data(), preds, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    TOR_HIP(hipStreamSynchronize(s));
    const double ltau = log10(tau);
    for (int i = 0; i < m; ++i) {
      const double* f = &hf[(size_t)i * TOR_NFEAT];
      const int nk = n[idx[i]];
      bool ood = !sel.trained || nk < sel.nmin || nk > sel.nmax || !std::isfinite(hp[i]);
      for (int j = 0; j < TOR_NFEAT && !ood; ++j) {
        const double span = sel.fmax[j] - sel.fmin[j];
        const double slack = 0.05 * span + 1e-12;
        if (!(f[j] >= sel.fmin[j] - slack && f[j] <= sel.fmax[j] + slack)) ood = true;
      }
      int t;
      if (ood) {
        const double bits = fallback_bits(f, tau);
        t = bits <= 53.0 ? TOR_FP64 : (bits <= 106.0 ? TOR_DD : TOR_QD);
        (*pred)[idx[i]] = bits * 0.30102999566398120;
        (*src)[idx[i]] = 1;
        st.n_fallback++;
      } else {
        t = TOR_QD;
        for (int c = TOR_FP64; c <= TOR_DD; ++c) {
          if (predicted_log10_err(sel, c, hp[i]) <= ltau) {
            t = c;
            break;
          }
        }
        (*pred)[idx[i]] = hp[i];
        (*src)[idx[i]] = 0;
      }
      tier_of[idx[i]] = t;
      if (t == TOR_FP64) st.n_fp64++;
      else if (t == TOR_DD) st.n_dd++;
      else st.n_qd++;
    }
  }
  std::lock_guard<std::mutex> lk(g_sel_mu);
  g_stats = st;
  return TOR_OK;
}

// Spot re-evaluation of TOR_AUTO choices one tier up.  Only network choices
// whose predicted error lies within `window` decades of tau are informative
// (a choice predicted far below tau cannot be checked against tau by a
// re-evaluation that is itself only as good as the next tier); a fraction
// of those is re-evaluated, at least one per tier.  The sample is drawn
// before the evaluation so that its re-evaluations run in the same batch
// (they join the groups of their n and tier, one launch sequence).
struct SpotSample {
  int32_t k, tier;  // instance, the tier it was chosen for
};

std::vector<SpotSample> spot_sample(int batch, const int32_t* n, const int32_t* tiers_req, double tau,
                                    const std::vector<int32_t>& tier_of, const std::vector<double>& pred,
                                    const std::vector<int32_t>& src) {
  double frac = 1.0 / 32.0;
  if (const char* e = getenv("TOR_SPOT_FRACTION")) {
    const double v = atof(e);
    if (v > 0.0 && v <= 1.0) frac = v;
  }
  double window = 4.0;
  if (const char* e = getenv("TOR_SPOT_WINDOW")) {
    const double v = atof(e);
    if (v > 0.0) window = v;
  }
  tor_selector_t sel;
  {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    sel = g_sel;
  }
  const double ltau = log10(tau);
  const int stride = std::max(1, (int)llround(1.0 / frac));
  std::vector<SpotSample> out;
  for (int t = TOR_FP64; t <= TOR_DD; ++t) {
    std::vector<int32_t> near;
    for (int k = 0; k < batch; ++k)
      if (n[k] > 0 && (tiers_req ? tiers_req[k] : TOR_AUTO) == TOR_AUTO && tier_of[k] == t && src[k] == 0 &&
          predicted_log10_err(sel, t, pred[k]) >= ltau - window)
        near.push_back(k);
    for (size_t i = 0; i < near.size(); i += stride) out.push_back(SpotSample{near[i], t});
  }
  return out;
}

// Compare each sampled result (res[k], chosen tier) with its re-evaluation
// one tier up (res[batch + i]); on a miss, move up every instance of that
// tier predicted at least as hard and evaluate those again into out.
int spot_verify(Workspace* w, const void* O_packed, const int64_t* offsets, const int32_t* n, int batch,
                const int32_t* tiers_req, double tau, std::vector<int32_t>& tier_of,
                const std::vector<double>& pred, const std::vector<int32_t>& src,
                const std::vector<SpotSample>& smp, const std::vector<tor_result_t>& res, tor_result_t* out,
                hipStream_t s) {
  int n_viol = 0, n_esc = 0;
  for (int t = TOR_FP64; t <= TOR_DD; ++t) {
    double thr = 1e300;
    bool viol = false;
    for (size_t i = 0; i < smp.size(); ++i) {
      if (smp[i].tier != t) continue;
      const tor_result_t& hi = res[batch + i];
      const tor_result_t& lo = res[smp[i].k];
      const double th = hi.tor[0] + hi.tor[1];
      const double tl = lo.tor[0] + lo.tor[1];
      if (!(fabs(tl - th) <= tau * fabs(th))) {
        viol = true;
        ++n_viol;
        thr = std::min(thr, pred[smp[i].k]);
      }
    }
    if (!viol) continue;
    std::vector<int32_t> esc;
    for (int k = 0; k < batch; ++k)
      if (n[k] > 0 && (tiers_req ? tiers_req[k] : TOR_AUTO) == TOR_AUTO && tier_of[k] == t &&
          (pred[k] >= thr - 1.0 || src[k] == 1))
        esc.push_back(k);
    for (int32_t k : esc) tier_of[k] = t + 1;
    n_esc += (int)esc.size();
    TOR_TRY(batch_core(w, O_packed, offsets, n, esc, tier_of, nullptr, out, false, s));
  }
  std::lock_guard<std::mutex> lk(g_sel_mu);
  g_stats.n_spot = (int)smp.size();
  g_stats.n_violations = n_viol;
  g_stats.n_escalated = n_esc;
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
  TOR_TRY(enqueue_schur_group(w, w->buf, w->cus, p, O, nullptr, ld, opt, nullptr, dres, timed, s));
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
    case TOR_EINPUT: return "O is not finite, not Hermitian, or lacks the block structure of Eq. 3";
    case TOR_EUNSUPPORTED: return "not supported: tier and n do not fit the kernel's storage plan, or the library was compiled without this facility";
    default: return "unknown error";
  }
}

int tor_init(void) {
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  // the fixed buffer of tor_eval_noalloc: look up its device address now
  void* base = nullptr;
  int cus = 0;
  return hip_err(noalloc_buffer(&base, &cus));
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
      drop_graphs(w);
      if (w->meta) (void)hipFree(w->meta);
      for (auto& sl : w->slots) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
      }
      if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
      if (w->aux) (void)hipFree(w->aux);
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
  if (wants_check(opt)) TOR_TRY(check_input(w, O, nullptr, nullptr, 1, n, ld, s));
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

int tor_eval_noalloc(const void* O, int32_t n, int64_t ld, int32_t tier, void* stream, tor_result_t* out) {
  if (out == nullptr) return TOR_EINVAL;
  TOR_TRY(check_common(O, n, ld, tier));
  if (n > tor_noalloc_nmax(tier)) return TOR_EUNSUPPORTED;
  void* base = nullptr;
  int cus = 0;
  TOR_HIP(noalloc_buffer(&base, &cus));
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) return hip_err(launch_trivial_one(out, tier, s));
  SchurPlan p;
  if (!plan_schur_fit(tier, n, 1, 0, TOR_NOALLOC_SCRATCH_BYTES, &p)) return TOR_EUNSUPPORTED;
  // the buffer keeps the last call's contents: the plan's counters and
  // status word are cleared by a kernel inside the sequence, and every
  // partial sum is written before it is read
  return enqueue_schur_group(nullptr, (char*)base, cus, p, O, nullptr, ld, nullptr, nullptr, out, false, s);
}

int32_t tor_noalloc_nmax(int32_t tier) {
  if (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD) return TOR_EINVAL;
  static std::mutex mu;
  static int cached[3] = {-1, -1, -1};
  std::lock_guard<std::mutex> lk(mu);
  if (cached[tier] < 0) {
    int nmax = 0;
    for (int n = 1; n <= TOR_NMAX; ++n) {
      SchurPlan p;
      if (!plan_schur_fit(tier, n, 1, 0, TOR_NOALLOC_SCRATCH_BYTES, &p)) break;
      nmax = n;
    }
    cached[tier] = nmax;
  }
  return cached[tier];
}

int tor_workspace_bytes(int32_t n, int32_t tier, int32_t bottom_modes, uint64_t* bytes) {
  if (bytes == nullptr || n < 0 || n > TOR_NMAX || bottom_modes < 0) return TOR_EINVAL;
  if (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD) return TOR_EINVAL;
  if (n == 0) {
    *bytes = 0;
    return TOR_OK;
  }
  SchurPlan p;
  plan_schur(tier, n, 1, bottom_modes, &p);
  *bytes = workspace_capacity(p.bytes);
  return TOR_OK;
}

int tor_batch_workspace_bytes(int32_t n, int32_t tier, int32_t count, int32_t bottom_modes, uint64_t* bytes) {
  if (bytes == nullptr || n < 0 || n > TOR_NMAX || count < 0 || bottom_modes < 0) return TOR_EINVAL;
  if (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD) return TOR_EINVAL;
  if (n == 0 || count == 0) {
    *bytes = 0;
    return TOR_OK;
  }
  const int per = group_share(tier, n, count, bottom_modes);
  SchurPlan p;
  plan_schur(tier, n, per, bottom_modes, &p);
  *bytes = workspace_capacity(p.bytes);
  return TOR_OK;
}

double tor_last_kernel_ms(int32_t* split_depth, int32_t* grid, int32_t* launches) {
  Workspace* w = nullptr;
  if (get_ws(&w) != TOR_OK) return -1.0;
  if (split_depth) *split_depth = w->last_d;
  if (grid) *grid = w->last_grid;
  if (launches) *launches = w->last_launches;
  return w->last_ms;
}

int tor_eval_part(const void* O, int32_t n, int64_t ld, int32_t tier, const tor_options_t* opt,
                  void* stream, int32_t part, int32_t nparts, tor_result_t* out) {
  if (out == nullptr || nparts < 1 || part < 0 || part >= nparts) return TOR_EINVAL;
  TOR_TRY(check_common(O, n, ld, tier));
  if (opt && opt->algo != TOR_ALGO_AUTO && opt->algo != TOR_ALGO_SCHUR) return TOR_EINVAL;
  int k = 0;  // prefix modes that number the parts
  while (((int64_t)1 << k) < (int64_t)nparts) ++k;
  if (n == 0) {
    if (nparts != 1) return TOR_EINVAL;
    fill_trivial(out, tier);
    return TOR_OK;
  }
  SchurPlan p;
  plan_schur(tier, n, 1, opt ? opt->bottom_modes : 0, &p);
  if (k > p.D_s) return TOR_EINVAL;  // more parts than depth-D_s states
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  if (wants_check(opt)) TOR_TRY(check_input(w, O, nullptr, nullptr, 1, n, ld, s));
  TOR_TRY(ensure_cap(w, p.bytes));
  const size_t codes = (size_t)1 << k;
  const size_t c_lo = (size_t)part * codes / (size_t)nparts;
  const size_t c_hi = (size_t)(part + 1) * codes / (size_t)nparts;
  const int sh = p.D_s - k;
  const bool timed = opt && (opt->flags & TOR_FLAG_TIME_KERNEL);
  w->ev_pairs = 0;
  tor_result_t* dres = (tor_result_t*)(w->buf + p.o_res);
  TOR_TRY(enqueue_schur_group(w, w->buf, w->cus, p, O, nullptr, ld, opt, nullptr, dres, timed, s, c_lo << sh,
                              c_hi << sh));
  TOR_HIP(hipMemcpyAsync(w->host_res, dres, sizeof(tor_result_t), hipMemcpyDeviceToHost, s));
  TOR_HIP(hipStreamSynchronize(s));
  if (w->ev_pairs > 0) TOR_TRY(collect_ev(w));
  *out = *w->host_res;
  return out->status;
}

int tor_combine_parts(int32_t tier, int32_t n, const tor_result_t* parts, int32_t nparts,
                      tor_result_t* out) {
  if (!parts || !out || nparts < 1 || n < 0 || n > TOR_NMAX) return TOR_EINVAL;
  if (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD) return TOR_EINVAL;
  int status = TOR_OK;
  prec::dd a{0.0, 0.0}, t2{0.0, 0.0};
  prec::qd t4{{0.0, 0.0, 0.0, 0.0}};
  for (int i = 0; i < nparts; ++i) {
    const tor_result_t& r = parts[i];
    if (r.tier_used != tier) return TOR_EINVAL;
    if (r.status != TOR_OK && status == TOR_OK) status = r.status;
    a = prec::dd_add(a, prec::dd{r.abs_sum[0], r.abs_sum[1]});
    if (tier == TOR_QD)
      t4 = prec::qd_add(t4, prec::qd{{r.tor[0], r.tor[1], r.tor[2], r.tor[3]}});
    else
      t2 = prec::dd_add(t2, prec::dd{r.tor[0], r.tor[1]});
  }
  memset(out, 0, sizeof(*out));
  if (tier == TOR_QD) {
    const prec::qd z = prec::qd_nonoverlapping(t4);
    for (int i = 0; i < 4; ++i) out->tor[i] = z.x[i];
  } else {
    out->tor[0] = t2.hi;
    out->tor[1] = t2.lo;
  }
  out->abs_sum[0] = a.hi;
  out->abs_sum[1] = a.lo;
  out->err_bound = (double)(4 * n * n + n + 8) * unit_roundoff(tier) * a.hi;
  out->tier_used = tier;
  out->status = status;
  return TOR_OK;
}

int tor_eval_batched(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                     const int32_t* tiers, double tau, const tor_options_t* opt, void* stream,
                     tor_result_t* out) {
  if (batch < 0) return TOR_EINVAL;
  if (batch == 0) return TOR_OK;
  if (!offsets || !n || !out) return TOR_EINVAL;
  if (opt && opt->algo != TOR_ALGO_AUTO && opt->algo != TOR_ALGO_SCHUR) return TOR_EINVAL;
  bool any_work = false, any_auto = false;
  for (int k = 0; k < batch; ++k) {
    if (n[k] < 0 || n[k] > TOR_NMAX || offsets[k] < 0) return TOR_EINVAL;
    const int t = tiers ? tiers[k] : TOR_AUTO;
    if (t != TOR_FP64 && t != TOR_DD && t != TOR_QD && t != TOR_AUTO) return TOR_EINVAL;
    if (n[k] > 0) any_work = true;
    if (n[k] > 0 && t == TOR_AUTO) any_auto = true;
  }
  if (any_work && !O_packed) return TOR_EINVAL;
  if (any_auto && !(tau > 0.0)) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  if (wants_check(opt)) TOR_TRY(check_input(w, O_packed, offsets, n, batch, 0, 0, s));
  std::vector<int32_t> tier_of(batch);
  for (int k = 0; k < batch; ++k) tier_of[k] = tiers ? tiers[k] : TOR_AUTO;
  std::vector<double> pred;
  std::vector<int32_t> src;
  if (any_auto) TOR_TRY(select_tiers(w, O_packed, offsets, n, batch, tau, tier_of.data(), &pred, &src, s));

  const bool use_graph = opt && (opt->flags & TOR_FLAG_GRAPH);
  std::vector<BatchItem> items(batch);
  for (int k = 0; k < batch; ++k) items[k] = BatchItem{k, tier_of[k], k};
  std::vector<SpotSample> smp;
  if (any_auto) smp = spot_sample(batch, n, tiers, tau, tier_of, pred, src);
  if (smp.empty()) {
    TOR_TRY(batch_core(w, O_packed, offsets, n, items, opt, out, use_graph, s));
    if (any_auto) {
      std::lock_guard<std::mutex> lk(g_sel_mu);
      g_stats.n_spot = g_stats.n_violations = g_stats.n_escalated = 0;
    }
    return TOR_OK;
  }
  // the chosen tiers and the sample's re-evaluations one tier up in one
  // batch, into a scratch result array: [0, batch) the batch, then the sample
  const int total = batch + (int)smp.size();
  for (size_t i = 0; i < smp.size(); ++i)
    items.push_back(BatchItem{smp[i].k, smp[i].tier + 1, batch + (int32_t)i});
  TOR_TRY(ensure_aux(w, sizeof(tor_result_t) * (size_t)total, s));
  tor_result_t* res_dev = (tor_result_t*)w->aux;
  TOR_TRY(batch_core(w, O_packed, offsets, n, items, opt, res_dev, use_graph, s));
  TOR_HIP(hipMemcpyAsync(out, res_dev, sizeof(tor_result_t) * (size_t)batch, hipMemcpyDeviceToDevice, s));
  std::vector<tor_result_t> res(total);
  TOR_HIP(hipMemcpyAsync(res.data(), res_dev, sizeof(tor_result_t) * (size_t)total, hipMemcpyDeviceToHost, s));
  TOR_HIP(hipStreamSynchronize(s));
  return spot_verify(w, O_packed, offsets, n, batch, tiers, tau, tier_of, pred, src, smp, res, out, s);
}

int tor_mcmc(const void* O_full, int32_t M, int64_t ld, int32_t N, int32_t chains, int32_t steps,
             const int32_t* proposals, const double* uniforms, int32_t tier, double tau,
             const tor_options_t* opt, void* stream, tor_result_t* cand_out, int32_t* state_step) {
  if (M < 1 || N < 0 || N > M || N > TOR_NMAX || chains < 1 || steps < 1) return TOR_EINVAL;
  if (ld < 2 * (int64_t)M) return TOR_EINVAL;
  if (!O_full || !uniforms || !cand_out || !state_step || (N > 0 && !proposals)) return TOR_EINVAL;
  if (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD && tier != TOR_AUTO) return TOR_EINVAL;
  if (tier == TOR_AUTO && !(tau > 0.0)) return TOR_EINVAL;
  if (opt && opt->algo != TOR_ALGO_AUTO && opt->algo != TOR_ALGO_SCHUR) return TOR_EINVAL;
  const int64_t total = (int64_t)chains * steps;
  if (total > INT32_MAX) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  // candidates are scored in chunks of at most 1 GiB of packed O_S
  const int64_t per = 4 * (int64_t)N * N;  // complex elements per candidate
  int64_t chunk = total;
  if (per > 0) chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, ((int64_t)1 << 26) / per));
  if (const char* e = getenv("TOR_MCMC_CHUNK")) {
    const long long c = atoll(e);
    if (c >= 1) chunk = std::min<int64_t>(chunk, c);
  }
  char* buf = nullptr;
  TOR_HIP(hipMalloc((void**)&buf, 256 + (size_t)(per > 0 ? chunk * per : 1) * sizeof(double2)));
  int32_t* flag = (int32_t*)buf;
  double2* packed = (double2*)(buf + 256);
  int32_t hflag = 0;
  auto read_flag = [&]() -> int {
    TOR_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TOR_HIP(hipStreamSynchronize(s));
    return TOR_OK;
  };
  auto run = [&]() -> int {
    TOR_HIP(launch_zero_words((uint32_t*)flag, 1, s));
    TOR_HIP(launch_mcmc_check(proposals, uniforms, total, N, M, flag, s));
    TOR_TRY(read_flag());
    if (hflag) return TOR_EINVAL;
    tor_options_t o;
    memset(&o, 0, sizeof(o));
    o.algo = TOR_ALGO_AUTO;
    o.split_depth = -1;
    if (opt) o = *opt;
    o.flags &= ~TOR_FLAG_GRAPH;  // every chunk has its own output range
    std::vector<int64_t> offs((size_t)chunk);
    std::vector<int32_t> ns((size_t)chunk, N), ts((size_t)chunk, tier);
    for (int64_t k = 0; k < chunk; ++k) offs[(size_t)k] = k * per;
    for (int64_t c0 = 0; c0 < total; c0 += chunk) {
      const int cnt = (int)std::min<int64_t>(chunk, total - c0);
      TOR_HIP(launch_mcmc_gather((const double2*)O_full, ld, M, proposals, N, c0, cnt, packed, s));
      TOR_TRY(tor_eval_batched(packed, offs.data(), ns.data(), cnt, ts.data(), tau, &o, stream,
                               cand_out + c0));
    }
    TOR_HIP(launch_mcmc_scan(cand_out, uniforms, chains, steps, state_step, flag, s));
    TOR_TRY(read_flag());
    return hflag & 4 ? TOR_ENOTPD : TOR_OK;
  };
  const int rc = run();
  (void)hipStreamSynchronize(s);  // nothing may still read the buffer
  (void)hipFree(buf);
  return rc;
}

int tor_select_tiers(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                     double tau, void* stream, int32_t* tiers, double* log10_kappa,
                     int32_t* source) {
  if (batch < 0 || !(tau > 0.0)) return TOR_EINVAL;
  if (batch == 0) return TOR_OK;
  if (!O_packed || !offsets || !n || !tiers) return TOR_EINVAL;
  for (int k = 0; k < batch; ++k)
    if (n[k] < 0 || n[k] > TOR_NMAX || offsets[k] < 0) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  TOR_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> tier_of(batch, TOR_AUTO);
  std::vector<double> pred;
  std::vector<int32_t> src;
  TOR_TRY(select_tiers(w, O_packed, offsets, n, batch, tau, tier_of.data(), &pred, &src, s));
  for (int k = 0; k < batch; ++k) {
    tiers[k] = n[k] == 0 ? TOR_FP64 : tier_of[k];
    if (log10_kappa) log10_kappa[k] = pred[k];
    if (source) source[k] = src[k];
  }
  return TOR_OK;
}

int tor_autotune(int32_t n, int32_t tier, void* stream, int32_t* best_bottom, double* ms) {
  if (n < 1 || n > TOR_NMAX || (tier != TOR_FP64 && tier != TOR_DD && tier != TOR_QD)) return TOR_EINVAL;
  load_default_tune_table();  // the result below overrides the shipped entry
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  // the shape the evaluations of this n run as: up to n = 24 a batch group
  // of R copies of one instance (the work does not depend on the values;
  // a thermal product O = 0.25 I), larger n one instance, timed on a share
  // of its depth-D_s frontier of about 2^28 subsets and scaled to the whole
  const int R = n <= AUTOTUNE_GROUP_NMAX ? AUTOTUNE_GROUP : 1;
  const size_t per = (size_t)4 * n * n;  // complex elements of one O
  std::vector<double> h(2 * per * R, 0.0);
  for (int r = 0; r < R; ++r)
    for (int i = 0; i < 2 * n; ++i) h[2 * (per * r + (size_t)i * 2 * n + i)] = 0.25;
  double* dO = nullptr;
  TOR_HIP(hipMalloc((void**)&dO, sizeof(double) * h.size()));
  int rc = hip_err(hipMemcpy(dO, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
  std::vector<int64_t> offs(R);
  std::vector<int32_t> ns(R, n), ts(R, tier), idx(R);
  for (int r = 0; r < R; ++r) {
    offs[r] = (int64_t)(per * r);
    idx[r] = r;
  }
  tor_result_t* dres = nullptr;
  if (rc == TOR_OK) rc = hip_err(hipMalloc((void**)&dres, sizeof(tor_result_t) * R));
  hipEvent_t ea = nullptr, eb = nullptr;
  if (rc == TOR_OK) rc = hip_err(hipEventCreate(&ea));
  if (rc == TOR_OK) rc = hip_err(hipEventCreate(&eb));
  const int cand_max = tier == TOR_FP64 ? 6 : (tier == TOR_DD ? 5 : 3);
  int best = 0;
  double best_ms = 1e300;
  for (int sb = 1; sb <= 6; ++sb) {
    if (ms) ms[sb - 1] = -1.0;
    if (rc != TOR_OK || sb > cand_max || sb > n) continue;
    tor_options_t o;
    memset(&o, 0, sizeof(o));
    o.algo = TOR_ALGO_SCHUR;
    o.split_depth = -1;
    o.bottom_modes = sb;
    // one run: the whole batch group, or the share [0, cnt) of the frontier
    double scale = 1.0;
    auto run = [&]() -> int {
      if (R > 1) return batch_core(w, dO, offs.data(), ns.data(), idx, ts, &o, dres, false, s);
      SchurPlan p;
      plan_schur(tier, n, 1, sb, &p);
      TOR_TRY(ensure_cap(w, p.bytes));
      const int sub = n - p.D_s;  // subsets per frontier state: 2^sub
      size_t cnt = sub >= 28 ? 1 : ((size_t)1 << (28 - sub));
      cnt = std::max(cnt, (size_t)p.Cr);
      cnt = std::min(cnt, p.Ns);
      scale = (double)p.Ns / (double)cnt;
      return enqueue_schur_group(w, w->buf, w->cus, p, dO, nullptr, 2 * (int64_t)n, &o, nullptr, dres, false, s, 0,
                                 cnt);
    };
    double tot = 0.0;
    for (int rep = 0; rep < 3 && rc == TOR_OK; ++rep) {
      rc = hip_err(hipEventRecord(ea, s));
      if (rc == TOR_OK) rc = run();
      if (rc == TOR_OK) rc = hip_err(hipEventRecord(eb, s));
      if (rc == TOR_OK) rc = hip_err(hipEventSynchronize(eb));
      float t = 0.0f;
      if (rc == TOR_OK) rc = hip_err(hipEventElapsedTime(&t, ea, eb));
      if (rep > 0) tot += t;  // the first run warms up
    }
    if (rc != TOR_OK) break;
    const double t = tot / 2.0 * scale;
    if (ms) ms[sb - 1] = t;
    if (t < best_ms) {
      best_ms = t;
      best = sb;
    }
  }
  (void)hipStreamSynchronize(s);
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  if (dres) (void)hipFree(dres);
  (void)hipFree(dO);
  if (rc != TOR_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_pair((int)n, (int)tier)] = best;
  }
  if (best_bottom) *best_bottom = best;
  return TOR_OK;
}

int tor_autotune_save(const char* path) {
  if (!path) return TOR_EINVAL;
  load_default_tune_table();
  FILE* f = fopen(path, "w");
  if (!f) return TOR_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tuned) fprintf(f, "%d %d %d\n", kv.first.first, kv.first.second, kv.second);
  return fclose(f) == 0 ? TOR_OK : TOR_EINVAL;
}

int tor_autotune_load(const char* path) {
  load_default_tune_table();  // a later load overrides the shipped table
  return load_tune_table(path);
}

}  // extern "C"

namespace tor {
namespace {
int load_tune_table(const char* path) {
  if (!path) return TOR_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return TOR_EINVAL;
  std::map<std::pair<int, int>, int> t;
  int a, b, c, rc = TOR_OK;
  while (fscanf(f, "%d %d %d", &a, &b, &c) == 3) {
    if (a < 1 || a > TOR_NMAX || b < TOR_FP64 || b > TOR_QD || c < 1 || c > 6) rc = TOR_EINVAL;
    t[std::make_pair(a, b)] = c;
  }
  fclose(f);
  if (rc != TOR_OK) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : t) g_tuned[kv.first] = kv.second;
  return TOR_OK;
}
}  // namespace
}  // namespace tor

extern "C" {

int tor_last_select_stats(tor_select_stats_t* o) {
  if (!o) return TOR_EINVAL;
  std::lock_guard<std::mutex> lk(g_sel_mu);
  *o = g_stats;
  return TOR_OK;
}

int tor_selector_set(const tor_selector_t* sel) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  if (sel) {
    if (sel->trained) {
      for (int i = 0; i < TOR_NFEAT; ++i)
        if (!(sel->std[i] > 0.0)) return TOR_EINVAL;
      if (sel->nmin < 1 || sel->nmax < sel->nmin || sel->nmax > TOR_NMAX) return TOR_EINVAL;
      if (sel->target != TOR_TARGET_KAPPA && sel->target != TOR_TARGET_ERR64) return TOR_EINVAL;
      for (int t = 0; t < 3; ++t)
        if (sel->target == TOR_TARGET_KAPPA && !(sel->slope[t] > 0.0 && sel->slope[t] <= 2.0)) return TOR_EINVAL;
    }
    g_sel = *sel;
  } else {
    memset(&g_sel, 0, sizeof(g_sel));
  }
  ++g_sel_version;
  return TOR_OK;
}

int tor_selector_get(tor_selector_t* sel) {
  if (!sel) return TOR_EINVAL;
  std::lock_guard<std::mutex> lk(g_sel_mu);
  *sel = g_sel;
  return TOR_OK;
}

int tor_selector_save(const char* path) {
  if (!path) return TOR_EINVAL;
  tor_selector_t sel;
  TOR_TRY(tor_selector_get(&sel));
  FILE* f = fopen(path, "w");
  if (!f) return TOR_EINVAL;
  auto arr = [&](const char* name, const double* v, int cnt) {
    fprintf(f, "%s %d", name, cnt);
    for (int i = 0; i < cnt; ++i) fprintf(f, " %.17g", v[i]);
    fprintf(f, "\n");
  };
  fprintf(f, "tor_selector 3\n");
  arr("theta", sel.theta, TOR_MLP_PARAMS);
  arr("mean", sel.mean, TOR_NFEAT);
  arr("std", sel.std, TOR_NFEAT);
  arr("fmin", sel.fmin, TOR_NFEAT);
  arr("fmax", sel.fmax, TOR_NFEAT);
  arr("log10_c", sel.log10_c, 3);
  arr("slope", sel.slope, 3);
  arr("margin", &sel.margin, 1);
  fprintf(f, "nrange %d %d\ntrained %d\ntarget %d\n", sel.nmin, sel.nmax, sel.trained, sel.target);
  const int ok = fclose(f) == 0;
  return ok ? TOR_OK : TOR_EINVAL;
}

int tor_selector_load(const char* path) {
  if (!path) return TOR_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return TOR_EINVAL;
  tor_selector_t sel;
  memset(&sel, 0, sizeof(sel));
  char name[64];
  int version = 0, rc = TOR_OK;
  // version 3: TOR_NFEAT = 20 features and the network's target; older
  // files hold networks of 12 features and are refused
  if (fscanf(f, "%63s %d", name, &version) != 2 || strcmp(name, "tor_selector") != 0 || version != 3)
    rc = TOR_EINVAL;
  auto arr = [&](const char* want, double* v, int cnt) {
    int c = 0;
    if (rc != TOR_OK) return;
    if (fscanf(f, "%63s %d", name, &c) != 2 || strcmp(name, want) != 0 || c != cnt) {
      rc = TOR_EINVAL;
      return;
    }
    for (int i = 0; i < cnt; ++i)
      if (fscanf(f, "%lf", &v[i]) != 1) rc = TOR_EINVAL;
  };
  arr("theta", sel.theta, TOR_MLP_PARAMS);
  arr("mean", sel.mean, TOR_NFEAT);
  arr("std", sel.std, TOR_NFEAT);
  arr("fmin", sel.fmin, TOR_NFEAT);
  arr("fmax", sel.fmax, TOR_NFEAT);
  arr("log10_c", sel.log10_c, 3);
  arr("slope", sel.slope, 3);
  arr("margin", &sel.margin, 1);
  if (rc == TOR_OK && fscanf(f, "%63s %d %d", name, &sel.nmin, &sel.nmax) != 3) rc = TOR_EINVAL;
  if (rc == TOR_OK && fscanf(f, "%63s %d", name, &sel.trained) != 2) rc = TOR_EINVAL;
  if (rc == TOR_OK && fscanf(f, "%63s %d", name, &sel.target) != 2) rc = TOR_EINVAL;
  fclose(f);
  if (rc != TOR_OK) return rc;
  return tor_selector_set(&sel);
}

double tor_fallback_bits(const double* feats, double tau) { return fallback_bits(feats, tau); }

int tor_features(const void* O_packed, const int64_t* offsets, const int32_t* n, int32_t batch,
                 void* stream, double* feats) {
  if (batch < 0) return TOR_EINVAL;
  if (batch == 0) return TOR_OK;
  if (!O_packed || !offsets || !n || !feats) return TOR_EINVAL;
  int nmax = 1;
  for (int k = 0; k < batch; ++k) {
    if (n[k] < 1 || n[k] > TOR_NMAX || offsets[k] < 0) return TOR_EINVAL;
    nmax = std::max(nmax, (int)n[k]);
  }
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  TOR_HIP(hipStreamSynchronize(s));
  std::vector<char> meta(sizeof(int64_t) * batch + sizeof(int32_t) * batch);
  memcpy(meta.data(), offsets, sizeof(int64_t) * batch);
  memcpy(meta.data() + sizeof(int64_t) * batch, n, sizeof(int32_t) * batch);
  TOR_TRY(upload_meta(w, meta.data(), meta.size(), s));
  TOR_HIP(launch_features((const double2*)O_packed, (const int64_t*)w->meta,
                          (const int32_t*)(w->meta + sizeof(int64_t) * batch), batch, nmax, feats, s));
  return TOR_OK;
}

int tor_mlp_forward(const double* theta, const double* mean, const double* std, const double* X,
                    int32_t B, void* stream, double* Y) {
  if (B < 0 || (B > 0 && (!theta || !mean || !std || !X || !Y))) return TOR_EINVAL;
  TOR_HIP(launch_mlp_forward(theta, mean, std, X, B, Y, (hipStream_t)stream));
  return TOR_OK;
}

int tor_mlp_grad(const double* theta, const double* mean, const double* std, const double* X,
                 const double* y, int32_t B, double under, double over, void* stream, double* grad,
                 double* loss) {
  if (B <= 0 || !theta || !mean || !std || !X || !y || !grad) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  const size_t need = sizeof(double) * ((size_t)B * TOR_MLP_PARAMS + B);
  TOR_TRY(ensure_aux(w, need, s));
  double* G = (double*)w->aux;
  double* lossb = G + (size_t)B * TOR_MLP_PARAMS;
  TOR_HIP(launch_mlp_grad(theta, mean, std, X, y, B, 0, under, over, G, lossb, grad, loss, s));
  return TOR_OK;
}

int tor_mlp_grad_quantile(const double* theta, const double* mean, const double* std, const double* X,
                          const double* y, int32_t B, double q, void* stream, double* grad, double* loss) {
  if (B <= 0 || !theta || !mean || !std || !X || !y || !grad || !(q > 0.0 && q < 1.0)) return TOR_EINVAL;
  Workspace* w = nullptr;
  TOR_TRY(get_ws(&w));
  hipStream_t s = (hipStream_t)stream;
  const size_t need = sizeof(double) * ((size_t)B * TOR_MLP_PARAMS + B);
  TOR_TRY(ensure_aux(w, need, s));
  double* G = (double*)w->aux;
  double* lossb = G + (size_t)B * TOR_MLP_PARAMS;
  TOR_HIP(launch_mlp_grad(theta, mean, std, X, y, B, 1, q, 0.0, G, lossb, grad, loss, s));
  return TOR_OK;
}

int tor_mlp_adam(double* theta, const double* grad, double* m, double* v, double lr, double beta1,
                 double beta2, double eps, int32_t step, void* stream) {
  if (!theta || !grad || !m || !v || step < 1) return TOR_EINVAL;
  TOR_HIP(launch_adam(theta, grad, m, v, lr, beta1, beta2, eps, step, (hipStream_t)stream));
  return TOR_OK;
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
  for (int m = 0; m <= n; ++m) {
    prec::qd v{{0.0, 0.0, 0.0, 0.0}};
    for (int k = 0; k < per && k < 4; ++k) v.x[k] = w->host_lev[per * m + k];
    if (per == 4) v = prec::qd_nonoverlapping(v);
    for (int k = 0; k < 4; ++k) out_levels[4 * m + k] = v.x[k];
  }
  return out->status;
}

int tor_debug_phase_clocks(int32_t reset, uint64_t* out) {
  if (!out) return TOR_EINVAL;
  const hipError_t e = phase_clocks(reset != 0, out);
  if (e == hipErrorNotSupported) return TOR_EUNSUPPORTED;
  TOR_HIP(e);
  return TOR_OK;
}

int tor_debug_level_sums_schur(const void* O, int32_t n, int64_t ld, int32_t tier, void* stream,
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
  SchurPlan p;
  plan_schur(tier, n, 1, level_sb_max(tier), &p);
  int occ = 0;
  TOR_HIP(leaf_levels_occupancy(tier, p.s_b, &occ));
  if (occ < 1) return TOR_EUNSUPPORTED;
  const size_t ab = acc_bytes(tier), cols = (size_t)n + 1;
  const size_t grid = std::min((size_t)occ * w->cus, p.mids);
  Carver c;
  c.off = p.bytes;
  const size_t o_part = c.take(ab * cols * grid), o_chunks = c.take(ab * cols * p.nchunks);
  const size_t o_out = c.take(ab * cols);
  const size_t o_sc = c.take(reduce_scratch_bytes(tier, (int)std::max(grid, (size_t)p.nchunks), (int)cols));
  TOR_TRY(ensure_cap(w, c.off));
  LevelOut lv{w->buf + o_part, w->buf + o_chunks, w->buf + o_out, w->buf + o_sc};
  tor_result_t* dres = (tor_result_t*)(w->buf + p.o_res);
  w->ev_pairs = 0;
  TOR_TRY(enqueue_schur_group(w, w->buf, w->cus, p, O, nullptr, ld, nullptr, nullptr, dres, false, s, 0, SIZE_MAX,
                              &lv));
  TOR_HIP(hipMemcpyAsync(w->host_res, dres, sizeof(tor_result_t), hipMemcpyDeviceToHost, s));
  TOR_HIP(hipMemcpyAsync(w->host_lev, lv.out, ab * cols, hipMemcpyDeviceToHost, s));
  TOR_HIP(hipStreamSynchronize(s));
  *out = *w->host_res;
  const int per = (int)(ab / sizeof(double));
  for (int m = 0; m <= n; ++m) {
    prec::qd v{{0.0, 0.0, 0.0, 0.0}};
    for (int k = 0; k < per && k < 4; ++k) v.x[k] = w->host_lev[per * m + k];
    if (per == 4) v = prec::qd_nonoverlapping(v);
    for (int k = 0; k < 4; ++k) out_levels[4 * m + k] = v.x[k];
  }
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
