// Host side of libmpcpcg: argument validation, workspace, schedules, launches, graphs.
// The C ABI is declared in include/mpcpcg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mpcpcg.h"
#include "pcg_kernel.h"
#include "ctrl_kernels.h"
#include "tri_kernel.h"
#include "wide_kernels.h"
#include "wide_pcg.h"

namespace {

using mpc::Gang;
using mpc::KArgs;
using mpc::ProbDesc;
using mpc::Task;

constexpr int kNX = 14, kNU = 7;        // register-resident fused path
constexpr int kWNX = 28, kWNU = 14;     // generic (workspace-staged) path
constexpr int kKpwChoices[] = {4, 8, 16, 24, 32, 48};

// Knots per workgroup of a single solve on a context with default settings: one workgroup
// when the horizon fits (no gang barrier; the smallest such shape has the cheapest workgroup
// barriers), else the smallest of 16, 32 and 48 whose gang has at most 32 parts (one XCD,
// one poll per barrier), else 32.  Measured on MI355X (us per N = 512 / 640 / 768 / 1024 /
// 1536 / 2048 solve): 16 knots 257 / 317 / 314 / 331 / 395 / -, 32 knots 273 / 288 / 278 /
// 287 / 402 / 408, 48 knots 317 / 335 / 321 / 328 / 338 / 453.
int default_single_kpw(int64_t N) {
  for (int k : kKpwChoices)
    if (N <= k) return k;
  for (int k : {16, 32, 48})
    if ((N + k - 1) / k <= 32) return k;
  return 32;
}
constexpr int kNumKpw = (int)(sizeof(kKpwChoices) / sizeof(kKpwChoices[0]));

// Device arrays owned by a cached schedule: freed with it.
struct DevArrays {
  std::vector<void *> ptrs;
  int64_t bytes = 0;
  DevArrays() = default;
  DevArrays(const DevArrays &) = delete;
  DevArrays &operator=(const DevArrays &) = delete;
  ~DevArrays() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  // device copy of n host elements (nullptr on failure)
  template <class T>
  T *upload(const T *src, size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (n ? n : 1)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    bytes += (int64_t)(sizeof(T) * (n ? n : 1));
    if (n && hipMemcpy(p, src, sizeof(T) * n, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return static_cast<T *>(p);
  }
};

// One schedule per (horizon signature, knots per workgroup): problem descriptors and the
// task list in longest-first order, resident on the device, plus the graph execs that
// replay the persistent launch for it ([mode][per-XCD lists used]).
struct Schedule {
  std::vector<int64_t> off;
  int kpw = 0;
  int ntasks = 0;
  int nprobs = 0;
  DevArrays mem;
  ProbDesc *d_probs = nullptr;
  ProbDesc *d_sorted = nullptr;  // the same descriptors, longest first (factorisation sweep)
  Task *d_tasks = nullptr;
  // the same tasks in eight per-XCD lists (batched PCG; nullptr when the batch does not
  // qualify), with their own problem descriptors (t0 indexes these lists)
  ProbDesc *d_xprobs = nullptr;
  Task *d_xtasks = nullptr;
  int32_t *d_xoff = nullptr;
  int xgrid = 0;
  hipGraph_t graph[4][2] = {};
  hipGraphExec_t exec[4][2] = {};
  hipGraphNode_t node[4][2] = {};
  KArgs args[4][2];
  int grid[4] = {0, 0, 0, 0};
  ~Schedule() {
    for (int m = 0; m < 4; ++m)
      for (int x = 0; x < 2; ++x) {
        if (exec[m][x]) (void)hipGraphExecDestroy(exec[m][x]);
        if (graph[m][x]) (void)hipGraphDestroy(graph[m][x]);
      }
  }
};

// chunks of the control-step kernels (linearisation, line search) for one horizon signature
struct CtrlSchedule {
  DevArrays mem;
  mpc::ctrl::Chunk *d_chunks = nullptr;
  int nchunks = 0;
};

// one captured control step per horizon signature: the graph is valid for the argument
// signature it was captured with
struct CtrlGraph {
  std::vector<uint64_t> sig;
  int calls = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~CtrlGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

struct WideSchedule {
  DevArrays mem;
  mpc::wide::KnotDesc *d_knots = nullptr;
  mpc::wide::ProbDescW *d_probs = nullptr;
  int nknots = 0, nprobs = 0, maxN = 0;
  // block tasks of the cyclic reduction: per level (stride 1, 2, 4, ...) the eliminated
  // blocks (also the back-substitution's) and the absorbing blocks; one root per problem
  std::vector<int> stride, n_odd, n_even;
  std::vector<int64_t> at_odd, at_even;  // offsets into d_tasks
  int64_t at_root = 0;
  mpc::wide::CrTask *d_tasks = nullptr;
  // tasks of the gang PCG: (problem, part) longest problem first, KW knots per part
  ProbDesc *d_gprobs = nullptr;
  Task *d_gtasks = nullptr;
  int gntasks = 0, gmax_parts = 0;
  // the same tasks in eight per-XCD lists (nullptr when a gang does not fit one XCD's share)
  ProbDesc *d_gxprobs = nullptr;
  Task *d_gxtasks = nullptr;
  int32_t *d_gxoff = nullptr;
};

// Schedule choice of the batched PCG launch for one horizon signature.
struct Tuned {
  int kpw = 16;
  int pin = 1;  // per-XCD task lists when the batch qualifies
};

// Least-recently-used map of per-signature state.  Values free what they own in their
// destructors; the context evicts the oldest entry before inserting beyond its limit.
template <class K, class V>
struct Lru {
  struct Ent {
    std::unique_ptr<V> v;
    uint64_t used = 0;
  };
  std::map<K, Ent> m;
  uint64_t tick = 0;
  V *get(const K &k) {
    auto it = m.find(k);
    if (it == m.end()) return nullptr;
    it->second.used = ++tick;
    return it->second.v.get();
  }
  V *put(const K &k, std::unique_ptr<V> v) {
    Ent &e = m[k];
    e.v = std::move(v);
    e.used = ++tick;
    return e.v.get();
  }
  typename std::map<K, Ent>::iterator oldest() {
    auto best = m.begin();
    for (auto it = m.begin(); it != m.end(); ++it)
      if (it->second.used < best->second.used) best = it;
    return best;
  }
  size_t size() const { return m.size(); }
};

using Sig = std::vector<int64_t>;

}  // namespace

struct mpcpcg_ctx {
  int nx = 0, nu = 0, device = 0, cus = 0;
  int64_t max_knots = 0;
  int max_batch = 0;
  int64_t max_tasks = 0;
  int kpw_override = 0;
  int fwd_cap[kNumKpw] = {};  // resident forward workgroups per shape of kKpwChoices (0: not queried yet)
  int use_graph = 1;
  // per-XCD task lists: only on a device that reports eight XCDs (one partition spanning
  // the whole MI355X), where workgroups are dispatched to the XCDs in turn
  int xcd_ok = 0;
  int xcd_pin = 1;  // batched PCG default placement when the batch qualifies
  int method = MPCPCG_METHOD_PCG;
  int64_t spin_ticks = 0;      // bound of every cross-workgroup wait (wall-clock ticks)
  int64_t clock_khz = 100000;  // wall-clock rate
  int stall = 0;               // test hook (mpcpcg_debug_set_wait)
  size_t cache_limit = 32;     // signatures kept per cache
  // factorisation path workspace (allocated on first use): S rows, rhs / y, D^-1, lambda
  double *f_s = nullptr, *f_rhs = nullptr, *f_dinv = nullptr, *f_lam = nullptr;
  int *f_flag = nullptr;  // breakdown flag of a split single solve (kept at 0 between solves)
  double *qinv_ws = nullptr, *rinv_ws = nullptr;
  void *tws = nullptr;
  Gang *gang = nullptr;
  int *queue = nullptr;
  Lru<std::pair<Sig, int>, Schedule> sched;
  Lru<Sig, Tuned> tuned;  // horizon signature -> batched PCG schedule choice
  // generic path (nx = 28)
  bool wide = false;
  double *w_S = nullptr, *w_Dinv = nullptr, *w_rhs = nullptr, *w_Qinv = nullptr, *w_RW = nullptr;
  double *w_lam = nullptr;  // lambda of the factorisation path
  int *w_flag = nullptr;    // per-problem breakdown flags of the factorisation path
  float *w_P = nullptr;
  void *w_tws = nullptr;  // tagged words of the gang PCG, one per task
  Gang *w_gang = nullptr;
  int *w_queue = nullptr;
  Lru<Sig, WideSchedule> wsched;
  // control step: chunk lists and the line search's per-chunk partial sums (on first use)
  Lru<Sig, CtrlSchedule> csched;
  double *ls_part = nullptr;
  // control step: the LQ problem and the step between its stages (on first use), graphs
  float *cs_ws = nullptr;
  hipStream_t cap_stream = nullptr;
  Lru<Sig, CtrlGraph> cgraph;
  std::string err;
};

namespace {

int fail(mpcpcg_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, MPCPCG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

using KernelFn = void (*)(KArgs);

const Sig &sig_of(const Sig &k) { return k; }
const Sig &sig_of(const std::pair<Sig, int> &k) { return k.first; }

// Makes room for one more entry in a cache of per-signature state by evicting the least
// recently used entries.  A captured control step may hold the device arrays of an evicted
// schedule, so the control-step graph of the same signature goes with it (drop_graphs).
// The device is synchronised first: a launch still in flight may read what is freed.
template <class Cache>
void make_room(mpcpcg_ctx *c, Cache &cache, bool drop_graphs) {
  if (cache.size() < c->cache_limit) return;
  (void)hipDeviceSynchronize();
  while (cache.size() > 0 && cache.size() >= c->cache_limit) {
    auto it = cache.oldest();
    if (drop_graphs) {
      auto g = c->cgraph.m.find(sig_of(it->first));
      if (g != c->cgraph.m.end()) c->cgraph.m.erase(g);
    }
    cache.m.erase(it);
  }
}

// launch mode of the adjoint that reads the forward's factor record (phase 3 of the
// adjoint kernel) beside mpc::kForm / kForward / kAdjoint
constexpr int kAdjointKept = 3;

template <int KPW>
KernelFn kernel_for(int mode) {
  switch (mode) {
    case mpc::kForm: return mpc::pcg_kernel<kNX, kNU, KPW, mpc::kForm>;
    case mpc::kForward: return mpc::pcg_kernel<kNX, kNU, KPW, mpc::kForward>;
    case kAdjointKept: return mpc::pcg_kernel<kNX, kNU, KPW, mpc::kAdjoint, 3>;
    default: return mpc::pcg_kernel<kNX, kNU, KPW, mpc::kAdjoint>;
  }
}

// formation-only (phase 1) and epilogue-only (phase 2) kernels of the factorisation path,
// built for 16 knots per workgroup
KernelFn phase_kernel(int mode, int phase) {
  if (mode == mpc::kForward)
    return phase == 1 ? mpc::pcg_kernel<kNX, kNU, 16, mpc::kForward, 1> : mpc::pcg_kernel<kNX, kNU, 16, mpc::kForward, 2>;
  return phase == 1 ? mpc::pcg_kernel<kNX, kNU, 16, mpc::kAdjoint, 1> : mpc::pcg_kernel<kNX, kNU, 16, mpc::kAdjoint, 2>;
}

KernelFn kernel_for(int kpw, int mode) {
  switch (kpw) {
    case 4: return kernel_for<4>(mode);
    case 8: return kernel_for<8>(mode);
    case 16: return kernel_for<16>(mode);
    case 24: return kernel_for<24>(mode);
    case 48: return kernel_for<48>(mode);
    default: return kernel_for<32>(mode);
  }
}

bool valid_kpw(int k) {
  for (int c : kKpwChoices)
    if (c == k) return true;
  return false;
}

// Workgroups of the fused kernel counted as resident on one compute unit at once.  The
// occupancy query counts registers per compute unit, but a workgroup's waves go to the four
// SIMDs in turn, so one of W waves takes ceil(W / 4) wave slots on some SIMD; at
// waves_per_eu slots per SIMD that allows waves_per_eu / ceil(W / 4) workgroups.  For 24
// knots (6 waves at three per SIMD) this gives one where the query reports two, and the
// measurements agree with one: the batched 24-knot launch on 256 x N = 512 runs 2.3x
// slower than the 16-knot one at the same knots per compute unit by the query, and a single
// solve of 43 parts of 24 knots placed on one XCD (32 compute units) timed out waiting for
// parts that never started.
int resident_per_cu(int occupancy, int kpw) {
  const int waves = kpw * mpc::kGroup / 64;
  const int per_simd = kpw == 32 ? 2 : 3;  // the kernel's waves per SIMD (waves_per_eu)
  const int by_simd = waves <= 4 ? per_simd * (4 / waves) : per_simd / ((waves + 3) / 4);
  return std::min(occupancy, by_simd);
}

// resident workgroups of this kernel on the whole device
int capacity(mpcpcg_ctx *c, int kpw, int mode, int *out) {
  int nb = 0;
  HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(kernel_for(kpw, mode)), kpw * mpc::kGroup, 0));
  *out = resident_per_cu(nb, kpw) * c->cus;
  return MPCPCG_OK;
}

size_t tws_bytes() { return sizeof(mpc::TaskWS<kNX>); }

int check_problem_ptrs(mpcpcg_ctx *c, const mpcpcg_problem *p, bool need_ctrl) {
  if (!p) return fail(c, MPCPCG_EINVAL, "problem is NULL");
  if (p->nx != c->nx || p->nu != c->nu)
    return fail(c, MPCPCG_EINVAL, "problem (nx, nu) = (%d, %d) differs from the context (%d, %d)",
                p->nx, p->nu, c->nx, c->nu);
  if (!p->Q || !p->q || !p->x0) return fail(c, MPCPCG_EINVAL, "Q, q and x0 must be non-NULL");
  if (need_ctrl && (!p->R || !p->A || !p->B || !p->r))
    return fail(c, MPCPCG_EINVAL, "R, A, B and r must be non-NULL when a horizon exceeds one knot");
  return MPCPCG_OK;
}

int check_opts(mpcpcg_ctx *c, const mpcpcg_opts *o) {
  if (!o) return fail(c, MPCPCG_EINVAL, "opts is NULL");
  if (!(o->eps >= 0.0f) || o->max_iter < 0)
    return fail(c, MPCPCG_EINVAL, "eps must be >= 0 and max_iter >= 0");
  if (o->stop_rule != MPCPCG_STOP_RELATIVE && o->stop_rule != MPCPCG_STOP_ABSOLUTE)
    return fail(c, MPCPCG_EINVAL, "stop_rule must be MPCPCG_STOP_RELATIVE or MPCPCG_STOP_ABSOLUTE");
  return MPCPCG_OK;
}

KArgs base_args(mpcpcg_ctx *c, const mpcpcg_problem *p, const mpcpcg_opts *o) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.Q = p->Q; a.R = p->R; a.A = p->A; a.B = p->B;
  a.q = p->q; a.r = p->r; a.x0 = p->x0; a.e = p->e;
  a.tws = c->tws; a.gang = c->gang; a.queue = c->queue;
  a.qinv_ws = c->qinv_ws; a.rinv_ws = c->rinv_ws;
  if (o) { a.eps = o->eps; a.max_iter = o->max_iter; a.warm = o->warm_start; a.stop_abs = o->stop_rule; }
  a.spin_limit = c->spin_ticks;
  a.stall = c->stall;
  return a;
}

int single_kpw(mpcpcg_ctx *c, int N) {
  if (c->kpw_override) return c->kpw_override;
  return default_single_kpw(N);
}

int launch_single(mpcpcg_ctx *c, KArgs &a, int N, int kpw, int mode, hipStream_t s) {
  const int g = (N + kpw - 1) / kpw;
  int cap = 0;
  int st = capacity(c, kpw, mode, &cap);
  if (st) return st;
  if (g > cap)
    return fail(c, MPCPCG_EINVAL, "horizon N=%d needs %d co-resident workgroups; the device holds %d", N, g, cap);
  if (g > c->max_tasks) return fail(c, MPCPCG_EINVAL, "N=%d exceeds the context's task workspace", N);
  a.single.k0 = 0; a.single.N = N; a.single.t0 = 0; a.single.nparts = g; a.single.id = 0;
  a.probs = nullptr; a.tasks = nullptr; a.ntasks = g; a.persistent = 0;
  // a gang that fits one XCD's share of the device runs there: launch 8 workgroups per
  // part; the ones running on XCD 0 take the parts and the loop barriers exchange through
  // that XCD's L2
  a.one_xcd = (c->xcd_ok && c->xcd_pin && g > 1 && 8 * g <= cap) ? 1 : 0;
  a.l2x = a.one_xcd;
  hipLaunchKernelGGL(kernel_for(kpw, mode), dim3(a.one_xcd ? 8 * g : g), dim3(kpw * mpc::kGroup), 0, s, a);
  HIPCHK(c, hipGetLastError());
  return MPCPCG_OK;
}

int validate_batch(mpcpcg_ctx *c, int batch, const int64_t *off, const mpcpcg_problem *p) {
  if (batch < 1) return fail(c, MPCPCG_EINVAL, "batch must be >= 1");
  if (batch > c->max_batch) return fail(c, MPCPCG_EINVAL, "batch %d exceeds the context limit %d", batch, c->max_batch);
  if (!off) return fail(c, MPCPCG_EINVAL, "knot_off is NULL");
  if (off[0] != 0) return fail(c, MPCPCG_EINVAL, "knot_off[0] must be 0");
  bool ctrl = false;
  for (int b = 0; b < batch; ++b) {
    const int64_t n = off[b + 1] - off[b];
    if (n < 1) return fail(c, MPCPCG_EINVAL, "problem %d has N=%lld < 1", b, (long long)n);
    if (n > (int64_t)1 << 30) return fail(c, MPCPCG_EINVAL, "problem %d horizon too long", b);
    if (n > 1) ctrl = true;
  }
  if (off[batch] > c->max_knots)
    return fail(c, MPCPCG_EINVAL, "total knots %lld exceed the context limit %lld", (long long)off[batch], (long long)c->max_knots);
  return check_problem_ptrs(c, p, ctrl);
}

// Schedule of the batched PCG launch for a signature: a fixed shape if one is set, else the
// autotuned choice, else 16 knots per workgroup with the context's default placement.
// Default shape of a batch with no tuned choice: 16 knots per workgroup (three workgroups
// per compute unit) unless the longest horizon needs more than 32 parts of 16 knots, where
// every barrier then polls twice.  Then 32 or 48 knots (one workgroup per compute unit) may
// cost fewer rounds x iteration time; the estimate takes every problem as the longest, the
// gangs that fit one XCD's share at once, and 1.27x the iteration time for two polls, as
// measured on MI355X (forward ms, 16 / 32 knots: 4 x N = 1024 0.349 / 0.307, 48 x N = 1024
// 2.22 / 1.74, 8 x N = 768 0.334 / 0.301, 32 x N = 768 0.771 / 1.142).
int default_batch_kpw(mpcpcg_ctx *c, const Sig &off) {
  const int B = (int)off.size() - 1;
  int64_t nmax = 0;
  for (int b = 0; b < B; ++b) nmax = std::max(nmax, off[b + 1] - off[b]);
  if ((nmax + 15) / 16 <= 32) return 16;
  int best = 16;
  double best_cost = 0.0;
  for (int i = 0; i < kNumKpw; ++i) {
    const int k = kKpwChoices[i];
    if (k != 16 && k != 32 && k != 48) continue;
    if (!c->fwd_cap[i] && capacity(c, k, mpc::kForward, &c->fwd_cap[i]) != MPCPCG_OK) return 16;
    const int64_t g = (nmax + k - 1) / k;
    const int64_t per_xcd = c->fwd_cap[i] / 8;
    if (g > per_xcd || per_xcd < 1) continue;
    const int64_t at_once = 8 * (per_xcd / g);
    const double cost = (double)((B + at_once - 1) / at_once) * (g > 32 ? 1.27 : 1.0);
    if (best_cost == 0.0 || cost < best_cost) {
      best = k;
      best_cost = cost;
    }
  }
  return best;
}

Tuned pick(mpcpcg_ctx *c, const Sig &off) {
  Tuned t;
  t.pin = c->xcd_pin;
  if (c->kpw_override) {
    t.kpw = c->kpw_override;
    return t;
  }
  if (const Tuned *u = c->tuned.get(off)) return *u;
  t.kpw = default_batch_kpw(c, off);
  return t;
}

int pick_kpw(mpcpcg_ctx *c, const Sig &off) { return pick(c, off).kpw; }

int get_schedule(mpcpcg_ctx *c, const std::vector<int64_t> &off, int kpw, Schedule **out) {
  auto key = std::make_pair(off, kpw);
  if (Schedule *hit = c->sched.get(key)) { *out = hit; return MPCPCG_OK; }
  const int B = (int)off.size() - 1;
  // longest-processing-time first: every problem runs ~the same number of iterations, so
  // its work is proportional to N; parts of one problem stay adjacent in the queue so a
  // gang is always completed by the next free workgroups
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return off[x + 1] - off[x] > off[y + 1] - off[y];
  });
  std::vector<ProbDesc> probs(B), sorted;
  std::vector<Task> tasks;
  for (int b : order) {
    ProbDesc d;
    d.k0 = off[b];
    d.N = (int32_t)(off[b + 1] - off[b]);
    d.nparts = (d.N + kpw - 1) / kpw;
    d.t0 = (int32_t)tasks.size();
    d.id = b;
    probs[b] = d;
    sorted.push_back(d);
    for (int j = 0; j < d.nparts; ++j) tasks.push_back(Task{b, j});
  }
  if ((int64_t)tasks.size() > c->max_tasks)
    return fail(c, MPCPCG_EINVAL, "batch needs %zu workgroup tasks; the context holds %lld", tasks.size(), (long long)c->max_tasks);
  int cap = 0;
  int st = capacity(c, kpw, mpc::kForward, &cap);
  if (st) return st;
  for (int m : {(int)mpc::kAdjoint, kAdjointKept}) {
    int capb = 0;
    st = capacity(c, kpw, m, &capb);
    if (st) return st;
    cap = std::min(cap, capb);
  }
  for (const auto &d : probs)
    if (d.nparts > cap)
      return fail(c, MPCPCG_EINVAL, "a horizon of %d knots needs %d co-resident workgroups; the device holds %d", d.N, d.nparts, cap);
  auto s = std::make_unique<Schedule>();
  s->off = off;
  s->kpw = kpw;
  s->ntasks = (int)tasks.size();
  s->nprobs = B;
  s->d_probs = s->mem.upload(probs.data(), probs.size());
  s->d_sorted = s->mem.upload(sorted.data(), sorted.size());
  s->d_tasks = s->mem.upload(tasks.data(), tasks.size());
  if (!s->d_probs || !s->d_sorted || !s->d_tasks) {
    (void)hipGetLastError();
    return fail(c, MPCPCG_ENOMEM, "cannot allocate the schedule of a %d-problem batch", B);
  }
  for (int m = 0; m < 4; ++m) s->grid[m] = std::min(s->ntasks, cap);
  // Per-XCD lists: workgroups are dispatched to the eight XCDs in turn, so a grid of 8 m
  // workgroups puts m on each (at most cap / 8 of them resident).  When every gang fits in
  // cap / 8, each problem (in longest-first order) goes to the XCD with the least work so
  // far, and all parts of a gang run on one XCD (each workgroup reads its XCD from the
  // hardware and pops only that XCD's list).  Its loop barriers then exchange through that
  // XCD's L2.  A batch of fewer than eight problems leaves some lists empty; the grid gives
  // every XCD as many workgroups as the longest list has tasks, up to cap / 8.
  constexpr int kXcds = 8;
  int max_parts = 0;
  for (const auto &d : sorted) max_parts = std::max(max_parts, d.nparts);
  if (c->xcd_ok && cap % kXcds == 0 && max_parts <= cap / kXcds) {
    std::vector<std::vector<int>> lists(kXcds);
    std::vector<int64_t> load(kXcds, 0);
    for (const auto &d : sorted) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      lists[x].push_back(d.id);
      load[x] += d.N;
    }
    std::vector<ProbDesc> xprobs(probs);
    std::vector<Task> xtasks;
    std::vector<int32_t> xoff(kXcds + 1, 0);
    for (int x = 0; x < kXcds; ++x) {
      xoff[x] = (int32_t)xtasks.size();
      for (int b : lists[x]) {
        xprobs[b].t0 = (int32_t)xtasks.size();
        for (int j = 0; j < xprobs[b].nparts; ++j) xtasks.push_back(Task{b, j});
      }
    }
    xoff[kXcds] = (int32_t)xtasks.size();
    s->d_xprobs = s->mem.upload(xprobs.data(), xprobs.size());
    s->d_xtasks = s->mem.upload(xtasks.data(), xtasks.size());
    s->d_xoff = s->mem.upload(xoff.data(), xoff.size());
    if (!s->d_xprobs || !s->d_xtasks || !s->d_xoff) {
      (void)hipGetLastError();
      return fail(c, MPCPCG_ENOMEM, "cannot allocate the per-XCD lists of a %d-problem batch", B);
    }
    int longest = 0;
    for (int x = 0; x < kXcds; ++x) longest = std::max(longest, xoff[x + 1] - xoff[x]);
    s->xgrid = kXcds * std::min(longest, cap / kXcds);
  }
  make_room(c, c->sched, true);
  *out = c->sched.put(key, std::move(s));
  return MPCPCG_OK;
}

int ensure_factor_ws(mpcpcg_ctx *c) {
  if (c->f_s) return MPCPCG_OK;
  const size_t K = (size_t)c->max_knots;
  // blocks stored by columns padded to 16 rows (see fws_index)
  if (hipMalloc(&c->f_s, K * 3 * kNX * mpc::kGroup * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->f_rhs, K * kNX * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->f_dinv, K * kNX * mpc::kGroup * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->f_lam, K * kNX * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->f_flag, sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    for (double **q : {&c->f_s, &c->f_rhs, &c->f_dinv, &c->f_lam})
      if (*q) { (void)hipFree(*q); *q = nullptr; }
    if (c->f_flag) { (void)hipFree(c->f_flag); c->f_flag = nullptr; }
    return fail(c, MPCPCG_ENOMEM, "cannot allocate the factorisation workspace (%zu knots)", K);
  }
  HIPCHK(c, hipMemset(c->f_flag, 0, sizeof(int)));
  HIPCHK(c, hipDeviceSynchronize());
  return MPCPCG_OK;
}

// Whether a call takes the factorisation path: always for MPCPCG_METHOD_FACTOR; for
// MPCPCG_METHOD_AUTO by a cost model measured on MI355X (nx = 14, microseconds):
//   PCG: rounds of resident problems (12,288 knots each), each ~40 + iters x (2.1 + 0.7 f)
//        with f the fraction of the device the batch fills (2.2 us per iteration for one
//        N = 512 solve, ~318 us per round of 256 x N = 512); iters ~100 for cold starts and
//        ~45 for warm-started receding-horizon solves;
//   factorisation: its two parallel phases, ~25 + 58 per 12,288 knots, plus the cyclic
//        reduction, one workgroup per problem: ~25 + 0.55 N for the longest horizon alone,
//        up to 2.2x that when every CU holds a problem; a lone problem, whose first levels
//        spread over the device, ~49 + 20.5 (log2 N - 4) in all, against ~95 + 2.1 iters
//        for its PCG solve.
// The adjoint (warm = false) is priced as a cold solve.
bool use_factor(mpcpcg_ctx *c, const std::vector<int64_t> &off, bool warm) {
  if (c->method == MPCPCG_METHOD_PCG) return false;
  if (c->method == MPCPCG_METHOD_FACTOR) return true;
  if (c->wide) return true;  // the 28-state PCG runs one workgroup per problem: always slower
  const int64_t B = (int64_t)off.size() - 1;
  int64_t nmax = 0;
  for (int64_t b = 0; b < B; ++b) nmax = std::max(nmax, off[b + 1] - off[b]);
  const double knots = (double)off.back(), per_round = 12288.0;
  const double rounds = std::ceil(knots / per_round);
  const double fill = std::min(1.0, knots / per_round);
  const double iters = warm ? 45.0 : 100.0;
  const double t_pcg = rounds * (40.0 + iters * (2.1 + 0.7 * fill));
  // a lone solve also pays its launch and setup outside the rounds: ~95 us end to end
  // beside the iterations (warm N = 128 receding-horizon solves take ~0.19 ms at p50)
  if (B == 1) return 49.0 + 20.5 * std::max(0.0, std::log2((double)nmax) - 4.0) < 95.0 + iters * 2.1;
  const double load = 1.0 + 1.2 * (double)std::min<int64_t>(B, c->cus) / (double)c->cus;
  const double t_cr = (25.0 + 0.55 * (double)nmax) * load * std::ceil((double)B / (double)c->cus);
  const double t_fac = 25.0 + 58.0 * knots / per_round + t_cr;
  return t_fac < t_pcg;
}

int launch_phase(mpcpcg_ctx *c, KArgs a, int mode, int phase, Schedule *s, int N, hipStream_t stream) {
  constexpr int kpw = 16;
  KernelFn fn = phase_kernel(mode, phase);
  int nb = 0;
  HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(fn), kpw * mpc::kGroup, 0));
  const int cap = nb * c->cus;
  int grid;
  a.xoff = nullptr;  // the phases pop the global queue
  if (s) {
    a.probs = s->d_probs; a.tasks = s->d_tasks; a.ntasks = s->ntasks; a.persistent = 1;
    grid = std::min(s->ntasks, cap);
    int need = 0;
    for (int64_t b = 0; b + 1 < (int64_t)s->off.size(); ++b)
      need = std::max<int>(need, (int)((s->off[b + 1] - s->off[b] + kpw - 1) / kpw));
    if (need > cap) return fail(c, MPCPCG_EINVAL, "a horizon needs %d co-resident workgroups; the device holds %d", need, cap);
  } else {
    grid = (N + kpw - 1) / kpw;
    if (grid > cap) return fail(c, MPCPCG_EINVAL, "horizon N=%d needs %d co-resident workgroups; the device holds %d", N, grid, cap);
    a.single.k0 = 0; a.single.N = N; a.single.t0 = 0; a.single.nparts = grid; a.single.id = 0;
    a.probs = nullptr; a.tasks = nullptr; a.ntasks = grid; a.persistent = 0;
  }
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kpw * mpc::kGroup), 0, stream, a);
  HIPCHK(c, hipGetLastError());
  return MPCPCG_OK;
}

// Factorisation path: formation to the workspace (phase 1), the block cyclic reduction of
// every problem, then the epilogue from the solved lambda (phase 2).  s == nullptr: one
// problem of N knots.
int run_factor(mpcpcg_ctx *c, KArgs a, int mode, Schedule *s, int N, hipStream_t stream) {
  int st = ensure_factor_ws(c);
  if (st) return st;
  const int64_t knots = s ? s->off.back() : N;
  if (!s && (N + 15) / 16 > c->max_tasks) return fail(c, MPCPCG_EINVAL, "N=%d exceeds the context's task workspace", N);
  if (knots > c->max_knots) return fail(c, MPCPCG_EINVAL, "knots exceed the context limit");
  a.s_ws = c->f_s; a.rhs_ws = c->f_rhs; a.lam_ws = c->f_lam;
  if ((st = launch_phase(c, a, mode, 1, s, N, stream))) return st;
  mpc::TriArgs t;
  std::memset(&t, 0, sizeof t);
  t.s_ws = c->f_s; t.rhs_ws = c->f_rhs; t.dinv_ws = c->f_dinv; t.lam_ws = c->f_lam;
  t.stats = a.stats;
  t.s0 = 1;
  t.flag = c->f_flag;
  if (s && s->nprobs > 1) {
    t.probs = s->d_sorted; t.nprobs = s->nprobs;
  } else {
    // a lone problem (a single solve or a batch of one): the levels with more block tasks
    // than one workgroup holds run as one launch per sub-step over the device, the rest
    // in one workgroup
    const int n1 = s ? (int)(s->off[1] - s->off[0]) : N;
    t.probs = nullptr; t.nprobs = 1;
    t.single.k0 = 0; t.single.N = n1; t.single.t0 = 0; t.single.nparts = 1; t.single.id = 0;
    while ((n1 - 1) / (2 * t.s0) + 1 > mpc::kCrGroups) t.s0 *= 2;
  }
  const int n1 = t.single.N;
  auto grid = [](int n) { return dim3((n + mpc::kCrGroups - 1) / mpc::kCrGroups); };
  auto n_odd = [n1](int sl) { return (n1 - sl + 2 * sl - 1) / (2 * sl); };
  for (int sl = 1; sl < t.s0; sl *= 2) {
    hipLaunchKernelGGL((mpc::cr_level<kNX, mpc::kLvlOdd>), grid(n_odd(sl)), dim3(mpc::kCrThreads), 0, stream, t, sl);
    hipLaunchKernelGGL((mpc::cr_level<kNX, mpc::kLvlEven>), grid((n1 - 1) / (2 * sl) + 1), dim3(mpc::kCrThreads), 0,
                       stream, t, sl);
  }
  hipLaunchKernelGGL(mpc::cr_solve<kNX>, dim3(t.nprobs), dim3(mpc::kCrThreads), 0, stream, t);
  if (t.s0 > 1) {
    for (int sl = t.s0 / 2; sl >= 1; sl /= 2)
      hipLaunchKernelGGL((mpc::cr_level<kNX, mpc::kLvlBack>), grid(n_odd(sl)), dim3(mpc::kCrThreads), 0, stream, t, sl);
    hipLaunchKernelGGL(mpc::cr_finish<kNX>, dim3(1), dim3(mpc::kCrThreads), 0, stream, t);
  }
  HIPCHK(c, hipGetLastError());
  return launch_phase(c, a, mode, 2, s, N, stream);
}

int launch_batched(mpcpcg_ctx *c, Schedule *s, KArgs &a, int mode, int want_pin, hipStream_t stream) {
  const bool pin = want_pin && s->d_xoff != nullptr;
  const int x = pin ? 1 : 0;
  a.probs = pin ? s->d_xprobs : s->d_probs;
  a.tasks = pin ? s->d_xtasks : s->d_tasks;
  a.xoff = pin ? s->d_xoff : nullptr;
  a.l2x = pin ? 1 : 0;  // a gang's workgroups all pop their XCD's list
  a.ntasks = s->ntasks;
  a.persistent = 1;
  const int grid = pin ? s->xgrid : s->grid[mode];
  const dim3 block(s->kpw * mpc::kGroup);
  if (!c->use_graph) {
    hipLaunchKernelGGL(kernel_for(s->kpw, mode), dim3(grid), block, 0, stream, a);
    HIPCHK(c, hipGetLastError());
    return MPCPCG_OK;
  }
  void *params[] = {&s->args[mode][x]};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof kp);
  kp.func = reinterpret_cast<void *>(kernel_for(s->kpw, mode));
  kp.gridDim = dim3(grid);
  kp.blockDim = block;
  kp.sharedMemBytes = 0;
  kp.kernelParams = params;
  kp.extra = nullptr;
  if (!s->exec[mode][x]) {
    s->args[mode][x] = a;
    HIPCHK(c, hipGraphCreate(&s->graph[mode][x], 0));
    HIPCHK(c, hipGraphAddKernelNode(&s->node[mode][x], s->graph[mode][x], nullptr, 0, &kp));
    HIPCHK(c, hipGraphInstantiate(&s->exec[mode][x], s->graph[mode][x], nullptr, nullptr, 0));
  } else if (std::memcmp(&s->args[mode][x], &a, sizeof a) != 0) {
    s->args[mode][x] = a;
    HIPCHK(c, hipGraphExecKernelNodeSetParams(s->exec[mode][x], s->node[mode][x], &kp));
  }
  HIPCHK(c, hipGraphLaunch(s->exec[mode][x], stream));
  return MPCPCG_OK;
}

// ---------------------------------------------------------------- generic path (nx = 28)
constexpr int kWKnots = mpc::wide::kGangKnots;  // knots per workgroup of the gang PCG

int64_t wide_max_tasks(const mpcpcg_ctx *c) { return c->max_knots / kWKnots + c->max_batch; }

int wide_schedule(mpcpcg_ctx *c, const std::vector<int64_t> &off, WideSchedule **out) {
  if (WideSchedule *hit = c->wsched.get(off)) { *out = hit; return MPCPCG_OK; }
  const int B = (int)off.size() - 1;
  std::vector<mpc::wide::KnotDesc> kd;
  std::vector<mpc::wide::ProbDescW> pd(B);
  int maxN = 0;
  for (int b = 0; b < B; ++b) {
    const int N = (int)(off[b + 1] - off[b]);
    maxN = std::max(maxN, N);
    pd[b] = mpc::wide::ProbDescW{off[b], N, b};
    for (int k = 0; k < N; ++k) kd.push_back(mpc::wide::KnotDesc{off[b], N, k, b, 0});
  }
  auto w = std::make_unique<WideSchedule>();
  w->nknots = (int)kd.size();
  w->nprobs = B;
  w->maxN = maxN;
  // gang PCG: problems longest first, the parts of a problem adjacent (a gang is always
  // completed by the next free workgroups)
  {
    std::vector<int> order(B);
    for (int b = 0; b < B; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pd[x].N > pd[y].N; });
    std::vector<ProbDesc> gp(B);
    std::vector<Task> gt;
    for (int b : order) {
      ProbDesc d;
      d.k0 = off[b];
      d.N = pd[b].N;
      d.nparts = (d.N + kWKnots - 1) / kWKnots;
      d.t0 = (int32_t)gt.size();
      d.id = b;
      gp[b] = d;
      w->gmax_parts = std::max(w->gmax_parts, d.nparts);
      for (int j = 0; j < d.nparts; ++j) gt.push_back(Task{b, j});
    }
    if ((int64_t)gt.size() > wide_max_tasks(c)) return fail(c, MPCPCG_EINVAL, "batch exceeds the gang workspace");
    w->gntasks = (int)gt.size();
    w->d_gprobs = w->mem.upload(gp.data(), gp.size());
    w->d_gtasks = w->mem.upload(gt.data(), gt.size());
    if (!w->d_gprobs || !w->d_gtasks) {
      (void)hipGetLastError();
      return fail(c, MPCPCG_ENOMEM, "cannot allocate the gang schedule of a %d-problem batch", B);
    }
    // Per-XCD lists (as for the 14-state batches): each problem, longest first, goes to the
    // XCD with the least work, and a workgroup pops only the list of the XCD it runs on, so
    // a gang's parts share that XCD's L2 for their barriers.  Needs every gang to fit the
    // cap / 8 workgroups of one XCD; XCDs left without problems just exit.
    int nb = 0;
    HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &nb, reinterpret_cast<const void *>(mpc::wide::wide_pcg_gang<kWNX, kWKnots>), kWKnots * 64, 0));
    const int cap = nb * c->cus;
    constexpr int kXcds = 8;
    if (c->xcd_ok && cap % kXcds == 0 && w->gmax_parts <= cap / kXcds) {
      std::vector<std::vector<int>> lists(kXcds);
      std::vector<int64_t> load(kXcds, 0);
      for (int b : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lists[x].push_back(b);
        load[x] += pd[b].N;
      }
      std::vector<ProbDesc> xp(gp);
      std::vector<Task> xt;
      std::vector<int32_t> xoff(kXcds + 1, 0);
      for (int x = 0; x < kXcds; ++x) {
        xoff[x] = (int32_t)xt.size();
        for (int b : lists[x]) {
          xp[b].t0 = (int32_t)xt.size();
          for (int j = 0; j < xp[b].nparts; ++j) xt.push_back(Task{b, j});
        }
      }
      xoff[kXcds] = (int32_t)xt.size();
      w->d_gxprobs = w->mem.upload(xp.data(), xp.size());
      w->d_gxtasks = w->mem.upload(xt.data(), xt.size());
      w->d_gxoff = w->mem.upload(xoff.data(), xoff.size());
      if (!w->d_gxprobs || !w->d_gxtasks || !w->d_gxoff) {
        (void)hipGetLastError();
        return fail(c, MPCPCG_ENOMEM, "cannot allocate the per-XCD gang lists of a %d-problem batch", B);
      }
    }
  }
  std::vector<mpc::wide::CrTask> tasks;
  for (int s = 1; s < maxN; s *= 2) {
    w->stride.push_back(s);
    w->at_odd.push_back((int64_t)tasks.size());
    for (int b = 0; b < B; ++b)
      for (int j = s; j < pd[b].N; j += 2 * s) tasks.push_back(mpc::wide::CrTask{b, j});
    w->n_odd.push_back((int)((int64_t)tasks.size() - w->at_odd.back()));
    w->at_even.push_back((int64_t)tasks.size());
    for (int b = 0; b < B; ++b)
      if (pd[b].N > s)
        for (int i = 0; i < pd[b].N; i += 2 * s) tasks.push_back(mpc::wide::CrTask{b, i});
    w->n_even.push_back((int)((int64_t)tasks.size() - w->at_even.back()));
  }
  w->at_root = (int64_t)tasks.size();
  for (int b = 0; b < B; ++b) tasks.push_back(mpc::wide::CrTask{b, 0});
  w->d_tasks = w->mem.upload(tasks.data(), tasks.size());
  w->d_knots = w->mem.upload(kd.data(), kd.size());
  w->d_probs = w->mem.upload(pd.data(), pd.size());
  if (!w->d_tasks || !w->d_knots || !w->d_probs) {
    (void)hipGetLastError();
    return fail(c, MPCPCG_ENOMEM, "cannot allocate the schedule of a %d-problem batch", B);
  }
  make_room(c, c->wsched, true);
  *out = c->wsched.put(off, std::move(w));
  return MPCPCG_OK;
}

mpc::wide::WArgs wide_args(mpcpcg_ctx *c, const mpcpcg_problem *p, const mpcpcg_opts *o) {
  mpc::wide::WArgs a;
  std::memset(&a, 0, sizeof a);
  a.Q = p->Q; a.R = p->R; a.A = p->A; a.B = p->B;
  a.q = p->q; a.r = p->r; a.x0 = p->x0; a.e = p->e;
  a.S = c->w_S; a.Dinv = c->w_Dinv; a.P = c->w_P; a.rhs = c->w_rhs; a.Qinv = c->w_Qinv; a.RW = c->w_RW;
  a.lamw = c->w_lam;
  if (o) { a.eps = o->eps; a.max_iter = o->max_iter; a.warm = o->warm_start; a.stop_abs = o->stop_rule; }
  return a;
}

// formation, preconditioner, then (unless form_only) PCG + epilogue
int wide_run(mpcpcg_ctx *c, const std::vector<int64_t> &off, mpc::wide::WArgs &a, bool form_only,
             hipStream_t s) {
  WideSchedule *w = nullptr;
  int st = wide_schedule(c, off, &w);
  if (st) return st;
  a.knots = w->d_knots;
  a.probs = w->d_probs;
  a.nknots = w->nknots;
  a.nprobs = w->nprobs;
  const bool fac = !form_only && use_factor(c, off, a.warm != 0);
  a.no_dinv = fac ? 1 : 0;
  {
    namespace mw = mpc::wide;
    const dim3 blk(mw::kFormWaves * 64);
    hipLaunchKernelGGL((mw::wide_form_inv<kWNX, kWNU>), dim3((2 * w->nknots + mw::kFormWaves - 1) / mw::kFormWaves),
                       blk, 0, s, a);
    hipLaunchKernelGGL((mw::wide_form_theta<kWNX, kWNU>), dim3((w->nknots + mw::kFormWaves - 1) / mw::kFormWaves),
                       blk, 0, s, a);
  }
  HIPCHK(c, hipGetLastError());
  if (!fac) {
    hipLaunchKernelGGL((mpc::wide::wide_precond<kWNX, kWNU>), dim3(w->nknots), dim3(256), 0, s, a);
    HIPCHK(c, hipGetLastError());
  }
  if (form_only) return MPCPCG_OK;
  if (fac) {
    // factorisation path: cyclic reduction, one launch per sub-step of a level over the
    // tasks of every problem, then the primal step (or adjoint gradients) per knot
    namespace mw = mpc::wide;
    const dim3 blk(mw::kCrWaves * 64);
    auto grid = [](int n) { return dim3((n + mw::kCrWaves - 1) / mw::kCrWaves); };
    hipLaunchKernelGGL(mw::wide_cr_init, dim3((w->nprobs + 255) / 256), dim3(256), 0, s, c->w_flag, w->nprobs);
    for (size_t l = 0; l < w->stride.size(); ++l) {
      if (w->n_odd[l])
        hipLaunchKernelGGL((mw::wide_cr_step<kWNX, mw::kCrOdd>), grid(w->n_odd[l]), blk, 0, s, a,
                           w->d_tasks + w->at_odd[l], w->n_odd[l], w->stride[l], c->w_flag);
      if (w->n_even[l])
        hipLaunchKernelGGL((mw::wide_cr_step<kWNX, mw::kCrEven>), grid(w->n_even[l]), blk, 0, s, a,
                           w->d_tasks + w->at_even[l], w->n_even[l], w->stride[l], c->w_flag);
    }
    hipLaunchKernelGGL((mw::wide_cr_step<kWNX, mw::kCrRoot>), grid(w->nprobs), blk, 0, s, a,
                       w->d_tasks + w->at_root, w->nprobs, 0, c->w_flag);
    for (size_t l = w->stride.size(); l-- > 0;)
      if (w->n_odd[l])
        hipLaunchKernelGGL((mw::wide_cr_step<kWNX, mw::kCrBack>), grid(w->n_odd[l]), blk, 0, s, a,
                           w->d_tasks + w->at_odd[l], w->n_odd[l], w->stride[l], c->w_flag);
    hipLaunchKernelGGL(mw::wide_cr_finish<kWNX>, dim3(w->nprobs), dim3(256), 0, s, a, (const int *)c->w_flag);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL((mw::wide_epilogue<kWNX, kWNU>), dim3((w->nknots + mw::kFormWaves - 1) / mw::kFormWaves),
                       dim3(mw::kFormWaves * 64), 0, s, a);
    HIPCHK(c, hipGetLastError());
    return MPCPCG_OK;
  }
  // PCG on gangs of workgroups (every gang co-resident), then the primal step or gradients
  {
    namespace mw = mpc::wide;
    auto fn = mw::wide_pcg_gang<kWNX, kWKnots>;
    int nb = 0;
    HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(fn), kWKnots * 64, 0));
    const int cap = nb * c->cus;
    if (w->gmax_parts > cap)
      return fail(c, MPCPCG_EINVAL, "a horizon needs %d co-resident workgroups; the device holds %d", w->gmax_parts, cap);
    mw::GangArgs ga;
    std::memset(&ga, 0, sizeof ga);
    ga.tws = c->w_tws; ga.gang = c->w_gang; ga.queue = c->w_queue;
    ga.ntasks = w->gntasks;
    ga.spin_limit = c->spin_ticks;
    int grid = std::min(w->gntasks, cap);
    if (w->d_gxoff && c->xcd_pin) {  // gangs on one XCD each: the full persistent grid
      ga.probs = w->d_gxprobs; ga.tasks = w->d_gxtasks; ga.xoff = w->d_gxoff; ga.l2x = 1;
      grid = cap;
    } else {
      ga.probs = w->d_gprobs; ga.tasks = w->d_gtasks;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kWKnots * 64), 0, s, a, ga);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL((mw::wide_epilogue<kWNX, kWNU>), dim3((w->nknots + mw::kFormWaves - 1) / mw::kFormWaves),
                       dim3(mw::kFormWaves * 64), 0, s, a);
    HIPCHK(c, hipGetLastError());
  }
  return MPCPCG_OK;
}

// ---- control step (linearisation, line search) ----------------------------------------

// Chunk length of the control-step kernels: short chunks spread a small batch over more
// workgroups (latency); long ones keep a large batch's per-workgroup overhead low.
constexpr int kCtrlShort = 8, kCtrlLong = mpc::ctrl::kMaxChunk;
constexpr int64_t kCtrlLongFrom = 16384;  // knots in the batch

int64_t ctrl_max_chunks(const mpcpcg_ctx *c) { return c->max_knots / kCtrlShort + c->max_batch; }

int ctrl_schedule(mpcpcg_ctx *c, const std::vector<int64_t> &off, CtrlSchedule **out) {
  if (CtrlSchedule *hit = c->csched.get(off)) { *out = hit; return MPCPCG_OK; }
  const int B = (int)off.size() - 1;
  const int len = off.back() >= kCtrlLongFrom ? kCtrlLong : kCtrlShort;
  std::vector<mpc::ctrl::Chunk> ch;
  for (int b = 0; b < B; ++b) {
    const int N = (int)(off[b + 1] - off[b]);
    const int nch = (N + len - 1) / len;
    const int c0 = (int)ch.size();
    for (int k = 0; k < N; k += len) {
      mpc::ctrl::Chunk x;
      x.pk0 = off[b]; x.b = b; x.N = N; x.lk0 = k; x.lk1 = std::min(N, k + len);
      x.c0 = c0; x.nch = nch;
      ch.push_back(x);
    }
  }
  if ((int64_t)ch.size() > ctrl_max_chunks(c)) return fail(c, MPCPCG_EINVAL, "batch exceeds the control-step workspace");
  auto cs = std::make_unique<CtrlSchedule>();
  cs->nchunks = (int)ch.size();
  cs->d_chunks = cs->mem.upload(ch.data(), ch.size());
  if (!cs->d_chunks) {
    (void)hipGetLastError();
    return fail(c, MPCPCG_ENOMEM, "cannot allocate the control-step chunk list");
  }
  make_room(c, c->csched, true);
  *out = c->csched.put(off, std::move(cs));
  return MPCPCG_OK;
}

int check_ctrl(mpcpcg_ctx *c, int batch, const int64_t *off, const mpcpcg_chain_model *m,
               const mpcpcg_trajectory *t, bool *ctrl) {
  if (batch < 1) return fail(c, MPCPCG_EINVAL, "batch must be >= 1");
  if (batch > c->max_batch) return fail(c, MPCPCG_EINVAL, "batch %d exceeds the context limit %d", batch, c->max_batch);
  if (!off) return fail(c, MPCPCG_EINVAL, "knot_off is NULL");
  if (off[0] != 0) return fail(c, MPCPCG_EINVAL, "knot_off[0] must be 0");
  *ctrl = false;
  for (int b = 0; b < batch; ++b) {
    const int64_t n = off[b + 1] - off[b];
    if (n < 1) return fail(c, MPCPCG_EINVAL, "problem %d has N=%lld < 1", b, (long long)n);
    if (n > (int64_t)1 << 30) return fail(c, MPCPCG_EINVAL, "problem %d horizon too long", b);
    if (n > 1) *ctrl = true;
  }
  if (off[batch] > c->max_knots)
    return fail(c, MPCPCG_EINVAL, "total knots %lld exceed the context limit %lld", (long long)off[batch], (long long)c->max_knots);
  if (!m || !t) return fail(c, MPCPCG_EINVAL, "model and trajectory must be non-NULL");
  if (t->nx != c->nx || t->nu != c->nu)
    return fail(c, MPCPCG_EINVAL, "trajectory (nx, nu) = (%d, %d) differs from the context (%d, %d)", t->nx, t->nu, c->nx, c->nu);
  if (!m->gravity) return fail(c, MPCPCG_EINVAL, "model gravity must be non-NULL");
  if (!std::isfinite(m->h) || !std::isfinite(m->damping) || !std::isfinite(m->coupling))
    return fail(c, MPCPCG_EINVAL, "model parameters must be finite");
  if (!t->X || !t->x_init || !t->xref || !t->Q) return fail(c, MPCPCG_EINVAL, "X, x_init, xref and Q must be non-NULL");
  if (*ctrl && (!t->U || !t->R)) return fail(c, MPCPCG_EINVAL, "U and R must be non-NULL when a horizon exceeds one knot");
  return MPCPCG_OK;
}

mpc::ctrl::CtrlArgs ctrl_args(const mpcpcg_chain_model *m, const mpcpcg_trajectory *t, const CtrlSchedule *cs) {
  mpc::ctrl::CtrlArgs a;
  std::memset(&a, 0, sizeof a);
  a.X = t->X; a.U = t->U; a.xs = t->x_init; a.xref = t->xref; a.Q = t->Q; a.R = t->R;
  a.grav = m->gravity; a.h = m->h; a.damp = m->damping; a.kap = m->coupling;
  a.chunks = cs->d_chunks; a.nchunks = cs->nchunks;
  return a;
}

// ---- allocation-free single solve (mpcpcg_solve_noalloc) -----------------------------
// Everything one single-problem PCG solve needs beyond its inputs and outputs: Q^-1 and
// (R^-1 | R^-1 B^T) by columns, the exchange words of the parts, one gang record and the
// launch queue, sized for horizons up to kNaMaxKnots.  The last three must be zero when a
// launch starts; every call clears the part of them it uses with a fill kernel on its
// stream (a kernel, not a memset, so the call may be captured into a graph).
constexpr int64_t kNaMaxKnots = 2048;
constexpr int kNaMaxParts = (int)(kNaMaxKnots / 16);  // horizons beyond 48 knots use 16 per part
constexpr size_t na_round(size_t n) { return (n + 255) / 256 * 256; }
constexpr size_t kNaQinv = na_round((size_t)kNaMaxKnots * kNX * mpc::kGroup * sizeof(double));
constexpr size_t kNaRinv = na_round((size_t)kNaMaxKnots * (kNU + kNX) * mpc::kURows * sizeof(double));
constexpr size_t kNaTws = na_round((size_t)kNaMaxParts * sizeof(mpc::TaskWS<kNX>));
constexpr size_t kNaGang = na_round(sizeof(Gang));
constexpr size_t kNaQueue = 256;
constexpr size_t kNaBytes = kNaQinv + kNaRinv + kNaTws + kNaGang + kNaQueue;
static_assert(sizeof(mpc::TaskWS<kNX>) % 16 == 0 && kNaQinv % 16 == 0 && kNaRinv % 16 == 0, "16-byte fill");

// Per device: the device address of `scratch` (each device holds its own copy of the
// array), resolved once with that device current, and the launch limits.
struct NaDevice {
  std::once_flag once;
  int rc = MPCPCG_OK;
  unsigned char *ptr = nullptr;
  int cap[kNumKpw] = {};  // co-resident workgroups per shape of kKpwChoices
  int xcd_ok = 0;
  int64_t spin = 0;
};
constexpr int kNaDevices = 64;
NaDevice g_na[kNaDevices];
thread_local std::string g_na_err;

int na_fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_na_err = buf;
  return code;
}

// zeroes [p, p + n16 * 16) and the n16b 16-byte words at q
__global__ void na_clear(uint4 *p, size_t n16, uint4 *q, size_t n16b) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16b; i += stride) q[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

// The scratch of mpcpcg_solve_noalloc (one copy per device, held until the process ends).
// In host code this name is not a device address: host code uses the per-device pointer
// that na_setup resolves with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

// Resolves this device's copy of `scratch` and the launch limits (once per device, with
// that device current).
void na_setup(NaDevice &d, int dev) {
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    d.rc = na_fail(MPCPCG_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    return;
  }
  d.ptr = static_cast<unsigned char *>(ptr);
  hipDeviceProp_t prop;
  int nxcc = 0, khz = 0;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    d.rc = na_fail(MPCPCG_EHIP, "hipGetDeviceProperties failed on device %d", dev);
    return;
  }
  if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess) nxcc = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
  (void)hipGetLastError();
  d.xcd_ok = (nxcc == 8 && prop.multiProcessorCount % 8 == 0) ? 1 : 0;
  d.spin = (int64_t)2000 * khz;  // 2 s
  for (int i = 0; i < kNumKpw; ++i) {
    const int k = kKpwChoices[i];
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(kernel_for(k, mpc::kForward)),
                                                     k * mpc::kGroup, 0) != hipSuccess) {
      (void)hipGetLastError();
      d.rc = na_fail(MPCPCG_EHIP, "occupancy query failed on device %d", dev);
      return;
    }
    d.cap[i] = resident_per_cu(nb, k) * prop.multiProcessorCount;
  }
}

}  // namespace

extern "C" {

int mpcpcg_create(mpcpcg_ctx **out, int32_t nx, int32_t nu, int64_t max_total_knots, int32_t max_batch) {
  if (!out) return MPCPCG_EINVAL;
  *out = nullptr;
  const bool wide = (nx == kWNX && nu == kWNU);
  if (!wide && (nx != kNX || nu != kNU)) return MPCPCG_EUNSUPPORTED;
  if (max_total_knots < 1 || max_batch < 1 || max_batch > max_total_knots) return MPCPCG_EINVAL;
  // the kernels address the parts' exchange records with 32-bit buffer offsets
  const int64_t records = wide ? (int64_t)sizeof(mpc::wide::WTag) * (max_total_knots / kWKnots + max_batch)
                               : (int64_t)tws_bytes() * (max_total_knots / 4 + max_batch);
  if (records > 0x7fffffff) return MPCPCG_EINVAL;
  auto c = std::make_unique<mpcpcg_ctx>();
  c->nx = nx;
  c->nu = nu;
  c->wide = wide;
  c->max_knots = max_total_knots;
  c->max_batch = max_batch;
  c->max_tasks = max_total_knots / 4 + max_batch;
  if (hipGetDevice(&c->device) != hipSuccess) return MPCPCG_EHIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return MPCPCG_EHIP;
  c->cus = prop.multiProcessorCount;
  int nxcc = 0, khz = 0;
  if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, c->device) != hipSuccess) nxcc = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || khz <= 0) khz = 100000;
  (void)hipGetLastError();
  c->xcd_ok = (nxcc == 8 && c->cus % 8 == 0) ? 1 : 0;
  c->clock_khz = khz;
  c->spin_ticks = (int64_t)2000 * khz;  // 2 s
  const size_t K = (size_t)max_total_knots;
  if (wide) {
    const size_t MM = (size_t)nx * nx;
    if (hipMalloc(&c->w_S, sizeof(double) * K * 3 * MM) != hipSuccess ||
        hipMalloc(&c->w_Dinv, sizeof(double) * K * MM) != hipSuccess ||
        hipMalloc(&c->w_P, sizeof(float) * K * 3 * MM) != hipSuccess ||
        hipMalloc(&c->w_rhs, sizeof(double) * K * nx) != hipSuccess ||
        hipMalloc(&c->w_lam, sizeof(double) * K * nx) != hipSuccess ||
        hipMalloc(&c->w_flag, sizeof(int) * (size_t)max_batch) != hipSuccess ||
        hipMalloc(&c->w_Qinv, sizeof(double) * K * MM) != hipSuccess ||
        hipMalloc(&c->w_RW, sizeof(double) * K * nu * (nu + nx)) != hipSuccess ||
        hipMalloc(&c->w_tws, sizeof(mpc::wide::WTag) * (size_t)wide_max_tasks(c.get())) != hipSuccess ||
        hipMalloc(&c->w_gang, sizeof(Gang) * (size_t)max_batch) != hipSuccess ||
        hipMalloc(&c->w_queue, 16 * sizeof(int)) != hipSuccess) {
      mpcpcg_destroy(c.release());
      return MPCPCG_ENOMEM;
    }
    if (hipMemset(c->w_tws, 0, sizeof(mpc::wide::WTag) * (size_t)wide_max_tasks(c.get())) != hipSuccess ||
        hipMemset(c->w_gang, 0, sizeof(Gang) * (size_t)max_batch) != hipSuccess ||
        hipMemset(c->w_queue, 0, 16 * sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      mpcpcg_destroy(c.release());
      return MPCPCG_EHIP;
    }
    *out = c.release();
    return MPCPCG_OK;
  }
  const size_t qb = sizeof(double) * K * nx * mpc::kGroup;        // Q^-1 by columns
  const size_t rb = sizeof(double) * K * (nu + nx) * mpc::kURows;  // (R^-1 | R^-1 B^T) by columns
  const size_t tb = tws_bytes() * (size_t)c->max_tasks;
  const size_t gb = sizeof(Gang) * (size_t)max_batch;
  if (hipMalloc(&c->qinv_ws, qb) != hipSuccess || hipMalloc(&c->rinv_ws, rb) != hipSuccess ||
      hipMalloc(&c->tws, tb) != hipSuccess || hipMalloc(&c->gang, gb) != hipSuccess ||
      hipMalloc(&c->queue, 16 * sizeof(int)) != hipSuccess) {
    mpcpcg_destroy(c.release());
    return MPCPCG_ENOMEM;
  }
  if (hipMemset(c->gang, 0, gb) != hipSuccess || hipMemset(c->queue, 0, 16 * sizeof(int)) != hipSuccess ||
      hipMemset(c->tws, 0, tb) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    mpcpcg_destroy(c.release());
    return MPCPCG_EHIP;
  }
  *out = c.release();
  return MPCPCG_OK;
}

int mpcpcg_destroy(mpcpcg_ctx *c) {
  if (!c) return MPCPCG_OK;
  (void)hipDeviceSynchronize();
  c->cgraph.m.clear();
  c->sched.m.clear();
  c->csched.m.clear();
  c->wsched.m.clear();
  for (double *q : {c->f_s, c->f_rhs, c->f_dinv, c->f_lam})
    if (q) (void)hipFree(q);
  if (c->f_flag) (void)hipFree(c->f_flag);
  if (c->qinv_ws) (void)hipFree(c->qinv_ws);
  if (c->rinv_ws) (void)hipFree(c->rinv_ws);
  if (c->tws) (void)hipFree(c->tws);
  if (c->gang) (void)hipFree(c->gang);
  if (c->queue) (void)hipFree(c->queue);
  if (c->ls_part) (void)hipFree(c->ls_part);
  if (c->cs_ws) (void)hipFree(c->cs_ws);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void *p : {(void *)c->w_S, (void *)c->w_Dinv, (void *)c->w_P, (void *)c->w_rhs, (void *)c->w_lam, (void *)c->w_Qinv,
                  (void *)c->w_RW, (void *)c->w_flag, c->w_tws, (void *)c->w_gang, (void *)c->w_queue})
    if (p) (void)hipFree(p);
  delete c;
  return MPCPCG_OK;
}

const char *mpcpcg_last_error(const mpcpcg_ctx *c) { return c ? c->err.c_str() : "null context"; }

int mpcpcg_form_schur(mpcpcg_ctx *c, const mpcpcg_problem *p, mpcpcg_schur *out, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  if (!p || !out) return fail(c, MPCPCG_EINVAL, "problem and out must be non-NULL");
  if (p->N < 1) return fail(c, MPCPCG_EINVAL, "N must be >= 1");
  if (p->N > c->max_knots) return fail(c, MPCPCG_EINVAL, "N exceeds the context limit");
  int st = check_problem_ptrs(c, p, p->N > 1);
  if (st) return st;
  if (c->wide) {
    if (!out->S || !out->Pinv || !out->gamma)
      return fail(c, MPCPCG_EINVAL, "the nx=28 path writes S, Pinv and gamma together: none may be NULL");
    mpc::wide::WArgs w = wide_args(c, p, nullptr);
    w.S_out = out->S; w.P_out = out->Pinv; w.gam_out = out->gamma;
    return wide_run(c, std::vector<int64_t>{0, p->N}, w, true, s);
  }
  KArgs a = base_args(c, p, nullptr);
  a.S_out = out->S;
  a.P_out = out->Pinv;
  a.gam_out = out->gamma;
  return launch_single(c, a, p->N, 16, mpc::kForm, s);
}

int mpcpcg_solve(mpcpcg_ctx *c, const mpcpcg_problem *p, const mpcpcg_opts *o, float *lambda,
                 float *dx, float *du, mpcpcg_stats *stats, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  if (!p) return fail(c, MPCPCG_EINVAL, "problem is NULL");
  if (p->N < 1) return fail(c, MPCPCG_EINVAL, "N must be >= 1");
  if (p->N > c->max_knots) return fail(c, MPCPCG_EINVAL, "N exceeds the context limit");
  int st = check_problem_ptrs(c, p, p->N > 1);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  if (!lambda || !dx || !stats || (p->N > 1 && !du))
    return fail(c, MPCPCG_EINVAL, "lambda, dx, du and stats must be non-NULL");
  if (c->wide) {
    mpc::wide::WArgs w = wide_args(c, p, o);
    w.lam = lambda; w.dx = dx; w.du = du; w.stats = stats;
    return wide_run(c, std::vector<int64_t>{0, p->N}, w, false, s);
  }
  KArgs a = base_args(c, p, o);
  a.lam = lambda; a.dx = dx; a.du = du; a.stats = stats;
  if (use_factor(c, std::vector<int64_t>{0, p->N}, o->warm_start != 0)) return run_factor(c, a, mpc::kForward, nullptr, p->N, s);
  return launch_single(c, a, p->N, single_kpw(c, p->N), mpc::kForward, s);
}

int mpcpcg_solve_batched(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_problem *p,
                         const mpcpcg_opts *o, float *lambda, float *dx, float *du,
                         mpcpcg_stats *stats, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  int st = validate_batch(c, batch, off, p);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  if (!lambda || !dx || !stats || (off[batch] > batch && !du))
    return fail(c, MPCPCG_EINVAL, "lambda, dx, du and stats must be non-NULL");
  std::vector<int64_t> key(off, off + batch + 1);
  if (c->wide) {
    mpc::wide::WArgs w = wide_args(c, p, o);
    w.lam = lambda; w.dx = dx; w.du = du; w.stats = stats;
    return wide_run(c, key, w, false, s);
  }
  const bool fac = use_factor(c, key, o->warm_start != 0);
  const Tuned tu = pick(c, key);
  Schedule *sc = nullptr;
  if ((st = get_schedule(c, key, fac ? 16 : tu.kpw, &sc))) return st;
  KArgs a = base_args(c, p, o);
  a.lam = lambda; a.dx = dx; a.du = du; a.stats = stats;
  if (fac) return run_factor(c, a, mpc::kForward, sc, 0, s);
  return launch_batched(c, sc, a, mpc::kForward, tu.pin, s);
}

int mpcpcg_backward(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_problem *p,
                    const mpcpcg_opts *o, const float *lambda, const float *dx, const float *du,
                    const float *gl, const float *gx, const float *gu, float *dQ, float *dR,
                    float *dA, float *dB, float *dq, float *dr, float *dx0, float *de,
                    float *dgamma, mpcpcg_stats *stats, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  int st = validate_batch(c, batch, off, p);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  const bool ctrl = off[batch] > batch;
  if (!lambda || !dx || !gl || !dQ || !dq || !dx0 || !stats)
    return fail(c, MPCPCG_EINVAL, "lambda, dx, dL_dlambda, dQ, dq, dx0 and stats must be non-NULL");
  if (ctrl && (!du || !dR || !dA || !dB || !dr))
    return fail(c, MPCPCG_EINVAL, "du, dR, dA, dB and dr must be non-NULL when a horizon exceeds one knot");
  std::vector<int64_t> key(off, off + batch + 1);
  if (c->wide) {
    mpc::wide::WArgs w = wide_args(c, p, o);
    w.warm = 0;
    w.adjoint = 1;
    w.lam_in = lambda; w.dx_in = dx; w.du_in = du;
    w.gl = gl; w.gx = gx; w.gu = gu;
    w.dQ = dQ; w.dR = dR; w.dA = dA; w.dB = dB; w.dq = dq; w.dr = dr; w.dx0 = dx0; w.de = de;
    w.dgamma = dgamma; w.stats = stats;
    return wide_run(c, key, w, false, s);
  }
  const bool fac = use_factor(c, key, false);  // the adjoint solve starts cold
  const Tuned tu = pick(c, key);
  Schedule *sc = nullptr;
  if ((st = get_schedule(c, key, fac ? 16 : tu.kpw, &sc))) return st;
  KArgs a = base_args(c, p, o);
  a.warm = 0;
  a.lam_in = lambda; a.dx_in = dx; a.du_in = du;
  a.gl = gl; a.gx = gx; a.gu = gu;
  a.dQ = dQ; a.dR = dR; a.dA = dA; a.dB = dB; a.dq = dq; a.dr = dr; a.dx0 = dx0; a.de = de;
  a.dgamma = dgamma; a.stats = stats;
  if (fac) return run_factor(c, a, mpc::kAdjoint, sc, 0, s);
  return launch_batched(c, sc, a, mpc::kAdjoint, tu.pin, s);
}

// Factor record of a forward solve, read back by its adjoint, for K knots: Phi^-1 (FP32) by
// columns in the factorisation workspace's layout, then the epilogue's Q^-1 and
// (R^-1 | R^-1 B^T) rows in the context workspace's layouts, each region 256-byte aligned.
struct FacLayout {
  int64_t p, q, r, total;
};
FacLayout fac_layout(int64_t K) {
  auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
  FacLayout L;
  L.p = 0;
  L.q = L.p + al(K * 3 * kNX * mpc::kGroup * (int64_t)sizeof(float));
  L.r = L.q + al(K * kNX * mpc::kGroup * (int64_t)sizeof(double));
  L.total = L.r + al(K * (kNU + kNX) * mpc::kURows * (int64_t)sizeof(double));
  return L;
}

void set_record(KArgs &a, const void *rec, int64_t K) {
  const FacLayout L = fac_layout(K);
  char *b = static_cast<char *>(const_cast<void *>(rec));
  a.fac_p = reinterpret_cast<float *>(b + L.p);
  a.qinv_ws = reinterpret_cast<double *>(b + L.q);
  a.rinv_ws = reinterpret_cast<double *>(b + L.r);
}

int check_record(mpcpcg_ctx *c, const void *rec) {
  if (c->wide) return fail(c, MPCPCG_EINVAL, "factor records are kept on the (14, 7) path only");
  if (!rec) return fail(c, MPCPCG_EINVAL, "factors is NULL");
  if (reinterpret_cast<uintptr_t>(rec) % 256) return fail(c, MPCPCG_EINVAL, "factors must be 256-byte aligned");
  return MPCPCG_OK;
}

int64_t mpcpcg_factor_bytes(const mpcpcg_ctx *c, int64_t total_knots) {
  if (!c || c->wide || total_knots < 1) return -1;
  return fac_layout(total_knots).total;
}

int mpcpcg_solve_batched_keep(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_problem *p,
                              const mpcpcg_opts *o, float *lambda, float *dx, float *du,
                              mpcpcg_stats *stats, void *factors, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  int st = validate_batch(c, batch, off, p);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  if (!lambda || !dx || !stats || (off[batch] > batch && !du))
    return fail(c, MPCPCG_EINVAL, "lambda, dx, du and stats must be non-NULL");
  if ((st = check_record(c, factors))) return st;
  std::vector<int64_t> key(off, off + batch + 1);
  const Tuned tu = pick(c, key);
  Schedule *sc = nullptr;
  if ((st = get_schedule(c, key, tu.kpw, &sc))) return st;
  KArgs a = base_args(c, p, o);
  a.lam = lambda; a.dx = dx; a.du = du; a.stats = stats;
  set_record(a, factors, off[batch]);
  a.fac_mode = 1;
  return launch_batched(c, sc, a, mpc::kForward, tu.pin, s);
}

int mpcpcg_backward_reuse(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_problem *p,
                          const mpcpcg_opts *o, const float *lambda, const float *dx, const float *du,
                          const float *gl, const float *gx, const float *gu, float *dQ, float *dR,
                          float *dA, float *dB, float *dq, float *dr, float *dx0, float *de,
                          float *dgamma, mpcpcg_stats *stats, const void *factors, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  int st = validate_batch(c, batch, off, p);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  const bool ctrl = off[batch] > batch;
  if (!lambda || !dx || !gl || !dQ || !dq || !dx0 || !stats)
    return fail(c, MPCPCG_EINVAL, "lambda, dx, dL_dlambda, dQ, dq, dx0 and stats must be non-NULL");
  if (ctrl && (!du || !dR || !dA || !dB || !dr))
    return fail(c, MPCPCG_EINVAL, "du, dR, dA, dB and dr must be non-NULL when a horizon exceeds one knot");
  if ((st = check_record(c, factors))) return st;
  std::vector<int64_t> key(off, off + batch + 1);
  const Tuned tu = pick(c, key);
  Schedule *sc = nullptr;
  if ((st = get_schedule(c, key, tu.kpw, &sc))) return st;
  KArgs a = base_args(c, p, o);
  a.warm = 0;
  a.lam_in = lambda; a.dx_in = dx; a.du_in = du;
  a.gl = gl; a.gx = gx; a.gu = gu;
  a.dQ = dQ; a.dR = dR; a.dA = dA; a.dB = dB; a.dq = dq; a.dr = dr; a.dx0 = dx0; a.de = de;
  a.dgamma = dgamma; a.stats = stats;
  set_record(a, factors, off[batch]);
  return launch_batched(c, sc, a, kAdjointKept, tu.pin, s);
}

int mpcpcg_set_knots_per_group(mpcpcg_ctx *c, int32_t k) {
  if (!c) return MPCPCG_EINVAL;
  if (k != 0 && !valid_kpw(k)) return fail(c, MPCPCG_EINVAL, "knots per group must be 0, 4, 8, 16 or 32");
  c->kpw_override = k;
  return MPCPCG_OK;
}

int mpcpcg_set_method(mpcpcg_ctx *c, int32_t method) {
  if (!c) return MPCPCG_EINVAL;
  if (method != MPCPCG_METHOD_PCG && method != MPCPCG_METHOD_FACTOR && method != MPCPCG_METHOD_AUTO)
    return fail(c, MPCPCG_EINVAL, "method must be MPCPCG_METHOD_PCG, _FACTOR or _AUTO");
  c->method = method;
  return MPCPCG_OK;
}

int mpcpcg_set_graph(mpcpcg_ctx *c, int32_t enable) {
  if (!c) return MPCPCG_EINVAL;
  c->use_graph = enable ? 1 : 0;
  return MPCPCG_OK;
}

int mpcpcg_autotune(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_problem *p,
                    const mpcpcg_opts *o, float *lambda, float *dx, float *du, mpcpcg_stats *stats,
                    hipStream_t s, int32_t *kpw_out) {
  if (!c) return MPCPCG_EINVAL;
  int st = validate_batch(c, batch, off, p);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  if (o->warm_start) return fail(c, MPCPCG_EINVAL, "autotune runs cold solves (warm_start must be 0)");
  if (c->wide) {  // one workgroup shape on the nx=28 path
    if (kpw_out) *kpw_out = 0;
    return MPCPCG_OK;
  }
  const Sig key(off, off + batch + 1);
  // the trials run PCG with a fixed shape and placement; the context's settings and the
  // events are restored / released on every exit
  struct Guard {
    mpcpcg_ctx *c;
    int kpw, pin, method;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Guard() {
      c->kpw_override = kpw;
      c->xcd_pin = pin;
      c->method = method;
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } g{c, c->kpw_override, c->xcd_pin, c->method};
  HIPCHK(c, hipEventCreate(&g.e0));
  HIPCHK(c, hipEventCreate(&g.e1));
  c->method = MPCPCG_METHOD_PCG;
  std::vector<mpcpcg_stats> hst((size_t)batch);
  Tuned best;
  best.kpw = 0;
  float best_ms = 0.f;
  for (int k : kKpwChoices) {
    Schedule *sc = nullptr;
    if (get_schedule(c, key, k, &sc) != MPCPCG_OK) continue;  // shape cannot hold a horizon
    for (int pin = 0; pin < 2; ++pin) {
      if (pin && !sc->d_xoff) continue;  // the batch does not qualify for per-XCD lists
      c->kpw_override = k;
      c->xcd_pin = pin;
      float ms_min = 0.f;
      bool ok = true;
      for (int rep = 0; rep < 4 && ok; ++rep) {
        HIPCHK(c, hipEventRecord(g.e0, s));
        if (mpcpcg_solve_batched(c, batch, off, p, o, lambda, dx, du, stats, s) != MPCPCG_OK) ok = false;
        HIPCHK(c, hipEventRecord(g.e1, s));
        HIPCHK(c, hipEventSynchronize(g.e1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, g.e0, g.e1));
        if (rep > 0 && (ms_min == 0.f || ms < ms_min)) ms_min = ms;
      }
      if (!ok) continue;
      // a shape whose solves broke down or timed out does not qualify
      HIPCHK(c, hipMemcpy(hst.data(), stats, sizeof(mpcpcg_stats) * (size_t)batch, hipMemcpyDeviceToHost));
      for (const auto &x : hst)
        if (x.status == MPCPCG_BREAKDOWN || x.status == MPCPCG_TIMEOUT) ok = false;
      if (ok && (best.kpw == 0 || ms_min < best_ms)) {
        best.kpw = k;
        best.pin = pin;
        best_ms = ms_min;
      }
    }
  }
  if (!best.kpw) return fail(c, MPCPCG_EINVAL, "no workgroup shape can run this batch");
  make_room(c, c->tuned, false);
  c->tuned.put(key, std::make_unique<Tuned>(best));
  if (kpw_out) *kpw_out = best.kpw;
  return MPCPCG_OK;
}

int mpcpcg_tuned_schedule(mpcpcg_ctx *c, int32_t batch, const int64_t *off, int32_t *kpw_out,
                          int32_t *pinned_out) {
  if (!c) return MPCPCG_EINVAL;
  if (batch < 1 || !off || off[0] != 0) return fail(c, MPCPCG_EINVAL, "batch must be >= 1 and knot_off[0] = 0");
  for (int b = 0; b < batch; ++b)
    if (off[b + 1] - off[b] < 1) return fail(c, MPCPCG_EINVAL, "problem %d has N < 1", b);
  if (c->wide) {
    if (kpw_out) *kpw_out = 0;
    if (pinned_out) *pinned_out = 0;
    return MPCPCG_OK;
  }
  const Sig key(off, off + batch + 1);
  const Tuned t = pick(c, key);
  Schedule *sc = nullptr;
  int st = get_schedule(c, key, t.kpw, &sc);
  if (st) return st;
  if (kpw_out) *kpw_out = t.kpw;
  if (pinned_out) *pinned_out = (t.pin && sc->d_xoff) ? 1 : 0;
  return MPCPCG_OK;
}

int mpcpcg_set_xcd_pinning(mpcpcg_ctx *c, int32_t enable) {
  if (!c) return MPCPCG_EINVAL;
  c->xcd_pin = enable ? 1 : 0;
  return MPCPCG_OK;
}

int mpcpcg_set_cache_limit(mpcpcg_ctx *c, int32_t max_signatures) {
  if (!c) return MPCPCG_EINVAL;
  if (max_signatures < 1) return fail(c, MPCPCG_EINVAL, "the cache limit must be >= 1");
  c->cache_limit = (size_t)max_signatures;
  // trim every cache to the new limit (make_room leaves limit - 1 entries)
  c->cache_limit += 1;
  make_room(c, c->sched, true);
  make_room(c, c->wsched, true);
  make_room(c, c->csched, true);
  make_room(c, c->cgraph, false);
  make_room(c, c->tuned, false);
  c->cache_limit -= 1;
  return MPCPCG_OK;
}

int mpcpcg_cache_info(const mpcpcg_ctx *c, int32_t *entries, int64_t *device_bytes) {
  if (!c) return MPCPCG_EINVAL;
  int64_t bytes = 0;
  for (const auto &kv : c->sched.m) bytes += kv.second.v->mem.bytes;
  for (const auto &kv : c->wsched.m) bytes += kv.second.v->mem.bytes;
  for (const auto &kv : c->csched.m) bytes += kv.second.v->mem.bytes;
  if (entries)
    *entries = (int32_t)(c->sched.size() + c->wsched.size() + c->csched.size() + c->cgraph.size() + c->tuned.size());
  if (device_bytes) *device_bytes = bytes;
  return MPCPCG_OK;
}

int mpcpcg_debug_set_wait(mpcpcg_ctx *c, int64_t limit_us, int32_t inject_stall) {
  if (!c) return MPCPCG_EINVAL;
  if (limit_us < 1 || limit_us > (int64_t)600 * 1000000) return fail(c, MPCPCG_EINVAL, "limit_us must be in [1, 6e8]");
  c->spin_ticks = limit_us * c->clock_khz / 1000;
  if (c->spin_ticks < 1) c->spin_ticks = 1;
  c->stall = inject_stall ? 1 : 0;
  return MPCPCG_OK;
}

int mpcpcg_linearize(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_chain_model *m,
                     const mpcpcg_trajectory *t, float *A, float *B, float *q, float *r, float *x0,
                     float *e, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  bool ctrl = false;
  int st = check_ctrl(c, batch, off, m, t, &ctrl);
  if (st) return st;
  if (!q || !x0) return fail(c, MPCPCG_EINVAL, "q and x0 must be non-NULL");
  if (ctrl && (!A || !B || !r || !e))
    return fail(c, MPCPCG_EINVAL, "A, B, r and e must be non-NULL when a horizon exceeds one knot");
  CtrlSchedule *cs = nullptr;
  if ((st = ctrl_schedule(c, std::vector<int64_t>(off, off + batch + 1), &cs))) return st;
  mpc::ctrl::CtrlArgs a = ctrl_args(m, t, cs);
  a.A = A; a.B = B; a.q = q; a.r = r; a.x0 = x0; a.e = e;
  if (c->wide)
    hipLaunchKernelGGL(mpc::ctrl::linearize_kernel<kWNX>, dim3(cs->nchunks), dim3(mpc::ctrl::kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(mpc::ctrl::linearize_kernel<kNX>, dim3(cs->nchunks), dim3(mpc::ctrl::kThreads), 0, s, a);
  HIPCHK(c, hipGetLastError());
  return MPCPCG_OK;
}

int mpcpcg_line_search(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_chain_model *m,
                       const mpcpcg_trajectory *t, const float *dX, const float *dU, const float *lambda,
                       float mu, float *X_out, float *U_out, double *merit, int32_t *choice, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  bool ctrl = false;
  int st = check_ctrl(c, batch, off, m, t, &ctrl);
  if (st) return st;
  if (!(mu >= 0.0f) || !std::isfinite(mu)) return fail(c, MPCPCG_EINVAL, "mu must be finite and >= 0");
  if (!dX || !X_out || !merit || !choice) return fail(c, MPCPCG_EINVAL, "dX, X_out, merit and choice must be non-NULL");
  if (ctrl && (!dU || !U_out)) return fail(c, MPCPCG_EINVAL, "dU and U_out must be non-NULL when a horizon exceeds one knot");
  CtrlSchedule *cs = nullptr;
  if ((st = ctrl_schedule(c, std::vector<int64_t>(off, off + batch + 1), &cs))) return st;
  if (!c->ls_part)
    HIPCHK(c, hipMalloc(&c->ls_part, sizeof(double) * mpc::ctrl::kParts * (size_t)ctrl_max_chunks(c)));
  mpc::ctrl::CtrlArgs a = ctrl_args(m, t, cs);
  a.dX = dX; a.dU = dU; a.lam = lambda; a.mu = mu;
  a.part = c->ls_part; a.X_out = X_out; a.U_out = U_out; a.merit = merit; a.choice = choice;
  const dim3 g(cs->nchunks), blk(mpc::ctrl::kThreads);
  if (c->wide) {
    hipLaunchKernelGGL(mpc::ctrl::merit_kernel<kWNX>, g, blk, 0, s, a);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(mpc::ctrl::ls_update_kernel<kWNX>, g, blk, 0, s, a);
  } else {
    hipLaunchKernelGGL(mpc::ctrl::merit_kernel<kNX>, g, blk, 0, s, a);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(mpc::ctrl::ls_update_kernel<kNX>, g, blk, 0, s, a);
  }
  HIPCHK(c, hipGetLastError());
  return MPCPCG_OK;
}

// The stages of one control step, launched on `s`: for each SQP iteration, linearise at
// the current iterate, solve the LQ problem, line-search; iterations after the first read
// the iterate from X_out / U_out.
static int control_body(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_chain_model *m,
                        const mpcpcg_trajectory *t, const mpcpcg_opts *o, int32_t iters, float mu,
                        float *lambda, float *X_out, float *U_out, double *merit, int32_t *choice,
                        mpcpcg_stats *stats, hipStream_t s) {
  const size_t K = (size_t)c->max_knots, nx = c->nx, nu = c->nu;
  float *A = c->cs_ws, *B = A + K * nx * nx, *q = B + K * nx * nu, *r = q + K * nx;
  float *x0 = r + K * nu, *e = x0 + (size_t)c->max_batch * nx, *dx = e + K * nx, *du = dx + K * nx;
  mpcpcg_trajectory cur = *t;
  mpcpcg_problem p;
  p.nx = c->nx; p.nu = c->nu; p.N = t->N;
  p.Q = t->Q; p.R = t->R; p.A = A; p.B = B; p.q = q; p.r = r; p.x0 = x0; p.e = e;
  for (int it = 0; it < iters; ++it) {
    int st = mpcpcg_linearize(c, batch, off, m, &cur, A, B, q, r, x0, e, s);
    if (!st) st = mpcpcg_solve_batched(c, batch, off, &p, o, lambda, dx, du, stats, s);
    if (!st) st = mpcpcg_line_search(c, batch, off, m, &cur, dx, du, lambda, mu, X_out, U_out, merit, choice, s);
    if (st) return st;
    cur.X = X_out;
    cur.U = U_out;
  }
  return MPCPCG_OK;
}

int mpcpcg_control_step(mpcpcg_ctx *c, int32_t batch, const int64_t *off, const mpcpcg_chain_model *m,
                        const mpcpcg_trajectory *t, const mpcpcg_opts *o, int32_t sqp_iters, float mu,
                        float *lambda, float *X_out, float *U_out, double *merit, int32_t *choice,
                        mpcpcg_stats *stats, hipStream_t s) {
  if (!c) return MPCPCG_EINVAL;
  bool ctrl = false;
  int st = check_ctrl(c, batch, off, m, t, &ctrl);
  if (st) return st;
  if ((st = check_opts(c, o))) return st;
  if (sqp_iters < 1 || sqp_iters > 16) return fail(c, MPCPCG_EINVAL, "sqp_iters must be in [1, 16]");
  if (!(mu >= 0.0f) || !std::isfinite(mu)) return fail(c, MPCPCG_EINVAL, "mu must be finite and >= 0");
  if (!lambda || !X_out || !merit || !choice || !stats || (ctrl && !U_out))
    return fail(c, MPCPCG_EINVAL, "lambda, X_out, U_out, merit, choice and stats must be non-NULL");
  if (!c->cs_ws) {
    const size_t K = (size_t)c->max_knots, nx = c->nx, nu = c->nu;
    const size_t n = K * (nx * nx + nx * nu + 3 * nx + 2 * nu) + (size_t)c->max_batch * nx;
    if (hipMalloc(&c->cs_ws, sizeof(float) * n) != hipSuccess) {
      (void)hipGetLastError();
      c->cs_ws = nullptr;
      return fail(c, MPCPCG_ENOMEM, "cannot allocate the control-step workspace");
    }
  }
  if (!c->use_graph) return control_body(c, batch, off, m, t, o, sqp_iters, mu, lambda, X_out, U_out, merit, choice, stats, s);

  // everything the launches depend on, so that a replay is exactly a fresh call
  std::vector<int64_t> key(off, off + batch + 1);
  auto u64 = [](const void *p) { return (uint64_t)(uintptr_t)p; };
  auto f32 = [](float v) { uint32_t b; std::memcpy(&b, &v, 4); return (uint64_t)b; };
  std::vector<uint64_t> sig = {
      f32(m->h), f32(m->damping), f32(m->coupling), u64(m->gravity),
      u64(t->X), u64(t->U), u64(t->x_init), u64(t->xref), u64(t->Q), u64(t->R),
      f32(o->eps), (uint64_t)(uint32_t)o->max_iter, (uint64_t)o->warm_start, (uint64_t)o->stop_rule,
      (uint64_t)sqp_iters, f32(mu), u64(lambda), u64(X_out), u64(U_out), u64(merit), u64(choice), u64(stats),
      (uint64_t)c->method, (uint64_t)c->kpw_override, (uint64_t)pick_kpw(c, key)};
  CtrlGraph *g = c->cgraph.get(key);
  if (!g) {
    make_room(c, c->cgraph, false);
    g = c->cgraph.put(key, std::make_unique<CtrlGraph>());
  }
  if (g->sig != sig) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr; g->graph = nullptr; g->calls = 0; g->sig = sig;
  }
  if (g->exec) {
    HIPCHK(c, hipGraphLaunch(g->exec, s));
    return MPCPCG_OK;
  }
  if (g->calls++ == 0)  // the first call runs eagerly and creates every schedule and workspace
    return control_body(c, batch, off, m, t, o, sqp_iters, mu, lambda, X_out, U_out, merit, choice, stats, s);
  // Nothing may be allocated or freed while the launches are captured: make sure every
  // schedule the step uses is cached (another signature may have evicted one since the
  // first call).  None of these inserts evicts this signature's graph, which is the newest.
  {
    CtrlSchedule *cs = nullptr;
    if ((st = ctrl_schedule(c, key, &cs))) return st;
    if (c->wide) {
      WideSchedule *w = nullptr;
      if ((st = wide_schedule(c, key, &w))) return st;
    } else {
      const bool fac = use_factor(c, key, o->warm_start != 0);
      Schedule *sc = nullptr;
      if ((st = get_schedule(c, key, fac ? 16 : pick_kpw(c, key), &sc))) return st;
    }
    g = c->cgraph.get(key);
    if (!g) {  // dropped with an evicted schedule of the same horizons: start it afresh
      make_room(c, c->cgraph, false);
      g = c->cgraph.put(key, std::make_unique<CtrlGraph>());
      g->sig = sig;
      g->calls = 2;
    }
  }
  // the second captures the same launches on the context's own stream and replays them
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const int saved = c->use_graph;
  c->use_graph = 0;  // the solve's launches go into this graph, not into a graph of their own
  st = control_body(c, batch, off, m, t, o, sqp_iters, mu, lambda, X_out, U_out, merit, choice, stats, c->cap_stream);
  c->use_graph = saved;
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
  if (st || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (st) return st;
    return fail(c, MPCPCG_EHIP, "capturing the control step failed: %s", hipGetErrorString(ec));
  }
  g->graph = graph;
  HIPCHK(c, hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  HIPCHK(c, hipGraphLaunch(g->exec, s));
  return MPCPCG_OK;
}


const char *mpcpcg_noalloc_last_error(void) { return g_na_err.c_str(); }

int mpcpcg_solve_noalloc(const mpcpcg_problem *p, const mpcpcg_opts *o, float *lambda, float *dx, float *du,
                         mpcpcg_stats *stats, hipStream_t s) {
  g_na_err.clear();
  if (!p) return na_fail(MPCPCG_EINVAL, "problem is NULL");
  if (p->nx != kNX || p->nu != kNU) return na_fail(MPCPCG_EUNSUPPORTED, "only (nx, nu) = (14, 7) is supported");
  if (p->N < 1 || p->N > kNaMaxKnots)
    return na_fail(MPCPCG_EINVAL, "N = %d outside [1, %lld], the horizons the static scratch holds", p->N,
                   (long long)kNaMaxKnots);
  if (!p->Q || !p->q || !p->x0) return na_fail(MPCPCG_EINVAL, "Q, q and x0 must be non-NULL");
  if (p->N > 1 && (!p->R || !p->A || !p->B || !p->r))
    return na_fail(MPCPCG_EINVAL, "R, A, B and r must be non-NULL when N > 1");
  if (!o) return na_fail(MPCPCG_EINVAL, "opts is NULL");
  if (!(o->eps >= 0.0f) || o->max_iter < 0) return na_fail(MPCPCG_EINVAL, "eps must be >= 0 and max_iter >= 0");
  if (o->stop_rule != MPCPCG_STOP_RELATIVE && o->stop_rule != MPCPCG_STOP_ABSOLUTE)
    return na_fail(MPCPCG_EINVAL, "stop_rule must be MPCPCG_STOP_RELATIVE or MPCPCG_STOP_ABSOLUTE");
  if (!lambda || !dx || !stats || (p->N > 1 && !du)) return na_fail(MPCPCG_EINVAL, "lambda, dx, du and stats must be non-NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaDevices) {
    (void)hipGetLastError();
    return na_fail(MPCPCG_EHIP, "no current device (or device index >= %d)", kNaDevices);
  }
  NaDevice &d = g_na[dev];
  std::call_once(d.once, [&] { na_setup(d, dev); });
  if (d.rc) return d.rc;
  const int N = p->N;
  const int kpw = default_single_kpw(N);  // the shape mpcpcg_solve takes by default
  int ki = 0;
  while (kKpwChoices[ki] != kpw) ++ki;
  const int g = (N + kpw - 1) / kpw;
  if (g > kNaMaxParts || g > d.cap[ki])
    return na_fail(MPCPCG_EINVAL, "horizon N=%d needs %d co-resident workgroups; the device holds %d", N, g, d.cap[ki]);
  unsigned char *const tws = d.ptr + kNaQinv + kNaRinv;
  unsigned char *const gq = tws + kNaTws;  // gang record, then the queue
  // the exchange words of the g parts, the gang record and the queue start at zero
  {
    const size_t n16 = (size_t)g * sizeof(mpc::TaskWS<kNX>) / 16, n16b = (kNaGang + kNaQueue) / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 512);
    hipLaunchKernelGGL(na_clear, dim3(blocks ? blocks : 1), dim3(256), 0, s, reinterpret_cast<uint4 *>(tws), n16,
                       reinterpret_cast<uint4 *>(gq), n16b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return na_fail(MPCPCG_EHIP, "clearing the scratch failed: %s", hipGetErrorString(e));
  }
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.Q = p->Q; a.R = p->R; a.A = p->A; a.B = p->B;
  a.q = p->q; a.r = p->r; a.x0 = p->x0; a.e = p->e;
  a.qinv_ws = reinterpret_cast<double *>(d.ptr);
  a.rinv_ws = reinterpret_cast<double *>(d.ptr + kNaQinv);
  a.tws = tws;
  a.gang = reinterpret_cast<Gang *>(gq);
  a.queue = reinterpret_cast<int *>(gq + kNaGang);
  a.eps = o->eps; a.max_iter = o->max_iter; a.warm = o->warm_start; a.stop_abs = o->stop_rule;
  a.spin_limit = d.spin;
  a.lam = lambda; a.dx = dx; a.du = du; a.stats = stats;
  a.single.k0 = 0; a.single.N = N; a.single.t0 = 0; a.single.nparts = g; a.single.id = 0;
  a.ntasks = g;
  // the placement rule of mpcpcg_solve: a gang that fits one XCD's share runs there
  a.one_xcd = (d.xcd_ok && g > 1 && 8 * g <= d.cap[ki]) ? 1 : 0;
  a.l2x = a.one_xcd;
  hipLaunchKernelGGL(kernel_for(kpw, mpc::kForward), dim3(a.one_xcd ? 8 * g : g), dim3(kpw * mpc::kGroup), 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return na_fail(MPCPCG_EHIP, "launch failed: %s", hipGetErrorString(e));
  return MPCPCG_OK;
}

}  // extern "C"
