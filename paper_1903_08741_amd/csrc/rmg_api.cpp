// C ABI of the batched Picard-multigrid sampler: validation, workspace,
// scheduling of grid-size classes, and the polling loop of the level-streaming
// path.  All arithmetic runs in the HIP kernels; this file only plans launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rmg.h"
#include "rmg_host.hpp"
#include "rmg_internal.hpp"

using namespace rmg;

constexpr int kTimerPairs = 1024;  // event pairs per timed kind and class
// Share of the compute units (whole XCDs of 32) the whole-sample classes of a batched
// MLMC call may use while level-streaming classes run beside them: a whole-sample
// workgroup holds its compute unit for milliseconds, and a streaming kernel's
// workgroups that land there wait; the streaming chains are the critical path.
// Measured on the 5-level Gardner MLMC workload: all CUs 253 ms per call, 50 % 244 ms,
// 25 % 239 ms; on the van Genuchten workload the heavy 32^2 whole-sample class then
// becomes the critical path (1776 ms against ~1500), so the restriction is requested
// per call (flag bit 7).  0 compiles it out.  Re-measured at the current kernels
// (Gardner call 195.6 ms): 12.5 % 195.7 ms, 37.5 % 197.5 ms.
#ifndef RMG_WHOLE_CU_PCT
#define RMG_WHOLE_CU_PCT 25
#endif
// Share of the compute units the other level-streaming classes of such a call may
// use, leaving the rest to the largest grid's chain (the critical path): 239 ms per
// call with every class on every CU, 232 ms at 75 %, 230 ms at 63 %, 258 ms at 50 %;
// at the current kernels 195.6 ms at 75 %, 195.3 ms at 63 % (within the run-to-run
// spread), 197.4 ms at 88 %.
#ifndef RMG_OTHER_CU_PCT
#define RMG_OTHER_CU_PCT 75
#endif
#ifndef RMG_WHOLE_MAX_N
#define RMG_WHOLE_MAX_N 32
#endif
// Largest grid solved by the whole-sample kernel (one workgroup per sample).
constexpr int kWholeMaxN = RMG_WHOLE_MAX_N;

// What a timed class's work counters mean in bytes and cells (see rmg_timed_kernel).
struct TimerMeta {
  int es = 4;                    // bytes per smoother-precision element
  double coarse_cells = 0.0;     // level cells one coarse-kernel cycle of a sample visits
  double coarse_bytes = 0.0;     // HBM bytes of that cycle
  double fine_bytes = 0.0;       // HBM bytes per fine-kernel cell
};

struct rmg_ctx {
  int device = 0;
  void* ws = nullptr;
  size_t ws_cap = 0;
  size_t ws_limit = 0;         // 0: no cap
  void* scratch = nullptr;     // device address of the fixed scratch array on this device
  int32_t* h_count = nullptr;  // pinned host mirror of the active-sample counters
  hipStream_t side[8] = {};
  hipEvent_t ev[8] = {};
  // completion markers of the iteration batches in flight, per class and slot
  hipEvent_t pev[16][4] = {};
  // one timer per concurrently running class (each on its own stream)
  KernelTimer timers[8] = {};
  TimerMeta tmeta[8] = {};
  unsigned long long* d_tcells = nullptr;  // 8 x kTimerCounters counters
  int timing = 0;
  // autotuner choices by key (device-qualified): streaming tile edges per class
  // signature ("t0 t1"), the schedule of a batched call signature ("confine G")
  std::map<std::string, std::string> tune;
  std::string tune_path;   // persisted here when non-empty
  std::string dev_key;     // architecture and compute units of the device
  // schedule tuning in progress: call signature -> measured wall ms per candidate
  std::map<std::string, std::vector<double>> sched_trials;
  bool tuned_now = false;  // a class's tiles were tuned during the current call
  hipEvent_t tev[2] = {};
  // set-up of each streaming class done (the whole-sample launches wait for them)
  hipEvent_t iev[16] = {};
  // compute-unit masks are available (the device has at least 32 compute units)
  bool can_mask = false;
  int cus = 0;
  // whole-sample classes' stream restricted to part of the compute units (null until the
  // context's first confined call)
  hipStream_t wstream = nullptr;
  hipEvent_t wev = nullptr;
  // streams for the streaming classes other than the largest grid, restricted too (or null)
  hipStream_t mside[7] = {};
  std::string err;
};

namespace {

int fail(rmg_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                       \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, RMG_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                     \
  } while (0)

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Bump allocator over the context workspace.
struct Arena {
  char* base = nullptr;
  size_t off = 0, cap = 0;
  void* take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

int reserve(rmg_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_cap && (ctx->ws_limit == 0 || ctx->ws_cap <= ctx->ws_limit)) return RMG_OK;
  if (ctx->ws_limit && bytes > ctx->ws_limit)
    return fail(ctx, RMG_ENOMEM, "workspace of %zu bytes needed, above the context's limit of %zu bytes", bytes,
                ctx->ws_limit);
  if (ctx->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
  }
  size_t want = bytes + bytes / 8 + (1 << 20);
  if (ctx->ws_limit && want > ctx->ws_limit) want = ctx->ws_limit;
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    return fail(ctx, RMG_ENOMEM, "workspace allocation of %zu bytes failed", want);
  }
  ctx->ws_cap = want;
  return RMG_OK;
}

int check_problem(rmg_ctx* ctx, const rmg_problem* p, int n_fields) {
  if (!p) return fail(ctx, RMG_EINVAL, "problem is NULL");
  if (p->model != RMG_GARDNER && p->model != RMG_VGM && p->model != RMG_LINEAR)
    return fail(ctx, RMG_EINVAL, "unknown closure model %d", p->model);
  const int need = p->model == RMG_VGM ? 3 : 1;
  if (n_fields < need) return fail(ctx, RMG_EINVAL, "model %d needs %d fields, got %d", p->model, need, n_fields);
  if (p->qoi != RMG_QOI_MEAN_SATURATION)
    return fail(ctx, RMG_EINVAL, "qoi %d is not supported by this library", p->qoi);
  if (!(p->dt > 0.0) || p->n_steps < 1) return fail(ctx, RMG_EINVAL, "need dt > 0 and n_steps >= 1");
  if (!(p->theta_s > p->theta_r)) return fail(ctx, RMG_EINVAL, "need theta_s > theta_r");
  if (p->init_profile != 0 && p->init_profile != 1) return fail(ctx, RMG_EINVAL, "init_profile must be 0 or 1");
  if (p->init_profile == 1 && !(p->init_rate > 0.0)) return fail(ctx, RMG_EINVAL, "init_profile 1 needs init_rate > 0");
  return RMG_OK;
}

int check_opts(rmg_ctx* ctx, const rmg_solver_opts* o, int n) {
  if (!o) return fail(ctx, RMG_EINVAL, "opts is NULL");
  if (o->precision != RMG_FP64 && o->precision != RMG_MIXED)
    return fail(ctx, RMG_EINVAL, "unknown precision %d", o->precision);
  if (o->cycle != RMG_CYCLE_V && o->cycle != RMG_CYCLE_W) return fail(ctx, RMG_EINVAL, "unknown cycle %d", o->cycle);
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 4 || o->nu2 > 4 || o->nu1 + o->nu2 == 0)
    return fail(ctx, RMG_EINVAL, "nu1, nu2 must be in 0..4 and not both 0");
  if (o->cycles_per_picard < 0 || o->cycles_per_picard > 16)
    return fail(ctx, RMG_EINVAL, "cycles_per_picard must be in 0..16");
  if (o->cycles_per_picard == 0 && !(o->eps_mg > 0.0))
    return fail(ctx, RMG_EINVAL, "cycles_per_picard = 0 needs eps_mg > 0");
  if (o->max_picard < 1) return fail(ctx, RMG_EINVAL, "max_picard must be >= 1");
  if (!(o->eps_picard > 0.0)) return fail(ctx, RMG_EINVAL, "eps_picard must be > 0");
  if (o->coarsest_n != 2 && o->coarsest_n != 4)
    return fail(ctx, RMG_EINVAL, "coarsest_n must be 2 or 4");
  if (o->fallback_cycles < 0 || o->fallback_cycles > 16)
    return fail(ctx, RMG_EINVAL, "fallback_cycles must be in 0..16");
  if (o->fallback_cycles > 0 && (o->cycles_per_picard == 0 || o->fallback_max_picard < 1))
    return fail(ctx, RMG_EINVAL, "a fallback needs cycles_per_picard >= 1 and fallback_max_picard >= 1");
  if (n < o->coarsest_n) return fail(ctx, RMG_EINVAL, "n=%d below coarsest_n=%d", n, o->coarsest_n);
  return RMG_OK;
}

// One grid-size class of a solve: its problems, fields and outputs.
struct ClassJob {
  SolveArgs a{};
  bool fp64 = false;
  bool whole = false;
  StreamPlan pl{};
  hipStream_t stream = nullptr;
  int32_t* d_count = nullptr;
  int32_t* h_count = nullptr;
  bool done = false;
  bool autotune = true;
};

// Workspace bytes a class needs beyond its caller-visible outputs.
size_t class_ws_bytes(const ClassJob& j) {
  const int64_t S = j.a.S;
  const int n = j.a.n;
  size_t b = 256 + 8 * (size_t)S * n * n;  // theta_old
  if (!j.whole) {
    for (int l = 0; l <= j.pl.ltop; ++l) b += 256 * 7 + level_bytes(n >> l, S, j.fp64);
    b += 7 * 256 + 2 * (sizeof(SampleState) * S + 8 * S + 8) + 8 * S;
  }
  return b;
}

void class_carve(ClassJob& j, Arena& ar) {
  const int64_t S = j.a.S;
  const int n = j.a.n;
  j.a.theta_old = (double*)ar.take(8 * (size_t)S * n * n);
  if (j.whole) return;
  const size_t es = j.fp64 ? 8 : 4;
  for (int l = 0; l <= j.pl.ltop; ++l) {
    const size_t m = (size_t)(n >> l);
    j.pl.lv.u[l] = ar.take(es * S * m * m);
    j.pl.lv.ub[l] = ar.take(es * S * m * m);
    j.pl.lv.f[l] = ar.take(es * S * m * m);
    j.pl.lv.cw[l] = ar.take(es * S * m * m);
    j.pl.lv.cs[l] = ar.take(es * S * m * m);
    j.pl.lv.cdt[l] = ar.take(es * S * m * m);
    j.pl.lv.ctop[l] = ar.take(es * S * m);
  }
  j.pl.state = (SampleState*)ar.take(sizeof(SampleState) * S);
  j.pl.state_prev = (SampleState*)ar.take(sizeof(SampleState) * S);
  j.pl.dpmax = (unsigned long long*)ar.take(8 * S);
  j.pl.dpmax_prev = (unsigned long long*)ar.take(8 * S);
  j.pl.active_count = (int32_t*)ar.take(8);
  j.pl.count_next = (int32_t*)ar.take(8);
  j.pl.mgres = j.a.cpp == 0 ? (unsigned long long*)ar.take(8 * S) : nullptr;
}

void class_plan(ClassJob& j, const rmg_solver_opts* o) {
  j.fp64 = o->precision == RMG_FP64;
  j.a.fb_cpp = o->fallback_cycles;
  j.a.fb_max_picard = o->fallback_cycles > 0 ? o->fallback_max_picard : 0;
  const int n = j.a.n;
  j.whole = !(o->flags & 1) && (n <= kWholeMaxN || (o->flags & 32)) &&
            whole_sample_lds_bytes(n, o->coarsest_n, j.fp64, j.a.F, nullptr) > 0;
  j.a.state_global = (o->flags & 4) != 0;
  j.autotune = (o->flags & (8 | 16)) == 0;
  j.pl.n = n;
  j.pl.nlev = j.a.nlev;
  j.pl.fp64 = j.fp64;
  j.pl.ltop = std::max(0, ilog2i(n) - ilog2i((o->flags & 64) ? 32 : coarse_top(j.fp64)));
  for (int l = 0; l < kMaxLevels; ++l) j.pl.ts[l] = (o->flags & 16) ? 16 : kTile;
}

std::string tune_key(const ClassJob& j) {
  char b[192];
  snprintf(b, sizeof b, "tiles n=%d S=%lld fp64=%d nu=%d,%d cpp=%d fb=%d F=%d g=%d", j.a.n, (long long)j.a.S,
           (int)j.fp64, j.a.nu1, j.a.nu2, j.a.cpp, j.a.fb_cpp, j.a.F, j.a.gamma);
  return b;
}

// The tune cache file: one "key<TAB>value" line per choice, keys qualified by the device.
void load_tune_cache(rmg_ctx* ctx) {
  if (ctx->tune_path.empty()) return;
  std::ifstream in(ctx->tune_path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t t = line.find('\t');
    if (t == std::string::npos) continue;
    ctx->tune[line.substr(0, t)] = line.substr(t + 1);
  }
}

void save_tune_cache(const rmg_ctx* ctx) {
  if (ctx->tune_path.empty()) return;
  // a temporary file of this context's own: contexts that share the cache file and tune at
  // the same time then never write into one another's copy (the last rename wins whole)
  char tag[32];
  snprintf(tag, sizeof tag, ".tmp%llx", (unsigned long long)(uintptr_t)ctx);
  const std::string tmp = ctx->tune_path + tag;
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;  // an unwritable cache only costs tuning time in later processes
    for (const auto& kv : ctx->tune) out << kv.first << '\t' << kv.second << '\n';
  }
  (void)std::rename(tmp.c_str(), ctx->tune_path.c_str());
}

bool tune_get(const rmg_ctx* ctx, const std::string& key, std::string* val) {
  auto it = ctx->tune.find(ctx->dev_key + " " + key);
  if (it == ctx->tune.end()) return false;
  *val = it->second;
  return true;
}

void tune_put(rmg_ctx* ctx, const std::string& key, const std::string& val) {
  ctx->tune[ctx->dev_key + " " + key] = val;
  save_tune_cache(ctx);
}

void set_tiles(ClassJob& j, int ts0, int tsr) {
  for (int l = 0; l < kMaxLevels; ++l) j.pl.ts[l] = l == 0 ? ts0 : tsr;
}

// Pick the tile edges of the down/up kernels of a streaming class by timing a few
// Picard iterations of the class itself for each candidate; the state is then
// re-initialised, so the tuning run leaves no trace in the results (every tile
// shape computes the same values).  Choices are cached per class signature.
int autotune_class(rmg_ctx* ctx, ClassJob& j) {
  const std::string key = tune_key(j);
  std::string val;
  int t0 = 0, t1 = 0;
  if (tune_get(ctx, key, &val) && sscanf(val.c_str(), "%d %d", &t0, &t1) == 2 && (t0 == 16 || t0 == 32) &&
      (t1 == 16 || t1 == 32)) {
    set_tiles(j, t0, t1);
    return RMG_OK;
  }
  ctx->tuned_now = true;
  KernelTimer* saved = j.pl.timer;
  j.pl.timer = nullptr;
  // The first candidate is the default; another one replaces it only when it is
  // at least 5 % faster, so that timing noise does not flip the choice from run to run.
  const int cand[4][2] = {{32, 32}, {32, 16}, {16, 16}, {16, 32}};
  float best = 1e30f;
  int b0 = kTile, b1 = kTile;
  bool first = true;
  for (auto& c : cand) {
    set_tiles(j, c[0], c[1]);
    const StreamPlan odd = flip(j.pl);
    HIP_TRY(ctx, launch_stream_init(j.a, j.pl, j.stream));
    const int J = std::max(1, j.a.cpp);
    HIP_TRY(ctx, launch_stream_iteration(j.a, j.pl, j.stream, J));
    HIP_TRY(ctx, launch_stream_iteration(j.a, odd, j.stream, J));
    HIP_TRY(ctx, hipEventRecord(ctx->tev[0], j.stream));
    for (int i = 0; i < 4; ++i) HIP_TRY(ctx, launch_stream_iteration(j.a, (i & 1) ? odd : j.pl, j.stream, J));
    HIP_TRY(ctx, hipEventRecord(ctx->tev[1], j.stream));
    HIP_TRY(ctx, hipEventSynchronize(ctx->tev[1]));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->tev[0], ctx->tev[1]));
    if (first) ms = ms * 0.95f;
    first = false;
    if (ms < best) {
      best = ms;
      b0 = c[0];
      b1 = c[1];
    }
  }
  char cv[32];
  snprintf(cv, sizeof cv, "%d %d", b0, b1);
  tune_put(ctx, key, cv);
  set_tiles(j, b0, b1);
  j.pl.timer = saved;
  HIP_TRY(ctx, launch_stream_init(j.a, j.pl, j.stream));
  return RMG_OK;
}

// Add the durations of the timed launches recorded before upto[k] in ring k (all complete).
struct RingMarks {
  int64_t tail[kTimedKinds] = {};
};
RingMarks ring_marks(const KernelTimer* t) {
  RingMarks m;
  if (t)
    for (int k = 0; k < kTimedKinds; ++k) m.tail[k] = t->ring[k].tail;
  return m;
}
int harvest_timer(rmg_ctx* ctx, KernelTimer* t, const RingMarks& upto) {
  if (!t) return RMG_OK;
  for (int k = 0; k < kTimedKinds; ++k) {
    EventRing& r = t->ring[k];
    for (; r.head < upto.tail[k]; ++r.head) {
      const int q = (int)(r.head % r.cap);
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, r.ev[2 * q], r.ev[2 * q + 1]));
      r.total_ms += ms;
      ++r.launches;
    }
  }
  return RMG_OK;
}

// Timer `ti` for a streaming class: reset its rings, record what its counters mean.
KernelTimer* attach_timer(rmg_ctx* ctx, int ti, const ClassJob& j) {
  KernelTimer* t = &ctx->timers[ti];
  for (auto& r : t->ring) r.head = r.tail = 0;
  TimerMeta& mt = ctx->tmeta[ti];
  mt.es = j.fp64 ? 8 : 4;
  const int lt = j.pl.ltop, m = j.a.n >> lt;
  double cells = 0.0, visits = 1.0;
  for (int l = lt; l < j.a.nlev; ++l, visits *= j.a.gamma) cells += visits * (double)(j.a.n >> l) * (j.a.n >> l);
  mt.coarse_cells = cells;
  mt.coarse_bytes = 5.0 * mt.es * (double)m * m;
  mt.fine_bytes = 8.0 * (2 + j.a.F) + 4.0 * mt.es * 4.0 / 3.0;
  return t;
}

// Run every class to completion.  Whole-sample classes are single launches.  A
// streaming class advances in batches of G passes (a replayed HIP graph, or eager
// launches) of alternating plan parity (G is even, so every batch starts with the even
// plan and ends with the odd one); each batch ends with an 8-byte read-back of the
// class's counters (active samples, and those of them in the fallback attempt, after
// its last pass) and an event.  A pass runs J cycle slots: J = the primary cycle count,
// or, once the read-back shows a sample in the fallback attempt, the larger of the
// primary and fallback counts (the kernels take each sample's cycles from its state,
// so the switch, seen a few batches late, never changes results).  D batches stay in
// flight per class, so the device never waits for the host; batches issued after the
// count reached zero find no active sample and do nothing.  Classes are polled
// independently.  With kernel timing on, the first pass of a timed batch is launched
// eagerly with its timed launches' events recorded by their dispatches (events recorded
// by graph nodes cannot be timed) and the other G - 1 replay a second graph.  An eager
// pass costs a roughly fixed extra host and queue time, so classes with short passes
// (fewer than kDenseCells cells per pass) time every kTimedEvery-th batch and the others
// every batch: a uniform sample of the launches, one in G * kTimedEvery or one in G.
int run_classes(rmg_ctx* ctx, std::vector<ClassJob>& jobs, bool use_graphs, int G = 8) {
  constexpr int D = 3, kTimedEvery = 8;
  constexpr int64_t kDenseCells = int64_t(1) << 22;
  if (G < 2 || G % 2 != 0) return fail(ctx, RMG_EINVAL, "internal: odd batch length");
  const bool timing = ctx->timing != 0;
  if (jobs.size() > 16) return fail(ctx, RMG_EINVAL, "too many grid-size classes");
  int ti = 0;
  for (auto& j : jobs) {
    j.pl.timer = nullptr;
    j.pl.tcells = nullptr;
    if (ctx->timing && !j.whole && ti < 8) {
      j.pl.timer = attach_timer(ctx, ti++, j);
    }
  }
  // Streaming classes first: their set-up (and a first call's synchronous tile
  // autotuning) must not wait behind, or be timed against, the whole-sample kernels;
  // the whole-sample launches also wait until every streaming class's initialisation
  // has run (a whole-sample launch occupies the compute units for milliseconds, and
  // an initialisation dispatched beside it waited that long).
  int nstream = 0;
  for (const auto& j : jobs) nstream += j.whole ? 0 : 1;
  for (auto& j : jobs) j.a.fuse_top = (!j.whole && nstream == 1) ? 1 : 0;
  int ninit = 0;
  for (auto& j : jobs) {
    if (j.whole) continue;
    HIP_TRY(ctx, prepare_stream(j.a, j.pl));
    HIP_TRY(ctx, launch_stream_init(j.a, j.pl, j.stream));
    if (j.autotune) {
      const int rc = autotune_class(ctx, j);
      if (rc != RMG_OK) return rc;
    }
    HIP_TRY(ctx, hipEventRecord(ctx->iev[ninit++], j.stream));
  }
  for (auto& j : jobs) {
    if (!j.whole) continue;
    for (int q = 0; q < ninit; ++q) HIP_TRY(ctx, hipStreamWaitEvent(j.stream, ctx->iev[q], 0));
    HIP_TRY(ctx, launch_whole_sample(j.a, j.fp64, j.stream));
    j.done = true;
  }
  // cycle slots per pass: primary, and with a sample in the fallback attempt
  auto slots = [](const ClassJob& j, int v) {
    return v == 0 ? std::max(1, j.a.cpp) : std::max(j.a.cpp, j.a.fb_cpp);
  };
  auto nvar = [](const ClassJob& j) { return j.a.fb_cpp > j.a.cpp ? 2 : 1; };
  // per class and slot variant v: a graph of the batch's G passes (index 4c + 2v) and,
  // with timing, one of its last G - 1 (4c + 2v + 1)
  std::vector<hipGraphExec_t> execs(4 * jobs.size(), nullptr);
  std::vector<hipGraph_t> graphs(4 * jobs.size(), nullptr);
  auto cleanup = [&]() {
    for (auto& e : execs)
      if (e) (void)hipGraphExecDestroy(e);
    for (auto& g : graphs)
      if (g) (void)hipGraphDestroy(g);
  };
  if (use_graphs) {
    for (size_t c = 0; c < jobs.size(); ++c) {
      ClassJob& j = jobs[c];
      if (j.done) continue;
      StreamPlan untimed = j.pl;
      untimed.timer = nullptr;
      const StreamPlan untimed_odd = flip(untimed);
      for (int v = 0; v < nvar(j); ++v)
        for (int first = 0; first < (timing ? 2 : 1); ++first) {
          const size_t gi = 4 * c + 2 * v + first;
          const char* what = "hipStreamBeginCapture";
          hipError_t e = hipStreamBeginCapture(j.stream, hipStreamCaptureModeThreadLocal);
          if (e == hipSuccess) what = "captured pass launches";
          for (int i = first; i < G && e == hipSuccess; ++i)
            e = launch_stream_iteration(j.a, (i & 1) ? untimed_odd : untimed, j.stream, slots(j, v));
          hipGraph_t g = nullptr;
          const hipError_t e2 = hipStreamEndCapture(j.stream, &g);
          graphs[gi] = g;
          if (e == hipSuccess) {
            e = e2;
            what = "hipStreamEndCapture";
          }
          if (e == hipSuccess) {
            e = hipGraphInstantiate(&execs[gi], g, nullptr, nullptr, 0);
            what = "hipGraphInstantiate";
          }
          if (e != hipSuccess) {
            cleanup();
            return fail(ctx, RMG_EHIP, "graph capture of the Picard pass failed in %s: %s", what,
                        hipGetErrorString(e));
          }
        }
    }
  }
  // every sample stops after at most n_steps * (max_picard * cpp + fallback limit * its
  // cycles) passes
  std::vector<int64_t> issued(jobs.size(), 0), retired(jobs.size(), 0);
  std::vector<int> var(jobs.size(), 0);
  std::vector<std::array<RingMarks, D>> mark(jobs.size());
  auto bound = [&](const ClassJob& j) {
    const int64_t steps = std::max(j.a.cp.prob[0].n_steps, j.a.cp.prob[1].n_steps);
    const int64_t cyc = j.a.cpp > 0 ? j.a.cpp : kMaxMgCycles;
    return steps * ((int64_t)j.a.max_picard * cyc + (int64_t)j.a.fb_max_picard * j.a.fb_cpp) + (int64_t)(D + 1) * G;
  };
  auto issue = [&](size_t c) -> hipError_t {
    ClassJob& j = jobs[c];
    const int k = (int)(issued[c] % D);
    const int v = var[c];
    StreamPlan untimed = j.pl;
    untimed.timer = nullptr;
    const StreamPlan untimed_odd = flip(untimed);
    hipError_t e = hipSuccess;
    const bool timed = timing && ((int64_t)j.a.S * j.a.n * j.a.n >= kDenseCells || issued[c] % kTimedEvery == 0);
    if (timed) e = launch_stream_iteration(j.a, j.pl, j.stream, slots(j, v));
    if (use_graphs) {
      if (e == hipSuccess) e = hipGraphLaunch(execs[4 * c + 2 * v + (timed ? 1 : 0)], j.stream);
    } else {
      for (int i = timed ? 1 : 0; i < G && e == hipSuccess; ++i)
        e = launch_stream_iteration(j.a, (i & 1) ? untimed_odd : untimed, j.stream, slots(j, v));
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(j.h_count + 2 * k, flip(j.pl).active_count, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                         j.stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->pev[c][k], j.stream);
    mark[c][k] = ring_marks(j.pl.timer);
    ++issued[c];
    return e;
  };
  int rc = RMG_OK;
  size_t active = 0;
  for (size_t c = 0; c < jobs.size() && rc == RMG_OK; ++c) {
    if (jobs[c].done) continue;
    ++active;
    for (int k = 0; k < D && rc == RMG_OK; ++k) {
      const hipError_t e = issue(c);
      if (e != hipSuccess) rc = fail(ctx, RMG_EHIP, "iteration launch failed: %s", hipGetErrorString(e));
    }
  }
  while (active > 0 && rc == RMG_OK) {
    bool progressed = false;
    for (size_t c = 0; c < jobs.size() && rc == RMG_OK; ++c) {
      ClassJob& j = jobs[c];
      if (j.done) continue;
      const int k = (int)(retired[c] % D);
      hipError_t e = hipEventQuery(ctx->pev[c][k]);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) {
        rc = fail(ctx, RMG_EHIP, "iteration batch: %s", hipGetErrorString(e));
        break;
      }
      progressed = true;
      if ((rc = harvest_timer(ctx, j.pl.timer, mark[c][k])) != RMG_OK) break;
      const int32_t left = ((volatile int32_t*)j.h_count)[2 * k];
      const int32_t in_fallback = ((volatile int32_t*)j.h_count)[2 * k + 1];
      ++retired[c];
      if (left == 0) {
        e = launch_stream_finish(j.a, flip(j.pl), j.stream);
        if (e != hipSuccess) rc = fail(ctx, RMG_EHIP, "finish launch: %s", hipGetErrorString(e));
        j.done = true;
        --active;
        continue;
      }
      if (in_fallback > 0 && nvar(j) == 2) var[c] = 1;
      if (issued[c] * G > bound(j)) {
        rc = fail(ctx, RMG_EHIP, "samples still active after %lld passes", (long long)(issued[c] * G));
        break;
      }
      e = issue(c);
      if (e != hipSuccess) rc = fail(ctx, RMG_EHIP, "iteration launch failed: %s", hipGetErrorString(e));
    }
    if (!progressed) std::this_thread::yield();
  }
  // leave nothing of this call running on an error; collect the last timed launches
  for (auto& j : jobs) {
    if (j.whole) continue;
    const hipError_t e = hipStreamSynchronize(j.stream);
    if (e != hipSuccess && rc == RMG_OK) rc = fail(ctx, RMG_EHIP, "stream synchronize: %s", hipGetErrorString(e));
    if (rc == RMG_OK && j.pl.timer) rc = harvest_timer(ctx, j.pl.timer, ring_marks(j.pl.timer));
  }
  cleanup();
  return rc;
}

}  // namespace

int rmg::set_error(rmg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int rmg::device_of(const rmg_ctx* c) { return c->device; }

extern "C" {

int64_t rmg_struct_size(const char* name) {
  if (!name) return -1;
  const std::string s(name);
  if (s == "rmg_problem") return sizeof(rmg_problem);
  if (s == "rmg_solver_opts") return sizeof(rmg_solver_opts);
  if (s == "rmg_sample_stats") return sizeof(rmg_sample_stats);
  if (s == "rmg_level_sums") return sizeof(rmg_level_sums);
  if (s == "rmg_level") return sizeof(rmg_level);
  if (s == "rmg_marginal") return sizeof(rmg_marginal);
  if (s == "rmg_kernel_timing") return sizeof(rmg_kernel_timing);
  if (s == "rmg_pc_level") return sizeof(rmg_pc_level);
  if (s == "rmg_pc_opts") return sizeof(rmg_pc_opts);
  if (s == "rmg_pc_level_out") return sizeof(rmg_pc_level_out);
  if (s == "rmg_pc_result") return sizeof(rmg_pc_result);
  return -1;
}

// The compute-unit-masked streams of confined calls, made by a context's first confined
// call: each holds a hardware queue of its own, and a context that never confines (such as
// one of several contexts driven at the same time, whose calls run unconfined) then holds
// none.  The whole-sample stream is made last, so that its presence means all are there.
static hipError_t ensure_masked_streams(rmg_ctx* c) {
  if (c->wstream) return hipSuccess;
  auto mask_of = [c](int pct) {
    const int keep = std::max(32, c->cus * pct / 100 / 32 * 32);
    std::vector<uint32_t> m((c->cus + 31) / 32, 0u);
    for (int k = 0; k < keep; ++k) m[k / 32] |= 1u << (k % 32);
    return m;
  };
  hipError_t e = hipSuccess;
#if RMG_OTHER_CU_PCT > 0
  const std::vector<uint32_t> m2 = mask_of(RMG_OTHER_CU_PCT);
  for (auto& ms : c->mside)
    if (!ms && (e = hipExtStreamCreateWithCUMask(&ms, (uint32_t)m2.size(), m2.data())) != hipSuccess) return e;
#endif
  if (!c->wev && (e = hipEventCreateWithFlags(&c->wev, hipEventDisableTiming)) != hipSuccess) return e;
  const std::vector<uint32_t> m = mask_of(RMG_WHOLE_CU_PCT);
  return hipExtStreamCreateWithCUMask(&c->wstream, (uint32_t)m.size(), m.data());
}

int rmg_ctx_create(rmg_ctx** out, int hip_device, const char* tune_cache_path) {
  if (!out) return RMG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return RMG_EINVAL;
  rmg_ctx* c = new (std::nothrow) rmg_ctx();
  if (!c) return RMG_ENOMEM;
  c->device = hip_device;
  // 8 counters per class: two per batch in flight
  if (hipSetDevice(hip_device) != hipSuccess ||
      hipHostMalloc((void**)&c->h_count, 256 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RMG_EHIP;
  }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
    char dk[128];
    snprintf(dk, sizeof dk, "[%s cu=%d]", prop.gcnArchName, prop.multiProcessorCount);
    c->dev_key = dk;
  }
  if (tune_cache_path && *tune_cache_path) {
    c->tune_path = tune_cache_path;
    load_tune_cache(c);
  }
  // the fixed scratch array's address on this device (each device holds its own copy)
  if (scratch_address(&c->scratch) != hipSuccess || !c->scratch) {
    rmg_ctx_destroy(c);
    return RMG_EHIP;
  }
  for (auto& s : c->side) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
  }
  for (auto& e : c->ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
  }
  for (auto& row : c->pev)
    for (auto& e : row)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        rmg_ctx_destroy(c);
        return RMG_EHIP;
      }
  for (auto& e : c->iev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
#if RMG_WHOLE_CU_PCT > 0
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess || cus < 32) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
    c->can_mask = true;  // the masked streams are made by the first confined call
    c->cus = cus;
  }
#endif
  for (auto& e : c->tev) {
    if (hipEventCreate(&e) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
  }
  constexpr size_t ncnt = 8 * kTimerCounters;
  if (hipMalloc((void**)&c->d_tcells, ncnt * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(c->d_tcells, 0, ncnt * sizeof(unsigned long long)) != hipSuccess) {
    rmg_ctx_destroy(c);
    return RMG_EHIP;
  }
  for (int t = 0; t < 8; ++t) c->timers[t].d_cells = c->d_tcells + kTimerCounters * t;
  *out = c;
  return RMG_OK;
}

int rmg_ctx_set_workspace_limit(rmg_ctx* c, int64_t bytes) {
  if (!c) return RMG_EINVAL;
  c->err.clear();
  if (bytes < 0) return fail(c, RMG_EINVAL, "workspace limit must be >= 0");
  c->ws_limit = (size_t)bytes;
  return RMG_OK;
}

int64_t rmg_ctx_tune_dump(rmg_ctx* c, char* buf, int64_t cap) {
  if (!c || cap < 0 || (cap > 0 && !buf)) return RMG_EINVAL;
  c->err.clear();
  std::string text;
  for (const auto& kv : c->tune) text += kv.first + '\t' + kv.second + '\n';
  if (cap > 0) {
    const size_t n = std::min<size_t>(text.size(), (size_t)cap - 1);
    std::memcpy(buf, text.data(), n);
    buf[n] = '\0';
  }
  return (int64_t)text.size();
}

static void free_timer_events(rmg_ctx* c) {
  for (auto& t : c->timers)
    for (auto& r : t.ring) {
      if (!r.ev) continue;
      for (int q = 0; q < 2 * r.cap; ++q)
        if (r.ev[q]) (void)hipEventDestroy(r.ev[q]);
      delete[] r.ev;
      r.ev = nullptr;
      r.cap = 0;
    }
}

int rmg_set_kernel_timing(rmg_ctx* c, int which) {
  if (!c) return RMG_EINVAL;
  c->err.clear();
  constexpr int all = RMG_TIME_SMOOTHER_DOWN | RMG_TIME_COARSE | RMG_TIME_FINE;
  if (which & ~all) return fail(c, RMG_EINVAL, "unknown timed kernel mask %d", which);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  const int bit[kTimedKinds] = {RMG_TIME_SMOOTHER_DOWN, RMG_TIME_COARSE, RMG_TIME_FINE};
  for (auto& t : c->timers)
    for (int k = 0; k < kTimedKinds; ++k) {
      EventRing& r = t.ring[k];
      if (!(which & bit[k]) || r.ev) continue;
      r.ev = new (std::nothrow) hipEvent_t[2 * kTimerPairs]();
      if (!r.ev) return fail(c, RMG_ENOMEM, "timer event pool");
      r.cap = kTimerPairs;
      for (int q = 0; q < 2 * kTimerPairs; ++q) HIP_TRY(c, hipEventCreate(&r.ev[q]));
    }
  for (auto& t : c->timers) {
    t.which = which;
    for (int k = 0; k < kTimedKinds; ++k) {
      EventRing& r = t.ring[k];
      r.head = r.tail = 0;
      r.launches = 0;
      r.total_ms = 0.0;
      // a ring of a kind that is not selected stays unused (room() is false without events)
      if (!(which & bit[k]) && r.ev) {
        for (int q = 0; q < 2 * r.cap; ++q) (void)hipEventDestroy(r.ev[q]);
        delete[] r.ev;
        r.ev = nullptr;
        r.cap = 0;
      }
    }
  }
  HIP_TRY(c, hipMemset(c->d_tcells, 0, 8 * kTimerCounters * sizeof(unsigned long long)));
  c->timing = which;
  return RMG_OK;
}

int rmg_get_kernel_timing(rmg_ctx* c, int kind, rmg_kernel_timing* out) {
  if (!c || !out) return RMG_EINVAL;
  c->err.clear();
  int k;
  if (kind == RMG_TIME_SMOOTHER_DOWN) k = 0;
  else if (kind == RMG_TIME_COARSE) k = 1;
  else if (kind == RMG_TIME_FINE) k = 2;
  else return fail(c, RMG_EINVAL, "kind %d is not a single timed kernel", kind);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  unsigned long long cnt[8 * kTimerCounters];
  HIP_TRY(c, hipMemcpy(cnt, c->d_tcells, sizeof cnt, hipMemcpyDeviceToHost));
  rmg_kernel_timing r = {0, 0, 0.0, 0.0};
  for (int t = 0; t < 8; ++t) {
    const EventRing& ring = c->timers[t].ring[k];
    const TimerMeta& m = c->tmeta[t];
    const unsigned long long* q = cnt + kTimerCounters * t;
    r.launches += ring.launches;
    r.total_ms += ring.total_ms;
    if (k == 0) {
      r.cells += (int64_t)(q[0] + q[1]);
      r.algo_bytes += m.es * (5.25 * (double)q[0] + 6.25 * (double)q[1]);
    } else if (k == 1) {
      r.cells += (int64_t)((double)q[2] * m.coarse_cells);
      r.algo_bytes += (double)q[2] * m.coarse_bytes;
    } else {
      r.cells += (int64_t)q[4];
      r.algo_bytes += (double)q[4] * m.fine_bytes;
    }
  }
  *out = r;
  return RMG_OK;
}

void rmg_ctx_destroy(rmg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_timer_events(c);
  for (auto& e : c->tev)
    if (e) (void)hipEventDestroy(e);
  if (c->d_tcells) (void)hipFree(c->d_tcells);
  for (auto& ms : c->mside)
    if (ms) (void)hipStreamDestroy(ms);
  if (c->wstream) (void)hipStreamDestroy(c->wstream);
  if (c->wev) (void)hipEventDestroy(c->wev);
  for (auto& e : c->iev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& row : c->pev)
    for (auto& e : row)
      if (e) (void)hipEventDestroy(e);
  for (auto& s : c->side)
    if (s) (void)hipStreamDestroy(s);
  if (c->ws) (void)hipFree(c->ws);
  if (c->h_count) (void)hipHostFree(c->h_count);
  delete c;
}

const char* rmg_last_error(const rmg_ctx* c) { return c ? c->err.c_str() : "null context"; }

int sample_fields(rmg_ctx* ctx, int n, int n_fields, int n_modes, const double* d_basis,
                  const double* d_xi, const rmg_marginal* h_marg, int64_t S, double* d_fields,
                  hipStream_t stream) {
  if (!ctx) return RMG_EINVAL;
  ctx->err.clear();
  if (!pow2_in(n, 4, 4096)) return fail(ctx, RMG_EINVAL, "n=%d must be a power of two in 4..4096", n);
  if (n_fields < 1 || n_fields > 4) return fail(ctx, RMG_EINVAL, "n_fields=%d not in 1..4", n_fields);
  if (n_modes < 1 || n_modes > 1024) return fail(ctx, RMG_EINVAL, "n_modes=%d not in 1..1024", n_modes);
  if (S < 1) return fail(ctx, RMG_EINVAL, "S must be >= 1");
  if (!d_basis || !d_xi || !h_marg || !d_fields) return fail(ctx, RMG_EINVAL, "NULL pointer");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_kl_fields(n * n, n_modes, S * n_fields, n_fields, d_basis, d_xi, h_marg, d_fields,
                                stream));
  return RMG_OK;
}

}  // extern "C"

namespace {
// picard_mg_solve, with its workspace in the context's workspace (grown with hipMalloc
// when needed) or, for the allocation-free variant, in the fixed device scratch array
// (the call then also launches its passes eagerly: no graph is instantiated).
int solve_impl(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
               const double* d_fields, int64_t S, double* d_h_out, double* d_qoi, int32_t* d_status,
               rmg_sample_stats* d_stats, hipStream_t stream, bool noalloc) {
  if (!ctx) return RMG_EINVAL;
  ctx->err.clear();
  if (!pow2_in(n, 2, 1024)) return fail(ctx, RMG_EINVAL, "n=%d must be a power of two in 2..1024", n);
  if (S < 1 || S > 65535) return fail(ctx, RMG_EINVAL, "S=%lld not in 1..65535", (long long)S);
  if (!d_fields || !d_h_out || !d_qoi || !d_status) return fail(ctx, RMG_EINVAL, "NULL pointer");
  int rc = check_problem(ctx, problem, problem ? (problem->model == RMG_VGM ? 3 : 1) : 1);
  if (rc) return rc;
  if ((rc = check_opts(ctx, opts, n))) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  std::vector<ClassJob> jobs(1);
  ClassJob& j = jobs[0];
  j.a.n = n;
  j.a.lg = ilog2i(n);
  j.a.nlev = ilog2i(n) - ilog2i(opts->coarsest_n) + 1;
  j.a.F = problem->model == RMG_VGM ? 3 : 1;
  j.a.S = S;
  j.a.fields = d_fields;
  j.a.cp.prob[0] = *problem;
  j.a.cp.prob[1] = *problem;
  j.a.cp.seg_split = S;
  j.a.nu1 = opts->nu1;
  j.a.nu2 = opts->nu2;
  j.a.gamma = opts->cycle == RMG_CYCLE_W ? 2 : 1;
  j.a.cpp = opts->cycles_per_picard;
  j.a.max_picard = opts->max_picard;
  j.a.eps = opts->eps_picard;
  j.a.eps_mg = opts->eps_mg;
  j.a.p = d_h_out;
  j.a.qoi = d_qoi;
  j.a.status = d_status;
  j.a.stats = d_stats;
  class_plan(j, opts);
  // the solve runs on a context stream ordered after the caller's stream (a
  // captured graph cannot be recorded on the legacy default stream)
  j.stream = ctx->side[0];
  j.h_count = ctx->h_count;
  Arena ar;
  if (noalloc) {
    // the allocation-free variant: the workspace is the fixed scratch array
    const size_t need = class_ws_bytes(j) + 256;
    if (need > kScratchBytes)
      return fail(ctx, RMG_EINVAL, "this solve needs %zu bytes of scratch; the fixed scratch of the allocation-free "
                  "entry point holds %zu bytes (use picard_mg_solve, or fewer samples per call)", need,
                  kScratchBytes);
    ar.base = (char*)ctx->scratch;
    ar.cap = kScratchBytes;
  } else {
    if ((rc = reserve(ctx, class_ws_bytes(j)))) return rc;
    ar.base = (char*)ctx->ws;
    ar.cap = ctx->ws_cap;
  }
  class_carve(j, ar);
  if (ar.off > ar.cap) return fail(ctx, RMG_ENOMEM, "internal error: workspace accounting (%zu > %zu)", ar.off, ar.cap);
  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], stream));
  HIP_TRY(ctx, hipStreamWaitEvent(j.stream, ctx->ev[0], 0));
  rc = run_classes(ctx, jobs, !noalloc && !(opts->flags & 2));
  HIP_TRY(ctx, hipEventRecord(ctx->ev[1], j.stream));
  HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->ev[1], 0));
  if (rc) return rc;
  // statuses checked in chunks through a fixed host buffer
  int32_t st[1024];
  bool all_ok = true;
  for (int64_t s0 = 0; s0 < S && all_ok; s0 += 1024) {
    const int64_t k = std::min<int64_t>(1024, S - s0);
    HIP_TRY(ctx, hipMemcpyAsync(st, d_status + s0, sizeof(int32_t) * k, hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    for (int64_t q = 0; q < k; ++q)
      if (st[q] != RMG_SAMPLE_OK) all_ok = false;
  }
  if (!all_ok) return fail(ctx, RMG_ENOTCONV, "some samples did not converge");
  return RMG_OK;
}
}  // namespace

extern "C" {

int picard_mg_solve(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                    const double* d_fields, int64_t S, double* d_h_out, double* d_qoi,
                    int32_t* d_status, rmg_sample_stats* d_stats, hipStream_t stream) {
  return solve_impl(ctx, n, problem, opts, d_fields, S, d_h_out, d_qoi, d_status, d_stats, stream, false);
}

int picard_mg_solve_noalloc(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                            const double* d_fields, int64_t S, double* d_h_out, double* d_qoi,
                            int32_t* d_status, rmg_sample_stats* d_stats, hipStream_t stream) {
  return solve_impl(ctx, n, problem, opts, d_fields, S, d_h_out, d_qoi, d_status, d_stats, stream, true);
}

int picard_mg_adjoint(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts, int n_modes,
                      const double* d_basis, const rmg_marginal* h_marg, const double* d_xi, int64_t S,
                      int ckpt_every, double eps_adjoint, double* d_q, double* d_grad, int32_t* d_status,
                      rmg_sample_stats* d_stats, hipStream_t stream) {
  if (!ctx) return RMG_EINVAL;
  ctx->err.clear();
  if (!pow2_in(n, 4, 1024)) return fail(ctx, RMG_EINVAL, "n=%d must be a power of two in 4..1024", n);
  if (S < 1 || S > 65535) return fail(ctx, RMG_EINVAL, "S=%lld not in 1..65535", (long long)S);
  if (n_modes < 1 || n_modes > 1024) return fail(ctx, RMG_EINVAL, "n_modes=%d not in 1..1024", n_modes);
  if (!problem || !d_basis || !h_marg || !d_xi || !d_q || !d_grad || !d_status)
    return fail(ctx, RMG_EINVAL, "NULL pointer");
  if (problem->model != RMG_GARDNER && problem->model != RMG_LINEAR)
    return fail(ctx, RMG_EINVAL, "the adjoint supports the Gardner and linear closures only");
  if (problem->qoi != RMG_QOI_BOTTOM_OUTFLUX)
    return fail(ctx, RMG_EINVAL, "the adjoint's quantity of interest is the bottom outflux (qoi = %d)",
                (int)RMG_QOI_BOTTOM_OUTFLUX);
  rmg_problem fprob = *problem;  // the forward kernels compute their own (unused) QoI
  fprob.qoi = RMG_QOI_MEAN_SATURATION;
  int rc = check_problem(ctx, &fprob, 1);
  if (rc) return rc;
  if ((rc = check_opts(ctx, opts, n))) return rc;
  const int nst = problem->n_steps;
  if (ckpt_every < 1 || ckpt_every > nst || nst % ckpt_every != 0)
    return fail(ctx, RMG_EINVAL, "ckpt_every=%d must divide n_steps=%d", ckpt_every, nst);
  if (!(eps_adjoint > 0.0)) return fail(ctx, RMG_EINVAL, "eps_adjoint must be > 0");
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  const int64_t N = (int64_t)n * n;
  const int K = ckpt_every, slots = nst / K + 1;
  // forward class (its own kernel choice) and adjoint class (level streaming)
  std::vector<ClassJob> fjobs(1);
  ClassJob& fj = fjobs[0];
  fj.a.n = n;
  fj.a.lg = ilog2i(n);
  fj.a.nlev = ilog2i(n) - ilog2i(opts->coarsest_n) + 1;
  fj.a.F = 1;
  fj.a.S = S;
  fj.a.cp.prob[0] = fprob;
  fj.a.cp.prob[1] = fprob;
  fj.a.cp.seg_split = S;
  fj.a.nu1 = opts->nu1;
  fj.a.nu2 = opts->nu2;
  fj.a.gamma = opts->cycle == RMG_CYCLE_W ? 2 : 1;
  fj.a.cpp = opts->cycles_per_picard;
  fj.a.max_picard = opts->max_picard;
  fj.a.eps = opts->eps_picard;
  fj.a.eps_mg = opts->eps_mg;
  class_plan(fj, opts);
  ClassJob aj = fj;
  rmg_solver_opts aopts = *opts;
  aopts.flags |= 1 | 8;  // level streaming, fixed tiles
  aopts.fallback_cycles = 0;
  class_plan(aj, &aopts);
  aj.a.cpp = std::max(1, opts->cycles_per_picard);

  // workspace: a dry carve sizes it, the second carve places it
  struct Bufs {
    double *fields, *p, *fq, *hist, *seg, *mu, *b, *g, *qn;
    int32_t *fst, *rst;
    rmg_sample_stats *fstats, *rstats;
  } bf{};
  auto carve_all = [&](Arena& ar) {
    bf.fields = (double*)ar.take(8 * S * N);
    bf.p = (double*)ar.take(8 * S * N);
    bf.fq = (double*)ar.take(8 * S);
    bf.fst = (int32_t*)ar.take(4 * S);
    bf.rst = (int32_t*)ar.take(4 * S);
    bf.fstats = (rmg_sample_stats*)ar.take(sizeof(rmg_sample_stats) * S);
    bf.rstats = (rmg_sample_stats*)ar.take(sizeof(rmg_sample_stats) * S);
    bf.hist = (double*)ar.take(8 * S * slots * N);
    bf.seg = K > 1 ? (double*)ar.take(8 * S * (K + 1) * N) : nullptr;
    bf.mu = (double*)ar.take(8 * S * N);
    bf.b = (double*)ar.take(8 * S * N);
    bf.g = (double*)ar.take(8 * S * N);
    bf.qn = (double*)ar.take(8 * S * nst);
    class_carve(fj, ar);
    class_carve(aj, ar);
  };
  Arena dry;
  carve_all(dry);
  if ((rc = reserve(ctx, dry.off + 256))) return rc;
  Arena ar;
  ar.base = (char*)ctx->ws;
  ar.cap = ctx->ws_cap;
  carve_all(ar);
  if (ar.off > ar.cap) return fail(ctx, RMG_ENOMEM, "internal error: workspace accounting (%zu > %zu)", ar.off, ar.cap);

  hipStream_t st = ctx->side[0];
  fj.stream = aj.stream = st;
  fj.h_count = aj.h_count = ctx->h_count;
  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], stream));
  HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->ev[0], 0));
  HIP_TRY(ctx, launch_kl_fields((int)N, n_modes, S, 1, d_basis, d_xi, h_marg, bf.fields, st));
  fj.a.fields = aj.a.fields = bf.fields;

  // forward pass: checkpoints p^0, p^K, p^2K, ...
  fj.a.p = bf.p;
  fj.a.qoi = bf.fq;
  fj.a.status = bf.fst;
  fj.a.stats = bf.fstats;
  fj.a.p_hist = bf.hist;
  fj.a.hist_every = K;
  fj.a.hist_slots = slots;
  const bool graphs = !(opts->flags & 2);
  if ((rc = run_classes(ctx, fjobs, graphs))) return rc;

  // backward pass, segment by segment
  aj.a.p = bf.mu;
  AdjArgs ad{};
  ad.mu = bf.mu;
  ad.b = bf.b;
  ad.g = bf.g;
  ad.qn = bf.qn;
  ad.n_steps = nst;
  ad.eps = eps_adjoint;
  ad.max_its = opts->max_picard;
  HIP_TRY(ctx, prepare_stream(aj.a, aj.pl));
  HIP_TRY(ctx, launch_adj_init(aj.a, aj.pl, ad, bf.fst, st));
  // kernel timing covers the adjoint iterations' launches too (eager launches: all timed
  // while the event ring has room; it is drained at every poll)
  KernelTimer* tm = nullptr;
  if (ctx->timing) {
    tm = attach_timer(ctx, 1, aj);
  }
  aj.pl.timer = tm;
  for (int seg = (K == 1 ? 0 : nst / K - 1); seg >= 0; --seg) {
    if (K == 1) {
      ad.hist = bf.hist;
      ad.slots = slots;
      ad.base = 0;
      ad.lo = 1;
      ad.hi = nst;
    } else {
      // recompute the segment's steps from its checkpoint, every step recorded
      fj.a.cp.prob[0].n_steps = fj.a.cp.prob[1].n_steps = K;
      fj.a.p0 = bf.hist + (int64_t)seg * N;
      fj.a.p0_stride = (int64_t)slots * N;
      fj.a.p_hist = bf.seg;
      fj.a.hist_every = 1;
      fj.a.hist_slots = K + 1;
      fj.a.status = bf.rst;
      fj.a.stats = bf.rstats;
      fj.done = false;
      if ((rc = run_classes(ctx, fjobs, graphs))) return rc;
      ad.hist = bf.seg;
      ad.slots = K + 1;
      ad.base = seg * K;
      ad.lo = seg * K + 1;
      ad.hi = seg * K + K;
    }
    HIP_TRY(ctx, launch_adj_reset(aj.a, aj.pl, ad, st));
    const int64_t bound = (int64_t)(ad.hi - ad.lo + 1) * ad.max_its + 16;
    int64_t its = 0;
    for (;;) {
      for (int i = 0; i < 8; ++i) HIP_TRY(ctx, launch_adj_iteration(aj.a, aj.pl, ad, st));
      its += 8;
      HIP_TRY(ctx, hipMemcpyAsync(ctx->h_count, aj.pl.active_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(ctx, hipStreamSynchronize(st));
      if ((rc = harvest_timer(ctx, tm, ring_marks(tm)))) return rc;
      if (((volatile int32_t*)ctx->h_count)[0] == 0) break;
      if (its > bound) return fail(ctx, RMG_EHIP, "adjoint samples still active after %lld iterations", (long long)its);
    }
    HIP_TRY(ctx, launch_adj_grad_final(aj.a, aj.pl, ad, st));
    HIP_TRY(ctx, launch_adj_outflux(aj.a, ad, st));
  }
  HIP_TRY(ctx, launch_adj_finish(aj.a, aj.pl, ad, bf.fst, d_q, d_status, d_stats ? d_stats + S : nullptr, st));
  if (d_stats)
    HIP_TRY(ctx, hipMemcpyAsync(d_stats, bf.fstats, sizeof(rmg_sample_stats) * S, hipMemcpyDeviceToDevice, st));
  HIP_TRY(ctx, launch_grad_xi(S, (int)N, n_modes, d_basis, bf.g, bf.fields, h_marg[0], d_status, d_grad, st));
  HIP_TRY(ctx, hipEventRecord(ctx->ev[1], st));
  HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->ev[1], 0));
  std::vector<int32_t> sv(S);
  HIP_TRY(ctx, hipMemcpyAsync(sv.data(), d_status, sizeof(int32_t) * S, hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  for (int32_t v : sv)
    if (v != RMG_SAMPLE_OK) return fail(ctx, RMG_ENOTCONV, "some samples did not converge");
  return RMG_OK;
}

int picard_mg_outflux(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts, int n_modes,
                      const double* d_basis, const rmg_marginal* h_marg, const double* d_xi, int64_t S,
                      double* d_q, int32_t* d_status, rmg_sample_stats* d_stats, hipStream_t stream) {
  if (!ctx) return RMG_EINVAL;
  ctx->err.clear();
  if (!pow2_in(n, 4, 1024)) return fail(ctx, RMG_EINVAL, "n=%d must be a power of two in 4..1024", n);
  if (S < 1 || S > 65535) return fail(ctx, RMG_EINVAL, "S=%lld not in 1..65535", (long long)S);
  if (n_modes < 1 || n_modes > 1024) return fail(ctx, RMG_EINVAL, "n_modes=%d not in 1..1024", n_modes);
  if (!problem || !d_basis || !h_marg || !d_xi || !d_q || !d_status) return fail(ctx, RMG_EINVAL, "NULL pointer");
  if (problem->model != RMG_GARDNER && problem->model != RMG_LINEAR)
    return fail(ctx, RMG_EINVAL, "the outflux entry point supports the Gardner and linear closures only");
  if (problem->qoi != RMG_QOI_BOTTOM_OUTFLUX)
    return fail(ctx, RMG_EINVAL, "problem->qoi must be RMG_QOI_BOTTOM_OUTFLUX (%d)", (int)RMG_QOI_BOTTOM_OUTFLUX);
  rmg_problem fprob = *problem;
  fprob.qoi = RMG_QOI_MEAN_SATURATION;
  int rc = check_problem(ctx, &fprob, 1);
  if (rc) return rc;
  if ((rc = check_opts(ctx, opts, n))) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int64_t N = (int64_t)n * n;
  const int nst = problem->n_steps, slots = nst + 1;
  std::vector<ClassJob> fjobs(1);
  ClassJob& fj = fjobs[0];
  fj.a.n = n;
  fj.a.lg = ilog2i(n);
  fj.a.nlev = ilog2i(n) - ilog2i(opts->coarsest_n) + 1;
  fj.a.F = 1;
  fj.a.S = S;
  fj.a.cp.prob[0] = fprob;
  fj.a.cp.prob[1] = fprob;
  fj.a.cp.seg_split = S;
  fj.a.nu1 = opts->nu1;
  fj.a.nu2 = opts->nu2;
  fj.a.gamma = opts->cycle == RMG_CYCLE_W ? 2 : 1;
  fj.a.cpp = opts->cycles_per_picard;
  fj.a.max_picard = opts->max_picard;
  fj.a.eps = opts->eps_picard;
  fj.a.eps_mg = opts->eps_mg;
  class_plan(fj, opts);
  // every step's pressure head is kept (the history is what the outflux is summed from)
  double *fields = nullptr, *p = nullptr, *fq = nullptr, *hist = nullptr, *qn = nullptr;
  rmg_sample_stats* fstats = nullptr;
  auto carve_all = [&](Arena& ar) {
    fields = (double*)ar.take(8 * S * N);
    p = (double*)ar.take(8 * S * N);
    fq = (double*)ar.take(8 * S);
    fstats = (rmg_sample_stats*)ar.take(sizeof(rmg_sample_stats) * S);
    hist = (double*)ar.take(8 * S * slots * N);
    qn = (double*)ar.take(8 * S * nst);
    class_carve(fj, ar);
  };
  Arena dry;
  carve_all(dry);
  if ((rc = reserve(ctx, dry.off + 256))) return rc;
  Arena ar;
  ar.base = (char*)ctx->ws;
  ar.cap = ctx->ws_cap;
  carve_all(ar);
  if (ar.off > ar.cap) return fail(ctx, RMG_ENOMEM, "internal error: workspace accounting (%zu > %zu)", ar.off, ar.cap);
  hipStream_t st = ctx->side[0];
  fj.stream = st;
  fj.h_count = ctx->h_count;
  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], stream));
  HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->ev[0], 0));
  HIP_TRY(ctx, launch_kl_fields((int)N, n_modes, S, 1, d_basis, d_xi, h_marg, fields, st));
  fj.a.fields = fields;
  fj.a.p = p;
  fj.a.qoi = fq;
  fj.a.status = d_status;
  fj.a.stats = d_stats ? d_stats : fstats;
  fj.a.p_hist = hist;
  fj.a.hist_every = 1;
  fj.a.hist_slots = slots;
  if ((rc = run_classes(ctx, fjobs, !(opts->flags & 2)))) return rc;
  AdjArgs ad{};
  ad.hist = hist;
  ad.slots = slots;
  ad.base = 0;
  ad.lo = 1;
  ad.hi = nst;
  ad.n_steps = nst;
  ad.qn = qn;
  HIP_TRY(ctx, launch_adj_outflux(fj.a, ad, st));
  HIP_TRY(ctx, launch_outflux_total(fj.a, ad, d_status, d_q, st));
  HIP_TRY(ctx, hipEventRecord(ctx->ev[1], st));
  HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->ev[1], 0));
  int32_t sv[1024];
  bool all_ok = true;
  for (int64_t s0 = 0; s0 < S && all_ok; s0 += 1024) {
    const int64_t k = std::min<int64_t>(1024, S - s0);
    HIP_TRY(ctx, hipMemcpyAsync(sv, d_status + s0, sizeof(int32_t) * k, hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    for (int64_t q = 0; q < k; ++q)
      if (sv[q] != RMG_SAMPLE_OK) all_ok = false;
  }
  if (!all_ok) return fail(ctx, RMG_ENOTCONV, "some samples did not converge");
  return RMG_OK;
}

int mlmc_level_estimate(rmg_ctx* ctx, int n_levels, const rmg_level* L, int n_fields, int n_modes,
                        const rmg_marginal* h_marg, const rmg_solver_opts* opts, rmg_level_sums* h_out,
                        double* d_qoi_out, hipStream_t stream) {
  if (!ctx) return RMG_EINVAL;
  ctx->err.clear();
  if (n_levels < 1 || n_levels > 16 || !L || !h_marg || !h_out)
    return fail(ctx, RMG_EINVAL, "bad level list");
  if (n_fields < 1 || n_fields > 4 || n_modes < 1 || n_modes > 1024)
    return fail(ctx, RMG_EINVAL, "bad n_fields / n_modes");
  int rc;
  // classes by grid size: (level, role) segments, at most one fine and one coarse per size
  struct Seg {
    int level, role;  // role 0 fine, 1 coarse
  };
  std::map<int, std::vector<Seg>> cls;
  for (int l = 0; l < n_levels; ++l) {
    const rmg_level& v = L[l];
    if (!pow2_in(v.n_fine, 4, 1024)) return fail(ctx, RMG_EINVAL, "level %d: bad n_fine %d", l, v.n_fine);
    // an entry is a base level (no coarse member, n_coarse = 0) or a correction
    // level (n_coarse = n_fine / 2); any entry may be either, so a caller can
    // add samples to one correction level alone
    const bool corr = v.n_coarse != 0;
    if (corr && v.n_coarse * 2 != v.n_fine)
      return fail(ctx, RMG_EINVAL, "level %d: n_coarse must be 0 or n_fine/2", l);
    if (v.n_samples < 1 || !v.d_basis_fine || !v.d_xi || (corr && !v.d_basis_coarse))
      return fail(ctx, RMG_EINVAL, "level %d: bad samples or NULL pointer", l);
    if ((rc = check_problem(ctx, &v.fine, n_fields))) return rc;
    if (corr && (rc = check_problem(ctx, &v.coarse, n_fields))) return rc;
    if ((rc = check_opts(ctx, opts, corr ? v.n_coarse : v.n_fine))) return rc;
    cls[v.n_fine].push_back({l, 0});
    if (corr) cls[v.n_coarse].push_back({l, 1});
  }
  for (auto& kv : cls) {
    if (kv.second.size() > 2) return fail(ctx, RMG_EINVAL, "grid %d used by more than two segments", kv.first);
    if (kv.second.size() == 2 && kv.second[0].role == kv.second[1].role)
      return fail(ctx, RMG_EINVAL, "grid %d appears twice in the same role", kv.first);
    std::sort(kv.second.begin(), kv.second.end(), [](const Seg& a, const Seg& b) { return a.role < b.role; });
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  // plan every class, then size the workspace once
  std::vector<ClassJob> jobs;
  std::vector<int> jn;
  struct Out {
    double *fields, *p, *qoi;
    int32_t* status;
    rmg_sample_stats* stats;
  };
  for (auto& kv : cls) {
    ClassJob j;
    const int n = kv.first;
    int64_t S = 0;
    for (auto& sg : kv.second) S += L[sg.level].n_samples;
    if (S > 65535) return fail(ctx, RMG_EINVAL, "grid %d: more than 65535 solves", n);
    j.a.n = n;
    j.a.lg = ilog2i(n);
    j.a.nlev = ilog2i(n) - ilog2i(opts->coarsest_n) + 1;
    j.a.F = n_fields;
    j.a.S = S;
    const Seg& s0 = kv.second[0];
    j.a.cp.prob[0] = s0.role == 0 ? L[s0.level].fine : L[s0.level].coarse;
    j.a.cp.prob[1] = j.a.cp.prob[0];
    j.a.cp.seg_split = L[s0.level].n_samples;
    if (kv.second.size() == 2) {
      const Seg& s1 = kv.second[1];
      j.a.cp.prob[1] = s1.role == 0 ? L[s1.level].fine : L[s1.level].coarse;
    }
    j.a.nu1 = opts->nu1;
    j.a.nu2 = opts->nu2;
  j.a.gamma = opts->cycle == RMG_CYCLE_W ? 2 : 1;
    j.a.cpp = opts->cycles_per_picard;
    j.a.max_picard = opts->max_picard;
    j.a.eps = opts->eps_picard;
  j.a.eps_mg = opts->eps_mg;
    class_plan(j, opts);
    jobs.push_back(j);
    jn.push_back(n);
  }
  size_t need = 0;
  for (auto& j : jobs) {
    const int64_t S = j.a.S;
    const size_t N = (size_t)j.a.n * j.a.n;
    need += class_ws_bytes(j) + 6 * 256 + 8 * S * n_fields * N + 8 * S * N + 8 * S + 4 * S +
            sizeof(rmg_sample_stats) * S;
  }
  need += 256 + sizeof(rmg_level_sums) * n_levels;
  if ((rc = reserve(ctx, need))) return rc;
  Arena ar;
  ar.base = (char*)ctx->ws;
  ar.cap = ctx->ws_cap;
  std::vector<Out> outs(jobs.size());
  for (size_t c = 0; c < jobs.size(); ++c) {
    ClassJob& j = jobs[c];
    const int64_t S = j.a.S;
    const size_t N = (size_t)j.a.n * j.a.n;
    outs[c].fields = (double*)ar.take(8 * S * n_fields * N);
    outs[c].p = (double*)ar.take(8 * S * N);
    outs[c].qoi = (double*)ar.take(8 * S);
    outs[c].status = (int32_t*)ar.take(4 * S);
    outs[c].stats = (rmg_sample_stats*)ar.take(sizeof(rmg_sample_stats) * S);
    j.a.fields = outs[c].fields;
    j.a.p = outs[c].p;
    j.a.qoi = outs[c].qoi;
    j.a.status = outs[c].status;
    j.a.stats = outs[c].stats;
    class_carve(j, ar);
  }
  rmg_level_sums* d_sums = (rmg_level_sums*)ar.take(sizeof(rmg_level_sums) * n_levels);
  if (ar.off > ar.cap) return fail(ctx, RMG_ENOMEM, "internal error: workspace accounting (%zu > %zu)", ar.off, ar.cap);

  // fields: both members of a pair draw from the same xi row through their own basis
  for (size_t c = 0; c < jobs.size(); ++c) {
    const size_t N = (size_t)jn[c] * jn[c];
    int64_t row = 0;
    for (auto& sg : cls[jn[c]]) {
      const rmg_level& v = L[sg.level];
      const double* B = sg.role == 0 ? v.d_basis_fine : v.d_basis_coarse;
      HIP_TRY(ctx, launch_kl_fields((int)N, n_modes, v.n_samples * n_fields, n_fields, B, v.d_xi, h_marg,
                                    outs[c].fields + (size_t)row * n_fields * N, stream));
      row += v.n_samples;
    }
  }
  // Every whole-sample class runs on the caller's stream, one after the other
  // (ordered after the fields); each streaming class gets a side stream of its
  // own, in creation order.  HIP multiplexes streams onto a few hardware queues
  // (four by default), and a streaming class whose stream shares a queue with a
  // long whole-sample kernel cannot start its chain of short launches until that
  // kernel ends; the caller's stream is otherwise idle until the level sums.
  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], stream));
  int nside = 0;
  bool any_whole = false;
  for (size_t c = 0; c < jobs.size(); ++c) {
    if (jobs[c].whole) {
      jobs[c].stream = stream;
      any_whole = true;
    } else {
      if (nside == 7) return fail(ctx, RMG_EINVAL, "more than seven level-streaming grid sizes");
      jobs[c].stream = ctx->side[nside++];
    }
    jobs[c].h_count = ctx->h_count + 8 * (int)c;
  }
  for (int q = 0; q < nside; ++q) HIP_TRY(ctx, hipStreamWaitEvent(ctx->side[q], ctx->ev[0], 0));
  // Schedule of the call: whether the whole-sample classes move to the restricted stream
  // while streaming classes run beside them (flag bit 7 forces it, bit 8 forbids it;
  // whether it helps depends on which class is critical), and the passes per batch G.
  // Otherwise the choice is tuned per call signature across calls: the candidates run
  // whole calls in turn, each timed twice (round robin, kSchedRounds rounds), then the one
  // with the fastest of its calls is kept (a later candidate must beat the first by 2 %,
  // about twice the call-to-call spread) and written to the tune cache.  Results never
  // depend on it.
  constexpr size_t kSchedRounds = 2;
  const bool can_confine = ctx->can_mask && any_whole && nside > 0;
  const bool tune_sched = (opts->flags & (8 | 16)) == 0;
  std::vector<std::pair<int, int>> cands;  // (confine, G)
  for (int G : {8, 16}) {
    if (!tune_sched && G != 8) continue;
    if (!can_confine || (opts->flags & 256)) {
      cands.push_back({0, G});
    } else if (opts->flags & 128) {
      cands.push_back({1, G});
    } else {
      cands.push_back({0, G});
      cands.push_back({1, G});
    }
  }
  std::string skey = "sched";
  for (auto& j : jobs) skey += " {" + tune_key(j) + (j.whole ? " whole" : "") + "}";
  {
    char fb[64];
    snprintf(fb, sizeof fb, " flags=%d", opts->flags & ~(8 | 16));
    skey += fb;
  }
  int sched_cand = -1;  // index being tried in this call, or -1 if the choice is settled
  std::pair<int, int> sched = cands[0];
  if (cands.size() > 1) {
    std::string val;
    int c0 = 0, g0 = 0;
    if (tune_get(ctx, skey, &val) && sscanf(val.c_str(), "%d %d", &c0, &g0) == 2 && (c0 == 0 || can_confine) &&
        (g0 == 8 || g0 == 16)) {
      sched = {c0, g0};
    } else {
      sched_cand = (int)(ctx->sched_trials[skey].size() % cands.size());
      sched = cands[sched_cand];
    }
  }
  const auto t_sched0 = std::chrono::steady_clock::now();
  ctx->tuned_now = false;
  const bool wmasked = can_confine && sched.first;
  std::vector<hipStream_t> sused(ctx->side, ctx->side + nside);
  if (wmasked) {
    HIP_TRY(ctx, ensure_masked_streams(ctx));
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->wstream, ctx->ev[0], 0));
    for (auto& j : jobs)
      if (j.whole) j.stream = ctx->wstream;
    // the largest grid's chain is the critical path: the other streaming classes move
    // to restricted streams, so that some compute units only ever see the largest grid
    if (ctx->mside[0] && nside > 1) {
      int k = 0;
      for (auto& j : jobs)
        if (!j.whole && k < nside - 1) {
          HIP_TRY(ctx, hipStreamWaitEvent(ctx->mside[k], ctx->ev[0], 0));
          j.stream = ctx->mside[k];
          sused[k] = ctx->mside[k];
          ++k;
        }
    }
  }
  if ((rc = run_classes(ctx, jobs, !(opts->flags & 2), sched.second))) return rc;
  for (int q = 0; q < nside; ++q) {
    HIP_TRY(ctx, hipEventRecord(ctx->ev[1 + q], sused[q]));
    HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->ev[1 + q], 0));
  }
  if (wmasked) {
    HIP_TRY(ctx, hipEventRecord(ctx->wev, ctx->wstream));
    HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->wev, 0));
  }
  // level sums and optional per-sample QoIs
  int64_t qoff = 0;
  for (int l = 0; l < n_levels; ++l) {
    const rmg_level& v = L[l];
    auto locate = [&](int n, int role, const double** q, const int32_t** st, const rmg_sample_stats** ss) {
      size_t c = std::find(jn.begin(), jn.end(), n) - jn.begin();
      int64_t off = 0;
      for (auto& sg : cls[n]) {
        if (sg.role == role && sg.level == l) break;
        off += L[sg.level].n_samples;
      }
      *q = outs[c].qoi + off;
      *st = outs[c].status + off;
      *ss = outs[c].stats + off;
    };
    const double *qf, *qc = nullptr;
    const int32_t *sf, *sc = nullptr;
    const rmg_sample_stats *tf, *tc = nullptr;
    locate(v.n_fine, 0, &qf, &sf, &tf);
    if (v.n_coarse) locate(v.n_coarse, 1, &qc, &sc, &tc);
    HIP_TRY(ctx, launch_level_sums(qf, qc, v.n_samples, sf, sc, tf, tc, d_sums + l, stream));
    if (d_qoi_out) {
      HIP_TRY(ctx, hipMemcpyAsync(d_qoi_out + qoff, qf, 8 * v.n_samples, hipMemcpyDeviceToDevice, stream));
      if (qc) {
        HIP_TRY(ctx, hipMemcpyAsync(d_qoi_out + qoff + v.n_samples, qc, 8 * v.n_samples,
                                    hipMemcpyDeviceToDevice, stream));
      } else {
        std::vector<double> nanv(v.n_samples, std::nan(""));
        HIP_TRY(ctx, hipMemcpyAsync(d_qoi_out + qoff + v.n_samples, nanv.data(), 8 * v.n_samples,
                                    hipMemcpyHostToDevice, stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
      }
      qoff += 2 * v.n_samples;
    }
  }
  HIP_TRY(ctx, hipMemcpyAsync(h_out, d_sums, sizeof(rmg_level_sums) * n_levels, hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  if (sched_cand >= 0 && !ctx->tuned_now) {  // a call that also tuned tiles is not a fair trial
    auto& tr = ctx->sched_trials[skey];
    tr.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_sched0).count());
    if (tr.size() == kSchedRounds * cands.size()) {
      const size_t nc = cands.size();
      std::vector<double> t(nc, 1e300);
      for (size_t q = 0; q < tr.size(); ++q) t[q % nc] = std::min(t[q % nc], tr[q]);
      size_t best = 0;
      for (size_t q = 1; q < nc; ++q)
        if (t[q] < 0.98 * t[0] && t[q] < t[best]) best = q;
      char cv[32];
      snprintf(cv, sizeof cv, "%d %d", cands[best].first, cands[best].second);
      tune_put(ctx, skey, cv);
      ctx->sched_trials.erase(skey);
    }
  }
  for (int l = 0; l < n_levels; ++l)
    if (h_out[l].n_failed) return fail(ctx, RMG_ENOTCONV, "level %d: %lld failed pairs", l, (long long)h_out[l].n_failed);
  return RMG_OK;
}

}  // extern "C"
