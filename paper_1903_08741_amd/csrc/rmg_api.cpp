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
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rmg.h"
#include "rmg_host.hpp"
#include "rmg_internal.hpp"

using namespace rmg;

constexpr int kTimerPairs = 4096;
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

struct rmg_ctx {
  int device = 0;
  void* ws = nullptr;
  size_t ws_cap = 0;
  int32_t* h_count = nullptr;  // pinned host mirror of the active-sample counters
  hipStream_t side[8] = {};
  hipEvent_t ev[8] = {};
  // completion markers of the iteration batches in flight, per class and slot
  hipEvent_t pev[16][4] = {};
  // one timer per concurrently running class (each on its own stream)
  KernelTimer timers[8] = {};
  int timer_es[8] = {};
  unsigned long long* d_tcells = nullptr;  // 8 x 2 counters
  int timing = 0;
  // autotuner: tile edges (level 0, coarser streaming levels) per class signature
  std::map<std::string, std::pair<int, int>> tune;
  hipEvent_t tev[2] = {};
  // set-up of each streaming class done (the whole-sample launches wait for them)
  hipEvent_t iev[16] = {};
  // whole-sample classes' stream restricted to part of the compute units (or null)
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
  if (bytes <= ctx->ws_cap) return RMG_OK;
  if (ctx->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
  }
  const size_t want = bytes + bytes / 8 + (1 << 20);
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
    return fail(ctx, RMG_EINVAL, "qoi %d is not supported by this build", p->qoi);
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
    b += 6 * 256 + 2 * (sizeof(SampleState) * S + 8 * S + 8);
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
}

void class_plan(ClassJob& j, const rmg_solver_opts* o) {
  j.fp64 = o->precision == RMG_FP64;
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
  char b[160];
  snprintf(b, sizeof b, "n=%d S=%lld fp64=%d nu=%d,%d cpp=%d F=%d", j.a.n, (long long)j.a.S, (int)j.fp64,
           j.a.nu1, j.a.nu2, j.a.cpp, j.a.F);
  return b;
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
  auto it = ctx->tune.find(key);
  if (it != ctx->tune.end()) {
    set_tiles(j, it->second.first, it->second.second);
    return RMG_OK;
  }
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
    HIP_TRY(ctx, launch_stream_iteration(j.a, j.pl, j.stream));
    HIP_TRY(ctx, launch_stream_iteration(j.a, odd, j.stream));
    HIP_TRY(ctx, hipEventRecord(ctx->tev[0], j.stream));
    for (int i = 0; i < 4; ++i) HIP_TRY(ctx, launch_stream_iteration(j.a, (i & 1) ? odd : j.pl, j.stream));
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
  ctx->tune[key] = {b0, b1};
  set_tiles(j, b0, b1);
  j.pl.timer = saved;
  HIP_TRY(ctx, launch_stream_init(j.a, j.pl, j.stream));
  return RMG_OK;
}

// Add the durations of the timed launches recorded before `upto` (all complete).
int harvest_timer(rmg_ctx* ctx, KernelTimer* t, int64_t upto) {
  if (!t) return RMG_OK;
  for (; t->head < upto; ++t->head) {
    const int q = (int)(t->head % t->cap);
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, t->ev[2 * q], t->ev[2 * q + 1]));
    t->total_ms += ms;
    ++t->launches;
  }
  return RMG_OK;
}

// Run every class to completion.  Whole-sample classes are single launches.  A
// streaming class advances in batches of G Picard iterations (a replayed HIP graph,
// or eager launches) of alternating plan parity (G is even, so every batch starts
// with the even plan and ends with the odd one); each batch ends with a 4-byte
// read-back of the class's active-sample count (of its last iteration) and an event.  D batches stay in flight per class, so the
// device never waits for the host; batches issued after the count reached zero
// find no active sample and do nothing.  Classes are polled independently.
// With kernel timing on, the first iteration of a timed batch is launched eagerly
// with its timed launches bracketed by events (events recorded by graph nodes
// cannot be timed) and the other G - 1 replay a second graph.  An eager iteration
// costs a roughly fixed extra host and queue time, so classes with short iterations
// (fewer than kDenseCells cells per iteration) time every kTimedEvery-th batch and
// the others every batch: a uniform sample of the launches, one in G * kTimedEvery
// or one in G.
int run_classes(rmg_ctx* ctx, std::vector<ClassJob>& jobs, bool use_graphs) {
  constexpr int G = 8, D = 3, kTimedEvery = 8;
  constexpr int64_t kDenseCells = int64_t(1) << 22;
  static_assert(G % 2 == 0, "a batch must end on the odd plan (double-buffered per-sample state)");
  const bool timing = ctx->timing != 0;
  if (jobs.size() > 16) return fail(ctx, RMG_EINVAL, "too many grid-size classes");
  int ti = 0;
  for (auto& j : jobs) {
    j.pl.timer = nullptr;
    j.pl.tcells = nullptr;
    if (ctx->timing && !j.whole && ti < 8) {
      j.pl.timer = &ctx->timers[ti];
      j.pl.timer->head = j.pl.timer->tail = 0;
      ctx->timer_es[ti] = j.fp64 ? 8 : 4;
      ++ti;
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
  // per class: a graph of the batch's G iterations, and (timing) one of its last G - 1
  std::vector<hipGraphExec_t> execs(2 * jobs.size(), nullptr);
  std::vector<hipGraph_t> graphs(2 * jobs.size(), nullptr);
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
      for (int first = 0; first < (timing ? 2 : 1); ++first) {
        const char* what = "hipStreamBeginCapture";
        hipError_t e = hipStreamBeginCapture(j.stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) what = "captured iteration launches";
        for (int i = first; i < G && e == hipSuccess; ++i)
          e = launch_stream_iteration(j.a, (i & 1) ? untimed_odd : untimed, j.stream);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(j.stream, &g);
        graphs[2 * c + first] = g;
        if (e == hipSuccess) {
          e = e2;
          what = "hipStreamEndCapture";
        }
        if (e == hipSuccess) {
          e = hipGraphInstantiate(&execs[2 * c + first], g, nullptr, nullptr, 0);
          what = "hipGraphInstantiate";
        }
        if (e != hipSuccess) {
          cleanup();
          return fail(ctx, RMG_EHIP, "graph capture of the Picard iteration failed in %s: %s", what,
                      hipGetErrorString(e));
        }
      }
    }
  }
  // every sample stops after at most n_steps * max_picard iterations
  std::vector<int64_t> issued(jobs.size(), 0), retired(jobs.size(), 0);
  std::vector<std::array<int64_t, D>> mark(jobs.size());
  auto bound = [&](const ClassJob& j) {
    const int64_t steps = std::max(j.a.cp.prob[0].n_steps, j.a.cp.prob[1].n_steps);
    return steps * (int64_t)j.a.max_picard + (int64_t)(D + 1) * G;
  };
#ifdef RMG_HOST_STATS
  double host_issue_s = 0.0;
  long n_issue = 0, n_poll = 0;
#endif
  auto issue = [&](size_t c) -> hipError_t {
#ifdef RMG_HOST_STATS
    const auto t0_ = std::chrono::steady_clock::now();
    struct Acc {
      double& s;
      std::chrono::steady_clock::time_point t;
      ~Acc() { s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count(); }
    } acc_{host_issue_s, t0_};
    ++n_issue;
#endif
    ClassJob& j = jobs[c];
    const int k = (int)(issued[c] % D);
    StreamPlan untimed = j.pl;
    untimed.timer = nullptr;
    const StreamPlan untimed_odd = flip(untimed);
    hipError_t e = hipSuccess;
    const bool timed = timing && ((int64_t)j.a.S * j.a.n * j.a.n >= kDenseCells || issued[c] % kTimedEvery == 0);
    if (timed) e = launch_stream_iteration(j.a, j.pl, j.stream);
    if (use_graphs) {
      if (e == hipSuccess) e = hipGraphLaunch(execs[2 * c + (timed ? 1 : 0)], j.stream);
    } else {
      for (int i = timed ? 1 : 0; i < G && e == hipSuccess; ++i)
        e = launch_stream_iteration(j.a, (i & 1) ? untimed_odd : untimed, j.stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(j.h_count + k, flip(j.pl).active_count, sizeof(int32_t), hipMemcpyDeviceToHost, j.stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->pev[c][k], j.stream);
    mark[c][k] = j.pl.timer ? j.pl.timer->tail : 0;
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
      const int32_t left = ((volatile int32_t*)j.h_count)[k];
      ++retired[c];
      if (left == 0) {
        e = launch_stream_finish(j.a, flip(j.pl), j.stream);
        if (e != hipSuccess) rc = fail(ctx, RMG_EHIP, "finish launch: %s", hipGetErrorString(e));
        j.done = true;
        --active;
        continue;
      }
      if (issued[c] * G > bound(j)) {
        rc = fail(ctx, RMG_EHIP, "samples still active after %lld iterations", (long long)(issued[c] * G));
        break;
      }
      e = issue(c);
      if (e != hipSuccess) rc = fail(ctx, RMG_EHIP, "iteration launch failed: %s", hipGetErrorString(e));
    }
    if (!progressed) std::this_thread::yield();
#ifdef RMG_HOST_STATS
    ++n_poll;
#endif
  }
#ifdef RMG_HOST_STATS
  fprintf(stderr, "[rmg host] issues %ld, %.1f us each, polls %ld\n", n_issue, 1e6 * host_issue_s / (n_issue ? n_issue : 1), n_poll);
#endif
  // leave nothing of this call running on an error; collect the last timed launches
  for (auto& j : jobs) {
    if (j.whole) continue;
    const hipError_t e = hipStreamSynchronize(j.stream);
    if (e != hipSuccess && rc == RMG_OK) rc = fail(ctx, RMG_EHIP, "stream synchronize: %s", hipGetErrorString(e));
    if (rc == RMG_OK && j.pl.timer) rc = harvest_timer(ctx, j.pl.timer, j.pl.timer->tail);
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

int rmg_ctx_create(rmg_ctx** out, int hip_device) {
  if (!out) return RMG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return RMG_EINVAL;
  rmg_ctx* c = new (std::nothrow) rmg_ctx();
  if (!c) return RMG_ENOMEM;
  c->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess ||
      hipHostMalloc((void**)&c->h_count, 64 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    delete c;
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
    const int keep = std::max(32, cus * RMG_WHOLE_CU_PCT / 100 / 32 * 32);
    std::vector<uint32_t> mask((cus + 31) / 32, 0u);
    for (int k = 0; k < keep; ++k) mask[k / 32] |= 1u << (k % 32);
    if (hipExtStreamCreateWithCUMask(&c->wstream, (uint32_t)mask.size(), mask.data()) != hipSuccess ||
        hipEventCreateWithFlags(&c->wev, hipEventDisableTiming) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
#if RMG_OTHER_CU_PCT > 0
    const int keep2 = std::max(32, cus * RMG_OTHER_CU_PCT / 100 / 32 * 32);
    std::vector<uint32_t> mask2((cus + 31) / 32, 0u);
    for (int k = 0; k < keep2; ++k) mask2[k / 32] |= 1u << (k % 32);
    for (auto& ms : c->mside)
      if (hipExtStreamCreateWithCUMask(&ms, (uint32_t)mask2.size(), mask2.data()) != hipSuccess) {
        rmg_ctx_destroy(c);
        return RMG_EHIP;
      }
#endif
  }
#endif
  for (auto& e : c->tev) {
    if (hipEventCreate(&e) != hipSuccess) {
      rmg_ctx_destroy(c);
      return RMG_EHIP;
    }
  }
  if (hipMalloc((void**)&c->d_tcells, 16 * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(c->d_tcells, 0, 16 * sizeof(unsigned long long)) != hipSuccess) {
    rmg_ctx_destroy(c);
    return RMG_EHIP;
  }
  for (int t = 0; t < 8; ++t) c->timers[t].d_cells = c->d_tcells + 2 * t;
  *out = c;
  return RMG_OK;
}

static void free_timer_events(rmg_ctx* c) {
  for (auto& t : c->timers) {
    if (!t.ev) continue;
    for (int q = 0; q < 2 * t.cap; ++q)
      if (t.ev[q]) (void)hipEventDestroy(t.ev[q]);
    delete[] t.ev;
    t.ev = nullptr;
    t.cap = 0;
  }
}

int rmg_set_kernel_timing(rmg_ctx* c, int which) {
  if (!c) return RMG_EINVAL;
  c->err.clear();
  if (which != RMG_TIME_NONE && which != RMG_TIME_SMOOTHER_DOWN)
    return fail(c, RMG_EINVAL, "unknown timed kernel %d", which);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  if (which != RMG_TIME_NONE) {
    for (auto& t : c->timers) {
      if (t.ev) continue;
      t.ev = new (std::nothrow) hipEvent_t[2 * kTimerPairs]();
      if (!t.ev) return fail(c, RMG_ENOMEM, "timer event pool");
      t.cap = kTimerPairs;
      for (int q = 0; q < 2 * kTimerPairs; ++q) HIP_TRY(c, hipEventCreate(&t.ev[q]));
    }
  }
  for (auto& t : c->timers) {
    t.which = which;
    t.head = t.tail = 0;
    t.launches = 0;
    t.total_ms = 0.0;
  }
  HIP_TRY(c, hipMemset(c->d_tcells, 0, 16 * sizeof(unsigned long long)));
  c->timing = which;
  return RMG_OK;
}

int rmg_get_kernel_timing(rmg_ctx* c, rmg_kernel_timing* out) {
  if (!c || !out) return RMG_EINVAL;
  c->err.clear();
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  unsigned long long cells[16];
  HIP_TRY(c, hipMemcpy(cells, c->d_tcells, sizeof cells, hipMemcpyDeviceToHost));
  rmg_kernel_timing r = {0, 0, 0.0, 0.0};
  for (int t = 0; t < 8; ++t) {
    r.launches += c->timers[t].launches;
    r.total_ms += c->timers[t].total_ms;
    r.cells += (int64_t)(cells[2 * t] + cells[2 * t + 1]);
    const double es = c->timer_es[t];
    r.algo_bytes += es * (5.25 * (double)cells[2 * t] + 6.25 * (double)cells[2 * t + 1]);
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

int picard_mg_solve(rmg_ctx* ctx, int n, const rmg_problem* problem, const rmg_solver_opts* opts,
                    const double* d_fields, int64_t S, double* d_h_out, double* d_qoi,
                    int32_t* d_status, rmg_sample_stats* d_stats, hipStream_t stream) {
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
  if (!j.whole && opts->cycles_per_picard == 0)
    return fail(ctx, RMG_EINVAL, "grid %d: the residual-controlled cycle count (cycles_per_picard = 0) is built "
                "for the whole-sample kernel only (grids up to 32 x 32, or 64 x 64 with flag bit 5)", j.a.n);
  // the solve runs on a context stream ordered after the caller's stream (a
  // captured graph cannot be recorded on the legacy default stream)
  j.stream = ctx->side[0];
  j.h_count = ctx->h_count;
  if ((rc = reserve(ctx, class_ws_bytes(j)))) return rc;
  Arena ar;
  ar.base = (char*)ctx->ws;
  ar.cap = ctx->ws_cap;
  class_carve(j, ar);
  if (ar.off > ar.cap) return fail(ctx, RMG_ENOMEM, "internal error: workspace accounting (%zu > %zu)", ar.off, ar.cap);
  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], stream));
  HIP_TRY(ctx, hipStreamWaitEvent(j.stream, ctx->ev[0], 0));
  rc = run_classes(ctx, jobs, !(opts->flags & 2));
  HIP_TRY(ctx, hipEventRecord(ctx->ev[1], j.stream));
  HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->ev[1], 0));
  if (rc) return rc;
  std::vector<int32_t> st(S);
  HIP_TRY(ctx, hipMemcpyAsync(st.data(), d_status, sizeof(int32_t) * S, hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  for (int32_t v : st)
    if (v != RMG_SAMPLE_OK) return fail(ctx, RMG_ENOTCONV, "some samples did not converge");
  return RMG_OK;
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
  if (!fj.whole && opts->cycles_per_picard == 0)
    return fail(ctx, RMG_EINVAL, "grid %d: cycles_per_picard = 0 needs the whole-sample kernel", n);
  ClassJob aj = fj;
  rmg_solver_opts aopts = *opts;
  aopts.flags |= 1 | 8;  // level streaming, fixed tiles
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
    tm = &ctx->timers[1];
    tm->head = tm->tail = 0;
    ctx->timer_es[1] = aj.fp64 ? 8 : 4;
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
      if ((rc = harvest_timer(ctx, tm, tm ? tm->tail : 0))) return rc;
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
    if (!j.whole && opts->cycles_per_picard == 0)
      return fail(ctx, RMG_EINVAL, "grid %d: the residual-controlled cycle count (cycles_per_picard = 0) is "
                  "built for the whole-sample kernel only (grids up to 32 x 32, or 64 x 64 with flag bit 5)", n);
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
    jobs[c].h_count = ctx->h_count + 4 * (int)c;
  }
  for (int q = 0; q < nside; ++q) HIP_TRY(ctx, hipStreamWaitEvent(ctx->side[q], ctx->ev[0], 0));
  // flag bit 7: the whole-sample classes move to the restricted stream when streaming
  // classes run beside them (whether that helps depends on which class is critical)
  const bool wmasked = ctx->wstream && any_whole && nside > 0 && (opts->flags & 128);
  std::vector<hipStream_t> sused(ctx->side, ctx->side + nside);
  if (wmasked) {
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
  if ((rc = run_classes(ctx, jobs, !(opts->flags & 2)))) return rc;
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
  for (int l = 0; l < n_levels; ++l)
    if (h_out[l].n_failed) return fail(ctx, RMG_ENOTCONV, "level %d: %lld failed pairs", l, (long long)h_out[l].n_failed);
  return RMG_OK;
}

}  // extern "C"
