// Internal interfaces between the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rmg.h"

namespace rmg {

constexpr int kMaxLevels = 12;
constexpr int kMaxMgCycles = 200;  // cap of the residual-controlled cycle count
// the per-sample cycle count of residual-controlled cycling: above the cap, so that no
// cycle slot is ever the sample's last (the residual check applies the correction)
constexpr int kMgCpp = kMaxMgCycles + 1;
constexpr int kTile = 32;       // output tile edge of the level-streaming kernels
#ifndef RMG_COARSE_TOP_F32
#define RMG_COARSE_TOP_F32 64
#endif
// Finest level of the one-workgroup-per-sample coarse V-cycle kernel; the
// level-streaming kernels handle the finer levels.  Its LDS hierarchy must fit in
// 160 KiB: 64 x 64 and below in FP32, 32 x 32 and below in FP64.
constexpr int coarse_top(bool fp64) { return fp64 ? 32 : RMG_COARSE_TOP_F32; }

// Per-sample iteration state of the level-streaming path (device memory).
// A Picard iteration takes cpp multigrid cycles.  The forward streaming path launches
// J cycle slots per pass (k_fine, then J cycles); a sample runs its cycles cyc0,
// cyc0 + 1, ... in the slots of consecutive passes, so samples whose cycle counts
// differ share one launch sequence (slot j of a pass is cycle cyc0 + j of the sample,
// skipped when cyc0 + j >= cpp).
struct SampleState {
  int32_t active, new_step, step, it;
  int32_t status, tot_its, cycles, nanflag;
  double final_dp;
  int32_t pend;    // adjoint: the step above `step` converged and its gradient term is pending
  int32_t fresh;   // streaming forward: no iteration has run yet (no stopping test pending)
  int32_t cpp;     // cycles per Picard iteration of the current attempt
  int32_t cyc0;    // cycles of the current iteration done before this pass
  int32_t jpass;   // cycle slots of the pass that last wrote this state
  int32_t attempt; // 0: primary setting; 1: fallback setting (restarted from the initial state)
  int32_t mgdone;  // residual-controlled cycling (cpp option 0): the iteration's correction
                   // met eps_mg (or the cycle cap) and was applied in the pass that wrote this
};

// Slot argument of the cycle kernels: kUniform runs the cycle for every active sample
// with the launch's own u_zero / final flags (adjoint); slot j >= 0 takes them from the
// sample's state (cycle cyc0 + j of its iteration).
constexpr int kUniform = -1;
__device__ __forceinline__ bool slot_runs(const SampleState& st, int slot) {
  return st.active && (slot < 0 || st.cyc0 + slot < st.cpp);
}
__device__ __forceinline__ bool slot_first(const SampleState& st, int slot, int uniform_flag) {
  return slot < 0 ? uniform_flag != 0 : st.cyc0 + slot == 0;
}
// (with residual-controlled cycling no cycle is known to be the last one: the correction
// is applied by the residual check after each cycle, so slot_last is false there)
__device__ __forceinline__ bool slot_last(const SampleState& st, int slot, int uniform_flag) {
  return slot < 0 ? uniform_flag != 0 : st.cyc0 + slot + 1 == st.cpp;
}

// The fields of a sample's state that the cycle kernels branch on (active, cyc0, cpp),
// read together: with the short-circuit in slot_runs the compiler would order the
// second load behind a branch on the first, one more memory round trip.
__device__ __forceinline__ SampleState slot_fields(const SampleState* p) {
  SampleState st{};
  st.active = p->active;
  st.cyc0 = p->cyc0;
  st.cpp = p->cpp;
  asm volatile("" ::"v"(st.active), "v"(st.cyc0), "v"(st.cpp));
  return st;
}

// Problems of one grid-size class: samples [0, seg_split) use prob[0], the rest prob[1].
struct ClassProblems {
  rmg_problem prob[2];
  int64_t seg_split;
};

// Per-level arrays of the streaming path.  A down or up kernel reads the iterate
// of its level over its tile plus a halo that other workgroups of the same launch
// own, so it never writes the array it reads: down legs write u, up legs read u and
// write ub, and a down leg that starts from a loaded iterate reads ub.
struct LevelPtrs {
  void* u[kMaxLevels];
  void* ub[kMaxLevels];
  void* f[kMaxLevels];
  void* cw[kMaxLevels];
  void* cs[kMaxLevels];
  void* cdt[kMaxLevels];
  void* ctop[kMaxLevels];
};

// Arrays of the level of one down or up launch, resolved on the host.  The kernel
// reads them at fixed argument offsets in its first batch of scalar loads; indexing
// the plan's per-level tables by a level argument would need a dependent load.
struct LegArgs {
  const void* f;
  const void* cw;
  const void* cs;
  const void* cdt;
  const void* ctop;
  const void* uin;  // iterate read (a down leg that starts from zero reads none)
  void* uout;       // iterate written
  void* fc;         // right-hand side of level l + 1 (the down legs write it)
  const void* uc;   // correction of level l + 1 (the up legs prolong it)
  int l, m;         // level and its edge
  int hb;           // halo of the kernel's region in 2 x 2 blocks
  int lgntx;        // log2 of the output tiles per row
  unsigned mg;      // ceil(2^32 / BW), BW = TS / 2 + 2 hb blocks per region row
};

struct SolveArgs {
  int n, lg, nlev;  // nlev levels from n down to the coarsest grid
  int F;
  int64_t S;
  const double* fields;
  ClassProblems cp;
  int nu1, nu2, cpp, max_picard;
  int fb_cpp, fb_max_picard;  // fallback attempt (fb_cpp = 0: none): a sample that fails with
                              // cpp / max_picard restarts from its initial state with these
  int gamma;  // coarse cycles per level visit: 1 = V-cycle, 2 = W-cycle
  int state_global;  // whole-sample kernel: keep the FP64 state in global memory even if LDS fits
  int fuse_top;      // level streaming with the coarse kernel's top level the finest: one launch
                     // per Picard iteration (set when the class is its call's only streaming class)
  double eps;     // Picard stopping tolerance on ||dp||_inf
  double eps_mg;  // cycles_per_picard == 0: cycle until max |f - A dp| < eps_mg
  double* p;
  double* theta_old;
  double* qoi;
  int32_t* status;
  rmg_sample_stats* stats;
  int64_t s0;  // whole-sample kernel: first sample of the launch (launches cover chunks of S)
  // optional initial pressure head p0 + s * p0_stride (else the problem's uniform h_init)
  const double* p0;
  int64_t p0_stride;
  // optional history: the pressure head after step k (k = 0: initial) for every k that is a
  // multiple of hist_every, at p_hist + (s * hist_slots + k / hist_every) * n * n
  double* p_hist;
  int hist_every, hist_slots;
};

// Level-streaming discrete adjoint (backward through the time steps): the state of one
// segment of steps lo .. hi, solved from hi down to lo.
struct AdjArgs {
  const double* hist;  // pressure heads p^k at hist + (s * slots + k - base) * n * n
  int slots, base;
  int lo, hi;
  int n_steps;         // of the whole integration (layout of qn)
  double* mu;          // [S][n*n] adjoint state (minus the Lagrange multiplier of the step)
  double* b;           // [S][n*n] right-hand side of the current step
  double* g;           // [S][n*n] dQ/dlog Ks accumulated over the converged steps
  double* qn;          // [S][n_steps] outflux F(p^k) of every step
  double eps;          // stop a step when ||d mu||_inf < eps
  int max_its;         // fixed-point iterations allowed per step
};

// Size of the fixed device scratch array of the allocation-free solve entry point.
constexpr size_t kScratchBytes = size_t(64) << 20;
// Device address of that array on the current device.
hipError_t scratch_address(void** ptr);

// LDS bytes of the whole-sample kernel for grid n (0 if it does not fit).
size_t whole_sample_lds_bytes(int n, int nc, bool fp64, int F, bool* state_in_lds);
hipError_t launch_whole_sample(const SolveArgs& a, bool fp64, hipStream_t st);

// Optional timing of the streaming kernels.  A timed launch goes out through
// hipExtLaunchKernelGGL with an event pair that the dispatch itself records, so the
// pair brackets the kernel's execution (not the queue time before it).  One ring of
// event pairs per timed kernel kind; device counters of the work the timed launches
// did (d_cells[0]: down-leg cells with a zero initial iterate, [1]: with a loaded
// iterate, [2]: coarse-kernel sample launches, [4]: fine-kernel cells).
struct EventRing {
  hipEvent_t* ev = nullptr;  // cap event pairs
  int cap = 0;
  int64_t head = 0, tail = 0;  // pairs harvested / recorded so far (tail - head <= cap in flight)
  int64_t launches = 0;
  double total_ms = 0.0;
  bool room() const { return ev && tail - head < cap; }
  hipEvent_t* next() {
    hipEvent_t* e = ev + 2 * (tail % cap);
    ++tail;
    return e;
  }
};
constexpr int kTimedKinds = 3;  // ring 0: down leg, 1: coarse kernel, 2: fine kernel
constexpr int kTimerCounters = 8;
struct KernelTimer {
  int which = 0;  // bit mask of rmg_timed_kernel
  EventRing ring[kTimedKinds];
  unsigned long long* d_cells = nullptr;  // kTimerCounters device counters
};

// Level-streaming path.
struct StreamPlan {
  int n, nlev, ltop;  // ltop: first level handled by the coarse LDS kernel
  int ts[kMaxLevels]; // output tile edge (16 or 32) of the down/up kernels per streaming level
  bool fp64;
  LevelPtrs lv;
  // The per-sample state, the ||dp||_inf maxima and the active-sample counter are
  // double-buffered by iteration parity: iteration i works on state / dpmax /
  // active_count and decides the stopping test of iteration i - 1 from state_prev /
  // dpmax_prev at its start (the fine kernel), so no separate control launch is
  // needed.  flip() gives the plan of the other parity.
  SampleState* state;
  SampleState* state_prev;
  unsigned long long* dpmax;
  unsigned long long* dpmax_prev;
  unsigned long long* mgres;  // residual-controlled cycling: max |f - A dp| of the pass's cycle
  int32_t* active_count;  // [0]: active samples, [1]: of them in the fallback attempt
  int32_t* count_next;    // the counters of the next iteration (cleared by this one)
  KernelTimer* timer;               // host object, never dereferenced on the device
  unsigned long long* tcells;       // device counters of a timed launch, else null
};
inline StreamPlan flip(const StreamPlan& p) {
  StreamPlan q = p;
  q.state = p.state_prev;
  q.state_prev = p.state;
  q.dpmax = p.dpmax_prev;
  q.dpmax_prev = p.dpmax;
  q.active_count = p.count_next;
  q.count_next = p.active_count;
  return q;
}
hipError_t launch_stream_init(const SolveArgs& a, const StreamPlan& pl, hipStream_t st);
// Kernel attributes of the streaming kernels (call once before launching or capturing).
hipError_t prepare_stream(const SolveArgs& a, const StreamPlan& pl);
// One pass of every active sample (the fine kernel, then J cycle slots; a sample whose
// iteration takes cpp <= J cycles completes one Picard iteration per pass): stream
// operations only, capturable.  Successive passes must alternate the plan's parity
// (pl, flip(pl), pl, ...), starting with the plan given to launch_stream_init; the
// state after a pass is in that pass's plan's `state` (its stopping test is taken by
// the next pass, or is pending: the loop ends after a pass in which no sample was
// active, counted in that pass's active_count).
hipError_t launch_stream_iteration(const SolveArgs& a, const StreamPlan& pl, hipStream_t st, int J);
hipError_t launch_stream_finish(const SolveArgs& a, const StreamPlan& pl, hipStream_t st);
// The a.cpp multigrid cycles of one iteration of every active sample (down legs, coarse
// kernel, up legs; the last cycle's finest up leg adds the correction to a.p), with
// uniform flags: the adjoint's fixed-point iteration.
hipError_t launch_stream_cycles(const SolveArgs& a, const StreamPlan& pl, hipStream_t st);

// Adjoint (streaming path).  a.p must point at ad.mu.
hipError_t launch_adj_init(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, const int32_t* fwd_status,
                           hipStream_t st);
hipError_t launch_adj_reset(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, hipStream_t st);
// One fixed-point iteration of every active sample (capturable).
hipError_t launch_adj_iteration(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, hipStream_t st);
// Gradient terms still pending when the segment's loop ended.
hipError_t launch_adj_grad_final(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, hipStream_t st);
hipError_t launch_adj_outflux(const SolveArgs& a, const AdjArgs& ad, hipStream_t st);
// Q[s] = sum_k dt qn[s][k] of a forward solve (NaN where fwd_status is not OK).
hipError_t launch_outflux_total(const SolveArgs& a, const AdjArgs& ad, const int32_t* fwd_status, double* q,
                                hipStream_t st);
hipError_t launch_adj_finish(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, const int32_t* fwd_status,
                             double* q, int32_t* status, rmg_sample_stats* stats, hipStream_t st);
// dQ/dxi[s][j] = sum_c B[j][c] g[s][c] scale (Ks - shift) / Ks (NaN for failed samples).
hipError_t launch_grad_xi(int64_t S, int N, int M, const double* B, const double* g, const double* Ks,
                          rmg_marginal marg, const int32_t* status, double* grad, hipStream_t st);
size_t level_bytes(int m, int64_t S, bool fp64);

// KL fields: out[r][c] = shift_f + exp(log_mean_f + scale_f * sum_k xi[r][k] B[k][c]), f = r mod F.
hipError_t launch_kl_fields(int N, int M, int64_t rows, int F, const double* B, const double* xi,
                            const rmg_marginal* marg, double* out, hipStream_t st);

// Neumaier level sums of one MLMC level.
hipError_t launch_level_sums(const double* qf, const double* qc, int64_t n, const int32_t* stf,
                             const int32_t* stc, const rmg_sample_stats* sf,
                             const rmg_sample_stats* sc, rmg_level_sums* out, hipStream_t st);

}  // namespace rmg
