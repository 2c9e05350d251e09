// Batched modified-Picard / cell-centred multigrid solver kernels (gfx950).
//
// Two execution shapes share the per-cell arithmetic of rmg_device.hpp and
// therefore produce bit-identical iterates:
//   * whole-sample kernel: one workgroup owns one sample for its whole time
//     integration; every multigrid level lives in LDS (used up to 32 x 32, where
//     the FP64 state p, theta_old and the fields live in LDS as well);
//   * level-streaming kernels: one launch per phase of a Picard iteration over
//     all samples of a grid size: the fine residual (k_fine), the down and up
//     legs of the levels finer than the coarse kernel's top (rmg_smoother.hpp),
//     the one-workgroup-per-sample coarse V-cycle in LDS (k_coarse_v) and the
//     stopping test of the previous iteration at the start of k_fine.
// Section 4.1 (modified Picard) and Section 4.2 (cell-centred multigrid).
#include <hip/hip_ext.h>
#include <math.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "rmg_device.hpp"
#include "rmg_internal.hpp"
#include "rmg_lds.hpp"
#include "rmg_smoother.hpp"
#include "rmg_tiles.hpp"

namespace rmg {

// Mean effective saturation (theta - theta_r)/(theta_s - theta_r) over the cells.
// The summation order is fixed independently of the block size: lane t <
// kQoiLanes sums cells t, t + kQoiLanes, ... (thread k computes lanes k, k + B,
// ... for a block of B threads), then a fixed binary tree over the lanes.
constexpr int kQoiLanes = 256;
template <int NT>
__device__ double mean_saturation(const rmg_problem& P, const double* fields, int F, int64_t N,
                                  int64_t s, const double* p, double* red) {
  __syncthreads();
  for (int t = threadIdx.x; t < kQoiLanes; t += NT) {
    double acc = 0.0;
    for (int64_t c = t; c < N; c += kQoiLanes) {
      const CellFields cf = load_fields(fields, F, N, s, c);
      const Closure cl = closure(P, p[c], cf.Ks, cf.alpha, cf.nvg);
      acc += (cl.theta - P.theta_r) / (P.theta_s - P.theta_r);
    }
    red[t] = acc;
  }
  __syncthreads();
  for (int w = kQoiLanes >> 1; w > 0; w >>= 1) {
    for (int t = threadIdx.x; t < w; t += NT) red[t] = red[t] + red[t + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r / (double)N;
}

// ============================================================ whole sample
// LDS doubles ahead of the level arrays: reduction lanes.
__host__ __device__ constexpr int whole_doubles() { return kQoiLanes; }

#ifndef RMG_WS_UNROLL
#define RMG_WS_UNROLL 1
#endif
#ifndef RMG_WS_THREADS
#define RMG_WS_THREADS 512
#endif
constexpr int kUnroll = RMG_WS_UNROLL;  // cells per thread whose global loads are issued together

// One workgroup integrates sample a.s0 + blockIdx.x.
// SL: the FP64 state (pressure head, old moisture content, fields) lives in LDS
// for the whole integration and the pressure head is written back once at the end;
// otherwise it stays in global memory and is read kUnroll cells at a time.
template <class R, int NT, bool SL>
__global__ __launch_bounds__(NT) void k_whole_sample(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t s = a.s0 + blockIdx.x;
  const rmg_problem P = class_problem(a.cp, s);
  const int n = a.n, lg = a.lg, F = a.F;
  const int N = n * n;

  RMG_LDS double* Kc = (RMG_LDS double*)smem;
  double* red = (double*)(Kc + N);
  double* dend = red + kQoiLanes;
  double* pS = dend;
  double* thS = pS + (SL ? N : 0);
  double* fS = thS + (SL ? N : 0);
  R* rbase = (R*)(fS + (SL ? F * N : 0));
  const LdsHier<R> lev = lds_hier(rbase, n);
  R* rend = lev.end(a.nlev);
  for (R* q = rbase + threadIdx.x; q < rend; q += NT) *q = (R)0;

  double* pg = a.p + s * N;
  double* const p = SL ? pS : pg;
  double* const thold = SL ? thS : a.theta_old + s * N;
  const double* const fld = SL ? fS : a.fields + s * F * N;  // field f of cell c at fld[f*N + c]
  for (int c = threadIdx.x; c < N; c += NT) {
    p[c] = a.p0 ? a.p0[s * a.p0_stride + c] : initial_head(P, c >> lg, n);
    if (SL)
      for (int f = 0; f < F; ++f) fS[f * N + c] = a.fields[(s * F + f) * N + c];
  }
  __syncthreads();

  int step = 0, it = 0, new_step = 1, status = RMG_SAMPLE_OK, tot_its = 0, cycles = 0;
  int attempt = 0, cpp = a.cpp, maxp = a.max_picard;  // the fallback attempt changes both
  double dp = 0.0;
  const LdsLevel<R> L0 = lev[0];
  // a sample whose fields hold a non-finite value is not solved (input validation)
  double fbad = 0.0;
  for (int c = threadIdx.x; c < N; c += NT)
    for (int f = 0; f < F; ++f)
      if (!isfinite(fld[f * N + c])) fbad = 1.0;
  if (block_max<NT>(fbad, red) > 0.0) status = RMG_SAMPLE_NONFINITE;
  while (status == RMG_SAMPLE_OK) {
    // conductivity at every cell (FP64)
    for (int c0 = threadIdx.x; c0 < N; c0 += kUnroll * NT) {
      double pv[kUnroll], k0[kUnroll], k1[kUnroll], k2[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int c = c0 + q * NT;
        if (c < N) {
          pv[q] = p[c];
          k0[q] = fld[c];
          k1[q] = F > 1 ? fld[N + c] : 0.0;
          k2[q] = F > 2 ? fld[2 * N + c] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int c = c0 + q * NT;
        if (c < N) Kc[c] = closure(P, pv[q], k0[q], k1[q], k2[q]).K;
      }
    }
    __syncthreads();
    // outer residual and fine-level coefficients
    double* hist = nullptr;  // history slot of the step that starts here, if recorded
    if (new_step && a.p_hist && step % a.hist_every == 0)
      hist = a.p_hist + (s * a.hist_slots + step / a.hist_every) * N;
    for (int c0 = threadIdx.x; c0 < N; c0 += kUnroll * NT) {
      double pc[kUnroll], pw[kUnroll], pe[kUnroll], ps[kUnroll], pn[kUnroll], to[kUnroll];
      double k0[kUnroll], k1[kUnroll], k2[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int c = c0 + q * NT;
        if (c < N) {
          const int j = c >> lg, i = c - (j << lg);
          pc[q] = p[c];
          pw[q] = i > 0 ? p[c - 1] : 0.0;
          pe[q] = i < n - 1 ? p[c + 1] : 0.0;
          ps[q] = j > 0 ? p[c - n] : 0.0;
          pn[q] = j < n - 1 ? p[c + n] : 0.0;
          to[q] = new_step ? 0.0 : thold[c];
          k0[q] = fld[c];
          k1[q] = F > 1 ? fld[N + c] : 0.0;
          k2[q] = F > 2 ? fld[2 * N + c] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int c = c0 + q * NT;
        if (c >= N) continue;
        const int j = c >> lg, i = c - (j << lg);
        const Closure cl = closure(P, pc[q], k0[q], k1[q], k2[q]);
        double th_old = to[q];
        if (new_step) {
          th_old = cl.theta;
          thold[c] = cl.theta;
          if (hist) hist[c] = pc[q];
        }
        const double Kw = i > 0 ? Kc[c - 1] : 0.0, Ke = i < n - 1 ? Kc[c + 1] : 0.0;
        const double Ks_ = j > 0 ? Kc[c - n] : 0.0, Kn = j < n - 1 ? Kc[c + n] : 0.0;
        const FineCell fc = fine_cell(i, j, n, pc[q], pw[q], pe[q], ps[q], pn[q], Kc[c], Kw, Ke, Ks_, Kn,
                                      cl.theta, th_old, cl.C, P.dt, P.h_bottom, P.h_top);
        L0.f[c] = (R)fc.f;
        L0.cw[c] = (R)fc.cw;
        L0.cs[c] = (R)fc.cs;
        L0.cdt[c] = (R)fc.cdt;
        if (j == n - 1) L0.cs[c + n] = (R)fc.ctop;
        L0.u[c] = (R)0;
      }
    }
    __syncthreads();
    // a fixed number of cycles, or (cpp == 0) cycles until the correction equation's
    // residual max_c |f - A dp| (level 0, smoother precision) is below eps_mg; the
    // first cycle forms the coarse levels' coefficients on its way down
    int ncyc = 0;
    for (;;) {
      lds_cycle_whole<R, NT>(lev, a.nlev, a.nu1, a.nu2, a.gamma, ncyc == 0, ncyc == 0);
      ++ncyc;
      if (cpp > 0) {
        if (ncyc == cpp) break;
        continue;
      }
      double rmax = 0.0;
      for (int c = threadIdx.x; c < N; c += NT)
        rmax = fmax(rmax, fabs((double)residual_value<R>(L0.f[c], L0.u[c], lds_st5(L0, c))));
      rmax = block_max<NT>(rmax, red);
      if (rmax < a.eps_mg || ncyc == kMaxMgCycles) break;
    }
    // Picard update p <- p + dp and ||dp||_inf
    double mx = 0.0, bad = 0.0;
    for (int c0 = threadIdx.x; c0 < N; c0 += kUnroll * NT) {
      double pv[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int c = c0 + q * NT;
        if (c < N) pv[q] = p[c];
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int c = c0 + q * NT;
        if (c >= N) continue;
        const double d = (double)L0.u[c];
        p[c] = pv[q] + d;
        mx = fmax(mx, fabs(d));
        if (!isfinite(d)) bad = 1.0;
      }
    }
    dp = block_max<NT>(mx, red);
    const double anybad = block_max<NT>(bad, red);
    ++it;
    ++tot_its;
    cycles += ncyc;
    int fail = RMG_SAMPLE_OK;
    if (anybad > 0.0) {
      fail = RMG_SAMPLE_NONFINITE;
    } else if (dp < a.eps) {
      ++step;
      it = 0;
      new_step = 1;
      if (step == P.n_steps) break;
    } else {
      new_step = 0;
      if (it >= maxp) fail = RMG_SAMPLE_MAXITER;
    }
    if (fail != RMG_SAMPLE_OK) {
      if (a.fb_cpp > 0 && attempt == 0) {
        // fallback: restart from the initial state with the fallback's cycles and limit
        attempt = 1;
        cpp = a.fb_cpp;
        maxp = a.fb_max_picard;
        step = 0;
        it = 0;
        new_step = 1;
        for (int c = threadIdx.x; c < N; c += NT) p[c] = a.p0 ? a.p0[s * a.p0_stride + c] : initial_head(P, c >> lg, n);
        __syncthreads();
        continue;
      }
      status = fail;
      break;
    }
  }
  __syncthreads();
  if (SL)
    for (int c = threadIdx.x; c < N; c += NT) pg[c] = p[c];
  if (a.p_hist && status == RMG_SAMPLE_OK && P.n_steps % a.hist_every == 0) {
    double* hist = a.p_hist + (s * a.hist_slots + P.n_steps / a.hist_every) * N;
    for (int c = threadIdx.x; c < N; c += NT) hist[c] = p[c];
  }
  const double q = mean_saturation<NT>(P, fld, F, N, 0, p, red);
  if (threadIdx.x == 0) {
    a.qoi[s] = status == RMG_SAMPLE_OK ? q : __longlong_as_double(0x7ff8000000000000ll);
    a.status[s] = status;
    if (a.stats) {
      rmg_sample_stats st;
      st.picard_its = tot_its;
      st.mg_cycles = cycles;
      st.steps_done = step;
      st.status = status;
      st.final_dp_inf = dp;
      st.attempts = attempt + 1;
      st.reserved = 0;
      a.stats[s] = st;
    }
  }
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// LDS bytes of the whole-sample kernel (0 if it does not fit); *state_in_lds tells
// whether the FP64 state fits as well (preferred up to 32 x 32).
static size_t ws_bytes(int n, int nc, bool fp64, int F, bool state) {
  const int nlev = ilog2(n) - ilog2(nc) + 1;
  size_t relems = 0;
  for (int l = 0, m = n; l < nlev; ++l, m >>= 1) relems += lds_level_elems(m);
  const size_t N = (size_t)n * n;
  return 8 * (N + whole_doubles() + (state ? (2 + F) * N : 0)) + relems * (fp64 ? 8 : 4);
}

size_t whole_sample_lds_bytes(int n, int nc, bool fp64, int F, bool* state_in_lds) {
  const size_t cap = 160 * 1024;
  const size_t with = ws_bytes(n, nc, fp64, F, true), without = ws_bytes(n, nc, fp64, F, false);
  const bool st = n <= 32 && with <= cap;
  if (state_in_lds) *state_in_lds = st;
  const size_t b = st ? with : without;
  return b <= cap ? b : 0;
}

// The dynamic-LDS limit of a kernel is a property of the kernel on its device, not of
// a context: it is only ever raised (to the largest size a launch has needed so far),
// under a lock, so that calls on separate contexts from separate host threads cannot
// lower it between another call's setting and its launch.
constexpr int kLdsDevices = 64;  // devices of one process whose limits are tracked
static hipError_t raise_dyn_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> set[kLdsDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kLdsDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = set[dev][fn];
  if (bytes <= cur) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) cur = bytes;
  return e;
}

template <class R, int NT, bool SL>
static hipError_t launch_ws(const SolveArgs& a, size_t lds, hipStream_t st) {
  hipError_t e = raise_dyn_lds((const void*)k_whole_sample<R, NT, SL>, lds);
  if (e != hipSuccess) return e;
  // grid dimension x holds at most 2^31 - 1 workgroups: larger classes go out in parts
  constexpr int64_t kMaxGrid = 1 << 30;
  for (int64_t s0 = 0; s0 < a.S; s0 += kMaxGrid) {
    SolveArgs b = a;
    b.s0 = s0;
    const int64_t g = a.S - s0 < kMaxGrid ? a.S - s0 : kMaxGrid;
    hipLaunchKernelGGL((k_whole_sample<R, NT, SL>), dim3((unsigned)g), dim3(NT), lds, st, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

#ifndef RMG_WS_NT16
#define RMG_WS_NT16 128
#endif
#ifndef RMG_WS_NT32
#define RMG_WS_NT32 256
#endif
// Threads per whole-sample workgroup (state in LDS) for grids up to 16 x 16 and
// 32 x 32.  The small-grid classes hold thousands of samples, so throughput is set
// by how many samples a compute unit keeps in flight, and one or two waves per
// sample turn most barriers into wave barriers.
template <class R>
static hipError_t launch_ws_sl(const SolveArgs& a, size_t lds, hipStream_t st) {
  if (a.n <= 16) return launch_ws<R, RMG_WS_NT16, true>(a, lds, st);
  if (a.n <= 32) return launch_ws<R, RMG_WS_NT32, true>(a, lds, st);
  return launch_ws<R, 256, true>(a, lds, st);
}

hipError_t launch_whole_sample(const SolveArgs& a, bool fp64, hipStream_t st) {
  const int nc = a.n >> (a.nlev - 1);
  bool sl = false;
  size_t lds = whole_sample_lds_bytes(a.n, nc, fp64, a.F, &sl);
  if (lds == 0) return hipErrorInvalidValue;
  if (sl && a.state_global) {
    sl = false;
    lds = ws_bytes(a.n, nc, fp64, a.F, false);
  }
  constexpr int T = RMG_WS_THREADS;
  if (fp64) return sl ? launch_ws_sl<double>(a, lds, st) : launch_ws<double, T, false>(a, lds, st);
  return sl ? launch_ws_sl<float>(a, lds, st) : launch_ws<float, T, false>(a, lds, st);
}

// ============================================================ level streaming
__global__ void k_stream_init(SolveArgs a, StreamPlan pl) {
  // n is a power of two: sample and cell of element e by shifts (no 64-bit division)
  const int lg = a.lg;
  const int64_t N = (int64_t)1 << (2 * lg);
  const int64_t tot = a.S * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e >> (2 * lg);
    const int c = (int)(e & (N - 1));
    a.p[e] = a.p0 ? a.p0[s * a.p0_stride + c] : initial_head(class_problem(a.cp, s), c >> lg, a.n);
  }
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < a.S;
       s += (int64_t)gridDim.x * blockDim.x) {
    SampleState z;
    z.active = 1;
    z.new_step = 1;
    z.step = 0;
    z.it = 0;
    z.status = RMG_SAMPLE_OK;
    z.tot_its = 0;
    z.cycles = 0;
    z.nanflag = 0;
    z.final_dp = 0.0;
    z.pend = 0;
    z.fresh = 1;
    z.cpp = a.cpp > 0 ? a.cpp : kMgCpp;
    z.cyc0 = 0;
    z.jpass = 0;
    z.attempt = 0;
    z.mgdone = 0;
    pl.state[s] = z;
    pl.state_prev[s] = z;
    pl.dpmax[s] = 0ull;
    pl.dpmax_prev[s] = 0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    pl.active_count[0] = pl.active_count[1] = 0;
    pl.count_next[0] = pl.count_next[1] = 0;
  }
}

// The stopping test and step bookkeeping of one sample after a Picard iteration
// whose ||dp||_inf is dp (Section 4.1: stop the step when ||dp||_inf < eps_PI;
// Section 4.3: give up after max_picard iterations in a step).  A sample that fails
// with the primary setting while a fallback is configured is not given up: it
// restarts from its initial state with the fallback's cycles per Picard iteration
// and iteration limit (the return value is true then; iteration and cycle totals
// keep counting).
__device__ __forceinline__ bool control_step(SampleState& st, double dp, const SolveArgs& a, const rmg_problem& P) {
  st.it += 1;
  st.tot_its += 1;
  st.cycles += st.cpp;
  st.final_dp = dp;
  int fail;
  if (st.nanflag) {
    fail = RMG_SAMPLE_NONFINITE;
  } else if (dp < a.eps) {
    st.step += 1;
    st.it = 0;
    st.new_step = 1;
    if (st.step == P.n_steps) st.active = 0;
    return false;
  } else {
    st.new_step = 0;
    if (st.it < (st.attempt ? a.fb_max_picard : a.max_picard)) return false;
    fail = RMG_SAMPLE_MAXITER;
  }
  if (a.fb_cpp > 0 && st.attempt == 0) {
    st.attempt = 1;
    st.cpp = a.fb_cpp;
    st.step = 0;
    st.it = 0;
    st.new_step = 1;
    st.nanflag = 0;
    return true;
  }
  st.status = fail;
  st.active = 0;
  return false;
}

// Pressure head of cell c = j n + i before the first step: the optional caller-given
// initial state, else the problem's initial condition.
__device__ __forceinline__ double start_head(const SolveArgs& a, const rmg_problem& P, int64_t s, int64_t c, int j,
                                             int n) {
  return a.p0 ? a.p0[s * a.p0_stride + c] : initial_head(P, j, n);
}

// Outer residual + fine coefficients for one tile, then the coarser levels
// 1 .. ltop of the same tile by in-tile coarsening (cells of level l inside a
// 32 x 32 fine tile are complete for 2^l <= 32).
// Start of a pass (J cycle slots follow): the stopping test of a sample whose iteration
// ended in the previous pass, the cycle count of one whose iteration is still running.
// Every workgroup of the sample takes the same decision; the first one stores it and
// clears this pass's maximum.  Returns whether the sample restarts from its initial state.
__device__ __forceinline__ bool pass_control(SampleState& st, const SolveArgs& a, const StreamPlan& pl,
                                             const rmg_problem& P, int64_t s, int J, bool store,
                                             unsigned long long dp_prev) {
  bool restart = false;
  if (st.fresh) {
    st.fresh = 0;
    st.cyc0 = 0;
  } else if (st.active) {
    const int done = st.cyc0 + st.jpass;
    if (a.cpp == 0) {  // residual-controlled cycling: the residual check applied the correction
      if (st.mgdone) {
        st.cpp = done;  // cycles of the iteration, for the totals
        restart = control_step(st, __longlong_as_double((long long)dp_prev), a, P);
        st.cpp = kMgCpp;
        st.cyc0 = 0;
        st.mgdone = 0;
      } else {
        st.cyc0 = done;
      }
    } else if (done >= st.cpp) {
      restart = control_step(st, __longlong_as_double((long long)dp_prev), a, P);
      st.cyc0 = 0;
    } else {
      st.cyc0 = done;
    }
  }
  st.jpass = J;
  if (store) {
    pl.state[s] = st;
    pl.dpmax[s] = 0ull;
    if (pl.mgres) pl.mgres[s] = 0ull;
    if (st.active) {
      atomicAdd(pl.active_count, 1);
      if (st.attempt) atomicAdd(pl.active_count + 1, 1);
    }
    if (s == 0) pl.count_next[0] = pl.count_next[1] = 0;
  }
  return restart;
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_fine(SolveArgs a, StreamPlan pl, int J) {
  __shared__ double sp[34 * 34], sK[34 * 34];
  __shared__ R bufA[3 * 32 * 32 + 32], bufB[3 * 16 * 16 + 16];
  // the arguments of the prologue in one batch of scalar loads; then the sample's
  // state and its previous iteration's ||dp||_inf together
  sgpr_ready_all((int)gridDim.x, (const void*)pl.state_prev, (const void*)pl.dpmax_prev, (const void*)pl.state,
                 (const void*)pl.dpmax, (const void*)pl.mgres, (const void*)pl.active_count,
                 (const void*)pl.count_next, (const void*)pl.tcells, (const void*)a.p, (const void*)a.theta_old,
                 (const void*)a.fields, (const void*)a.p0, a.n, a.F, a.cpp, a.max_picard, a.fb_cpp,
                 a.fb_max_picard, J);
  const SampleTile w = xcd_sample_tile();
  const int64_t s = w.s;
  const rmg_problem P = class_problem(a.cp, s);
  SampleState st = pl.state_prev[s];
  const unsigned long long dp_prev = pl.dpmax_prev[s];
  asm volatile("" ::"v"(st.active), "v"(st.fresh), "v"(st.cyc0), "v"(st.jpass), "v"(dp_prev));
  const bool restart = pass_control(st, a, pl, P, s, J, w.tile == 0 && threadIdx.x == 0, dp_prev);
  // a sample in the middle of its iteration keeps the coefficients formed at its start
  if (!st.active || st.cyc0 > 0) return;
  const int new_step = st.new_step;
  const int n = a.n;
  if (pl.tcells && w.tile == 0 && threadIdx.x == 0)  // timed: cells (once per sample)
    atomicAdd(pl.tcells, (unsigned long long)n * (unsigned long long)n);
  const int T = n < kTile ? n : kTile, TL = T + 2;
  const int ntx = n / T;
  const int tile = w.tile;
  const int x0 = (tile % ntx) * T, y0 = (tile / ntx) * T;
  const int64_t N = (int64_t)n * n;
  double* p = a.p + s * N;
  double* thold = a.theta_old + s * N;
  // The tile's own cells (T = 32 or n, a power of two; k = threadIdx.x + q kBlock):
  // pressure head and closure once per cell, K and p to LDS for the neighbours, the
  // moisture content and capacity kept in registers for the cell phase after the
  // barrier; the old moisture content is loaded here as well, so that its loads are
  // in flight meanwhile.  Then the halo ring (one cell per thread): p and K only.
  constexpr int Q = (kTile * kTile + kBlock - 1) / kBlock;
  const int lgT = 31 - __clz(T);
  double cth[Q], cC[Q], pth[Q], pvq[Q];
  CellFields cfq[Q];
  // every global load of the own cells first (a thread beyond a smaller tile reads the
  // tile's last cell and discards it), so that they are in flight together
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = min((int)threadIdx.x + q * kBlock, T * T - 1);
    const int64_t c = (int64_t)(y0 + (k >> lgT)) * n + x0 + (k & (T - 1));
    cfq[q] = load_fields(a.fields, a.F, N, s, c);
    pth[q] = new_step ? 0.0 : thold[c];
    pvq[q] = restart ? 0.0 : p[c];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = (int)threadIdx.x + q * kBlock;
    cth[q] = cC[q] = 0.0;
    if (k < T * T) {
      const int lj = k >> lgT, li = k & (T - 1);
      const int64_t c = (int64_t)(y0 + lj) * n + x0 + li;
      double pv = pvq[q];
      if (restart) {  // a restart re-initialises the head (every workgroup of the sample reads
        pv = start_head(a, P, s, c, y0 + lj, n);  // it from the initial state, not from p)
        p[c] = pv;
      }
      const Closure cl = closure(P, pv, cfq[q].Ks, cfq[q].alpha, cfq[q].nvg);
      const int le = (lj + 1) * TL + li + 1;
      sp[le] = pv;
      sK[le] = cl.K;
      cth[q] = cl.theta;
      cC[q] = cl.C;
    } else {
      pth[q] = 0.0;
    }
  }
  for (int r = threadIdx.x; r < 4 * TL - 4; r += kBlock) {
    int li, lj;  // bottom row, top row, then the left and right columns without corners
    if (r < TL) {
      li = r;
      lj = 0;
    } else if (r < 2 * TL) {
      li = r - TL;
      lj = TL - 1;
    } else {
      const int q = r - 2 * TL;
      li = (q & 1) ? TL - 1 : 0;
      lj = 1 + (q >> 1);
    }
    const int gi = x0 - 1 + li, gj = y0 - 1 + lj;
    const int le = lj * TL + li;
    double pv = 0.0, K = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      const int64_t c = (int64_t)gj * n + gi;
      pv = restart ? start_head(a, P, s, c, gj, n) : p[c];
      const CellFields cf = load_fields(a.fields, a.F, N, s, c);
      K = closure(P, pv, cf.Ks, cf.alpha, cf.nvg).K;
    }
    sp[le] = pv;
    sK[le] = K;
  }
  __syncthreads();
  R* tcw = bufA;
  R* tcdt = bufA + T * T;
  R* tcs = bufA + 2 * T * T;  // (T+1) x T, row T = top Dirichlet weights
  R* f0 = (R*)pl.lv.f[0] + s * N;
  R* cw0 = (R*)pl.lv.cw[0] + s * N;
  R* cs0 = (R*)pl.lv.cs[0] + s * N;
  R* cdt0 = (R*)pl.lv.cdt[0] + s * N;
  R* ctop0 = (R*)pl.lv.ctop[0] + s * n;
  double* hist = nullptr;  // history slot of the step that starts here, if recorded
  if (new_step && a.p_hist) {
    const int k = st.step;
    if (k % a.hist_every == 0) hist = a.p_hist + (s * a.hist_slots + k / a.hist_every) * N;
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = (int)threadIdx.x + q * kBlock;
    if (k >= T * T) continue;
    const int lj = k >> lgT, li = k & (T - 1);
    const int e = lj * T + li;
    const int gi = x0 + li, gj = y0 + lj;
    const int64_t c = (int64_t)gj * n + gi;
    const int le = (lj + 1) * TL + li + 1;
    double th_old;
    if (new_step) {
      th_old = cth[q];
      thold[c] = cth[q];
      if (hist) hist[c] = sp[le];
    } else {
      th_old = pth[q];
    }
    const FineCell fc = fine_cell(gi, gj, n, sp[le], sp[le - 1], sp[le + 1], sp[le - TL], sp[le + TL],
                                  sK[le], sK[le - 1], sK[le + 1], sK[le - TL], sK[le + TL], cth[q],
                                  th_old, cC[q], P.dt, P.h_bottom, P.h_top);
    const R rf = (R)fc.f, rcw = (R)fc.cw, rcs = (R)fc.cs, rcdt = (R)fc.cdt;
    f0[c] = rf;
    cw0[c] = rcw;
    cs0[c] = rcs;
    cdt0[c] = rcdt;
    tcw[e] = rcw;
    tcs[e] = rcs;
    tcdt[e] = rcdt;
    if (lj == T - 1) {
      const R rct = (R)fc.ctop;
      tcs[T * T + li] = rct;
      if (gj == n - 1) ctop0[gi] = rct;
    }
  }
  tile_coarsen<R>(pl, s, n, T, x0, y0, bufA, bufB);
}

// Levels ltop .. nlev-1 of one sample in LDS: load level ltop, coarsen, V-cycle,
// store its correction (or, when ltop is the finest level, apply the Picard update).
#ifndef RMG_COARSE_THREADS
#define RMG_COARSE_THREADS 512
#endif
// Threads per sample of the coarse kernel.  The coarse V-cycle is a long chain of
// small sweeps on the critical path of every Picard iteration; few samples run
// it at once, so its latency falls with the threads per sample (measured on the
// 256^2 class: 64 threads 102, 256 threads 85, 512 threads 82 us per iteration).
constexpr int kCoarseThreads = RMG_COARSE_THREADS;
// 16-byte vectors for the global loads and stores of the coarse kernel.
template <class R> struct Vec16;
template <> struct Vec16<float> { using T = float4; };
template <> struct Vec16<double> { using T = double2; };

// ---------------------------------------------------------------------------
// The 64 x 64 top level of the coarse kernel in the register-block form of the
// streaming smoother (FP32, 512 threads, two 2 x 2 blocks per thread).  Each thread
// loads its blocks' right-hand side, coefficients and iterate from global memory
// straight into registers (no staging of the level in LDS); LDS mirrors only the
// iterate, with a zero ring, in the top level's place of the hierarchy.  A red-black
// update reads two neighbours from LDS, the residual restriction eight per block and
// no coefficient, and the coarsening of the coefficients (Section 4.2) uses the
// block's registers.  The first red half-sweep after the coarse correction reads
// its neighbours as iterate plus the prolongated correction (eq. transfer), so the
// up leg needs no separate prolongation phase.  Per cell the operations and their
// order are those of lds_cycle_top_cached, so the results are bit-identical.
constexpr int kTopBlkM = 64;
template <class R, int NT>
struct TopBlk {
  static constexpr int NB = kTopBlkM * kTopBlkM / 4 / NT;
  Blk<R> b[NB];
  R cdt[NB][4];
  int bx[NB], by[NB];
  bool live[NB];
};

template <class R, int NT>
__device__ __forceinline__ void top_blk_setup(TopBlk<R, NT>& T, BlkRegion& g, RMG_LDS R* L, const R* F, const R* CW,
                                              const R* CS, const R* CDT, const R* CT, const R* U, bool u_zero,
                                              const LdsHier<R>& lev, int nlev) {
  constexpr int M = kTopBlkM, NB = TopBlk<R, NT>::NB;
  g.hb = 0;
  g.BW = M / 2;
  g.UW = M + 2;
  g.gbx0 = g.gby0 = 0;
  g.mb = M / 2;
  // the loads of all of the thread's blocks are in flight before the first is used
  BlkRaw<R> raw[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int k = (int)threadIdx.x + q * NT;
    T.by[q] = k / (M / 2);
    T.bx[q] = k % (M / 2);
    T.live[q] = true;
    blk_fetch(raw[q], g, T.bx[q], T.by[q], M, F, CW, CS, CDT, CT, (const R*)nullptr, M / 2);
  }
  if (!u_zero) {
#pragma unroll
    for (int q = 0; q < NB; ++q) blk_fetch_u(raw[q], g, T.bx[q], T.by[q], M, U);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) blk_build(T.b[q], raw[q], u_zero, false, T.cdt[q]);
  // the padding of the levels below, while the global loads above are in flight
  lds_zero_padding<R, NT>(lev.base + lev.offset(1), M / 2, nlev - 1);
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int k = 0; k < 4; ++k) L[blk_lds(g, 2 * T.bx[q] + (k & 1), 2 * T.by[q] + (k >> 1))] = T.b[q].u[k];
  for (int e = threadIdx.x; e < 4 * (M + 1); e += NT) {
    const int side = e / (M + 1), i = e - side * (M + 1);
    int lx, ly;
    if (side == 0) { lx = i - 1; ly = -1; }
    else if (side == 1) { lx = i; ly = M; }
    else if (side == 2) { lx = -1; ly = i; }
    else { lx = M; ly = i - 1; }
    L[blk_lds(g, lx, ly)] = (R)0;
  }
  __syncthreads();
}

template <class R, int NT>
__device__ __forceinline__ void top_blk_sweeps(TopBlk<R, NT>& T, const BlkRegion& g, RMG_LDS R* L, int nu) {
  for (int st = 0; st < 2 * nu; ++st) {
    if (st & 1)
      blk_half_sweep<R, TopBlk<R, NT>::NB, 1>(T.b, T.live, T.bx, T.by, g, L);
    else
      blk_half_sweep<R, TopBlk<R, NT>::NB, 0>(T.b, T.live, T.bx, T.by, g, L);
    __syncthreads();
  }
}

// Residual, its restriction to level 1 (zero iterate there) and, with `coarsen`, the
// level-1 coefficients.
template <class R, int NT>
__device__ __forceinline__ void top_blk_restrict(const TopBlk<R, NT>& T, const BlkRegion& g, const RMG_LDS R* L,
                                                 const LdsLevel<R>& C, bool coarsen) {
  constexpr int MC = kTopBlkM / 2;
#pragma unroll
  for (int q = 0; q < TopBlk<R, NT>::NB; ++q) {
    const Blk<R>& b = T.b[q];
    R r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const R snb = blk_cell_snb(b, g, L, T.bx[q], T.by[q], k);
      r[k] = (b.f[k] + snb) - b.d[k] * b.u[k];
    }
    const int kc = T.by[q] * MC + T.bx[q];
    C.f[kc] = restrict4<R>(r[0], r[1], r[2], r[3]);
    C.u[kc] = (R)0;
    if (coarsen) {
      C.cw[kc] = coarse_face<R>(b.vx[0][0], b.vx[1][0]);
      C.cs[kc] = coarse_face<R>(b.vy[0][0], b.vy[1][0]);
      C.cdt[kc] = coarse_cdt<R>(T.cdt[q][0], T.cdt[q][1], T.cdt[q][2], T.cdt[q][3]);
      if (T.by[q] == MC - 1) C.cs[MC * MC + T.bx[q]] = coarse_face<R>(b.vy[0][2], b.vy[1][2]);
    }
  }
}

// Up leg: nu2 sweeps after the coarse correction of level 1 (prolongation folded into
// the first red half-sweep), or the plain prolongation when nu2 = 0.
template <class R, int NT>
__device__ __forceinline__ void top_blk_up(TopBlk<R, NT>& T, const BlkRegion& g, RMG_LDS R* L, const LdsLevel<R>& C,
                                           int nu2) {
  constexpr int MC = kTopBlkM / 2, NB = TopBlk<R, NT>::NB;
  if (nu2 == 0) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const R uc = C.u[T.by[q] * MC + T.bx[q]];
#pragma unroll
      for (int k = 0; k < 4; ++k) T.b[q].u[k] = T.b[q].u[k] + uc;
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    Blk<R>& b = T.b[q];
    const int bx = T.bx[q], by = T.by[q];
    const int x = 2 * bx, y = 2 * by;
    const R uc = C.u[by * MC + bx];
    const R z = (R)0;
    // cell 0 = (x, y) and cell 3 = (x + 1, y + 1); their in-block neighbours are black
    const R w0 = bx > 0 ? L[blk_lds(g, x - 1, y)] + C.u[by * MC + bx - 1] : z;
    const R e0 = b.u[1] + uc;
    const R s0 = by > 0 ? L[blk_lds(g, x, y - 1)] + C.u[(by - 1) * MC + bx] : z;
    const R n0 = b.u[2] + uc;
    const R w3 = b.u[2] + uc;
    const R e3 = bx < MC - 1 ? L[blk_lds(g, x + 2, y + 1)] + C.u[by * MC + bx + 1] : z;
    const R s3 = b.u[1] + uc;
    const R n3 = by < MC - 1 ? L[blk_lds(g, x + 1, y + 2)] + C.u[(by + 1) * MC + bx] : z;
    const R sn0 = blk_snb<R>(b.vx[0][0], b.vx[0][1], b.vy[0][0], b.vy[0][1], w0, e0, s0, n0);
    const R sn3 = blk_snb<R>(b.vx[1][1], b.vx[1][2], b.vy[1][1], b.vy[1][2], w3, e3, s3, n3);
    b.u[0] = blk_gs(b.f[0], sn0, b.d[0], b.rd[0]);
    b.u[3] = blk_gs(b.f[3], sn3, b.d[3], b.rd[3]);
    // red cells read only black ones, so they can be published at once
    L[blk_lds(g, x, y)] = b.u[0];
    L[blk_lds(g, x + 1, y + 1)] = b.u[3];
  }
  __syncthreads();
  blk_half_sweep<R, NB, 1>(T.b, T.live, T.bx, T.by, g, L);
  __syncthreads();
  top_blk_sweeps<R, NT>(T, g, L, nu2 - 1);
}

#ifndef RMG_TOP_BLK
#define RMG_TOP_BLK 1
#endif
// k_coarse_v on a 64 x 64 top level (FP32): the register-block top level, the levels
// below it as lds_cycle_top_cached runs them, then the store of the correction or
// (fin) the Picard update.
template <class R, int NT>
__device__ void coarse_v_top_blk(const SolveArgs& a, const StreamPlan& pl, const LegArgs& lg, int64_t s,
                                 const LdsHier<R>& lev, int nlev, bool u_zero, bool fin) {
  constexpr int M = kTopBlkM, NB = TopBlk<R, NT>::NB;
  constexpr int64_t M2 = (int64_t)M * M;
  RMG_LDS R* L = (RMG_LDS R*)lev.base;
  TopBlk<R, NT> T;
  BlkRegion g;
  R* U = (R*)lg.uout + s * M2;
  top_blk_setup<R, NT>(T, g, L, (const R*)lg.f + s * M2, (const R*)lg.cw + s * M2, (const R*)lg.cs + s * M2,
                       (const R*)lg.cdt + s * M2, (const R*)lg.ctop + s * M, U, u_zero, lev, nlev);
  top_blk_sweeps<R, NT>(T, g, L, a.nu1);
  top_blk_restrict<R, NT>(T, g, L, lev[1], true);
  __syncthreads();
  for (int gg = 0; gg < a.gamma; ++gg) {
    if (RMG_NEST_CACHE && nlev >= 3)
      lds_cycle_top_cached<R, NT, M / 2, 0, 1>(lev, nlev, a.nu1, a.nu2, a.gamma, gg == 0, gg == 0);
    else
      lds_cycle<R, NT>(lev, 1, nlev, a.nu1, a.nu2, a.gamma, gg == 0, gg == 0);
  }
  top_blk_up<R, NT>(T, g, L, lev[1], a.nu2);
  using V = typename Vec2<R>::T;
  if (!fin) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int64_t c0 = (int64_t)(2 * T.by[q]) * M + 2 * T.bx[q];
      V o0, o1;
      o0.x = T.b[q].u[0];
      o0.y = T.b[q].u[1];
      o1.x = T.b[q].u[2];
      o1.y = T.b[q].u[3];
      *(V*)(U + c0) = o0;
      *(V*)(U + c0 + M) = o1;
    }
    return;
  }
  double* p = a.p + s * M2;
  double* red = (double*)lev.base - (NT / 64 + 1);
  double mx = 0.0, bad = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int64_t c0 = (int64_t)(2 * T.by[q]) * M + 2 * T.bx[q];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t c = c0 + (k >> 1) * M + (k & 1);
      const double d = (double)T.b[q].u[k];
      p[c] += d;
      mx = fmax(mx, fabs(d));
      if (!isfinite(d)) bad = 1.0;
    }
  }
  mx = block_max<NT>(mx, red);
  bad = block_max<NT>(bad, red);
  if (threadIdx.x == 0) {
    pl.dpmax[s] = (unsigned long long)__double_as_longlong(mx);
    if (bad > 0.0) pl.state[s].nanflag = 1;
  }
}

template <class R, int NT>
__global__ __launch_bounds__(NT) void k_coarse_v(SolveArgs a, StreamPlan pl, LegArgs lg, int u_zero_, int final_,
                                                 int slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t s = blockIdx.x;
  // every argument of the prologue in one batch of scalar loads, then the sample's state
  sgpr_ready_all((const void*)pl.state, (const void*)pl.tcells, (const void*)pl.dpmax, (const void*)a.p, lg.f,
                 lg.cw, lg.cs, lg.cdt, lg.ctop, lg.uout, lg.l, a.n, a.nlev, a.nu1, a.nu2, a.gamma, u_zero_, final_,
                 slot);
  const SampleState sst = slot_fields(pl.state + s);
  if (!slot_runs(sst, slot)) return;
  const int lt = lg.l;
  // on the finest level (lt = 0) the first and last cycle of the sample's iteration
  // follow from its state in a cycle slot; on coarser levels from the enclosing cycle
  const int u_zero = lt == 0 ? slot_first(sst, slot, u_zero_) : u_zero_;
  const int fin = lt == 0 && slot_last(sst, slot, final_);
  if (pl.tcells && threadIdx.x == 0) atomicAdd(pl.tcells, 1ull);  // timed: sample launches
  const int m = a.n >> lt;
  const int nlev = a.nlev - lt;
  const int M2 = m * m;
  double* red = (double*)smem;
  R* rbase = (R*)(red + NT / 64 + 1);
  const LdsHier<R> lev = lds_hier(rbase, m);
  if constexpr (RMG_TOP_BLK && sizeof(R) == 4 && NT == 512) {
    if (m == kTopBlkM && nlev >= 2) {
      coarse_v_top_blk<R, NT>(a, pl, lg, s, lev, nlev, u_zero != 0, fin != 0);
      return;
    }
  }
  lds_zero_padding<R, NT>(rbase, m, nlev);
  // the top level is loaded before the first barrier: its global loads overlap the
  // start-up of the workgroup's waves
  const LdsLevel<R> T = lev[0];
  using V = typename Vec16<R>::T;
  constexpr int E = 16 / sizeof(R);  // elements per vector; M2 is a multiple of E
  const V* F = (const V*)((const R*)lg.f + s * M2);
  const V* CW = (const V*)((const R*)lg.cw + s * M2);
  const V* CS = (const V*)((const R*)lg.cs + s * M2);
  const V* CDT = (const V*)((const R*)lg.cdt + s * M2);
  const R* CT = (const R*)lg.ctop + s * m;
  R* U = (R*)lg.uout + s * M2;
  const int nv = M2 / E;
  constexpr int VB = 4;  // vectors per array and lane whose loads are in flight together
  for (int v0 = threadIdx.x; v0 < nv; v0 += VB * NT) {
    V f[VB], cw[VB], cs[VB], cdt[VB], u[VB];
#pragma unroll
    for (int q = 0; q < VB; ++q) {
      const int v = v0 + q * NT;
      if (v < nv) {
        f[q] = F[v];
        cw[q] = CW[v];
        cs[q] = CS[v];
        cdt[q] = CDT[v];
        if (!u_zero) u[q] = ((const V*)U)[v];
      }
    }
#pragma unroll
    for (int q = 0; q < VB; ++q) {
      const int v = v0 + q * NT;
      if (v >= nv) continue;
      const R* fe = (const R*)&f[q];
      const R* cwe = (const R*)&cw[q];
      const R* cse = (const R*)&cs[q];
      const R* cde = (const R*)&cdt[q];
      const R* ue = (const R*)&u[q];
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int c = v * E + k;
        T.f[c] = fe[k];
        T.cw[c] = cwe[k];
        T.cs[c] = cse[k];
        T.cdt[c] = cde[k];
        T.u[c] = u_zero ? (R)0 : ue[k];
      }
    }
  }
  for (int i = threadIdx.x; i < m; i += NT) T.cs[M2 + i] = CT[i];
  __syncthreads();
  lds_cycle_coarse<R, NT>(lev, nlev, a.nu1, a.nu2, a.gamma, u_zero != 0, true);
  if (!fin) {
    for (int v = threadIdx.x; v < nv; v += NT) {
      V o;
      R* oe = (R*)&o;
#pragma unroll
      for (int k = 0; k < E; ++k) oe[k] = T.u[v * E + k];
      ((V*)U)[v] = o;
    }
    return;
  }
  double* p = a.p + s * M2;
  double mx = 0.0, bad = 0.0;
  for (int c = threadIdx.x; c < M2; c += NT) {
    const double d = (double)T.u[c];
    p[c] += d;
    mx = fmax(mx, fabs(d));
    if (!isfinite(d)) bad = 1.0;
  }
  mx = block_max<NT>(mx, red);
  bad = block_max<NT>(bad, red);
  if (threadIdx.x == 0) {
    pl.dpmax[s] = (unsigned long long)__double_as_longlong(mx);
    if (bad > 0.0) pl.state[s].nanflag = 1;
  }
}

// One Picard iteration of an M x M sample whose finest level is the coarse kernel's
// top level, in one workgroup: the stopping test of the previous iteration (as in
// k_fine), the fine coefficients formed as k_fine forms them (closure once per cell;
// p and K of the cells and of the zero ring around the grid staged in LDS where the
// top level will lie: each thread keeps its cells' coefficients in registers until
// the staging is dead, then writes them into the top level of the LDS hierarchy, so
// the kernel needs no more LDS than k_coarse_v), the cycles of k_coarse_v, and its
// Picard update.  One launch per iteration instead of two, and the top level's
// coefficients never go through global memory; every value is computed by the same
// operations in the same order as on the two-kernel path.
#ifndef RMG_FUSED_FINE_COARSE
#define RMG_FUSED_FINE_COARSE 1
#endif
constexpr int kFusedM = 64;  // the float coarse kernel's top level

template <class R, int NT, int M>
__global__ __launch_bounds__(NT) void k_fine_coarse(SolveArgs a, StreamPlan pl) {
  static_assert((M * M) % NT == 0, "every thread forms the same number of cells");
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t s = blockIdx.x;
  const rmg_problem P = class_problem(a.cp, s);
  SampleState st = pl.state_prev[s];
  // every launch is a whole Picard iteration of its sample (all its cycles)
  st.jpass = st.cpp;
  const bool restart = pass_control(st, a, pl, P, s, st.cpp, threadIdx.x == 0, pl.dpmax_prev[s]);
  if (!st.active) return;
  if (pl.tcells && threadIdx.x == 0) atomicAdd(pl.tcells, 1ull);  // timed: sample launches
  constexpr int M2 = M * M, TL = M + 2, LG = M == 64 ? 6 : M == 32 ? 5 : 4, Q = M2 / NT;
  static_assert((1 << LG) == M, "unsupported grid size");
  const int nlev = a.nlev;
  const int new_step = st.new_step;
  double* red = (double*)smem;
  R* rbase = (R*)(red + NT / 64 + 1);
  const LdsHier<R> lev = lds_hier(rbase, M);
  const LdsLevel<R> T = lev[0];
  static_assert(8 * (NT / 64 + 1) + 2 * sizeof(double) * TL * TL <= 8 * (NT / 64 + 1) + lds_level_elems(M) * sizeof(R),
                "the staging fits in the top level's place");
  double* sp = (double*)rbase;  // 8-byte aligned: rbase follows NT / 64 + 1 doubles
  double* sK = sp + TL * TL;
  double* pg = a.p + s * M2;
  double* thold = a.theta_old + s * M2;
  double cth[Q], cC[Q], pth[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = (int)threadIdx.x + q * NT;
    const int lj = c >> LG, li = c & (M - 1);
    pth[q] = 0.0;
    if (!new_step) pth[q] = thold[c];
    double pv;
    if (restart) {
      pv = start_head(a, P, s, c, lj, M);
      pg[c] = pv;
    } else {
      pv = pg[c];
    }
    const CellFields cf = load_fields(a.fields, a.F, (int64_t)M2, s, c);
    const Closure cl = closure(P, pv, cf.Ks, cf.alpha, cf.nvg);
    const int le = (lj + 1) * TL + li + 1;
    sp[le] = pv;
    sK[le] = cl.K;
    cth[q] = cl.theta;
    cC[q] = cl.C;
  }
  for (int r = threadIdx.x; r < 4 * TL - 4; r += NT) {
    int li, lj;  // bottom row, top row, then the left and right columns without corners
    if (r < TL) {
      li = r;
      lj = 0;
    } else if (r < 2 * TL) {
      li = r - TL;
      lj = TL - 1;
    } else {
      const int q = r - 2 * TL;
      li = (q & 1) ? TL - 1 : 0;
      lj = 1 + (q >> 1);
    }
    sp[lj * TL + li] = 0.0;
    sK[lj * TL + li] = 0.0;
  }
  __syncthreads();
  double* hist = nullptr;  // history slot of the step that starts here, if recorded
  if (new_step && a.p_hist) {
    const int k = st.step;
    if (k % a.hist_every == 0) hist = a.p_hist + (s * a.hist_slots + k / a.hist_every) * M2;
  }
  R rf[Q], rcw[Q], rcs[Q], rcdt[Q], rct = (R)0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = (int)threadIdx.x + q * NT;
    const int lj = c >> LG, li = c & (M - 1);
    const int le = (lj + 1) * TL + li + 1;
    double th_old;
    if (new_step) {
      th_old = cth[q];
      thold[c] = cth[q];
      if (hist) hist[c] = sp[le];
    } else {
      th_old = pth[q];
    }
    const FineCell fc = fine_cell(li, lj, M, sp[le], sp[le - 1], sp[le + 1], sp[le - TL], sp[le + TL], sK[le],
                                  sK[le - 1], sK[le + 1], sK[le - TL], sK[le + TL], cth[q], th_old, cC[q], P.dt,
                                  P.h_bottom, P.h_top);
    rf[q] = (R)fc.f;
    rcw[q] = (R)fc.cw;
    rcs[q] = (R)fc.cs;
    rcdt[q] = (R)fc.cdt;
    if (q == Q - 1) rct = (R)fc.ctop;  // the top row's cells are every thread's last ones
  }
  static_assert(M <= NT, "the top row lies in the last NT cells, every thread's last ones");
  __syncthreads();  // the staging is dead: the hierarchy takes its place
  lds_zero_padding<R, NT>(rbase, M, nlev);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = (int)threadIdx.x + q * NT;
    T.f[c] = rf[q];
    T.cw[c] = rcw[q];
    T.cs[c] = rcs[q];
    T.cdt[c] = rcdt[q];
    T.u[c] = (R)0;
    if (q == Q - 1 && (c >> LG) == M - 1) T.cs[M2 + (c & (M - 1))] = rct;
  }
  __syncthreads();
  for (int cyc = 0; cyc < st.cpp; ++cyc) lds_cycle_coarse<R, NT>(lev, nlev, a.nu1, a.nu2, a.gamma, cyc == 0, cyc == 0);
  double* p = a.p + s * M2;
  double mx = 0.0, bad = 0.0;
  for (int c = threadIdx.x; c < M2; c += NT) {
    const double d = (double)T.u[c];
    p[c] += d;
    mx = fmax(mx, fabs(d));
    if (!isfinite(d)) bad = 1.0;
  }
  mx = block_max<NT>(mx, red);
  bad = block_max<NT>(bad, red);
  if (threadIdx.x == 0) {
    pl.dpmax[s] = (unsigned long long)__double_as_longlong(mx);
    if (bad > 0.0) pl.state[s].nanflag = 1;
  }
}

// Residual-controlled cycling on the streaming path (Section 4.2: cycle until
// max_c |f - A dp| < eps_mg): after each cycle, the correction equation's residual on
// the finest level in the smoother precision (the per-cell arithmetic of
// residual_value / st5, as the whole-sample kernel's check), reduced per sample.
template <class R>
__global__ __launch_bounds__(kBlock) void k_mg_residual(SolveArgs a, StreamPlan pl) {
  __shared__ double red[kBlock / 64];
  const int64_t s = blockIdx.y;
  const SampleState st = pl.state[s];
  if (!slot_runs(st, 0)) return;
  const int m = a.n, lg = a.lg;
  const int64_t M2 = (int64_t)m * m;
  const R* F = (const R*)pl.lv.f[0] + s * M2;
  const R* CW = (const R*)pl.lv.cw[0] + s * M2;
  const R* CS = (const R*)pl.lv.cs[0] + s * M2;
  const R* CDT = (const R*)pl.lv.cdt[0] + s * M2;
  const R* CT = (const R*)pl.lv.ctop[0] + s * m;
  const R* U = (const R*)(pl.ltop == 0 ? pl.lv.u[0] : pl.lv.ub[0]) + s * M2;
  double mx = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x; c < M2; c += (int64_t)gridDim.x * kBlock) {
    const int j = (int)(c >> lg), i = (int)(c - ((int64_t)j << lg));
    const R z = (R)0;
    const St5<R> t = st5<R>(CDT[c], CW[c], i < m - 1 ? CW[c + 1] : z, CS[c], j < m - 1 ? CS[c + m] : CT[i],
                            i > 0 ? U[c - 1] : z, i < m - 1 ? U[c + 1] : z, j > 0 ? U[c - m] : z,
                            j < m - 1 ? U[c + m] : z);
    mx = fmax(mx, fabs((double)residual_value<R>(F[c], U[c], t)));
  }
  mx = block_max<kBlock>(mx, red);
  if (threadIdx.x == 0) atomic_max_nonneg(pl.mgres + s, mx);
}

// The correction of a sample whose residual met eps_mg (or that reached the cycle cap)
// is applied: p += dp, ||dp||_inf and the non-finite flag as the finest up leg does, and
// the state records that the iteration's cycling is over.
template <class R>
__global__ __launch_bounds__(kBlock) void k_mg_apply(SolveArgs a, StreamPlan pl) {
  __shared__ double red[kBlock / 64];
  const int64_t s = blockIdx.y;
  const SampleState st = pl.state[s];
  if (!slot_runs(st, 0)) return;
  const double r = __longlong_as_double((long long)pl.mgres[s]);
  if (!(r < a.eps_mg) && st.cyc0 + 1 < kMaxMgCycles) return;
  const int64_t M2 = (int64_t)a.n * a.n;
  const R* U = (const R*)(pl.ltop == 0 ? pl.lv.u[0] : pl.lv.ub[0]) + s * M2;
  double* p = a.p + s * M2;
  double mx = 0.0, bad = 0.0;
  for (int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x; c < M2; c += (int64_t)gridDim.x * kBlock) {
    const double d = (double)U[c];
    p[c] += d;
    mx = fmax(mx, fabs(d));
    if (!isfinite(d)) bad = 1.0;
  }
  mx = block_max<kBlock>(mx, red);
  bad = block_max<kBlock>(bad, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(pl.dpmax + s, mx);
    if (bad > 0.0) atomicOr(&pl.state[s].nanflag, 1);
    if (blockIdx.x == 0) pl.state[s].mgdone = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_stream_finish(SolveArgs a, StreamPlan pl) {
  __shared__ double red[kBlock];
  const int64_t s = blockIdx.x;
  const rmg_problem P = class_problem(a.cp, s);
  const int64_t N = (int64_t)a.n * a.n;
  const double q = mean_saturation<kBlock>(P, a.fields, a.F, N, s, a.p + s * N, red);
  if (a.p_hist && pl.state[s].status == RMG_SAMPLE_OK && P.n_steps % a.hist_every == 0) {
    double* hist = a.p_hist + (s * a.hist_slots + P.n_steps / a.hist_every) * N;
    for (int64_t c = threadIdx.x; c < N; c += kBlock) hist[c] = a.p[s * N + c];
  }
  if (threadIdx.x == 0) {
    const SampleState st = pl.state[s];
    a.qoi[s] = st.status == RMG_SAMPLE_OK ? q : __longlong_as_double(0x7ff8000000000000ll);
    a.status[s] = st.status;
    if (a.stats) {
      rmg_sample_stats o;
      o.picard_its = st.tot_its;
      o.mg_cycles = st.cycles;
      o.steps_done = st.step;
      o.status = st.status;
      o.final_dp_inf = st.final_dp;
      o.attempts = st.attempt + 1;
      o.reserved = 0;
      a.stats[s] = o;
    }
  }
}

size_t level_bytes(int m, int64_t S, bool fp64) {
  const size_t es = fp64 ? 8 : 4;
  return es * (size_t)S * (6 * (size_t)m * m + (size_t)m);
}

// Input validation: a sample whose fields hold a non-finite value is marked
// RMG_SAMPLE_NONFINITE and never iterated (both parities of its state).
__global__ __launch_bounds__(kBlock) void k_check_fields(SolveArgs a, StreamPlan pl) {
  __shared__ double red[kBlock / 64];
  const int64_t s = blockIdx.x;
  const int64_t FN = (int64_t)a.F << (2 * a.lg);
  const double* fld = a.fields + s * FN;
  double bad = 0.0;
  for (int64_t e = threadIdx.x; e < FN; e += kBlock)
    if (!isfinite(fld[e])) bad = 1.0;
  bad = block_max<kBlock>(bad, red);
  if (threadIdx.x == 0 && bad > 0.0) {
    pl.state[s].active = pl.state_prev[s].active = 0;
    pl.state[s].status = pl.state_prev[s].status = RMG_SAMPLE_NONFINITE;
  }
}

hipError_t launch_stream_init(const SolveArgs& a, const StreamPlan& pl, hipStream_t st) {
  const int64_t tot = a.S * (int64_t)a.n * a.n;
  int64_t blocks = (tot + kBlock - 1) / kBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_stream_init, dim3((unsigned)blocks), dim3(kBlock), 0, st, a, pl);
  hipLaunchKernelGGL(k_check_fields, dim3((unsigned)a.S), dim3(kBlock), 0, st, a, pl);
  return hipGetLastError();
}

static size_t coarse_lds(int m, int nc, bool fp64) {
  size_t relems = 0;
  for (int mm = m; mm >= nc; mm >>= 1) relems += lds_level_elems(mm);
  return 8 * (kCoarseThreads / 64 + 1) + relems * (fp64 ? 8 : 4);
}

// Down and up kernels by tile edge and blocks per thread (nu <= 4: at most 3 blocks).
// A timed launch (ev != null) goes through hipExtLaunchKernelGGL with the event pair
// recorded by the dispatch itself: the events then bracket the kernel's execution, not
// the queue time before it.
template <class K, class... Args>
static void launch_k(K kern, dim3 grid, dim3 blk, size_t lds, hipStream_t st, hipEvent_t* ev, Args... args) {
  if (ev)
    hipExtLaunchKernelGGL(kern, grid, blk, (uint32_t)lds, st, ev[0], ev[1], 0u, args...);
  else
    hipLaunchKernelGGL(kern, grid, blk, lds, st, args...);
}

// The level's arrays of a down or up launch on level l (ts x ts tiles, a halo of hb
// blocks), with the iterate read and written and the neighbouring level's array.
static LegArgs leg_args(const SolveArgs& a, const StreamPlan& pl, int l, int ts, int hb, const void* uin,
                        void* uout, void* fc, const void* uc) {
  LegArgs g;
  g.f = pl.lv.f[l];
  g.cw = pl.lv.cw[l];
  g.cs = pl.lv.cs[l];
  g.cdt = pl.lv.cdt[l];
  g.ctop = pl.lv.ctop[l];
  g.uin = uin;
  g.uout = uout;
  g.fc = fc;
  g.uc = uc;
  g.l = l;
  g.m = a.n >> l;
  g.hb = hb;
  int lgt = 0;
  while ((ts << lgt) < g.m) ++lgt;
  g.lgntx = lgt;
  g.mg = blk_magic_host(ts, hb);
  return g;
}

template <class R>
static void launch_down(int ts, dim3 grid, hipStream_t st, hipEvent_t* ev, const SolveArgs& a,
                        const StreamPlan& pl, int l, int u_zero, int slot) {
  const int hb = a.nu1 + 1, nb = blk_nb(ts, hb);
  const size_t lds = blk_lds_bytes<R>(ts, hb);
  const dim3 b(kBlock);
  const LegArgs lg = leg_args(a, pl, l, ts, hb, pl.lv.ub[l], pl.lv.u[l], pl.lv.f[l + 1], nullptr);
  if (ts == 16) {
    if (nb <= 1)
      launch_k(k_down<R, 16, 1>, grid, b, lds, st, ev, a, pl, lg, u_zero, slot);
    else
      launch_k(k_down<R, 16, 2>, grid, b, lds, st, ev, a, pl, lg, u_zero, slot);
  } else {
    if (nb <= 2)
      launch_k(k_down<R, 32, 2>, grid, b, lds, st, ev, a, pl, lg, u_zero, slot);
    else
      launch_k(k_down<R, 32, 3>, grid, b, lds, st, ev, a, pl, lg, u_zero, slot);
  }
}

template <class R>
static void launch_up(int ts, dim3 grid, hipStream_t st, const SolveArgs& a, const StreamPlan& pl, int l,
                      int final_, int slot) {
  const int hb = a.nu2, nb = blk_nb(ts, hb);
  const size_t lds = blk_lds_bytes<R>(ts, hb);
  const LegArgs lg = leg_args(a, pl, l, ts, hb, pl.lv.u[l], pl.lv.ub[l], nullptr,
                              l + 1 == pl.ltop ? pl.lv.u[l + 1] : pl.lv.ub[l + 1]);
  if (ts == 16) {
    hipLaunchKernelGGL((k_up<R, 16, 1>), grid, dim3(kBlock), lds, st, a, pl, lg, final_, slot);
  } else {
    if (nb <= 1)
      hipLaunchKernelGGL((k_up<R, 32, 1>), grid, dim3(kBlock), lds, st, a, pl, lg, final_, slot);
    else if (nb == 2)
      hipLaunchKernelGGL((k_up<R, 32, 2>), grid, dim3(kBlock), lds, st, a, pl, lg, final_, slot);
    else
      hipLaunchKernelGGL((k_up<R, 32, 3>), grid, dim3(kBlock), lds, st, a, pl, lg, final_, slot);
  }
}
static_assert(blk_nb(16, 5) <= 2 && blk_nb(16, 4) <= 1 && blk_nb(32, 5) <= 3 && blk_nb(32, 4) <= 3,
              "blocks per thread of the instantiated down/up kernels (nu <= 4)");

// Cycles from the finest level: `ncyc` cycles with uniform flags (slot = kUniform: cycle
// k starts from zero iff k = 0 and applies the Picard update iff k = ncyc - 1), or one
// cycle in cycle slot `slot` (flags from each sample's state).
// Parts of a cycle from the finest level that stream_cycles launches.
enum CyclePart { kCycleFull = 0, kCycleDown0 = 1, kCycleBelow0 = 2 };

template <class R>
static hipError_t stream_cycles(const SolveArgs& a, const StreamPlan& pl, hipStream_t st, int ncyc, int slot,
                                CyclePart part = kCycleFull) {
  const bool fp64 = sizeof(R) == 8;
  const int n = a.n;
  const int nc = n >> (a.nlev - 1);
  const size_t lcv = coarse_lds(n >> pl.ltop, nc, fp64);
  hipError_t err = hipSuccess;
  // One cycle from level l (its iterate zero on entry if `zero`): the down leg, gamma
  // coarse cycles (the coarse kernel below ltop), the up leg; `last`: the final cycle of
  // the Picard iteration, whose finest up leg applies the Picard update.
  auto cycle = [&](auto&& self, int l, bool zero, bool last) -> void {
    if (err != hipSuccess) return;
    KernelTimer* tm = pl.timer;
    if (l == pl.ltop) {
      const bool timed = tm && (tm->which & RMG_TIME_COARSE) && tm->ring[1].room();
      hipEvent_t* ev = timed ? tm->ring[1].next() : nullptr;
      StreamPlan plx = pl;
      plx.tcells = timed ? tm->d_cells + 2 : nullptr;
      const LegArgs lg = leg_args(a, pl, l, n >> l, 0, pl.lv.u[l], pl.lv.u[l], nullptr, nullptr);
      launch_k(k_coarse_v<R, kCoarseThreads>, dim3((unsigned)a.S), dim3(kCoarseThreads), lcv, st, ev, a, plx, lg,
               zero ? 1 : 0, last ? 1 : 0, slot);
      return;
    }
    const int m = n >> l, ts = pl.ts[l];
    const unsigned tiles = (unsigned)((m / ts) * (m / ts));
    if (!(l == 0 && part == kCycleBelow0)) {
      const bool timed = tm && (tm->which & RMG_TIME_SMOOTHER_DOWN) && tm->ring[0].room();
      hipEvent_t* ev = timed ? tm->ring[0].next() : nullptr;
      StreamPlan plx = pl;
      plx.tcells = timed ? tm->d_cells : nullptr;
      launch_down<R>(ts, dim3(tiles, (unsigned)a.S), st, ev, a, plx, l, zero ? 1 : 0, slot);
    }
    if (l == 0 && part == kCycleDown0) return;
    for (int k = 0; k < a.gamma; ++k) self(self, l + 1, k == 0, last);
    if (!(l == 0 && part == kCycleBelow0)) launch_up<R>(ts, dim3(tiles, (unsigned)a.S), st, a, pl, l, (l == 0 && last) ? 1 : 0, slot);
  };
  if (slot >= 0)
    cycle(cycle, 0, false, false);
  else
    for (int cyc = 0; cyc < ncyc; ++cyc) cycle(cycle, 0, cyc == 0, cyc == ncyc - 1);
  return err;
}

#ifndef RMG_FUSE_UP_DOWN
#define RMG_FUSE_UP_DOWN 1
#endif
template <class R>
static void launch_up_down(int ts, dim3 grid, hipStream_t st, const SolveArgs& a, const StreamPlan& pl, int slot) {
  const int hb = a.nu1 + a.nu2 + 1, nb = blk_nb(ts, hb);
  const size_t lds = blk_lds_bytes<R>(ts, hb);
  const LegArgs lg = leg_args(a, pl, 0, ts, hb, pl.lv.u[0], pl.lv.ub[0], pl.lv.f[1],
                              1 == pl.ltop ? pl.lv.u[1] : pl.lv.ub[1]);
  if (ts == 16) {
    if (nb <= 2)
      hipLaunchKernelGGL((k_up_down<R, 16, 2>), grid, dim3(kBlock), lds, st, a, pl, lg, slot);
    else
      hipLaunchKernelGGL((k_up_down<R, 16, 3>), grid, dim3(kBlock), lds, st, a, pl, lg, slot);
  } else {
    if (nb <= 3)
      hipLaunchKernelGGL((k_up_down<R, 32, 3>), grid, dim3(kBlock), lds, st, a, pl, lg, slot);
    else
      hipLaunchKernelGGL((k_up_down<R, 32, 4>), grid, dim3(kBlock), lds, st, a, pl, lg, slot);
  }
}
static_assert(blk_nb(16, 5) <= 2 && blk_nb(16, 9) <= 3 && blk_nb(32, 5) <= 3 && blk_nb(32, 7) <= 4,
              "blocks per thread of the instantiated fused kernels (nu1 + nu2 <= 6 with 32 x 32 tiles)");
// Whether the J cycle slots of a pass run with the finest level's up and down legs
// fused between consecutive slots: several slots, a streaming finest level, fixed
// cycle counts (residual-controlled cycling checks between cycles) and a halo that
// the instantiated kernels cover.
static bool fuse_up_down(const SolveArgs& a, const StreamPlan& pl, int J) {
  const int hb = a.nu1 + a.nu2 + 1;
  return RMG_FUSE_UP_DOWN && J >= 2 && a.cpp > 0 && pl.ltop >= 1 &&
         blk_nb(pl.ts[0], hb) <= (pl.ts[0] == 16 ? 3 : 4);
}

// LDS of k_fine_coarse: that of k_coarse_v (the p / K staging lies in the top level's place).
static size_t fine_coarse_lds(int m, int nc) { return coarse_lds(m, nc, false); }

template <class R>
static bool fine_coarse_fits(const SolveArgs& a, const StreamPlan& pl) {
  return RMG_FUSED_FINE_COARSE && sizeof(R) == 4 && pl.ltop == 0 && a.n == kFusedM && a.nlev >= 2;
}
// Measured: with the class alone on the GPU the fused launch shortens the 64 x 64
// class by 8 %; beside the larger streaming classes of a multilevel call it makes
// the call 2 % slower (its one workgroup per sample holds a compute unit through the
// coefficient assembly that k_fine spreads over four), so it is taken only when the
// class is its call's only streaming class.
template <class R>
static bool fused_fine_coarse(const SolveArgs& a, const StreamPlan& pl) {
  return a.fuse_top && a.cpp > 0 && fine_coarse_fits<R>(a, pl);
}

template <class R>
static hipError_t stream_iteration(const SolveArgs& a, const StreamPlan& pl, hipStream_t st, int J) {
  const dim3 blk(kBlock);
  const int n = a.n;
  KernelTimer* tm = pl.timer;
  if constexpr (sizeof(R) == 4) {
    if (fused_fine_coarse<R>(a, pl)) {
      const bool timed = tm && (tm->which & RMG_TIME_COARSE) && tm->ring[1].room();
      StreamPlan plx = pl;
      plx.tcells = timed ? tm->d_cells + 2 : nullptr;
      launch_k(k_fine_coarse<R, kCoarseThreads, kFusedM>, dim3((unsigned)a.S), dim3(kCoarseThreads),
               fine_coarse_lds(n, n >> (a.nlev - 1)), st, timed ? tm->ring[1].next() : nullptr, a, plx);
      return hipGetLastError();
    }
  }
  {
    const int T = n < kTile ? n : kTile;
    const unsigned tiles = (unsigned)((n / T) * (n / T));
    const bool timed = tm && (tm->which & RMG_TIME_FINE) && tm->ring[2].room();
    StreamPlan plx = pl;
    plx.tcells = timed ? tm->d_cells + 4 : nullptr;
    launch_k(k_fine<R>, dim3(tiles, (unsigned)a.S), blk, 0, st, timed ? tm->ring[2].next() : nullptr, a, plx, J);
  }
  if (fuse_up_down(a, pl, J)) {
    // slot j's finest up leg and slot j + 1's down leg in one launch; the fused kernel of
    // slot j reads u and writes ub of the plan of parity j, so the plans alternate
    StreamPlan sw = pl;
    std::swap(sw.lv.u[0], sw.lv.ub[0]);
    const unsigned tiles = (unsigned)((n / pl.ts[0]) * (n / pl.ts[0]));
    hipError_t err = stream_cycles<R>(a, pl, st, 1, 0, kCycleDown0);
    for (int j = 0; j < J && err == hipSuccess; ++j) {
      err = stream_cycles<R>(a, pl, st, 1, j, kCycleBelow0);
      const StreamPlan& pj = (j & 1) ? sw : pl;
      if (j + 1 < J)
        launch_up_down<R>(pl.ts[0], dim3(tiles, (unsigned)a.S), st, a, pj, j);
      else
        launch_up<R>(pl.ts[0], dim3(tiles, (unsigned)a.S), st, a, pj, 0, 0, j);
    }
    if (err != hipSuccess) return err;
  } else {
    for (int j = 0; j < J; ++j) {
      const hipError_t err = stream_cycles<R>(a, pl, st, 1, j);
      if (err != hipSuccess) return err;
    }
  }
  if (a.cpp == 0) {  // residual-controlled cycling: one cycle per pass, then the check
    const int64_t M2 = (int64_t)n * n;
    const unsigned g = (unsigned)std::min<int64_t>((M2 + kBlock - 1) / kBlock, 256);
    hipLaunchKernelGGL(k_mg_residual<R>, dim3(g, (unsigned)a.S), blk, 0, st, a, pl);
    hipLaunchKernelGGL(k_mg_apply<R>, dim3(g, (unsigned)a.S), blk, 0, st, a, pl);
  }
  return hipGetLastError();
}

template <class R>
static hipError_t set_stream_lds(const SolveArgs& a, const StreamPlan& pl) {
  const bool fp64 = sizeof(R) == 8;
  const int nc = a.n >> (a.nlev - 1);
  // (the down and up kernels need at most 23 KiB of LDS, below the default limit)
  hipError_t e = raise_dyn_lds((const void*)k_coarse_v<R, kCoarseThreads>, coarse_lds(a.n >> pl.ltop, nc, fp64));
  if constexpr (sizeof(R) == 4) {
    if (e == hipSuccess && fine_coarse_fits<R>(a, pl))
      e = raise_dyn_lds((const void*)k_fine_coarse<R, kCoarseThreads, kFusedM>, fine_coarse_lds(a.n, nc));
  }
  return e;
}

hipError_t prepare_stream(const SolveArgs& a, const StreamPlan& pl) {
  return pl.fp64 ? set_stream_lds<double>(a, pl) : set_stream_lds<float>(a, pl);
}

hipError_t launch_stream_iteration(const SolveArgs& a, const StreamPlan& pl, hipStream_t st, int J) {
  return pl.fp64 ? stream_iteration<double>(a, pl, st, J) : stream_iteration<float>(a, pl, st, J);
}

hipError_t launch_stream_cycles(const SolveArgs& a, const StreamPlan& pl, hipStream_t st) {
  const hipError_t e = pl.fp64 ? stream_cycles<double>(a, pl, st, a.cpp, kUniform)
                               : stream_cycles<float>(a, pl, st, a.cpp, kUniform);
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_stream_finish(const SolveArgs& a, const StreamPlan& pl, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_finish, dim3((unsigned)a.S), dim3(kBlock), 0, st, a, pl);
  return hipGetLastError();
}

// ------------------------------------------------- fixed scratch (no allocation)
// Workspace of picard_mg_solve_noalloc: a file-scope device array, one per GPU, held
// until the process ends.  Host code must not pass the array's name to a kernel (on
// the host it is only a stand-in symbol): it takes the device address from
// scratch_address() once per device, with that device current, and uses that.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** ptr) {
  *ptr = nullptr;
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace rmg
