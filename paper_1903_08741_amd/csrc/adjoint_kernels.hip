// Discrete adjoint of the backward-Euler / modified-Picard solve on the
// level-streaming path (gfx950).
//
// Step n of the forward model solves R^n(p^n, p^{n-1}) = 0 with R the outer
// Picard residual of eq. Mixed_based_3 (Section 4.1), harmonic-mean faces and
// mirror-ghost Dirichlet faces (Section 4.2).  For Q = sum_n dt F(p^n), F the
// downward flux through the bottom Dirichlet face, the multipliers lambda_n of
// the steps satisfy J_n^T lambda_n = dt dF/dp^n - diag(C(p^n)/dt) lambda_{n+1}
// (lambda_{N+1} = 0), J_n = dR/dp at p^n.  With mu = -lambda and J = -A + D,
// A the symmetric modified-Picard operator (the one the forward multigrid
// solves) and D the terms of dK/dp, this reads
//     A mu_n - K' * s(mu_n) = b_n,   b_n = dt dF/dp^n + (C(p^n)/dt) mu_{n+1},
// with, per cell c and over its faces f (neighbour nb, absent on a Dirichlet face),
//     s_c(mu) = sum_f w_{f,c} t_{f,c} (mu_c - mu_nb),
// t_{f,c} the face's inflow per unit conductivity into c and w_{f,c} = dK_f/dK_c
// (2 K_nb^2 / (K_c + K_nb)^2 for the harmonic mean, 1 on a Dirichlet face).  It is
// solved by the fixed-point iteration mu <- mu + MG_A(b + K' * s(mu) - A mu),
// which converges at the rate of the forward Picard iteration (its iteration
// matrix is the transpose of Picard's); each MG_A is the forward's own multigrid
// cycle on the coefficients of A at p^n.  The gradient accumulates
//     dQ/dlog Ks_c = sum_n [dt dF/dlog Ks_c(p^n) + K_c(p^n) s_c(mu_n)].
#include <math.h>

#include "rmg_device.hpp"
#include "rmg_internal.hpp"
#include "rmg_smoother.hpp"
#include "rmg_tiles.hpp"

namespace rmg {

// dK/dp of the closure at p (Gardner a K in the unsaturated range; the linear
// test law has K independent of p).  The van Genuchten closure is not differentiated here.
__device__ __forceinline__ double dK_dp(const rmg_problem& P, double p, double K) {
  return (P.model == RMG_GARDNER && p < 0.0) ? P.gardner_a * K : 0.0;
}

__device__ __forceinline__ double dhm(double Kc, double Knb) {
  const double s = Kc + Knb;
  return s > 0.0 ? 2.0 * (Knb * Knb) / (s * s) : 0.0;
}

// Per-cell adjoint quantities at p^n of one cell: (A mu)_c, s_c(mu) and the five
// coefficients of A (in FP64).
struct AdjCell {
  double Amu, smu, cw, cs, cdt, ctop;
};

__device__ __forceinline__ AdjCell adj_cell(int i, int j, int n, double pc, double pw, double pe, double ps,
                                            double pn, double Kc, double Kw, double Ke, double Ks_, double Kn,
                                            double mc, double mw, double me, double ms, double mn, double C,
                                            double dt, double g_bottom, double g_top) {
  const double inv_h = (double)n;
  const double inv_h2 = inv_h * inv_h;
  AdjCell r;
  r.cdt = C / dt;
  double Amu = r.cdt * mc, smu = 0.0;
  if (i > 0) {
    const double a = hmean(Kw, Kc) * inv_h2;
    Amu += a * (mc - mw);
    smu += dhm(Kc, Kw) * ((pw - pc) * inv_h2) * (mc - mw);
    r.cw = a;
  } else {
    r.cw = 0.0;
  }
  if (i < n - 1) {
    const double a = hmean(Kc, Ke) * inv_h2;
    Amu += a * (mc - me);
    smu += dhm(Kc, Ke) * ((pe - pc) * inv_h2) * (mc - me);
  }
  if (j > 0) {
    const double a = hmean(Ks_, Kc) * inv_h2;
    Amu += a * (mc - ms);
    smu += dhm(Kc, Ks_) * (((ps - pc) * inv_h - 1.0) * inv_h) * (mc - ms);
    r.cs = a;
  } else {
    const double a = 2.0 * Kc * inv_h2;
    Amu += a * mc;
    smu += (((g_bottom - pc) * (2.0 * inv_h) - 1.0) * inv_h) * mc;
    r.cs = a;
  }
  if (j < n - 1) {
    const double a = hmean(Kc, Kn) * inv_h2;
    Amu += a * (mc - mn);
    smu += dhm(Kc, Kn) * (((pn - pc) * inv_h + 1.0) * inv_h) * (mc - mn);
    r.ctop = 0.0;
  } else {
    const double a = 2.0 * Kc * inv_h2;
    Amu += a * mc;
    smu += (((g_top - pc) * (2.0 * inv_h) + 1.0) * inv_h) * mc;
    r.ctop = a;
  }
  r.Amu = Amu;
  r.smu = smu;
  return r;
}

// Load the (T+2)^2 halo tile of p^k, K(p^k) and mu of sample s into LDS.
__device__ __forceinline__ void adj_load_tile(const SolveArgs& a, const rmg_problem& P, int64_t s,
                                              const double* pk, const double* mu, int n, int x0, int y0, int TL,
                                              double* sp, double* sK, double* sm) {
  const int64_t N = (int64_t)n * n;
  for (int k = threadIdx.x; k < TL * TL; k += kBlock) {
    const int lj = k / TL, li = k - lj * TL;
    const int gi = x0 - 1 + li, gj = y0 - 1 + lj;
    double pv = 0.0, Kv = 0.0, mv = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      const int64_t c = (int64_t)gj * n + gi;
      pv = pk[c];
      mv = mu[c];
      const CellFields cf = load_fields(a.fields, a.F, N, s, c);
      Kv = closure(P, pv, cf.Ks, cf.alpha, cf.nvg).K;
    }
    sp[k] = pv;
    sK[k] = Kv;
    sm[k] = mv;
  }
}

// Pending gradient terms: for every sample whose step `state.step + 1` has
// converged (pend), g += dt dF/dlog Ks + K s(mu) at that step.  final_pass: the
// loop of the segment has ended and the samples are no longer active.
__global__ __launch_bounds__(kBlock) void k_adj_grad(SolveArgs a, StreamPlan pl, AdjArgs ad, int final_pass) {
  __shared__ double sp[34 * 34], sK[34 * 34], sm[34 * 34];
  const int64_t s = blockIdx.y;
  const SampleState st = pl.state[s];
  if (!st.pend || st.status != RMG_SAMPLE_OK || (!final_pass && !st.active)) return;
  const rmg_problem P = class_problem(a.cp, s);
  const int n = a.n;
  const int T = n < kTile ? n : kTile, TL = T + 2;
  const int ntx = n / T;
  const int x0 = (blockIdx.x % ntx) * T, y0 = (blockIdx.x / ntx) * T;
  const int64_t N = (int64_t)n * n;
  const int k = st.step + 1;
  const double* pk = ad.hist + (s * ad.slots + (k - ad.base)) * N;
  adj_load_tile(a, P, s, pk, ad.mu + s * N, n, x0, y0, TL, sp, sK, sm);
  __syncthreads();
  const double h = 1.0 / (double)n;
  RMG_TILE_FOR(T, li, lj) {
    const int gi = x0 + li, gj = y0 + lj;
    const int64_t c = (int64_t)gj * n + gi;
    const int le = (lj + 1) * TL + li + 1;
    const double pc = sp[le], Kc = sK[le];
    const AdjCell ac = adj_cell(gi, gj, n, pc, sp[le - 1], sp[le + 1], sp[le - TL], sp[le + TL], Kc, sK[le - 1],
                                sK[le + 1], sK[le - TL], sK[le + TL], sm[le], sm[le - 1], sm[le + 1], sm[le - TL],
                                sm[le + TL], 0.0, P.dt, P.h_bottom, P.h_top);
    double d = Kc * ac.smu;
    if (gj == 0) d += P.dt * (h * Kc * ((pc - P.h_bottom) * (2.0 * (double)n) + 1.0));
    ad.g[s * N + c] += d;
  }
}

// Fine level of one adjoint fixed-point iteration: (at a new step) the right-hand
// side b, the residual b + K' s(mu) - A mu as the multigrid right-hand side, the
// coefficients of A at p^n on every streaming level.
template <class R>
__global__ __launch_bounds__(kBlock) void k_adj_fine(SolveArgs a, StreamPlan pl, AdjArgs ad) {
  __shared__ double sp[34 * 34], sK[34 * 34], sm[34 * 34];
  __shared__ R bufA[3 * 32 * 32 + 32], bufB[3 * 16 * 16 + 16];
  const int64_t s = blockIdx.y;
  if (blockIdx.x == 0 && s == 0 && threadIdx.x == 0) *pl.active_count = 0;
  const SampleState st = pl.state[s];
  if (!st.active) return;
  const rmg_problem P = class_problem(a.cp, s);
  const int n = a.n;
  const int T = n < kTile ? n : kTile, TL = T + 2;
  const int ntx = n / T;
  const int x0 = (blockIdx.x % ntx) * T, y0 = (blockIdx.x / ntx) * T;
  const int64_t N = (int64_t)n * n;
  const double* pk = ad.hist + (s * ad.slots + (st.step - ad.base)) * N;
  const double* mu = ad.mu + s * N;
  double* bb = ad.b + s * N;
  // The tile's own cells (k = threadIdx.x + q kBlock; T = 32 or n, a power of two):
  // p, mu and the closure once per cell, K to LDS for the neighbours and C kept in
  // registers for the cell phase, the stored right-hand side (a step already
  // started) loaded here so that its loads are in flight during this phase; then
  // the halo ring (one cell per thread): p, K and mu only.
  constexpr int Q = (kTile * kTile + kBlock - 1) / kBlock;
  const int lgT = 31 - __clz(T);
  double cC[Q], pb[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = (int)threadIdx.x + q * kBlock;
    cC[q] = pb[q] = 0.0;
    if (k < T * T) {
      const int lj = k >> lgT, li = k & (T - 1);
      const int64_t c = (int64_t)(y0 + lj) * n + x0 + li;
      if (!st.new_step) pb[q] = bb[c];
      const double pv = pk[c];
      const CellFields cf = load_fields(a.fields, a.F, N, s, c);
      const Closure cl = closure(P, pv, cf.Ks, cf.alpha, cf.nvg);
      const int le = (lj + 1) * TL + li + 1;
      sp[le] = pv;
      sK[le] = cl.K;
      sm[le] = mu[c];
      cC[q] = cl.C;
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
    double pv = 0.0, Kv = 0.0, mv = 0.0;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      const int64_t c = (int64_t)gj * n + gi;
      pv = pk[c];
      mv = mu[c];
      const CellFields cf = load_fields(a.fields, a.F, N, s, c);
      Kv = closure(P, pv, cf.Ks, cf.alpha, cf.nvg).K;
    }
    sp[le] = pv;
    sK[le] = Kv;
    sm[le] = mv;
  }
  __syncthreads();
  R* tcw = bufA;
  R* tcdt = bufA + T * T;
  R* tcs = bufA + 2 * T * T;
  R* f0 = (R*)pl.lv.f[0] + s * N;
  R* cw0 = (R*)pl.lv.cw[0] + s * N;
  R* cs0 = (R*)pl.lv.cs[0] + s * N;
  R* cdt0 = (R*)pl.lv.cdt[0] + s * N;
  R* ctop0 = (R*)pl.lv.ctop[0] + s * n;
  const double h = 1.0 / (double)n;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k = (int)threadIdx.x + q * kBlock;
    if (k >= T * T) continue;
    const int lj = k >> lgT, li = k & (T - 1);
    const int e = lj * T + li;
    const int gi = x0 + li, gj = y0 + lj;
    const int64_t c = (int64_t)gj * n + gi;
    const int le = (lj + 1) * TL + li + 1;
    const double pc = sp[le], Kc = sK[le];
    const AdjCell ac = adj_cell(gi, gj, n, pc, sp[le - 1], sp[le + 1], sp[le - TL], sp[le + TL], Kc, sK[le - 1],
                                sK[le + 1], sK[le - TL], sK[le + TL], sm[le], sm[le - 1], sm[le + 1], sm[le - TL],
                                sm[le + TL], cC[q], P.dt, P.h_bottom, P.h_top);
    const double Kp = dK_dp(P, pc, Kc);
    double b;
    if (st.new_step) {
      b = ac.cdt * sm[le];
      if (gj == 0) {
        const double dF = h * (Kp * ((pc - P.h_bottom) * (2.0 * (double)n) + 1.0) + Kc * (2.0 * (double)n));
        b += P.dt * dF;
      }
      bb[c] = b;
    } else {
      b = pb[q];
    }
    const double r = (b + Kp * ac.smu) - ac.Amu;
    const R rcw = (R)ac.cw, rcs = (R)ac.cs, rcdt = (R)ac.cdt;
    f0[c] = (R)r;
    cw0[c] = rcw;
    cs0[c] = rcs;
    cdt0[c] = rcdt;
    tcw[e] = rcw;
    tcs[e] = rcs;
    tcdt[e] = rcdt;
    if (lj == T - 1) {
      const R rct = (R)ac.ctop;
      tcs[T * T + li] = rct;
      if (gj == n - 1) ctop0[gi] = rct;
    }
  }
  tile_coarsen<R>(pl, s, n, T, x0, y0, bufA, bufB);
}

// Per-sample stopping test of the fixed point and step bookkeeping (steps run
// downwards from ad.hi to ad.lo).
__global__ void k_adj_control(SolveArgs a, StreamPlan pl, AdjArgs ad) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  SampleState st = pl.state[s];
  if (!st.active) return;
  const double dm = __longlong_as_double((long long)pl.dpmax[s]);
  pl.dpmax[s] = 0ull;
  st.pend = 0;
  st.it += 1;
  st.tot_its += 1;
  st.cycles += a.cpp;
  st.final_dp = dm;
  if (st.nanflag) {
    st.status = RMG_SAMPLE_NONFINITE;
    st.active = 0;
  } else if (dm < ad.eps) {
    st.pend = 1;
    st.step -= 1;
    st.it = 0;
    st.new_step = 1;
    if (st.step < ad.lo) st.active = 0;
  } else {
    st.new_step = 0;
    if (st.it >= ad.max_its) {
      st.status = RMG_SAMPLE_MAXITER;
      st.active = 0;
    }
  }
  pl.state[s] = st;
  if (st.active) atomicAdd(pl.active_count, 1);
}

__global__ void k_adj_init(SolveArgs a, StreamPlan pl, AdjArgs ad, const int32_t* fwd_status) {
  const int64_t N = (int64_t)a.n * a.n;
  const int64_t tot = a.S * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    ad.mu[e] = 0.0;
    ad.g[e] = 0.0;
  }
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < a.S; s += (int64_t)gridDim.x * blockDim.x) {
    SampleState z;
    z.active = 0;
    z.new_step = 1;
    z.step = 0;
    z.it = 0;
    z.status = fwd_status[s];
    z.tot_its = 0;
    z.cycles = 0;
    z.nanflag = 0;
    z.final_dp = 0.0;
    z.pend = 0;
    z.fresh = 0;
    z.cpp = a.cpp;
    z.cyc0 = 0;
    z.jpass = 0;
    z.attempt = 0;
    pl.state[s] = z;
    pl.dpmax[s] = 0ull;
  }
}

__global__ void k_adj_reset(SolveArgs a, StreamPlan pl, AdjArgs ad) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  SampleState st = pl.state[s];
  st.pend = 0;
  st.active = st.status == RMG_SAMPLE_OK ? 1 : 0;
  st.step = ad.hi;
  st.new_step = 1;
  st.it = 0;
  pl.state[s] = st;
  pl.dpmax[s] = 0ull;
}

// F(p^k) = h sum_i K_i0 ((p_i0 - g_B) / (h/2) + 1) for the steps of a segment; one
// workgroup per (sample, step), fixed-order reduction.
__global__ __launch_bounds__(kBlock) void k_adj_outflux(SolveArgs a, AdjArgs ad) {
  __shared__ double red[kBlock];
  const int64_t s = blockIdx.x;
  const int k = ad.lo + (int)blockIdx.y;
  const rmg_problem P = class_problem(a.cp, s);
  const int n = a.n;
  const int64_t N = (int64_t)n * n;
  const double* pk = ad.hist + (s * ad.slots + (k - ad.base)) * N;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const CellFields cf = load_fields(a.fields, a.F, N, s, i);
    const double K = closure(P, pk[i], cf.Ks, cf.alpha, cf.nvg).K;
    acc += K * ((pk[i] - P.h_bottom) * (2.0 * (double)n) + 1.0);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock >> 1; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) ad.qn[s * ad.n_steps + (k - 1)] = red[0] / (double)n;
}

__global__ void k_adj_finish(SolveArgs a, StreamPlan pl, AdjArgs ad, const int32_t* fwd_status, double* q,
                             int32_t* status, rmg_sample_stats* stats) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  const rmg_problem& P = class_problem(a.cp, s);
  const SampleState st = pl.state[s];
  const int32_t sts = fwd_status[s] != RMG_SAMPLE_OK ? fwd_status[s] : st.status;
  double Q = 0.0;
  for (int k = 0; k < ad.n_steps; ++k) Q += P.dt * ad.qn[s * ad.n_steps + k];
  q[s] = sts == RMG_SAMPLE_OK ? Q : __longlong_as_double(0x7ff8000000000000ll);
  status[s] = sts;
  if (stats) {
    rmg_sample_stats o;
    o.picard_its = st.tot_its;
    o.mg_cycles = st.cycles;
    o.steps_done = P.n_steps - (st.status == RMG_SAMPLE_OK ? 0 : st.step);
    o.status = st.status;
    o.final_dp_inf = st.final_dp;
    o.attempts = 1;
    o.reserved = 0;
    stats[s] = o;
  }
}

// dQ/dxi = B (g * dlogKs/dG): grid (S, ceil(M / 8)); thread t sums cells t, t + 256, ...
// for 8 coefficients, then a fixed-order tree over the threads.
constexpr int kGradJ = 8;
__global__ __launch_bounds__(kBlock) void k_grad_xi(int64_t S, int N, int M, const double* B, const double* g,
                                                    const double* Ks, rmg_marginal marg, const int32_t* status,
                                                    double* grad) {
  __shared__ double red[kGradJ][kBlock];
  const int64_t s = blockIdx.x;
  const int j0 = blockIdx.y * kGradJ;
  double acc[kGradJ];
#pragma unroll
  for (int q = 0; q < kGradJ; ++q) acc[q] = 0.0;
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    const double k = Ks[s * N + c];
    const double w = g[s * N + c] * (marg.scale * ((k - marg.shift) / k));
#pragma unroll
    for (int q = 0; q < kGradJ; ++q)
      if (j0 + q < M) acc[q] += B[(int64_t)(j0 + q) * N + c] * w;
  }
#pragma unroll
  for (int q = 0; q < kGradJ; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = kBlock >> 1; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < kGradJ; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < kGradJ && j0 + (int)threadIdx.x < M)
    grad[s * M + j0 + threadIdx.x] =
        status[s] == RMG_SAMPLE_OK ? red[threadIdx.x][0] : __longlong_as_double(0x7ff8000000000000ll);
}

// ------------------------------------------------------------------ launchers
static unsigned per_sample_blocks(int64_t S) { return (unsigned)((S + kBlock - 1) / kBlock); }

hipError_t launch_adj_init(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, const int32_t* fwd_status,
                           hipStream_t st) {
  const int64_t tot = a.S * (int64_t)a.n * a.n;
  int64_t blocks = (tot + kBlock - 1) / kBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_adj_init, dim3((unsigned)blocks), dim3(kBlock), 0, st, a, pl, ad, fwd_status);
  return hipGetLastError();
}

hipError_t launch_adj_reset(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_reset, dim3(per_sample_blocks(a.S)), dim3(kBlock), 0, st, a, pl, ad);
  return hipGetLastError();
}

static dim3 tile_grid(const SolveArgs& a) {
  const int T = a.n < kTile ? a.n : kTile;
  return dim3((unsigned)((a.n / T) * (a.n / T)), (unsigned)a.S);
}

hipError_t launch_adj_iteration(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_grad, tile_grid(a), dim3(kBlock), 0, st, a, pl, ad, 0);
  if (pl.fp64)
    hipLaunchKernelGGL(k_adj_fine<double>, tile_grid(a), dim3(kBlock), 0, st, a, pl, ad);
  else
    hipLaunchKernelGGL(k_adj_fine<float>, tile_grid(a), dim3(kBlock), 0, st, a, pl, ad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_stream_cycles(a, pl, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_control, dim3(per_sample_blocks(a.S)), dim3(kBlock), 0, st, a, pl, ad);
  return hipGetLastError();
}

hipError_t launch_adj_grad_final(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_grad, tile_grid(a), dim3(kBlock), 0, st, a, pl, ad, 1);
  return hipGetLastError();
}

// Q = sum_k dt F(p^k) of the forward solve alone (the sum of k_adj_finish, in the same
// order), NaN for a sample the forward solve did not converge on.
__global__ void k_outflux_total(SolveArgs a, AdjArgs ad, const int32_t* fwd_status, double* q) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  const rmg_problem& P = class_problem(a.cp, s);
  double Q = 0.0;
  for (int k = 0; k < ad.n_steps; ++k) Q += P.dt * ad.qn[s * ad.n_steps + k];
  q[s] = fwd_status[s] == RMG_SAMPLE_OK ? Q : __longlong_as_double(0x7ff8000000000000ll);
}

hipError_t launch_outflux_total(const SolveArgs& a, const AdjArgs& ad, const int32_t* fwd_status, double* q,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_outflux_total, dim3(per_sample_blocks(a.S)), dim3(kBlock), 0, st, a, ad, fwd_status, q);
  return hipGetLastError();
}

hipError_t launch_adj_outflux(const SolveArgs& a, const AdjArgs& ad, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_outflux, dim3((unsigned)a.S, (unsigned)(ad.hi - ad.lo + 1)), dim3(kBlock), 0, st, a,
                     ad);
  return hipGetLastError();
}

hipError_t launch_adj_finish(const SolveArgs& a, const StreamPlan& pl, const AdjArgs& ad, const int32_t* fwd_status,
                             double* q, int32_t* status, rmg_sample_stats* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_finish, dim3(per_sample_blocks(a.S)), dim3(kBlock), 0, st, a, pl, ad, fwd_status, q,
                     status, stats);
  return hipGetLastError();
}

hipError_t launch_grad_xi(int64_t S, int N, int M, const double* B, const double* g, const double* Ks,
                          rmg_marginal marg, const int32_t* status, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_xi, dim3((unsigned)S, (unsigned)((M + kGradJ - 1) / kGradJ)), dim3(kBlock), 0, st, S, N,
                     M, B, g, Ks, marg, status, grad);
  return hipGetLastError();
}

}  // namespace rmg
