// Karhunen-Loeve field sampling on FP64 matrix cores (gfx950).
//
// Section 3 eq. KLexp truncated at M terms, for a batch of rows r = s*F + f:
//   G[r][c] = sum_k xi[r][k] * B[k][c],   B[k][c] = sqrt(lambda_k) Psi_k(x_c),
// followed by the pointwise marginal of eq. RandK (lognormal, optionally shifted):
//   out[r][c] = shift_f + exp(log_mean_f + scale_f * G[r][c]).
// One wave computes a 16-row x 64-column block with four 16x16 FP64 MFMA
// accumulators (v_mfma_f64_16x16x4f64, K = 4 per instruction); a workgroup of
// four waves covers 64 rows x 64 columns.
#include <hip/hip_runtime.h>
#include <math.h>

#include "rmg_internal.hpp"

namespace rmg {

typedef double v4d __attribute__((ext_vector_type(4)));

struct Marg4 {
  rmg_marginal m[4];
};

__global__ __launch_bounds__(256) void k_kl_fields(int N, int M, int64_t rows, int F,
                                                   const double* __restrict__ B,
                                                   const double* __restrict__ xi, Marg4 mg,
                                                   double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * 64 + wave * 16;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int li = lane & 15, lk = lane >> 4;
  // operand layouts: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k
  const int64_t arow = r0 + li;
  v4d acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < M; k0 += 4) {
    const int k = k0 + lk;
    const double a = (arow < rows && k < M) ? xi[arow * M + k] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t col = c0 + 16 * t + li;
      const double b = (k < M && col < N) ? B[(int64_t)k * N + col] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  // result layout of v_mfma_f64_16x16x4f64: D[i][j] in lane j + 16*(i%4), element i/4
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t col = c0 + 16 * t + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = r0 + 4 * e + lk;
      if (row < rows && col < N) {
        const rmg_marginal& q = mg.m[(int)(row % F)];
        out[row * N + col] = q.shift + exp(q.log_mean + q.scale * acc[t][e]);
      }
    }
  }
}

hipError_t launch_kl_fields(int N, int M, int64_t rows, int F, const double* B, const double* xi,
                            const rmg_marginal* marg, double* out, hipStream_t st) {
  Marg4 mg;
  for (int f = 0; f < 4; ++f) mg.m[f] = f < F ? marg[f] : rmg_marginal{0.0, 0.0, 0.0};
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((rows + 63) / 64));
  hipLaunchKernelGGL(k_kl_fields, grid, dim3(256), 0, st, N, M, rows, F, B, xi, mg, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- level sums
// Compensated sums over the pairs of one level (Section 5.1 eqs. SMC, MC_var need
// sum Y, sum Y^2 and the same for Q_f, Q_c).  Thread t of the workgroup takes pairs
// t, t + 256, ... with Neumaier compensation; the 256 partial sums (value + its
// compensation) are then added in thread order as double-double numbers by thread
// 0.  The order is fixed, so the result does not depend on scheduling.
constexpr int kSumThreads = 256;
struct Neu {
  double s, c;
};
__device__ __forceinline__ void neu_add(Neu& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}
// a += (b.s + b.c) in double-double arithmetic (TwoSum of the leading parts).
__device__ __forceinline__ void dd_acc(Neu& a, const Neu& b) {
  const double s = a.s + b.s;
  const double bb = s - a.s;
  const double e = (a.s - (s - bb)) + (b.s - bb);
  a.s = s;
  a.c += e + b.c;
}

__global__ __launch_bounds__(kSumThreads) void k_level_sums(const double* qf, const double* qc, int64_t n,
                                                            const int32_t* stf, const int32_t* stc,
                                                            const rmg_sample_stats* sf,
                                                            const rmg_sample_stats* sc, rmg_level_sums* out) {
  __shared__ Neu part[6][kSumThreads];
  __shared__ long long cnt[6][kSumThreads];
  Neu acc[6];
  for (int k = 0; k < 6; ++k) acc[k] = Neu{0.0, 0.0};
  long long ok = 0, bad = 0, its = 0, cyc = 0, cyc_c = 0, retried = 0;
  for (int64_t i = threadIdx.x; i < n; i += kSumThreads) {
    its += sf[i].picard_its + (sc ? sc[i].picard_its : 0);
    cyc += sf[i].mg_cycles + (sc ? sc[i].mg_cycles : 0);
    cyc_c += sc ? sc[i].mg_cycles : 0;
    retried += (sf[i].attempts > 1 || (sc && sc[i].attempts > 1)) ? 1 : 0;
    const bool good = stf[i] == RMG_SAMPLE_OK && (!stc || stc[i] == RMG_SAMPLE_OK);
    if (!good) {
      ++bad;
      continue;
    }
    ++ok;
    const double a = qf[i], b = qc ? qc[i] : 0.0, d = a - b;
    neu_add(acc[0], d);
    neu_add(acc[1], d * d);
    neu_add(acc[2], a);
    neu_add(acc[3], a * a);
    neu_add(acc[4], b);
    neu_add(acc[5], b * b);
  }
  for (int k = 0; k < 6; ++k) part[k][threadIdx.x] = acc[k];
  cnt[0][threadIdx.x] = ok;
  cnt[1][threadIdx.x] = bad;
  cnt[2][threadIdx.x] = its;
  cnt[3][threadIdx.x] = cyc;
  cnt[4][threadIdx.x] = cyc_c;
  cnt[5][threadIdx.x] = retried;
  __syncthreads();
  if (threadIdx.x != 0) return;
  Neu tot[6];
  long long c5[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 6; ++k) tot[k] = Neu{0.0, 0.0};
  for (int t = 0; t < kSumThreads; ++t) {
    for (int k = 0; k < 6; ++k) dd_acc(tot[k], part[k][t]);
    for (int k = 0; k < 6; ++k) c5[k] += cnt[k][t];
  }
  rmg_level_sums o;
  o.n = c5[0];
  o.n_failed = c5[1];
  o.picard_its = c5[2];
  o.mg_cycles = c5[3];
  o.mg_cycles_coarse = c5[4];
  o.n_retried = c5[5];
  rmg_dd* dst[6] = {&o.sY, &o.sY2, &o.sQf, &o.sQf2, &o.sQc, &o.sQc2};
  for (int k = 0; k < 6; ++k) {
    // renormalise: hi = fl(s + c), lo = the rounding error of that sum
    const double hi = tot[k].s + tot[k].c;
    const double bb = hi - tot[k].s;
    const double lo = (tot[k].s - (hi - bb)) + (tot[k].c - bb);
    *dst[k] = {hi, lo};
  }
  *out = o;
}

hipError_t launch_level_sums(const double* qf, const double* qc, int64_t n, const int32_t* stf,
                             const int32_t* stc, const rmg_sample_stats* sf,
                             const rmg_sample_stats* sc, rmg_level_sums* out, hipStream_t st) {
  hipLaunchKernelGGL(k_level_sums, dim3(1), dim3(kSumThreads), 0, st, qf, qc, n, stf, stc, sf, sc, out);
  return hipGetLastError();
}

}  // namespace rmg
