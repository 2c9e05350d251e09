// Device-side arithmetic shared by every solver kernel (gfx950).
//
// Everything a kernel computes per cell lives here, so that the level-streaming
// kernels and the whole-sample-in-LDS kernels perform the identical sequence of
// floating-point operations (the library is built with -ffp-contract=off; fused
// multiply-adds appear only where written).
//
// Notation (Section 4.2, eq. five_stencil): on a level of m x m cells the
// correction equation is   d_c u_c - sum_nb a_nb u_nb = f_c   with
//   a_w = cw[c], a_e = cw[c+1]     x-face coefficients K_face / H^2 (0 on the no-flux sides)
//   a_s = cs[c], a_n = cs[c+m]     z-face coefficients; on the Dirichlet faces the
//                                  coefficient is 2 K / H^2 and the neighbour is absent
//   d_c = cdt_c + a_w + a_e + a_s + a_n,   cdt = C / dt.
// Storage keeps the top Dirichlet coefficients in a separate row `ctop`.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rmg.h"

// Pointers into LDS carry address space 3 in their type, so that every access is
// a ds_read/ds_write even when the pointer itself was stored and reloaded (a
// generic pointer would compile to the slower flat instructions).
#define RMG_LDS __attribute__((address_space(3)))

namespace rmg {

constexpr int kBlock = 256;  // threads per workgroup for every solver kernel

// ---------------------------------------------------------------- closure laws
// Gardner: Se = e^{a p} (p < 0); van Genuchten-Mualem: Section 2.1 eqs. Sw, sc_van,
// Krw with 1 - S^{1/m} rewritten exactly as u/(1+u), u = |alpha p|^n.
struct Closure {
  double K, theta, C;
};

__device__ __forceinline__ Closure closure(const rmg_problem& P, double p, double Ks, double alpha,
                                           double nvg) {
  Closure r;
  const double dth = P.theta_s - P.theta_r;
  if (P.model == RMG_GARDNER) {
    if (p < 0.0) {
      const double e = exp(P.gardner_a * p);
      r.K = Ks * e;
      r.theta = P.theta_r + dth * e;
      r.C = dth * P.gardner_a * e;
    } else {
      r.K = Ks;
      r.theta = P.theta_s;
      r.C = 0.0;
    }
  } else if (P.model == RMG_VGM) {
    if (p < 0.0) {
      const double a = alpha + P.vg_alpha_shift;
      const double n = nvg + P.vg_n_shift;
      const double m = 1.0 - 1.0 / n;
      const double ap = fabs(a * p);
      const double lap = log(ap);
      const double u = exp(n * lap);
      const double l1u = log1p(u);
      const double S = exp(-m * l1u);
      const double w = u / (1.0 + u);
      const double t = 1.0 - exp(m * log(w));
      r.K = Ks * sqrt(S) * t * t;
      r.theta = P.theta_r + dth * S;
      // dS/d|ap| = m n (1+u)^-(m+1) |ap|^(n-1) with (1+u)^-(m+1) = S / (1+u) and
      // |ap|^(n-1) = u / |ap|: no further exponentials
      r.C = dth * a * m * n * (S / (1.0 + u)) * (u / ap);
    } else {
      r.K = Ks;
      r.theta = P.theta_s;
      r.C = 0.0;
    }
  } else {  // RMG_LINEAR (test law)
    r.K = Ks;
    r.theta = P.theta_r + P.linear_c0 * p;
    r.C = P.linear_c0;
  }
  return r;
}

// Initial pressure head of a cell in row j of an n x n grid: uniform, or the
// exponential profile of the infiltration problem (Section 4.3, eq. travellingwave).
__device__ __forceinline__ double initial_head(const rmg_problem& P, int j, int n) {
  if (P.init_profile == 1) return P.h_init * (1.0 - exp(-P.init_rate * (((double)j + 0.5) / (double)n)));
  return P.h_init;
}

// Field values of sample s at cell c in [S][F][N] layout.
struct CellFields {
  double Ks, alpha, nvg;
};
__device__ __forceinline__ CellFields load_fields(const double* fields, int F, int64_t N, int64_t s,
                                                  int64_t c) {
  const double* b = fields + (s * F) * N + c;
  CellFields f;
  f.Ks = b[0];
  f.alpha = F > 1 ? b[N] : 0.0;
  f.nvg = F > 2 ? b[2 * N] : 0.0;
  return f;
}

// Reciprocal by the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r), each doubling its correct bits (about 1 ulp at the end).  Unlike
// the correctly rounded division sequence it does not pass through the VCC register,
// so independent quotients of one thread overlap instead of running one after another.
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Harmonic mean 2ab/(a+b) of eq. five_stencil; symmetric bit-for-bit in (a, b).
__device__ __forceinline__ double hmean(double a, double b) {
  const double s = a + b;
  return s > 0.0 ? (2.0 * (a * b)) * recip_nr(s) : 0.0;
}

// ------------------------------------------------------- outer Picard residual
// Fine-level quantities of one cell (Section 4.1 eq. Mixed_based_3 with f = 0):
//   f~ = sum_faces K_f ((p_nb - p_c)/d_f + g_f) / h - (theta - theta_old)/dt
// with d_f = h inside, h/2 to a Dirichlet face; g_f = -1 (bottom face), +1 (top
// face), 0 (x-faces); K_f harmonic mean inside, the cell's own K on a Dirichlet
// face; no-flux sides carry nothing.  Coefficients are those of the correction
// equation on the fine mesh.
struct FineCell {
  double f, cw, cs, cdt, ctop;
};

__device__ __forceinline__ FineCell fine_cell(int i, int j, int n, double pc, double pw, double pe,
                                              double ps, double pn, double Kc, double Kw, double Ke,
                                              double Ks_, double Kn, double theta, double theta_old,
                                              double C, double dt, double g_bottom, double g_top) {
  const double inv_h = (double)n;
  const double inv_h2 = inv_h * inv_h;
  FineCell r;
  double flow = 0.0;
  if (i > 0) {
    const double k = hmean(Kw, Kc);
    flow += k * ((pw - pc) * inv_h2);
    r.cw = k * inv_h2;
  } else {
    r.cw = 0.0;
  }
  if (i < n - 1) {
    const double k = hmean(Kc, Ke);
    flow += k * ((pe - pc) * inv_h2);
  }
  if (j > 0) {
    const double k = hmean(Ks_, Kc);
    flow += k * (((ps - pc) * inv_h - 1.0) * inv_h);
    r.cs = k * inv_h2;
  } else {
    flow += Kc * (((g_bottom - pc) * (2.0 * inv_h) - 1.0) * inv_h);
    r.cs = 2.0 * Kc * inv_h2;
  }
  if (j < n - 1) {
    const double k = hmean(Kc, Kn);
    flow += k * (((pn - pc) * inv_h + 1.0) * inv_h);
    r.ctop = 0.0;
  } else {
    flow += Kc * (((g_top - pc) * (2.0 * inv_h) + 1.0) * inv_h);
    r.ctop = 2.0 * Kc * inv_h2;
  }
  const double inv_dt = recip_nr(dt);
  r.cdt = C * inv_dt;
  r.f = flow - (theta - theta_old) * inv_dt;
  return r;
}

// ------------------------------------------------------------- level stencil
// Diagonal and neighbour sum of one cell; absent neighbours enter with u = 0
// (their coefficient is either 0 or a Dirichlet weight that belongs to d only).
template <class R>
struct St5 {
  R d, snb;
};
template <class R>
__device__ __forceinline__ St5<R> st5(R cdt, R aw, R ae, R as, R an, R uw, R ue, R us, R un) {
  St5<R> r;
  R d = cdt;
  d = d + aw;
  d = d + ae;
  d = d + as;
  d = d + an;
  R t1 = aw * uw;
  t1 = t1 + ae * ue;
  R t2 = as * us;
  t2 = t2 + an * un;
  r.d = d;
  r.snb = t1 + t2;
  return r;
}
// Gauss-Seidel update of one cell: u = (f + sum a_nb u_nb) / d.
template <class R>
__device__ __forceinline__ R gs_value(R f, const St5<R>& s) {
  return (f + s.snb) / s.d;
}
// FP32 (the multigrid of the mixed-precision solver): multiply by the hardware
// reciprocal (1 ulp) instead of the correctly rounded division sequence.
template <>
__device__ __forceinline__ float gs_value<float>(float f, const St5<float>& s) {
  return (f + s.snb) * __builtin_amdgcn_rcpf(s.d);
}
// Residual f - A u of one cell.
template <class R>
__device__ __forceinline__ R residual_value(R f, R u, const St5<R>& s) {
  return (f + s.snb) - s.d * u;
}

// Coarse coefficients (Section 4.2, upscaling figure): a coarse face's
// conductivity is the arithmetic mean of the two fine faces it covers; with the
// mesh doubling this is (a1 + a2) / 8 for interior and Dirichlet faces alike.
template <class R>
__device__ __forceinline__ R coarse_face(R a1, R a2) {
  return (a1 + a2) * (R)0.125;
}
// Coarse C/dt: mean of the four fine values.
template <class R>
__device__ __forceinline__ R coarse_cdt(R c00, R c01, R c10, R c11) {
  return ((c00 + c01) + (c10 + c11)) * (R)0.25;
}
// Restriction R = P^T/4 (eq. transfer): mean of the four fine residuals.
template <class R>
__device__ __forceinline__ R restrict4(R r00, R r01, R r10, R r11) {
  return ((r00 + r01) + (r10 + r11)) * (R)0.25;
}

// ------------------------------------------------------------ block helpers
// NT: the workgroup size (compile-time constant).
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  // wave64 reduction through LDS; every thread returns the block maximum
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < NT / 64; ++w) r = fmax(r, red[w]);
  return r;
}

// Non-negative doubles order like their bit patterns: max via integer atomics.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v) {
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

}  // namespace rmg
