// Tile helpers shared by the level-streaming fine-level kernels (forward residual
// and adjoint residual): tile enumeration and the in-tile coarsening of the
// multigrid coefficients (Section 4.2, coarse operators by face upscaling).
#pragma once

#include "rmg_device.hpp"
#include "rmg_internal.hpp"
#include "rmg_smoother.hpp"

namespace rmg {

__device__ __forceinline__ const rmg_problem& class_problem(const ClassProblems& cp, int64_t s) {
  return s < cp.seg_split ? cp.prob[0] : cp.prob[1];
}

// Cells (ri, rj) of a w x w tile, distributed over the kBlock threads of the workgroup.
#define RMG_TILE_FOR(w, ri, rj)                                                                 \
  for (int w_ = (w), once_ = 1; once_; once_ = 0)                                                 \
    for (unsigned mg_ = rmg_magic(w_), once2_ = 1u; once2_; once2_ = 0u)                          \
      for (int k_ = (int)threadIdx.x, rj = 0, ri = 0; k_ < w_ * w_; k_ += kBlock)                   \
        if ((rj = (int)__umulhi((unsigned)k_, mg_), ri = k_ - rj * w_), true)

// Coefficients of the streaming levels 1 .. ltop inside the T x T fine tile at
// (x0, y0) of sample s: bufA holds the tile's fine coefficients (cw [T*T], cdt
// [T*T], cs [(T+1)*T] whose last row is the top Dirichlet weights); each level is
// coarsened from the previous one, ping-ponging between bufA and bufB, and stored
// to the level's global arrays.  Cells of level l inside a 32 x 32 fine tile are
// complete for 2^l <= 32.
template <class R>
__device__ void tile_coarsen(const StreamPlan& pl, int64_t s, int n, int T, int x0, int y0, R* bufA, R* bufB) {
  R* src = bufA;
  R* dst = bufB;
  int t = T;
  for (int l = 1; l <= pl.ltop; ++l) {
    __syncthreads();
    const int tc = t >> 1;
    const int m = n >> l;
    const int64_t M2 = (int64_t)m * m;
    R* scw = src;
    R* scdt = src + t * t;
    R* scs = src + 2 * t * t;
    R* dcw = dst;
    R* dcdt = dst + tc * tc;
    R* dcs = dst + 2 * tc * tc;
    R* gcw = (R*)pl.lv.cw[l] + s * M2;
    R* gcs = (R*)pl.lv.cs[l] + s * M2;
    R* gcdt = (R*)pl.lv.cdt[l] + s * M2;
    R* gctop = (R*)pl.lv.ctop[l] + s * m;
    const int X0 = x0 >> l, Y0 = y0 >> l;
    RMG_TILE_FOR(tc, I, J) {
      const int e = J * tc + I;
      const int f00 = (2 * J) * t + 2 * I;
      const R cw = coarse_face<R>(scw[f00], scw[f00 + t]);
      const R cs = coarse_face<R>(scs[f00], scs[f00 + 1]);
      const R cd = coarse_cdt<R>(scdt[f00], scdt[f00 + 1], scdt[f00 + t], scdt[f00 + t + 1]);
      dcw[e] = cw;
      dcs[e] = cs;
      dcdt[e] = cd;
      const int64_t gc = (int64_t)(Y0 + J) * m + X0 + I;
      gcw[gc] = cw;
      gcs[gc] = cs;
      gcdt[gc] = cd;
    }
    for (int I = threadIdx.x; I < tc; I += kBlock) {
      const R ct = coarse_face<R>(scs[t * t + 2 * I], scs[t * t + 2 * I + 1]);
      dcs[tc * tc + I] = ct;
      if (y0 + T == n) gctop[X0 + I] = ct;
    }
    R* tmp = src;
    src = dst;
    dst = tmp;
    t = tc;
  }
}

}  // namespace rmg
