// Whole-grid multigrid levels held in LDS by one workgroup (gfx950, 160 KiB LDS per CU).
// NT is the workgroup size (a compile-time constant, so that loops stride by a
// constant instead of reading the launch size from the dispatch packet).
//
// Layout of a level with m x m cells (element type R):
//   u   : one zero row, m*m cells, one zero row (plus one guard each end), so
//         u[c - m], u[c + m], u[c - 1], u[c + 1] are always readable; a neighbour
//         outside the domain (a zero row below or above, or across the left or
//         right side the end cell of the adjacent row) meets a zero or
//         Dirichlet-only coefficient;
//   f, cdt : m*m;
//   cw  : m*m + 1, cw[j*m] = 0 (no-flux left face) and cw[m*m] = 0, so the east
//         coefficient cw[c + 1] of a right-edge cell is the next row's left face = 0;
//   cs  : (m+1)*m, rows 0..m-1 are south faces (row 0: bottom Dirichlet weight),
//         row m holds the top Dirichlet weights, so the north coefficient is cs[c + m].
// The zero rows and guards are written once when the workgroup starts; levels follow
// one another in that order of arrays (LdsHier).
#pragma once

#include "rmg_device.hpp"

namespace rmg {


template <class R>
struct LdsLevel {
  RMG_LDS R* u;
  RMG_LDS R* f;
  RMG_LDS R* cw;
  RMG_LDS R* cs;
  RMG_LDS R* cdt;
  int m, lg;  // m = 1 << lg
};

// Elements of R needed by one level.
__host__ __device__ constexpr int lds_level_elems(int m) {
  return ((m + 2) * m + 2) + m * m + (m * m + 1) + (m + 1) * m + m * m;
}

// The levels m_top, m_top/2, ... laid out one after another from `base`.  Level l
// starts sum_{k<l} lds_level_elems(m_top >> k) elements in, which in closed form
// is 20 (m^2 - m_l^2) / 3 + 6 (m - m_l) + 3 l with m = m_top, m_l = m >> l, so a
// level's pointers are a few scalar operations away and need no table: a table in
// LDS would put one more LDS round trip in front of every phase's loads, and a
// runtime-indexed table in registers would live in scratch memory.
template <class R>
struct LdsHier {
  R* base;
  int m_top, lg_top;
  __device__ __forceinline__ int offset(int l) const {
    const int ml = m_top >> l;
    return (20 * (m_top * m_top - ml * ml)) / 3 + 6 * (m_top - ml) + 3 * l;
  }
  __device__ __forceinline__ LdsLevel<R> operator[](int l) const {
    LdsLevel<R> L;
    const int m = m_top >> l;
    L.m = m;
    L.lg = lg_top - l;
    R* p = base + offset(l);
    L.u = (RMG_LDS R*)(p + 1 + m);
    p += (m + 2) * m + 2;
    L.f = (RMG_LDS R*)p;
    p += m * m;
    L.cw = (RMG_LDS R*)p;
    p += m * m + 1;
    L.cs = (RMG_LDS R*)p;
    p += (m + 1) * m;
    L.cdt = (RMG_LDS R*)p;
    return L;
  }
  // one past the last element of levels 0 .. nlev-1
  __device__ __forceinline__ R* end(int nlev) const { return base + offset(nlev); }
};

template <class R>
__device__ __forceinline__ LdsHier<R> lds_hier(R* base, int m_top) {
  LdsHier<R> H;
  H.base = base;
  H.m_top = m_top;
  H.lg_top = 31 - __clz(m_top);
  return H;
}

// Zero the elements of a hierarchy (LdsHier) that no routine writes: the
// zero rows and guards around each level's u and the trailing guard of its cw.
// Every other element (cells of u, f, cw, cs including the top weights, cdt) is
// written before it is read: loaded or computed on the top level, produced by
// lds_residual_restrict (right-hand side, zero iterate, coefficients) below it.
template <class R, int NT>
__device__ void lds_zero_padding(R* base, int m_top, int nlev) {
  R* p = base;
  int m = m_top;
  for (int l = 0; l < nlev; ++l) {
    const int span = (m + 2) * m + 2;  // u with its rows and guards
    for (int k = threadIdx.x; k <= m; k += NT) {
      p[k] = (R)0;
      p[span - 1 - k] = (R)0;
    }
    p += span + m * m;  // past u and f: p is cw
    if (threadIdx.x == 0) p[m * m] = (R)0;
    p += (m * m + 1) + (m + 1) * m + m * m;
    m >>= 1;
  }
}

template <class R>
__device__ __forceinline__ St5<R> lds_st5(const LdsLevel<R>& L, int c) {
  const int m = L.m;
  return st5<R>(L.cdt[c], L.cw[c], L.cw[c + 1], L.cs[c], L.cs[c + m], L.u[c - 1], L.u[c + 1],
                L.u[c - m], L.u[c + m]);
}

// Cell (i, j) of the k-th cell of `colour` on an m x m level (m = 2^(hlg+1)).  The
// cells of one colour in a row lie two apart, so a row's worth of lanes would meet
// every LDS bank it touches twice; lanes therefore take chunks of up to 16 cells
// alternately from rows 2r and 2r+1, whose cells of that colour sit on the other
// bank parity (a row is a multiple of 32 elements apart from the next-but-one), so
// consecutive lanes cover all banks.  Any order of the cells of one colour gives
// the same sweep.  (Keeping the plain row order below 32 x 32, where the chunks are
// shorter, was measured slower: the branch cost more than the index operations.)
// LGC: log2 of the chunk; LGC >= hlg gives the plain order (row 2r, then row 2r+1).
// The chunks pay in the 512-thread coarse kernel (5-level step -1.5 %); the smaller
// workgroups of the whole-sample kernel keep the plain order (with it, rather than
// the chunks, the robustness sweep takes 1814 ms against 1829 ms and the 5-level
// step 194.7 ms against 195.7 ms).
template <int NT>
__host__ __device__ constexpr int rb_chunk_lg() {
  return NT >= 512 ? 4 : 30;
}

template <int LGC>
__device__ __forceinline__ void rb_cell(int k, int m, int hlg, int colour, int& i, int& j) {
  const int lgc = hlg < LGC ? hlg : LGC;  // chunk of min(2^LGC, m/2) cells
  const int w = k & (m - 1);          // position within the row pair
  const int q = ((w >> (lgc + 1)) << lgc) | (w & ((1 << lgc) - 1));
  j = 2 * (k >> (hlg + 1)) + ((w >> lgc) & 1);
  i = 2 * q + ((j + colour) & 1);
}

// One colour of a red-black Gauss-Seidel sweep (colour 0 = red = (i+j) even).
template <class R, int NT>
__device__ void lds_half_sweep(const LdsLevel<R>& L, int colour) {
  const int m = L.m, hlg = L.lg - 1;
  const int tot = (m * m) >> 1;
  for (int k = threadIdx.x; k < tot; k += NT) {
    int i, j;
    rb_cell<rb_chunk_lg<NT>()>(k, m, hlg, colour, i, j);
    const int c = j * m + i;
    L.u[c] = gs_value<R>(L.f[c], lds_st5(L, c));
  }
}

// Red half-sweep when the current iterate is zero: the neighbour sum vanishes, so
// u = f / d without reading neighbours (the same operations as lds_half_sweep on a
// zero iterate).
template <class R, int NT>
__device__ void lds_half_sweep_from_zero(const LdsLevel<R>& L) {
  const int m = L.m, hlg = L.lg - 1;
  const int tot = (m * m) >> 1;
  for (int k = threadIdx.x; k < tot; k += NT) {
    int i, j;
    rb_cell<rb_chunk_lg<NT>()>(k, m, hlg, 0, i, j);
    const int c = j * m + i;
    const St5<R> s = st5<R>(L.cdt[c], L.cw[c], L.cw[c + 1], L.cs[c], L.cs[c + m], (R)0, (R)0, (R)0, (R)0);
    L.u[c] = gs_value<R>(L.f[c], s);
  }
}

// Red half-sweep right after the coarse-grid correction: the black neighbours are
// read as u + (prolongated coarse correction); the red cells' own corrected values
// are never needed (they are overwritten), and the black cells are overwritten by
// the following black half-sweep, so no separate prolongation pass is required.
template <class R, int NT>
__device__ void lds_half_sweep_prolong(const LdsLevel<R>& L, const LdsLevel<R>& C) {
  const int m = L.m, hlg = L.lg - 1, mc = C.m;
  const int tot = (m * m) >> 1;
  for (int k = threadIdx.x; k < tot; k += NT) {
    int i, j;
    rb_cell<rb_chunk_lg<NT>()>(k, m, hlg, 0, i, j);
    const int c = j * m + i;
    const R uw = i > 0 ? L.u[c - 1] + C.u[(j >> 1) * mc + ((i - 1) >> 1)] : (R)0;
    const R ue = i < m - 1 ? L.u[c + 1] + C.u[(j >> 1) * mc + ((i + 1) >> 1)] : (R)0;
    const R us = j > 0 ? L.u[c - m] + C.u[((j - 1) >> 1) * mc + (i >> 1)] : (R)0;
    const R un = j < m - 1 ? L.u[c + m] + C.u[((j + 1) >> 1) * mc + (i >> 1)] : (R)0;
    const St5<R> s = st5<R>(L.cdt[c], L.cw[c], L.cw[c + 1], L.cs[c], L.cs[c + m], uw, ue, us, un);
    L.u[c] = gs_value<R>(L.f[c], s);
  }
}

// Ordering between phases: a workgroup barrier, or (WAVE: the levels that the first
// wavefront runs alone) a wavefront-scope fence -- LDS operations of one wavefront
// complete in issue order, so only the compiler must be kept from moving them.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <class R, int NT, bool WAVE = false>
__device__ void lds_sweeps(const LdsLevel<R>& L, int nu, bool from_zero = false) {
  for (int s = 0; s < nu; ++s) {
    if (s == 0 && from_zero)
      lds_half_sweep_from_zero<R, NT>(L);
    else
      lds_half_sweep<R, NT>(L, 0);
    lds_sync<WAVE>();
    lds_half_sweep<R, NT>(L, 1);
    lds_sync<WAVE>();
  }
}

// Coarse right-hand side = R (f - A u); coarse initial iterate 0.  COARSEN: also
// the coefficients of C in the same pass over the coarse cells (Section 4.2: each
// coarse face the arithmetic mean of the two fine faces it covers, C/dt the mean of
// the four fine cells, the top Dirichlet weights likewise).
template <class R, int NT, bool COARSEN = false>
__device__ void lds_residual_restrict(const LdsLevel<R>& F, const LdsLevel<R>& C) {
  const int mc = C.m, m = F.m;
  for (int kc = threadIdx.x; kc < mc * mc; kc += NT) {
    const int J = kc >> C.lg, I = kc - (J << C.lg);
    const int c00 = (2 * J) * m + 2 * I;
    // alternate 16-lane chunks take the two cells of a fine row in the other order,
    // so that one load instruction touches both bank parities (the workgroups that
    // sweep in chunks; the order does not change the values)
    const int sw = rb_chunk_lg<NT>() <= 4 ? ((threadIdx.x >> 4) & 1) : 0;
    const int ca = c00 + sw, cb = c00 + 1 - sw;
    const R ra0 = residual_value<R>(F.f[ca], F.u[ca], lds_st5(F, ca));
    const R rb0 = residual_value<R>(F.f[cb], F.u[cb], lds_st5(F, cb));
    const R ra1 = residual_value<R>(F.f[ca + m], F.u[ca + m], lds_st5(F, ca + m));
    const R rb1 = residual_value<R>(F.f[cb + m], F.u[cb + m], lds_st5(F, cb + m));
    const R r00 = sw ? rb0 : ra0, r01 = sw ? ra0 : rb0;
    const R r10 = sw ? rb1 : ra1, r11 = sw ? ra1 : rb1;
    C.f[kc] = restrict4<R>(r00, r01, r10, r11);
    C.u[kc] = (R)0;
    if (COARSEN) {
      C.cw[kc] = coarse_face<R>(F.cw[c00], F.cw[c00 + m]);
      C.cs[kc] = coarse_face<R>(F.cs[c00], F.cs[c00 + 1]);
      C.cdt[kc] = coarse_cdt<R>(F.cdt[c00], F.cdt[c00 + 1], F.cdt[c00 + m], F.cdt[c00 + m + 1]);
    }
  }
  if (COARSEN)
    for (int I = threadIdx.x; I < mc; I += NT)
      C.cs[mc * mc + I] = coarse_face<R>(F.cs[m * m + 2 * I], F.cs[m * m + 2 * I + 1]);
}

// Piecewise-constant prolongation of the coarse correction (eq. transfer).
template <class R, int NT>
__device__ void lds_prolong_add(const LdsLevel<R>& F, const LdsLevel<R>& C) {
  const int m = F.m;
  for (int c = threadIdx.x; c < m * m; c += NT) {
    const int j = c >> F.lg, i = c - (j << F.lg);
    F.u[c] = F.u[c] + C.u[(j >> 1) * C.m + (i >> 1)];
  }
}

// Value of v in lane `lane` of the wavefront, for every lane (two readlanes).
__device__ __forceinline__ double wave_read(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Pivot order of the coarsest solve: the red cells ((i + j) even) first, then the
// black ones.  The five-point operator couples red cells only to black cells, so a
// red pivot row holds its diagonal and its black neighbours only (earlier red pivots
// leave it untouched: its entries in their columns are zero) and the eight red steps
// do not depend on one another; the black steps then eliminate the dense 8 x 8 (or
// 2 x 2) Schur complement.
template <int M>
struct CoarsestOrder {
  int piv[M * M];
  constexpr CoarsestOrder() : piv() {
    int t = 0;
    for (int colour = 0; colour < 2; ++colour)
      for (int c = 0; c < M * M; ++c)
        if ((((c % M) + (c / M)) & 1) == colour) piv[t++] = c;
  }
};
// Reciprocal of a pivot: recip_nr (no VCC-serialised division sequence, so the
// independent red pivots' reciprocals overlap).
__device__ __forceinline__ double pivot_recip(double x) { return recip_nr(x); }
__host__ __device__ constexpr bool grid_adjacent(int m, int a, int b) {
  const int di = a % m - b % m, dj = a / m - b / m;
  return (di == 1 || di == -1) ? dj == 0 : ((dj == 1 || dj == -1) && di == 0);
}

// Exact solve on the coarsest level (N = m*m = 4 or 16 unknowns) in FP64:
// Gauss-Jordan elimination without pivoting on the symmetric positive definite
// matrix, in the registers of the first wavefront.  Lane c holds row c of the
// matrix (columns 0..N-1) and its right-hand side; the step of pivot k reads the
// pivot row from lane k (a wave-uniform value, so no LDS round trip and no barrier)
// and replaces every row c != k by row_c - (a_ck / a_kk) row_k on the columns of
// the pivots still to come (column k is then logically zero and never read again).
// Pivots are taken in CoarsestOrder, and a red pivot's step touches only the
// columns of its neighbours (its other entries are zero, so the skipped updates
// would subtract exact zeros).  The unknown is the row's right-hand side times the
// reciprocal of its pivot.  Lanes N..63 duplicate rows.
// Kept out of line: inlined, its unrolled rows and scalar pivot-row reads raised
// the register pressure of the calling kernels, whose sweep loops then reloaded
// spilled scalar registers (every level and class ran slower).
template <class R, int N>
__device__ __attribute__((noinline)) void coarsest_gauss_jordan(RMG_LDS R* Lu, const RMG_LDS R* Lf,
                                                               const RMG_LDS R* Lcw, const RMG_LDS R* Lcs,
                                                               const RMG_LDS R* Lcdt) {
  constexpr int m = N == 16 ? 4 : 2, lg = N == 16 ? 2 : 1;
  struct {
    RMG_LDS R* u;
    const RMG_LDS R *f, *cw, *cs, *cdt;
  } const L = {Lu, Lf, Lcw, Lcs, Lcdt};
  constexpr CoarsestOrder<m> ord{};
  const int c = (int)(threadIdx.x & (N - 1));
  const int j = c >> lg, i = c - (j << lg);
  const double aw = (double)L.cw[c], ae = (double)L.cw[c + 1];
  const double as = (double)L.cs[c], an = (double)L.cs[c + m];
  const St5<double> s = st5<double>((double)L.cdt[c], aw, ae, as, an, 0.0, 0.0, 0.0, 0.0);
  double a[N];
#pragma unroll
  for (int col = 0; col < N; ++col) {
    double v = 0.0;
    if (col == c) v = s.d;
    if (i > 0 && col == c - 1) v = -aw;
    if (i < m - 1 && col == c + 1) v = -ae;
    if (j > 0 && col == c - m) v = -as;
    if (j < m - 1 && col == c + m) v = -an;
    a[col] = v;
  }
  double b = (double)L.f[c], rpiv = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const int k = ord.piv[t];
    // lane k's row is not modified in its own step, so each pivot-row entry can be
    // read just before the column it updates
    const double pk = pivot_recip(wave_read(a[k], k));
    rpiv = c == k ? pk : rpiv;
    const double mk = c != k ? a[k] * pk : 0.0;
#pragma unroll
    for (int u = t + 1; u < N; ++u) {
      const int col = ord.piv[u];
      if (t < N / 2 && !grid_adjacent(m, k, col)) continue;
      const double akj = wave_read(a[col], k);
      if (c != k) a[col] = a[col] - mk * akj;
    }
    const double bk = wave_read(b, k);
    if (c != k) b = b - mk * bk;
  }
  if ((int)threadIdx.x < N) L.u[c] = (R)(b * rpiv);
}

// Value of v in lane `src` (0..63), for each lane its own src.
__device__ __forceinline__ double lane_value(double v, int src) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(x & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Exact solve on a 4 x 4 coarsest level (16 unknowns) in FP64 by the Schur complement
// of the red cells, in the first wavefront.  The five-point operator couples red cells
// ((i + j) even) only to black ones, so the red block is diagonal and eliminating it
// leaves, for the black unknowns,
//   S u_b = g,  S = D_b - C^T D_r^{-1} C,  g = f_b + C^T D_r^{-1} f_r,
// with C the (positive) face coefficients between red and black cells.  Lane 8 r + c
// forms S[r][c] (and lane 8 r + anything g[r]) from the level's coefficients;
// Gauss-Jordan elimination on the 8 x 8 system follows, step k reading the pivot from
// lane 9 k and the pivot column of a lane's row and the pivot row by lane permutes;
// finally the red unknowns follow from their black neighbours,
// u_r = (f_r + sum_b a_rb u_b) / d_r.  Reciprocals: pivot_recip.
// (Measured on one wavefront with its caches warm: 3930 clocks per solve; 4330 with
// a branch per neighbour direction, whose LDS loads and reciprocals then ran one
// direction after the other; 4990 for a variant that gathers rows into lanes for
// elimination with wave-uniform pivot rows: single-wavefront code pays the full
// latency of every instruction, and that variant's readlanes outnumbered the
// permutes it saved.)
template <class R>
__device__ __attribute__((noinline)) void coarsest_schur16(RMG_LDS R* Lu, const RMG_LDS R* Lf, const RMG_LDS R* Lcw,
                                                          const RMG_LDS R* Lcs, const RMG_LDS R* Lcdt) {
  constexpr int m = 4;
  const int lane = (int)(threadIdx.x & 63);
  const int r8 = lane >> 3, c8 = lane & 7;
  // black cell q: row q >> 1, column 2 (q & 1) + (row + 1) mod 2; red cell q: 2 (q & 1) + row mod 2
  const int jb = r8 >> 1, ib = 2 * (r8 & 1) + ((jb + 1) & 1);
  const int jp = c8 >> 1, ip = 2 * (c8 & 1) + ((jp + 1) & 1);
  const int b = jb * m + ib;
  // diagonal of a cell (st5 order: C/dt, west, east, south, north faces)
  auto diag = [&](int c) {
    double d = (double)Lcdt[c];
    d = d + (double)Lcw[c];
    d = d + (double)Lcw[c + 1];
    d = d + (double)Lcs[c];
    d = d + (double)Lcs[c + m];
    return d;
  };
  double sv = r8 == c8 ? diag(b) : 0.0;
  double g = (double)Lf[b];
  // red neighbours of b in the order west, east, south, north; a neighbour outside the
  // grid is read at b itself and its terms are selected away, so the four directions
  // are straight-line code whose LDS loads and reciprocals overlap
  double t[4], fr[4], krp[4];
  bool in[4];
#pragma unroll
  for (int dir = 0; dir < 4; ++dir) {
    const int di = dir == 0 ? -1 : dir == 1 ? 1 : 0, dj = dir == 2 ? -1 : dir == 3 ? 1 : 0;
    const int ir = ib + di, jr = jb + dj;
    in[dir] = ir >= 0 && ir < m && jr >= 0 && jr < m;
    const int r = in[dir] ? jr * m + ir : b;
    const double kbr = dir == 0 ? (double)Lcw[b] : dir == 1 ? (double)Lcw[b + 1]
                     : dir == 2 ? (double)Lcs[b] : (double)Lcs[b + m];
    t[dir] = kbr * pivot_recip(diag(r));
    fr[dir] = (double)Lf[r];
    // coupling of r with the column's black cell, if they are neighbours
    const int ei = ip - ir, ej = jp - jr;
    const double kw = (double)Lcw[r], ke = (double)Lcw[r + 1], ks = (double)Lcs[r], kn = (double)Lcs[r + m];
    double k = 0.0;
    k = (ei == -1 && ej == 0) ? kw : k;
    k = (ei == 1 && ej == 0) ? ke : k;
    k = (ei == 0 && ej == -1) ? ks : k;
    k = (ei == 0 && ej == 1) ? kn : k;
    krp[dir] = k;
  }
#pragma unroll
  for (int dir = 0; dir < 4; ++dir) {
    if (in[dir]) g = g + t[dir] * fr[dir];
    if (in[dir]) sv = sv - t[dir] * krp[dir];
  }
  double rpiv = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double pk = pivot_recip(wave_read(sv, 9 * k));
    const double ark = lane_value(sv, 8 * r8 + k);
    const double akc = lane_value(sv, 8 * k + c8);
    const double gk = wave_read(g, 8 * k);
    rpiv = r8 == k ? pk : rpiv;
    const double mk = r8 != k ? ark * pk : 0.0;
    if (r8 != k && c8 > k) sv = sv - mk * akc;
    if (r8 != k) g = g - mk * gk;
  }
  const double ub = g * rpiv;
  if (c8 == 0) Lu[b] = (R)ub;
  // every black value is in LDS before the red cells read them (one wavefront)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane < 8) {
    const int jr = lane >> 1, ir = 2 * (lane & 1) + (jr & 1);
    const int r = jr * m + ir;
    // neighbours outside the grid are read at r and replaced by zero
    const double vw = (double)Lu[ir > 0 ? r - 1 : r], ve = (double)Lu[ir < m - 1 ? r + 1 : r];
    const double vs = (double)Lu[jr > 0 ? r - m : r], vn = (double)Lu[jr < m - 1 ? r + m : r];
    const double uw = ir > 0 ? vw : 0.0, ue = ir < m - 1 ? ve : 0.0;
    const double us = jr > 0 ? vs : 0.0, un = jr < m - 1 ? vn : 0.0;
    double t1 = (double)Lcw[r] * uw;
    t1 = t1 + (double)Lcw[r + 1] * ue;
    double t2 = (double)Lcs[r] * us;
    t2 = t2 + (double)Lcs[r + m] * un;
    Lu[r] = (R)(((double)Lf[r] + (t1 + t2)) * pivot_recip(diag(r)));
  }
}

template <class R, int NT, bool WAVE = false>
__device__ void lds_coarsest_solve(const LdsLevel<R>& L) {
  static_assert(NT >= 64, "the coarsest solve runs on the first wavefront");
  // (the level's arrays go to the out-of-line solvers as separate pointers: a struct
  // passed by reference would be written to scratch memory and read back there)
  if (threadIdx.x < 64) {
    if (L.m == 4)
      coarsest_schur16<R>(L.u, L.f, L.cw, L.cs, L.cdt);
    else
      coarsest_gauss_jordan<R, 4>(L.u, L.f, L.cw, L.cs, L.cdt);
  }
  lds_sync<WAVE>();
}

#ifndef RMG_ZERO_SWEEP
#define RMG_ZERO_SWEEP 1
#endif
#ifndef RMG_FUSED_PROLONG
#define RMG_FUSED_PROLONG 1
#endif

// Post-smoothing of level l after its coarse correction (prolongation fused into the
// first red half-sweep when nu2 > 0).
template <class R, int NT, bool WAVE = false>
__device__ void lds_up_leg(const LdsHier<R>& lev, int l, int nu2) {
  if (RMG_FUSED_PROLONG && nu2 > 0) {
    lds_half_sweep_prolong<R, NT>(lev[l], lev[l + 1]);
    lds_sync<WAVE>();
    lds_half_sweep<R, NT>(lev[l], 1);
    lds_sync<WAVE>();
    lds_sweeps<R, NT, WAVE>(lev[l], nu2 - 1);
  } else {
    lds_prolong_add<R, NT>(lev[l], lev[l + 1]);
    lds_sync<WAVE>();
    lds_sweeps<R, NT, WAVE>(lev[l], nu2);
  }
}

#ifndef RMG_WS_WAVE_M
#define RMG_WS_WAVE_M 8
#endif

// One multigrid cycle from level `top` of the LDS hierarchy (levels top .. nlev-1;
// gamma = 1: V-cycle, gamma = 2: W-cycle; Section 4.2), written as a loop: descend
// with pre-smoothing and restriction to the coarsest level, solve it exactly, then
// ascend with prolongation and post-smoothing; a W-cycle descends once more from
// every level before ascending past it.  A level's first visit starts from a zero
// iterate (its restriction set it to zero), a second visit from the current
// iterate.  `top_zero`: the iterate on level `top` is zero on entry.  `coarsen`:
// the coefficients of the levels below `top` are formed on the first descent, each
// in the restriction pass that enters its level (before the level is first used).
// WM > 0: the levels below `top` of at most WM x WM cells are cycled by the first
// wavefront alone, without workgroup barriers, as the bottom solve of the levels
// above them (the same operations in the same order per cell).  Measured: it pays
// in the whole-sample kernel's W-cycles (WM = 8: robustness sweep -2 %), not in the
// coarse kernel's V-cycle (WM = 16 there: +1 % per MLMC step).
template <class R, int NT, bool WAVE = false, int WM = 0>
__device__ void lds_cycle(const LdsHier<R>& lev, int top, int nlev, int nu1, int nu2, int gamma,
                          bool top_zero, bool coarsen = false) {
  int nb = nlev - 1;  // bottom: the coarsest level, or the first wavefront's levels
  if constexpr (!WAVE && NT > 64 && WM > 0) {
    for (int l = top + 1; l < nlev - 1; ++l)
      if ((lev.m_top >> l) <= WM) {
        nb = l;
        break;
      }
  }
  int l = top;
  bool zero = top_zero;
  unsigned again = 0;  // bit l: level l owes one more coarse cycle (W-cycle)
  for (;;) {
    for (; l < nb; ++l) {
      lds_sweeps<R, NT, WAVE>(lev[l], nu1, RMG_ZERO_SWEEP && zero);
      if (coarsen)
        lds_residual_restrict<R, NT, true>(lev[l], lev[l + 1]);
      else
        lds_residual_restrict<R, NT>(lev[l], lev[l + 1]);
      lds_sync<WAVE>();
      if (gamma == 2) again |= 1u << l;
      zero = true;
    }
    if constexpr (!WAVE && NT > 64 && WM > 0) {
      if (nb < nlev - 1) {
        if (threadIdx.x < 64) lds_cycle<R, 64, true>(lev, nb, nlev, nu1, nu2, gamma, zero, coarsen);
        __syncthreads();
      } else {
        lds_coarsest_solve<R, NT>(lev[nlev - 1]);
      }
    } else {
      lds_coarsest_solve<R, NT, WAVE>(lev[nlev - 1]);
    }
    coarsen = false;
    bool descend = false;
    while (l > top) {
      --l;
      if (again & (1u << l)) {
        again &= ~(1u << l);
        ++l;
        zero = false;
        descend = true;
        break;
      }
      lds_up_leg<R, NT, WAVE>(lev, l, nu2);
    }
    if (!descend) return;
  }
}

// ---------------------------------------------------------------------------
// Top level of the coarse kernel with its coefficients in registers.  Within one
// cycle the coefficients of a level do not change, so each thread keeps, for the
// CPT cells of each colour it updates (the cells the loop of lds_half_sweep gives
// it), the diagonal, the four face coefficients and the right-hand side in
// registers: a half-sweep then reads only the four neighbour values from LDS
// (instead of ten values per cell), all of a thread's loads issued before its
// stores.  The arithmetic is that of st5 / gs_value in the same order, so the
// results are bit-identical to lds_cycle's.

#ifndef RMG_NEST_CACHE
#define RMG_NEST_CACHE 1
#endif

template <class R, int CPT>
struct SweepCache {
  R d[2][CPT], aw[2][CPT], ae[2][CPT], as[2][CPT], an[2][CPT], f[2][CPT];
};

// Cell (i, j) of the r-th cell of `colour` of this thread on an M x M level.
template <int NT, int M>
__device__ __forceinline__ int sweep_cell(int colour, int r, int& i, int& j) {
  constexpr int hlg = (M == 64 ? 6 : M == 32 ? 5 : M == 16 ? 4 : 3) - 1;
  static_assert((1 << (hlg + 1)) == M, "unsupported level size");
  rb_cell<rb_chunk_lg<NT>()>((int)threadIdx.x + r * NT, M, hlg, colour, i, j);
  return j * M + i;
}

template <class R>
__device__ __forceinline__ R cached_gs(R d, R aw, R ae, R as, R an, R f, R uw, R ue, R us, R un) {
  R t1 = aw * uw;
  t1 = t1 + ae * ue;
  R t2 = as * us;
  t2 = t2 + an * un;
  St5<R> s;
  s.d = d;
  s.snb = t1 + t2;
  return gs_value<R>(f, s);
}

template <class R, int NT, int M, int CPT>
__device__ __forceinline__ void sweep_cache_load(SweepCache<R, CPT>& K, const LdsLevel<R>& L) {
#pragma unroll
  for (int colour = 0; colour < 2; ++colour)
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      int i, j;
      const int c = sweep_cell<NT, M>(colour, r, i, j);
      const R aw = L.cw[c], ae = L.cw[c + 1], as = L.cs[c], an = L.cs[c + M];
      R d = L.cdt[c];
      d = d + aw;
      d = d + ae;
      d = d + as;
      d = d + an;
      K.d[colour][r] = d;
      K.aw[colour][r] = aw;
      K.ae[colour][r] = ae;
      K.as[colour][r] = as;
      K.an[colour][r] = an;
      K.f[colour][r] = L.f[c];
    }
}

// One colour of a sweep from the cache.  MODE 0: neighbours from u; 1: the iterate
// is zero (lds_half_sweep_from_zero); 2: neighbours are u plus the prolongated
// coarse correction of C (lds_half_sweep_prolong).
template <class R, int NT, int M, int CPT, int MODE>
__device__ __forceinline__ void cached_half_sweep(const SweepCache<R, CPT>& K, const LdsLevel<R>& L,
                                                  const LdsLevel<R>& C, int colour) {
  R uw[CPT], ue[CPT], us[CPT], un[CPT];
  int cc[CPT];
#pragma unroll
  for (int r = 0; r < CPT; ++r) {
    int i, j;
    const int c = sweep_cell<NT, M>(colour, r, i, j);
    cc[r] = c;
    if (MODE == 1) {
      uw[r] = ue[r] = us[r] = un[r] = (R)0;
    } else if (MODE == 0) {
      uw[r] = L.u[c - 1];
      ue[r] = L.u[c + 1];
      us[r] = L.u[c - M];
      un[r] = L.u[c + M];
    } else {
      constexpr int mc = M / 2;
      uw[r] = i > 0 ? L.u[c - 1] + C.u[(j >> 1) * mc + ((i - 1) >> 1)] : (R)0;
      ue[r] = i < M - 1 ? L.u[c + 1] + C.u[(j >> 1) * mc + ((i + 1) >> 1)] : (R)0;
      us[r] = j > 0 ? L.u[c - M] + C.u[((j - 1) >> 1) * mc + (i >> 1)] : (R)0;
      un[r] = j < M - 1 ? L.u[c + M] + C.u[((j + 1) >> 1) * mc + (i >> 1)] : (R)0;
    }
  }
#pragma unroll
  for (int r = 0; r < CPT; ++r)
    L.u[cc[r]] = cached_gs<R>(K.d[colour][r], K.aw[colour][r], K.ae[colour][r], K.as[colour][r],
                              K.an[colour][r], K.f[colour][r], uw[r], ue[r], us[r], un[r]);
}

// lds_cycle from level LVL (M x M cells, M*M = 2*CPT*NT) with that level's sweeps
// from registers: pre-smoothing, restriction, gamma cycles of level LVL+1 (the
// first from a zero iterate), post-smoothing with the prolongation fused into its
// first red half-sweep -- the same sequence of operations as lds_cycle(lev, LVL,
// ...).  Where level LVL+1 has one cell of each colour per thread, its cycles are
// register-cached too.
template <class R, int NT, int M, int WM = 0, int LVL = 0>
__device__ void lds_cycle_top_cached(const LdsHier<R>& lev, int nlev, int nu1, int nu2, int gamma,
                                     bool top_zero, bool coarsen) {
  constexpr int CPT = M * M / (2 * NT);
  static_assert(CPT >= 1 && 2 * CPT * NT == M * M, "every cell of the top level needs one owner");
  constexpr bool kNest = RMG_NEST_CACHE && WM == 0 && (M / 2) * (M / 2) == 2 * NT;
  const LdsLevel<R> L = lev[LVL];
  {
    SweepCache<R, CPT> K;
    sweep_cache_load<R, NT, M, CPT>(K, L);
    for (int s = 0; s < nu1; ++s) {
      if (s == 0 && RMG_ZERO_SWEEP && top_zero)
        cached_half_sweep<R, NT, M, CPT, 1>(K, L, L, 0);
      else
        cached_half_sweep<R, NT, M, CPT, 0>(K, L, L, 0);
      __syncthreads();
      cached_half_sweep<R, NT, M, CPT, 0>(K, L, L, 1);
      __syncthreads();
    }
  }
  if (coarsen)
    lds_residual_restrict<R, NT, true>(lev[LVL], lev[LVL + 1]);
  else
    lds_residual_restrict<R, NT>(lev[LVL], lev[LVL + 1]);
  __syncthreads();
  for (int g = 0; g < gamma; ++g) {
    if constexpr (kNest) {
      if (nlev >= LVL + 3) {
        lds_cycle_top_cached<R, NT, M / 2, WM, LVL + 1>(lev, nlev, nu1, nu2, gamma, g == 0, coarsen && g == 0);
        continue;
      }
    }
    lds_cycle<R, NT, false, WM>(lev, LVL + 1, nlev, nu1, nu2, gamma, g == 0, coarsen && g == 0);
  }
  if (RMG_FUSED_PROLONG && nu2 > 0) {
    SweepCache<R, CPT> K;
    sweep_cache_load<R, NT, M, CPT>(K, L);
    cached_half_sweep<R, NT, M, CPT, 2>(K, L, lev[LVL + 1], 0);
    __syncthreads();
    cached_half_sweep<R, NT, M, CPT, 0>(K, L, L, 1);
    __syncthreads();
    for (int s = 1; s < nu2; ++s) {
      cached_half_sweep<R, NT, M, CPT, 0>(K, L, L, 0);
      __syncthreads();
      cached_half_sweep<R, NT, M, CPT, 0>(K, L, L, 1);
      __syncthreads();
    }
  } else {
    lds_up_leg<R, NT>(lev, LVL, nu2);
  }
}

// One cycle from the top level of the coarse kernel: register-cached top-level
// sweeps where the level size has a specialisation, lds_cycle otherwise.
template <class R, int NT>
__device__ void lds_cycle_coarse(const LdsHier<R>& lev, int nlev, int nu1, int nu2, int gamma, bool top_zero,
                                 bool coarsen) {
  const int m = lev.m_top;
  if constexpr (sizeof(R) == 4 && 64 * 64 == 8 * NT) {
    if (nlev >= 2 && m == 64) {
      lds_cycle_top_cached<R, NT, 64>(lev, nlev, nu1, nu2, gamma, top_zero, coarsen);
      return;
    }
  }
  if constexpr (32 * 32 == 2 * NT) {
    if (nlev >= 2 && m == 32) {
      lds_cycle_top_cached<R, NT, 32>(lev, nlev, nu1, nu2, gamma, top_zero, coarsen);
      return;
    }
  }
  lds_cycle<R, NT>(lev, 0, nlev, nu1, nu2, gamma, top_zero, coarsen);
}

// One cycle of the whole-sample kernel: register-cached top-level sweeps for 32 x 32
// grids on 256 threads (two cells of each colour per thread); other sizes use
// lds_cycle (on 16 x 16 grids the cache's registers cost more occupancy than it
// saves).
template <class R, int NT>
__device__ void lds_cycle_whole(const LdsHier<R>& lev, int nlev, int nu1, int nu2, int gamma, bool top_zero,
                                bool coarsen) {
  if constexpr (NT == 256) {
    if (nlev >= 2 && lev.m_top == 32) {
      lds_cycle_top_cached<R, NT, 32, RMG_WS_WAVE_M>(lev, nlev, nu1, nu2, gamma, top_zero, coarsen);
      return;
    }
  }
  lds_cycle<R, NT, false, RMG_WS_WAVE_M>(lev, 0, nlev, nu1, nu2, gamma, top_zero, coarsen);
}

}  // namespace rmg
