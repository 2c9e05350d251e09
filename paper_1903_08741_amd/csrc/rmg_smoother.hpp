// Level-streaming smoother of the batched Picard-multigrid solver (gfx950):
// the down leg (nu1 red-black Gauss-Seidel sweeps fused with the residual and
// its restriction) and the up leg (prolongation of the coarse correction fused
// with nu2 sweeps, and on the finest level the Picard update) of one level, over
// TS x TS output tiles of all samples of a grid size.  Section 4.2: five-point
// cell-centred operator, red-black Gauss-Seidel, R = P^T / 4 with piecewise
// constant P (eq. transfer).
#pragma once

#include "rmg_device.hpp"
#include "rmg_internal.hpp"

namespace rmg {

// Flat traversal of a w x w region of a tile without integer division: for
// k < 2^16 and w < 2^16, floor(k / w) = umulhi(k, ceil(2^32 / w)) exactly (the
// rounding error of the reciprocal, k (ceil(2^32/w) w - 2^32) / (w 2^32) < k / 2^32,
// stays below 1/w).
// (w = 1 has no 32-bit magic number: the table holds 0, which is right only for a
// single-element loop; the loops below use w >= 2 whenever they have several rows.)
// Widths up to kMagicMax come from a table (a 64-bit division per loop would cost
// a software division routine on the scalar unit).
constexpr int kMagicMax = 128;
struct MagicTable {
  unsigned v[kMagicMax + 1];
  constexpr MagicTable() : v() {
    for (int w = 1; w <= kMagicMax; ++w)
      v[w] = (unsigned)((0x100000000ull + (unsigned long long)w - 1ull) / (unsigned long long)w);
  }
};
__constant__ constexpr MagicTable kMagic{};
__device__ __forceinline__ unsigned rmg_magic(int w) {
  if (w >= 1 && w <= kMagicMax) return kMagic.v[w];
  return (unsigned)((0x100000000ull + (unsigned long long)w - 1ull) / (unsigned long long)w);
}
// Sample and tile of this workgroup of a (tiles x samples) launch.  Workgroups are
// handed to the 8 XCDs round-robin by linear id; when the tile count is a multiple of
// 8 the tiles are renumbered so that each XCD receives a contiguous band of every
// sample's tiles and the halos its workgroups share can stay in that XCD's L2.
// (Renumbering whole samples onto one XCD instead measured slower: the 256^2 class
// of the 5-level workload 379 ms against 359 ms, the large-batch smoother 2.78
// against 2.82 TB/s.)
struct SampleTile {
  int64_t s;
  int tile;
};
__device__ __forceinline__ SampleTile xcd_sample_tile() {
  const int g = (int)gridDim.x, x = (int)blockIdx.x;
  SampleTile w;
  w.s = blockIdx.y;
  w.tile = (g & 7) ? x : (x & 7) * (g >> 3) + (x >> 3);
  return w;
}

// ------------------------------------------------------------ streaming smoother
// A down or up kernel works on a TS x TS output tile of one level plus a halo,
// both made of 2 x 2 cell blocks aligned with the coarse grid.  Each thread owns
// whole blocks for the whole kernel and keeps their right-hand side, face
// coefficients, diagonal and iterate in registers; LDS mirrors only the iterate,
// for the neighbours.  A red-black update of a block cell then reads two
// neighbours from LDS (the other two are cells of its own block); the residual
// restriction of a block and the prolongation of its coarse cell need no
// exchange at all.  Per cell the arithmetic is that of st5 / gs_value /
// residual_value, in the same order, so the result equals the whole-level LDS
// path bit for bit.
//
// Cell k = 2 cy + cx of a block: 0 = (0,0) red, 1 = (1,0) black, 2 = (0,1) black,
// 3 = (1,1) red ((i + j) even is red; blocks start at even coordinates).
template <class R>
struct Blk {
  R f[4], d[4], rd[4];  // right-hand side, diagonal, reciprocal of the diagonal (FP32)
  R vx[2][3];           // x-face coefficients of row r at local x = 0, 1, 2
  R vy[2][3];           // y-face coefficients of column c at local y = 0, 1, 2
  R u[4];
};

template <class R> struct Vec2;
template <> struct Vec2<float> { using T = float2; };
template <> struct Vec2<double> { using T = double2; };

// Smoother update of one cell from its neighbour sum (gs_value with d precomputed).
__device__ __forceinline__ float blk_gs(float f, float snb, float d, float rd) { return (f + snb) * rd; }
__device__ __forceinline__ double blk_gs(double f, double snb, double d, double) { return (f + snb) / d; }
template <class R>
__device__ __forceinline__ R blk_snb(R aw, R ae, R as, R an, R uw, R ue, R us, R un) {
  R t1 = aw * uw;
  t1 = t1 + ae * ue;
  R t2 = as * us;
  t2 = t2 + an * un;
  return t1 + t2;
}

// Region of a kernel: BW x BW blocks, the output tile's TS/2 x TS/2 blocks plus hb
// halo blocks on each side.  LDS holds the iterate of the region's cells with a
// ring of zero cells around it (UW = 2 BW + 2 cells per row).
struct BlkRegion {
  int BW, hb, UW;
  int gbx0, gby0;  // coarse (block) coordinates of region block (0, 0)
  int mb;          // blocks per side of the level (m / 2)
};

__device__ __forceinline__ int blk_lds(const BlkRegion& g, int lx, int ly) { return (ly + 1) * g.UW + lx + 1; }

// Raw global values of one block: its two rows of f, C/dt and the west and south
// faces, the east faces of its right column, the south faces of the block above (or
// the top-boundary faces), its iterate and the coarse correction of its coarse cell.
template <class R>
struct BlkRaw {
  using V = typename Vec2<R>::T;
  V f0, f1, t0, t1, w0, w1, s0, s1, n0, u0, u1;
  R e0, e1, uc;
};

// Issue the loads of block (bx, by) of the region, which must lie inside the domain
// (the caller clamps the coordinates of blocks outside it and masks them later).
// Every load is unconditional, so the loads of all of a thread's blocks are in flight
// before the first value is used.
template <class R>
__device__ __forceinline__ void blk_fetch(BlkRaw<R>& r, const BlkRegion& g, int bx, int by, int m, const R* F,
                                          const R* CW, const R* CS, const R* CDT, const R* CTOP, const R* UC,
                                          int mc) {
  using V = typename Vec2<R>::T;
  const int gx = 2 * (g.gbx0 + bx), gy = 2 * (g.gby0 + by);
  const int64_t c0 = (int64_t)gy * m + gx, c2 = c0 + m;
  const bool east = gx + 2 < m, north = gy + 2 < m;
  r.f0 = *(const V*)(F + c0);
  r.f1 = *(const V*)(F + c2);
  r.t0 = *(const V*)(CDT + c0);
  r.t1 = *(const V*)(CDT + c2);
  r.w0 = *(const V*)(CW + c0);
  r.w1 = *(const V*)(CW + c2);
  r.s0 = *(const V*)(CS + c0);
  r.s1 = *(const V*)(CS + c2);
  r.e0 = CW[east ? c0 + 2 : c0];
  r.e1 = CW[east ? c2 + 2 : c2];
  r.e0 = east ? r.e0 : (R)0;
  r.e1 = east ? r.e1 : (R)0;
  r.n0 = *(const V*)(north ? CS + c2 + m : CTOP + gx);
  r.uc = UC ? UC[(int64_t)(g.gby0 + by) * mc + g.gbx0 + bx] : (R)0;
}
template <class R>
__device__ __forceinline__ void blk_fetch_u(BlkRaw<R>& r, const BlkRegion& g, int bx, int by, int m, const R* U) {
  using V = typename Vec2<R>::T;
  const int64_t c0 = (int64_t)(2 * (g.gby0 + by)) * m + 2 * (g.gbx0 + bx);
  r.u0 = *(const V*)(U + c0);
  r.u1 = *(const V*)(U + c0 + m);
}

// Registers of a block from its raw values (u_zero: the iterate is zero; with UC the
// coarse correction is added to it); with cdt_out, also its four C/dt values.
template <class R>
__device__ __forceinline__ void blk_build(Blk<R>& b, const BlkRaw<R>& r, bool u_zero, bool with_uc,
                                          R* cdt_out = nullptr) {
  using V = typename Vec2<R>::T;
  V u0, u1;
  if (u_zero) {
    u0.x = u0.y = u1.x = u1.y = (R)0;
  } else {
    u0 = r.u0;
    u1 = r.u1;
  }
  if (with_uc) {
    u0.x = u0.x + r.uc;
    u0.y = u0.y + r.uc;
    u1.x = u1.x + r.uc;
    u1.y = u1.y + r.uc;
  }
  b.f[0] = r.f0.x; b.f[1] = r.f0.y; b.f[2] = r.f1.x; b.f[3] = r.f1.y;
  b.u[0] = u0.x; b.u[1] = u0.y; b.u[2] = u1.x; b.u[3] = u1.y;
  b.vx[0][0] = r.w0.x; b.vx[0][1] = r.w0.y; b.vx[0][2] = r.e0;
  b.vx[1][0] = r.w1.x; b.vx[1][1] = r.w1.y; b.vx[1][2] = r.e1;
  b.vy[0][0] = r.s0.x; b.vy[0][1] = r.s1.x; b.vy[0][2] = r.n0.x;
  b.vy[1][0] = r.s0.y; b.vy[1][1] = r.s1.y; b.vy[1][2] = r.n0.y;
  const R cdt[4] = {r.t0.x, r.t0.y, r.t1.x, r.t1.y};
  if (cdt_out)
    for (int k = 0; k < 4; ++k) cdt_out[k] = cdt[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cx = k & 1, cy = k >> 1;
    R d = cdt[k];
    d = d + b.vx[cy][cx];
    d = d + b.vx[cy][cx + 1];
    d = d + b.vy[cx][cy];
    d = d + b.vy[cx][cy + 1];
    b.d[k] = d;
    b.rd[k] = sizeof(R) == 4 ? (R)__builtin_amdgcn_rcpf((float)d) : (R)0;
  }
}

// Neighbour sums of the four cells of block (bx, by) from the current iterate.
template <class R>
__device__ __forceinline__ R blk_cell_snb(const Blk<R>& b, const BlkRegion& g, const RMG_LDS R* L, int bx, int by,
                                          int k) {
  const int cx = k & 1, cy = k >> 1;
  const int lx = 2 * bx + cx, ly = 2 * by + cy;
  const R uw = cx ? b.u[k - 1] : L[blk_lds(g, lx - 1, ly)];
  const R ue = cx ? L[blk_lds(g, lx + 1, ly)] : b.u[k + 1];
  const R us = cy ? b.u[k - 2] : L[blk_lds(g, lx, ly - 1)];
  const R un = cy ? L[blk_lds(g, lx, ly + 1)] : b.u[k + 2];
  return blk_snb<R>(b.vx[cy][cx], b.vx[cy][cx + 1], b.vy[cx][cy], b.vy[cx][cy + 1], uw, ue, us, un);
}

// One colour of a red-black sweep over the thread's blocks (cells 0, 3 or 1, 2).
template <class R, int NB, int COLOUR>
__device__ __forceinline__ void blk_half_sweep(Blk<R> (&b)[NB], const bool (&live)[NB], const int (&bx)[NB],
                                               const int (&by)[NB], const BlkRegion& g, RMG_LDS R* L) {
  constexpr int ka = COLOUR ? 1 : 0, kb = COLOUR ? 2 : 3;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (!live[q]) continue;
    const R sa = blk_cell_snb(b[q], g, L, bx[q], by[q], ka);
    const R sb = blk_cell_snb(b[q], g, L, bx[q], by[q], kb);
    b[q].u[ka] = blk_gs(b[q].f[ka], sa, b[q].d[ka], b[q].rd[ka]);
    b[q].u[kb] = blk_gs(b[q].f[kb], sb, b[q].d[kb], b[q].rd[kb]);
    L[blk_lds(g, 2 * bx[q] + (ka & 1), 2 * by[q] + (ka >> 1))] = b[q].u[ka];
    L[blk_lds(g, 2 * bx[q] + (kb & 1), 2 * by[q] + (kb >> 1))] = b[q].u[kb];
  }
}

// Common set-up: the thread's blocks, their registers, the LDS iterate (zero outside
// the domain and on the ring).  The loads of all of the thread's blocks are issued
// first (a block outside the domain or the region loads a clamped in-domain block and
// is masked), the LDS ring is cleared while they are in flight.  Returns after the
// barrier that publishes the iterate.
template <class R, int TS, int NB>
__device__ __forceinline__ void blk_setup(Blk<R> (&b)[NB], bool (&live)[NB], bool (&own)[NB], int (&bx)[NB],
                                          int (&by)[NB], BlkRegion& g, RMG_LDS R* L, int hb, unsigned mg, int m,
                                          int x0, int y0, const R* F, const R* CW, const R* CS, const R* CDT,
                                          const R* CTOP, const R* U, const R* UC, int mc, bool u_zero) {
  g.hb = hb;
  g.BW = TS / 2 + 2 * hb;
  g.UW = 2 * g.BW + 2;
  g.gbx0 = x0 / 2 - hb;
  g.gby0 = y0 / 2 - hb;
  g.mb = m / 2;
  const int nblk = g.BW * g.BW;
  const int t = (int)threadIdx.x;
  BlkRaw<R> raw[NB];
  int cbx[NB], cby[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    // a thread slot beyond the region takes the region's last block (its loads then
    // hit lines the region fetches anyway) and stays masked
    const int k = t + q * kBlock, kk = min(k, nblk - 1);
    by[q] = (int)__umulhi((unsigned)kk, mg);
    bx[q] = kk - by[q] * g.BW;
    const int gbx = g.gbx0 + bx[q], gby = g.gby0 + by[q];
    live[q] = k < nblk && gbx >= 0 && gbx < g.mb && gby >= 0 && gby < g.mb;
    own[q] = live[q] && bx[q] >= hb && bx[q] < hb + TS / 2 && by[q] >= hb && by[q] < hb + TS / 2;
    cbx[q] = min(max(gbx, 0), g.mb - 1) - g.gbx0;
    cby[q] = min(max(gby, 0), g.mb - 1) - g.gby0;
    blk_fetch(raw[q], g, cbx[q], cby[q], m, F, CW, CS, CDT, CTOP, UC, mc);
  }
  if (!u_zero) {
#pragma unroll
    for (int q = 0; q < NB; ++q) blk_fetch_u(raw[q], g, cbx[q], cby[q], m, U);
  }
  const int W2 = 2 * g.BW;
  for (int e = t; e < 4 * (W2 + 1); e += kBlock) {
    const int side = e / (W2 + 1), i = e - side * (W2 + 1);
    int lx, ly;
    if (side == 0) { lx = i - 1; ly = -1; }        // bottom ring row, from the corner
    else if (side == 1) { lx = i; ly = W2; }       // top ring row
    else if (side == 2) { lx = -1; ly = i; }       // left ring column
    else { lx = W2; ly = i - 1; }                  // right ring column
    L[blk_lds(g, lx, ly)] = (R)0;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) blk_build(b[q], raw[q], u_zero, UC != nullptr);
  // LDS iterate: every block of the region (zero outside the domain)
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (t + q * kBlock >= nblk) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      L[blk_lds(g, 2 * bx[q] + (k & 1), 2 * by[q] + (k >> 1))] = live[q] ? b[q].u[k] : (R)0;
  }
  __syncthreads();
}

// Region width of a kernel's tiles: its magic number for the block enumeration.
inline unsigned blk_magic_host(int ts, int hb) {
  const unsigned long long w = (unsigned long long)(ts / 2 + 2 * hb);
  return (unsigned)((0x100000000ull + w - 1ull) / w);
}

// The prologue's uniform values in scalar registers before the sample's state is
// read: the compiler then issues every argument load in one batch instead of
// interleaving them with the dependent loads that follow.
__device__ __forceinline__ void sgpr_ready(const void* p) { asm volatile("" ::"s"(p)); }
__device__ __forceinline__ void sgpr_ready(int v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void sgpr_ready(unsigned v) { asm volatile("" ::"s"(v)); }
template <class... T>
__device__ __forceinline__ void sgpr_ready_all(const T&... v) {
  (sgpr_ready(v), ...);
}

constexpr int blk_nb(int ts, int hb) {
  return ((ts / 2 + 2 * hb) * (ts / 2 + 2 * hb) + kBlock - 1) / kBlock;
}
template <class R>
constexpr size_t blk_lds_bytes(int ts, int hb) {
  return sizeof(R) * (size_t)(2 * (ts / 2 + 2 * hb) + 2) * (size_t)(2 * (ts / 2 + 2 * hb) + 2);
}

// Down leg on a streaming level l: nu1 red-black sweeps, residual, restriction.
// Halo: nu1 + 1 blocks (2 nu1 + 2 >= 2 nu1 + 1 cells: the residual of a tile cell
// depends on data up to 2 nu1 + 1 cells away).
// slot: kUniform, or the cycle slot of the pass (the finest level's u_zero then follows
// from the sample's state: zero on the first cycle of its Picard iteration).
template <class R, int TS, int NB>
__global__ __launch_bounds__(kBlock) void k_down(SolveArgs a, StreamPlan pl, LegArgs lg, int u_zero_, int slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = lg.m, mc = m >> 1;
  const int64_t M2 = (int64_t)m * m, MC2 = (int64_t)mc * mc;
  sgpr_ready_all((int)gridDim.x, (const void*)pl.state, lg.f, lg.cw, lg.cs, lg.cdt, lg.ctop, lg.uin, lg.uout, lg.fc, m, lg.hb, lg.lgntx, lg.mg, lg.l,
                 u_zero_, slot, (const void*)pl.tcells);
  const SampleTile w = xcd_sample_tile();
  const int64_t s = w.s;
  const SampleState sst = slot_fields(pl.state + s);
  if (!slot_runs(sst, slot)) return;
  const int u_zero = lg.l == 0 ? (int)slot_first(sst, slot, u_zero_) : u_zero_;
  // timed launches count the cells they process: once per active sample (one
  // counter update per workgroup would serialise thousands of atomics on one address)
  if (pl.tcells && w.tile == 0 && threadIdx.x == 0)
    atomicAdd(pl.tcells + (u_zero ? 0 : 1), (unsigned long long)m * (unsigned long long)m);
  const int tile = w.tile;
  const int x0 = (tile & ((1 << lg.lgntx) - 1)) * TS, y0 = (tile >> lg.lgntx) * TS;
  RMG_LDS R* L = (RMG_LDS R*)smem;
  Blk<R> b[NB];
  bool live[NB], own[NB];
  int bx[NB], by[NB];
  BlkRegion g;
  blk_setup<R, TS, NB>(b, live, own, bx, by, g, L, lg.hb, lg.mg, m, x0, y0, (const R*)lg.f + s * M2,
                       (const R*)lg.cw + s * M2, (const R*)lg.cs + s * M2, (const R*)lg.cdt + s * M2,
                       (const R*)lg.ctop + s * m, (const R*)lg.uin + s * M2, nullptr, mc, u_zero != 0);
  for (int st = 0; st < 2 * a.nu1; ++st) {
    if (st & 1)
      blk_half_sweep<R, NB, 1>(b, live, bx, by, g, L);
    else
      blk_half_sweep<R, NB, 0>(b, live, bx, by, g, L);
    __syncthreads();
  }
  using V = typename Vec2<R>::T;
  R* U = (R*)lg.uout + s * M2;
  R* FC = (R*)lg.fc + s * MC2;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (!own[q]) continue;
    R r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const R snb = blk_cell_snb(b[q], g, L, bx[q], by[q], k);
      r[k] = (b[q].f[k] + snb) - b[q].d[k] * b[q].u[k];
    }
    const int gbx = g.gbx0 + bx[q], gby = g.gby0 + by[q];
    FC[(int64_t)gby * mc + gbx] = restrict4<R>(r[0], r[1], r[2], r[3]);
    const int64_t c0 = (int64_t)(2 * gby) * m + 2 * gbx;
    V o0, o1;
    o0.x = b[q].u[0];
    o0.y = b[q].u[1];
    o1.x = b[q].u[2];
    o1.y = b[q].u[3];
    *(V*)(U + c0) = o0;
    *(V*)(U + c0 + m) = o1;
  }
}

// Up leg on a streaming level l: prolongation of level l+1 (one coarse value per
// block), nu2 sweeps; on the finest level (final != 0) the Picard update p += dp
// and ||dp||_inf instead of a store.  Halo: nu2 blocks (2 nu2 cells).
// slot as for k_down: on the finest level the Picard update follows the sample's last cycle.
template <class R, int TS, int NB>
__global__ __launch_bounds__(kBlock) void k_up(SolveArgs a, StreamPlan pl, LegArgs lg, int final__, int slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kBlock / 64];
  const int m = lg.m, mc = m >> 1;
  const int64_t M2 = (int64_t)m * m, MC2 = (int64_t)mc * mc;
  sgpr_ready_all((int)gridDim.x, (const void*)pl.state, lg.f, lg.cw, lg.cs, lg.cdt, lg.ctop, lg.uin, lg.uout, lg.uc, m, lg.hb, lg.lgntx, lg.mg, lg.l,
                 final__, slot);
  const SampleTile w = xcd_sample_tile();
  const int64_t s = w.s;
  const SampleState sst = slot_fields(pl.state + s);
  if (!slot_runs(sst, slot)) return;
  const int final_ = lg.l == 0 ? (int)slot_last(sst, slot, final__) : final__;
  const int tile = w.tile;
  const int x0 = (tile & ((1 << lg.lgntx) - 1)) * TS, y0 = (tile >> lg.lgntx) * TS;
  RMG_LDS R* L = (RMG_LDS R*)smem;
  Blk<R> b[NB];
  bool live[NB], own[NB];
  int bx[NB], by[NB];
  BlkRegion g;
  blk_setup<R, TS, NB>(b, live, own, bx, by, g, L, lg.hb, lg.mg, m, x0, y0, (const R*)lg.f + s * M2,
                       (const R*)lg.cw + s * M2, (const R*)lg.cs + s * M2, (const R*)lg.cdt + s * M2,
                       (const R*)lg.ctop + s * m, (const R*)lg.uin + s * M2, (const R*)lg.uc + s * MC2, mc,
                       false);
  // the Picard update's FP64 head values are loaded before the sweeps, which hide
  // their latency
  double* p = a.p + s * M2;
  double2 pv[NB][2];
  if (final_) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!own[q]) continue;
      const int64_t c0 = (int64_t)(2 * (g.gby0 + by[q])) * m + 2 * (g.gbx0 + bx[q]);
      pv[q][0] = *(const double2*)(p + c0);
      pv[q][1] = *(const double2*)(p + c0 + m);
    }
  }
  for (int st = 0; st < 2 * a.nu2; ++st) {
    if (st & 1)
      blk_half_sweep<R, NB, 1>(b, live, bx, by, g, L);
    else
      blk_half_sweep<R, NB, 0>(b, live, bx, by, g, L);
    __syncthreads();
  }
  if (!final_) {
    using V = typename Vec2<R>::T;
    R* U = (R*)lg.uout + s * M2;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!own[q]) continue;
      const int64_t c0 = (int64_t)(2 * (g.gby0 + by[q])) * m + 2 * (g.gbx0 + bx[q]);
      V o0, o1;
      o0.x = b[q].u[0];
      o0.y = b[q].u[1];
      o1.x = b[q].u[2];
      o1.y = b[q].u[3];
      *(V*)(U + c0) = o0;
      *(V*)(U + c0 + m) = o1;
    }
    return;
  }
  double mx = 0.0, bad = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (!own[q]) continue;
    const int64_t c0 = (int64_t)(2 * (g.gby0 + by[q])) * m + 2 * (g.gbx0 + bx[q]);
    const double2 p0 = pv[q][0], p1 = pv[q][1];
    const double d0 = (double)b[q].u[0], d1 = (double)b[q].u[1], d2 = (double)b[q].u[2], d3 = (double)b[q].u[3];
    double2 o0, o1;
    o0.x = p0.x + d0;
    o0.y = p0.y + d1;
    o1.x = p1.x + d2;
    o1.y = p1.y + d3;
    *(double2*)(p + c0) = o0;
    *(double2*)(p + c0 + m) = o1;
    mx = fmax(fmax(mx, fabs(d0)), fmax(fabs(d1), fmax(fabs(d2), fabs(d3))));
    if (!isfinite(d0) || !isfinite(d1) || !isfinite(d2) || !isfinite(d3)) bad = 1.0;
  }
  mx = block_max<kBlock>(mx, red);
  bad = block_max<kBlock>(bad, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(pl.dpmax + s, mx);
    if (bad > 0.0) atomicOr(&pl.state[s].nanflag, 1);
  }
}

// Up leg of cycle slot `slot` fused with the down leg of slot + 1 on the finest level
// (the two are adjacent when a Picard iteration runs several cycles): prolongation
// of level 1, nu2 sweeps, then - for a sample whose iteration continues - nu1 sweeps
// of the next cycle, its residual and restriction, in one launch.  The halo is nu1 +
// nu2 + 1 blocks, so the owned cells see exactly the values the two separate
// kernels would compute (bit-identical results).  Input: lv.u[0] (the correction
// the down leg of slot wrote) and level 1's correction; output: the continuing
// samples' corrections in lv.ub[0] (the next up leg reads them there) and level 1's
// right-hand side; a sample whose iteration ends in slot applies the Picard update
// instead, as k_up does.
template <class R, int TS, int NB>
__global__ __launch_bounds__(kBlock) void k_up_down(SolveArgs a, StreamPlan pl, LegArgs lg, int slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kBlock / 64];
  const int m = lg.m, mc = m >> 1;
  const int64_t M2 = (int64_t)m * m, MC2 = (int64_t)mc * mc;
  sgpr_ready_all((int)gridDim.x, (const void*)pl.state, lg.f, lg.cw, lg.cs, lg.cdt, lg.ctop, lg.uin, lg.uout, lg.fc, lg.uc, m, lg.hb, lg.lgntx, lg.mg,
                 slot);
  const SampleTile w = xcd_sample_tile();
  const int64_t s = w.s;
  const SampleState sst = slot_fields(pl.state + s);
  if (!slot_runs(sst, slot)) return;
  const bool final_ = slot_last(sst, slot, 0);
  const int tile = w.tile;
  const int x0 = (tile & ((1 << lg.lgntx) - 1)) * TS, y0 = (tile >> lg.lgntx) * TS;
  RMG_LDS R* L = (RMG_LDS R*)smem;
  Blk<R> b[NB];
  bool live[NB], own[NB];
  int bx[NB], by[NB];
  BlkRegion g;
  blk_setup<R, TS, NB>(b, live, own, bx, by, g, L, lg.hb, lg.mg, m, x0, y0, (const R*)lg.f + s * M2,
                       (const R*)lg.cw + s * M2, (const R*)lg.cs + s * M2, (const R*)lg.cdt + s * M2,
                       (const R*)lg.ctop + s * m, (const R*)lg.uin + s * M2, (const R*)lg.uc + s * MC2, mc,
                       false);
  double* p = a.p + s * M2;
  double2 pv[NB][2];
  if (final_) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!own[q]) continue;
      const int64_t c0 = (int64_t)(2 * (g.gby0 + by[q])) * m + 2 * (g.gbx0 + bx[q]);
      pv[q][0] = *(const double2*)(p + c0);
      pv[q][1] = *(const double2*)(p + c0 + m);
    }
  }
  const int nsweep = 2 * a.nu2 + (final_ ? 0 : 2 * a.nu1);
  for (int st = 0; st < nsweep; ++st) {
    // the up leg's sweeps, then the down leg's: both start with a red half-sweep
    const int colour = st < 2 * a.nu2 ? (st & 1) : ((st - 2 * a.nu2) & 1);
    if (colour)
      blk_half_sweep<R, NB, 1>(b, live, bx, by, g, L);
    else
      blk_half_sweep<R, NB, 0>(b, live, bx, by, g, L);
    __syncthreads();
  }
  using V = typename Vec2<R>::T;
  if (!final_) {
    R* U = (R*)lg.uout + s * M2;
    R* FC = (R*)lg.fc + s * MC2;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (!own[q]) continue;
      R r[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const R snb = blk_cell_snb(b[q], g, L, bx[q], by[q], k);
        r[k] = (b[q].f[k] + snb) - b[q].d[k] * b[q].u[k];
      }
      const int gbx = g.gbx0 + bx[q], gby = g.gby0 + by[q];
      FC[(int64_t)gby * mc + gbx] = restrict4<R>(r[0], r[1], r[2], r[3]);
      const int64_t c0 = (int64_t)(2 * gby) * m + 2 * gbx;
      V o0, o1;
      o0.x = b[q].u[0];
      o0.y = b[q].u[1];
      o1.x = b[q].u[2];
      o1.y = b[q].u[3];
      *(V*)(U + c0) = o0;
      *(V*)(U + c0 + m) = o1;
    }
    return;
  }
  double mx = 0.0, bad = 0.0;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (!own[q]) continue;
    const int64_t c0 = (int64_t)(2 * (g.gby0 + by[q])) * m + 2 * (g.gbx0 + bx[q]);
    const double2 p0 = pv[q][0], p1 = pv[q][1];
    const double d0 = (double)b[q].u[0], d1 = (double)b[q].u[1], d2 = (double)b[q].u[2], d3 = (double)b[q].u[3];
    double2 o0, o1;
    o0.x = p0.x + d0;
    o0.y = p0.y + d1;
    o1.x = p1.x + d2;
    o1.y = p1.y + d3;
    *(double2*)(p + c0) = o0;
    *(double2*)(p + c0 + m) = o1;
    mx = fmax(fmax(mx, fabs(d0)), fmax(fabs(d1), fmax(fabs(d2), fabs(d3))));
    if (!isfinite(d0) || !isfinite(d1) || !isfinite(d2) || !isfinite(d3)) bad = 1.0;
  }
  mx = block_max<kBlock>(mx, red);
  bad = block_max<kBlock>(bad, red);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(pl.dpmax + s, mx);
    if (bad > 0.0) atomicOr(&pl.state[s].nanflag, 1);
  }
}

}  // namespace rmg
