// Red-black Newton-Gauss-Seidel relaxation (Sec. II.A.2, Eq. 17) and the fused defect +
// restriction of the FAS cycle (Sec. II.A.3, Eq. 18 and R), FP64, on colour-split meshes.
//
// Data: every field is colour-split ([c][i][j][m], m = k >> 1; see mr_device.h), so a
// half-sweep streams exactly one colour: it reads the other colour's face neighbours and its own
// colour's edge neighbours (old values, snapshot semantics) and writes the new values of its
// colour to a separate buffer (never in place). HBM traffic per half-sweep and cell of the
// colour: 16 B of theta in, 8 B delta in (+ 8 B of FAS right-hand side on coarse meshes), 8 B out.
//
// Work decomposition ("2.5D"): a block owns a TJ x TM tile of (j, m) and marches along i over a
// chunk of planes. Both colours of planes i-1, i, i+1 (tile plus a one-cell periodic halo) sit in
// a 4-slot LDS ring; while plane i is computed from LDS, plane i+2 is prefetched into registers
// and stored into the free slot afterwards, so each plane step needs a single barrier and every
// theta value is read from HBM about once per launch. Every thread updates exactly one cell per
// plane (perfect balance); the block's tiles are mapped so that each XCD walks a contiguous
// range of tiles and shares halos in its own L2.
#include <algorithm>
#include <type_traits>
#include <map>
#include <tuple>
#include <mutex>
#include <utility>
#include <vector>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"
#include "tuning.h"

namespace mr {

constexpr int kMaxPrefetch = 8;

// LDS ring of both colours of theta for a TJ x TM tile plus halo, 4 plane slots.
template <int TM>
struct PlaneRing {
  double* lds;
  int tj;
  // value of colour c, plane p, halo-tile row r in [0, tj+2), column s in [0, TM+2)
  __device__ __forceinline__ double at(int c, int p, int r, int s) const {
    return lds[((c * 4 + (p & 3)) * (tj + 2) + r) * (TM + 2) + s];
  }
};

// Per-thread element list of the plane loader: global offset inside a plane (both colours) and
// LDS offset inside a slot. Computed once per block.
template <int TM>
struct PlaneLoader {
  unsigned goff[kMaxPrefetch];
  int loff[kMaxPrefetch];
  int count;
  __device__ void init(int tid, int nthreads, int tj, int j0, int m0, int n) {
    const int nh = n >> 1;
    const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
    const int per_colour = (tj + 2) * (TM + 2);
    const int total = 2 * per_colour;
    count = 0;
#pragma unroll
    for (int t = 0; t < kMaxPrefetch; ++t) {
      const int e = tid + t * nthreads;
      goff[t] = 0;
      loff[t] = 0;
      if (e < total) {
        const int c = e / per_colour;
        const int rem = e - c * per_colour;
        const int r = rem / (TM + 2);
        const int s = rem - r * (TM + 2);
        const int gj = wrapi(j0 - 1 + r, n), gm = wrapi(m0 - 1 + s, nh);
        goff[t] = c * half + (unsigned)gj * nh + gm;
        loff[t] = (c * 4 * (tj + 2) + r) * (TM + 2) + s;   // slot offset added at store time
        count = t + 1;
      }
    }
  }
  __device__ __forceinline__ void store(double* lds, int tj, int p, const double (&v)[kMaxPrefetch]) const {
    const int slot_off = (p & 3) * (tj + 2) * (TM + 2);
#pragma unroll
    for (int t = 0; t < kMaxPrefetch; ++t)
      if (t < count) lds[loff[t] + slot_off] = v[t];
  }
};

// Gather the 18 neighbours of the colour-c cell at tile position (r, s) of plane i from the ring.
template <int TM>
__device__ __forceinline__ void ring_gather(const PlaneRing<TM>& R, int c, int i, int q, int r, int s, Nb18& t) {
  const int o = 1 - c;
  const int sp = s + q, sm = s + q - 1;   // columns of k+1 and k-1
  t.xm = R.at(o, i - 1, r, s); t.xp = R.at(o, i + 1, r, s);
  t.ym = R.at(o, i, r - 1, s); t.yp = R.at(o, i, r + 1, s);
  t.zm = R.at(o, i, r, sm);    t.zp = R.at(o, i, r, sp);
  t.xpyp = R.at(c, i + 1, r + 1, s); t.xmym = R.at(c, i - 1, r - 1, s);
  t.xpym = R.at(c, i + 1, r - 1, s); t.xmyp = R.at(c, i - 1, r + 1, s);
  t.xpzp = R.at(c, i + 1, r, sp);    t.xmzm = R.at(c, i - 1, r, sm);
  t.xpzm = R.at(c, i + 1, r, sm);    t.xmzp = R.at(c, i - 1, r, sp);
  t.ypzp = R.at(c, i, r + 1, sp);    t.ymzm = R.at(c, i, r - 1, sm);
  t.ypzm = R.at(c, i, r + 1, sm);    t.ymzp = R.at(c, i, r - 1, sp);
}

__device__ __forceinline__ void tile_coords(int nblocks, int tiles_m, int tiles_j, int tj, int tm, int ci,
                                            int& j0, int& m0, int& i0) {
  const int logical = xcd_remap(blockIdx.x, nblocks);
  const int tm_i = logical % tiles_m;
  const int tj_i = (logical / tiles_m) % tiles_j;
  const int chunk = logical / (tiles_m * tiles_j);
  j0 = tj_i * tj;
  m0 = tm_i * tm;
  i0 = chunk * ci;
}

// Fetch plane p of both colours into registers. th holds both colours; if red_new is given the
// red colour is taken from it instead (the black half-sweep reads the new red values).
template <int TM>
__device__ __forceinline__ void fetch_plane(const PlaneLoader<TM>& ld, const double* __restrict__ th,
                                            const double* __restrict__ red_new, int p, int n,
                                            double (&v)[kMaxPrefetch]) {
  const unsigned plane = (unsigned)n * (unsigned)(n >> 1);
  const unsigned half = plane * (unsigned)n;
  const unsigned base = (unsigned)wrapi(p, n) * plane;
#pragma unroll
  for (int t = 0; t < kMaxPrefetch; ++t) {
    if (t < ld.count) {
      const unsigned g = ld.goff[t];
      const double* src = (red_new != nullptr && g < half) ? red_new : th;
      v[t] = src[base + g];
    }
  }
}

// ---- half-sweep (compile-time tile) --------------------------------------------------------
// Tile TM columns x TJ rows, NT = TM * TJ / CPT threads; each thread updates CPT cells per plane
// (rows r, r + TJ/CPT, ...), which gives independent dependency chains to interleave. The plane
// loader is branch-free: NPF elements per thread, out-of-range elements clamped onto the last
// element (duplicate stores of the same value). The colour-0 and colour-1 sources are separate
// pointers so the black half-sweep reads the new red values without a per-element select.
template <int TM, int TJ, int CPT>
__global__ void __launch_bounds__(TM * TJ / CPT) half_sweep_tiled(HalfSweepArgs a) {
  constexpr int NT = TM * TJ / CPT;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;                 // one colour, one plane
  constexpr int TOTAL = 2 * SLOT;               // both colours of one plane
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  constexpr int ROWSTEP = TJ / CPT;
  __shared__ double lds[2 * 4 * SLOT];
  const int n = a.n, nh = n >> 1, c = a.colour;
  const int tid = threadIdx.x;
  int j0, m0, i0;
  tile_coords(gridDim.x, a.tiles_m, a.tiles_j, TJ, TM, a.ci, j0, m0, i0);
  const int i1 = i0 + a.ci;
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
  const double* __restrict__ src0 = a.th_red_new ? a.th_red_new : a.th_in;   // colour 0 values
  const double* __restrict__ src1 = a.th_in + half;                          // colour 1 values

  // loader element table
  unsigned goff[NPF];
  int loff[NPF];
  bool col1[NPF];
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    int e = tid + t * NT;
    e = e < TOTAL ? e : TOTAL - 1;
    const int cc = e / SLOT;
    const int rem = e - cc * SLOT;
    const int r = rem / RW;
    const int s = rem - r * RW;
    goff[t] = (unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + s, nh);
    loff[t] = cc * 4 * SLOT + rem;
    col1[t] = cc != 0;
  }
  auto fetch = [&](int p, double (&v)[NPF]) {
    const unsigned base = (unsigned)wrapi(p, n) * plane;
#pragma unroll
    for (int t = 0; t < NPF; ++t) v[t] = (col1[t] ? src1 : src0)[base + goff[t]];
  };
  auto store = [&](int p, const double (&v)[NPF]) {
    const int so = (p & 3) * SLOT;
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[loff[t] + so] = v[t];
  };
  auto L = [&](int cc, int p, int r, int s) -> double { return lds[(cc * 4 + (p & 3)) * SLOT + r * RW + s]; };

  double v[NPF];
  {
    // prologue: all three planes in flight before the first store
    double va[NPF], vb[NPF];
    fetch(i0 - 1, va);
    fetch(i0, vb);
    fetch(i0 + 1, v);
    store(i0 - 1, va);
    store(i0, vb);
    store(i0 + 1, v);
  }
  __syncthreads();

  const int s = tid % TM, r0 = tid / TM;
  const int m = m0 + s;
  const double C = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const double h2 = a.h2, ih2 = a.ih2;
  const double* __restrict__ dl = a.delta + c * half;
  const double* __restrict__ ff = a.f ? a.f + c * half : nullptr;
  double* __restrict__ out = a.th_out + c * half;
  const int o = 1 - c;
  double acc = 0.0;

  for (int i = i0; i < i1; ++i) {
    const bool pre = (i + 2 <= i1);
    if (pre) fetch(i + 2, v);
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int r = r0 + u * ROWSTEP;
      const int j = j0 + r;
      const int q = (i + j + c) & 1;
      const int R = r + 1, S = s + 1, sp = S + q, sm = S + q - 1;
      Nb18 t;
      t.xm = L(o, i - 1, R, S); t.xp = L(o, i + 1, R, S);
      t.ym = L(o, i, R - 1, S); t.yp = L(o, i, R + 1, S);
      t.zm = L(o, i, R, sm);    t.zp = L(o, i, R, sp);
      t.xpyp = L(c, i + 1, R + 1, S); t.xmym = L(c, i - 1, R - 1, S);
      t.xpym = L(c, i + 1, R - 1, S); t.xmyp = L(c, i - 1, R + 1, S);
      t.xpzp = L(c, i + 1, R, sp);    t.xmzm = L(c, i - 1, R, sm);
      t.xpzm = L(c, i + 1, R, sm);    t.xmzp = L(c, i - 1, R, sp);
      t.ypzp = L(c, i, R + 1, sp);    t.ymzm = L(c, i, R - 1, sm);
      t.ypzm = L(c, i, R + 1, sm);    t.ymzp = L(c, i, R - 1, sp);
      const unsigned e = (unsigned)i * plane + (unsigned)j * nh + m;
      const double fc = ff ? ff[e] : 0.0;
      double Ssum;
      const double sig = sigma_cell(t, 1.0 + dl[e], ih2, Ssum);
      const bool keep = a.row_filter != 0 && (4 + 2 * (i & 1) + (j & 1)) != a.row_filter;
      out[e] = keep ? L(c, i, R, S) : (Ssum - h2 * (sig + fc - C)) * (1.0 / 6.0);
      acc += sig + fc;
    }
    if (pre) store(i + 2, v);
    __syncthreads();
  }

  double vv[1] = {acc};
  const bool last = grid_sum<1>(vv, a.partials, a.counter, a.sum_out, gridDim.x, blockIdx.x);
  if (last && tid == 0 && a.copy_to) *a.copy_to = *a.copy_from;
}

// ---- pipelined half-sweep ------------------------------------------------------------------
// The same decomposition and arithmetic as half_sweep_tiled with one cell per thread, for the
// large tiles of the fine meshes. The colour and the presence of f are compile-time, and the plane
// loop is unrolled by the ring length (4) with slots taken relative to the chunk, so every LDS
// access is a per-thread base plus an immediate. Old planes are fetched into registers two steps
// before they enter LDS and delta / f two steps before use (rotating register sets), and every
// memory operation of the loop body is unconditional (clamped plane indices), so the loads of
// later steps stay in flight across the barrier. Requires ci % 4 == 0.
template <int TM, int TJ, int COL, bool HAS_F>
__global__ void __launch_bounds__(TM * TJ) half_sweep_pipe(HalfSweepArgs a) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int O = 1 - COL;
  __shared__ double lds[2 * 4 * SLOT];
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  int j0, m0, i0;
  tile_coords(gridDim.x, a.tiles_m, a.tiles_j, TJ, TM, a.ci, j0, m0, i0);
  const int ci = a.ci;
  const size_t plane = (size_t)n * nh;
  const size_t half = plane * n;
  const unsigned pbytes = (unsigned)plane * 8u;
  const double* __restrict__ src0 = COL == 1 ? a.th_red_new : a.th_in;   // colour 0 values
  const double* __restrict__ src1 = a.th_in + half;                      // colour 1 values
  // every global access goes through a buffer resource of one plane (uniform) and a per-lane
  // byte offset inside it
  auto prs = [&](const double* arr, int p) { return plane_rsrc(arr + (size_t)p * plane, pbytes); };

  // loader: element t of a thread is e = tid + t NT of the two slots laid end to end, colour 0
  // over e < SLOTP and colour 1 from SLOTP on, where SLOTP is SLOT rounded up to whole waves, so
  // that the colour of an element is the same on every lane of a wave and the buffer resource is
  // chosen in scalar registers (a per-lane choice of resource makes the compiler loop over the
  // distinct resources, one load at a time). Out-of-range elements are clamped onto the last one
  // of their colour (duplicate stores of the same value).
  static_assert(NT % 64 == 0, "whole waves per block");
  constexpr int SLOTP = (SLOT + 63) / 64 * 64;
  constexpr int NPF = (SLOTP + SLOT + NT - 1) / NT;
  const int wave0 = __builtin_amdgcn_readfirstlane(tid) & ~63;   // first thread of this wave
  unsigned gb[NPF];
  int le[NPF];
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    const int cc = wave0 + t * NT >= SLOTP ? 1 : 0;
    int rem = tid + t * NT - cc * SLOTP;
    rem = rem < SLOT ? rem : SLOT - 1;
    const int r = rem / RW;
    const int c = rem - r * RW;
    gb[t] = ((unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh)) * 8u;
    le[t] = cc * 4 * SLOT + rem;
  }
  // plane i0 - 1 + rel sits in slot rel & 3
  auto fetch = [&](int rel, double (&v)[NPF]) {
    const int p = wrapi(i0 - 1 + rel, n);
    const auto b0 = prs(src0, p), b1 = prs(src1, p);
#pragma unroll
    for (int t = 0; t < NPF; ++t) v[t] = ld_rs(wave0 + t * NT >= SLOTP ? b1 : b0, gb[t]);
  };
  auto store = [&](int slot, const double (&v)[NPF]) {
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[le[t] + slot * SLOT] = v[t];
  };

  const int s = tid % TM, r = tid / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned o_c = ((unsigned)j * nh + m) * 8u;      // own cell inside a plane (bytes)
  const int ob = (r + 1) * RW + (s + 1);                 // own cell inside a slot
  const int q0 = (i0 + j + COL) & 1;                     // z-parity at even t
  const int oq0 = ob + q0, oq1 = ob + (q0 ^ 1);
  const double C = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const double h2 = a.h2, ih2 = a.ih2;
  const double* __restrict__ dl = a.delta + COL * half;
  const double* __restrict__ ff = HAS_F ? a.f + COL * half : nullptr;
  double* __restrict__ out = a.th_out + COL * half;
  const int last_plane = n - 1;
  double acc = 0.0;

  double V0[NPF], V1[NPF];
  double D[4], Fv[4];
  {
    double va[NPF], vb[NPF], vc[NPF];
    fetch(0, va);
    fetch(1, vb);
    fetch(2, vc);
    store(0, va);
    store(1, vb);
    store(2, vc);
  }
  fetch(3, V0);
  D[0] = ld_rs_nt(prs(dl, i0), o_c);
  D[1] = ld_rs_nt(prs(dl, min(i0 + 1, last_plane)), o_c);
  if (HAS_F) {
    Fv[0] = ld_rs(prs(ff, i0), o_c);
    Fv[1] = ld_rs(prs(ff, min(i0 + 1, last_plane)), o_c);
  }
  __syncthreads();

  // step t (K = t & 3): plane i = i0 + t (rel t + 1); LDS holds rel t, t+1, t+2
  auto step = [&](auto kc, int t, double (&vst)[NPF], double (&vft)[NPF]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = (K + 0) & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    const int pn = min(i0 + t + 2, last_plane);
    D[(K + 2) & 3] = ld_rs_nt(prs(dl, pn), o_c);
    if (HAS_F) Fv[(K + 2) & 3] = ld_rs(prs(ff, pn), o_c);
    const int oq = (K & 1) ? oq1 : oq0;
    const double* __restrict__ lo = lds + O * 4 * SLOT;     // other colour
    const double* __restrict__ lc = lds + COL * 4 * SLOT;   // own colour
    Nb18 c;
    c.xm = lo[SM * SLOT + ob];         c.xp = lo[SP * SLOT + ob];
    c.ym = lo[S0 * SLOT + ob - RW];    c.yp = lo[S0 * SLOT + ob + RW];
    c.zm = lo[S0 * SLOT + oq - 1];     c.zp = lo[S0 * SLOT + oq];
    c.xpyp = lc[SP * SLOT + ob + RW];  c.xmym = lc[SM * SLOT + ob - RW];
    c.xpym = lc[SP * SLOT + ob - RW];  c.xmyp = lc[SM * SLOT + ob + RW];
    c.xpzp = lc[SP * SLOT + oq];       c.xmzm = lc[SM * SLOT + oq - 1];
    c.xpzm = lc[SP * SLOT + oq - 1];   c.xmzp = lc[SM * SLOT + oq];
    c.ypzp = lc[S0 * SLOT + oq + RW];  c.ymzm = lc[S0 * SLOT + oq - RW - 1];
    c.ypzm = lc[S0 * SLOT + oq + RW - 1]; c.ymzp = lc[S0 * SLOT + oq - RW];
    const double fc = HAS_F ? Fv[K] : 0.0;
    double S;
    const double sig = sigma_cell(c, 1.0 + D[K], ih2, S);
    st_rs_nt(prs(out, i0 + t), o_c, (S - h2 * (sig + fc - C)) * (1.0 / 6.0));
    acc += sig + fc;
    store(SN, vst);
    __syncthreads();
  };
  for (int t = 0; t < ci; t += 4) {
    step(std::integral_constant<int, 0>(), t, V0, V1);
    step(std::integral_constant<int, 1>(), t + 1, V1, V0);
    step(std::integral_constant<int, 2>(), t + 2, V0, V1);
    step(std::integral_constant<int, 3>(), t + 3, V1, V0);
  }

  double vv[1] = {acc};
  const bool last = grid_sum<1>(vv, a.partials, a.counter, a.sum_out, gridDim.x, blockIdx.x);
  if (last && tid == 0 && a.copy_to) *a.copy_to = *a.copy_from;
}

// ---- fused defect + restriction -----------------------------------------------------------
// d = nabla^2 theta - Sigma - f + C at every fine cell, then the 8-son averages of d and theta
// (Eq. 18 and R). A thread owns fine rows 2J, 2J+1 and the cell pair k = 2m, 2m+1 (both colours
// at column m), so over the two planes 2I, 2I+1 it holds all 8 sons of coarse cell (I, J, m).
// Also accumulates sum d and sum d^2 (the projected residual norm of this level).
template <int TM>
__global__ void __launch_bounds__(256) defect_restrict_kernel(DefectArgs a) {
  extern __shared__ double lds[];
  const int n = a.n, nh = n >> 1, nc = n >> 1, nch = nc >> 1;
  const int tj = a.tj;               // fine rows per tile (even)
  const int ncomp = TM * (tj >> 1);  // threads that own a coarse cell; the rest only load
  const int nthreads = blockDim.x;
  const int tid = threadIdx.x;
  int j0, m0, i0;
  tile_coords(gridDim.x, a.tiles_m, a.tiles_j, tj, TM, a.ci, j0, m0, i0);
  const int i1 = i0 + a.ci;
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
  const unsigned halfc = (unsigned)nc * (unsigned)nc * (unsigned)nch;

  PlaneLoader<TM> ld;
  ld.init(tid, nthreads, tj, j0, m0, n);
  PlaneRing<TM> R{lds, tj};
  const double* __restrict__ th = a.theta;
  double v[kMaxPrefetch];
  for (int p = i0 - 1; p <= i0 + 1; ++p) {
    fetch_plane<TM>(ld, th, nullptr, p, n, v);
    ld.store(lds, tj, p, v);
  }
  __syncthreads();

  const int s = tid % TM, rr = tid / TM;   // coarse row within the tile
  const int m = m0 + s;
  const double C = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const double ih2 = a.ih2;
  double n1 = 0.0, n2 = 0.0, sd = 0.0, st = 0.0;

  const bool active = tid < ncomp;
  for (int i = i0; i < i1; ++i) {
    const bool pre = (i + 2 <= i1);
    if (pre) fetch_plane<TM>(ld, th, nullptr, i + 2, n, v);
    if (active) {
#pragma unroll
      for (int dr = 0; dr < 2; ++dr) {
        const int r = 2 * rr + dr;
        const int j = j0 + r;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int q = (i + j + c) & 1;
          Nb18 t;
          ring_gather<TM>(R, c, i, q, r + 1, s + 1, t);
          const unsigned e = c * half + (unsigned)i * plane + (unsigned)j * nh + m;
          const double tc = R.at(c, i, r + 1, s + 1);
          double S;
          const double sig = sigma_cell(t, 1.0 + a.delta[e], ih2, S);
          const double d = (S - 6.0 * tc) * ih2 - sig - (a.f ? a.f[e] : 0.0) + C;
          n1 += d;
          n2 += d * d;
          sd += d;
          st += tc;
        }
      }
      if (i & 1) {
        const int I = i >> 1, J = (j0 >> 1) + rr, K = m;
        const unsigned ec = ((I + J + K) & 1) * halfc + ((unsigned)I * nc + J) * (unsigned)nch + (unsigned)(K >> 1);
        a.theta_c[ec] = 0.125 * st;
        if (a.theta_c2) a.theta_c2[ec] = 0.125 * st;
        a.dr[ec] = 0.125 * sd;
        sd = 0.0;
        st = 0.0;
      }
    }
    if (pre) ld.store(lds, tj, i + 2, v);
    __syncthreads();
  }
  double vv[2] = {n1, n2};
  grid_sum<2>(vv, a.partials, a.counter, a.sums_out, gridDim.x, blockIdx.x);
}

// ---- pipelined defect + restriction ------------------------------------------------------------
// The outputs of defect_restrict_kernel on the decomposition of the pipelined sweep: a thread owns
// column (j, m) and evaluates both colours (two independent roots) per plane; it accumulates the
// defect and theta over the plane pair 2I, 2I+1, and after the odd plane the thread of the even row
// adds its neighbour's partial sums from LDS to complete the 8 sons of coarse cell (I, j/2, m).
// Chunks are multiples of 4 planes (uneven lengths), the plane loop is unrolled by the ring length
// (compile-time slots), planes are fetched two steps ahead and delta / f two steps before use.
template <int TM, int TJ, bool HAS_F>
__global__ void __launch_bounds__(TM * TJ) defect_restrict_pipe(DefectArgs a, int nchunks) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int TOTAL = 2 * SLOT;
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  static_assert(TJ % 2 == 0, "row pairs");
  __shared__ double lds[2 * 4 * SLOT];
  __shared__ double xb[NT][2];
  const int n = a.n, nh = n >> 1, nc = n >> 1, nch = nc >> 1;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = a.tiles_m * a.tiles_j;
  const int tile = logical % ntile, chunk = logical / ntile;
  const int m0 = (tile % a.tiles_m) * TM, j0 = (tile / a.tiles_m) * TJ;
  const int q4 = n / 4;
  const int i0 = 4 * (int)(((long)chunk * q4) / nchunks);
  const int i1 = 4 * (int)(((long)(chunk + 1) * q4) / nchunks);
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
  const unsigned halfc = (unsigned)nc * (unsigned)nc * (unsigned)nch;
  const double* __restrict__ th = a.theta;

  unsigned goff[NPF];
  int loff[NPF];
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    int e = tid + t * NT;
    e = e < TOTAL ? e : TOTAL - 1;
    const int cc = e / SLOT;
    const int rem = e - cc * SLOT;
    const int r = rem / RW;
    const int c = rem - r * RW;
    goff[t] = (unsigned)cc * half + (unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh);
    loff[t] = cc * 4 * SLOT + rem;
  }
  auto fetch = [&](int rel, double (&v)[NPF]) {
    const unsigned base = (unsigned)wrapi(i0 - 1 + rel, n) * plane;
#pragma unroll
    for (int t = 0; t < NPF; ++t) v[t] = th[base + goff[t]];
  };
  auto store = [&](int slot, const double (&v)[NPF]) {
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[loff[t] + slot * SLOT] = v[t];
  };

  const int s = tid % TM, r = tid / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned own = (unsigned)j * nh + m;
  const int ob = (r + 1) * RW + (s + 1);
  const int qa = (i0 + j) & 1;
  const int oq00 = ob + qa, oq01 = ob + (qa ^ 1);
  const double C = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const double ih2 = a.ih2;
  const double* __restrict__ dl = a.delta + own;
  const double* __restrict__ ff = HAS_F ? a.f + own : nullptr;
  const int last_plane = n - 1;
  double n1 = 0.0, n2 = 0.0, sd = 0.0, st = 0.0;

  double V0[NPF], V1[NPF];
  double D[4][2], Fv[4][2];
  {
    double va[NPF], vb[NPF], vc[NPF];
    fetch(0, va);
    fetch(1, vb);
    fetch(2, vc);
    store(0, va);
    store(1, vb);
    store(2, vc);
  }
  fetch(3, V0);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const unsigned pk = (unsigned)min(i0 + k, last_plane) * plane;
    D[k][0] = dl[pk];
    D[k][1] = dl[half + pk];
    if (HAS_F) {
      Fv[k][0] = ff[pk];
      Fv[k][1] = ff[half + pk];
    }
  }
  __syncthreads();

  auto gather = [&](const double* lo, const double* lc, int SM, int S0, int SP, int oq, Nb18& c) {
    c.xm = lo[SM * SLOT + ob];         c.xp = lo[SP * SLOT + ob];
    c.ym = lo[S0 * SLOT + ob - RW];    c.yp = lo[S0 * SLOT + ob + RW];
    c.zm = lo[S0 * SLOT + oq - 1];     c.zp = lo[S0 * SLOT + oq];
    c.xpyp = lc[SP * SLOT + ob + RW];  c.xmym = lc[SM * SLOT + ob - RW];
    c.xpym = lc[SP * SLOT + ob - RW];  c.xmyp = lc[SM * SLOT + ob + RW];
    c.xpzp = lc[SP * SLOT + oq];       c.xmzm = lc[SM * SLOT + oq - 1];
    c.xpzm = lc[SP * SLOT + oq - 1];   c.xmzp = lc[SM * SLOT + oq];
    c.ypzp = lc[S0 * SLOT + oq + RW];  c.ymzm = lc[S0 * SLOT + oq - RW - 1];
    c.ypzm = lc[S0 * SLOT + oq + RW - 1]; c.ymzp = lc[S0 * SLOT + oq - RW];
  };
  auto step = [&](auto kc, int t, double (&vst)[NPF], double (&vft)[NPF]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = K & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    const unsigned pn = (unsigned)min(i0 + t + 2, last_plane) * plane;
    D[(K + 2) & 3][0] = dl[pn];
    D[(K + 2) & 3][1] = dl[half + pn];
    if (HAS_F) {
      Fv[(K + 2) & 3][0] = ff[pn];
      Fv[(K + 2) & 3][1] = ff[half + pn];
    }
    const double* l0 = lds;
    const double* l1 = lds + 4 * SLOT;
    const int oqc0 = (K & 1) ? oq01 : oq00;
    const int oqc1 = (K & 1) ? oq00 : oq01;
    // the two colours' roots one after the other (fewer live registers than iterating both)
    double S[2], sr[2];
    {
      Nb18 c0;
      gather(l1, l0, SM, S0, SP, oqc0, c0);
      double pp[1], qq[1], r1[1];
      cell_pq(c0, 1.0 + D[K][0], ih2, S[0], pp[0], qq[0]);
      largest_roots<1>(pp, qq, r1);
      sr[0] = r1[0];
    }
    {
      Nb18 c1;
      gather(l0, l1, SM, S0, SP, oqc1, c1);
      double pp[1], qq[1], r1[1];
      cell_pq(c1, 1.0 + D[K][1], ih2, S[1], pp[0], qq[0]);
      largest_roots<1>(pp, qq, r1);
      sr[1] = r1[0];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double tc = (c == 0 ? l0 : l1)[S0 * SLOT + ob];
      const double d = (S[c] - 6.0 * tc) * ih2 - (sr[c] - 3.0) - (HAS_F ? Fv[K][c] : 0.0) + C;
      n1 += d;
      n2 += d * d;
      sd += d;
      st += tc;
    }
    if (K & 1) {   // odd plane: partial sums of the plane pair to LDS
      xb[tid][0] = sd;
      xb[tid][1] = st;
    }
    store(SN, vst);
    __syncthreads();
    if (K & 1) {
      if ((r & 1) == 0) {
        const double sdt = sd + xb[tid + TM][0];
        const double stt = st + xb[tid + TM][1];
        const int i = i0 + t;
        const int I = i >> 1, J = j >> 1, Kc = m;
        const unsigned ec = ((I + J + Kc) & 1) * halfc + ((unsigned)I * nc + J) * (unsigned)nch + (unsigned)(Kc >> 1);
        a.theta_c[ec] = 0.125 * stt;
        if (a.theta_c2) a.theta_c2[ec] = 0.125 * stt;
        a.dr[ec] = 0.125 * sdt;
      }
      sd = 0.0;
      st = 0.0;
    }
  };
  for (int t = 0; t < i1 - i0; t += 4) {
    step(std::integral_constant<int, 0>(), t, V0, V1);
    step(std::integral_constant<int, 1>(), t + 1, V1, V0);
    step(std::integral_constant<int, 2>(), t + 2, V0, V1);
    step(std::integral_constant<int, 3>(), t + 3, V1, V0);
  }
  double vv[2] = {n1, n2};
  grid_sum<2>(vv, a.partials, a.counter, a.sums_out, gridDim.x, blockIdx.x);
}

// ---- pipelined FAS right-hand side ---------------------------------------------------------------
// tau_kernel's outputs (Eq. 19: f = nabla^2 th - Sigma(th) - rd, in place over rd allowed; sums of
// Sigma + f) on the decomposition of the pipelined sweep: a thread owns column (j, m) and both
// colours per plane (two roots per step); chunks are multiples of 4 planes.
template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) tau_pipe(const double* __restrict__ th, const double* __restrict__ delta,
                                                    const double* rd, double* f, int n, double ih2, Reduce red,
                                                    int tiles_j, int tiles_m, int nchunks) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int TOTAL = 2 * SLOT;
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  __shared__ double lds[2 * 4 * SLOT];
  const int nh = n >> 1;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = tiles_m * tiles_j;
  const int tile = logical % ntile, chunk = logical / ntile;
  const int m0 = (tile % tiles_m) * TM, j0 = (tile / tiles_m) * TJ;
  const int q4 = n / 4;
  const int i0 = 4 * (int)(((long)chunk * q4) / nchunks);
  const int i1 = 4 * (int)(((long)(chunk + 1) * q4) / nchunks);
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;

  unsigned goff[NPF];
  int loff[NPF];
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    int e = tid + t * NT;
    e = e < TOTAL ? e : TOTAL - 1;
    const int cc = e / SLOT;
    const int rem = e - cc * SLOT;
    const int r = rem / RW;
    const int c = rem - r * RW;
    goff[t] = (unsigned)cc * half + (unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh);
    loff[t] = cc * 4 * SLOT + rem;
  }
  auto fetch = [&](int rel, double (&v)[NPF]) {
    const unsigned base = (unsigned)wrapi(i0 - 1 + rel, n) * plane;
#pragma unroll
    for (int t = 0; t < NPF; ++t) v[t] = th[base + goff[t]];
  };
  auto store = [&](int slot, const double (&v)[NPF]) {
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[loff[t] + slot * SLOT] = v[t];
  };

  const int s = tid % TM, r = tid / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned own = (unsigned)j * nh + m;
  const int ob = (r + 1) * RW + (s + 1);
  const int qa = (i0 + j) & 1;
  const int oq00 = ob + qa, oq01 = ob + (qa ^ 1);
  const double* __restrict__ dl = delta + own;
  const int last_plane = n - 1;
  double acc = 0.0;

  double V0[NPF], V1[NPF];
  double D[4][2];
  {
    double va[NPF], vb[NPF], vc[NPF];
    fetch(0, va);
    fetch(1, vb);
    fetch(2, vc);
    store(0, va);
    store(1, vb);
    store(2, vc);
  }
  fetch(3, V0);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const unsigned pk = (unsigned)min(i0 + k, last_plane) * plane;
    D[k][0] = dl[pk];
    D[k][1] = dl[half + pk];
  }
  __syncthreads();

  auto gather = [&](const double* lo, const double* lc, int SM, int S0, int SP, int oq, Nb18& c) {
    c.xm = lo[SM * SLOT + ob];         c.xp = lo[SP * SLOT + ob];
    c.ym = lo[S0 * SLOT + ob - RW];    c.yp = lo[S0 * SLOT + ob + RW];
    c.zm = lo[S0 * SLOT + oq - 1];     c.zp = lo[S0 * SLOT + oq];
    c.xpyp = lc[SP * SLOT + ob + RW];  c.xmym = lc[SM * SLOT + ob - RW];
    c.xpym = lc[SP * SLOT + ob - RW];  c.xmyp = lc[SM * SLOT + ob + RW];
    c.xpzp = lc[SP * SLOT + oq];       c.xmzm = lc[SM * SLOT + oq - 1];
    c.xpzm = lc[SP * SLOT + oq - 1];   c.xmzp = lc[SM * SLOT + oq];
    c.ypzp = lc[S0 * SLOT + oq + RW];  c.ymzm = lc[S0 * SLOT + oq - RW - 1];
    c.ypzm = lc[S0 * SLOT + oq + RW - 1]; c.ymzp = lc[S0 * SLOT + oq - RW];
  };
  auto step = [&](auto kc, int t, double (&vst)[NPF], double (&vft)[NPF]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = K & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    const unsigned pn = (unsigned)min(i0 + t + 2, last_plane) * plane;
    D[(K + 2) & 3][0] = dl[pn];
    D[(K + 2) & 3][1] = dl[half + pn];
    const double* l0 = lds;
    const double* l1 = lds + 4 * SLOT;
    const int oqc0 = (K & 1) ? oq01 : oq00;
    const int oqc1 = (K & 1) ? oq00 : oq01;
    // the two colours' roots one after the other (fewer live registers than iterating both)
    double S[2], sr[2];
    {
      Nb18 c0;
      gather(l1, l0, SM, S0, SP, oqc0, c0);
      double pp[1], qq[1], r1[1];
      cell_pq(c0, 1.0 + D[K][0], ih2, S[0], pp[0], qq[0]);
      largest_roots<1>(pp, qq, r1);
      sr[0] = r1[0];
    }
    {
      Nb18 c1;
      gather(l0, l1, SM, S0, SP, oqc1, c1);
      double pp[1], qq[1], r1[1];
      cell_pq(c1, 1.0 + D[K][1], ih2, S[1], pp[0], qq[0]);
      largest_roots<1>(pp, qq, r1);
      sr[1] = r1[0];
    }
    const unsigned e0 = (unsigned)(i0 + t) * plane + own;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double tc = (c == 0 ? l0 : l1)[S0 * SLOT + ob];
      const double sig = sr[c] - 3.0;
      const unsigned e = (unsigned)c * half + e0;
      const double fv = (S[c] - 6.0 * tc) * ih2 - sig - rd[e];
      f[e] = fv;
      acc += sig + fv;
    }
    store(SN, vst);
    __syncthreads();
  };
  for (int t = 0; t < i1 - i0; t += 4) {
    step(std::integral_constant<int, 0>(), t, V0, V1);
    step(std::integral_constant<int, 1>(), t + 1, V1, V0);
    step(std::integral_constant<int, 2>(), t + 2, V0, V1);
    step(std::integral_constant<int, 3>(), t + 3, V1, V0);
  }
  double vv[2] = {acc, 0.0};
  grid_sum<2>(vv, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// Tile and chunk count of the pipelined FAS right-hand side (as for the defect + restriction).
bool tau_pipe_cfg(int n, int& tm, int& tj, int& nchunks) {
  static const int pref[][2] = {{64, 8}, {32, 8}, {16, 8}, {8, 8}, {4, 8}};
  if (n % 8 != 0) return false;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return false;
  for (const auto& p : pref) {
    if ((n / 2) % p[0] != 0 || n % p[1] != 0) continue;
    const void* k = nullptr;
#define MR_TP_PTR(TM, TJ) \
    if (p[0] == TM && p[1] == TJ) k = reinterpret_cast<const void*>(&tau_pipe<TM, TJ>);
    MR_TP_PTR(64, 8) MR_TP_PTR(32, 8) MR_TP_PTR(16, 8) MR_TP_PTR(8, 8) MR_TP_PTR(4, 8)
#undef MR_TP_PTR
    int bpc = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k, p[0] * p[1], 0) != hipSuccess || bpc < 1) continue;
    const long tiles = (long)(n / p[1]) * (n / 2 / p[0]);
    long ch = ((long)cus * bpc) / tiles;
    ch = std::max(1L, std::min(ch, (long)(n / 8)));
    while (ch > 1 && tiles * ch > kMaxReduceBlocks) --ch;
    if (tiles * ch > kMaxReduceBlocks) return false;
    tm = p[0];
    tj = p[1];
    nchunks = (int)ch;
    return true;
  }
  return false;
}

hipError_t launch_tau_pipe(const double* th, const double* delta, const double* rd, double* f, int n, double h,
                           Reduce red, hipStream_t s, bool* done) {
  int tm = 0, tj = 0, nch = 0;
  *done = false;
  if (!tau_pipe_cfg(n, tm, tj, nch)) return hipSuccess;
  const int tiles_j = n / tj, tiles_m = n / 2 / tm;
  const unsigned blocks = (unsigned)(tiles_j * tiles_m * nch);
  const double ih2 = 1.0 / (h * h);
#define MR_TP_LAUNCH(TM, TJ)                                                                                   \
  if (tm == TM && tj == TJ) {                                                                                  \
    hipLaunchKernelGGL((tau_pipe<TM, TJ>), dim3(blocks), dim3(TM * TJ), 0, s, th, delta, rd, f, n, ih2, red,      \
                       tiles_j, tiles_m, nch);                                                                 \
    *done = true;                                                                                              \
    return hipGetLastError();                                                                                  \
  }
  MR_TP_LAUNCH(64, 8) MR_TP_LAUNCH(32, 8) MR_TP_LAUNCH(16, 8) MR_TP_LAUNCH(8, 8) MR_TP_LAUNCH(4, 8)
#undef MR_TP_LAUNCH
  return hipSuccess;
}

// Coarsest mesh (at most 12^3 cells): nsweeps red-black sweeps by one block with the whole
// mesh in LDS (natural order inside the block). Same update and snapshot semantics as the tiled
// half-sweeps; the uniform shift is lagged by one sweep and refreshed in-block after every sweep.
__global__ void __launch_bounds__(256) coarsest_kernel(CoarsestArgs a) {
  __shared__ double th[kMaxCoarsest], dd[kMaxCoarsest], fv[kMaxCoarsest], nv[kMaxCoarsest];
  __shared__ double red[16][1];
  __shared__ double cnew;
  const int n = a.n, n3 = n * n * n;
  const int tid = threadIdx.x;
  for (int e = tid; e < n3; e += blockDim.x) {
    const int i = e / (n * n), j = (e / n) % n, k = e % n;
    const unsigned g = split_idx(n, i, j, k);
    th[e] = a.theta[g];
    dd[e] = 1.0 + a.delta[g];
    fv[e] = a.f ? a.f[g] : 0.0;
  }
  double C = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  __syncthreads();
  const double h2 = a.h2, ih2 = a.ih2;
  auto at = [&](int i, int j, int k) { return th[(wrapi(i, n) * n + wrapi(j, n)) * n + wrapi(k, n)]; };
  for (int sw = 0; sw < a.nsweeps; ++sw) {
    double acc = 0.0;
    for (int colour = 0; colour < 2; ++colour) {
      for (int e = tid; e < n3; e += blockDim.x) {
        const int i = e / (n * n), j = (e / n) % n, k = e % n;
        if (((i + j + k) & 1) != colour) continue;
        Nb18 t;
        t.xm = at(i - 1, j, k); t.xp = at(i + 1, j, k);
        t.ym = at(i, j - 1, k); t.yp = at(i, j + 1, k);
        t.zm = at(i, j, k - 1); t.zp = at(i, j, k + 1);
        t.xpyp = at(i + 1, j + 1, k); t.xmym = at(i - 1, j - 1, k);
        t.xpym = at(i + 1, j - 1, k); t.xmyp = at(i - 1, j + 1, k);
        t.xpzp = at(i + 1, j, k + 1); t.xmzm = at(i - 1, j, k - 1);
        t.xpzm = at(i + 1, j, k - 1); t.xmzp = at(i - 1, j, k + 1);
        t.ypzp = at(i, j + 1, k + 1); t.ymzm = at(i, j - 1, k - 1);
        t.ypzm = at(i, j + 1, k - 1); t.ymzp = at(i, j - 1, k + 1);
        double S;
        const double sig = sigma_cell(t, dd[e], ih2, S);
        nv[e] = (S - h2 * (sig + fv[e] - C)) * (1.0 / 6.0);
        acc += sig + fv[e];
      }
      __syncthreads();
      for (int e = tid; e < n3; e += blockDim.x) {
        const int i = e / (n * n), j = (e / n) % n, k = e % n;
        if (((i + j + k) & 1) == colour) th[e] = nv[e];
      }
      __syncthreads();
    }
    double v[1] = {acc};
    block_sum<1>(v, red, tid, blockDim.x);
    if (tid == 0) cnew = v[0] / (double)n3;
    __syncthreads();
    C = cnew;
    __syncthreads();
  }
  for (int e = tid; e < n3; e += blockDim.x) {
    const int i = e / (n * n), j = (e / n) % n, k = e % n;
    a.theta[split_idx(n, i, j, k)] = th[e];
  }
  if (tid == 0 && a.c_sum_out) {
    a.c_sum_out[0] = C * (double)n3;
    a.c_sum_out[1] = 0.0;
  }
}

// ---- fused red-black sweep (one launch per sweep) -----------------------------------------
// Both half-sweeps of Eq. 17 in one pass over the mesh. A cell's update reads only its 18
// neighbours (never its own old value), so a block can compute the new red values of plane p on
// its tile plus a one-cell halo (the halo cells are recomputed identically by the neighbouring
// blocks), and the new black values of plane p - 2 on its tile from red values already in LDS.
// Old theta of both colours (tile plus a two-cell halo) streams through LDS rings: red needs
// planes p-1..p+1, black p-3..p+1 (faces of red at plane p, edges of black at p-3..p-1); the
// new red values live in a 4-plane ring. One barrier per plane; every old value, delta and f is
// read from HBM once (plus halos) and every new value written once: 24 B per cell update.
// Latency: old planes are fetched into registers three plane steps before they enter LDS, and
// the per-cell inputs (delta, f) two steps before use, from three rotating register sets (the
// plane loop is unrolled by three so that each set is a fixed group of registers).
// Sums of Sigma + f over the block's own cells of each colour go to sum_out[0] (red) and
// sum_out[1] (black).
template <int TM, int TJ>
struct FusedTile {
  static constexpr int NT = TM * TJ;
  static constexpr int DW = TM + 4, DH = TJ + 4, DS = DW * DH;   // old values: tile + 2-cell halo
  static constexpr int EW = TM + 2, EH = TJ + 2, ES = EW * EH;   // new red: tile + 1-cell halo
  static constexpr int H = 2 * EW + 2 * TJ;                      // red halo cells per plane
  static constexpr int LTOT = 2 * DS;                            // old values loaded per plane
  static constexpr int NPF = (LTOT + NT - 1) / NT;
  static constexpr int LDS = 4 * DS + 6 * DS + 4 * ES;           // doubles
  static_assert(H <= NT, "tile too small for its halo");
};

__device__ __forceinline__ int slot6(int p) { return ((p % 6) + 6) % 6; }

// Per-cell inputs of one plane step: delta and f of the own red cell, the red halo cell and the
// own black cell.
struct StepIn {
  double dRo, dRh, dB, fRo, fRh, fB;
};

// The plane loop runs over steps t = 0, 1, ... (red plane p = i0 - 1 + t, black plane p - 2).
// Ring slots are taken relative to the first old plane P0 = i0 - 2 (rel = plane - P0), and the
// loop is unrolled by 12 (a multiple of both ring lengths), so that every slot and the parity of
// every z-neighbour offset is a compile-time constant of the unrolled step: each LDS access is a
// per-thread base address plus an immediate offset.
template <int TM, int TJ, bool HAS_F>
struct FusedSweep {
  using F = FusedTile<TM, TJ>;
  static constexpr int NT = F::NT, DW = F::DW, DS = F::DS, EW = F::EW, ES = F::ES, NPF = F::NPF;
  static constexpr int OR0 = 0, OB0 = 4 * DS, NR0 = 10 * DS;   // ring bases (doubles)
  static constexpr int s4(int rel) { return rel & 3; }
  static constexpr int s6(int rel) { return rel % 6; }

  double* lds;
  const double* __restrict__ th;
  const double* __restrict__ dl;
  const double* __restrict__ ff;
  double* __restrict__ out;
  int n, P0, i0, i1, tlast;          // tlast: last step; planes P0 .. P0 + tlast + 2 are loaded
  unsigned plane, half, own_off, halo_off;
  bool has_halo;
  double C, h2, ih2, accR, accB;
  unsigned goff[NPF];
  int soff_r[NPF], soff_b[NPF];
  bool blk[NPF];
  // per-thread LDS element offsets: own red cell (D coords), red halo cell (D coords), own black
  // cell (E coords in the new-red ring, D coords in the old-black ring); *_q[k]: the same plus the
  // z-parity of the cell when rel is even (k = 0) or odd (k = 1)
  int pro, pro_q[2], prh, prh_q[2], pbE, pbE_q[2], pbD, pbD_q[2];
  int wro, wrh;   // new red of the own and the halo cell (E coords, ring base)
  double B0[NPF], B1[NPF], B2[NPF];
  StepIn I0, I1, I2;

  __device__ __forceinline__ void fetch(int rel, double (&v)[NPF]) const {
    const unsigned base = (unsigned)wrapi(P0 + rel, n) * plane;
#pragma unroll
    for (int t = 0; t < NPF; ++t) v[t] = th[base + goff[t]];
  }
  template <int REL>
  __device__ __forceinline__ void store(const double (&v)[NPF]) {
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[blk[t] ? soff_b[t] + s6(REL) * DS : soff_r[t] + s4(REL) * DS] = v[t];
  }
  __device__ __forceinline__ void store_rt(int rel, const double (&v)[NPF]) {
    const int sr = (rel & 3) * DS, sb = (rel % 6) * DS;
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[blk[t] ? soff_b[t] + sb : soff_r[t] + sr] = v[t];
  }
  __device__ __forceinline__ double cell_in(const double* __restrict__ fld, int colour, int rel, unsigned off) const {
    return fld[(unsigned)colour * half + (unsigned)wrapi(P0 + rel, n) * plane + off];
  }
  // inputs of step t: red plane rel t + 1 (if plane <= i1), black plane rel t - 1 (if in [i0, i1))
  __device__ __forceinline__ StepIn load_in(int t) const {
    double dRo = 0.0, dRh = 0.0, dB = 0.0, fRo = 0.0, fRh = 0.0, fB = 0.0;
    if (P0 + t + 1 <= i1) {
      dRo = cell_in(dl, 0, t + 1, own_off);
      if (has_halo) dRh = cell_in(dl, 0, t + 1, halo_off);
      if (HAS_F) {
        fRo = cell_in(ff, 0, t + 1, own_off);
        if (has_halo) fRh = cell_in(ff, 0, t + 1, halo_off);
      }
    }
    const int pb = P0 + t - 1;
    if (pb >= i0 && pb < i1) {
      dB = cell_in(dl, 1, t - 1, own_off);
      if (HAS_F) fB = cell_in(ff, 1, t - 1, own_off);
    }
    return StepIn{dRo, dRh, dB, fRo, fRh, fB};
  }
  // red cell of plane REL from the old rings; pc at the cell (D coords), pq = pc + q
  template <int REL>
  __device__ __forceinline__ void gather_red(int c0, int q0, Nb18& t) const {
    const double* pc = lds + c0;
    const double* pq = lds + q0;
    constexpr int bm = OB0 + s6(REL + 5) * DS, b0 = OB0 + s6(REL) * DS, bp = OB0 + s6(REL + 1) * DS;
    constexpr int rm = OR0 + s4(REL + 3) * DS, r0 = OR0 + s4(REL) * DS, rp = OR0 + s4(REL + 1) * DS;
    t.xm = pc[bm]; t.xp = pc[bp];
    t.ym = pc[b0 - DW]; t.yp = pc[b0 + DW];
    t.zm = pq[b0 - 1];  t.zp = pq[b0];
    t.xpyp = pc[rp + DW]; t.xmym = pc[rm - DW];
    t.xpym = pc[rp - DW]; t.xmyp = pc[rm + DW];
    t.xpzp = pq[rp];      t.xmzm = pq[rm - 1];
    t.xpzm = pq[rp - 1];  t.xmzp = pq[rm];
    t.ypzp = pq[r0 + DW]; t.ymzm = pq[r0 - DW - 1];
    t.ypzm = pq[r0 + DW - 1]; t.ymzp = pq[r0 - DW];
  }
  // black own cell of plane REL: faces from the new-red ring (E coords), edges from old black
  template <int REL>
  __device__ __forceinline__ void gather_black(Nb18& t) const {
    const double* eq = lds + pbE_q[REL & 1];
    const double* dq = lds + pbD_q[REL & 1];
    const double* pE = lds + pbE;
    const double* pD = lds + pbD;
    constexpr int nm = s4(REL + 3) * ES, n0 = s4(REL) * ES, np = s4(REL + 1) * ES;
    constexpr int bm = s6(REL + 5) * DS, b0 = s6(REL) * DS, bp = s6(REL + 1) * DS;
    t.xm = pE[nm]; t.xp = pE[np];
    t.ym = pE[n0 - EW]; t.yp = pE[n0 + EW];
    t.zm = eq[n0 - 1];   t.zp = eq[n0];
    t.xpyp = pD[bp + DW]; t.xmym = pD[bm - DW];
    t.xpym = pD[bp - DW]; t.xmyp = pD[bm + DW];
    t.xpzp = dq[bp];       t.xmzm = dq[bm - 1];
    t.xpzm = dq[bp - 1];   t.xmzp = dq[bm];
    t.ypzp = dq[b0 + DW];  t.ymzm = dq[b0 - DW - 1];
    t.ypzm = dq[b0 + DW - 1]; t.ymzp = dq[b0 - DW];
  }

  // Step t = 12 u + K: red plane rel t + 1, black plane rel t - 1; store old plane rel t + 3
  // (fetched two steps earlier), fetch rel t + 5, load the inputs of step t + 2.
  template <int K>
  __device__ __forceinline__ void step(int t) {
    if (t > tlast) return;
    constexpr int kS = (K + 2) % 3, kF = (K + 1) % 3;          // store / fetch buffer
    constexpr int kC = K % 3, kN = (K + 2) % 3;                // current / next inputs
    double(&vs)[NPF] = kS == 0 ? B0 : (kS == 1 ? B1 : B2);
    double(&vf)[NPF] = kF == 0 ? B0 : (kF == 1 ? B1 : B2);
    const StepIn& cur = kC == 0 ? I0 : (kC == 1 ? I1 : I2);
    StepIn& nxt = kN == 0 ? I0 : (kN == 1 ? I1 : I2);
    if (t + 4 <= tlast) fetch(t + 5, vf);
    if (t + 2 <= tlast) nxt = load_in(t + 2);
    constexpr int REL = K + 1;            // red plane rel modulo 12 (t = 12 u + K)
    constexpr int RELB = K + 11;          // black plane rel (t - 1) modulo 12, kept non-negative
    const int pr = P0 + t + 1, pb = P0 + t - 1;
    const bool do_red = pr <= i1;
    const bool do_black = pb >= i0;
    if (do_red && has_halo) {
      Nb18 c;
      gather_red<REL>(prh, prh_q[REL & 1], c);
      double S, pp[1], qq[1], sr[1];
      cell_pq(c, 1.0 + cur.dRh, ih2, S, pp[0], qq[0]);
      largest_roots<1>(pp, qq, sr);
      lds[wrh + s4(REL) * ES] = (S - h2 * (sr[0] - 3.0 + cur.fRh - C)) * (1.0 / 6.0);
    }
    if (do_red || do_black) {
      Nb18 tr, tb;
      double Sr = 0.0, Sb = 0.0, pp[2] = {0.0, 0.0}, qq[2] = {-27.0, -27.0}, sr[2];
      if (do_red) {
        gather_red<REL>(pro, pro_q[REL & 1], tr);
        cell_pq(tr, 1.0 + cur.dRo, ih2, Sr, pp[0], qq[0]);
      }
      if (do_black) {
        gather_black<RELB>(tb);
        cell_pq(tb, 1.0 + cur.dB, ih2, Sb, pp[1], qq[1]);
      }
      largest_roots<2>(pp, qq, sr);
      if (do_red) {
        const double sig = sr[0] - 3.0;
        const double nv = (Sr - h2 * (sig + cur.fRo - C)) * (1.0 / 6.0);
        lds[wro + s4(REL) * ES] = nv;
        if (pr >= i0 && pr < i1) {
          out[(unsigned)pr * plane + own_off] = nv;
          accR += sig + cur.fRo;
        }
      }
      if (do_black) {
        const double sig = sr[1] - 3.0;
        out[half + (unsigned)pb * plane + own_off] = (Sb - h2 * (sig + cur.fB - C)) * (1.0 / 6.0);
        accB += sig + cur.fB;
      }
    }
    if (t + 2 <= tlast) store<K + 3>(vs);
    __syncthreads();
  }
};

template <int TM, int TJ, bool HAS_F>
__global__ void __launch_bounds__(TM * TJ) sweep_fused(FusedSweepArgs a) {
  using FS = FusedSweep<TM, TJ, HAS_F>;
  using F = FusedTile<TM, TJ>;
  constexpr int NT = F::NT, DW = F::DW, DS = F::DS, EW = F::EW, NPF = F::NPF;
  __shared__ double lds[F::LDS];
  FS st;
  st.lds = lds;
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = a.tiles_m * a.tiles_j;
  const int tile = logical % ntile, chunk = logical / ntile;
  const int m0 = (tile % a.tiles_m) * TM, j0 = (tile / a.tiles_m) * TJ;
  st.n = n;
  st.i0 = (int)(((long)chunk * n) / a.nchunks);
  st.i1 = (int)(((long)(chunk + 1) * n) / a.nchunks);
  st.P0 = st.i0 - 2;
  st.tlast = st.i1 + 1 - (st.i0 - 1);
  st.plane = (unsigned)n * (unsigned)nh;
  st.half = st.plane * (unsigned)n;
  st.th = a.th_in;
  st.dl = a.delta;
  st.ff = a.f;
  st.out = a.th_out;
  st.C = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  st.h2 = a.h2;
  st.ih2 = a.ih2;
  st.accR = 0.0;
  st.accB = 0.0;
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    int e = tid + t * NT;
    e = e < F::LTOT ? e : F::LTOT - 1;
    const int cc = e / DS;
    const int rem = e - cc * DS;
    const int r = rem / DW;
    const int c = rem - r * DW;
    st.goff[t] = (unsigned)cc * st.half + (unsigned)wrapi(j0 - 2 + r, n) * nh + (unsigned)wrapi(m0 - 2 + c, nh);
    st.soff_r[t] = FS::OR0 + rem;
    st.soff_b[t] = FS::OB0 + rem;
    st.blk[t] = cc != 0;
  }
  const int s = tid % TM, r = tid / TM;
  st.has_halo = tid < F::H;
  int rh = 0, sh = 0;
  if (tid < EW) {
    rh = 0;
    sh = tid;
  } else if (tid < 2 * EW) {
    rh = TJ + 1;
    sh = tid - EW;
  } else {
    const int k = tid - 2 * EW;
    rh = 1 + (k >> 1);
    sh = (k & 1) ? TM + 1 : 0;
  }
  const int jm = j0 + r, mm = m0 + s;
  const int jh = wrapi(j0 - 1 + rh, n), mh = wrapi(m0 - 1 + sh, nh);
  st.own_off = (unsigned)jm * nh + mm;
  st.halo_off = (unsigned)jh * nh + mh;
  // z-parity of a colour-c cell of row j in plane P0 + rel: q = (P0 + rel + j + c) & 1
  const int qro = (st.P0 + jm) & 1, qrh = (st.P0 + jh) & 1, qb = (st.P0 + jm + 1) & 1;
  st.pro = (r + 2) * DW + (s + 2);
  st.pro_q[0] = st.pro + qro;
  st.pro_q[1] = st.pro + (qro ^ 1);
  st.prh = (rh + 1) * DW + (sh + 1);
  st.prh_q[0] = st.prh + qrh;
  st.prh_q[1] = st.prh + (qrh ^ 1);
  st.pbE = FS::NR0 + (r + 1) * EW + (s + 1);
  st.pbE_q[0] = st.pbE + qb;
  st.pbE_q[1] = st.pbE + (qb ^ 1);
  st.pbD = FS::OB0 + (r + 2) * DW + (s + 2);
  st.pbD_q[0] = st.pbD + qb;
  st.pbD_q[1] = st.pbD + (qb ^ 1);
  st.wro = FS::NR0 + (r + 1) * EW + (s + 1);
  st.wrh = FS::NR0 + rh * EW + sh;

  // prologue: old planes rel 0..2 into LDS, rel 3 and 4 in flight, inputs of steps 0 and 1
  {
    double va[NPF], vb[NPF], vc[NPF];
    st.fetch(0, va);
    st.fetch(1, vb);
    st.fetch(2, vc);
    st.store_rt(0, va);
    st.store_rt(1, vb);
    st.store_rt(2, vc);
  }
  st.fetch(3, st.B2);
  if (st.tlast >= 3) st.fetch(4, st.B0);
  st.I0 = st.load_in(0);
  st.I1 = st.load_in(1);
  st.I2 = StepIn{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  for (int t = 0; t <= st.tlast; t += 12) {
    st.template step<0>(t);
    st.template step<1>(t + 1);
    st.template step<2>(t + 2);
    st.template step<3>(t + 3);
    st.template step<4>(t + 4);
    st.template step<5>(t + 5);
    st.template step<6>(t + 6);
    st.template step<7>(t + 7);
    st.template step<8>(t + 8);
    st.template step<9>(t + 9);
    st.template step<10>(t + 10);
    st.template step<11>(t + 11);
  }
  double vv[2] = {st.accR, st.accB};
  grid_sum<2>(vv, a.partials, a.counter, a.sum_out, gridDim.x, blockIdx.x);
}

// ---- launchers ----------------------------------------------------------------------------

size_t tile_lds_bytes(int tj, int tm) { return sizeof(double) * 2 * 4 * (size_t)(tj + 2) * (tm + 2); }

// Block size: the compute threads, raised if needed so that every halo element of a plane has a
// loader slot (kMaxPrefetch per thread).
static int tile_threads(const TileCfg& t, int ncomp) {
  const int need = (2 * (t.tj + 2) * (t.tm + 2) + kMaxPrefetch - 1) / kMaxPrefetch;
  return ncomp > need ? ncomp : need;
}

static bool tile_ok(const TileCfg& t, int n, int threads) {
  const long blocks = (long)t.tiles_j * t.tiles_m * (n / t.ci);
  return blocks >= 1 && blocks <= kMaxReduceBlocks && t.tj * t.tiles_j == n && t.tm * t.tiles_m == n / 2 &&
         n % t.ci == 0 && threads >= 1 && threads <= 256 &&
         2 * (t.tj + 2) * (t.tm + 2) <= kMaxPrefetch * threads;
}

// Compiled half-sweep tiles (TM, TJ, CPT). TileCfg selects by (tm, tj, cpt).
#define MR_HS_TILES(X) \
  X(64, 8, 2) X(64, 4, 1) X(64, 8, 1) X(64, 16, 4) X(32, 8, 1) X(32, 16, 2) X(16, 16, 1) \
  X(16, 32, 2) X(8, 16, 1) X(8, 8, 1) X(4, 8, 1) X(4, 16, 2) X(2, 4, 1) X(2, 8, 1)

#define MR_HP_TILES(X) X(64, 8) X(64, 4) X(64, 16) X(32, 8) X(32, 16) X(16, 16)

bool half_sweep_tile_supported(int tm, int tj, int cpt) {
#define MR_HS_MATCH(TM, TJ, CPT) if (tm == TM && tj == TJ && cpt == CPT) return true;
  MR_HS_TILES(MR_HS_MATCH)
#undef MR_HS_MATCH
  return false;
}

hipError_t launch_half_sweep(const HalfSweepArgs& a, const TileCfg& t, hipStream_t s) {
  const long blocks_l = (long)t.tiles_j * t.tiles_m * (a.n / t.ci);
  if (blocks_l < 1 || blocks_l > kMaxReduceBlocks || t.tj * t.tiles_j != a.n || t.tm * t.tiles_m != a.n / 2 ||
      a.n % t.ci != 0)
    return hipErrorInvalidValue;
  HalfSweepArgs b = a;
  b.tj = t.tj;
  b.tiles_j = t.tiles_j;
  b.tiles_m = t.tiles_m;
  b.ci = t.ci;
  const int blocks = (int)blocks_l;
  if (t.pipe) {
    if (t.ci % 4 != 0 || t.cpt != 1 || (a.colour == 1 && !a.th_red_new) || a.row_filter != 0)
      return hipErrorInvalidValue;
#define MR_HP_LAUNCH(TM, TJ)                                                                            \
    if (t.tm == TM && t.tj == TJ) {                                                                     \
      if (a.colour == 0 && !a.f)                                                                        \
        hipLaunchKernelGGL((half_sweep_pipe<TM, TJ, 0, false>), dim3(blocks), dim3(TM * TJ), 0, s, b);  \
      else if (a.colour == 0)                                                                           \
        hipLaunchKernelGGL((half_sweep_pipe<TM, TJ, 0, true>), dim3(blocks), dim3(TM * TJ), 0, s, b);   \
      else if (!a.f)                                                                                    \
        hipLaunchKernelGGL((half_sweep_pipe<TM, TJ, 1, false>), dim3(blocks), dim3(TM * TJ), 0, s, b);  \
      else                                                                                              \
        hipLaunchKernelGGL((half_sweep_pipe<TM, TJ, 1, true>), dim3(blocks), dim3(TM * TJ), 0, s, b);   \
      return hipGetLastError();                                                                         \
    }
    MR_HP_TILES(MR_HP_LAUNCH)
#undef MR_HP_LAUNCH
    return hipErrorInvalidValue;
  }
#define MR_HS_LAUNCH(TM, TJ, CPT)                                                                  \
  if (t.tm == TM && t.tj == TJ && t.cpt == CPT) {                                                  \
    hipLaunchKernelGGL((half_sweep_tiled<TM, TJ, CPT>), dim3(blocks), dim3(TM * TJ / CPT), 0, s, b); \
    return hipGetLastError();                                                                      \
  }
  MR_HS_TILES(MR_HS_LAUNCH)
#undef MR_HS_LAUNCH
  return hipErrorInvalidValue;
}

bool half_sweep_pipe_supported(int tm, int tj) {
#define MR_HP_MATCH(TM, TJ) if (tm == TM && tj == TJ) return true;
  MR_HP_TILES(MR_HP_MATCH)
#undef MR_HP_MATCH
  return false;
}

#define MR_DR_TILES(X) X(64, 8) X(64, 4) X(32, 8) X(32, 4) X(16, 8) X(8, 8) X(4, 8)

// Tile and chunk count of the pipelined defect + restriction (chunks are multiples of 4 planes).
struct DefectCfg {
  int tm = 0, tj = 0, nchunks = 0;
};
static std::mutex g_defect_tune_mu;
static std::map<std::tuple<int, int, bool>, DefectCfg> g_defect_tuned;   // (device, n, has f)

// Untimed choice: the compiled tile dividing the mesh with the most resident waves per CU (ties: the
// larger tile), and the largest number of chunks (at least 8 planes each) whose grid still fits in
// one round of the device's resident blocks. A timed choice (tune_defect) takes precedence.
static bool defect_pipe_cfg(int n, bool has_f, int& tm, int& tj, int& nchunks) {
  if (n % 8 != 0) return false;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  {
    std::lock_guard<std::mutex> lk(g_defect_tune_mu);
    auto it = g_defect_tuned.find(std::make_tuple(dev, n, has_f));
    if (it != g_defect_tuned.end()) {
      tm = it->second.tm;
      tj = it->second.tj;
      nchunks = it->second.nchunks;
      return true;
    }
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return false;
  int best_waves = 0, best_bpc = 0;
  auto consider = [&](int ctm, int ctj, const void* k) {
    if ((n / 2) % ctm != 0 || n % ctj != 0 || ctj > n) return;
    int bpc = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k, ctm * ctj, 0) != hipSuccess || bpc < 1) return;
    const int waves = bpc * ((ctm * ctj + 63) / 64);
    if (waves > best_waves || (waves == best_waves && ctm * ctj > tm * tj)) {
      best_waves = waves;
      best_bpc = bpc;
      tm = ctm;
      tj = ctj;
    }
  };
  tm = 0;
  tj = 0;
#define MR_DR_CONSIDER(TM, TJ)                                                                                \
  consider(TM, TJ, has_f ? reinterpret_cast<const void*>(&defect_restrict_pipe<TM, TJ, true>)                 \
                         : reinterpret_cast<const void*>(&defect_restrict_pipe<TM, TJ, false>));
  MR_DR_TILES(MR_DR_CONSIDER)
#undef MR_DR_CONSIDER
  if (best_waves == 0) return false;
  const long tiles = (long)(n / tj) * (n / 2 / tm);
  const long cap = (long)cus * best_bpc;
  long ch = cap / tiles;
  ch = std::max(1L, std::min(ch, (long)(n / 8)));
  while (ch > 1 && tiles * ch > kMaxReduceBlocks) --ch;
  if (tiles * ch > kMaxReduceBlocks) return false;
  nchunks = (int)ch;
  return true;
}

static hipError_t launch_defect_pipe(const DefectArgs& a, int tm, int tj, int nch, hipStream_t s) {
  const int n = a.n;
  if (tm < 1 || tj < 2 || (n / 2) % tm != 0 || n % tj != 0 || nch < 1 || nch > n / 8 || n % 8 != 0 ||
      (long)(n / tj) * (n / 2 / tm) * nch > kMaxReduceBlocks)
    return hipErrorInvalidValue;
  DefectArgs b = a;
  b.tj = tj;
  b.tiles_j = n / tj;
  b.tiles_m = n / 2 / tm;
  const unsigned blocks = (unsigned)(b.tiles_j * b.tiles_m * nch);
#define MR_DR_GO(TM, TJ)                                                                                   \
  if (tm == TM && tj == TJ) {                                                                              \
    if (a.f)                                                                                               \
      hipLaunchKernelGGL((defect_restrict_pipe<TM, TJ, true>), dim3(blocks), dim3(TM * TJ), 0, s, b, nch);  \
    else                                                                                                   \
      hipLaunchKernelGGL((defect_restrict_pipe<TM, TJ, false>), dim3(blocks), dim3(TM * TJ), 0, s, b, nch); \
    return hipGetLastError();                                                                              \
  }
  MR_DR_TILES(MR_DR_GO)
#undef MR_DR_GO
  return hipErrorInvalidValue;
}

// Times the pipelined defect + restriction on every compiled tile with 1 to n/8 chunks (powers of
// two, plus the occupancy-derived default) on the caller's buffers (the kernel only reads theta,
// delta, f and overwrites its outputs, so repeated launches are harmless) and caches the fastest
// per (device, n, f present).
int tune_defect(const DefectArgs& a, hipStream_t s) {
  const int n = a.n, nh = n / 2;
  const bool has_f = a.f != nullptr;
  int dev = 0;
  if (n % 8 != 0) return MR_OK;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorInvalidDevice, "defect tuner");
  {
    std::lock_guard<std::mutex> lk(g_defect_tune_mu);
    static int gen = -1;
    tuning_sync(gen, g_defect_tuned);
    if (g_defect_tuned.count(std::make_tuple(dev, n, has_f))) return MR_OK;
  }
  std::vector<DefectCfg> cand;
  int tm0 = 0, tj0 = 0, nch0 = 0;
  if (defect_pipe_cfg(n, has_f, tm0, tj0, nch0)) cand.push_back(DefectCfg{tm0, tj0, nch0});
  auto add = [&](int tm, int tj) {
    if (nh % tm != 0 || n % tj != 0 || tj > n) return;
    for (int nch = 1; nch <= n / 8; nch *= 2)
      if ((long)(n / tj) * (nh / tm) * nch <= kMaxReduceBlocks) cand.push_back(DefectCfg{tm, tj, nch});
  };
#define MR_DR_ADD(TM, TJ) add(TM, TJ);
  MR_DR_TILES(MR_DR_ADD)
#undef MR_DR_ADD
  if (cand.empty()) return MR_OK;
  const char* kind = has_f ? "defect64f.v1" : "defect64.v1";
  {
    std::vector<int> rec;
    if (tuning_lookup(kind, dev, n, rec))
      for (const DefectCfg& c : cand)
        if (rec == std::vector<int>{c.tm, c.tj, c.nchunks}) {
          std::lock_guard<std::mutex> lk(g_defect_tune_mu);
          g_defect_tuned[std::make_tuple(dev, n, has_f)] = c;
          return MR_OK;
        }
  }
  const size_t cells = (size_t)n * n * n;
  const int reps = cells >= ((size_t)1 << 24) ? 2 : 4;
  size_t bi = 0;
  const hipError_t e = pick_fastest(cand.size(), reps, s,
                                    [&](size_t i) { return launch_defect_pipe(a, cand[i].tm, cand[i].tj, cand[i].nchunks, s); },
                                    &bi);
  if (e != hipSuccess) return hip_fail(e, "defect tuner");
  {
    std::lock_guard<std::mutex> lk(g_defect_tune_mu);
    g_defect_tuned[std::make_tuple(dev, n, has_f)] = cand[bi];
  }
  tuning_record(kind, dev, n, {cand[bi].tm, cand[bi].tj, cand[bi].nchunks});
  return MR_OK;
}

hipError_t launch_defect_restrict_tiled(const DefectArgs& a, const TileCfg& t, hipStream_t s) {
  {
    int tm = 0, tj = 0, nch = 0;
    if (defect_pipe_cfg(a.n, a.f != nullptr, tm, tj, nch)) return launch_defect_pipe(a, tm, tj, nch, s);
  }
  const int threads = tile_threads(t, t.tm * (t.tj / 2));
  if (!tile_ok(t, a.n, threads) || t.tj % 2 != 0 || t.ci % 2 != 0) return hipErrorInvalidValue;
  DefectArgs b = a;
  b.tj = t.tj;
  b.tiles_j = t.tiles_j;
  b.tiles_m = t.tiles_m;
  b.ci = t.ci;
  const int blocks = t.tiles_j * t.tiles_m * (a.n / t.ci);
  const size_t lds = tile_lds_bytes(t.tj, t.tm);
  switch (t.tm) {
    case 2: hipLaunchKernelGGL(defect_restrict_kernel<2>, dim3(blocks), dim3(threads), lds, s, b); break;
    case 4: hipLaunchKernelGGL(defect_restrict_kernel<4>, dim3(blocks), dim3(threads), lds, s, b); break;
    case 8: hipLaunchKernelGGL(defect_restrict_kernel<8>, dim3(blocks), dim3(threads), lds, s, b); break;
    case 16: hipLaunchKernelGGL(defect_restrict_kernel<16>, dim3(blocks), dim3(threads), lds, s, b); break;
    case 32: hipLaunchKernelGGL(defect_restrict_kernel<32>, dim3(blocks), dim3(threads), lds, s, b); break;
    case 64: hipLaunchKernelGGL(defect_restrict_kernel<64>, dim3(blocks), dim3(threads), lds, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_coarsest(const CoarsestArgs& a, hipStream_t s) {
  if ((long)a.n * a.n * a.n > kMaxCoarsest) return hipErrorInvalidValue;
  hipLaunchKernelGGL(coarsest_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mr

namespace mr {

#define MR_FUSED_TILES(X) X(64, 16) X(64, 8) X(32, 16) X(32, 8) X(16, 16) X(16, 8) X(8, 8) X(8, 4) X(4, 8)

static const void* fused_kernel(int tm, int tj) {
#define MR_FZ_PTR(TM, TJ) \
  if (tm == TM && tj == TJ) return reinterpret_cast<const void*>(&sweep_fused<TM, TJ, true>);
  MR_FUSED_TILES(MR_FZ_PTR)
#undef MR_FZ_PTR
  return nullptr;
}

// Candidate configurations for an n^3 mesh: every compiled tile that fits, each with the chunk
// counts (chunks of at least 4 planes) whose fill * ci / (ci + 3) is within 15% of the best for
// that tile, where fill is the fraction of the device's resident block slots the grid occupies
// over its rounds and a chunk of ci planes takes ci + 3 plane steps. Ordered by that score.
static std::vector<std::pair<double, FusedCfg>> fused_candidates(int n) {
  std::vector<std::pair<double, FusedCfg>> out;
  static const int pref[][2] = {{64, 16}, {64, 8}, {32, 16}, {32, 8}, {16, 16}, {16, 8}, {8, 8}, {8, 4}, {4, 8}};
  const int nh = n / 2;
  int dev = 0, cus = 0;
  if (n < 8 || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return out;
  for (const auto& t : pref) {
    const int tm = t[0], tj = t[1];
    if (nh % tm != 0 || n % tj != 0) continue;
    const void* k = fused_kernel(tm, tj);
    int bpc = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k, tm * tj, 0) != hipSuccess || bpc < 1) continue;
    const long tiles = (long)(n / tj) * (nh / tm);
    const long cap = (long)cus * bpc;
    std::vector<std::pair<double, int>> ch;
    for (int c = 1; c <= n; ++c) {
      if (n / c < 4 && c > 1) break;
      const long blocks = tiles * c;
      if (blocks > kMaxReduceBlocks) break;
      const long rounds = (blocks + cap - 1) / cap;
      const double fill = (double)blocks / (double)(rounds * cap);
      const double ci = (double)n / c;
      ch.push_back({fill * ci / (ci + 3.0), c});
    }
    if (ch.empty()) continue;
    std::sort(ch.begin(), ch.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (size_t i = 0; i < ch.size() && i < 3 && ch[i].first >= 0.85 * ch[0].first; ++i) {
      FusedCfg c;
      c.tm = tm;
      c.tj = tj;
      c.tiles_j = n / tj;
      c.tiles_m = nh / tm;
      c.nchunks = ch[i].second;
      out.push_back({ch[i].first, c});
    }
  }
  std::stable_sort(out.begin(), out.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  return out;
}

bool fused_tile_supported(int tm, int tj) {
#define MR_FZ_MATCH(TM, TJ) if (tm == TM && tj == TJ) return true;
  MR_FUSED_TILES(MR_FZ_MATCH)
#undef MR_FZ_MATCH
  return false;
}

bool pick_fused(int n, FusedCfg& cfg) {
  const auto c = fused_candidates(n);
  if (c.empty()) return false;
  cfg = c.front().second;
  return true;
}

// Synthetic state for timing, colour-split: a potential of three periodic plane waves of about
// ten cells' wavelength whose Hessian is of order one (as in a converged solution of a strongly
// non-linear field, so that the root iteration counts are representative), and a lognormal-like
// density with the same contrast.
__global__ void tune_fill_kernel(double* __restrict__ th, double* __restrict__ delta, int n) {
  const int nh = n >> 1;
  const size_t half = (size_t)n * n * nh, cells = 2 * half;
  const double tw = 6.283185307179586 / n;
  const double sc = n / 10.0;
  const double k1[3] = {3.0 / 9.11, 5.0 / 9.11, 7.0 / 9.11}, k2[3] = {-4.0 / 6.71, 2.0 / 6.71, 5.0 / 6.71},
               k3[3] = {6.0 / 7.0, -3.0 / 7.0, 2.0 / 7.0};
  double w1[3], w2[3], w3[3];
  for (int d = 0; d < 3; ++d) {
    w1[d] = tw * fmax(1.0, rint(sc * k1[d] * (k1[d] < 0 ? -1.0 : 1.0))) * (k1[d] < 0 ? -1.0 : 1.0);
    w2[d] = tw * fmax(1.0, rint(sc * k2[d] * (k2[d] < 0 ? -1.0 : 1.0))) * (k2[d] < 0 ? -1.0 : 1.0);
    w3[d] = tw * fmax(1.0, rint(sc * k3[d] * (k3[d] < 0 ? -1.0 : 1.0))) * (k3[d] < 0 ? -1.0 : 1.0);
  }
  const double a1 = 0.8 / (w1[0] * w1[0] + w1[1] * w1[1] + w1[2] * w1[2]);
  const double a2 = 0.8 / (w2[0] * w2[0] + w2[1] * w2[1] + w2[2] * w2[2]);
  const double a3 = 0.8 / (w3[0] * w3[0] + w3[1] * w3[1] + w3[2] * w3[2]);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / half);
    const size_t rem = e - c * half;
    const int i = (int)(rem / ((size_t)n * nh));
    const int j = (int)((rem / nh) % n);
    const int m = (int)(rem % nh);
    const int k = 2 * m + ((i + j + c) & 1);
    const double x = i, y = j, z = k;
    th[e] = a1 * sin(w1[0] * x + w1[1] * y + w1[2] * z) + a2 * sin(w2[0] * x + w2[1] * y + w2[2] * z + 1.0) +
            a3 * sin(w3[0] * x + w3[1] * y + w3[2] * z + 2.0);
    delta[e] = exp(0.9 * sin(w2[0] * z - w1[1] * x + w3[2] * y + 0.5) - 0.405) - 1.0;
  }
}

static std::mutex g_sweep_tune_mu;
static std::map<std::pair<int, int>, std::pair<bool, FusedCfg>> g_sweep_tuned;   // (device, n)
static std::map<std::pair<int, int>, TileCfg> g_half_tuned;                       // (device, n)

bool tuned_sweep(int n, FusedCfg* cfg) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_sweep_tune_mu);
  auto it = g_sweep_tuned.find({dev, n});
  if (it == g_sweep_tuned.end() || !it->second.first) return false;
  *cfg = it->second.second;
  return true;
}

// Every schedule the sweep tuner times for an n^3 level: two launches per sweep with the general
// kernel on the default tile `two`, two launches with the pipelined kernel on every compiled tile that
// fits with chunks of 16 to 256 planes, and the fused launch on the candidates of fused_candidates.
std::vector<SweepCand> sweep_candidates(int n, const TileCfg& two) {
  std::vector<SweepCand> all{SweepCand{false, two, FusedCfg{}}};
  auto add_pipe = [&](int tm, int tj) {
    if ((n / 2) % tm != 0 || n % tj != 0 || tj > n) return;
    for (int ci = 16; ci <= 256 && ci <= n; ci *= 2) {
      TileCfg tp;
      tp.tm = tm;
      tp.tj = tj;
      tp.cpt = 1;
      tp.ci = ci;
      tp.tiles_j = n / tj;
      tp.tiles_m = (n / 2) / tm;
      tp.pipe = true;
      const long blocks = (long)tp.tiles_j * tp.tiles_m * (n / ci);
      if (n % ci == 0 && blocks <= kMaxReduceBlocks) all.push_back(SweepCand{false, tp, FusedCfg{}});
    }
  };
#define MR_HP_ADD(TM, TJ) add_pipe(TM, TJ);
  MR_HP_TILES(MR_HP_ADD)
#undef MR_HP_ADD
  for (const auto& c : fused_candidates(n)) all.push_back(SweepCand{true, two, c.second});
  return all;
}

int tune_sweep(int n, double* th_a, double* th_b, double* delta, double* partials, unsigned* counter, double* sums,
               TileCfg* two, hipStream_t s, bool* use_fused, FusedCfg* cfg) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorInvalidDevice, "sweep tuner");
  {
    std::lock_guard<std::mutex> lk(g_sweep_tune_mu);
    static int gen = -1, gen_half = -1;
    tuning_sync(gen, g_sweep_tuned);
    tuning_sync(gen_half, g_half_tuned);
    auto it = g_sweep_tuned.find({dev, n});
    if (it != g_sweep_tuned.end()) {
      *use_fused = it->second.first;
      *cfg = it->second.second;
      auto jt = g_half_tuned.find({dev, n});
      if (jt != g_half_tuned.end()) *two = jt->second;
      return MR_OK;
    }
  }
  const size_t cells = (size_t)n * n * n;
  hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, s, th_a, delta, n);
  hipError_t e = hipGetLastError();
  const int reps = cells >= ((size_t)1 << 24) ? 2 : 4;
  FusedCfg best_cfg;
  bool best_fused = false;
  const std::vector<SweepCand> all = sweep_candidates(n, *two);
  // a recorded choice (this or an earlier process) that is still a candidate
  const TileCfg def_two = *two;
  auto code = [&](const SweepCand& c) {
    std::vector<int> v{c.fused ? 1 : 0};
    for (int x : tile_code(c.fused ? def_two : c.two)) v.push_back(x);
    const FusedCfg f = c.fused ? c.fz : FusedCfg{};
    for (int x : {f.tm, f.tj, f.tiles_j, f.tiles_m, f.nchunks}) v.push_back(x);
    return v;
  };
  {
    std::vector<int> rec;
    if (tuning_lookup("sweep64.v1", dev, n, rec))
      for (const SweepCand& c : all)
        if (code(c) == rec) {
          *use_fused = c.fused;
          *cfg = c.fused ? c.fz : FusedCfg{};
          if (!c.fused) *two = c.two;
          std::lock_guard<std::mutex> lk(g_sweep_tune_mu);
          g_sweep_tuned[{dev, n}] = {*use_fused, *cfg};
          g_half_tuned[{dev, n}] = *two;
          return MR_OK;
        }
  }
  using Cand = SweepCand;
  auto run = [&](const Cand& c) -> hipError_t {
    if (c.fused) {
      FusedSweepArgs a{};
      a.th_in = th_a;
      a.th_out = th_b;
      a.delta = delta;
      a.n = n;
      a.h2 = 1.0;
      a.ih2 = 1.0;
      a.sum_out = sums;
      a.partials = partials;
      a.counter = counter;
      return launch_sweep_fused(a, c.fz, s);
    }
    HalfSweepArgs a{};
    a.th_in = th_a;
    a.th_out = th_b;
    a.delta = delta;
    a.n = n;
    a.h2 = 1.0;
    a.ih2 = 1.0;
    a.partials = partials;
    a.counter = counter;
    a.colour = 0;
    a.sum_out = sums;
    hipError_t x = launch_half_sweep(a, c.two, s);
    a.colour = 1;
    a.th_red_new = th_b;
    a.sum_out = sums + 1;
    return x == hipSuccess ? launch_half_sweep(a, c.two, s) : x;
  };
  size_t bk = 0;
  if (e == hipSuccess) e = pick_fastest(all.size(), reps, s, [&](size_t i) { return run(all[i]); }, &bk);
  // when the fused launch wins, the two-launch schedule (used only on request, MR_FLAG_TWO_PASS)
  // stays the default tile
  TileCfg best_two = *two;
  if (!all.empty()) {
    best_fused = all[bk].fused;
    if (best_fused) {
      best_cfg = all[bk].fz;
    } else {
      best_two = all[bk].two;
    }
  }
  if (e != hipSuccess) return hip_fail(e, "sweep tuner");
  {
    std::lock_guard<std::mutex> lk(g_sweep_tune_mu);
    g_sweep_tuned[{dev, n}] = {best_fused, best_cfg};
    g_half_tuned[{dev, n}] = best_two;
  }
  if (!all.empty()) tuning_record("sweep64.v1", dev, n, code(all[bk]));
  *use_fused = best_fused;
  *cfg = best_cfg;
  *two = best_two;
  return MR_OK;
}

hipError_t launch_sweep_fused(const FusedSweepArgs& a, const FusedCfg& cfg, hipStream_t s) {
  const long blocks = (long)cfg.tiles_j * cfg.tiles_m * cfg.nchunks;
  if (blocks < 1 || blocks > kMaxReduceBlocks || cfg.tj * cfg.tiles_j != a.n || cfg.tm * cfg.tiles_m != a.n / 2 ||
      cfg.nchunks > a.n)
    return hipErrorInvalidValue;
  FusedSweepArgs b = a;
  b.tiles_j = cfg.tiles_j;
  b.tiles_m = cfg.tiles_m;
  b.nchunks = cfg.nchunks;
#define MR_FZ_LAUNCH(TM, TJ)                                                                           \
  if (cfg.tm == TM && cfg.tj == TJ) {                                                                  \
    if (b.f)                                                                                           \
      hipLaunchKernelGGL((sweep_fused<TM, TJ, true>), dim3((unsigned)blocks), dim3(TM * TJ), 0, s, b);  \
    else                                                                                               \
      hipLaunchKernelGGL((sweep_fused<TM, TJ, false>), dim3((unsigned)blocks), dim3(TM * TJ), 0, s, b); \
    return hipGetLastError();                                                                          \
  }
  MR_FUSED_TILES(MR_FZ_LAUNCH)
#undef MR_FZ_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace mr
