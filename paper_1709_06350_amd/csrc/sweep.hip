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
#include "mr_device.h"
#include "mr_kernels.h"

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
      out[e] = (Ssum - h2 * (sig + fc - C)) * (1.0 / 6.0);
      acc += sig + fc;
    }
    if (pre) store(i + 2, v);
    __syncthreads();
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
#define MR_HS_LAUNCH(TM, TJ, CPT)                                                                  \
  if (t.tm == TM && t.tj == TJ && t.cpt == CPT) {                                                  \
    hipLaunchKernelGGL((half_sweep_tiled<TM, TJ, CPT>), dim3(blocks), dim3(TM * TJ / CPT), 0, s, b); \
    return hipGetLastError();                                                                      \
  }
  MR_HS_TILES(MR_HS_LAUNCH)
#undef MR_HS_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_defect_restrict_tiled(const DefectArgs& a, const TileCfg& t, hipStream_t s) {
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
