// Mixed-precision form of the solve: an FP64 defect-correction (Newton) outer loop on the finest
// mesh around an FP32 linear multigrid for the Jacobian of the mean-projected operator.
//
// Outer step: r = -F(theta) in FP64 (F the mean-projected operator of Sec. II.A.1, Eq. 15; the
// residual also decides convergence), then J_p e = r is solved approximately by FP32 V-cycles,
// and theta += e in FP64. Representing e separately keeps FP32 rounding out of theta itself.
//
// Linearisation (differentiating the physical root of the cubic, Sec. II, Eqs. 8-10):
// dSigma(e) = tr(W dMbar(e)), W = (9 s Mbar - 27 Mbar^2) / (3 s^2 + p), so with the traceless
// part Wbar of W, h^2 dSigma(e) = sum_a Wbar_aa S_a(e) + sum_{a<b} W_ab D_ab(e) / 2 (S_a the pair
// sum along axis a, D_ab the cross difference of e). The Jacobian J_p e = nabla^2 e - dSigma(e)
// + <dSigma(e)> keeps the -6/h^2 diagonal of the nonlinear operator, so the inner smoother is the
// same red-black point update with the source replaced by dSigma(e) and no root finding:
//     e_c <- (sum of 6 face neighbours of e - h^2 (dSigma_c(e) + rhs_c - C)) / 6.
// W is rebuilt on the fly in every sweep from an FP32 copy of the base potential (both colours in
// LDS with e) and the FP32 base root s; coarse meshes use the restricted base potential and
// their own root (rediscretisation).
#include <algorithm>
#include <type_traits>

#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"
#include "mixed_device.h"

namespace mr {

// Compiled tile shapes (tm columns of m, tj rows) of the FP32 linear sweeps.
#define MR_LIN_TILES(X) X(64, 8) X(64, 4) X(32, 16) X(32, 8) X(16, 16) X(8, 16) X(4, 8) X(2, 4)

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) lin_half_sweep_tiled(LinSweepArgs a) {
  __shared__ float lds[LinTile<TM, TJ>::LDS];
  lin_sweep_body<TM, TJ>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(256) mixed_resid64_kernel(const double* __restrict__ theta,
    const double* __restrict__ delta, int n, ShiftRef cref, float* __restrict__ rhs32, float* __restrict__ base32,
    float* __restrict__ sb32, Reduce red) {
  mixed_resid64_body(theta, delta, n, cref, rhs32, base32, sb32, red, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) base_root_kernel(const float* __restrict__ base32,
    const double* __restrict__ delta, int n, double ih2, float* __restrict__ sb32) {
  base_root_body(base32, delta, n, ih2, sb32, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(512) restrict32_kernel(const float* __restrict__ fine, float* __restrict__ coarse, int n) {
  restrict32_body(fine, coarse, n, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) lin_resid_restrict_kernel(const float* __restrict__ e,
    const float* __restrict__ base, const float* __restrict__ sb, const float* __restrict__ rhs, int n, float ih2,
    ShiftRef cref, float* __restrict__ rhs_c, Reduce red) {
  lin_resid_restrict_body(e, base, sb, rhs, n, ih2, cref, rhs_c, red, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(512) prolong_add32_kernel(const float* __restrict__ ec, float* __restrict__ e, int n) {
  prolong_add32_body(ec, e, n, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) lin_coarsest_kernel(float* __restrict__ e, const float* __restrict__ base,
    const float* __restrict__ sb, const float* __restrict__ rhs, int n, int nsweeps, float h2, float ih2,
    const double* c_sum, double c_scale) {
  __shared__ LinCoarsestShared sh;
  lin_coarsest_body(e, base, sb, rhs, n, nsweeps, h2, ih2, c_sum, c_scale, sh);
}

__global__ void __launch_bounds__(256) update64_kernel(double* __restrict__ theta, const float* __restrict__ e, size_t cells) {
  update64_body(theta, e, cells, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) fill32_kernel(float* __restrict__ a, float v, size_t cells) {
  fill32_body(a, v, cells, blockIdx.x, gridDim.x);
}

// ---- pipelined FP32 linear half-sweep --------------------------------------------------------
// lin_sweep_body's decomposition and arithmetic with the colour compile-time and the plane loop
// unrolled by the ring length (compile-time LDS slots); planes are fetched two steps before they
// enter LDS and the base root / right-hand side two steps before use. Requires ci % 4 == 0.
template <int TM, int TJ, int COL>
__global__ void __launch_bounds__(TM * TJ) lin_sweep_pipe(LinSweepArgs a) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2;
  constexpr int SLOT = LinTile<TM, TJ>::SLOT;
  constexpr int PER = (SLOT + NT - 1) / NT;   // loads per field and thread
  constexpr int NPF = 4 * PER;
  constexpr int O = 1 - COL;
  __shared__ float lds[LinTile<TM, TJ>::LDS];
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tm_i = logical % a.tiles_m;
  const int tj_i = (logical / a.tiles_m) % a.tiles_j;
  const int chunk = logical / (a.tiles_m * a.tiles_j);
  const int j0 = tj_i * TJ, m0 = tm_i * TM, i0 = chunk * a.ci, ci = a.ci;
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
  const float* __restrict__ f0 = COL == 1 ? a.e_red_new : a.e_in;   // e red
  const float* __restrict__ f1 = a.e_in + half;                      // e black
  const float* __restrict__ f2 = a.base;                             // base red
  const float* __restrict__ f3 = a.base + half;                      // base black

  // loader: element k of field f is f * SLOT + (k % PER) * NT + tid (clamped inside the field), so
  // that the source field of every load is a compile-time constant
  unsigned goff[PER];
  int loff[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int e = tid + k * NT;
    e = e < SLOT ? e : SLOT - 1;
    const int r = e / RW;
    const int c = e - r * RW;
    goff[k] = (unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh);
    loff[k] = e;
  }
  auto fetch = [&](int rel, float (&v)[NPF]) {
    const unsigned base = (unsigned)wrapi(i0 - 1 + rel, n) * plane;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[0 * PER + k] = f0[base + goff[k]];
      v[1 * PER + k] = f1[base + goff[k]];
      v[2 * PER + k] = f2[base + goff[k]];
      v[3 * PER + k] = f3[base + goff[k]];
    }
  };
  auto store = [&](int slot, const float (&v)[NPF]) {
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int k = 0; k < PER; ++k) lds[(f * 4 + slot) * SLOT + loff[k]] = v[f * PER + k];
  };

  const int s = tid % TM, r = tid / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned own = (unsigned)j * nh + m;
  const int ob = (r + 1) * RW + (s + 1);
  const int q0 = (i0 + j + COL) & 1;
  const int oq0 = ob + q0, oq1 = ob + (q0 ^ 1);
  const double Cd = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const float C = (float)Cd;
  const float h2 = a.h2, ih2 = a.ih2;
  const float* __restrict__ sbc = a.sb + COL * half + own;
  const float* __restrict__ rc = a.rhs + COL * half + own;
  float* __restrict__ out = a.e_out + COL * half + own;
  const int last_plane = n - 1;
  double acc = 0.0;

  float V0[NPF], V1[NPF];
  float SB[4], RH[4];
  {
    float va[NPF], vb[NPF], vc[NPF];
    fetch(0, va);
    fetch(1, vb);
    fetch(2, vc);
    store(0, va);
    store(1, vb);
    store(2, vc);
  }
  fetch(3, V0);
  SB[0] = sbc[(unsigned)i0 * plane];
  RH[0] = rc[(unsigned)i0 * plane];
  SB[1] = sbc[(unsigned)min(i0 + 1, last_plane) * plane];
  RH[1] = rc[(unsigned)min(i0 + 1, last_plane) * plane];
  __syncthreads();

  auto step = [&](auto kc, int t, float (&vst)[NPF], float (&vft)[NPF]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = K & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    const unsigned pn = (unsigned)min(i0 + t + 2, last_plane) * plane;
    SB[(K + 2) & 3] = sbc[pn];
    RH[(K + 2) & 3] = rc[pn];
    const int oq = (K & 1) ? oq1 : oq0;
    Nb18f te, tb;
#define MR_LP_GATHER(T, LO, LC)                                                        \
    {                                                                                  \
      const float* lo = lds + (LO) * 4 * SLOT;                                          \
      const float* lc = lds + (LC) * 4 * SLOT;                                          \
      T.xm = lo[SM * SLOT + ob];         T.xp = lo[SP * SLOT + ob];                     \
      T.ym = lo[S0 * SLOT + ob - RW];    T.yp = lo[S0 * SLOT + ob + RW];                \
      T.zm = lo[S0 * SLOT + oq - 1];     T.zp = lo[S0 * SLOT + oq];                     \
      T.xpyp = lc[SP * SLOT + ob + RW];  T.xmym = lc[SM * SLOT + ob - RW];              \
      T.xpym = lc[SP * SLOT + ob - RW];  T.xmyp = lc[SM * SLOT + ob + RW];              \
      T.xpzp = lc[SP * SLOT + oq];       T.xmzm = lc[SM * SLOT + oq - 1];               \
      T.xpzm = lc[SP * SLOT + oq - 1];   T.xmzp = lc[SM * SLOT + oq];                   \
      T.ypzp = lc[S0 * SLOT + oq + RW];  T.ymzm = lc[S0 * SLOT + oq - RW - 1];          \
      T.ypzm = lc[S0 * SLOT + oq + RW - 1]; T.ymzp = lc[S0 * SLOT + oq - RW];           \
    }
    MR_LP_GATHER(te, O, COL)
    MR_LP_GATHER(tb, 2 + O, 2 + COL)
#undef MR_LP_GATHER
    float Se;
    const float g = lin_source(tb, SB[K], ih2, te, Se) * ih2;
    const float rhs = RH[K];
    out[(unsigned)(i0 + t) * plane] = (Se - h2 * (g + rhs - C)) * (1.0f / 6.0f);
    acc += (double)(g + rhs);
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

// ---- tiled linear residual + restriction ---------------------------------------------------
// lin_resid_restrict_body's outputs on a 2.5D tile: e and the base potential (both colours) of
// planes i-1..i+1 in a 4-slot LDS ring; a thread owns fine rows 2J, 2J+1 and the cell pair
// k = 2m, 2m+1 (both colours of column m), so over planes 2I, 2I+1 it holds the 8 sons of coarse
// cell (I, J, m) and writes their mean residual after the odd plane. Chunks are multiples of 4
// planes; the plane loop is unrolled by the ring length (compile-time slots) with planes fetched
// two steps ahead.
struct LinRRArgs {
  const float* e;
  const float* base;
  const float* sb;
  const float* rhs;
  int n;
  float ih2;
  ShiftRef cref;
  float* rhs_c;
  Reduce red;
  int tiles_j, tiles_m, nchunks;
};

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ / 2) lin_resid_restrict_tiled(LinRRArgs a) {
  constexpr int NT = TM * TJ / 2;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int PER = (SLOT + NT - 1) / NT;   // loads per field and thread
  constexpr int NPF = 4 * PER;
  __shared__ float lds[4 * 4 * SLOT];
  const int n = a.n, nh = n >> 1, nc = n >> 1, nch = nc >> 1;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = a.tiles_m * a.tiles_j;
  const int tile = logical % ntile, chunk = logical / ntile;
  const int m0 = (tile % a.tiles_m) * TM, j0 = (tile / a.tiles_m) * TJ;
  const int q4 = n / 4;
  const int i0 = 4 * (int)(((long)chunk * q4) / a.nchunks);
  const int i1 = 4 * (int)(((long)(chunk + 1) * q4) / a.nchunks);
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
  const unsigned halfc = (unsigned)nc * (unsigned)nc * (unsigned)nch;
  const float* __restrict__ f0 = a.e;
  const float* __restrict__ f1 = a.e + half;
  const float* __restrict__ f2 = a.base;
  const float* __restrict__ f3 = a.base + half;

  // loader: element k of field f is f * SLOT + (k % PER) * NT + tid (clamped inside the field), so
  // that the source field of every load is a compile-time constant
  unsigned goff[PER];
  int loff[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int e = tid + k * NT;
    e = e < SLOT ? e : SLOT - 1;
    const int r = e / RW;
    const int c = e - r * RW;
    goff[k] = (unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh);
    loff[k] = e;
  }
  auto fetch = [&](int rel, float (&v)[NPF]) {
    const unsigned base = (unsigned)wrapi(i0 - 1 + rel, n) * plane;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[0 * PER + k] = f0[base + goff[k]];
      v[1 * PER + k] = f1[base + goff[k]];
      v[2 * PER + k] = f2[base + goff[k]];
      v[3 * PER + k] = f3[base + goff[k]];
    }
  };
  auto store = [&](int slot, const float (&v)[NPF]) {
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int k = 0; k < PER; ++k) lds[(f * 4 + slot) * SLOT + loff[k]] = v[f * PER + k];
  };

  const int s = tid % TM, rr = tid / TM;            // coarse row within the tile
  const int m = m0 + s;
  const double Cd = (a.cref.c_sum ? (a.cref.c_sum[0] + a.cref.c_sum[1]) * a.cref.c_scale : 0.0) + a.cref.c_add;
  const float C = (float)Cd;
  const float ih2 = a.ih2;
  double acc = 0.0;
  float sres = 0.0f;

  float V0[NPF], V1[NPF];
  {
    float va[NPF], vb[NPF], vc[NPF];
    fetch(0, va);
    fetch(1, vb);
    fetch(2, vc);
    store(0, va);
    store(1, vb);
    store(2, vc);
  }
  fetch(3, V0);
  __syncthreads();

  auto step = [&](auto kc, int t, float (&vst)[NPF], float (&vft)[NPF]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = K & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    const int i = i0 + t;
#pragma unroll 1
    for (int cell = 0; cell < 4; ++cell) {
      const int dr = cell >> 1, c = cell & 1;
      const int r = 2 * rr + dr;
      const int j = j0 + r;
      const int ob = (r + 1) * RW + (s + 1);
      const unsigned o = (unsigned)c * half + (unsigned)i * plane + (unsigned)j * nh + m;
      const float sbv = a.sb[o], rhv = a.rhs[o];
      {
        const int q = (i + j + c) & 1;
        const int oq = ob + q;
        const int O = 1 - c;
        Nb18f te, tb;
#define MR_RR_GATHER(T, LO, LC)                                                        \
        {                                                                              \
          const float* lo = lds + (LO) * 4 * SLOT;                                      \
          const float* lc = lds + (LC) * 4 * SLOT;                                      \
          T.xm = lo[SM * SLOT + ob];         T.xp = lo[SP * SLOT + ob];                 \
          T.ym = lo[S0 * SLOT + ob - RW];    T.yp = lo[S0 * SLOT + ob + RW];            \
          T.zm = lo[S0 * SLOT + oq - 1];     T.zp = lo[S0 * SLOT + oq];                 \
          T.xpyp = lc[SP * SLOT + ob + RW];  T.xmym = lc[SM * SLOT + ob - RW];          \
          T.xpym = lc[SP * SLOT + ob - RW];  T.xmyp = lc[SM * SLOT + ob + RW];          \
          T.xpzp = lc[SP * SLOT + oq];       T.xmzm = lc[SM * SLOT + oq - 1];           \
          T.xpzm = lc[SP * SLOT + oq - 1];   T.xmzp = lc[SM * SLOT + oq];               \
          T.ypzp = lc[S0 * SLOT + oq + RW];  T.ymzm = lc[S0 * SLOT + oq - RW - 1];      \
          T.ypzm = lc[S0 * SLOT + oq + RW - 1]; T.ymzp = lc[S0 * SLOT + oq - RW];       \
        }
        MR_RR_GATHER(te, O, c)
        MR_RR_GATHER(tb, 2 + O, 2 + c)
#undef MR_RR_GATHER
        float Se;
        const float src = lin_source(tb, sbv, ih2, te, Se) * ih2;
        const float ec = lds[(c * 4 + S0) * SLOT + ob];
        const float lap = (Se - 6.0f * ec) * ih2;
        sres += rhv + src - lap - C;
      }
    }
    if (K & 1) {   // odd plane (chunks start at even planes): the coarse cell is complete
      const int I = i >> 1, J = (j0 >> 1) + rr, Kc = m;
      const unsigned ec = ((I + J + Kc) & 1) * halfc + ((unsigned)I * nc + J) * (unsigned)nch + (unsigned)(Kc >> 1);
      const float v = 0.125f * sres;
      a.rhs_c[ec] = v;
      acc += v;
      sres = 0.0f;
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
  grid_sum<2>(vv, a.red.partials, a.red.counter, a.red.result, gridDim.x, blockIdx.x);
}

#define MR_RR_TILES(X) X(64, 8) X(32, 8) X(16, 8) X(8, 8) X(4, 8)

static const void* rr_tiled_kernel(int tm, int tj) {
#define MR_RR_PTR(TM, TJ) \
  if (tm == TM && tj == TJ) return reinterpret_cast<const void*>(&lin_resid_restrict_tiled<TM, TJ>);
  MR_RR_TILES(MR_RR_PTR)
#undef MR_RR_PTR
  return nullptr;
}

// ---- tiled FP64 outer residual ------------------------------------------------------------
// The same outputs as mixed_resid64_body, on the 2.5D decomposition of the sweeps: a block owns a
// TM x TJ tile of (m, j) and a chunk of planes [i0, i1) (a multiple of 4 long); both colours of
// theta for planes i-1..i+1 sit in a 4-slot LDS ring. Per plane step a thread evaluates the two
// cells of its (j, m) column (one per colour), so that two independent roots overlap. The plane
// loop is unrolled by the ring length (compile-time slots), planes are fetched two steps before
// they enter LDS and delta two steps before use.
struct ResidTiledArgs {
  const double* theta;
  const double* delta;
  int n;
  ShiftRef cref;
  float* rhs32;
  float* base32;
  float* sb32;
  Reduce red;
  int tiles_j, tiles_m, nchunks;
};

template <int TM, int TJ>
__global__ void __launch_bounds__(TM * TJ) mixed_resid64_tiled(ResidTiledArgs a) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int TOTAL = 2 * SLOT;
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  __shared__ double lds[2 * 4 * SLOT];
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = a.tiles_m * a.tiles_j;
  const int tile = logical % ntile, chunk = logical / ntile;
  const int m0 = (tile % a.tiles_m) * TM, j0 = (tile / a.tiles_m) * TJ;
  const int q4 = n / 4;
  const int i0 = 4 * (int)(((long)chunk * q4) / a.nchunks);
  const int i1 = 4 * (int)(((long)(chunk + 1) * q4) / a.nchunks);
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
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
  // z-parity of the colour-c cell of this column at plane i0 + t: (i0 + j + c + t) & 1
  const int qa = (i0 + j) & 1;
  const int oq00 = ob + qa, oq01 = ob + (qa ^ 1);          // colour 0 at even / odd t
  const double C = (a.cref.c_sum ? (a.cref.c_sum[0] + a.cref.c_sum[1]) * a.cref.c_scale : 0.0) + a.cref.c_add;
  const double* __restrict__ dl = a.delta + own;
  const int last_plane = n - 1;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;

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
  D[0][0] = dl[(unsigned)i0 * plane];
  D[0][1] = dl[half + (unsigned)i0 * plane];
  D[1][0] = dl[(unsigned)min(i0 + 1, last_plane) * plane];
  D[1][1] = dl[half + (unsigned)min(i0 + 1, last_plane) * plane];
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
    const double* l0 = lds;              // colour 0
    const double* l1 = lds + 4 * SLOT;   // colour 1
    // colour 0 cell: parity q = (i + j) & 1; colour 1 cell: the opposite parity
    const int oqc0 = (K & 1) ? oq01 : oq00;
    const int oqc1 = (K & 1) ? oq00 : oq01;
    Nb18 c0, c1;
    gather(l1, l0, SM, S0, SP, oqc0, c0);
    gather(l0, l1, SM, S0, SP, oqc1, c1);
    double S[2], pp[2], qq[2], sr[2];
    cell_pq(c0, 1.0 + D[K][0], 1.0, S[0], pp[0], qq[0]);
    cell_pq(c1, 1.0 + D[K][1], 1.0, S[1], pp[1], qq[1]);
    largest_roots<2>(pp, qq, sr);
    const unsigned e0 = (unsigned)(i0 + t) * plane + own;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double thc = (c == 0 ? l0 : l1)[S0 * SLOT + ob];
      const double sig = sr[c] - 3.0;
      const double b = (S[c] - 6.0 * thc) - sig + C;
      const unsigned e = (unsigned)c * half + e0;
      a.rhs32[e] = (float)(-b);
      a.base32[e] = (float)thc;
      a.sb32[e] = (float)sr[c];
      a0 += b;
      a1 += b * b;
      a2 += sig;
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
  double v[4] = {a2, 0.0, a0, a1};
  grid_sum<4>(v, a.red.partials, a.red.counter, a.red.result, gridDim.x, blockIdx.x);
}

#define MR_RT_TILES(X) X(64, 8) X(32, 8) X(16, 8) X(8, 8) X(4, 8)

static const void* resid_tiled_kernel(int tm, int tj) {
#define MR_RT_PTR(TM, TJ) \
  if (tm == TM && tj == TJ) return reinterpret_cast<const void*>(&mixed_resid64_tiled<TM, TJ>);
  MR_RT_TILES(MR_RT_PTR)
#undef MR_RT_PTR
  return nullptr;
}

// Tile and chunking of a 2.5D kernel for an n^3 mesh: the largest tile (tm x tj of (m, j),
// threads = tm * tj / per) that divides the mesh, the plane axis split in units of 4 planes so
// that the grid fills whole waves of the device's resident block slots as well as possible.
// Returns false when no tile applies.
static const int kPref8[][2] = {{64, 8}, {32, 8}, {16, 8}, {8, 8}, {4, 8}};

template <typename Get, size_t NP>
static bool tiled_cfg(int n, Get get, int per, int& tm, int& tj, int& nchunks, const int (&pref)[NP][2]) {
  if (n % 8 != 0) return false;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return false;
  for (const auto& t : pref) {
    if ((n / 2) % t[0] != 0 || n % t[1] != 0) continue;
    int bpc = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, get(t[0], t[1]), t[0] * t[1] / per, 0) != hipSuccess ||
        bpc < 1)
      continue;
    const long tiles = (long)(n / t[1]) * (n / 2 / t[0]);
    const long cap = (long)cus * bpc;
    double best = -1.0;
    int bc = 1;
    for (int c = 1; c <= n / 4; ++c) {
      const long blocks = tiles * c;
      if (blocks > kMaxReduceBlocks) break;
      const long rounds = (blocks + cap - 1) / cap;
      const double fill = (double)blocks / (double)(rounds * cap);
      const double ci = (double)n / c;
      const double eff = fill * ci / (ci + 3.0);
      if (eff > best + 1e-9) {
        best = eff;
        bc = c;
      }
    }
    tm = t[0];
    tj = t[1];
    nchunks = bc;
    return true;
  }
  return false;
}

static bool resid_tiled_cfg(int n, int& tm, int& tj, int& nchunks) {
  return tiled_cfg(n, resid_tiled_kernel, 1, tm, tj, nchunks, kPref8);
}

// Inner shift of level 0 from the outer residual sums: (sum of rhs, 0) = (-sum b, 0).
__global__ void inner_shift_kernel(const double* __restrict__ res, double* __restrict__ lsum0) {
  if (threadIdx.x == 0) {
    lsum0[0] = -res[2];
    lsum0[1] = 0.0;
  }
}

// ---- launchers ----------------------------------------------------------------------------

static int lin_blocks(size_t cells) {
  size_t b = (cells + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}
static int rows_blocks(int n) { return n * n < 4096 ? n * n : 4096; }
static int row_threads(int n) { return n < 64 ? 64 : (n < 256 ? n : 256); }


bool lin_tile_supported(int tm, int tj) {
#define MR_LIN_MATCH(TM, TJ) if (tm == TM && tj == TJ) return true;
  MR_LIN_TILES(MR_LIN_MATCH)
#undef MR_LIN_MATCH
  return false;
}

hipError_t launch_lin_half_sweep(const LinSweepArgs& a, const TileCfg& t, hipStream_t s) {
  const long blocks_l = (long)t.tiles_j * t.tiles_m * (a.n / std::max(t.ci, 1));
  if (blocks_l < 1 || blocks_l > kMaxReduceBlocks || t.tj * t.tiles_j != a.n || t.tm * t.tiles_m != a.n / 2 ||
      t.ci < 1 || a.n % t.ci != 0)
    return hipErrorInvalidValue;
  LinSweepArgs b = a;
  b.tiles_j = t.tiles_j;
  b.tiles_m = t.tiles_m;
  b.ci = t.ci;
  const int blocks = (int)blocks_l;
  if (t.pipe) {
    if (b.ci % 4 != 0 || (a.colour == 1 && !a.e_red_new)) return hipErrorInvalidValue;
#define MR_LP_LAUNCH(TM, TJ)                                                                          \
    if (t.tm == TM && t.tj == TJ) {                                                                   \
      if (a.colour == 0)                                                                              \
        hipLaunchKernelGGL((lin_sweep_pipe<TM, TJ, 0>), dim3(blocks), dim3(TM * TJ), 0, s, b);        \
      else                                                                                            \
        hipLaunchKernelGGL((lin_sweep_pipe<TM, TJ, 1>), dim3(blocks), dim3(TM * TJ), 0, s, b);        \
      return hipGetLastError();                                                                       \
    }
    MR_LIN_TILES(MR_LP_LAUNCH)
#undef MR_LP_LAUNCH
    return hipErrorInvalidValue;
  }
#define MR_LIN_LAUNCH(TM, TJ)                                                                  \
  if (t.tm == TM && t.tj == TJ) {                                                              \
    hipLaunchKernelGGL((lin_half_sweep_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ), 0, s, b);  \
    return hipGetLastError();                                                                  \
  }
  MR_LIN_TILES(MR_LIN_LAUNCH)
#undef MR_LIN_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_mixed_resid64(const double* theta, const double* delta, int n, ShiftRef C, float* rhs32, float* base32,
                                float* sb32, Reduce red, hipStream_t s) {
  int tm = 0, tj = 0, nch = 0;
  if (resid_tiled_cfg(n, tm, tj, nch)) {
    ResidTiledArgs a{theta, delta, n, C, rhs32, base32, sb32, red, n / tj, n / 2 / tm, nch};
    const unsigned blocks = (unsigned)(a.tiles_j * a.tiles_m * nch);
#define MR_RT_LAUNCH(TM, TJ)                                                                   \
    if (tm == TM && tj == TJ) {                                                                \
      hipLaunchKernelGGL((mixed_resid64_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ), 0, s, a); \
      return hipGetLastError();                                                                \
    }
    MR_RT_TILES(MR_RT_LAUNCH)
#undef MR_RT_LAUNCH
  }
  hipLaunchKernelGGL(mixed_resid64_kernel, dim3(rows_blocks(n)), dim3(row_threads(n)), 0, s, theta, delta, n, C, rhs32,
                     base32, sb32, red);
  return hipGetLastError();
}

hipError_t launch_base_root(const float* base32, const double* delta, int n, double h, float* sb32, hipStream_t s) {
  hipLaunchKernelGGL(base_root_kernel, dim3((unsigned)n * n), dim3(n < 256 ? n : 256), 0, s, base32, delta, n,
                     1.0 / (h * h), sb32);
  return hipGetLastError();
}

hipError_t launch_restrict32(const float* fine, float* coarse, int n, hipStream_t s) {
  const int m = n / 2;
  hipLaunchKernelGGL(restrict32_kernel, dim3((unsigned)m * m), dim3(m), 0, s, fine, coarse, n);
  return hipGetLastError();
}

hipError_t launch_lin_resid_restrict(const float* e, const float* base, const float* sb, const float* rhs, int n, double h,
                                     ShiftRef c, float* rhs_c, Reduce red, hipStream_t s) {
  int tm = 0, tj = 0, nch = 0;
  if (tiled_cfg(n, rr_tiled_kernel, 2, tm, tj, nch, kPref8)) {
    LinRRArgs a{e, base, sb, rhs, n, (float)(1.0 / (h * h)), c, rhs_c, red, n / tj, n / 2 / tm, nch};
    const unsigned blocks = (unsigned)(a.tiles_j * a.tiles_m * nch);
#define MR_RR_LAUNCH(TM, TJ)                                                                           \
    if (tm == TM && tj == TJ) {                                                                        \
      hipLaunchKernelGGL((lin_resid_restrict_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ / 2), 0, s, a); \
      return hipGetLastError();                                                                        \
    }
    MR_RR_TILES(MR_RR_LAUNCH)
#undef MR_RR_LAUNCH
  }
  const int m = n / 2;
  hipLaunchKernelGGL(lin_resid_restrict_kernel, dim3(rows_blocks(m)), dim3(row_threads(m)), 0, s, e, base, sb, rhs, n,
                     (float)(1.0 / (h * h)), c, rhs_c, red);
  return hipGetLastError();
}

hipError_t launch_prolong_add32(const float* ec, float* e, int n, hipStream_t s) {
  hipLaunchKernelGGL(prolong_add32_kernel, dim3((unsigned)n * n), dim3(n / 2), 0, s, ec, e, n);
  return hipGetLastError();
}

hipError_t launch_lin_coarsest(float* e, const float* base, const float* sb, const float* rhs, int n, int nsweeps, double h,
                               const double* c_sum, double c_scale, hipStream_t s) {
  if ((long)n * n * n > kMaxCoarsest) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lin_coarsest_kernel, dim3(1), dim3(256), 0, s, e, base, sb, rhs, n, nsweeps, (float)(h * h),
                     (float)(1.0 / (h * h)), c_sum, c_scale);
  return hipGetLastError();
}

hipError_t launch_update64(double* theta, const float* e, size_t cells, hipStream_t s) {
  hipLaunchKernelGGL(update64_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, theta, e, cells);
  return hipGetLastError();
}

hipError_t launch_fill32(float* a, float v, size_t cells, hipStream_t s) {
  hipLaunchKernelGGL(fill32_kernel, dim3(lin_blocks(cells)), dim3(256), 0, s, a, v, cells);
  return hipGetLastError();
}

// ---- driver -------------------------------------------------------------------------------

// FP32 buffers of one level of the inner linear multigrid (colour-split).
struct LinLevel {
  float* e[2] = {nullptr, nullptr};
  int cur = 0;
  float* rhs = nullptr;
  float* base = nullptr;
  float* sb = nullptr;
  TileCfg sw;
};

struct MixedState {
  std::vector<LinLevel> lv;
  std::vector<void*> owned;
};

static TileCfg lin_tiles(int n) {
  TileCfg t;
  const int nh = n / 2;
  int tm = 64;
  while (tm > 2 && (nh % tm != 0 || tm > nh)) tm /= 2;
  static const int pref[][2] = {{64, 4}, {32, 8}, {16, 16}, {8, 16}, {4, 8}, {2, 4}};
  t.tm = 0;
  for (const auto& p : pref)
    if (p[0] == tm && n % p[1] == 0 && p[1] <= n) {
      t.tm = p[0];
      t.tj = p[1];
      break;
    }
  if (t.tm == 0) return t;
  t.tiles_j = n / t.tj;
  t.tiles_m = nh / t.tm;
  const long tiles = (long)t.tiles_j * t.tiles_m;
  t.ci = n;
  while (t.ci % 2 == 0 && t.ci / 2 >= 8 && tiles * (n / t.ci) < 1024) t.ci /= 2;
  while (tiles * (n / t.ci) > kMaxReduceBlocks && t.ci * 2 <= n && n % (t.ci * 2) == 0) t.ci *= 2;
  t.pipe = t.ci % 4 == 0;
  return t;
}

static int mixed_alloc(Ctx* c) {
  if (c->mixed) return MR_OK;
  MixedState* m = new MixedState();
  c->mixed = m;
  m->lv.resize(c->nlev);
  for (int l = 0; l < c->nlev; ++l) {
    const size_t cells = c->lv[l].cells;
    LinLevel& L = m->lv[l];
    float** bufs[] = {&L.e[0], &L.e[1], &L.rhs, &L.base, &L.sb};
    for (float** b : bufs) {
      hipError_t e = hipMalloc((void**)b, cells * sizeof(float));
      if (e != hipSuccess) return fail(MR_ENOMEM, "mixed precision buffers: %s", hipGetErrorString(e));
      m->owned.push_back(*b);
    }
    if (l < c->nlev - 1) L.sw = lin_tiles(c->lv[l].n);
  }
  return MR_OK;
}

void Ctx::release_extra() {
  if (cic_grid) {
    (void)hipFree(cic_grid);
    cic_grid = nullptr;
  }
  if (mixed) {
    for (void* p : mixed->owned) (void)hipFree(p);
    delete mixed;
    mixed = nullptr;
  }
  release_adjoint();
}

double* Ctx::linsum(int l) { return scal + kSlotLin + 3 * l; }

int Ctx::lin_sweep(int l) {
  LinLevel& L = mixed->lv[l];
  Level& F = lv[l];
  double* cs = linsum(l);
  LinSweepArgs a{};
  a.e_in = L.e[L.cur];
  a.e_red_new = nullptr;
  a.e_out = L.e[L.cur ^ 1];
  a.base = L.base;
  a.sb = L.sb;
  a.rhs = L.rhs;
  a.n = F.n;
  a.colour = 0;
  a.h2 = (float)(F.h * F.h);
  a.ih2 = (float)(1.0 / (F.h * F.h));
  a.c_sum = cs;
  a.c_scale = 1.0 / (double)F.cells;
  a.sum_out = cs + 2;
  a.partials = partials;
  a.counter = counter;
  const int ev = (l == 0) ? timer.begin(stream) : -1;
  hipError_t e = launch_lin_half_sweep(a, L.sw, stream);
  if (e != hipSuccess) return hip_fail(e, "linear red half-sweep");
  a.colour = 1;
  a.e_red_new = L.e[L.cur ^ 1];
  a.sum_out = cs + 1;
  a.copy_from = cs + 2;
  a.copy_to = cs + 0;
  e = launch_lin_half_sweep(a, L.sw, stream);
  if (e != hipSuccess) return hip_fail(e, "linear black half-sweep");
  timer.end(1, ev, stream);
  L.cur ^= 1;
  return MR_OK;
}

int Ctx::lin_vcycle(int l) {
  LinLevel& L = mixed->lv[l];
  Level& F = lv[l];
  hipError_t e;
  if (l == nlev - 1) {
    e = launch_lin_coarsest(L.e[L.cur], L.base, L.sb, L.rhs, F.n, opts.ncoarse, F.h, linsum(l), 1.0 / (double)F.cells,
                            stream);
    return e == hipSuccess ? MR_OK : hip_fail(e, "linear coarsest");
  }
  int rc;
  for (int s = 0; s < opts.npre; ++s)
    if ((rc = lin_sweep(l)) != MR_OK) return rc;
  LinLevel& Lc = mixed->lv[l + 1];
  Level& Fc = lv[l + 1];
  e = launch_lin_resid_restrict(L.e[L.cur], L.base, L.sb, L.rhs, F.n, F.h, ShiftRef{linsum(l), 1.0 / (double)F.cells, 0.0},
                                Lc.rhs, Reduce{partials, counter, linsum(l + 1)}, stream);
  if (e == hipSuccess) e = launch_fill32(Lc.e[Lc.cur], 0.0f, Fc.cells, stream);
  if (e != hipSuccess) return hip_fail(e, "linear restriction");
  if ((rc = lin_vcycle(l + 1)) != MR_OK) return rc;
  e = launch_prolong_add32(Lc.e[Lc.cur], L.e[L.cur], F.n, stream);
  if (e != hipSuccess) return hip_fail(e, "linear prolongation");
  for (int s = 0; s < opts.npost; ++s)
    if ((rc = lin_sweep(l)) != MR_OK) return rc;
  return MR_OK;
}

int Ctx::solve_mixed(const double* delta, double* theta, mr_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  int rc = mixed_alloc(this);
  if (rc != MR_OK) return rc;
  if ((rc = prepare(delta)) != MR_OK) return rc;
  Level& L0 = lv[0];
  const double N3 = (double)L0.cells;
  L0.cur = 0;
  hipError_t e = opts.warm_start ? launch_to_split(theta, L0.th[0], L0.n, stream)
                                 : hipMemsetAsync(L0.th[0], 0, L0.cells * sizeof(double), stream);
  if (e != hipSuccess) return hip_fail(e, "initial theta");
  double r0, m0;
  if ((rc = finest_norm(nullptr, ShiftRef{nullptr, 0.0, 0.0}, &r0, &m0)) != MR_OK) return rc;
  if (r0 == 0.0) r0 = 1.0;
  // running sum of Sigma for the shift of the outer residual: (sum Sigma, 0) at theta = 0
  if ((rc = write_scalar(kSlotRes, m0 * N3)) != MR_OK) return rc;
  if ((rc = write_scalar(kSlotRes + 1, 0.0)) != MR_OK) return rc;
  mr_info loc{};
  loc.r0_norm = r0;
  int it = 0, status = MR_OK;
  double rel = 1.0, best = 1e300, msig = m0;
  LinLevel& M0 = mixed->lv[0];
  for (;;) {
    e = launch_mixed_resid64(L0.th[0], L0.delta, L0.n, ShiftRef{scal + kSlotRes, 1.0 / N3, 0.0}, M0.rhs, M0.base, M0.sb,
                             reducer(kSlotRes), stream);
    if (e != hipSuccess) return hip_fail(e, "mixed residual");
    double r[4];
    if ((rc = read_scalars(kSlotRes, 4, r)) != MR_OK) return rc;
    const double var = r[3] - r[2] * r[2] / N3;
    rel = std::sqrt(var > 0.0 ? var : 0.0) / r0;
    msig = r[0] / N3;
    if (it < 128) loc.history[it] = rel;
    if (!std::isfinite(rel) || rel > 1e6 * (best < 1.0 ? 1.0 : best)) {
      status = fail(MR_EDIVERGED, "residual diverged at outer iteration %d (%g)", it, rel);
      break;
    }
    if (rel < best) best = rel;
    if (rel <= opts.tol || it >= opts.max_cycles) break;
    // base hierarchy for the linear operator
    for (int l = 1; l < nlev; ++l) {
      e = launch_restrict32(mixed->lv[l - 1].base, mixed->lv[l].base, lv[l - 1].n, stream);
      if (e == hipSuccess) e = launch_base_root(mixed->lv[l].base, lv[l].delta, lv[l].n, lv[l].h, mixed->lv[l].sb, stream);
      if (e != hipSuccess) return hip_fail(e, "linear base hierarchy");
    }
    // inner solve from e = 0; the shift starts at <rhs> = -<b>
    M0.cur = 0;
    if ((e = launch_fill32(M0.e[0], 0.0f, L0.cells, stream)) != hipSuccess) return hip_fail(e, "fill");
    hipLaunchKernelGGL(inner_shift_kernel, dim3(1), dim3(64), 0, stream, (const double*)(scal + kSlotRes), linsum(0));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "inner shift");
    for (int k = 0; k < opts.inner_cycles; ++k)
      if ((rc = lin_vcycle(0)) != MR_OK) return rc;
    if ((e = launch_update64(L0.th[0], M0.e[M0.cur], L0.cells, stream)) != hipSuccess) return hip_fail(e, "update");
    ++it;
  }
  if (status == MR_OK && rel > opts.tol) {
    status = MR_NOT_CONVERGED;
    fail(MR_NOT_CONVERGED, "not converged after %d outer iterations (rel residual %g)", it, rel);
  }
  e = launch_sum(L0.th[0], L0.cells, reducer(kSlotGauge), stream);
  if (e == hipSuccess) e = launch_from_split(L0.th[0], theta, L0.n, scal + kSlotGauge, 1.0 / N3, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "gauge");
  loc.status = status;
  loc.cycles = it;
  loc.rel_residual = rel;
  loc.m_shift = msig;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return status;
}

}  // namespace mr
