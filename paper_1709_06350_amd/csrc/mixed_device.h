// Device bodies of the mixed-precision kernels. Each body processes the share of one mesh given
// by (bid, nblocks), so that the same code serves one-mesh launches (bid = blockIdx.x) and
// multi-box launches (bid = the block's rank within its box).
#pragma once

#include <type_traits>

#include "mr_device.h"
#include "mr_kernels.h"

namespace mr {

struct Nb18f {
  float xm, xp, ym, yp, zm, zp;
  float xpyp, xmym, xpym, xmyp;
  float xpzp, xmzm, xpzm, xmzp;
  float ypzp, ymzm, ypzm, ymzp;
};

template <typename T, typename N>
__device__ __forceinline__ void gather18_split_t(const T* __restrict__ a, int n, int i, int j, int k, N& t) {
  const int im = wrapi(i - 1, n), ip = wrapi(i + 1, n);
  const int jm = wrapi(j - 1, n), jp = wrapi(j + 1, n);
  const int km = wrapi(k - 1, n), kp = wrapi(k + 1, n);
  t.xm = a[split_idx(n, im, j, k)]; t.xp = a[split_idx(n, ip, j, k)];
  t.ym = a[split_idx(n, i, jm, k)]; t.yp = a[split_idx(n, i, jp, k)];
  t.zm = a[split_idx(n, i, j, km)]; t.zp = a[split_idx(n, i, j, kp)];
  t.xpyp = a[split_idx(n, ip, jp, k)]; t.xmym = a[split_idx(n, im, jm, k)];
  t.xpym = a[split_idx(n, ip, jm, k)]; t.xmyp = a[split_idx(n, im, jp, k)];
  t.xpzp = a[split_idx(n, ip, j, kp)]; t.xmzm = a[split_idx(n, im, j, km)];
  t.xpzm = a[split_idx(n, ip, j, km)]; t.xmzp = a[split_idx(n, im, j, kp)];
  t.ypzp = a[split_idx(n, i, jp, kp)]; t.ymzm = a[split_idx(n, i, jm, km)];
  t.ypzm = a[split_idx(n, i, jp, km)]; t.ymzp = a[split_idx(n, i, jm, kp)];
}

// The base potential of the linearisation is stored as 32-bit fixed point, q = round(theta 2^s)
// with |q| < 2^29 (the scale chosen from max |theta|), so that second differences of the base are
// exact integers: an FP32 copy of theta would round it to about 1e-7 of max |theta| (1.2e-4 for
// |theta| ~ 1000 cells^2 on a 512^3 mesh) and the Hessian of a void cell, its eigenvalues near -1
// and W = (9 s Mbar - 27 Mbar^2) / (3 s^2 + p) sensitive to them, would be wrong by several per
// cent. With |q| < 2^29 every difference below fits int32: a neighbour minus the centre is below
// 2^30 and the sum of two such, or the difference of two such, below 2^31. The fixed-point values
// travel through the FP32 loaders and LDS slots as raw bits (qbits / qval).
constexpr int kBaseBits = 29;
__device__ __forceinline__ float qbits(int q) { return __builtin_bit_cast(float, q); }
__device__ __forceinline__ int qval(float bits) { return __builtin_bit_cast(int, bits); }

// Fixed-point base value of theta for the scale 2^s (s from base_scale_exp).
__device__ __forceinline__ int base_quantise(double theta, double scale) { return __double2int_rn(theta * scale); }

// Scale exponent for a potential with max |theta| = tmax: the largest s with tmax 2^s < 2^kBaseBits - 1
// (at most 60, for theta = 0).
__host__ __device__ inline int base_scale_exp(double tmax) {
  int s = 60;
  const double lim = (double)((1 << kBaseBits) - 1);
  while (s > -60 && tmax * ldexp(1.0, s) >= lim) --s;
  return s;
}

// h^2 dSigma(e) for a cell with base neighbours b and centre bc (fixed-point bits, scale bscl =
// 2^-s), base root s and perturbation neighbours e; also returns the face-neighbour sum of e. FP32.
// With Mbar the traceless (scaled) Hessian of the base and W = (9 s Mbar - 27 Mbar^2 + 9 T2 I) /
// (3 s^2 - 4.5 T2) the result is sum_a W_aa eS_a + (1/2) sum_{a<b} W_ab eD_ab, evaluated as
// (9 s A - 27 B + 9 T2 Se) / (3 s^2 - 4.5 T2) with A and B the same contractions of Mbar and Mbar^2;
// the off-diagonal entries of Mbar^2 use the zero trace (Mbar_xx + Mbar_yy = -Mbar_zz, ...).
__device__ __forceinline__ float lin_source(const Nb18f& b, float bc, float bscl, float s, float ih2, const Nb18f& e,
                                            float& Se) {
  const int c = qval(bc);
  // exact integer second differences of the base (pair sums minus twice the centre: with |q| < 2^29
  // a pair sum and twice the centre are below 2^30, their difference below 2^31) and cross differences
  const int c2 = c + c;
  const int dx = (qval(b.xm) + qval(b.xp)) - c2;
  const int dy = (qval(b.ym) + qval(b.yp)) - c2;
  const int dz = (qval(b.zm) + qval(b.zp)) - c2;
  const int cxy = (qval(b.xpyp) - qval(b.xpym)) - (qval(b.xmyp) - qval(b.xmym));
  const int cxz = (qval(b.xpzp) - qval(b.xpzm)) - (qval(b.xmzp) - qval(b.xmzm));
  const int cyz = (qval(b.ypzp) - qval(b.ypzm)) - (qval(b.ymzp) - qval(b.ymzm));
  const float sc = bscl * ih2;
  const float sc4 = 0.25f * sc;
  const float fx = (float)dx * sc, fy = (float)dy * sc, fz = (float)dz * sc;
  const float f3 = (fx + fy + fz) * (1.0f / 3.0f);
  const float mx = fx - f3, my = fy - f3, mz = fz - f3;
  const float mxy = sc4 * (float)cxy;
  const float mxz = sc4 * (float)cxz;
  const float myz = sc4 * (float)cyz;
  const float mx2 = mx * mx, my2 = my * my, mz2 = mz * mz;
  const float xy2 = mxy * mxy, xz2 = mxz * mxz, yz2 = myz * myz;
  const float T2 = (mx2 + my2 + mz2) + 2.0f * (xy2 + xz2 + yz2);
  // hardware reciprocal: the linearised operator only steers the defect correction
  const float inv = __builtin_amdgcn_rcpf(3.0f * s * s - 4.5f * T2);
  const float eSx = e.xm + e.xp, eSy = e.ym + e.yp, eSz = e.zm + e.zp;
  Se = eSx + eSy + eSz;
  const float eDxy = (e.xpyp + e.xmym) - (e.xpym + e.xmyp);
  const float eDxz = (e.xpzp + e.xmzm) - (e.xpzm + e.xmzp);
  const float eDyz = (e.ypzp + e.ymzm) - (e.ypzm + e.ymzp);
  // Mbar^2
  const float Nxx = mx2 + xy2 + xz2, Nyy = xy2 + my2 + yz2, Nzz = xz2 + yz2 + mz2;
  const float Nxy = mxz * myz - mxy * mz, Nxz = mxy * myz - mxz * my, Nyz = mxy * mxz - myz * mx;
  const float A = (mx * eSx + my * eSy + mz * eSz) + 0.5f * (mxy * eDxy + mxz * eDxz + myz * eDyz);
  const float B = (Nxx * eSx + Nyy * eSy + Nzz * eSz) + 0.5f * (Nxy * eDxy + Nxz * eDxz + Nyz * eDyz);
  return ((9.0f * s) * A - 27.0f * B + (9.0f * T2) * Se) * inv;
}

// ---- FP32 linear half-sweep (compile-time tile, same decomposition as the FP64 sweep) -------
// LDS holds four colour fields per plane: e red, e black, base red, base black.
template <int TM, int TJ>
struct LinTile {
  static constexpr int NT = TM * TJ;
  static constexpr int SLOT = (TJ + 2) * (TM + 2);
  static constexpr int LDS = 4 * 4 * SLOT;   // floats
};

// Body of the FP32 linear half-sweep for one tile (logical tile id), reduction over nblocks
// blocks with this block as number bid. Shared by the single-mesh and the multi-box launches.
template <int TM, int TJ>
inline __device__ void lin_sweep_body(const LinSweepArgs& a, int logical, int bid, int nblocks, float* lds) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2;
  constexpr int SLOT = LinTile<TM, TJ>::SLOT;
  constexpr int TOTAL = 4 * SLOT;
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  const int n = a.n, nh = n >> 1, c = a.colour;
  const int tid = threadIdx.x;
  const int tm_i = logical % a.tiles_m;
  const int tj_i = (logical / a.tiles_m) % a.tiles_j;
  const int chunk = logical / (a.tiles_m * a.tiles_j);
  const int j0 = tj_i * TJ, m0 = tm_i * TM, i0 = chunk * a.ci, i1 = i0 + a.ci;
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned plane = (unsigned)n * (unsigned)nh;
  const float* __restrict__ f0 = a.e_red_new ? a.e_red_new : a.e_in;   // e red
  const float* __restrict__ f1 = a.e_in + half;                        // e black
  const float* __restrict__ f2 = reinterpret_cast<const float*>(a.base);          // base red (fixed-point bits)
  const float* __restrict__ f3 = reinterpret_cast<const float*>(a.base) + half;   // base black

  unsigned goff[NPF];
  int loff[NPF];
  int fld[NPF];
#pragma unroll
  for (int t = 0; t < NPF; ++t) {
    int e = tid + t * NT;
    e = e < TOTAL ? e : TOTAL - 1;
    const int ff = e / SLOT;
    const int rem = e - ff * SLOT;
    const int r = rem / RW;
    const int s = rem - r * RW;
    goff[t] = (unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + s, nh);
    loff[t] = ff * 4 * SLOT + rem;
    fld[t] = ff;
  }
  auto fetch = [&](int p, float (&v)[NPF]) {
    const unsigned base = (unsigned)wrapi(p, n) * plane;
#pragma unroll
    for (int t = 0; t < NPF; ++t) {
      const float* src = fld[t] == 0 ? f0 : (fld[t] == 1 ? f1 : (fld[t] == 2 ? f2 : f3));
      v[t] = src[base + goff[t]];
    }
  };
  auto store = [&](int p, const float (&v)[NPF]) {
    const int so = (p & 3) * SLOT;
#pragma unroll
    for (int t = 0; t < NPF; ++t) lds[loff[t] + so] = v[t];
  };
  auto L = [&](int ff, int p, int r, int s) -> float { return lds[(ff * 4 + (p & 3)) * SLOT + r * RW + s]; };

  float v[NPF];
  {
    float va[NPF], vb[NPF];
    fetch(i0 - 1, va);
    fetch(i0, vb);
    fetch(i0 + 1, v);
    store(i0 - 1, va);
    store(i0, vb);
    store(i0 + 1, v);
  }
  __syncthreads();

  const int s = tid % TM, r = tid / TM;
  const int m = m0 + s, j = j0 + r;
  const double Cd = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const float C = (float)Cd;
  const float h2 = a.h2, ih2 = a.ih2;
  const float bscl = (float)a.bq[0];
  const float* __restrict__ sbc = a.sb + c * half;
  const float* __restrict__ rc = a.rhs + c * half;
  float* __restrict__ out = a.e_out + c * half;
  const int o = 1 - c;
  double acc = 0.0;

  for (int i = i0; i < i1; ++i) {
    const bool pre = (i + 2 <= i1);
    if (pre) fetch(i + 2, v);
    const int q = (i + j + c) & 1;
    const int R = r + 1, S = s + 1, sp = S + q, sm = S + q - 1;
    Nb18f te, tb;
#define MR_LIN_GATHER(T, OF, SF)                                                   \
    T.xm = L(OF, i - 1, R, S); T.xp = L(OF, i + 1, R, S);                          \
    T.ym = L(OF, i, R - 1, S); T.yp = L(OF, i, R + 1, S);                          \
    T.zm = L(OF, i, R, sm);    T.zp = L(OF, i, R, sp);                             \
    T.xpyp = L(SF, i + 1, R + 1, S); T.xmym = L(SF, i - 1, R - 1, S);              \
    T.xpym = L(SF, i + 1, R - 1, S); T.xmyp = L(SF, i - 1, R + 1, S);              \
    T.xpzp = L(SF, i + 1, R, sp);    T.xmzm = L(SF, i - 1, R, sm);                 \
    T.xpzm = L(SF, i + 1, R, sm);    T.xmzp = L(SF, i - 1, R, sp);                 \
    T.ypzp = L(SF, i, R + 1, sp);    T.ymzm = L(SF, i, R - 1, sm);                 \
    T.ypzm = L(SF, i, R + 1, sm);    T.ymzp = L(SF, i, R - 1, sp);
    MR_LIN_GATHER(te, o, c)
    MR_LIN_GATHER(tb, 2 + o, 2 + c)
#undef MR_LIN_GATHER
    const unsigned e = (unsigned)i * plane + (unsigned)j * nh + m;
    float Se;
    const float g = lin_source(tb, L(2 + c, i, R, S), bscl, sbc[e], ih2, te, Se) * ih2;
    const float rhs = rc[e];
    out[e] = (Se - h2 * (g + rhs - C)) * (1.0f / 6.0f);
    acc += (double)(g + rhs);
    if (pre) store(i + 2, v);
    __syncthreads();
  }
  double vv[1] = {acc};
  const bool last = grid_sum<1>(vv, a.partials, a.counter, a.sum_out, nblocks, bid);
  if (last && tid == 0 && a.copy_to) *a.copy_to = *a.copy_from;
}
// ---- simple kernels of the mixed form (row mapping as in transfer.hip) ----------------------

// FP64 outer residual on the finest mesh: b = nabla^2 theta - Sigma + C; rhs32 = -b, base32 =
// theta, sb32 = the physical root s. result = (sum Sigma, 0, sum b, sum b^2), so that the first two
// entries serve as the running sum that sets C of the next pass.
inline __device__ bool mixed_resid64_body(const double* __restrict__ theta, const double* __restrict__ delta, int n,
                                   ShiftRef cref, float* __restrict__ rhs32, int* __restrict__ baseq,
                                   const double* __restrict__ bq, float* __restrict__ sb32, Reduce red, int bid,
                                   int nblocks) {
  const double C = (cref.c_sum ? (cref.c_sum[0] + cref.c_sum[1]) * cref.c_scale : 0.0) + cref.c_add;
  const double qs = bq[1];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const int rows = n * n;
  const int rpb = (rows + nblocks - 1) / nblocks;
  const int r0 = xcd_remap(bid, nblocks) * rpb;
  const int r1 = r0 + rpb < rows ? r0 + rpb : rows;
  for (int row = r0; row < r1; ++row) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned e = split_idx(n, i, j, k);
      Nb18 t;
      gather18_split(theta, n, i, j, k, t);
      double S;
      const double sig = sigma_cell(t, 1.0 + delta[e], 1.0, S);
      const double th = theta[e];
      const double b = (S - 6.0 * th) - sig + C;
      rhs32[e] = (float)(-b);
      baseq[e] = base_quantise(th, qs);
      sb32[e] = (float)(sig + 3.0);
      a0 += b;
      a1 += b * b;
      a2 += sig;
    }
  }
  double v[4] = {a2, 0.0, a0, a1};
  return grid_sum<4>(v, red.partials, red.counter, red.result, nblocks, bid);
}
// Base root on a coarse mesh (cell size h) from the restricted fixed-point base potential (its
// value bq[0] q, exact in FP64); rows bid, bid + nblocks, ... of the mesh.
// Largest real root of s^3 + p s + q = 0 in FP32 (the root of the linearisation's base, which
// only weights the FP32 operator): the upper-bound seed of the FP64 iteration, then Newton steps in
// FP32 until every lane of the wave has a step below 1e-6 of its root (at most 12).
__device__ __forceinline__ float largest_root_f32(float p, float q) {
  const float mq = fmaxf(-q, 0.0f);
  const float c = mq > 0.0f ? __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(mq) * (1.0f / 3.0f)) : 0.0f;
  const float b1 = __builtin_amdgcn_sqrtf(fmaxf(-p, 0.0f)) + c;
  const float b2 = c > 0.0f ? c - p * __builtin_amdgcn_rcpf(3.0f * c) : b1;
  float s = fminf(b1, b2);
  bool done = false;
#pragma unroll 1
  for (int it = 0; it < 12; ++it) {
    const float s2 = s * s;
    const float t = s2 + p;
    const float g = __builtin_fmaf(s, t, q);
    const float gp = __builtin_fmaf(2.0f, s2, t);
    const float d = g * __builtin_amdgcn_rcpf(gp);
    const float sn = s - d;
    s = done ? s : sn;
    done = done || !(__builtin_fabsf(d) > 1e-6f * sn);
    if (it >= 3 && __ballot(!done) == 0) break;
  }
  return s;
}

// Root of the linearisation at every cell of a coarse level from its fixed-point base, FP32: the
// traceless Hessian from exact integer differences (as in lin_source), T2 and T3 of it, and
// p = -(9/2) T2, q = 9 T3 - 27 (1 + delta).
inline __device__ void base_root_body(const int* __restrict__ baseq, const double* __restrict__ bq,
                               const double* __restrict__ delta, int n, double ih2, float* __restrict__ sb32, int bid,
                               int nblocks) {
  const float sc = (float)bq[0] * (float)ih2;
  const float sc4 = 0.25f * sc;
  for (int row = xcd_remap(bid, nblocks); row < n * n; row += nblocks) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned e = split_idx(n, i, j, k);
      Nb18f b;
      gather18_split_t(reinterpret_cast<const float*>(baseq), n, i, j, k, b);
      const int c2 = 2 * baseq[e];
      const int dx = (qval(b.xm) + qval(b.xp)) - c2;
      const int dy = (qval(b.ym) + qval(b.yp)) - c2;
      const int dz = (qval(b.zm) + qval(b.zp)) - c2;
      const int cxy = (qval(b.xpyp) - qval(b.xpym)) - (qval(b.xmyp) - qval(b.xmym));
      const int cxz = (qval(b.xpzp) - qval(b.xpzm)) - (qval(b.xmzp) - qval(b.xmzm));
      const int cyz = (qval(b.ypzp) - qval(b.ypzm)) - (qval(b.ymzp) - qval(b.ymzm));
      const float fx = (float)dx * sc, fy = (float)dy * sc, fz = (float)dz * sc;
      const float f3 = (fx + fy + fz) * (1.0f / 3.0f);
      const float mx = fx - f3, my = fy - f3, mz = fz - f3;
      const float mxy = sc4 * (float)cxy, mxz = sc4 * (float)cxz, myz = sc4 * (float)cyz;
      const float xy2 = mxy * mxy, xz2 = mxz * mxz, yz2 = myz * myz;
      const float T2 = (mx * mx + my * my + mz * mz) + 2.0f * (xy2 + xz2 + yz2);
      const float T3 = 3.0f * (mx * my * mz - (mz * xy2 + my * xz2 + mx * yz2)) + 6.0f * mxy * mxz * myz;
      sb32[e] = largest_root_f32(-4.5f * T2, 9.0f * T3 - 27.0f * (float)(1.0 + delta[e]));
    }
  }
}
// 8-son mean of the fixed-point base (rounded to nearest; |q| < 2^kBaseBits keeps the sum in range
// of int64 and the mean in range of int32), coarse rows bid, bid + nblocks, ...
inline __device__ void restrictq_body(const int* __restrict__ fine, int* __restrict__ coarse, int n, int bid, int nblocks) {
  const int m = n >> 1;
  for (int row = xcd_remap(bid, nblocks); row < m * m; row += nblocks) {
    const int I = row / m, J = row - I * m;
    for (int K = threadIdx.x; K < m; K += blockDim.x) {
      long long s = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += fine[split_idx(n, 2 * I + (q >> 2), 2 * J + ((q >> 1) & 1), 2 * K + (q & 1))];
      coarse[split_idx(m, I, J, K)] = (int)((s >= 0 ? s + 4 : s - 4) / 8);
    }
  }
}
// Block maximum of v over the calling block, then one atomic maximum on the bit pattern of a
// non-negative double (whose order is that of unsigned integers) at *slot.
inline __device__ void block_absmax_to(double v, double* slot) {
  __shared__ double red[16];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int tid = threadIdx.x, nw = (blockDim.x + 63) >> 6;
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
    atomicMax(reinterpret_cast<unsigned long long*>(slot), (unsigned long long)__double_as_longlong(m));
  }
}
// max |a| over cells into *slot (atomic maximum; the slot must hold a value <= the result).
inline __device__ void absmax_body(const double* __restrict__ a, size_t cells, double* slot, int bid, int nblocks) {
  double m = 0.0;
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x) m = fmax(m, fabs(a[x]));
  block_absmax_to(m, slot);
}
// Scale of the fixed-point base from max |theta| (*tmax): bq[0] = 2^-s, bq[1] = 2^s; *tmax is
// returned to zero for the next maximum. One thread.
inline __device__ void base_scale_body(double* tmax, double* bq) {
  const int sx = base_scale_exp(*tmax);
  bq[0] = ldexp(1.0, -sx);
  bq[1] = ldexp(1.0, sx);
  *tmax = 0.0;
}
// Residual of the linear level equation and its restriction: res = rhs + dSigma(e) - lap(e) - C,
// rhs_c = R res (one thread per coarse cell). result[0..1] = (sum of rhs_c, 0).
inline __device__ void lin_resid_restrict_body(const float* __restrict__ e, const int* __restrict__ baseq,
    const double* __restrict__ bq, const float* __restrict__ sb, const float* __restrict__ rhs, int n, float ih2,
    ShiftRef cref, float* __restrict__ rhs_c, Reduce red, int bid, int nblocks) {
  const int m = n >> 1;
  const float* __restrict__ base = reinterpret_cast<const float*>(baseq);
  const float bscl = (float)bq[0];
  const double Cd = (cref.c_sum ? (cref.c_sum[0] + cref.c_sum[1]) * cref.c_scale : 0.0) + cref.c_add;
  const float C = (float)Cd;
  double acc = 0.0;
  const int rows = m * m;
  const int rpb = (rows + nblocks - 1) / nblocks;
  const int r0 = xcd_remap(bid, nblocks) * rpb;
  const int r1 = r0 + rpb < rows ? r0 + rpb : rows;
  for (int row = r0; row < r1; ++row) {
    const int I = row / m, J = row - I * m;
    for (int K = threadIdx.x; K < m; K += blockDim.x) {
      float sres = 0.0f;
#pragma unroll 1
      for (int q = 0; q < 8; ++q) {
        const int i = 2 * I + (q >> 2), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q & 1);
        const unsigned g = split_idx(n, i, j, k);
        Nb18f te, tb;
        gather18_split_t(e, n, i, j, k, te);
        gather18_split_t(base, n, i, j, k, tb);
        float Se;
        const float src = lin_source(tb, base[g], bscl, sb[g], ih2, te, Se) * ih2;
        const float lap = (Se - 6.0f * e[g]) * ih2;
        sres += rhs[g] + src - lap - C;
      }
      const float v = 0.125f * sres;
      rhs_c[split_idx(m, I, J, K)] = v;
      acc += v;
    }
  }
  double vv[2] = {acc, 0.0};
  grid_sum<2>(vv, red.partials, red.counter, red.result, nblocks, bid);
}
// e += P(ec) (trilinear: a fine cell takes 3/4 of its coarse parent and 1/4 of the neighbour
// towards it in each direction, the weights multiplied across x, y, z). A thread per coarse cell
// (I, J, K): it loads the 3 x 3 x 3 coarse neighbourhood once and updates the 8 fine sons (rows
// 2I + a, 2J + b, the cell pair k = 2K, 2K + 1), all 8 fine loads issued before any store.
// Coarse cells are dealt to blocks bid, bid + nblocks, ... of blockDim.x cells each.
inline __device__ void prolong_add32_body(const float* __restrict__ ec, float* __restrict__ e, int n, int bid,
                                          int nblocks) {
  const int nc = n >> 1, nh = nc;
  const long total = (long)nc * nc * nc;
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const float wI[2] = {0.75f, 0.25f};
  for (long gid = (long)xcd_remap(bid, nblocks) * blockDim.x + threadIdx.x; gid < total;
       gid += (long)nblocks * blockDim.x) {
    const int K = (int)(gid % nc);
    const long rest = gid / nc;
    const int J = (int)(rest % nc), I = (int)(rest / nc);
    float c[3][3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          c[a][b][k] = ec[split_idx(nc, wrapi(I - 1 + a, nc), wrapi(J - 1 + b, nc), wrapi(K - 1 + k, nc))];
    unsigned off[2][2];
    int c0[2][2];
    float t[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = 2 * I + a, j = 2 * J + b;
        off[a][b] = ((unsigned)i * n + j) * (unsigned)nh + K;
        c0[a][b] = (i + j) & 1;
        t[a][b][0] = e[c0[a][b] * half + off[a][b]];
        t[a][b][1] = e[(1 - c0[a][b]) * half + off[a][b]];
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int a2 = a ? 2 : 0, b2 = b ? 2 : 0;
        float lo = 0.0f, hi = 0.0f;   // cells k = 2K (neighbour K - 1) and k = 2K + 1 (neighbour K + 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ia = (q & 2) ? a2 : 1, jb = (q & 1) ? b2 : 1;
          const float w = wI[(q >> 1) & 1] * wI[q & 1];
          const float ek = c[ia][jb][1];
          lo += w * (0.75f * ek + 0.25f * c[ia][jb][0]);
          hi += w * (0.75f * ek + 0.25f * c[ia][jb][2]);
        }
        e[c0[a][b] * half + off[a][b]] = t[a][b][0] + lo;
        e[(1 - c0[a][b]) * half + off[a][b]] = t[a][b][1] + hi;
      }
  }
}

// The same update with the coarse neighbourhood staged in LDS, for coarse sizes nc = n / 2 that
// divide 256 with 16 <= nc <= 256: row group blk (of nc^3 / 256) covers coarse plane I, rows
// J0 .. J0 + R - 1 (R = 256 / nc) and every column; its 256 threads first copy coarse rows
// I-1..I+1 x J0-1..J0+R of both colours into cl (3 (256 + 2 nc) floats) in natural k order, then
// each thread updates the 8 fine sons of its coarse cell from the staged neighbourhood.
inline __host__ __device__ bool prolong_rows_ok(int n) {
  const int nc = n / 2;
  return nc >= 16 && nc <= 256 && 256 % nc == 0;
}
inline __device__ void prolong_rows32_body(const float* __restrict__ ec, float* __restrict__ e, int n, int blk,
                                           float* __restrict__ cl) {
  const int nc = n >> 1, nh = nc, nch = nc >> 1;
  const int R = 256 / nc;
  const int groups = nc / R;
  const int I = blk / groups, J0 = (blk - I * groups) * R;
  const int tid = threadIdx.x;
  const unsigned halfc = (unsigned)nc * (unsigned)nc * (unsigned)nch;
  const int r = tid / nc, K = tid - r * nc;
  const int J = J0 + r;
  // the fine values this thread corrects are loaded first, so that their latency overlaps the
  // staging of the coarse rows
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  unsigned off[2][2];
  int c0[2][2];
  float t[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = 2 * I + a, j = 2 * J + b;
      off[a][b] = ((unsigned)i * n + j) * (unsigned)nh + K;
      c0[a][b] = (i + j) & 1;
      t[a][b][0] = __builtin_nontemporal_load(e + c0[a][b] * half + off[a][b]);
      t[a][b][1] = __builtin_nontemporal_load(e + (1 - c0[a][b]) * half + off[a][b]);
    }
  const int rows = 3 * (R + 2);
  for (int x = tid; x < rows * nc; x += 256) {
    const int w = x / nc, pos = x - w * nc;
    const int a = w / (R + 2), b = w - a * (R + 2);
    const int c = pos / nch, m = pos - c * nch;
    const int ii = wrapi(I - 1 + a, nc), jj = wrapi(J0 - 1 + b, nc);
    cl[w * nc + 2 * m + ((ii + jj + c) & 1)] = ec[(unsigned)c * halfc + ((unsigned)ii * nc + jj) * (unsigned)nch + m];
  }
  __syncthreads();
  const int km = K == 0 ? nc - 1 : K - 1, kp = K == nc - 1 ? 0 : K + 1;
  float c3[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float* row = cl + (a * (R + 2) + r + b) * nc;
      c3[a][b][0] = row[km];
      c3[a][b][1] = row[K];
      c3[a][b][2] = row[kp];
    }
  const float wI[2] = {0.75f, 0.25f};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int a2 = a ? 2 : 0, b2 = b ? 2 : 0;
      float lo = 0.0f, hi = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ia = (q & 2) ? a2 : 1, jb = (q & 1) ? b2 : 1;
        const float w = wI[(q >> 1) & 1] * wI[q & 1];
        const float ek = c3[ia][jb][1];
        lo += w * (0.75f * ek + 0.25f * c3[ia][jb][0]);
        hi += w * (0.75f * ek + 0.25f * c3[ia][jb][2]);
      }
      __builtin_nontemporal_store(t[a][b][0] + lo, e + c0[a][b] * half + off[a][b]);
      __builtin_nontemporal_store(t[a][b][1] + hi, e + (1 - c0[a][b]) * half + off[a][b]);
    }
}
constexpr int kProlongRowsLds = 3 * (256 + 2 * 256);   // floats of cl

// Pipelined form of the same prolongation for 128 <= nc <= 256: a block of 1024 threads owns
// TJC = 1024 / nc coarse rows (all nc columns) and marches through a chunk of coarse planes. Each
// coarse plane is staged once (rows J0-1 .. J0+TJC, natural k order) in a two-slot LDS ring, and
// each thread keeps the in-plane (j, k) interpolation of planes I-1, I, I+1 at its four fine
// (j, k) positions in registers, so a plane step reads one staged plane and interpolates in i
// from registers. Coarse planes are fetched one step before they are staged.
inline __host__ __device__ bool prolong_pipe_ok(int n) {
  const int nc = n / 2;
  return nc == 128 || nc == 256;
}
constexpr int kProlongPipeLds = 2 * 10 * 256;   // floats: 2 slots of (TJC + 2) rows x nc

inline __device__ void prolong_pipe32_body(const float* __restrict__ ec, float* __restrict__ e, int n, int logical,
                                           int nchunks, float* __restrict__ cl) {
  const int nc = n >> 1, nh = nc, nch = nc >> 1;
  const int tjc = 1024 / nc;
  const int rows = tjc + 2;
  const int slab = rows * nc;                  // floats of one staged plane
  const int tiles = nc / tjc;
  const int tile = logical % tiles, chunk = logical / tiles;
  const int J0 = tile * tjc;
  const int I0 = (int)(((long)chunk * nc) / nchunks), I1 = (int)(((long)(chunk + 1) * nc) / nchunks);
  const int tid = threadIdx.x;
  const unsigned halfc = (unsigned)nc * (unsigned)nc * (unsigned)nch;
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  // staging: element x < slab of a plane is row w = x / nc, colour cc and column m of that row;
  // two elements per thread (slab <= 2048)
  float pf[2];
  auto fetch = [&](int I) {
    const int ii = wrapi(I, nc);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int x = tid + q * 1024;
      if (x < slab) {
        const int w = x / nc, pos = x - w * nc;
        const int cc = pos / nch, m = pos - cc * nch;
        const int jj = wrapi(J0 - 1 + w, nc);
        pf[q] = ec[(unsigned)cc * halfc + ((unsigned)ii * nc + jj) * (unsigned)nch + m];
      }
    }
  };
  auto stage = [&](int I, int slot) {
    const int ii = wrapi(I, nc);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int x = tid + q * 1024;
      if (x < slab) {
        const int w = x / nc, pos = x - w * nc;
        const int cc = pos / nch, m = pos - cc * nch;
        const int jj = wrapi(J0 - 1 + w, nc);
        cl[slot * slab + w * nc + 2 * m + ((ii + jj + cc) & 1)] = pf[q];
      }
    }
  };
  const int r = tid / nc, K = tid - r * nc;
  const int J = J0 + r;
  const int km = K == 0 ? nc - 1 : K - 1, kp = K == nc - 1 ? 0 : K + 1;
  // in-plane interpolation of a staged plane at fine rows 2J + b and columns 2K + kk:
  // q[2 b + kk]; 3/4 of the own coarse row / column and 1/4 of the neighbour on that side
  auto interp = [&](int slot, float (&q)[4]) {
    const float* c = cl + slot * slab + r * nc;   // rows J-1, J, J+1 at c, c + nc, c + 2 nc
    float lo[3], hi[3];
    const int kk[3] = {km, K, kp};
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const float cm = c[kk[u]], c0 = c[nc + kk[u]], cp = c[2 * nc + kk[u]];
      lo[u] = 0.75f * c0 + 0.25f * cm;
      hi[u] = 0.75f * c0 + 0.25f * cp;
    }
    q[0] = 0.75f * lo[1] + 0.25f * lo[0];
    q[1] = 0.75f * lo[1] + 0.25f * lo[2];
    q[2] = 0.75f * hi[1] + 0.25f * hi[0];
    q[3] = 0.75f * hi[1] + 0.25f * hi[2];
  };
  float Qm[4], Q0[4], Qp[4];
  fetch(I0 - 1);
  stage(I0 - 1, 0);
  fetch(I0);
  stage(I0, 1);
  __syncthreads();
  interp(0, Qm);
  interp(1, Q0);
  fetch(I0 + 1);
  __syncthreads();   // slot 0 is read
  stage(I0 + 1, 0);
  __syncthreads();
  for (int I = I0; I < I1; ++I) {
    const int slot = (I - I0) & 1;               // plane I + 1 is staged here
    fetch(I + 2);                                 // (one plane past the chunk on the last step: unused)
    unsigned off[2][2];
    int c0[2][2];
    float t[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = 2 * I + a, j = 2 * J + b;
        off[a][b] = ((unsigned)i * n + j) * (unsigned)nh + K;
        c0[a][b] = (i + j) & 1;
        t[a][b][0] = __builtin_nontemporal_load(e + c0[a][b] * half + off[a][b]);
        t[a][b][1] = __builtin_nontemporal_load(e + (1 - c0[a][b]) * half + off[a][b]);
      }
    interp(slot, Qp);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float* nb = a ? Qp : Qm;
        const float lo = 0.75f * Q0[2 * b] + 0.25f * nb[2 * b];
        const float hi = 0.75f * Q0[2 * b + 1] + 0.25f * nb[2 * b + 1];
        __builtin_nontemporal_store(t[a][b][0] + lo, e + c0[a][b] * half + off[a][b]);
        __builtin_nontemporal_store(t[a][b][1] + hi, e + (1 - c0[a][b]) * half + off[a][b]);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Qm[u] = Q0[u];
      Q0[u] = Qp[u];
    }
    stage(I + 2, slot ^ 1);                       // the slot read in the previous step
    __syncthreads();
  }
}

// ---- the small levels of an inner V-cycle in one workgroup -----------------------------------
// Every level with n <= kTailMaxN (down to the coarsest) of a zero-start inner V-cycle, in one
// block of kTailThreads threads with all fields in LDS (natural order): on each level e = 0,
// npre sweeps, the defect rhs + dSigma(e) - lap(e) - C restricted to the next level (8-son mean,
// whose mean starts that level's shift), the coarsest level ncoarse sweeps, then on the way up
// e += P e_coarse and npost sweeps. A sweep is the red then the black half with snapshot
// semantics within a colour; its shift C is the mean of dSigma(e) + rhs over the previous sweep
// (the first from the level's right-hand side), as on the larger levels. The launch overhead of
// these levels' kernels, not their arithmetic, is what they cost when launched one by one.
constexpr int kTailMaxN = 16;
constexpr int kTailMaxLev = 3;                       // 16, 8, 4 (or 12, 6)
constexpr int kTailCells = 4096 + 512 + 64 + 8;      // sum of n^3 over the levels, rounded up
constexpr int kTailThreads = 1024;
struct LinTailArgs {
  float* e_out;                      // split e of the first tail level
  const float* rhs;                  // split rhs of the first tail level
  const int* base[kTailMaxLev];      // split fixed-point base of each tail level
  const float* sb[kTailMaxLev];      // split root of each tail level
  const double* bq;
  const double* c_sum;               // (sum rhs, 0) of the first tail level
  int n0, levels, npre, npost, ncoarse;
  float h0;
};
struct LinTailShared {
  float e[kTailCells], b[kTailCells], s[kTailCells], r[kTailCells];
  float t[4096];
  float C[kTailMaxLev];
  double red[16][1];   // (a half level, at most 2048 cells, is 2 cells per thread)
};

inline __device__ void tail_gather(const float* __restrict__ a, int n, int i, int j, int k, Nb18f& t) {
  const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
  const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
  const int km = k == 0 ? n - 1 : k - 1, kp = k == n - 1 ? 0 : k + 1;
  auto at = [&](int ii, int jj, int kk) { return a[(ii * n + jj) * n + kk]; };
  t.xm = at(im, j, k); t.xp = at(ip, j, k); t.ym = at(i, jm, k); t.yp = at(i, jp, k);
  t.zm = at(i, j, km); t.zp = at(i, j, kp);
  t.xpyp = at(ip, jp, k); t.xmym = at(im, jm, k); t.xpym = at(ip, jm, k); t.xmyp = at(im, jp, k);
  t.xpzp = at(ip, j, kp); t.xmzm = at(im, j, km); t.xpzm = at(ip, j, km); t.xmzp = at(im, j, kp);
  t.ypzp = at(i, jp, kp); t.ymzm = at(i, jm, km); t.ypzm = at(i, jp, km); t.ymzp = at(i, jm, kp);
}

inline __device__ void lin_tail_body(const LinTailArgs& a, LinTailShared& sh) {
  const int tid = threadIdx.x;
  const float bscl = (float)a.bq[0];
  // level l: n0 >> l cells a side, cell size h0 2^l, fields at offset sum_{t<l} (n0 >> t)^3
  // (computed, not indexed, so that nothing is kept in per-lane scratch memory)
  auto nn = [&](int l) { return a.n0 >> l; };
  auto hh = [&](int l) { return a.h0 * (float)(1 << l); };
  auto off = [&](int l) {
    int o = 0;
    for (int t = 0; t < l; ++t) o += (a.n0 >> t) * (a.n0 >> t) * (a.n0 >> t);
    return o;
  };
  // fields of every level, and the first level's right-hand side, into natural order
  for (int l = 0; l < a.levels; ++l) {
    const int n = nn(l), n3 = n * n * n;
    // (selects, not a dynamic index into the argument block)
    const float* bsrc = reinterpret_cast<const float*>(l == 0 ? a.base[0] : l == 1 ? a.base[1] : a.base[2]);
    const float* ssrc = l == 0 ? a.sb[0] : l == 1 ? a.sb[1] : a.sb[2];
    for (int x = tid; x < n3; x += kTailThreads) {
      const int i = x / (n * n), j = (x / n) % n, k = x % n;
      const unsigned g = split_idx(n, i, j, k);
      sh.b[off(l) + x] = bsrc[g];
      sh.s[off(l) + x] = ssrc[g];
      if (l == 0) sh.r[x] = a.rhs[g];
    }
  }
  __syncthreads();

  // one sweep of level l (shift C in, next shift out)
  auto sweep = [&](int l) {
    const float C = sh.C[l];
    const int n = nn(l), nh = n >> 1, n3 = n * n * n, half = n3 >> 1;
    float* e = sh.e + off(l);
    const float* b = sh.b + off(l);
    const float* sv = sh.s + off(l);
    const float* r = sh.r + off(l);
    const float h2 = hh(l) * hh(l), ih2 = 1.0f / h2;
    double acc = 0.0;
    for (int c = 0; c < 2; ++c) {
      float nv[2];
      int nx[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int y = tid + q * kTailThreads;
        nx[q] = -1;
        if (y < half) {
          const int i = y / (n * nh), j = (y / nh) % n, m = y % nh;
          const int k = 2 * m + ((i + j + c) & 1);
          const int x = (i * n + j) * n + k;
          Nb18f te, tb;
          tail_gather(e, n, i, j, k, te);
          tail_gather(b, n, i, j, k, tb);
          float Se;
          const float g = lin_source(tb, b[x], bscl, sv[x], ih2, te, Se) * ih2;
          nv[q] = (Se - h2 * (g + r[x] - C)) * (1.0f / 6.0f);
          nx[q] = x;
          acc += (double)(g + r[x]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (nx[q] >= 0) e[nx[q]] = nv[q];
      __syncthreads();
    }
    double v[1] = {acc};
    block_sum<1>(v, sh.red, tid, kTailThreads);
    if (tid == 0) sh.C[l] = (float)(v[0] / (double)n3);
    __syncthreads();
  };

  float* Cl = sh.C;   // shift of each level (uniform values, kept in LDS)
  if (tid == 0) Cl[0] = (float)((a.c_sum[0] + a.c_sum[1]) / (double)(a.n0 * a.n0 * a.n0));
  __syncthreads();
  const int last = a.levels - 1;
  // down: smooth from zero, restrict the defect
  for (int l = 0; l <= last; ++l) {
    const int n = nn(l), n3 = n * n * n;
    for (int x = tid; x < n3; x += kTailThreads) sh.e[off(l) + x] = 0.0f;
    __syncthreads();
    const int ns = l == last ? a.ncoarse : a.npre;
    for (int sw = 0; sw < ns; ++sw) sweep(l);
    if (l == last) break;
    // defect at every cell into t, then its 8-son means into the next level's rhs
    {
      const float* e = sh.e + off(l);
      const float* b = sh.b + off(l);
      const float* sv = sh.s + off(l);
      const float* r = sh.r + off(l);
      const float ih2 = 1.0f / (hh(l) * hh(l));
      for (int x = tid; x < n3; x += kTailThreads) {
        const int i = x / (n * n), j = (x / n) % n, k = x % n;
        Nb18f te, tb;
        tail_gather(e, n, i, j, k, te);
        tail_gather(b, n, i, j, k, tb);
        float Se;
        const float g = lin_source(tb, b[x], bscl, sv[x], ih2, te, Se) * ih2;
        sh.t[x] = r[x] + g - (Se - 6.0f * e[x]) * ih2 - Cl[l];
      }
      __syncthreads();
      const int nc = n >> 1, nc3 = nc * nc * nc;
      float* rc = sh.r + off(l + 1);
      double acc = 0.0;
      for (int X = tid; X < nc3; X += kTailThreads) {
        const int I = X / (nc * nc), J = (X / nc) % nc, K = X % nc;
        float sum = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          sum += sh.t[((2 * I + (q >> 2)) * n + 2 * J + ((q >> 1) & 1)) * n + 2 * K + (q & 1)];
        rc[X] = 0.125f * sum;
        acc += (double)(0.125f * sum);
      }
      double v[1] = {acc};
      block_sum<1>(v, sh.red, tid, kTailThreads);
      if (tid == 0) Cl[l + 1] = (float)(v[0] / (double)nc3);
      __syncthreads();
    }
  }
  // up: correct from the coarser level, smooth
  for (int l = last - 1; l >= 0; --l) {
    const int n = nn(l), n3 = n * n * n, nc = n >> 1;
    float* e = sh.e + off(l);
    const float* ec = sh.e + off(l + 1);
    for (int x = tid; x < n3; x += kTailThreads) {
      const int i = x / (n * n), j = (x / n) % n, k = x % n;
      const int I = i >> 1, J = j >> 1, K = k >> 1;
      const int I2 = (i & 1) ? (I + 1 == nc ? 0 : I + 1) : (I == 0 ? nc - 1 : I - 1);
      const int J2 = (j & 1) ? (J + 1 == nc ? 0 : J + 1) : (J == 0 ? nc - 1 : J - 1);
      const int K2 = (k & 1) ? (K + 1 == nc ? 0 : K + 1) : (K == 0 ? nc - 1 : K - 1);
      auto at = [&](int ii, int jj, int kk) { return ec[(ii * nc + jj) * nc + kk]; };
      const float z0 = 0.75f * at(I, J, K) + 0.25f * at(I, J, K2);
      const float z1 = 0.75f * at(I, J2, K) + 0.25f * at(I, J2, K2);
      const float z2 = 0.75f * at(I2, J, K) + 0.25f * at(I2, J, K2);
      const float z3 = 0.75f * at(I2, J2, K) + 0.25f * at(I2, J2, K2);
      e[x] += 0.75f * (0.75f * z0 + 0.25f * z1) + 0.25f * (0.75f * z2 + 0.25f * z3);
    }
    __syncthreads();
    for (int sw = 0; sw < a.npost; ++sw) sweep(l);
  }
  // the first level's e back to the split layout
  {
    const int n = nn(0), n3 = n * n * n;
    for (int x = tid; x < n3; x += kTailThreads) {
      const int i = x / (n * n), j = (x / n) % n, k = x % n;
      a.e_out[split_idx(n, i, j, k)] = sh.e[x];
    }
  }
}

// Linear coarsest solve: nsweeps red-black sweeps in one block (FP32, natural order in LDS).
struct LinCoarsestShared {
  float te[kMaxCoarsest], tb[kMaxCoarsest], ts[kMaxCoarsest], tr[kMaxCoarsest], tn[kMaxCoarsest];
  double red[16][1];
  float cnew;
};

inline __device__ void lin_coarsest_body(float* __restrict__ e, const int* __restrict__ baseq, const double* __restrict__ bq,
                                  const float* __restrict__ sb, const float* __restrict__ rhs, int n, int nsweeps,
                                  float h2, float ih2, const double* c_sum, double c_scale, LinCoarsestShared& sh) {
  const float* __restrict__ base = reinterpret_cast<const float*>(baseq);
  const float bscl = (float)bq[0];
  float* te = sh.te;
  float* tb = sh.tb;
  float* ts = sh.ts;
  float* tr = sh.tr;
  float* tn = sh.tn;
  auto& red = sh.red;
  float& cnew = sh.cnew;
  const int n3 = n * n * n, tid = threadIdx.x;
  for (int x = tid; x < n3; x += blockDim.x) {
    const int i = x / (n * n), j = (x / n) % n, k = x % n;
    const unsigned g = split_idx(n, i, j, k);
    te[x] = e[g];
    tb[x] = base[g];
    ts[x] = sb[g];
    tr[x] = rhs[g];
  }
  float C = c_sum ? (float)((c_sum[0] + c_sum[1]) * c_scale) : 0.0f;
  __syncthreads();
  auto nb = [&](const float* a, int i, int j, int k, Nb18f& t) {
    auto at = [&](int ii, int jj, int kk) { return a[(wrapi(ii, n) * n + wrapi(jj, n)) * n + wrapi(kk, n)]; };
    t.xm = at(i - 1, j, k); t.xp = at(i + 1, j, k); t.ym = at(i, j - 1, k); t.yp = at(i, j + 1, k);
    t.zm = at(i, j, k - 1); t.zp = at(i, j, k + 1);
    t.xpyp = at(i + 1, j + 1, k); t.xmym = at(i - 1, j - 1, k); t.xpym = at(i + 1, j - 1, k); t.xmyp = at(i - 1, j + 1, k);
    t.xpzp = at(i + 1, j, k + 1); t.xmzm = at(i - 1, j, k - 1); t.xpzm = at(i + 1, j, k - 1); t.xmzp = at(i - 1, j, k + 1);
    t.ypzp = at(i, j + 1, k + 1); t.ymzm = at(i, j - 1, k - 1); t.ypzm = at(i, j + 1, k - 1); t.ymzp = at(i, j - 1, k + 1);
  };
  for (int sw = 0; sw < nsweeps; ++sw) {
    double acc = 0.0;
    for (int colour = 0; colour < 2; ++colour) {
      for (int x = tid; x < n3; x += blockDim.x) {
        const int i = x / (n * n), j = (x / n) % n, k = x % n;
        if (((i + j + k) & 1) != colour) continue;
        Nb18f ve, vb;
        nb(te, i, j, k, ve);
        nb(tb, i, j, k, vb);
        float Se;
        const float g = lin_source(vb, tb[x], bscl, ts[x], ih2, ve, Se) * ih2;
        tn[x] = (Se - h2 * (g + tr[x] - C)) * (1.0f / 6.0f);
        acc += (double)(g + tr[x]);
      }
      __syncthreads();
      for (int x = tid; x < n3; x += blockDim.x) {
        const int i = x / (n * n), j = (x / n) % n, k = x % n;
        if (((i + j + k) & 1) == colour) te[x] = tn[x];
      }
      __syncthreads();
    }
    double v[1] = {acc};
    block_sum<1>(v, red, tid, blockDim.x);
    if (tid == 0) cnew = (float)(v[0] / (double)n3);
    __syncthreads();
    C = cnew;
    __syncthreads();
  }
  for (int x = tid; x < n3; x += blockDim.x) {
    const int i = x / (n * n), j = (x / n) % n, k = x % n;
    e[split_idx(n, i, j, k)] = te[x];
  }
}
// theta += e; max |theta| of the result into *tmax (atomic maximum) when tmax is given.
inline __device__ void update64_body(double* __restrict__ theta, const float* __restrict__ e, size_t cells, int bid,
                                     int nblocks, double* tmax) {
  double m = 0.0;
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x) {
    const double v = theta[x] + (double)e[x];
    theta[x] = v;
    m = fmax(m, fabs(v));
  }
  if (tmax) block_absmax_to(m, tmax);
}

inline __device__ void fill32_body(float* __restrict__ a, float v, size_t cells, int bid, int nblocks) {
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x) a[x] = v;
}

// ---- pipelined FP32 linear half-sweep --------------------------------------------------------
// lin_sweep_body's decomposition and arithmetic with the colour compile-time and the plane loop
// unrolled by the ring length (compile-time LDS slots); planes are fetched two steps before they
// enter LDS and the base root / right-hand side two steps before use. Requires ci % 4 == 0.
// ZB (black half only): the old black values are zero, so they are not loaded.
template <int TM, int TJ, int COL, bool ZB = false>
__device__ void lin_sweep_pipe_body(const LinSweepArgs& a, int logical, int bid, int nblocks, float* lds) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2;
  constexpr int SLOT = LinTile<TM, TJ>::SLOT;
  constexpr int PER = (SLOT + NT - 1) / NT;   // loads per field and thread
  constexpr int NPF = 4 * PER;
  constexpr int O = 1 - COL;
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  const int tm_i = logical % a.tiles_m;
  const int tj_i = (logical / a.tiles_m) % a.tiles_j;
  const int chunk = logical / (a.tiles_m * a.tiles_j);
  const int j0 = tj_i * TJ, m0 = tm_i * TM, i0 = chunk * a.ci, ci = a.ci;
  const size_t plane = (size_t)n * nh;
  const size_t half = plane * n;
  const unsigned pbytes = (unsigned)plane * 4u;
  const float* __restrict__ f0 = COL == 1 ? a.e_red_new : a.e_in;   // e red
  const float* __restrict__ f1 = a.e_in + half;                      // e black
  const float* __restrict__ f2 = reinterpret_cast<const float*>(a.base);          // base red (fixed-point bits)
  const float* __restrict__ f3 = reinterpret_cast<const float*>(a.base) + half;   // base black
  // global accesses through a buffer resource of one plane (uniform) and a per-lane byte offset
  auto prs = [&](const float* arr, int p) { return plane_rsrc(arr + (size_t)p * plane, pbytes); };

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
    goff[k] = ((unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh)) * 4u;
    loff[k] = e;
  }
  auto fetch = [&](int rel, float (&v)[NPF]) {
    const int p = wrapi(i0 - 1 + rel, n);
    const auto b0 = prs(f0, p), b2 = prs(f2, p), b3 = prs(f3, p);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[0 * PER + k] = ld_rs_f(b0, goff[k]);
      v[2 * PER + k] = ld_rs_f(b2, goff[k]);
      v[3 * PER + k] = ld_rs_f(b3, goff[k]);
    }
    if (!ZB) {
      const auto b1 = prs(f1, p);
#pragma unroll
      for (int k = 0; k < PER; ++k) v[1 * PER + k] = ld_rs_f(b1, goff[k]);
    } else {
#pragma unroll
      for (int k = 0; k < PER; ++k) v[1 * PER + k] = 0.0f;
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
  const unsigned o_c = ((unsigned)j * nh + m) * 4u;   // own cell inside a plane (bytes)
  const int ob = (r + 1) * RW + (s + 1);
  const int q0 = (i0 + j + COL) & 1;
  const int oq0 = ob + q0, oq1 = ob + (q0 ^ 1);
  const double Cd = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const float C = (float)Cd;
  const float h2 = a.h2, ih2 = a.ih2;
  const float bscl = (float)a.bq[0];
  const float* __restrict__ sbc = a.sb + COL * half;
  const float* __restrict__ rc = a.rhs + COL * half;
  float* __restrict__ out = a.e_out + COL * half;
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
  SB[0] = ld_rs_f_nt(prs(sbc, i0), o_c);
  RH[0] = ld_rs_f_nt(prs(rc, i0), o_c);
  SB[1] = ld_rs_f_nt(prs(sbc, min(i0 + 1, last_plane)), o_c);
  RH[1] = ld_rs_f_nt(prs(rc, min(i0 + 1, last_plane)), o_c);
  __syncthreads();

  auto step = [&](auto kc, int t, float (&vst)[NPF], float (&vft)[NPF]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = K & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    const int pn = min(i0 + t + 2, last_plane);
    SB[(K + 2) & 3] = ld_rs_f_nt(prs(sbc, pn), o_c);
    RH[(K + 2) & 3] = ld_rs_f_nt(prs(rc, pn), o_c);
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
    const float g = lin_source(tb, lds[(2 + COL) * 4 * SLOT + S0 * SLOT + ob], bscl, SB[K], ih2, te, Se) * ih2;
    const float rhs = RH[K];
    st_rs_f_nt(prs(out, i0 + t), o_c, (Se - h2 * (g + rhs - C)) * (1.0f / 6.0f));
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
  const bool last = grid_sum<1>(vv, a.partials, a.counter, a.sum_out, nblocks, bid);
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
  const int* base;
  const double* bq;
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
__device__ void lin_resid_restrict_tiled_body(const LinRRArgs& a, int logical, int bid, int nblocks, float* lds) {
  constexpr int NT = TM * TJ / 2;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int PER = (SLOT + NT - 1) / NT;   // loads per field and thread
  constexpr int NPF = 4 * PER;
  const int n = a.n, nh = n >> 1, nc = n >> 1, nch = nc >> 1;
  const int tid = threadIdx.x;
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
  const float* __restrict__ f2 = reinterpret_cast<const float*>(a.base);          // fixed-point bits
  const float* __restrict__ f3 = reinterpret_cast<const float*>(a.base) + half;
  const float bscl = (float)a.bq[0];

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
  // root and right-hand side of the thread's 4 cells of a plane, fetched one plane step ahead
  // (the last fetch of a chunk reads a clamped plane and is not used)
  auto pre = [&](int t, float (&p)[8]) {
    const int i = min(i0 + t, n - 1);
#pragma unroll
    for (int cell = 0; cell < 4; ++cell) {
      const int j = j0 + 2 * rr + (cell >> 1);
      const unsigned o = (unsigned)(cell & 1) * half + (unsigned)i * plane + (unsigned)j * nh + m;
      p[cell] = __builtin_nontemporal_load(a.sb + o);
      p[4 + cell] = __builtin_nontemporal_load(a.rhs + o);
    }
  };
  float PA[8], PB[8];
  pre(0, PA);
  fetch(3, V0);
  __syncthreads();

  auto step = [&](auto kc, int t, float (&vst)[NPF], float (&vft)[NPF], const float (&pc)[8], float (&pn)[8]) {
    constexpr int K = decltype(kc)::value;
    constexpr int SM = K & 3, S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    fetch(t + 4, vft);
    pre(t + 1, pn);
    const int i = i0 + t;
#pragma unroll 1
    for (int cell = 0; cell < 4; ++cell) {
      const int dr = cell >> 1, c = cell & 1;
      const int r = 2 * rr + dr;
      const int j = j0 + r;
      const int ob = (r + 1) * RW + (s + 1);
      // register selects (a dynamic index would put the arrays in scratch memory)
      const float sbv = cell == 0 ? pc[0] : cell == 1 ? pc[1] : cell == 2 ? pc[2] : pc[3];
      const float rhv = cell == 0 ? pc[4] : cell == 1 ? pc[5] : cell == 2 ? pc[6] : pc[7];
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
        const float src = lin_source(tb, lds[((2 + c) * 4 + S0) * SLOT + ob], bscl, sbv, ih2, te, Se) * ih2;
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
    step(std::integral_constant<int, 0>(), t, V0, V1, PA, PB);
    step(std::integral_constant<int, 1>(), t + 1, V1, V0, PB, PA);
    step(std::integral_constant<int, 2>(), t + 2, V0, V1, PA, PB);
    step(std::integral_constant<int, 3>(), t + 3, V1, V0, PB, PA);
  }
  double vv[2] = {acc, 0.0};
  grid_sum<2>(vv, a.red.partials, a.red.counter, a.red.result, nblocks, bid);
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
  int* baseq;
  const double* bq;
  float* sb32;
  Reduce red;
  int tiles_j, tiles_m, nchunks;
};

template <int TM, int TJ>
__device__ bool mixed_resid64_tiled_body(const ResidTiledArgs& a, int logical, int bid, int nblocks, double* lds) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int TOTAL = 2 * SLOT;
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
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
  const double qs = a.bq[1];
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
    // the two colours' roots one after the other (fewer live registers than iterating both)
    double S[2], sr[2];
    {
      Nb18 c0;
      gather(l1, l0, SM, S0, SP, oqc0, c0);
      double pp[1], qq[1], r1[1];
      cell_pq(c0, 1.0 + D[K][0], 1.0, S[0], pp[0], qq[0]);
      largest_roots<1>(pp, qq, r1);
      sr[0] = r1[0];
    }
    {
      Nb18 c1;
      gather(l0, l1, SM, S0, SP, oqc1, c1);
      double pp[1], qq[1], r1[1];
      cell_pq(c1, 1.0 + D[K][1], 1.0, S[1], pp[0], qq[0]);
      largest_roots<1>(pp, qq, r1);
      sr[1] = r1[0];
    }
    const unsigned e0 = (unsigned)(i0 + t) * plane + own;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double thc = (c == 0 ? l0 : l1)[S0 * SLOT + ob];
      const double sig = sr[c] - 3.0;
      const double b = (S[c] - 6.0 * thc) - sig + C;
      const unsigned e = (unsigned)c * half + e0;
      a.rhs32[e] = (float)(-b);
      a.baseq[e] = base_quantise(thc, qs);
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
  return grid_sum<4>(v, a.red.partials, a.red.counter, a.red.result, nblocks, bid);
}

}  // namespace mr

namespace mr {

// ---- one-launch (fused) FP32 linear sweep -----------------------------------------------------
// Both colours of a red-black sweep of the linear level equation in one pass over the mesh. A block
// owns a TM x TJ tile of (m, j) and marches over a chunk of planes [i0, i1). At step t it updates the
// red cells of plane t (its tile plus the one-cell ring around it that the black update of its tile
// reads: the two halo rows and columns, no corners), then, after a barrier, the black cells of plane
// t - 1 from the new red values of planes t - 2 .. t. A red cell's update reads only black values and
// red values of the snapshot (never its own old value), so a ring cell recomputed here equals the
// neighbouring block's result bit for bit: the blocks need no communication. Old e and the base
// (both colours) of planes t - 2 .. t + 2 sit in 5-slot LDS rings with a two-cell halo, the new red
// values in a 5-slot ring with a one-cell halo. Plane t + 3 is fetched into registers at step t and
// stored into the ring's free slot at the end of step t + 1; the root and right-hand side of a step
// are loaded one step ahead. The step loop is unrolled by 10 (the ring length times the two row
// parities), so every LDS slot offset is a compile-time constant. Per cell update the kernel moves
// 20 bytes (e read and written, base, root and right-hand side read once) against 28 for the two
// one-colour launches, which each read both colours of e and of the base.
template <int TM, int TJ>
struct LinFusedTile {
  static constexpr int NT = TM * TJ;
  static constexpr int W2 = TM + 4, S2 = (TJ + 4) * W2;   // old e / base planes (halo 2)
  static constexpr int W1 = TM + 2, S1 = (TJ + 2) * W1;   // new red planes (halo 1)
  static constexpr int HC = 2 * TM + 2 * TJ;              // red ring cells per plane
  static constexpr int PER = (S2 + NT - 1) / NT;          // loads per field and thread
  static constexpr int NPF = 4 * PER;                     // e red, e black, base red, base black
  static constexpr int OFF_B = 10 * S2, OFF_N = 20 * S2;
  static constexpr int LDS = 20 * S2 + 5 * S1;            // floats
};

template <int TM, int TJ>
__device__ void lin_fused_body(const LinFusedArgs& a, int logical, int bid, int nblocks, float* lds) {
  using T = LinFusedTile<TM, TJ>;
  constexpr int NT = T::NT, W2 = T::W2, S2 = T::S2, W1 = T::W1, S1 = T::S1, PER = T::PER, NPF = T::NPF;
  constexpr int OB = T::OFF_B, ON = T::OFF_N;
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  const int ntile = a.tiles_m * a.tiles_j;
  const int tile = logical % ntile, chunk = logical / ntile;
  const int m0 = (tile % a.tiles_m) * TM, j0 = (tile / a.tiles_m) * TJ;
  const int ci = n / a.nchunks, i0 = chunk * ci, i1 = i0 + ci;
  const int U = ci + 2;   // steps: red planes i0 - 1 .. i1, black planes i0 .. i1 - 1
  const size_t plane = (size_t)n * nh, half = plane * n;
  const unsigned pbytes = (unsigned)plane * 4u;
  const float* __restrict__ f0 = a.e_in;
  const float* __restrict__ f1 = a.e_in + half;
  const float* __restrict__ f2 = reinterpret_cast<const float*>(a.base);          // fixed-point bits
  const float* __restrict__ f3 = reinterpret_cast<const float*>(a.base) + half;
  auto prs = [&](const float* arr, int p) { return plane_rsrc(arr + (size_t)wrapi(p, n) * plane, pbytes); };

  // loader: element k of each field is min(k NT + tid, S2 - 1) of its tile-plus-halo plane
  unsigned goff[PER];
  int loff[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int e = k * NT + tid;
    e = e < S2 ? e : S2 - 1;
    const int rr = e / W2, cc = e - rr * W2;
    goff[k] = ((unsigned)wrapi(j0 - 2 + rr, n) * nh + (unsigned)wrapi(m0 - 2 + cc, nh)) * 4u;
    loff[k] = e;
  }
  auto fetch = [&](int p, float (&v)[NPF]) {
    const auto r0 = prs(f0, p), r1 = prs(f1, p), r2 = prs(f2, p), r3 = prs(f3, p);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[k] = ld_rs_f(r0, goff[k]);
      v[PER + k] = ld_rs_f(r1, goff[k]);
      v[2 * PER + k] = ld_rs_f(r2, goff[k]);
      v[3 * PER + k] = ld_rs_f(r3, goff[k]);
    }
  };
  // plane with ring slot sl (compile-time): e red, e black, base red, base black
  auto store = [&](int sl, const float (&v)[NPF]) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      lds[(sl * 2 + 0) * S2 + loff[k]] = v[k];
      lds[(sl * 2 + 1) * S2 + loff[k]] = v[PER + k];
      lds[OB + (sl * 2 + 0) * S2 + loff[k]] = v[2 * PER + k];
      lds[OB + (sl * 2 + 1) * S2 + loff[k]] = v[3 * PER + k];
    }
  };

  const int s = tid % TM, r = tid / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned o_c = ((unsigned)j * nh + m) * 4u;
  // red ring cell of this thread (tid < HC): rows -1 and TJ, then columns -1 and TM
  const bool has_halo = tid < T::HC;
  int hr, hs;
  if (tid < TM) {
    hr = -1;
    hs = tid;
  } else if (tid < 2 * TM) {
    hr = TJ;
    hs = tid - TM;
  } else if (tid < 2 * TM + TJ) {
    hr = tid - 2 * TM;
    hs = -1;
  } else {
    hr = has_halo ? tid - 2 * TM - TJ : 0;
    hs = has_halo ? TM : 0;
  }
  const unsigned o_h = ((unsigned)wrapi(j0 + hr, n) * nh + (unsigned)wrapi(m0 + hs, nh)) * 4u;
  // per-thread LDS offsets: cell (halo-2 and halo-1 planes) and its z neighbour k - 1 for the row
  // parity of even (index 0) and odd (index 1) steps; the parity of a row at step u is p0 ^ (u & 1)
  const int q0 = (i0 - 1 + j) & 1, qh0 = (i0 - 1 + j0 + hr) & 1;
  const int ob2 = (r + 2) * W2 + (s + 2), ob1 = (r + 1) * W1 + (s + 1);
  const int hb2 = (hr + 2) * W2 + (hs + 2), hb1 = (hr + 1) * W1 + (hs + 1);
  const int oz2[2] = {ob2 + q0 - 1, ob2 + (q0 ^ 1) - 1};
  const int oz1[2] = {ob1 + q0 - 1, ob1 + (q0 ^ 1) - 1};
  const int hz2[2] = {hb2 + qh0 - 1, hb2 + (qh0 ^ 1) - 1};
  const double Cd = (a.c_sum ? (a.c_sum[0] + a.c_sum[1]) * a.c_scale : 0.0) + a.c_add;
  const float C = (float)Cd;
  const float h2 = a.h2, ih2 = a.ih2, bscl = (float)a.bq[0];
  const float* __restrict__ sbR = a.sb;
  const float* __restrict__ sbB = a.sb + half;
  const float* __restrict__ rhR = a.rhs;
  const float* __restrict__ rhB = a.rhs + half;
  float* __restrict__ outR = a.e_out;
  float* __restrict__ outB = a.e_out + half;
  double accR = 0.0, accB = 0.0;

  // red update of the cell at LDS offsets (c2 in the halo-2 planes, z2 its k - 1 neighbour) with old
  // slots SM, S0, SP of planes t - 1, t, t + 1
  auto red_at = [&](auto smc, auto s0c, auto spc, int c2, int z2, float sbv, float rhv, float& g) -> float {
    constexpr int SM = decltype(smc)::value, S0 = decltype(s0c)::value, SP = decltype(spc)::value;
    const float* eR_m = lds + (SM * 2) * S2;
    const float* eR_p = lds + (SP * 2) * S2;
    const float* eR_0 = lds + (S0 * 2) * S2;
    const float* eB_m = lds + (SM * 2 + 1) * S2;
    const float* eB_p = lds + (SP * 2 + 1) * S2;
    const float* eB_0 = lds + (S0 * 2 + 1) * S2;
    Nb18f te, tb;
#define MR_LF_RED(T_, O)                                                                             \
    T_.xm = eB_m[O + c2];         T_.xp = eB_p[O + c2];                                              \
    T_.ym = eB_0[O + c2 - W2];    T_.yp = eB_0[O + c2 + W2];                                         \
    T_.zm = eB_0[O + z2];         T_.zp = eB_0[O + z2 + 1];                                          \
    T_.xpyp = eR_p[O + c2 + W2];  T_.xmym = eR_m[O + c2 - W2];                                       \
    T_.xpym = eR_p[O + c2 - W2];  T_.xmyp = eR_m[O + c2 + W2];                                       \
    T_.xpzp = eR_p[O + z2 + 1];   T_.xmzm = eR_m[O + z2];                                            \
    T_.xpzm = eR_p[O + z2];       T_.xmzp = eR_m[O + z2 + 1];                                        \
    T_.ypzp = eR_0[O + z2 + 1 + W2]; T_.ymzm = eR_0[O + z2 - W2];                                    \
    T_.ypzm = eR_0[O + z2 + W2];  T_.ymzp = eR_0[O + z2 + 1 - W2];
    MR_LF_RED(te, 0)
    MR_LF_RED(tb, OB)
#undef MR_LF_RED
    float Se;
    g = lin_source(tb, eR_0[OB + c2], bscl, sbv, ih2, te, Se) * ih2;
    return (Se - h2 * (g + rhv - C)) * (1.0f / 6.0f);
  };

  float X0[NPF], X1[NPF];
  float SR[2], RR[2], SH[2], RH[2], SBk[2], RBk[2];
  {
    float va[NPF];
    fetch(i0 - 2, va);
    store(0, va);
    fetch(i0 - 1, va);
    store(1, va);
    fetch(i0, va);
    store(2, va);
  }
  fetch(i0 + 1, X1);   // stored at the end of step 0
  SR[0] = ld_rs_f(prs(sbR, i0 - 1), o_c);
  RR[0] = ld_rs_f(prs(rhR, i0 - 1), o_c);
  SH[0] = has_halo ? ld_rs_f(prs(sbR, i0 - 1), o_h) : 0.0f;
  RH[0] = has_halo ? ld_rs_f(prs(rhR, i0 - 1), o_h) : 0.0f;
  SBk[0] = 0.0f;
  RBk[0] = 0.0f;
  __syncthreads();

  auto step = [&](auto kc, int u) {
    constexpr int K = decltype(kc)::value;
    constexpr int P = K & 1;                                   // parity index of this step
    constexpr int OM = (K + 0) % 5, O0 = (K + 1) % 5, OP = (K + 2) % 5, OQ = (K + 3) % 5;  // old planes t-1..t+2
    constexpr int OMM = (K + 4) % 5;                           // old plane t - 2
    constexpr int N0 = K % 5, NM = (K + 4) % 5, NMM = (K + 3) % 5;   // new red planes t, t - 1, t - 2
    constexpr int CUR = K & 1, NXT = (K + 1) & 1;
    if (u >= U) return;
    const int t = i0 - 1 + u;
    float(&xf)[NPF] = (K & 1) ? X1 : X0;   // fetched now (plane t + 3)
    float(&xs)[NPF] = (K & 1) ? X0 : X1;   // fetched last step (plane t + 2), stored at the end
    if (t + 3 <= i1 + 1) fetch(t + 3, xf);
    // inputs of the next step: red of plane t + 1 (own, ring), black of plane t
    if (u + 1 < U) {
      SR[NXT] = ld_rs_f_nt(prs(sbR, t + 1), o_c);
      RR[NXT] = ld_rs_f_nt(prs(rhR, t + 1), o_c);
      if (has_halo) {
        SH[NXT] = ld_rs_f(prs(sbR, t + 1), o_h);
        RH[NXT] = ld_rs_f(prs(rhR, t + 1), o_h);
      }
      if (t >= i0) {
        SBk[NXT] = ld_rs_f_nt(prs(sbB, t), o_c);
        RBk[NXT] = ld_rs_f_nt(prs(rhB, t), o_c);
      }
    }
    // phase A: red cells of plane t
    {
      float g;
      const float v = red_at(std::integral_constant<int, OM>(), std::integral_constant<int, O0>(),
                             std::integral_constant<int, OP>(), ob2, oz2[P], SR[CUR], RR[CUR], g);
      lds[ON + N0 * S1 + ob1] = v;
      if (t >= i0 && t < i1) {
        st_rs_f_nt(prs(outR, t), o_c, v);
        accR += (double)(g + RR[CUR]);
      }
      if (has_halo) {
        float gh;
        lds[ON + N0 * S1 + hb1] = red_at(std::integral_constant<int, OM>(), std::integral_constant<int, O0>(),
                                         std::integral_constant<int, OP>(), hb2, hz2[P], SH[CUR], RH[CUR], gh);
      }
    }
    __syncthreads();
    // phase B: black cells of plane t - 1 (own tile); the black row parity at plane t - 1 is that of
    // the red cells of plane t
    if (t - 1 >= i0) {
      const float* nRm = lds + ON + NMM * S1;   // new red, plane t - 2
      const float* nR0 = lds + ON + NM * S1;    // plane t - 1
      const float* nRp = lds + ON + N0 * S1;    // plane t
      const float* eBm = lds + (OMM * 2 + 1) * S2;   // old black, planes t - 2, t - 1, t
      const float* eB0 = lds + (OM * 2 + 1) * S2;
      const float* eBp = lds + (O0 * 2 + 1) * S2;
      const float* bRm = lds + OB + (OMM * 2) * S2;  // base red, planes t - 2, t - 1, t
      const float* bR0 = lds + OB + (OM * 2) * S2;
      const float* bRp = lds + OB + (O0 * 2) * S2;
      const int c2 = ob2, z2 = oz2[P], c1 = ob1, z1 = oz1[P];
      Nb18f te, tb;
      te.xm = nRm[c1];       te.xp = nRp[c1];
      te.ym = nR0[c1 - W1];  te.yp = nR0[c1 + W1];
      te.zm = nR0[z1];       te.zp = nR0[z1 + 1];
      tb.xm = bRm[c2];       tb.xp = bRp[c2];
      tb.ym = bR0[c2 - W2];  tb.yp = bR0[c2 + W2];
      tb.zm = bR0[z2];       tb.zp = bR0[z2 + 1];
#define MR_LF_EDGES(T_, O)                                                                           \
      T_.xpyp = eBp[O + c2 + W2];  T_.xmym = eBm[O + c2 - W2];                                       \
      T_.xpym = eBp[O + c2 - W2];  T_.xmyp = eBm[O + c2 + W2];                                       \
      T_.xpzp = eBp[O + z2 + 1];   T_.xmzm = eBm[O + z2];                                            \
      T_.xpzm = eBp[O + z2];       T_.xmzp = eBm[O + z2 + 1];                                        \
      T_.ypzp = eB0[O + z2 + 1 + W2]; T_.ymzm = eB0[O + z2 - W2];                                    \
      T_.ypzm = eB0[O + z2 + W2];  T_.ymzp = eB0[O + z2 + 1 - W2];
      MR_LF_EDGES(te, 0)
      MR_LF_EDGES(tb, OB)
#undef MR_LF_EDGES
      float Se;
      const float g = lin_source(tb, eB0[OB + c2], bscl, SBk[CUR], ih2, te, Se) * ih2;
      st_rs_f_nt(prs(outB, t - 1), o_c, (Se - h2 * (g + RBk[CUR] - C)) * (1.0f / 6.0f));
      accB += (double)(g + RBk[CUR]);
    }
    if (t + 2 <= i1 + 1) store(OQ, xs);
    __syncthreads();
  };
  for (int u0 = 0; u0 < U; u0 += 10) {
    step(std::integral_constant<int, 0>(), u0);
    step(std::integral_constant<int, 1>(), u0 + 1);
    step(std::integral_constant<int, 2>(), u0 + 2);
    step(std::integral_constant<int, 3>(), u0 + 3);
    step(std::integral_constant<int, 4>(), u0 + 4);
    step(std::integral_constant<int, 5>(), u0 + 5);
    step(std::integral_constant<int, 6>(), u0 + 6);
    step(std::integral_constant<int, 7>(), u0 + 7);
    step(std::integral_constant<int, 8>(), u0 + 8);
    step(std::integral_constant<int, 9>(), u0 + 9);
  }
  double vv[2] = {accR, accB};
  grid_sum<2>(vv, a.partials, a.counter, a.sum_out, nblocks, bid);
}

// ---- vector kernels of the Krylov-accelerated inner solve -------------------------------------
constexpr int kKryMax = 8;          // longest Krylov space of the inner solve
constexpr int kKryBlocks = 1024;    // blocks of the reducing vector kernels
constexpr int kApplyBlocks = 256;   // preferred block count of the fused operator product
constexpr int kKryNV = kKryMax + 2; // values reduced per block
struct KryPtrs {
  const float* p[kKryMax + 1];
};
struct KryCoef {
  double c[kKryMax + 1];
};

// ---- the linear operator applied to both colours in one pass, with the Krylov projections ------
// w = nabla^2 z - dSigma(z) at every cell, and the sums w v_j (j < K), w and w^2. The pipelined
// sweep's tile decomposition and 4-slot plane ring (z and the base, both colours, one-cell halo);
// the block has two threads per (j, m) column of its TM x TJ tile, the first half evaluating the red
// cell of each plane and the second half the black one. No cell depends on another's result, so one
// launch covers both colours, and the projections are accumulated where w is produced.
struct LinApplyArgs {
  const float* z;
  const int* base;
  const double* bq;
  const float* sb;
  float* w;
  int n;
  float ih2;
  int tiles_j, tiles_m, ci;
  KryPtrs v;
  double* partials;
  unsigned* counter;
  double* result;
};

template <int TM, int TJ, int K>
__device__ void lin_apply_dots_body(const LinApplyArgs& a, int logical, int bid, int nblocks, float* lds) {
  constexpr int NC = TM * TJ;        // columns of the tile
  constexpr int NT = 2 * NC;         // threads
  constexpr int RW = TM + 2;
  constexpr int SLOT = LinTile<TM, TJ>::SLOT;
  constexpr int PER = (SLOT + NT - 1) / NT;
  constexpr int NPF = 4 * PER;
  const int n = a.n, nh = n >> 1;
  const int tid = threadIdx.x;
  const int tm_i = logical % a.tiles_m;
  const int tj_i = (logical / a.tiles_m) % a.tiles_j;
  const int chunk = logical / (a.tiles_m * a.tiles_j);
  const int j0 = tj_i * TJ, m0 = tm_i * TM, i0 = chunk * a.ci, ci = a.ci;
  const size_t plane = (size_t)n * nh;
  const size_t half = plane * n;
  const unsigned pbytes = (unsigned)plane * 4u;
  const float* __restrict__ f0 = a.z;
  const float* __restrict__ f1 = a.z + half;
  const float* __restrict__ f2 = reinterpret_cast<const float*>(a.base);
  const float* __restrict__ f3 = reinterpret_cast<const float*>(a.base) + half;
  auto prs = [&](const float* arr, int p) { return plane_rsrc(arr + (size_t)p * plane, pbytes); };
  unsigned goff[PER];
  int loff[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int e = tid + k * NT;
    e = e < SLOT ? e : SLOT - 1;
    const int r = e / RW;
    const int c = e - r * RW;
    goff[k] = ((unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh)) * 4u;
    loff[k] = e;
  }
  auto fetch = [&](int rel, float (&v)[NPF]) {
    const int p = wrapi(i0 - 1 + rel, n);
    const auto b0 = prs(f0, p), b1 = prs(f1, p), b2 = prs(f2, p), b3 = prs(f3, p);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[0 * PER + k] = ld_rs_f(b0, goff[k]);
      v[1 * PER + k] = ld_rs_f(b1, goff[k]);
      v[2 * PER + k] = ld_rs_f(b2, goff[k]);
      v[3 * PER + k] = ld_rs_f(b3, goff[k]);
    }
  };
  auto store = [&](int slot, const float (&v)[NPF]) {
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int k = 0; k < PER; ++k) lds[(f * 4 + slot) * SLOT + loff[k]] = v[f * PER + k];
  };
  // colour of this thread's cells: the same on every lane of a wave (NC is a multiple of 64), taken
  // from the wave's first lane so that the compiler keeps the colour's pointers in scalar registers
  static_assert(NC % 64 == 0, "whole waves per colour");
  const int c = __builtin_amdgcn_readfirstlane(tid) / NC;
  const int col = tid - c * NC;
  const int s = col % TM, r = col / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned o_c = ((unsigned)j * nh + m) * 4u;
  const int ob = (r + 1) * RW + (s + 1);
  const int q0 = (i0 + j + c) & 1;
  const int oq0 = ob + q0, oq1 = ob + (q0 ^ 1);
  const float ih2 = a.ih2, bscl = (float)a.bq[0];
  const float* __restrict__ sbc = a.sb + c * half;
  float* __restrict__ out = a.w + c * half;
  const int last_plane = n - 1;
  const float* lo = lds + (1 - c) * 4 * SLOT;       // z of the other colour
  const float* lc = lds + c * 4 * SLOT;             // z of this colour
  const float* bo = lds + (3 - c) * 4 * SLOT;       // base of the other colour
  const float* bc = lds + (2 + c) * 4 * SLOT;       // base of this colour
  // projections: FP32 partial sums over the four plane steps of a ring cycle, added into FP64
  // accumulators at its end
  double acc[K + 2];
  float accf[K + 2];
#pragma unroll
  for (int q = 0; q < K + 2; ++q) {
    acc[q] = 0.0;
    accf[q] = 0.0f;
  }
  float V0[NPF], V1[NPF];
  float SB[4];
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
  SB[0] = ld_rs_f_nt(prs(sbc, i0), o_c);
  SB[1] = ld_rs_f_nt(prs(sbc, min(i0 + 1, last_plane)), o_c);
  // the Krylov vectors at the thread's cell, one plane step ahead (two register sets)
  constexpr int KV = K > 0 ? K : 1;
  float VJ[2][KV];
#pragma unroll
  for (int q = 0; q < K; ++q) VJ[0][q] = ld_rs_f_nt(prs(a.v.p[q] + c * half, i0), o_c);
  __syncthreads();
  auto step = [&](auto kc, int t, float (&vst)[NPF], float (&vft)[NPF]) {
    constexpr int KK = decltype(kc)::value;
    constexpr int SM = KK & 3, S0 = (KK + 1) & 3, SP = (KK + 2) & 3, SN = (KK + 3) & 3;
    fetch(t + 4, vft);
    SB[(KK + 2) & 3] = ld_rs_f_nt(prs(sbc, min(i0 + t + 2, last_plane)), o_c);
    const float (&vj)[KV] = VJ[KK & 1];
#pragma unroll
    for (int q = 0; q < K; ++q) VJ[(KK + 1) & 1][q] = ld_rs_f_nt(prs(a.v.p[q] + c * half, min(i0 + t + 1, last_plane)), o_c);
    const int oq = (KK & 1) ? oq1 : oq0;
    Nb18f te, tb;
#define MR_AD_GATHER(T, LO, LC)                                                        \
    T.xm = LO[SM * SLOT + ob];         T.xp = LO[SP * SLOT + ob];                       \
    T.ym = LO[S0 * SLOT + ob - RW];    T.yp = LO[S0 * SLOT + ob + RW];                  \
    T.zm = LO[S0 * SLOT + oq - 1];     T.zp = LO[S0 * SLOT + oq];                       \
    T.xpyp = LC[SP * SLOT + ob + RW];  T.xmym = LC[SM * SLOT + ob - RW];                \
    T.xpym = LC[SP * SLOT + ob - RW];  T.xmyp = LC[SM * SLOT + ob + RW];                \
    T.xpzp = LC[SP * SLOT + oq];       T.xmzm = LC[SM * SLOT + oq - 1];                 \
    T.xpzm = LC[SP * SLOT + oq - 1];   T.xmzp = LC[SM * SLOT + oq];                     \
    T.ypzp = LC[S0 * SLOT + oq + RW];  T.ymzm = LC[S0 * SLOT + oq - RW - 1];            \
    T.ypzm = LC[S0 * SLOT + oq + RW - 1]; T.ymzp = LC[S0 * SLOT + oq - RW];
    MR_AD_GATHER(te, lo, lc)
    MR_AD_GATHER(tb, bo, bc)
#undef MR_AD_GATHER
    float Se;
    const float g = lin_source(tb, bc[S0 * SLOT + ob], bscl, SB[KK], ih2, te, Se) * ih2;
    const float wv = (Se - 6.0f * lc[S0 * SLOT + ob]) * ih2 - g;
    st_rs_f_nt(prs(out, i0 + t), o_c, wv);
#pragma unroll
    for (int q = 0; q < K; ++q) accf[q] = __builtin_fmaf(wv, vj[q], accf[q]);
    accf[K] += wv;
    accf[K + 1] = __builtin_fmaf(wv, wv, accf[K + 1]);
    if (KK == 3) {
#pragma unroll
      for (int q = 0; q < K + 2; ++q) {
        acc[q] += (double)accf[q];
        accf[q] = 0.0f;
      }
    }
    store(SN, vst);
    __syncthreads();
  };
  for (int t = 0; t < ci; t += 4) {
    step(std::integral_constant<int, 0>(), t, V0, V1);
    step(std::integral_constant<int, 1>(), t + 1, V1, V0);
    step(std::integral_constant<int, 2>(), t + 2, V0, V1);
    step(std::integral_constant<int, 3>(), t + 3, V1, V0);
  }
  grid_sum<K + 2>(acc, a.partials, a.counter, a.result, nblocks, bid);
}

// Sums over all cells of w v_j (j < K) into result[j], of w into result[K] and of w^2 into
// result[K + 1]: 16-byte loads, four FP32 products per lane and step added into FP64 accumulators.
template <int K>
__device__ void kry_dots_body(const float* __restrict__ w, const KryPtrs& v, size_t cells, double* partials,
                              unsigned* counter, double* result, int bid, int nblocks) {
  double acc[K + 2];
#pragma unroll
  for (int j = 0; j < K + 2; ++j) acc[j] = 0.0;
  const float4* __restrict__ w4 = reinterpret_cast<const float4*>(w);
  const size_t n4 = cells / 4;
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < n4; x += (size_t)nblocks * blockDim.x) {
    const float4 a = w4[x];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const float4 b = reinterpret_cast<const float4*>(v.p[j])[x];
      acc[j] += (double)(a.x * b.x + a.y * b.y) + (double)(a.z * b.z + a.w * b.w);
    }
    acc[K] += (double)(a.x + a.y) + (double)(a.z + a.w);
    acc[K + 1] += (double)(a.x * a.x + a.y * a.y) + (double)(a.z * a.z + a.w * a.w);
  }
  grid_sum<K + 2>(acc, partials, counter, result, nblocks, bid);
}

// out = (w - sum_{j<k} c_j v_j - c_k) c_{k+1}: the next orthonormal Krylov vector (classical
// Gram-Schmidt against mean-free orthonormal v_j, the mean c_k removed, scaled by c_{k+1}).
inline __device__ void kry_orth_body(const float* __restrict__ w, const KryPtrs& v, KryCoef c, int k, size_t cells,
                                     float* __restrict__ out, int bid, int nblocks) {
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x) {
    double s = (double)w[x] - c.c[k];
#pragma unroll
    for (int j = 0; j < kKryMax; ++j)
      if (j < k) s -= c.c[j] * (double)v.p[j][x];
    out[x] = (float)(s * c.c[k + 1]);
  }
}

// theta += sum_{j<m} y_j z_j; max |theta| of the result into *tmax (atomic maximum) when given.
inline __device__ void kry_update_body(double* __restrict__ theta, const KryPtrs& z, KryCoef y, int m, size_t cells,
                                       double* tmax, int bid, int nblocks) {
  double mx = 0.0;
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x) {
    double s = theta[x];
#pragma unroll
    for (int j = 0; j < kKryMax; ++j)
      if (j < m) s += y.c[j] * (double)z.p[j][x];
    theta[x] = s;
    mx = fmax(mx, fabs(s));
  }
  if (tmax) block_absmax_to(mx, tmax);
}

}  // namespace mr
