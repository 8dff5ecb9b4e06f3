// Device bodies of the mixed-precision kernels. Each body processes the share of one mesh given
// by (bid, nblocks), so that the same code serves one-mesh launches (bid = blockIdx.x) and
// multi-box launches (bid = the block's rank within its box).
#pragma once

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

// h^2 dSigma(e) for a cell with base neighbours b, base root s and perturbation neighbours e;
// also returns the face-neighbour sum of e. FP32.
__device__ __forceinline__ float lin_source(const Nb18f& b, float s, float ih2, const Nb18f& e, float& Se) {
  const float bSx = b.xm + b.xp, bSy = b.ym + b.yp, bSz = b.zm + b.zp;
  const float bS3 = (bSx + bSy + bSz) * (1.0f / 3.0f);
  const float mx = (bSx - bS3) * ih2, my = (bSy - bS3) * ih2, mz = (bSz - bS3) * ih2;
  const float mxy = 0.25f * ((b.xpyp + b.xmym) - (b.xpym + b.xmyp)) * ih2;
  const float mxz = 0.25f * ((b.xpzp + b.xmzm) - (b.xpzm + b.xmzp)) * ih2;
  const float myz = 0.25f * ((b.ypzp + b.ymzm) - (b.ypzm + b.ymzp)) * ih2;
  const float xy2 = mxy * mxy, xz2 = mxz * mxz, yz2 = myz * myz;
  const float T2 = mx * mx + my * my + mz * mz + 2.0f * (xy2 + xz2 + yz2);
  // hardware reciprocal: the linearised operator only steers the defect correction
  const float inv = __builtin_amdgcn_rcpf(3.0f * s * s - 4.5f * T2);
  const float s9 = 9.0f * s;
  const float q9 = 9.0f * T2;
  const float Wxx = (s9 * mx - 27.0f * (mx * mx + xy2 + xz2) + q9) * inv;
  const float Wyy = (s9 * my - 27.0f * (xy2 + my * my + yz2) + q9) * inv;
  const float Wzz = (s9 * mz - 27.0f * (xz2 + yz2 + mz * mz) + q9) * inv;
  const float Wxy = (s9 * mxy - 27.0f * (mx * mxy + mxy * my + mxz * myz)) * inv;
  const float Wxz = (s9 * mxz - 27.0f * (mx * mxz + mxy * myz + mxz * mz)) * inv;
  const float Wyz = (s9 * myz - 27.0f * (mxy * mxz + my * myz + myz * mz)) * inv;
  const float eSx = e.xm + e.xp, eSy = e.ym + e.yp, eSz = e.zm + e.zp;
  Se = eSx + eSy + eSz;
  const float eDxy = (e.xpyp + e.xmym) - (e.xpym + e.xmyp);
  const float eDxz = (e.xpzp + e.xmzm) - (e.xpzm + e.xmzp);
  const float eDyz = (e.ypzp + e.ymzm) - (e.ypzm + e.ymzp);
  return Wxx * eSx + Wyy * eSy + Wzz * eSz + 0.5f * (Wxy * eDxy + Wxz * eDxz + Wyz * eDyz);
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
  const float* __restrict__ f2 = a.base;                               // base red
  const float* __restrict__ f3 = a.base + half;                        // base black

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
    const float g = lin_source(tb, sbc[e], ih2, te, Se) * ih2;
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
                                   ShiftRef cref, float* __restrict__ rhs32, float* __restrict__ base32,
                                   float* __restrict__ sb32, Reduce red, int bid, int nblocks) {
  const double C = (cref.c_sum ? (cref.c_sum[0] + cref.c_sum[1]) * cref.c_scale : 0.0) + cref.c_add;
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
      base32[e] = (float)th;
      sb32[e] = (float)(sig + 3.0);
      a0 += b;
      a1 += b * b;
      a2 += sig;
    }
  }
  double v[4] = {a2, 0.0, a0, a1};
  return grid_sum<4>(v, red.partials, red.counter, red.result, nblocks, bid);
}
// Base root on a coarse mesh (cell size h) from the restricted FP32 base potential; rows
// bid, bid + nblocks, ... of the mesh.
inline __device__ void base_root_body(const float* __restrict__ base32, const double* __restrict__ delta, int n, double ih2,
                               float* __restrict__ sb32, int bid, int nblocks) {
  for (int row = xcd_remap(bid, nblocks); row < n * n; row += nblocks) {
    const int i = row / n, j = row - i * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const unsigned e = split_idx(n, i, j, k);
      Nb18f tf;
      gather18_split_t(base32, n, i, j, k, tf);
      Nb18 t{tf.xm, tf.xp, tf.ym, tf.yp, tf.zm, tf.zp, tf.xpyp, tf.xmym, tf.xpym, tf.xmyp,
             tf.xpzp, tf.xmzm, tf.xpzm, tf.xmzp, tf.ypzp, tf.ymzm, tf.ypzm, tf.ymzp};
      double S;
      sb32[e] = (float)(sigma_cell(t, 1.0 + delta[e], ih2, S) + 3.0);
    }
  }
}
// 8-son mean, coarse rows bid, bid + nblocks, ...
inline __device__ void restrict32_body(const float* __restrict__ fine, float* __restrict__ coarse, int n, int bid, int nblocks) {
  const int m = n >> 1;
  for (int row = xcd_remap(bid, nblocks); row < m * m; row += nblocks) {
    const int I = row / m, J = row - I * m;
    for (int K = threadIdx.x; K < m; K += blockDim.x) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += fine[split_idx(n, 2 * I + (q >> 2), 2 * J + ((q >> 1) & 1), 2 * K + (q & 1))];
      coarse[split_idx(m, I, J, K)] = 0.125f * s;
    }
  }
}
// Residual of the linear level equation and its restriction: res = rhs + dSigma(e) - lap(e) - C,
// rhs_c = R res (one thread per coarse cell). result[0..1] = (sum of rhs_c, 0).
inline __device__ void lin_resid_restrict_body(const float* __restrict__ e, const float* __restrict__ base,
    const float* __restrict__ sb, const float* __restrict__ rhs, int n, float ih2, ShiftRef cref,
    float* __restrict__ rhs_c, Reduce red, int bid, int nblocks) {
  const int m = n >> 1;
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
        const float src = lin_source(tb, sb[g], ih2, te, Se) * ih2;
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
// e += P(ec) (trilinear, cell pair per thread; see prolong_correct_kernel).
inline __device__ void prolong_add32_row(const float* __restrict__ ec, float* __restrict__ e, int n, int row, int m) {
  const int nh = n >> 1;
  const int i = row / n, j = row - i * n;
  if (m >= nh) return;
  const int nc = n >> 1;
  const int I = i >> 1, J = j >> 1, K = m;
  const int I2 = wrapi((i & 1) ? I + 1 : I - 1, nc);
  const int J2 = wrapi((j & 1) ? J + 1 : J - 1, nc);
  const int Km = wrapi(K - 1, nc), Kp = wrapi(K + 1, nc);
  const float wI[2] = {0.75f, 0.25f};
  float lo = 0.0f, hi = 0.0f;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int ii = (s & 2) ? I2 : I, jj = (s & 1) ? J2 : J;
    const float w = wI[(s >> 1) & 1] * wI[s & 1];
    const float ek = ec[split_idx(nc, ii, jj, K)];
    lo += w * (0.75f * ek + 0.25f * ec[split_idx(nc, ii, jj, Km)]);
    hi += w * (0.75f * ek + 0.25f * ec[split_idx(nc, ii, jj, Kp)]);
  }
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)nh;
  const unsigned off = ((unsigned)i * n + j) * (unsigned)nh + m;
  const int c0 = (i + j) & 1;
  e[c0 * half + off] += lo;
  e[(1 - c0) * half + off] += hi;
}

inline __device__ void prolong_add32_body(const float* __restrict__ ec, float* __restrict__ e, int n, int bid, int nblocks) {
  for (int row = xcd_remap(bid, nblocks); row < n * n; row += nblocks)
    for (int m = threadIdx.x; m < n / 2; m += blockDim.x) prolong_add32_row(ec, e, n, row, m);
}
// Linear coarsest solve: nsweeps red-black sweeps in one block (FP32, natural order in LDS).
struct LinCoarsestShared {
  float te[kMaxCoarsest], tb[kMaxCoarsest], ts[kMaxCoarsest], tr[kMaxCoarsest], tn[kMaxCoarsest];
  double red[16][1];
  float cnew;
};

inline __device__ void lin_coarsest_body(float* __restrict__ e, const float* __restrict__ base, const float* __restrict__ sb,
                                  const float* __restrict__ rhs, int n, int nsweeps, float h2, float ih2,
                                  const double* c_sum, double c_scale, LinCoarsestShared& sh) {
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
        const float g = lin_source(vb, ts[x], ih2, ve, Se) * ih2;
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
inline __device__ void update64_body(double* __restrict__ theta, const float* __restrict__ e, size_t cells, int bid, int nblocks) {
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x)
    theta[x] += (double)e[x];
}

inline __device__ void fill32_body(float* __restrict__ a, float v, size_t cells, int bid, int nblocks) {
  for (size_t x = bid * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)nblocks * blockDim.x) a[x] = v;
}

}  // namespace mr
