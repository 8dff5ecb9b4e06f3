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
#include "mr_ctx.h"
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
  const float inv = 1.0f / (3.0f * s * s - 4.5f * T2);
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
__global__ void __launch_bounds__(TM * TJ) lin_half_sweep_tiled(LinSweepArgs a) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int TOTAL = 4 * SLOT;
  constexpr int NPF = (TOTAL + NT - 1) / NT;
  __shared__ float lds[4 * 4 * SLOT];
  const int n = a.n, nh = n >> 1, c = a.colour;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
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
  const bool last = grid_sum<1>(vv, a.partials, a.counter, a.sum_out, gridDim.x, blockIdx.x);
  if (last && tid == 0 && a.copy_to) *a.copy_to = *a.copy_from;
}

// ---- simple kernels of the mixed form (row mapping as in transfer.hip) ----------------------

// FP64 outer residual on the finest mesh: b = nabla^2 theta - Sigma + C; rhs32 = -b, base32 =
// theta, sb32 = the physical root s. Sums: b, b^2, Sigma.
__global__ void __launch_bounds__(256) mixed_resid64_kernel(const double* __restrict__ theta,
    const double* __restrict__ delta, int n, double C, float* __restrict__ rhs32, float* __restrict__ base32,
    float* __restrict__ sb32, Reduce red) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const int rows = n * n;
  const int rpb = (rows + gridDim.x - 1) / gridDim.x;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rpb;
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
  double v[3] = {a0, a1, a2};
  grid_sum<3>(v, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// Base root on a coarse mesh (cell size h) from the restricted FP32 base potential.
__global__ void __launch_bounds__(256) base_root_kernel(const float* __restrict__ base32,
    const double* __restrict__ delta, int n, double ih2, float* __restrict__ sb32) {
  const int row = xcd_remap(blockIdx.x, gridDim.x);
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

__global__ void __launch_bounds__(512) restrict32_kernel(const float* __restrict__ fine, float* __restrict__ coarse, int n) {
  const int m = n >> 1;
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int I = row / m, J = row - I * m;
  const int K = threadIdx.x;
  if (K >= m) return;
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += fine[split_idx(n, 2 * I + (q >> 2), 2 * J + ((q >> 1) & 1), 2 * K + (q & 1))];
  coarse[split_idx(m, I, J, K)] = 0.125f * s;
}

// Residual of the linear level equation and its restriction: res = rhs + dSigma(e) - lap(e) - C,
// rhs_c = R res (one thread per coarse cell). result[0..1] = (sum of rhs_c, 0).
__global__ void __launch_bounds__(256) lin_resid_restrict_kernel(const float* __restrict__ e,
    const float* __restrict__ base, const float* __restrict__ sb, const float* __restrict__ rhs, int n, float h2,
    float ih2, ShiftRef cref, float* __restrict__ rhs_c, Reduce red) {
  const int m = n >> 1;
  const double Cd = (cref.c_sum ? (cref.c_sum[0] + cref.c_sum[1]) * cref.c_scale : 0.0) + cref.c_add;
  const float C = (float)Cd;
  double acc = 0.0;
  const int rows = m * m;
  const int rpb = (rows + gridDim.x - 1) / gridDim.x;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rpb;
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
  grid_sum<2>(vv, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// e += P(ec) (trilinear, cell pair per thread; see prolong_correct_kernel).
__global__ void __launch_bounds__(512) prolong_add32_kernel(const float* __restrict__ ec, float* __restrict__ e, int n) {
  const int nh = n >> 1;
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int i = row / n, j = row - i * n;
  const int m = threadIdx.x;
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

// Linear coarsest solve: nsweeps red-black sweeps in one block (FP32, natural order in LDS).
__global__ void __launch_bounds__(256) lin_coarsest_kernel(float* __restrict__ e, const float* __restrict__ base,
    const float* __restrict__ sb, const float* __restrict__ rhs, int n, int nsweeps, float h2, float ih2,
    const double* c_sum, double c_scale) {
  __shared__ float te[kMaxCoarsest], tb[kMaxCoarsest], ts[kMaxCoarsest], tr[kMaxCoarsest], tn[kMaxCoarsest];
  __shared__ double red[16][1];
  __shared__ float cnew;
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

__global__ void __launch_bounds__(256) update64_kernel(double* __restrict__ theta, const float* __restrict__ e, size_t cells) {
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)gridDim.x * blockDim.x)
    theta[x] += (double)e[x];
}

__global__ void __launch_bounds__(256) fill32_kernel(float* __restrict__ a, float v, size_t cells) {
  for (size_t x = blockIdx.x * (size_t)blockDim.x + threadIdx.x; x < cells; x += (size_t)gridDim.x * blockDim.x) a[x] = v;
}

// ---- launchers ----------------------------------------------------------------------------

static int lin_blocks(size_t cells) {
  size_t b = (cells + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}
static int rows_blocks(int n) { return n * n < 4096 ? n * n : 4096; }
static int row_threads(int n) { return n < 64 ? 64 : (n < 256 ? n : 256); }

#define MR_LIN_TILES(X) X(64, 4) X(32, 8) X(16, 16) X(8, 16) X(4, 8) X(2, 4)

bool lin_tile_supported(int tm, int tj) {
#define MR_LIN_MATCH(TM, TJ) if (tm == TM && tj == TJ) return true;
  MR_LIN_TILES(MR_LIN_MATCH)
#undef MR_LIN_MATCH
  return false;
}

hipError_t launch_lin_half_sweep(const LinSweepArgs& a, const TileCfg& t, hipStream_t s) {
  const long blocks_l = (long)t.tiles_j * t.tiles_m * (a.n / t.ci);
  if (blocks_l < 1 || blocks_l > kMaxReduceBlocks || t.tj * t.tiles_j != a.n || t.tm * t.tiles_m != a.n / 2 ||
      a.n % t.ci != 0)
    return hipErrorInvalidValue;
  LinSweepArgs b = a;
  b.tiles_j = t.tiles_j;
  b.tiles_m = t.tiles_m;
  b.ci = t.ci;
  const int blocks = (int)blocks_l;
#define MR_LIN_LAUNCH(TM, TJ)                                                                  \
  if (t.tm == TM && t.tj == TJ) {                                                              \
    hipLaunchKernelGGL((lin_half_sweep_tiled<TM, TJ>), dim3(blocks), dim3(TM * TJ), 0, s, b);  \
    return hipGetLastError();                                                                  \
  }
  MR_LIN_TILES(MR_LIN_LAUNCH)
#undef MR_LIN_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_mixed_resid64(const double* theta, const double* delta, int n, double C, float* rhs32, float* base32,
                                float* sb32, Reduce red, hipStream_t s) {
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
  const int m = n / 2;
  hipLaunchKernelGGL(lin_resid_restrict_kernel, dim3(rows_blocks(m)), dim3(row_threads(m)), 0, s, e, base, sb, rhs, n,
                     (float)(h * h), (float)(1.0 / (h * h)), c, rhs_c, red);
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
  double C64 = m0;  // shift of the outer residual (mean of Sigma at the previous iterate)
  mr_info loc{};
  loc.r0_norm = r0;
  int it = 0, status = MR_OK;
  double rel = 1.0, best = 1e300, msig = m0;
  LinLevel& M0 = mixed->lv[0];
  for (;;) {
    e = launch_mixed_resid64(L0.th[0], L0.delta, L0.n, C64, M0.rhs, M0.base, M0.sb, reducer(kSlotRes), stream);
    if (e != hipSuccess) return hip_fail(e, "mixed residual");
    double r[3];
    if ((rc = read_scalars(kSlotRes, 3, r)) != MR_OK) return rc;
    const double var = r[1] - r[0] * r[0] / N3;
    rel = std::sqrt(var > 0.0 ? var : 0.0) / r0;
    msig = r[2] / N3;
    if (it < 128) loc.history[it] = rel;
    if (!std::isfinite(rel) || rel > 1e6 * (best < 1.0 ? 1.0 : best)) {
      status = fail(MR_EDIVERGED, "residual diverged at outer iteration %d (%g)", it, rel);
      break;
    }
    if (rel < best) best = rel;
    if (rel <= opts.tol || it >= opts.max_cycles) break;
    C64 = msig;
    // base hierarchy for the linear operator
    for (int l = 1; l < nlev; ++l) {
      e = launch_restrict32(mixed->lv[l - 1].base, mixed->lv[l].base, lv[l - 1].n, stream);
      if (e == hipSuccess) e = launch_base_root(mixed->lv[l].base, lv[l].delta, lv[l].n, lv[l].h, mixed->lv[l].sb, stream);
      if (e != hipSuccess) return hip_fail(e, "linear base hierarchy");
    }
    // inner solve from e = 0; the shift starts at <rhs> = -<b>
    M0.cur = 0;
    if ((e = launch_fill32(M0.e[0], 0.0f, L0.cells, stream)) != hipSuccess) return hip_fail(e, "fill");
    host[0] = -r[0];
    host[1] = 0.0;
    if ((e = hipMemcpyAsync(linsum(0), host, 2 * sizeof(double), hipMemcpyHostToDevice, stream)) != hipSuccess)
      return hip_fail(e, "inner shift");
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
