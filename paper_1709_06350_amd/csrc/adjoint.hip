// Adjoint of the solve: gradient of a loss L(theta(delta)) with respect to delta, FP64.
//
// With F(theta, delta) = nabla^2 theta - Sigma + <Sigma> (the mean-projected operator of Sec. II.A.1,
// Eq. 15) and the gauge <theta> = 0, dL/d(delta) = D * (lambda - <lambda>) where
// J_p^T lambda = g - <g>, g = dL/dtheta, J_p the Jacobian of F and D = dSigma/d(delta) =
// 27 / (3 s^2 + p) (implicit differentiation of the physical root of the cubic, Sec. II,
// Eqs. 8-10). For mean-free lambda, J_p^T lambda = J^T lambda with J the 19-point stencil
//   (J e)_c = [sum_a A_a(c) S_a(e) - 6 e_c - sum_{a<b} W_ab(c) D_ab(e) / 2] / h^2,
//   A_a = 1 - Wbar_aa, W = (9 s Mbar - 27 Mbar^2) / (3 s^2 + p),
// so the transpose gathers each neighbour's coefficient times its lambda:
//   (J^T l)_c = [sum_a (A_a l)(c +- e_a) - 6 l_c - sum_{a<b} D_ab(W_ab l)(c) / 2] / h^2.
// It is solved by a linear multigrid (red-black Gauss-Seidel on J^T with the -6/h^2 diagonal,
// 8-son restriction, trilinear prolongation) whose coefficients are rebuilt on every level from
// the restricted theta_star and delta (no forward V-cycle state is stored). lambda is kept
// mean-free after every sweep: each level's array is stored with a uniform offset mu (the mean of
// the last sweep's output), which every read subtracts.
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"
#include "tuning.h"

namespace mr {

struct AdjLevel {
  double* lam[2] = {nullptr, nullptr};
  int cur = 0;
  double* rhs = nullptr;
  double* coef = nullptr;   // 6 fields: A_x, A_y, A_z, W_xy, W_xz, W_yz (each colour-split n^3)
  int tm = 0, tj = 0, ci = 0;   // half-sweep tile and chunk; tm == 0: the row kernel
  bool pfc = false;             // coefficient prefetch of the tiled half-sweep
};

struct AdjointState {
  std::vector<AdjLevel> lv;
  double* D = nullptr;      // dSigma/d(delta) on the finest mesh (colour-split)
  std::vector<void*> owned;
};

// ---- coefficient fields --------------------------------------------------------------------

__global__ void __launch_bounds__(256) adj_coef_kernel(const double* __restrict__ theta, const double* __restrict__ delta,
                                                       int n, double ih2, double* __restrict__ coef,
                                                       double* __restrict__ Dout) {
  const size_t cells = (size_t)n * n * n;
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int i = row / n, j = row - i * n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const unsigned e = split_idx(n, i, j, k);
    Nb18 t;
    gather18_split(theta, n, i, j, k, t);
    double S;
    const double sig = sigma_cell(t, 1.0 + delta[e], ih2, S);
    const double s = sig + 3.0;
    const double Sx = t.xm + t.xp, Sy = t.ym + t.yp, Sz = t.zm + t.zp;
    const double s3 = (Sx + Sy + Sz) * (1.0 / 3.0);
    const double mx = (Sx - s3) * ih2, my = (Sy - s3) * ih2, mz = (Sz - s3) * ih2;
    const double mxy = 0.25 * ((t.xpyp + t.xmym) - (t.xpym + t.xmyp)) * ih2;
    const double mxz = 0.25 * ((t.xpzp + t.xmzm) - (t.xpzm + t.xmzp)) * ih2;
    const double myz = 0.25 * ((t.ypzp + t.ymzm) - (t.ypzm + t.ymzp)) * ih2;
    const double xy2 = mxy * mxy, xz2 = mxz * mxz, yz2 = myz * myz;
    const double T2 = mx * mx + my * my + mz * mz + 2.0 * (xy2 + xz2 + yz2);
    const double den = 3.0 * s * s - 4.5 * T2;
    const double inv = 1.0 / den;
    const double s9 = 9.0 * s, q9 = 9.0 * T2;
    coef[0 * cells + e] = 1.0 - (s9 * mx - 27.0 * (mx * mx + xy2 + xz2) + q9) * inv;
    coef[1 * cells + e] = 1.0 - (s9 * my - 27.0 * (xy2 + my * my + yz2) + q9) * inv;
    coef[2 * cells + e] = 1.0 - (s9 * mz - 27.0 * (xz2 + yz2 + mz * mz) + q9) * inv;
    coef[3 * cells + e] = (s9 * mxy - 27.0 * (mx * mxy + mxy * my + mxz * myz)) * inv;
    coef[4 * cells + e] = (s9 * mxz - 27.0 * (mx * mxz + mxy * myz + mxz * mz)) * inv;
    coef[5 * cells + e] = (s9 * myz - 27.0 * (mxy * mxz + my * myz + myz * mz)) * inv;
    if (Dout) Dout[e] = 27.0 * inv;
  }
}

// Off-diagonal part of h^2 (J^T l)_c from neighbours' coefficients and (mean-adjusted) lambda.
// lam(i,j,k) is supplied by the caller (it knows which colour carries which offset).
template <class LamAt>
__device__ __forceinline__ double adj_offdiag(const double* __restrict__ coef, size_t cells, int n, int i, int j, int k,
                                              LamAt lam) {
  const int im = wrapi(i - 1, n), ip = wrapi(i + 1, n);
  const int jm = wrapi(j - 1, n), jp = wrapi(j + 1, n);
  const int km = wrapi(k - 1, n), kp = wrapi(k + 1, n);
  auto AL = [&](int f, int a, int b, int c) {
    const unsigned g = split_idx(n, a, b, c);
    return coef[f * cells + g] * lam(a, b, c, g);
  };
  double off = AL(0, im, j, k) + AL(0, ip, j, k) + AL(1, i, jm, k) + AL(1, i, jp, k) + AL(2, i, j, km) + AL(2, i, j, kp);
  const double dxy = (AL(3, ip, jp, k) + AL(3, im, jm, k)) - (AL(3, ip, jm, k) + AL(3, im, jp, k));
  const double dxz = (AL(4, ip, j, kp) + AL(4, im, j, km)) - (AL(4, ip, j, km) + AL(4, im, j, kp));
  const double dyz = (AL(5, i, jp, kp) + AL(5, i, jm, km)) - (AL(5, i, jp, km) + AL(5, i, jm, kp));
  return off - 0.5 * (dxy + dxz + dyz);
}

// One colour of a red-black Gauss-Seidel sweep on J^T l = rhs. Stored arrays carry the offset mu
// (mean of the previous sweep's output): the red pass subtracts it from both colours, the black
// pass from the old black values only (the new red values are read as written). Sums the new
// values (the next offset).
__global__ void __launch_bounds__(256) adj_half_sweep_kernel(const double* __restrict__ lam_in,
    const double* __restrict__ red_new, double* __restrict__ out, const double* __restrict__ rhs,
    const double* __restrict__ coef, int n, int colour, double h2, const double* mu_sum, double mu_scale,
    double* sum_out, const double* copy_from, double* copy_to, Reduce red) {
  const size_t cells = (size_t)n * n * n;
  const unsigned half = (unsigned)(cells / 2);
  const double mu = mu_sum ? (mu_sum[0] + mu_sum[1]) * mu_scale : 0.0;
  double acc = 0.0;
  const int nh = n >> 1;
  const int rows = n * n;
  const int rpb = (rows + gridDim.x - 1) / gridDim.x;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rpb;
  const int r1 = r0 + rpb < rows ? r0 + rpb : rows;
  auto lam = [&](int, int, int, unsigned g) -> double {
    if (red_new && g < half) return red_new[g];
    return lam_in[g] - mu;
  };
  for (int row = r0; row < r1; ++row) {
    const int i = row / n, j = row - i * n;
    const int q = (i + j + colour) & 1;
    for (int m = threadIdx.x; m < nh; m += blockDim.x) {
      const int k = 2 * m + q;
      const unsigned e = split_idx(n, i, j, k);
      const double off = adj_offdiag(coef, cells, n, i, j, k, lam);
      const double v = (off - h2 * rhs[e]) * (1.0 / 6.0);
      out[e] = v;
      acc += v;
    }
  }
  double vv[1] = {acc};
  const bool last = grid_sum<1>(vv, red.partials, red.counter, sum_out, gridDim.x, blockIdx.x);
  if (last && threadIdx.x == 0 && copy_to) *copy_to = *copy_from;
}

// ---- pipelined half-sweep (fine meshes) ----------------------------------------------------
// The same update as adj_half_sweep_kernel on a TJ x TM tile of (j, m) marching along i over a
// chunk of ci planes (ci % 4 == 0). lambda of both colours (mean offset already removed) sits in a
// 4-slot LDS plane ring filled two planes ahead, as in the forward pipelined half-sweep. The
// coefficients are read from global memory one step ahead into registers; they are used exactly
// once per cell, so staging them in LDS would buy nothing. The x-direction part of the transpose
// stencil splits by plane: a plane p contributes X(p) = (A_x l)(p) and
// E(p) = [(W_xy l)(j+1) - (W_xy l)(j-1)] + [(W_xz l)(k+1) - (W_xz l)(k-1)] to both cells that sit
// on top of and below it with opposite signs of E, so each is computed once and reused two planes
// later. Order of the sums differs from adj_offdiag (rounding only).
struct AdjSweepArgs {
  const double* lam_in;     // old lambda, both colours, stored with offset mu
  const double* red_new;    // black pass: the new red values (no offset); red pass: unused
  double* out;              // receives the new values of the swept colour
  const double* rhs;
  const double* coef;
  int n;
  double h2;
  const double* mu_sum;     // mu = (mu_sum[0] + mu_sum[1]) * mu_scale
  double mu_scale;
  double* sum_out;          // sum of the new values
  const double* copy_from;  // last block copies *copy_from to *copy_to (if copy_to)
  double* copy_to;
  const double* add_from;   // last block adds *add_from to *sum_out (if set)
  Reduce red;
};

// PFC: coefficients of step t + 1 are loaded at the end of step t (in flight across the barrier),
// else at the start of their own step (fewer registers, higher occupancy).
// RES: instead of the update, the residual r = rhs - (J^T l) of the colour's cells (both colours
// read from lam_in with the offset removed), its sum of squares into sum_out.
template <int TM, int TJ, int COL, bool PFC, bool RES = false>
__global__ void __launch_bounds__(TM * TJ) adj_half_sweep_pipe(AdjSweepArgs a, int tiles_m, int tiles_j, int ci) {
  constexpr int NT = TM * TJ;
  constexpr int RW = TM + 2, RH = TJ + 2;
  constexpr int SLOT = RH * RW;
  constexpr int NPC = (SLOT + NT - 1) / NT;   // loader elements per thread and colour
  constexpr int O = 1 - COL;
  __shared__ double lds[2 * 4 * SLOT];
  const int n = a.n, nh = n >> 1;
  const double h2 = a.h2, ih2 = 1.0 / a.h2;
  const int tid = threadIdx.x;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int m0 = (logical % tiles_m) * TM;
  const int j0 = ((logical / tiles_m) % tiles_j) * TJ;
  const int i0 = (logical / (tiles_m * tiles_j)) * ci;
  const size_t plane = (size_t)n * nh;
  const size_t half = plane * n;
  const double mu = a.mu_sum ? (a.mu_sum[0] + a.mu_sum[1]) * a.mu_scale : 0.0;
  // colour-0 values: the new red values in the black pass (no offset), else the old ones
  const double* __restrict__ src0 = COL == 1 && !RES ? a.red_new : a.lam_in;
  const double* __restrict__ src1 = a.lam_in + half;
  const double mu0 = COL == 1 && !RES ? 0.0 : mu;

  // loader: element e of a slot is halo-tile row e / RW, column e % RW (same for both colours);
  // byte offsets inside a plane, out-of-range elements clamped onto the last one
  unsigned gb[NPC];
  int le[NPC];
#pragma unroll
  for (int t = 0; t < NPC; ++t) {
    int e = tid + t * NT;
    e = e < SLOT ? e : SLOT - 1;
    const int r = e / RW;
    const int c = e - r * RW;
    gb[t] = ((unsigned)wrapi(j0 - 1 + r, n) * nh + (unsigned)wrapi(m0 - 1 + c, nh)) * 8u;
    le[t] = e;
  }
  // every global access goes through a buffer resource of one plane (uniform) and a per-lane
  // byte offset inside it
  const unsigned pbytes = (unsigned)plane * 8u;
  auto prs = [&](const double* arr, int p) { return plane_rsrc(arr + (size_t)p * plane, pbytes); };
  auto fetch = [&](int rel, double (&v)[2][NPC]) {
    const int p = wrapi(i0 - 1 + rel, n);
    const auto b0 = prs(src0, p), b1 = prs(src1, p);
#pragma unroll
    for (int t = 0; t < NPC; ++t) {
      v[0][t] = ld_rs(b0, gb[t]);
      v[1][t] = ld_rs(b1, gb[t]);
    }
  };
  auto store = [&](int slot, const double (&v)[2][NPC]) {
#pragma unroll
    for (int t = 0; t < NPC; ++t) {
      lds[le[t] + slot * SLOT] = v[0][t] - mu0;
      lds[le[t] + (4 + slot) * SLOT] = v[1][t] - mu;
    }
  };

  const int s = tid % TM, r = tid / TM;
  const int j = j0 + r, m = m0 + s;
  const unsigned rc = (unsigned)j * nh, rm = (unsigned)wrapi(j - 1, n) * nh, rp = (unsigned)wrapi(j + 1, n) * nh;
  const int q0 = (i0 + j + COL) & 1;   // z-parity of the own cell at even steps
  // byte offsets inside a plane: own cell, rows j -+ 1, and the k +- 1 columns at even (index 0)
  // and odd (index 1) steps
  const unsigned zp[2] = {(unsigned)wrapi(m + q0, nh), (unsigned)wrapi(m + (q0 ^ 1), nh)};
  const unsigned zm[2] = {(unsigned)wrapi(m + q0 - 1, nh), (unsigned)wrapi(m + (q0 ^ 1) - 1, nh)};
  const unsigned o_c = (rc + m) * 8u, o_ym = (rm + m) * 8u, o_yp = (rp + m) * 8u;
  unsigned o_zp[2], o_zm[2], o_pp[2], o_mm[2], o_pm[2], o_mp[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    o_zp[b] = (rc + zp[b]) * 8u;
    o_zm[b] = (rc + zm[b]) * 8u;
    o_pp[b] = (rp + zp[b]) * 8u;
    o_mm[b] = (rm + zm[b]) * 8u;
    o_pm[b] = (rp + zm[b]) * 8u;
    o_mp[b] = (rm + zp[b]) * 8u;
  }
  const int ob = (r + 1) * RW + (s + 1);
  const int oq0 = ob + q0, oq1 = ob + (q0 ^ 1);
  const size_t cells = half * 2;
  const double* __restrict__ cAx = a.coef + 0 * cells + O * half;
  const double* __restrict__ cAy = a.coef + 1 * cells + O * half;
  const double* __restrict__ cAz = a.coef + 2 * cells + O * half;
  const double* __restrict__ cWxy = a.coef + 3 * cells + COL * half;
  const double* __restrict__ cWxz = a.coef + 4 * cells + COL * half;
  const double* __restrict__ cWyz = a.coef + 5 * cells + COL * half;
  const double* __restrict__ rh = a.rhs + COL * half;
  double* __restrict__ out = a.out + COL * half;
  const int last_plane = n - 1;
  const double* __restrict__ lo_all = lds + O * 4 * SLOT;
  const double* __restrict__ lc_all = lds + COL * 4 * SLOT;

  // coefficients of one step: x-part on plane i+1, in-plane part on plane i
  struct Coef {
    double ax, wxyp, wxym, wxzp, wxzm;
    double aym, ayp, azm, azp, wpp, wmm, wpm, wmp;
  };
  auto load_x = [&](Coef& c, int p, int b) {
    const auto rx = prs(cAx, p), rxy = prs(cWxy, p), rxz = prs(cWxz, p);
    c.ax = ld_rs(rx, o_c);
    c.wxyp = ld_rs(rxy, o_yp);
    c.wxym = ld_rs(rxy, o_ym);
    c.wxzp = ld_rs(rxz, o_zp[b]);
    c.wxzm = ld_rs(rxz, o_zm[b]);
  };
  auto load_in = [&](Coef& c, int p, int b) {
    const auto ry = prs(cAy, p), rz = prs(cAz, p), ryz = prs(cWyz, p);
    c.aym = ld_rs(ry, o_ym);
    c.ayp = ld_rs(ry, o_yp);
    c.azm = ld_rs(rz, o_zm[b]);
    c.azp = ld_rs(rz, o_zp[b]);
    c.wpp = ld_rs(ryz, o_pp[b]);
    c.wmm = ld_rs(ryz, o_mm[b]);
    c.wpm = ld_rs(ryz, o_pm[b]);
    c.wmp = ld_rs(ryz, o_mp[b]);
  };
  auto wrapp = [&](int p) { return p >= n ? p - n : (p < 0 ? p + n : p); };
  // X and E of the plane held in LDS slot sl, for cells whose z-parity index is b
  auto xe = [&](const Coef& c, int sl, int b, double& X, double& E) {
    const int oq = b ? oq1 : oq0;
    const double* __restrict__ lo = lo_all + sl * SLOT;
    const double* __restrict__ lc = lc_all + sl * SLOT;
    X = c.ax * lo[ob];
    E = (c.wxyp * lc[ob + RW] - c.wxym * lc[ob - RW]) + (c.wxzp * lc[oq] - c.wxzm * lc[oq - 1]);
  };

  double V0[2][NPC], V1[2][NPC];
  double Rv[4];
  double Xr[2], Er[2];
  Coef cf;
  {
    double va[2][NPC], vb[2][NPC], vc[2][NPC];
    fetch(0, va);
    fetch(1, vb);
    fetch(2, vc);
    store(0, va);
    store(1, vb);
    store(2, vc);
  }
  fetch(3, V0);
  Rv[0] = ld_rs(prs(rh, i0), o_c);
  Rv[1] = ld_rs(prs(rh, min(i0 + 1, last_plane)), o_c);
  {
    Coef pa, pb;
    load_x(pa, wrapp(i0 - 1), 0);
    load_x(pb, i0, 1);
    if (PFC) {
      load_x(cf, wrapp(i0 + 1), 0);
      load_in(cf, i0, 0);
    }
    __syncthreads();
    xe(pa, 0, 0, Xr[0], Er[0]);
    xe(pb, 1, 1, Xr[1], Er[1]);
  }
  double acc = 0.0;

  // step t (K = t & 3): plane i = i0 + t sits in slot (K + 1) & 3, plane i + 1 in (K + 2) & 3
  auto step = [&](auto kc, int t, double (&vst)[2][NPC], double (&vft)[2][NPC]) {
    constexpr int K = decltype(kc)::value;
    constexpr int S0 = (K + 1) & 3, SP = (K + 2) & 3, SN = (K + 3) & 3;
    constexpr int B = K & 1;
    fetch(t + 4, vft);
    Rv[(K + 2) & 3] = ld_rs(prs(rh, min(i0 + t + 2, last_plane)), o_c);
    if (!PFC) {
      load_x(cf, wrapp(i0 + t + 1), B);
      load_in(cf, i0 + t, B);
    }
    double Xp, Ep;
    xe(cf, SP, B, Xp, Ep);
    const int oq = B ? oq1 : oq0;
    const double* __restrict__ lo = lo_all + S0 * SLOT;
    const double* __restrict__ lc = lc_all + S0 * SLOT;
    const double P = (cf.aym * lo[ob - RW] + cf.ayp * lo[ob + RW]) + (cf.azm * lo[oq - 1] + cf.azp * lo[oq]);
    const double dyz = (cf.wpp * lc[oq + RW] + cf.wmm * lc[oq - RW - 1]) - (cf.wpm * lc[oq + RW - 1] + cf.wmp * lc[oq - RW]);
    const double off = (Xr[B] + Xp) + P - 0.5 * ((Ep - Er[B]) + dyz);
    Xr[B] = Xp;
    Er[B] = Ep;
    if (RES) {
      const double v = Rv[K] - (off - 6.0 * lc[ob]) * ih2;
      st_rs(prs(out, i0 + t), o_c, v);
      acc += v * v;
    } else {
      const double v = (off - h2 * Rv[K]) * (1.0 / 6.0);
      st_rs(prs(out, i0 + t), o_c, v);
      acc += v;
    }
    if (PFC) {
      const int ip = i0 + t + 1;
      load_x(cf, wrapp(ip + 1), B ^ 1);
      load_in(cf, min(ip, last_plane), B ^ 1);
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

  double vv[1] = {acc};
  const bool last = grid_sum<1>(vv, a.red.partials, a.red.counter, a.sum_out, gridDim.x, blockIdx.x);
  if (last && tid == 0 && a.copy_to) *a.copy_to = *a.copy_from;
  if (last && tid == 0 && a.add_from) *a.sum_out += *a.add_from;
}

// res = rhs - J^T l on the fine mesh and rhs_c = R res; sums res^2 (the level's residual norm).
__global__ void __launch_bounds__(256) adj_resid_restrict_kernel(const double* __restrict__ lam_in,
    const double* __restrict__ rhs, const double* __restrict__ coef, int n, double ih2, const double* mu_sum,
    double mu_scale, double* __restrict__ rhs_c, Reduce red) {
  const size_t cells = (size_t)n * n * n;
  const double mu = mu_sum ? (mu_sum[0] + mu_sum[1]) * mu_scale : 0.0;
  const int m = n >> 1;
  double a2 = 0.0;
  const int rows = m * m;
  const int rpb = (rows + gridDim.x - 1) / gridDim.x;
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * rpb;
  const int r1 = r0 + rpb < rows ? r0 + rpb : rows;
  auto lam = [&](int, int, int, unsigned g) -> double { return lam_in[g] - mu; };
  for (int row = r0; row < r1; ++row) {
    const int I = row / m, J = row - I * m;
    for (int K = threadIdx.x; K < m; K += blockDim.x) {
      double s = 0.0;
#pragma unroll 1
      for (int q = 0; q < 8; ++q) {
        const int i = 2 * I + (q >> 2), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q & 1);
        const unsigned g = split_idx(n, i, j, k);
        const double off = adj_offdiag(coef, cells, n, i, j, k, lam);
        const double r = rhs[g] - (off - 6.0 * (lam_in[g] - mu)) * ih2;
        s += r;
        a2 += r * r;
      }
      rhs_c[split_idx(m, I, J, K)] = 0.125 * s;
    }
  }
  double vv[2] = {0.0, a2};
  grid_sum<2>(vv, red.partials, red.counter, red.result, gridDim.x, blockIdx.x);
}

// Coarsest level: nsweeps projected red-black sweeps in one block (lambda and rhs in LDS,
// coefficients from global memory). Writes the mean-free result and sets its offset to 0.
__global__ void __launch_bounds__(256) adj_coarsest_kernel(double* __restrict__ lam, const double* __restrict__ rhs,
    const double* __restrict__ coef, int n, int nsweeps, double h2, const double* mu_sum, double mu_scale,
    double* mu_out) {
  __shared__ double tl[kMaxCoarsest], tr[kMaxCoarsest], tn[kMaxCoarsest];
  __shared__ double red[16][1];
  __shared__ double mnew;
  const int n3 = n * n * n, tid = threadIdx.x;
  const size_t cells = (size_t)n3;
  const double mu0 = mu_sum ? (mu_sum[0] + mu_sum[1]) * mu_scale : 0.0;
  for (int x = tid; x < n3; x += blockDim.x) {
    const unsigned g = split_idx(n, x / (n * n), (x / n) % n, x % n);
    tl[x] = lam[g] - mu0;
    tr[x] = rhs[g];
  }
  __syncthreads();
  auto lamv = [&](int a, int b, int c, unsigned) -> double { return tl[(a * n + b) * n + c]; };
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int colour = 0; colour < 2; ++colour) {
      for (int x = tid; x < n3; x += blockDim.x) {
        const int i = x / (n * n), j = (x / n) % n, k = x % n;
        if (((i + j + k) & 1) != colour) continue;
        const double off = adj_offdiag(coef, cells, n, i, j, k, lamv);
        tn[x] = (off - h2 * tr[x]) * (1.0 / 6.0);
      }
      __syncthreads();
      for (int x = tid; x < n3; x += blockDim.x) {
        const int i = x / (n * n), j = (x / n) % n, k = x % n;
        if (((i + j + k) & 1) == colour) tl[x] = tn[x];
      }
      __syncthreads();
    }
    double acc = 0.0;
    for (int x = tid; x < n3; x += blockDim.x) acc += tl[x];
    double v[1] = {acc};
    block_sum<1>(v, red, tid, blockDim.x);
    if (tid == 0) mnew = v[0] / (double)n3;
    __syncthreads();
    for (int x = tid; x < n3; x += blockDim.x) tl[x] -= mnew;
    __syncthreads();
  }
  for (int x = tid; x < n3; x += blockDim.x) lam[split_idx(n, x / (n * n), (x / n) % n, x % n)] = tl[x];
  if (tid == 0 && mu_out) {
    mu_out[0] = 0.0;
    mu_out[1] = 0.0;
  }
}

// grad = D * (lambda - mu), natural order.
__global__ void __launch_bounds__(1024) adj_grad_kernel(const double* __restrict__ lam, const double* mu_sum,
                                                        double mu_scale, const double* __restrict__ D,
                                                        double* __restrict__ grad, int n) {
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int i = row / n, j = row - i * n;
  const int k = threadIdx.x;
  if (k >= n) return;
  const double mu = (mu_sum[0] + mu_sum[1]) * mu_scale;
  const unsigned g = split_idx(n, i, j, k);
  grad[((size_t)i * n + j) * n + k] = D[g] * (lam[g] - mu);
}

__global__ void __launch_bounds__(256) center_kernel(double* __restrict__ a, size_t cells, const double* sum, double scale) {
  const double m = (*sum) * scale;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x)
    a[e] -= m;
}

// ---- driver -------------------------------------------------------------------------------

static int rows_blocks_a(int n) { return n * n < 4096 ? n * n : 4096; }
static int row_threads_a(int n) { return n < 64 ? 64 : (n < 256 ? n : 256); }
static int lin_blocks_a(size_t cells) {
  size_t b = (cells + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// ---- half-sweep launch and tile choice ----------------------------------------------------

#define MR_AP_TILES(X) X(64, 4) X(64, 8) X(32, 8) X(16, 16) X(8, 16) X(8, 8) X(4, 8)

struct AdjCfg {
  int tm = 0, tj = 0, ci = 0;   // tm == 0: the row kernel
  bool pfc = false;
};

// One colour of a sweep (res = false), or of the residual r = rhs - J^T l (res = true: tiled
// configurations only, the offset removed from both colours of lam_in).
static hipError_t launch_adj_half(const AdjSweepArgs& a, int colour, const AdjCfg& c, hipStream_t s, bool res = false) {
  if (colour == 1 && !a.red_new && !res) return hipErrorInvalidValue;
  if (res && c.tm == 0) return hipErrorInvalidValue;
  if (c.tm == 0) {
    hipLaunchKernelGGL(adj_half_sweep_kernel, dim3(rows_blocks_a(a.n)), dim3(row_threads_a(a.n / 2)), 0, s, a.lam_in,
                       colour == 1 ? a.red_new : (const double*)nullptr, a.out, a.rhs, a.coef, a.n, colour, a.h2,
                       a.mu_sum, a.mu_scale, a.sum_out, a.copy_from, a.copy_to, a.red);
    return hipGetLastError();
  }
  const int nh = a.n / 2;
  if (c.tj > a.n || nh % c.tm != 0 || a.n % c.tj != 0 || c.ci % 4 != 0 || a.n % c.ci != 0) return hipErrorInvalidValue;
  const int tiles_m = nh / c.tm, tiles_j = a.n / c.tj;
  const long blocks = (long)tiles_m * tiles_j * (a.n / c.ci);
  if (blocks < 1 || blocks > kMaxReduceBlocks) return hipErrorInvalidValue;
#define MR_AP_GO(TM, TJ, COL, PFC, RES)                                                                     \
  hipLaunchKernelGGL((adj_half_sweep_pipe<TM, TJ, COL, PFC, RES>), dim3(blocks), dim3(TM * TJ), 0, s, a, tiles_m, \
                     tiles_j, c.ci)
#define MR_AP_LAUNCH(TM, TJ)                         \
  if (c.tm == TM && c.tj == TJ) {                    \
    if (res && colour == 0)                          \
      MR_AP_GO(TM, TJ, 0, true, true);               \
    else if (res)                                    \
      MR_AP_GO(TM, TJ, 1, true, true);               \
    else if (colour == 0 && c.pfc)                   \
      MR_AP_GO(TM, TJ, 0, true, false);              \
    else if (colour == 0)                            \
      MR_AP_GO(TM, TJ, 0, false, false);             \
    else if (c.pfc)                                  \
      MR_AP_GO(TM, TJ, 1, true, false);              \
    else                                             \
      MR_AP_GO(TM, TJ, 1, false, false);             \
    return hipGetLastError();                        \
  }
  MR_AP_TILES(MR_AP_LAUNCH)
#undef MR_AP_LAUNCH
#undef MR_AP_GO
  return hipErrorInvalidValue;
}

// The tiled schedule without timing: the first compiled tile that fits, chunks of 8 planes (4 on
// meshes that 8 does not divide), the coefficient prefetch on even levels (so one solve runs both
// load schedules). tm == 0 if none fits.
static AdjCfg fixed_tiled_cfg(int n, int level) {
  const int nh = n / 2;
  AdjCfg c;
  c.pfc = level % 2 == 0;
  auto take = [&](int tm, int tj) {
    if (c.tm != 0 || nh % tm != 0 || n % tj != 0 || tj > n) return;
    const int ci = n % 8 == 0 ? 8 : 4;
    if (n % ci != 0 || (long)(nh / tm) * (n / tj) * (n / ci) > kMaxReduceBlocks) return;
    c.tm = tm;
    c.tj = tj;
    c.ci = ci;
  };
#define MR_AP_TAKE(TM, TJ) take(TM, TJ);
  MR_AP_TILES(MR_AP_TAKE)
#undef MR_AP_TAKE
  return c;
}

static std::mutex g_adj_tune_mu;
static std::map<std::pair<int, int>, AdjCfg> g_adj_tuned;   // (device, n)

// Times both colours of a sweep for the row kernel and every compiled tile (of at least 128
// threads where one fits) with chunks of 8 to 256 planes, with and without the coefficient
// prefetch, on the level's own (zeroed) buffers, and keeps the fastest. Cached per (device, n).
static int tune_adj_sweep(const AdjSweepArgs& base, hipStream_t s, AdjCfg* out) {
  const int n = base.n, nh = n / 2;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorInvalidDevice, "adjoint tuner");
  {
    std::lock_guard<std::mutex> lk(g_adj_tune_mu);
    static int gen = -1;
    tuning_sync(gen, g_adj_tuned);
    auto it = g_adj_tuned.find({dev, n});
    if (it != g_adj_tuned.end()) {
      *out = it->second;
      return MR_OK;
    }
  }
  std::vector<AdjCfg> cand{AdjCfg{}};
  // tiles of at least 128 threads where one fits (smaller ones only on small meshes)
  bool big = false;
  auto fits = [&](int tm, int tj) { return nh % tm == 0 && n % tj == 0 && tj <= n; };
#define MR_AP_BIG(TM, TJ) big = big || (fits(TM, TJ) && TM * TJ >= 128);
  MR_AP_TILES(MR_AP_BIG)
#undef MR_AP_BIG
  auto add = [&](int tm, int tj) {
    if (!fits(tm, tj) || (big && tm * tj < 128)) return;
    const long tiles = (long)(nh / tm) * (n / tj);
    for (int ci = 8; ci <= 256 && ci <= n; ci *= 2) {
      if (n % ci != 0 || tiles * (n / ci) > kMaxReduceBlocks) continue;
      for (int pf = 0; pf < 2; ++pf) {
        AdjCfg c;
        c.tm = tm;
        c.tj = tj;
        c.ci = ci;
        c.pfc = pf != 0;
        cand.push_back(c);
      }
    }
  };
#define MR_AP_ADD(TM, TJ) add(TM, TJ);
  MR_AP_TILES(MR_AP_ADD)
#undef MR_AP_ADD
  const size_t cells = (size_t)n * n * n;
  const int reps = cells >= ((size_t)1 << 24) ? 2 : 4;
  auto run = [&](const AdjCfg& c) {
    hipError_t r = launch_adj_half(base, 0, c, s);
    return r == hipSuccess ? launch_adj_half(base, 1, c, s) : r;
  };
  auto code = [](const AdjCfg& c) { return std::vector<int>{c.tm, c.tj, c.ci, c.pfc ? 1 : 0}; };
  size_t bi = 0;
  bool recorded = false;
  {
    std::vector<int> rec;
    if (tuning_lookup("adj64.v1", dev, n, rec))
      for (size_t i = 0; i < cand.size() && !recorded; ++i)
        if (code(cand[i]) == rec) {
          bi = i;
          recorded = true;
        }
  }
  hipError_t e = recorded ? hipSuccess : pick_fastest(cand.size(), reps, s, [&](size_t i) { return run(cand[i]); }, &bi);
  const AdjCfg best_c = cand[bi];
  if (e != hipSuccess) return hip_fail(e, "adjoint tuner");
  {
    std::lock_guard<std::mutex> lk(g_adj_tune_mu);
    g_adj_tuned[{dev, n}] = best_c;
  }
  if (!recorded) tuning_record("adj64.v1", dev, n, code(best_c));
  *out = best_c;
  return MR_OK;
}

static int adjoint_alloc(Ctx* c) {
  if (c->adj) return MR_OK;
  AdjointState* a = new AdjointState();
  c->adj = a;
  a->lv.resize(c->nlev);
  auto get = [&](double** p, size_t count) -> int {
    hipError_t e = hipMalloc((void**)p, count * sizeof(double));
    if (e != hipSuccess) return fail(MR_ENOMEM, "adjoint buffers: %s", hipGetErrorString(e));
    a->owned.push_back(*p);
    return MR_OK;
  };
  int rc;
  for (int l = 0; l < c->nlev; ++l) {
    const size_t cells = c->lv[l].cells;
    AdjLevel& L = a->lv[l];
    if ((rc = get(&L.lam[0], cells)) != MR_OK || (rc = get(&L.lam[1], cells)) != MR_OK ||
        (rc = get(&L.rhs, cells)) != MR_OK || (rc = get(&L.coef, 6 * cells)) != MR_OK)
      return rc;
  }
  if ((rc = get(&a->D, c->lv[0].cells)) != MR_OK) return rc;
  // half-sweep schedule per level, timed on the level's zeroed buffers
  for (int l = 0; l + 1 < c->nlev; ++l) {
    AdjLevel& L = a->lv[l];
    const size_t cells = c->lv[l].cells;
    hipError_t e = hipMemsetAsync(L.lam[0], 0, cells * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L.lam[1], 0, cells * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L.rhs, 0, cells * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L.coef, 0, 6 * cells * sizeof(double), c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint tuner");
    AdjSweepArgs t{};
    t.lam_in = L.lam[0];
    t.red_new = L.lam[1];
    t.out = L.lam[1];
    t.rhs = L.rhs;
    t.coef = L.coef;
    t.n = c->lv[l].n;
    t.h2 = 1.0;
    t.sum_out = c->scal + kSlotAux;
    t.red = c->reducer(kSlotAux);
    AdjCfg cfg;
    if ((rc = tune_adj_sweep(t, c->stream, &cfg)) != MR_OK) return rc;
    L.tm = cfg.tm;
    L.tj = cfg.tj;
    L.ci = cfg.ci;
    L.pfc = cfg.pfc;
  }
  return MR_OK;
}

void Ctx::release_adjoint() {
  if (!adj) return;
  for (void* p : adj->owned) (void)hipFree(p);
  delete adj;
  adj = nullptr;
}

// The level's half-sweep schedule: the timed choice, or the one a flag forces.
static AdjCfg adj_level_cfg(const AdjLevel& A, int n, int l, int flags) {
  AdjCfg cfg;
  if (flags & MR_FLAG_ADJ_TILED) {
    cfg = fixed_tiled_cfg(n, l);
  } else if (!(flags & MR_FLAG_ADJ_ROWS)) {
    cfg.tm = A.tm;
    cfg.tj = A.tj;
    cfg.ci = A.ci;
    cfg.pfc = A.pfc;
  }
  return cfg;
}

int Ctx::adj_sweep(int l) {
  AdjLevel& A = adj->lv[l];
  Level& F = lv[l];
  double* ms = linsum(l);
  const double scale = 1.0 / (double)F.cells;
  const AdjCfg cfg = adj_level_cfg(adj->lv[l], lv[l].n, l, opts.flags);
  AdjSweepArgs a{};
  a.lam_in = A.lam[A.cur];
  a.red_new = A.lam[A.cur ^ 1];
  a.out = A.lam[A.cur ^ 1];
  a.rhs = A.rhs;
  a.coef = A.coef;
  a.n = F.n;
  a.h2 = F.h * F.h;
  a.mu_sum = ms;
  a.mu_scale = scale;
  a.red = reducer(kSlotAux);
  a.sum_out = ms + 2;   // red: its sum parks in the third slot
  hipError_t e = launch_adj_half(a, 0, cfg, stream);
  a.sum_out = ms + 1;   // black: then the red sum moves to the first slot
  a.copy_from = ms + 2;
  a.copy_to = ms + 0;
  if (e == hipSuccess) e = launch_adj_half(a, 1, cfg, stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint sweep");
  A.cur ^= 1;
  return MR_OK;
}

int Ctx::adj_vcycle(int l, double* norm2) {
  AdjLevel& A = adj->lv[l];
  Level& F = lv[l];
  const double scale = 1.0 / (double)F.cells;
  hipError_t e;
  if (l == nlev - 1) {
    hipLaunchKernelGGL(adj_coarsest_kernel, dim3(1), dim3(256), 0, stream, A.lam[A.cur], A.rhs, A.coef, F.n, opts.ncoarse,
                       F.h * F.h, linsum(l), scale, linsum(l));
    e = hipGetLastError();
    return e == hipSuccess ? MR_OK : hip_fail(e, "adjoint coarsest");
  }
  int rc;
  for (int s = 0; s < opts.npre; ++s)
    if ((rc = adj_sweep(l)) != MR_OK) return rc;
  AdjLevel& Ac = adj->lv[l + 1];
  Level& Fc = lv[l + 1];
  const int m = F.n / 2;
  double* nrm = norm2 ? norm2 : scal + kSlotAux + 4;
  const AdjCfg cfg = adj_level_cfg(adj->lv[l], lv[l].n, l, opts.flags);
  if (cfg.tm != 0) {
    // tiled: r of each colour into the free lambda buffer (sum of squares red -> aux slot, black
    // plus red -> nrm[1]), then its 8-son average
    AdjSweepArgs a{};
    a.lam_in = A.lam[A.cur];
    a.out = A.lam[A.cur ^ 1];
    a.rhs = A.rhs;
    a.coef = A.coef;
    a.n = F.n;
    a.h2 = F.h * F.h;
    a.mu_sum = linsum(l);
    a.mu_scale = scale;
    a.red = reducer(kSlotAux);
    a.sum_out = scal + kSlotAux + 10;
    e = launch_adj_half(a, 0, cfg, stream, true);
    a.sum_out = nrm + 1;
    a.add_from = scal + kSlotAux + 10;
    if (e == hipSuccess) e = launch_adj_half(a, 1, cfg, stream, true);
    if (e == hipSuccess) e = launch_restrict(A.lam[A.cur ^ 1], Ac.rhs, F.n, stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint residual");
  } else {
    hipLaunchKernelGGL(adj_resid_restrict_kernel, dim3(rows_blocks_a(m)), dim3(row_threads_a(m)), 0, stream,
                       A.lam[A.cur], A.rhs, A.coef, F.n, 1.0 / (F.h * F.h), linsum(l), scale, Ac.rhs,
                       Reduce{partials, counter, nrm});
  }
  Ac.cur = 0;
  if ((e = hipMemsetAsync(Ac.lam[0], 0, Fc.cells * sizeof(double), stream)) != hipSuccess) return hip_fail(e, "zero");
  if ((e = hipMemsetAsync(linsum(l + 1), 0, 2 * sizeof(double), stream)) != hipSuccess) return hip_fail(e, "zero");
  if (norm2) {
    // convergence test of the finest level before the coarse correction
    double r[2];
    if ((rc = read_scalars((int)(norm2 - scal), 2, r)) != MR_OK) return rc;
    adj_last_norm = std::sqrt(r[1] > 0.0 ? r[1] : 0.0);
    if (adj_last_norm <= adj_stop) return MR_OK;
  }
  if ((rc = adj_vcycle(l + 1, nullptr)) != MR_OK) return rc;
  // l += P(lc - mu_c)
  if ((e = launch_prolong_add(Ac.lam[Ac.cur], linsum(l + 1), 1.0 / (double)Fc.cells, A.lam[A.cur], F.n, stream)) !=
      hipSuccess)
    return hip_fail(e, "adjoint prolongation");
  for (int s = 0; s < opts.npost; ++s)
    if ((rc = adj_sweep(l)) != MR_OK) return rc;
  return MR_OK;
}

int Ctx::adjoint_solve(const double* delta, const double* theta_star, const double* g, double* grad, mr_info* info,
                       int aa_depth) {
  auto t0 = std::chrono::steady_clock::now();
  if (nlev == 1) return fail(MR_EINVAL, "adjoint needs at least two levels (n >= 8)");
  int rc = adjoint_alloc(this);
  if (rc != MR_OK) return rc;
  if (aa_depth > 0 && (rc = aa_reserve(aa_depth)) != MR_OK) return rc;
  AAState aa(aa_depth, aa_depth + 1);
  if ((rc = prepare(delta)) != MR_OK) return rc;
  Level& L0 = lv[0];
  AdjLevel& A0 = adj->lv[0];
  const double N3 = (double)L0.cells;
  // theta_star hierarchy (in the forward buffers) and per-level coefficients
  hipError_t e = launch_to_split(theta_star, L0.th[0], L0.n, stream);
  for (int l = 1; l < nlev && e == hipSuccess; ++l) e = launch_restrict(lv[l - 1].th[0], lv[l].th[0], lv[l - 1].n, stream);
  for (int l = 0; l < nlev && e == hipSuccess; ++l) {
    hipLaunchKernelGGL(adj_coef_kernel, dim3((unsigned)lv[l].n * lv[l].n), dim3(lv[l].n < 256 ? lv[l].n : 256), 0, stream,
                       lv[l].th[0], lv[l].delta, lv[l].n, 1.0 / (lv[l].h * lv[l].h), adj->lv[l].coef,
                       l == 0 ? adj->D : (double*)nullptr);
    e = hipGetLastError();
  }
  // rhs = g - <g>, lambda = 0
  if (e == hipSuccess) e = launch_to_split(g, A0.rhs, L0.n, stream);
  if (e == hipSuccess) e = launch_sum(A0.rhs, L0.cells, reducer(kSlotGauge), stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(center_kernel, dim3(lin_blocks_a(L0.cells)), dim3(256), 0, stream, A0.rhs, L0.cells,
                       (const double*)(scal + kSlotGauge), 1.0 / N3);
    e = hipGetLastError();
  }
  A0.cur = 0;
  if (e == hipSuccess) e = hipMemsetAsync(A0.lam[0], 0, L0.cells * sizeof(double), stream);
  if (e == hipSuccess) e = hipMemsetAsync(linsum(0), 0, 3 * sizeof(double), stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint setup");
  // ||rhs||: the residual pass at lambda = 0
  hipLaunchKernelGGL(adj_resid_restrict_kernel, dim3(rows_blocks_a(L0.n / 2)), dim3(row_threads_a(L0.n / 2)), 0, stream,
                     A0.lam[0], A0.rhs, A0.coef, L0.n, 1.0, linsum(0), 1.0 / N3, adj->lv[1].rhs,
                     Reduce{partials, counter, scal + kSlotAux + 6});
  double r[2];
  if ((rc = read_scalars(kSlotAux + 6, 2, r)) != MR_OK) return rc;
  double r0 = std::sqrt(r[1] > 0.0 ? r[1] : 0.0);
  mr_info loc{};
  loc.r0_norm = r0;
  loc.history[0] = 1.0;
  if (r0 == 0.0) r0 = 1.0;
  adj_stop = opts.tol * r0;
  int cyc = 0, status = MR_OK;
  double rel = (loc.r0_norm == 0.0) ? 0.0 : 1.0;
  while (rel > opts.tol && cyc < opts.max_cycles) {
    if (aa_depth > 0 && aa.steps == 0 && (e = aa_save(*this, A0.lam[A0.cur])) != hipSuccess)
      return hip_fail(e, "Anderson save");
    if ((rc = adj_vcycle(0, scal + kSlotAux + 6)) != MR_OK) return rc;
    ++cyc;
    rel = adj_last_norm / r0;
    if (cyc < 128) loc.history[cyc] = rel;
    if (!std::isfinite(rel)) {
      status = fail(MR_EDIVERGED, "adjoint diverged at cycle %d", cyc);
      break;
    }
    // Anderson mixing of lambda between cycles (not after the last one, whose running sums the
    // gradient uses); the mixed lambda stays mean-free up to the lag of those sums
    if (aa_depth > 0 && rel > opts.tol && cyc < opts.max_cycles && (rc = aa_step(aa, A0.lam[A0.cur])) != MR_OK)
      return rc;
  }
  if (status == MR_OK && rel > opts.tol) {
    status = MR_NOT_CONVERGED;
    fail(MR_NOT_CONVERGED, "adjoint not converged after %d cycles (rel residual %g)", cyc, rel);
  }
  hipLaunchKernelGGL(adj_grad_kernel, dim3((unsigned)L0.n * L0.n), dim3(L0.n), 0, stream, A0.lam[A0.cur],
                     (const double*)linsum(0), 1.0 / N3, adj->D, grad, L0.n);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint gradient");
  loc.status = status;
  loc.cycles = cyc;
  loc.rel_residual = rel;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return status;
}

}  // namespace mr

extern "C" int mr_adjoint_solve(mr_ctx* h, const double* delta, const double* theta_star, const double* g,
                                double* grad_delta, mr_info* info) {
  if (!h || !delta || !theta_star || !g || !grad_delta) return mr::fail(MR_EINVAL, "mr_adjoint_solve: null argument");
  return reinterpret_cast<mr::Ctx*>(h)->adjoint_solve(delta, theta_star, g, grad_delta, info);
}

extern "C" int mr_adjoint_solve_anderson(mr_ctx* h, const double* delta, const double* theta_star, const double* g,
                                         double* grad_delta, int depth, mr_info* info) {
  if (!h || !delta || !theta_star || !g || !grad_delta)
    return mr::fail(MR_EINVAL, "mr_adjoint_solve_anderson: null argument");
  if (depth < 1 || depth > mr::kAAMaxDepth)
    return mr::fail(MR_EINVAL, "mr_adjoint_solve_anderson: depth %d not in 1..%d", depth, mr::kAAMaxDepth);
  return reinterpret_cast<mr::Ctx*>(h)->adjoint_solve(delta, theta_star, g, grad_delta, info, depth);
}
