// Red-black Newton-Gauss-Seidel relaxation (Sec. II.A.2, Eq. 17) of the reconstruction
// equation on one periodic mesh, FP64.
//
// One launch performs a whole sweep -- the red half-sweep followed by the black half-sweep --
// in a single pass over HBM (read theta, delta [, f], write theta: 24 B per cell update on the
// finest mesh, 32 B with the FAS right-hand side f on coarse meshes). Within a colour every cell
// is updated from the same snapshot: red from theta_in, black from the new red values and
// theta_in's black values; results go to theta_out (never in place), so the outcome does not
// depend on the order of cells or blocks.
//
// Work decomposition: a block owns a TJ x TK tile of (j, k) and marches along i through a chunk
// of planes. Planes of theta_in (tile plus a 2-cell periodic ring) stream through a 4-slot LDS
// ring; the red update of plane i+1 (tile plus a 1-cell ring, the ring computed redundantly)
// goes to a 3-slot LDS ring; the black update of plane i then reads its six red face neighbours
// from LDS. Each thread owns a pair of cells along k (one red, one black), so every lane does
// useful work in both half-sweeps and stores are 16-byte (double2) and coalesced.
#include "mr_device.h"
#include "mr_kernels.h"

namespace mr {

template <int TK>
__global__ void __launch_bounds__(1024) sweep_tile_kernel(SweepArgs a) {
  extern __shared__ double lds[];
  constexpr int OW = TK + 4;       // old-plane row width (2-cell ring each side)
  constexpr int RW = TK + 2;       // red-plane row width (1-cell ring each side)
  constexpr int PX = TK / 2;       // threads along k (one cell pair each)
  const int TJ = a.tj;
  const int OH = TJ + 4, RH = TJ + 2;
  const int n = a.n;
  const size_t N = (size_t)n;
  double* old = lds;                          // [4][OH][OW]
  double* rnew = lds + 4 * OH * OW;           // [3][RH][RW]

  const int nthreads = PX * TJ;
  const int tid = threadIdx.x;
  const int tx = tid % PX, ty = tid / PX;

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tk_i = logical % a.tiles_k;
  const int tj_i = (logical / a.tiles_k) % a.tiles_j;
  const int chunk = logical / (a.tiles_k * a.tiles_j);
  const int j0 = tj_i * TJ, k0 = tk_i * TK;
  const int i0 = chunk * a.ci;
  const int i1 = i0 + a.ci;

  const double C = (a.c_sum ? (*a.c_sum) * a.c_scale : 0.0) + a.c_add;
  const double h2 = a.h2, ih2 = a.ih2;
  const double* __restrict__ th = a.th_in;
  const double* __restrict__ dl = a.delta;
  const double* __restrict__ ff = a.f;

  auto OLD = [&](int p, int r, int c) -> double& { return old[((p & 3) * OH + r) * OW + c]; };
  auto RN = [&](int p, int r, int c) -> double& { return rnew[(((p % 3 + 3) % 3) * RH + r) * RW + c]; };

  // Load plane p (periodic) of theta_in, tile + 2-ring, into its old slot.
  auto load_plane = [&](int p) {
    const int pi = wrapi(p, n);
    const size_t base = (size_t)pi * N * N;
    for (int e = tid; e < OH * OW; e += nthreads) {
      const int r = e / OW, c = e - r * OW;
      const int gj = wrapi(j0 - 2 + r, n), gk = wrapi(k0 - 2 + c, n);
      OLD(p, r, c) = th[base + (size_t)gj * N + gk];
    }
  };

  // Red update at ring-1 coordinates (r, c) of plane q; returns Sigma + f for accounting.
  auto red_at = [&](int q, int r, int c, double opd, double fc) -> double {
    const int R = r + 1, Cc = c + 1;  // old-slot coordinates
    Nb18 t;
    t.xm = OLD(q - 1, R, Cc); t.xp = OLD(q + 1, R, Cc);
    t.ym = OLD(q, R - 1, Cc); t.yp = OLD(q, R + 1, Cc);
    t.zm = OLD(q, R, Cc - 1); t.zp = OLD(q, R, Cc + 1);
    t.xpyp = OLD(q + 1, R + 1, Cc); t.xmym = OLD(q - 1, R - 1, Cc);
    t.xpym = OLD(q + 1, R - 1, Cc); t.xmyp = OLD(q - 1, R + 1, Cc);
    t.xpzp = OLD(q + 1, R, Cc + 1); t.xmzm = OLD(q - 1, R, Cc - 1);
    t.xpzm = OLD(q + 1, R, Cc - 1); t.xmzp = OLD(q - 1, R, Cc + 1);
    t.ypzp = OLD(q, R + 1, Cc + 1); t.ymzm = OLD(q, R - 1, Cc - 1);
    t.ypzm = OLD(q, R + 1, Cc - 1); t.ymzp = OLD(q, R - 1, Cc + 1);
    double S;
    const double sig = sigma_cell(t, 1.0 + opd, ih2, S);
    RN(q, r, c) = (S - h2 * (sig + fc - C)) * (1.0 / 6.0);
    return sig + fc;
  };

  // Ring red cells of plane q: rows r = 0 and r = TJ+1 (all columns), columns c = 0 and
  // c = TK+1 (rows 1..TJ). A ring cell (r, c) is red iff (q + j0 + r + c) is even.
  const int nring = (TK + 2) + TJ;
  auto ring_red = [&](int q) {
    for (int e = tid; e < nring; e += nthreads) {
      int r, c;
      if (e < PX + 1) { r = 0; c = 2 * e + ((q + j0) & 1); }
      else if (e < 2 * (PX + 1)) { r = TJ + 1; c = 2 * (e - PX - 1) + ((q + j0 + TJ + 1) & 1); }
      else if (e < 2 * (PX + 1) + TJ / 2) { c = 0; r = 1 + 2 * (e - 2 * (PX + 1)) + ((q + j0 + 1) & 1); }
      else { c = TK + 1; r = 1 + 2 * (e - 2 * (PX + 1) - TJ / 2) + ((q + j0) & 1); }
      const int gq = wrapi(q, n);
      const size_t g = ((size_t)gq * N + (size_t)wrapi(j0 - 1 + r, n)) * N + (size_t)wrapi(k0 - 1 + c, n);
      red_at(q, r, c, dl[g], ff ? ff[g] : 0.0);
    }
  };

  // Interior red cell of this thread at plane q; delta/f of the black partner are returned for
  // the black update of the same plane one step later.
  auto interior_red = [&](int q, double& d_black, double& f_black) -> double {
    const int gq = wrapi(q, n);
    const size_t g = ((size_t)gq * N + (size_t)(j0 + ty)) * N + (size_t)(k0 + 2 * tx);
    const double2 d2 = *reinterpret_cast<const double2*>(dl + g);
    double2 f2 = make_double2(0.0, 0.0);
    if (ff) f2 = *reinterpret_cast<const double2*>(ff + g);
    const int ro = (q + j0 + ty) & 1;  // offset of the red cell within the pair
    d_black = ro ? d2.x : d2.y;
    f_black = ro ? f2.x : f2.y;
    return red_at(q, ty + 1, 2 * tx + 1 + ro, ro ? d2.y : d2.x, ro ? f2.y : f2.x);
  };

  double acc = 0.0;
  double db_next = 0.0, fb_next = 0.0, dummy_d, dummy_f;

  // Prologue: planes i0-2 .. i0+1 and the red planes i0-1, i0.
  load_plane(i0 - 2);
  load_plane(i0 - 1);
  load_plane(i0);
  load_plane(i0 + 1);
  __syncthreads();
  interior_red(i0 - 1, dummy_d, dummy_f);
  ring_red(i0 - 1);
  acc += interior_red(i0, db_next, fb_next);
  ring_red(i0);

  for (int i = i0; i < i1; ++i) {
    __syncthreads();
    load_plane(i + 2);
    __syncthreads();
    double db = db_next, fb = fb_next;
    {
      const double v = interior_red(i + 1, db_next, fb_next);
      if (i + 1 < i1) acc += v;
    }
    ring_red(i + 1);
    __syncthreads();
    // Black update of this thread's pair at plane i.
    const int ro = (i + j0 + ty) & 1;
    const int bo = 1 - ro;
    const int R = ty + 1, Cr = 2 * tx + 1 + bo;  // red-ring coordinates of the black cell
    const int RO = ty + 2, CO = 2 * tx + 2 + bo; // old-slot coordinates
    Nb18 t;
    t.xm = RN(i - 1, R, Cr); t.xp = RN(i + 1, R, Cr);
    t.ym = RN(i, R - 1, Cr); t.yp = RN(i, R + 1, Cr);
    t.zm = RN(i, R, Cr - 1); t.zp = RN(i, R, Cr + 1);
    t.xpyp = OLD(i + 1, RO + 1, CO); t.xmym = OLD(i - 1, RO - 1, CO);
    t.xpym = OLD(i + 1, RO - 1, CO); t.xmyp = OLD(i - 1, RO + 1, CO);
    t.xpzp = OLD(i + 1, RO, CO + 1); t.xmzm = OLD(i - 1, RO, CO - 1);
    t.xpzm = OLD(i + 1, RO, CO - 1); t.xmzp = OLD(i - 1, RO, CO + 1);
    t.ypzp = OLD(i, RO + 1, CO + 1); t.ymzm = OLD(i, RO - 1, CO - 1);
    t.ypzm = OLD(i, RO + 1, CO - 1); t.ymzp = OLD(i, RO - 1, CO + 1);
    double S;
    const double sig = sigma_cell(t, 1.0 + db, ih2, S);
    const double vb = (S - h2 * (sig + fb - C)) * (1.0 / 6.0);
    acc += sig + fb;
    const double vr = RN(i, R, 2 * tx + 1 + ro);
    const size_t g = ((size_t)i * N + (size_t)(j0 + ty)) * N + (size_t)(k0 + 2 * tx);
    *reinterpret_cast<double2*>(a.th_out + g) = ro ? make_double2(vb, vr) : make_double2(vr, vb);
  }

  double v[1] = {acc};
  grid_sum<1>(v, a.partials, a.counter, a.sum_out, gridDim.x, blockIdx.x);
}

// Coarsest mesh (at most 12^3 cells): nsweeps red-black sweeps by one block with the whole
// mesh in LDS. Same update and snapshot semantics as the tiled sweep; the uniform shift is
// lagged by one sweep and refreshed in-block after every sweep.
__global__ void __launch_bounds__(256) coarsest_kernel(CoarsestArgs a) {
  __shared__ double th[kMaxCoarsest], dd[kMaxCoarsest], fv[kMaxCoarsest], nv[kMaxCoarsest];
  __shared__ double red[16][1];
  __shared__ double cnew;
  const int n = a.n, n3 = n * n * n;
  const int tid = threadIdx.x;
  for (int e = tid; e < n3; e += blockDim.x) {
    th[e] = a.theta[e];
    dd[e] = 1.0 + a.delta[e];
    fv[e] = a.f ? a.f[e] : 0.0;
  }
  double C = (a.c_sum ? (*a.c_sum) * a.c_scale : 0.0) + a.c_add;
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
  for (int e = tid; e < n3; e += blockDim.x) a.theta[e] = th[e];
  if (tid == 0 && a.c_sum_out) *a.c_sum_out = C * (double)n3;
}

// ---- launchers ----------------------------------------------------------------------------

size_t sweep_lds_bytes(int tj, int tk) {
  return sizeof(double) * (4 * (size_t)(tj + 4) * (tk + 4) + 3 * (size_t)(tj + 2) * (tk + 2));
}

hipError_t launch_sweep(const SweepArgs& a0, int tk, hipStream_t s) {
  SweepArgs a = a0;
  const int threads = (tk / 2) * a.tj;
  const size_t lds = sweep_lds_bytes(a.tj, tk);
  const long blocks_l = (long)a.tiles_j * a.tiles_k * (a.n / a.ci);
  if (blocks_l < 1 || blocks_l > kMaxReduceBlocks || a.tj * a.tiles_j != a.n || tk * a.tiles_k != a.n ||
      a.n % a.ci != 0 || threads > 1024 || threads < 1)
    return hipErrorInvalidValue;
  const int blocks = (int)blocks_l;
  switch (tk) {
    case 4: hipLaunchKernelGGL(sweep_tile_kernel<4>, dim3(blocks), dim3(threads), lds, s, a); break;
    case 8: hipLaunchKernelGGL(sweep_tile_kernel<8>, dim3(blocks), dim3(threads), lds, s, a); break;
    case 16: hipLaunchKernelGGL(sweep_tile_kernel<16>, dim3(blocks), dim3(threads), lds, s, a); break;
    case 32: hipLaunchKernelGGL(sweep_tile_kernel<32>, dim3(blocks), dim3(threads), lds, s, a); break;
    case 64: hipLaunchKernelGGL(sweep_tile_kernel<64>, dim3(blocks), dim3(threads), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_coarsest(const CoarsestArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(coarsest_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mr
