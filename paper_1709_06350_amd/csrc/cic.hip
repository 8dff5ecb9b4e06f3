// Density assignment (the paper's footnote in Sec. I allows NGP, CIC or TSC): each particle
// spreads its mass over the 1, 8 or 27 mesh points around it with weights prod_d w_d, mesh points at
// integer coordinates, periodic wrap; then delta = rho / <rho> - 1 with <rho> = np * mass / n^3.
// Per axis, with b = floor(x) and f = x - b: NGP puts weight 1 on the nearest point (b, or b + 1
// when f >= 1/2); CIC puts 1 - f on b and f on b + 1; TSC, with i the NGP point and d = x - i,
// puts (1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2 on i - 1, i, i + 1 (the quadratic B-spline).
//
// Accumulation is in unsigned 64-bit fixed point (2^40 units per particle mass): every weight is
// rounded once, the integer sums are exact and independent of the order in which atomics land,
// so the result is bitwise reproducible. Particles are processed in their input order by
// consecutive threads; for lattice-ordered catalogues (as produced by displacing a lattice)
// neighbouring lanes hit neighbouring cells, which keeps the L2 atomics local.
#include <algorithm>
#include <cmath>

#include "mr.h"
#include "mr_ctx.h"
#include "mr_device.h"
#include "mr_kernels.h"

namespace mr {

constexpr double kFixScale = 1099511627776.0;  // 2^40

__device__ __forceinline__ void wrap_coord(double x, int n, int& i0, int& i1, double& f) {
  const double dn = (double)n;
  double xw = x - dn * floor(x / dn);
  if (xw >= dn) xw -= dn;
  if (xw < 0.0) xw = 0.0;
  const double fl = floor(xw);
  i0 = (int)fl;
  if (i0 >= n) i0 = n - 1;
  f = xw - fl;
  i1 = i0 + 1 == n ? 0 : i0 + 1;
}

// Per-axis points and weights of one coordinate for a scheme of S points (1 NGP, 2 CIC, 3 TSC).
template <int S>
__device__ __forceinline__ void axis_assign(double x, int n, int (&idx)[S], double (&w)[S]) {
  int i0, i1;
  double f;
  wrap_coord(x, n, i0, i1, f);  // i0 = floor of the wrapped coordinate, f its fraction (exact)
  if constexpr (S == 2) {
    idx[0] = i0;
    idx[1] = i1;
    w[0] = 1.0 - f;
    w[1] = f;
  } else {
    const bool up = f >= 0.5;
    const int c = up ? i1 : i0;  // nearest point, a tie goes up
    if constexpr (S == 1) {
      idx[0] = c;
      w[0] = 1.0;
    } else {
      const double d = up ? f - 1.0 : f;  // x - c, exact
      idx[0] = c == 0 ? n - 1 : c - 1;
      idx[1] = c;
      idx[2] = c == n - 1 ? 0 : c + 1;
      const double lo = 0.5 - d, hi = 0.5 + d;
      w[0] = 0.5 * (lo * lo);
      w[1] = 0.75 - d * d;
      w[2] = 0.5 * (hi * hi);
    }
  }
}

// A particle with a non-finite coordinate deposits nothing and adds 1 to *bad_count (relaxed
// atomic: an exact integer count that needs no grid-wide reduction).
template <int S>
__global__ void __launch_bounds__(256) deposit_scatter_kernel(const double* __restrict__ pos, long long np, int n,
                                                              unsigned long long* __restrict__ grid,
                                                              double* __restrict__ bad_count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < np; p += stride) {
    const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
    if (!__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(z)) {
      __hip_atomic_fetch_add(bad_count, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    int ix[S], iy[S], iz[S];
    double wx[S], wy[S], wz[S];
    axis_assign<S>(x, n, ix, wx);
    axis_assign<S>(y, n, iy, wy);
    axis_assign<S>(z, n, iz, wz);
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) {
        const size_t row = ((size_t)ix[a] * n + iy[b]) * n;
#pragma unroll
        for (int d = 0; d < S; ++d) {
          const double w = wx[a] * wy[b] * wz[d];
          const unsigned long long q = (unsigned long long)__double2ull_rn(w * kFixScale);
          if (q) atomicAdd(&grid[row + iz[d]], q);
        }
      }
  }
}

// The same deposit with each wave's contributions binned in LDS first. A wave takes 64 consecutive
// particles, finds the bounding box of the mesh points they reach (wrapped base indices, so a wave
// straddling the periodic seam gets a wide box) and, when the box holds at most CAP points,
// accumulates into a private LDS box with LDS atomics and then adds every non-zero box point to the
// grid with one global atomic; otherwise it adds to the grid directly. For lattice-ordered
// catalogues consecutive particles are neighbours, so a box point collects several contributions
// and the global atomics (performed beyond the L2, the bound of the plain scatter) drop by that
// factor. The integer sums per cell are the plain scatter's, so the result is bitwise identical.
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// lattice > 0: the catalogue holds lattice^3 particles in lattice order (k fastest) and lattice is a
// multiple of 8; a wave then takes a block of 2 (i) x 4 (j) x 8 (k) particles of the lattice, whose
// assignment points overlap along all three axes, instead of 64 consecutive particles of one row.
// Either way every particle is taken exactly once. (A 4 x 4 x 4 cube needs fewer global adds but
// timed slower, probably from more lanes meeting on the same LDS box entries.)
template <int S, int CAP>
__global__ void __launch_bounds__(256) deposit_scatter_binned_kernel(const double* __restrict__ pos, long long np, int n,
                                                                     unsigned long long* __restrict__ grid,
                                                                     double* __restrict__ bad_count, int lattice) {
  __shared__ unsigned long long boxes[4][CAP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long* box = boxes[w];
  const long long nwaves = (long long)gridDim.x * 4;
  const long long kb_n = lattice / 8, jb_n = lattice / 4;
  for (long long seg = (long long)blockIdx.x * 4 + w; seg * 64 < np; seg += nwaves) {
    long long p = seg * 64 + lane;
    if (lattice > 0) {
      const long long kb = seg % kb_n, jb = (seg / kb_n) % jb_n, ib = seg / (kb_n * jb_n);
      p = ((ib * 2 + (lane >> 5)) * lattice + jb * 4 + ((lane >> 3) & 3)) * lattice + kb * 8 + (lane & 7);
    }
    bool valid = p < np;
    double x = 0.0, y = 0.0, z = 0.0;
    if (valid) {
      x = pos[3 * p];
      y = pos[3 * p + 1];
      z = pos[3 * p + 2];
      if (!__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(z)) {
        __hip_atomic_fetch_add(bad_count, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        valid = false;
      }
    }
    int ix[S], iy[S], iz[S];
    double wx[S], wy[S], wz[S];
    if (valid) {
      axis_assign<S>(x, n, ix, wx);
      axis_assign<S>(y, n, iy, wy);
      axis_assign<S>(z, n, iz, wz);
    }
    // first point per axis before wrapping: ix[0] for CIC and NGP; for TSC ix[0] may have wrapped
    // from -1 to n - 1, which only widens the box (then the wave takes the direct path)
    const int bx = valid ? ix[0] : 0x3fffffff, by = valid ? iy[0] : 0x3fffffff, bz = valid ? iz[0] : 0x3fffffff;
    const int lox = wave_min_i(bx), loy = wave_min_i(by), loz = wave_min_i(bz);
    const int hix = wave_max_i(valid ? bx : -1), hiy = wave_max_i(valid ? by : -1), hiz = wave_max_i(valid ? bz : -1);
    if (hix < 0) continue;  // no valid particle in this segment (wave-uniform)
    const int ex = hix - lox + S, ey = hiy - loy + S, ez = hiz - loz + S;
    const bool binned = (long long)ex * ey * ez <= CAP;  // wave-uniform
    if (binned) {
      const int vol = ex * ey * ez;
      for (int t = lane; t < vol; t += 64) box[t] = 0ull;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (valid) {
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
          for (int b = 0; b < S; ++b)
#pragma unroll
            for (int d = 0; d < S; ++d) {
              const double wgt = wx[a] * wy[b] * wz[d];
              const unsigned long long q = (unsigned long long)__double2ull_rn(wgt * kFixScale);
              // local coordinates from the unwrapped neighbours of the first point
              const int l = ((bx + a - lox) * ey + (by + b - loy)) * ez + (bz + d - loz);
              if (q) atomicAdd(&box[l], q);
            }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int t = lane; t < vol; t += 64) {
        const unsigned long long v = box[t];
        if (v) {
          const int lz = t % ez, ly = (t / ez) % ey, lx = t / (ez * ey);
          int gx = lox + lx, gy = loy + ly, gz = loz + lz;
          gx -= gx >= n ? n : 0;
          gy -= gy >= n ? n : 0;
          gz -= gz >= n ? n : 0;
          atomicAdd(&grid[((size_t)gx * n + gy) * n + gz], v);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else if (valid) {
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) {
          const size_t row = ((size_t)ix[a] * n + iy[b]) * n;
#pragma unroll
          for (int d = 0; d < S; ++d) {
            const double wgt = wx[a] * wy[b] * wz[d];
            const unsigned long long q = (unsigned long long)__double2ull_rn(wgt * kFixScale);
            if (q) atomicAdd(&grid[row + iz[d]], q);
          }
        }
    }
  }
}

// ---- deposit through particles sorted by mesh tile (any particle order) ------------------------
// The mesh is cut into tiles of 16 x 16 x 32 points. A particle belongs to the tile of the lowest
// mesh point it reaches (the first of its S points per axis, wrapped); its S^3 points then lie in
// the tile's box of (16 + S - 1) x (16 + S - 1) x (32 + S - 1) points. Counting sort of the
// particles by tile: count per (block of particles, tile), exclusive scan, scatter of the
// positions into tile order. One block per tile then accumulates its particles' contributions in
// its box in LDS (64-bit fixed point, the same rounded contribution per particle and point as the
// scatter kernels above, so the integer sums and the result are bitwise those of the scatter) and
// writes the whole box out; a last pass adds to every point of a tile the boxes of the (up to 7)
// lower neighbour tiles that reach it and writes delta. No global atomics: the result does not
// depend on particle order, and the traffic is that of reading the catalogue three times.
constexpr int kDepTX = 16, kDepTY = 16, kDepTZ = 32;

struct DepGeom {
  int n, tnx, tny, tnz, ntiles;
};

template <int S>
struct DepBox {
  static constexpr int BX = kDepTX + S - 1, BY = kDepTY + S - 1, BZ = kDepTZ + S - 1;
  static constexpr int CELLS = BX * BY * BZ;
};

// The particle's tile and its first mesh point inside the tile (false for a non-finite position).
template <int S>
__device__ __forceinline__ bool dep_place(const double* __restrict__ pos, long long p, const DepGeom& g, int& tile,
                                          int (&ix)[S], int (&iy)[S], int (&iz)[S], double (&wx)[S], double (&wy)[S],
                                          double (&wz)[S]) {
  const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
  if (!__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(z)) return false;
  axis_assign<S>(x, g.n, ix, wx);
  axis_assign<S>(y, g.n, iy, wy);
  axis_assign<S>(z, g.n, iz, wz);
  tile = ((ix[0] / kDepTX) * g.tny + iy[0] / kDepTY) * g.tnz + iz[0] / kDepTZ;
  return true;
}

// hist[b][t]: particles of block b's range [b per, (b + 1) per) in tile t.
template <int S>
__global__ void __launch_bounds__(256) dep_count_kernel(const double* __restrict__ pos, long long np, DepGeom g,
                                                        long long per, unsigned* __restrict__ hist,
                                                        double* __restrict__ bad_count) {
  extern __shared__ unsigned dep_lds[];
  for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) dep_lds[t] = 0u;
  __syncthreads();
  const long long p0 = (long long)blockIdx.x * per, p1 = min(np, p0 + per);
  for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    int tile, ix[S], iy[S], iz[S];
    double wx[S], wy[S], wz[S];
    if (dep_place<S>(pos, p, g, tile, ix, iy, iz, wx, wy, wz))
      atomicAdd(&dep_lds[tile], 1u);
    else
      __hip_atomic_fetch_add(bad_count, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  unsigned* row = hist + (size_t)blockIdx.x * g.ntiles;
  for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) row[t] = dep_lds[t];
}

// hist[b][t] <- particles of tile t in blocks before b; total[t]. A block takes 64 consecutive tiles
// (one per lane, coalesced rows) and splits the blocks into 16 segments, one per wave: each wave
// sums its segment, the segment sums are scanned in LDS, then each wave writes its prefixes.
constexpr int kDepScanSeg = 16;
__global__ void __launch_bounds__(64 * kDepScanSeg) dep_scan_blocks_kernel(unsigned* __restrict__ hist, int nblocks,
                                                                           int ntiles, unsigned* __restrict__ total) {
  __shared__ unsigned seg[kDepScanSeg][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const int b0 = (int)(((long)w * nblocks) / kDepScanSeg), b1 = (int)(((long)(w + 1) * nblocks) / kDepScanSeg);
  unsigned s = 0u;
  if (t < ntiles)
    for (int b = b0; b < b1; ++b) s += hist[(size_t)b * ntiles + t];
  seg[w][lane] = s;
  __syncthreads();
  unsigned run = 0u;
  for (int k = 0; k < w; ++k) run += seg[k][lane];
  if (t < ntiles) {
    for (int b = b0; b < b1; ++b) {
      unsigned* c = hist + (size_t)b * ntiles + t;
      const unsigned v = *c;
      *c = run;
      run += v;
    }
    if (w == kDepScanSeg - 1) total[t] = run;
  }
}

// One block of 1024 threads: start[t] = particles of tiles before t, start[ntiles] = all of them.
__global__ void __launch_bounds__(1024) dep_scan_tiles_kernel(const unsigned* __restrict__ total, int ntiles,
                                                              unsigned* __restrict__ start) {
  __shared__ unsigned part[1024];
  const int tid = threadIdx.x;
  const int per = (ntiles + 1023) / 1024;
  const int t0 = tid * per, t1 = min(ntiles, t0 + per);
  unsigned s = 0u;
  for (int t = t0; t < t1; ++t) s += total[t];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan of the per-thread sums
    const unsigned v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  unsigned run = tid == 0 ? 0u : part[tid - 1];
  for (int t = t0; t < t1; ++t) {
    start[t] = run;
    run += total[t];
  }
  if (tid == 1023) start[ntiles] = part[1023];
}

// The positions of block b's particles into tile order (the order inside a tile is immaterial).
template <int S>
__global__ void __launch_bounds__(256) dep_scatter_kernel(const double* __restrict__ pos, long long np, DepGeom g,
                                                          long long per, const unsigned* __restrict__ hist,
                                                          const unsigned* __restrict__ start,
                                                          double* __restrict__ sorted) {
  extern __shared__ unsigned dep_lds[];
  const unsigned* row = hist + (size_t)blockIdx.x * g.ntiles;
  for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) dep_lds[t] = start[t] + row[t];
  __syncthreads();
  const long long p0 = (long long)blockIdx.x * per, p1 = min(np, p0 + per);
  for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    int tile, ix[S], iy[S], iz[S];
    double wx[S], wy[S], wz[S];
    if (!dep_place<S>(pos, p, g, tile, ix, iy, iz, wx, wy, wz)) continue;
    const unsigned slot = atomicAdd(&dep_lds[tile], 1u);
    double* r = sorted + 3 * (size_t)slot;
    r[0] = pos[3 * p];
    r[1] = pos[3 * p + 1];
    r[2] = pos[3 * p + 2];
  }
}

// One block per tile: the tile's particles into its box (LDS), the box out to boxes[tile].
template <int S>
__global__ void __launch_bounds__(256) dep_tile_kernel(const double* __restrict__ sorted,
                                                       const unsigned* __restrict__ start, DepGeom g,
                                                       unsigned long long* __restrict__ boxes) {
  using B = DepBox<S>;
  __shared__ unsigned long long box[B::CELLS];
  const int t = blockIdx.x;
  for (int c = threadIdx.x; c < B::CELLS; c += blockDim.x) box[c] = 0ull;
  __syncthreads();
  const int tz = t % g.tnz, ty = (t / g.tnz) % g.tny, tx = t / (g.tnz * g.tny);
  const unsigned q0 = start[t], q1 = start[t + 1];
  for (unsigned q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    int tile, ix[S], iy[S], iz[S];
    double wx[S], wy[S], wz[S];
    (void)dep_place<S>(sorted, (long long)q, g, tile, ix, iy, iz, wx, wy, wz);   // finite by construction
    const int lx = ix[0] - tx * kDepTX, ly = iy[0] - ty * kDepTY, lz = iz[0] - tz * kDepTZ;
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b)
#pragma unroll
        for (int d = 0; d < S; ++d) {
          const double w = wx[a] * wy[b] * wz[d];
          const unsigned long long v = (unsigned long long)__double2ull_rn(w * kFixScale);
          if (v) atomicAdd(&box[((lx + a) * B::BY + (ly + b)) * B::BZ + (lz + d)], v);
        }
  }
  __syncthreads();
  unsigned long long* out = boxes + (size_t)t * B::CELLS;
  for (int c = threadIdx.x; c < B::CELLS; c += blockDim.x) out[c] = box[c];
}

// One block per tile: every point of the tile sums its own box and the lower neighbours' boxes that
// reach it; delta = count n^3 / (np 2^40) - 1; partials[tile] = the tile's sum of counts / 2^40.
// Writes nothing when a particle had a non-finite position (*bad_count != 0, complete since the
// counting launch): the call then fails and leaves delta unchanged.
template <int S>
__global__ void __launch_bounds__(256) dep_combine_kernel(const unsigned long long* __restrict__ boxes, DepGeom g,
                                                          double scale, double* __restrict__ delta,
                                                          double* __restrict__ partials, const double* bad_count) {
  using B = DepBox<S>;
  __shared__ double red[16][1];
  const int t = blockIdx.x;
  if (*bad_count != 0.0) {
    if (threadIdx.x == 0) partials[t] = 0.0;
    return;
  }
  const int tz = t % g.tnz, ty = (t / g.tnz) % g.tny, tx = t / (g.tnz * g.tny);
  const int n = g.n;
  double acc = 0.0;
  for (int c = threadIdx.x; c < kDepTX * kDepTY * kDepTZ; c += blockDim.x) {
    const int lz = c % kDepTZ, ly = (c / kDepTZ) % kDepTY, lx = c / (kDepTZ * kDepTY);
    unsigned long long v = 0ull;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = k >> 2, dy = (k >> 1) & 1, dz = k & 1;
      if ((dx && lx >= S - 1) || (dy && ly >= S - 1) || (dz && lz >= S - 1)) continue;
      const int nx = tx - dx < 0 ? g.tnx - 1 : tx - dx;
      const int ny = ty - dy < 0 ? g.tny - 1 : ty - dy;
      const int nz = tz - dz < 0 ? g.tnz - 1 : tz - dz;
      const int nt = (nx * g.tny + ny) * g.tnz + nz;
      v += boxes[(size_t)nt * B::CELLS + ((lx + dx * kDepTX) * B::BY + (ly + dy * kDepTY)) * B::BZ + (lz + dz * kDepTZ)];
    }
    const size_t cell = ((size_t)(tx * kDepTX + lx) * n + (ty * kDepTY + ly)) * n + (tz * kDepTZ + lz);
    const double cnt = (double)v;
    delta[cell] = cnt * scale - 1.0;
    acc += cnt * (1.0 / kFixScale);
  }
  double vv[1] = {acc};
  block_sum<1>(vv, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0) partials[t] = vv[0];
}

// delta = count * n^3 / (np * 2^40) - 1; partials[block] = the block's sum of counts / 2^40. The
// partials are added by sum_partials_kernel in the next launch (fixed order, no per-block fences).
__global__ void __launch_bounds__(256) cic_normalise_kernel(const unsigned long long* __restrict__ grid, size_t cells,
                                                            double scale, double* __restrict__ delta,
                                                            double* __restrict__ partials) {
  __shared__ double red[16][1];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) {
    const double cnt = (double)grid[e];
    delta[e] = cnt * scale - 1.0;
    acc += cnt * (1.0 / kFixScale);
  }
  double v[1] = {acc};
  block_sum<1>(v, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// out[0] = sum of partials[0 .. count) in a fixed order (one block).
__global__ void __launch_bounds__(256) sum_partials_kernel(const double* __restrict__ partials, int count,
                                                           double* __restrict__ out) {
  __shared__ double red[16][1];
  double acc = 0.0;
  for (int b = threadIdx.x; b < count; b += blockDim.x) acc += partials[b];
  double v[1] = {acc};
  block_sum<1>(v, red, threadIdx.x, blockDim.x);
  if (threadIdx.x == 0) out[0] = v[0];
}

// Clears the accumulation grid; block 0 also clears the non-finite particle count.
__global__ void __launch_bounds__(256) zero_u64_kernel(unsigned long long* __restrict__ a, size_t cells,
                                                       double* __restrict__ bad_count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *bad_count = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < cells; e += (size_t)gridDim.x * blockDim.x) a[e] = 0ull;
}

static int blocks_for(size_t work, int cap) {
  size_t b = (work + 255) / 256;
  return (int)(b < 1 ? 1 : (b > (size_t)cap ? cap : b));
}

// The tile-sorted deposit (CIC, TSC) on meshes with n a multiple of 32 up to 512.
template <int S>
static int deposit_sorted(Ctx* c, const double* pos, long long np, double* delta_out) {
  const int n = c->n;
  DepGeom g{n, n / kDepTX, n / kDepTY, n / kDepTZ, 0};
  g.ntiles = g.tnx * g.tny * g.tnz;
  const size_t cells = (size_t)n * n * n;
  // particle ranges: at most 1024 blocks and 4M (block, tile) counters
  int nb = (int)std::min<long long>(1024, std::max<long long>(1, (4 << 20) / g.ntiles));
  nb = (int)std::min<long long>(nb, (np + 255) / 256);
  const long long per = (np + nb - 1) / nb;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_hist = al((size_t)nb * g.ntiles * 4), b_tot = al((size_t)g.ntiles * 4),
               b_start = al(((size_t)g.ntiles + 1) * 4), b_sorted = al((size_t)np * 24),
               b_boxes = al((size_t)g.ntiles * DepBox<3>::CELLS * 8);
  const size_t need = b_hist + b_tot + b_start + b_sorted + b_boxes;
  if (c->dep_bytes < need) {
    if (c->dep_mem) (void)hipFree(c->dep_mem);
    c->dep_mem = nullptr;
    c->dep_bytes = 0;
    hipError_t e = hipMalloc(&c->dep_mem, need);
    if (e != hipSuccess) return fail(MR_ENOMEM, "density assignment: %.1f MiB of sort buffers", need / 1048576.0);
    c->dep_bytes = need;
  }
  char* m = (char*)c->dep_mem;
  unsigned* hist = (unsigned*)m;
  unsigned* total = (unsigned*)(m + b_hist);
  unsigned* start = (unsigned*)(m + b_hist + b_tot);
  double* sorted = (double*)(m + b_hist + b_tot + b_start);
  unsigned long long* boxes = (unsigned long long*)(m + b_hist + b_tot + b_start + b_sorted);
  double* bad_count = c->scal + kSlotRes;
  const size_t lds = (size_t)g.ntiles * 4;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, c->stream, (unsigned long long*)nullptr, (size_t)0, bad_count);
  hipLaunchKernelGGL(dep_count_kernel<S>, dim3(nb), dim3(256), lds, c->stream, pos, np, g, per, hist, bad_count);
  hipLaunchKernelGGL(dep_scan_blocks_kernel, dim3((g.ntiles + 63) / 64), dim3(64 * kDepScanSeg), 0, c->stream, hist, nb,
                     g.ntiles, total);
  hipLaunchKernelGGL(dep_scan_tiles_kernel, dim3(1), dim3(1024), 0, c->stream, (const unsigned*)total, g.ntiles, start);
  hipLaunchKernelGGL(dep_scatter_kernel<S>, dim3(nb), dim3(256), lds, c->stream, pos, np, g, per, (const unsigned*)hist,
                     (const unsigned*)start, sorted);
  hipLaunchKernelGGL(dep_tile_kernel<S>, dim3(g.ntiles), dim3(256), 0, c->stream, (const double*)sorted,
                     (const unsigned*)start, g, boxes);
  const double scale = (double)cells / ((double)np * kFixScale);
  hipLaunchKernelGGL(dep_combine_kernel<S>, dim3(g.ntiles), dim3(256), 0, c->stream, (const unsigned long long*)boxes, g,
                     scale, delta_out, c->partials, (const double*)bad_count);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, c->stream, (const double*)c->partials, g.ntiles,
                     c->scal + kSlotRes + 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mr_deposit");
  double r[2];
  int rc = c->read_scalars(kSlotRes, 2, r);
  if (rc != MR_OK) return rc;
  if (r[0] != 0.0) return fail(MR_EINVAL, "mr_deposit: %.0f particles with non-finite coordinates", r[0]);
  if (!(std::fabs(r[1] - (double)np) <= 0.5 + 1e-9 * (double)np))
    return fail(MR_EINVAL, "mr_deposit: fixed-point overflow (deposited %.6g of %lld particles)", r[1], np);
  return MR_OK;
}

static bool deposit_sorted_applies(int n, long long np) {
  return n % 32 == 0 && n >= 32 && n <= 512 && np < ((long long)1 << 31);
}

int Ctx::deposit(const double* pos, long long np, double mass, int scheme, double* delta_out) {
  const size_t cells = lv[0].cells;
  (void)mass;
  if (!(opts.flags & MR_FLAG_DEPOSIT_SCATTER) && scheme != MR_DEPOSIT_NGP && deposit_sorted_applies(n, np))
    return scheme == MR_DEPOSIT_CIC ? deposit_sorted<2>(this, pos, np, delta_out)
                                    : deposit_sorted<3>(this, pos, np, delta_out);
  if (!cic_grid) {
    hipError_t e = hipMalloc((void**)&cic_grid, cells * sizeof(unsigned long long));
    if (e != hipSuccess) return fail(MR_ENOMEM, "density assignment grid: %s", hipGetErrorString(e));
  }
  double* bad_count = scal + kSlotRes;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(blocks_for(cells, 1 << 16)), dim3(256), 0, stream, cic_grid, cells,
                     bad_count);
  const dim3 pg(blocks_for((size_t)np, 1 << 16));
  // CIC and TSC bin each wave's contributions in LDS (boxes of up to 1024 / 2048 mesh points);
  // NGP has one contribution per particle and little to combine.
  const dim3 wg((unsigned)std::min<long long>((np + 255) / 256, 1 << 16));
  // np = m^3 with m a multiple of 8: let each wave take a 2 x 4 x 8 block of the particle lattice
  long long m = (long long)std::llround(std::cbrt((double)np));
  while (m > 0 && m * m * m > np) --m;
  while ((m + 1) * (m + 1) * (m + 1) <= np) ++m;
  const int lattice = (m * m * m == np && m % 8 == 0 && m <= (1 << 20)) ? (int)m : 0;
  if (scheme == MR_DEPOSIT_NGP)
    hipLaunchKernelGGL(deposit_scatter_kernel<1>, pg, dim3(256), 0, stream, pos, np, n, cic_grid, bad_count);
  else if (scheme == MR_DEPOSIT_CIC)
    hipLaunchKernelGGL((deposit_scatter_binned_kernel<2, 1024>), wg, dim3(256), 0, stream, pos, np, n, cic_grid,
                       bad_count, lattice);
  else
    hipLaunchKernelGGL((deposit_scatter_binned_kernel<3, 2048>), wg, dim3(256), 0, stream, pos, np, n, cic_grid,
                       bad_count, lattice);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mr_deposit");
  double bad;
  int rc = read_scalars(kSlotRes, 1, &bad);
  if (rc != MR_OK) return rc;
  if (bad != 0.0) return fail(MR_EINVAL, "mr_deposit: %.0f particles with non-finite coordinates", bad);
  const double scale = (double)cells / ((double)np * kFixScale);
  const int nb = blocks_for(cells, kMaxReduceBlocks);
  hipLaunchKernelGGL(cic_normalise_kernel, dim3(nb), dim3(256), 0, stream, cic_grid, cells, scale, delta_out, partials);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, stream, partials, nb, scal + kSlotRes);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mr_deposit");
  double total;
  if ((rc = read_scalars(kSlotRes, 1, &total)) != MR_OK) return rc;
  // Each particle contributes 1 up to 27 roundings of 2^-41; a wrapped 64-bit cell loses 2^24.
  if (!(std::fabs(total - (double)np) <= 0.5 + 1e-9 * (double)np))
    return fail(MR_EINVAL, "mr_deposit: fixed-point overflow (deposited %.6g of %lld particles)", total, np);
  (void)mass;
  return MR_OK;
}

// ---- Lagrangian mapping -----------------------------------------------------------------------
// q = grad Theta = x + grad theta (Theta_0 = |x|^2 / 2, Sec. II; x - q = -grad theta, Sec. III), so
// the displacement is psi = grad theta: the central difference (theta(i+1) - theta(i-1)) / 2 per
// axis on the mesh (cell units), interpolated to each particle with the CIC weights above (the
// transpose of the deposit).

// psi[(i n + j) n + k][a], a = x, y, z; one row (i, j) per block, theta in natural order. The row's
// 3n outputs are assembled in LDS and written with consecutive lanes on consecutive doubles.
constexpr int kLagRowMax = 1024;  // largest mesh a context accepts
// Block 0 also clears the non-finite particle count that the gather that follows accumulates.
__global__ void __launch_bounds__(256) lag_grad_kernel(const double* __restrict__ theta, int n,
                                                       double* __restrict__ psi, double* __restrict__ bad_count) {
  __shared__ double stage[3 * kLagRowMax];
  if (blockIdx.x == 0 && threadIdx.x == 0) *bad_count = 0.0;
  const int row = xcd_remap(blockIdx.x, gridDim.x);
  const int i = row / n, j = row - i * n;
  const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
  const int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
  const double* __restrict__ r0 = theta + ((size_t)i * n + j) * n;
  const double* __restrict__ rxm = theta + ((size_t)im * n + j) * n;
  const double* __restrict__ rxp = theta + ((size_t)ip * n + j) * n;
  const double* __restrict__ rym = theta + ((size_t)i * n + jm) * n;
  const double* __restrict__ ryp = theta + ((size_t)i * n + jp) * n;
  double* __restrict__ out = psi + ((size_t)i * n + j) * n * 3;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int km = k == 0 ? n - 1 : k - 1, kp = k == n - 1 ? 0 : k + 1;
    stage[3 * k + 0] = (rxp[k] - rxm[k]) * 0.5;
    stage[3 * k + 1] = (ryp[k] - rym[k]) * 0.5;
    stage[3 * k + 2] = (r0[kp] - r0[km]) * 0.5;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) out[t] = stage[t];
}

// disp[p] = sum over the 8 mesh points around x_p of w * psi (corners in x-major order). A particle
// with a non-finite coordinate is not interpolated (its output is NaN) and adds 1 to *bad_count
// with a relaxed atomic: an exact, order-independent integer count that needs no grid-wide
// reduction (whose per-block release/acquire would write back and invalidate the L2 that the
// concurrently running blocks reuse mesh lines from).
__global__ void __launch_bounds__(256) lag_gather_kernel(const double* __restrict__ pos, long long np, int n,
                                                        const double* __restrict__ psi, double* __restrict__ disp,
                                                        double* __restrict__ bad_count) {
  // consecutive particles on one XCD: lattice-ordered catalogues then reuse mesh lines in its L2
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = xcd_remap(blockIdx.x, gridDim.x) * (long long)blockDim.x + threadIdx.x; p < np; p += stride) {
    const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
    if (!__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(z)) {
      __hip_atomic_fetch_add(bad_count, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      disp[3 * p] = disp[3 * p + 1] = disp[3 * p + 2] = __builtin_nan("");
      continue;
    }
    int ix0, ix1, iy0, iy1, iz0, iz1;
    double fx, fy, fz;
    wrap_coord(x, n, ix0, ix1, fx);
    wrap_coord(y, n, iy0, iy1, fy);
    wrap_coord(z, n, iz0, iz1, fz);
    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    const int ix[2] = {ix0, ix1}, iy[2] = {iy0, iy1}, iz[2] = {iz0, iz1};
    // all 24 loads are issued before the first use so that their latencies overlap
    double v[8][3];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = c >> 2, b = (c >> 1) & 1, d = c & 1;
      const double* __restrict__ src = psi + (((size_t)ix[a] * n + iy[b]) * n + iz[d]) * 3;
      v[c][0] = src[0];
      v[c][1] = src[1];
      v[c][2] = src[2];
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = c >> 2, b = (c >> 1) & 1, d = c & 1;
      const double w = wx[a] * wy[b] * wz[d];
      a0 += w * v[c][0];
      a1 += w * v[c][1];
      a2 += w * v[c][2];
    }
    disp[3 * p] = a0;
    disp[3 * p + 1] = a1;
    disp[3 * p + 2] = a2;
  }
}

// Without the mesh field: the central differences of the 8 corners are formed at the particle from
// theta itself (32 loads: per (y, z) corner pair the 4 points of the x line, per (x, z) and (x, y)
// pair the 2 outer points of the y and z lines), with the same operations in the same order as
// lag_grad_kernel followed by lag_gather_kernel, so the result is bitwise the same; theta (1/3 of the
// mesh field) is read instead of writing and reading psi.
__global__ void __launch_bounds__(256) lag_gather_theta_kernel(const double* __restrict__ pos, long long np, int n,
                                                              const double* __restrict__ theta,
                                                              double* __restrict__ disp,
                                                              double* __restrict__ bad_count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = xcd_remap(blockIdx.x, gridDim.x) * (long long)blockDim.x + threadIdx.x; p < np; p += stride) {
    const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
    if (!__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(z)) {
      __hip_atomic_fetch_add(bad_count, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      disp[3 * p] = disp[3 * p + 1] = disp[3 * p + 2] = __builtin_nan("");
      continue;
    }
    int ix0, ix1, iy0, iy1, iz0, iz1;
    double fx, fy, fz;
    wrap_coord(x, n, ix0, ix1, fx);
    wrap_coord(y, n, iy0, iy1, fy);
    wrap_coord(z, n, iz0, iz1, fz);
    const int xm = ix0 == 0 ? n - 1 : ix0 - 1, xp = ix1 == n - 1 ? 0 : ix1 + 1;
    const int ym = iy0 == 0 ? n - 1 : iy0 - 1, yp = iy1 == n - 1 ? 0 : iy1 + 1;
    const int zm = iz0 == 0 ? n - 1 : iz0 - 1, zp = iz1 == n - 1 ? 0 : iz1 + 1;
    const int xs[4] = {xm, ix0, ix1, xp}, ys[4] = {ym, iy0, iy1, yp}, zs[4] = {zm, iz0, iz1, zp};
    auto T = [&](int i, int j, int k) { return theta[((size_t)i * n + j) * n + k]; };
    double lx[2][2][4];   // [b][d][x line]
    double ly[2][2][2];   // [a][d][y minus / plus]
    double lz[2][2][2];   // [a][b][z minus / plus]
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int t = 0; t < 4; ++t) lx[b][d][t] = T(xs[t], ys[b + 1], zs[d + 1]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        ly[a][d][0] = T(xs[a + 1], ys[0], zs[d + 1]);
        ly[a][d][1] = T(xs[a + 1], ys[3], zs[d + 1]);
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        lz[a][b][0] = T(xs[a + 1], ys[b + 1], zs[0]);
        lz[a][b][1] = T(xs[a + 1], ys[b + 1], zs[3]);
      }
    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    double v[8][3];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = c >> 2, b = (c >> 1) & 1, d = c & 1;
      // the x, y and z central differences at corner (a, b, d), as lag_grad_kernel forms them
      v[c][0] = (lx[b][d][a + 2] - lx[b][d][a]) * 0.5;
      const double ylo = b == 0 ? ly[a][d][0] : lx[0][d][a + 1];
      const double yhi = b == 0 ? lx[1][d][a + 1] : ly[a][d][1];
      v[c][1] = (yhi - ylo) * 0.5;
      const double zlo = d == 0 ? lz[a][b][0] : lx[b][0][a + 1];
      const double zhi = d == 0 ? lx[b][1][a + 1] : lz[a][b][1];
      v[c][2] = (zhi - zlo) * 0.5;
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = c >> 2, b = (c >> 1) & 1, d = c & 1;
      const double w = wx[a] * wy[b] * wz[d];
      a0 += w * v[c][0];
      a1 += w * v[c][1];
      a2 += w * v[c][2];
    }
    disp[3 * p] = a0;
    disp[3 * p + 1] = a1;
    disp[3 * p + 2] = a2;
  }
}

__global__ void zero_scalar_kernel(double* __restrict__ v) { *v = 0.0; }

int Ctx::lagrangian(const double* theta, const double* pos, long long np, double* disp_out, double* psi_out) {
  double* bad_count = scal + kSlotRes;
  // one particle per thread up to 2^28 particles, a grid-stride loop beyond
  const long long gb = std::min<long long>((np + 255) / 256, 1 << 20);
  if (psi_out) {
    hipLaunchKernelGGL(lag_grad_kernel, dim3((unsigned)n * n), dim3(n < 256 ? (n < 64 ? 64 : n) : 256), 0, stream, theta,
                       n, psi_out, bad_count);
    hipLaunchKernelGGL(lag_gather_kernel, dim3((unsigned)gb), dim3(256), 0, stream, pos, np, n, psi_out, disp_out,
                       bad_count);
  } else {
    hipLaunchKernelGGL(zero_scalar_kernel, dim3(1), dim3(1), 0, stream, bad_count);
    hipLaunchKernelGGL(lag_gather_theta_kernel, dim3((unsigned)gb), dim3(256), 0, stream, pos, np, n, theta, disp_out,
                       bad_count);
  }
  hipError_t e = hipGetLastError();
  double bad = 0.0;
  int rc = e == hipSuccess ? read_scalars(kSlotRes, 1, &bad) : hip_fail(e, "mr_lagrangian");
  if (rc != MR_OK) return rc;
  if (bad != 0.0) return fail(MR_EINVAL, "mr_lagrangian: %.0f particles with non-finite coordinates", bad);
  return MR_OK;
}

}  // namespace mr

extern "C" int mr_deposit(mr_ctx* h, const double* pos, int64_t np, double mass, int scheme, double* delta_out) {
  if (!h || !pos || !delta_out) return mr::fail(MR_EINVAL, "mr_deposit: null argument");
  if (np < 1) return mr::fail(MR_EINVAL, "mr_deposit: no particles");
  if (!(mass > 0.0) || !std::isfinite(mass)) return mr::fail(MR_EINVAL, "mr_deposit: mass must be positive");
  if (scheme != MR_DEPOSIT_NGP && scheme != MR_DEPOSIT_CIC && scheme != MR_DEPOSIT_TSC)
    return mr::fail(MR_EINVAL, "mr_deposit: unknown scheme %d", scheme);
  return reinterpret_cast<mr::Ctx*>(h)->deposit(pos, (long long)np, mass, scheme, delta_out);
}

extern "C" int mr_deposit_cic(mr_ctx* h, const double* pos, int64_t np, double mass, double* delta_out) {
  return mr_deposit(h, pos, np, mass, MR_DEPOSIT_CIC, delta_out);
}

extern "C" int mr_lagrangian(mr_ctx* h, const double* theta, const double* pos, int64_t np, double* disp_out,
                             double* psi_out) {
  if (!h || !theta || !pos || !disp_out) return mr::fail(MR_EINVAL, "mr_lagrangian: null argument");
  if (np < 1) return mr::fail(MR_EINVAL, "mr_lagrangian: no particles");
  return reinterpret_cast<mr::Ctx*>(h)->lagrangian(theta, pos, (long long)np, disp_out, psi_out);
}
