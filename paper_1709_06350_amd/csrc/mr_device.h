// Device helpers shared by the kernels of the library: the 19-point stencil of the
// reconstruction equation, the physical root of its cubic, periodic indexing and a
// deterministic block/grid reduction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mr {

// theta at the 18 non-central points of the 3x3x3 neighbourhood used by the discrete
// Laplacian and cross derivatives (Sec. II.A.1, Eqs. 11-14); corners are not used.
struct Nb18 {
  double xm, xp, ym, yp, zm, zp;      // face neighbours (i-1,i+1), (j-1,j+1), (k-1,k+1)
  double xpyp, xmym, xpym, xmyp;      // (i+-1, j+-1)
  double xpzp, xmzm, xpzm, xmzp;      // (i+-1, k+-1)
  double ypzp, ymzm, ypzm, ymzp;      // (j+-1, k+-1)
};

__device__ __forceinline__ int wrapi(int x, int n) {
  return x < 0 ? x + n : (x >= n ? x - n : x);
}

// Largest real root of s^3 + p s + q = 0 (the physical branch of Sec. II, Eq. 10; p <= 0).
// Newton's method from an upper bound of that root. With c = cbrt(max(-q, 0)) two upper bounds
// are available: sqrt(-p) + c, and c - p/(3c) (the cubic at c + e with e = -p/(3c) equals
// e^3 >= 0, and c + e >= sqrt(-p/3)), so the iteration starts on the convex, increasing branch
// right of the root and decreases monotonically onto it. The seed is formed in FP32 with the
// hardware log2/exp2/sqrt/rcp; each FP64 step uses the approximate hardware reciprocal, whose
// error only scales the already-small step. Every root takes four steps; a root whose last step
// is still above 1e-8 of it keeps stepping until one is below (Newton's error is then below
// ~1e-15). The result depends only on (p, q), never on the other lanes of the wavefront.
// N independent roots are iterated together to overlap their latencies.
__device__ __forceinline__ float root_seed(double p, double q) {
  const float pf = (float)p;
  const float mq = fmaxf(-(float)q, 0.0f);
  const float c = mq > 0.0f ? __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(mq) * (1.0f / 3.0f)) : 0.0f;
  const float b1 = __builtin_amdgcn_sqrtf(fmaxf(-pf, 0.0f)) + c;
  const float b2 = c > 0.0f ? c - pf * __builtin_amdgcn_rcpf(3.0f * c) : b1;
  return fminf(b1, b2);
}

template <int N>
__device__ __forceinline__ void largest_roots(const double (&p)[N], const double (&q)[N], double (&s)[N]) {
  double ds[N];
#pragma unroll
  for (int u = 0; u < N; ++u) s[u] = (double)root_seed(p[u], q[u]);
  // Four steps for every root: from the upper-bound seed (typically ~1e-4 away) this reaches the
  // stopping test for nearly every cell, with no per-lane control in the common path.
  // One step: with s2 = s^2 and t = s2 + p, the cubic is s t + q and its derivative 3 s2 + p is
  // 2 s2 + t (a multiply-add by 2, which the hardware takes as an inline constant).
#pragma unroll
  for (int it = 0; it < 4; ++it) {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const double s2 = s[u] * s[u];
      const double t = s2 + p[u];
      const double g = __builtin_fma(s[u], t, q[u]);
      const double gp = __builtin_fma(2.0, s2, t);
      ds[u] = g * __builtin_amdgcn_rcp(gp);
      s[u] -= ds[u];
    }
  }
  bool done[N];
  bool any = false;
#pragma unroll
  for (int u = 0; u < N; ++u) {
    done[u] = !(__builtin_fabs(ds[u]) > 1e-8 * s[u]);
    any = any || !done[u];
  }
  if (__ballot(any) == 0) return;
  // the few roots that still move (near a double root or from a poor seed) continue alone
#pragma unroll 1
  for (int it = 4; it < 24; ++it) {
    any = false;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const double s2 = s[u] * s[u];
      const double t = s2 + p[u];
      const double g = __builtin_fma(s[u], t, q[u]);
      const double gp = __builtin_fma(2.0, s2, t);
      const double d = g * __builtin_amdgcn_rcp(gp);
      const double sn = s[u] - d;
      s[u] = done[u] ? s[u] : sn;
      done[u] = done[u] || !(__builtin_fabs(d) > 1e-8 * sn);
      any = any || !done[u];
    }
    if (__ballot(any) == 0) break;
  }
}

__device__ __forceinline__ double largest_root(double p, double q) {
  double pp[1] = {p}, qq[1] = {q}, s[1];
  largest_roots<1>(pp, qq, s);
  return s[0];
}

// Cubic coefficients p, q of one cell and S = sum of the 6 face neighbours (see sigma_cell).
// Evaluated on U_a = 4 u_a and D_ab = 4 w_ab, so that no quarter is applied per term: every
// factor 4 is exact in binary, h^4 T2 = (sum U_a^2 + 2 sum D_ab^2) / 16 and h^6 T3 = (3 U_x U_y U_z
// - 3 (U_z D_xy^2 + U_y D_xz^2 + U_x D_yz^2) + 6 D_xy D_xz D_yz) / 64, and the powers of two
// 1/16 and 1/64 go into the constants -9/2 and 9, so p and q round exactly as with u and w.
__device__ __forceinline__ void cell_pq(const Nb18& t, double opd, double ih2, double& S, double& p, double& q) {
  const double Sx = t.xm + t.xp;
  const double Sy = t.ym + t.yp;
  const double Sz = t.zm + t.zp;
  S = Sx + Sy + Sz;
  const double s3 = S * (4.0 / 3.0);
  const double ux = __builtin_fma(4.0, Sx, -s3), uy = __builtin_fma(4.0, Sy, -s3), uz = __builtin_fma(4.0, Sz, -s3);
  const double wxy = (t.xpyp + t.xmym) - (t.xpym + t.xmyp);
  const double wxz = (t.xpzp + t.xmzm) - (t.xpzm + t.xmzp);
  const double wyz = (t.ypzp + t.ymzm) - (t.ypzm + t.ymzp);
  const double wxy2 = wxy * wxy, wxz2 = wxz * wxz, wyz2 = wyz * wyz;
  const double P = __builtin_fma(ux, ux, __builtin_fma(uy, uy, uz * uz)) + 2.0 * (wxy2 + wxz2 + wyz2);
  const double Q = 3.0 * (ux * uy * uz - (__builtin_fma(uz, wxy2, __builtin_fma(uy, wxz2, ux * wyz2))))
                   + 6.0 * wxy * wxz * wyz;
  const double ih4 = ih2 * ih2;
  p = (-4.5 / 16.0) * P * ih4;
  q = __builtin_fma((9.0 / 64.0) * Q, ih4 * ih2, -27.0 * opd);
}

// Sigma = s* - 3 of one cell and S = sum of the 6 face neighbours.
// With u_a = S_a - S/3 (h^2 times the barred diagonal) and w_ab = D_ab/4 (h^2 times the barred
// off-diagonal), h^4 T2 = sum u_a^2 + 2 sum w_ab^2 and h^6 T3 = 3 u_x u_y u_z
// - 3 (u_z w_xy^2 + u_y w_xz^2 + u_x w_yz^2) + 6 w_xy w_xz w_yz (tr of the cube of a traceless
// symmetric matrix); p = -(9/2) T2, q = 9 T3 - 27 (1 + delta) (Sec. II, Eq. 9; Appendix A).
__device__ __forceinline__ double sigma_cell(const Nb18& t, double opd, double ih2, double& S) {
  double p, q;
  cell_pq(t, opd, ih2, S, p, q);
  return largest_root(p, q) - 3.0;
}

// ---- colour-split layout --------------------------------------------------------------------
// Inside the solver every n^3 field is stored colour-split: [c][i][j][m] with c = (i+j+k) & 1
// (0 red, 1 black) and m = k >> 1, so that each half-sweep streams one contiguous colour.
// In row (i, j) the cells of colour c sit at k = 2m + ((i + j + c) & 1).
__device__ __forceinline__ unsigned split_idx(int n, int i, int j, int k) {
  const unsigned half = (unsigned)n * (unsigned)n * (unsigned)(n >> 1);
  return ((i + j + k) & 1) * half + ((unsigned)i * n + j) * (unsigned)(n >> 1) + (unsigned)(k >> 1);
}

// Gather the 18 neighbours of (i, j, k) from a colour-split periodic n^3 field.
__device__ __forceinline__ void gather18_split(const double* __restrict__ a, int n, int i, int j, int k, Nb18& t) {
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

// Gather the 18 neighbours of (i, j, k) from a periodic n^3 array in global memory.
__device__ __forceinline__ void gather18(const double* __restrict__ a, int n, int i, int j, int k, Nb18& t) {
  const int im = wrapi(i - 1, n), ip = wrapi(i + 1, n);
  const int jm = wrapi(j - 1, n), jp = wrapi(j + 1, n);
  const int km = wrapi(k - 1, n), kp = wrapi(k + 1, n);
  const size_t N = (size_t)n;
#define MR_AT(I, J, K) a[((size_t)(I) * N + (size_t)(J)) * N + (size_t)(K)]
  t.xm = MR_AT(im, j, k); t.xp = MR_AT(ip, j, k);
  t.ym = MR_AT(i, jm, k); t.yp = MR_AT(i, jp, k);
  t.zm = MR_AT(i, j, km); t.zp = MR_AT(i, j, kp);
  t.xpyp = MR_AT(ip, jp, k); t.xmym = MR_AT(im, jm, k); t.xpym = MR_AT(ip, jm, k); t.xmyp = MR_AT(im, jp, k);
  t.xpzp = MR_AT(ip, j, kp); t.xmzm = MR_AT(im, j, km); t.xpzm = MR_AT(ip, j, km); t.xmzp = MR_AT(im, j, kp);
  t.ypzp = MR_AT(i, jp, kp); t.ymzm = MR_AT(i, jm, km); t.ypzm = MR_AT(i, jp, km); t.ymzp = MR_AT(i, jm, kp);
#undef MR_AT
}

// ---- deterministic reductions -------------------------------------------------------------
// Every block reduces its values with a fixed tree (wavefront butterfly, then waves in order),
// writes one partial per value, and the last block to finish (agent-scope counter) sums the
// partials in index order and writes the totals. The counter is returned to zero by that
// block, so consecutive launches need no reset. Results are independent of scheduling.
// Each block's counter increment is a release (its partial is visible before the count); only
// the last block then takes the matching acquire. An acquire in every block would invalidate each
// XCD's L2 once per block, which costs ~25 ns per block on a single address.

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*red)[NV], int tid, int nthreads) {
  const int lane = tid & 63, wid = tid >> 6;
  const int nw = (nthreads + 63) >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) red[wid][c] = v[c];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w][c];
      v[c] = s;
    }
  }
  __syncthreads();
}

// All threads of the block must call this. On return, thread 0 of the last block has written
// result[0..NV-1]. nblocks is the number of blocks of the launch, bid this block's index.
template <int NV>
__device__ bool grid_sum(double (&v)[NV], double* __restrict__ partials, unsigned int* counter,
                         double* result, int nblocks, int bid) {
  __shared__ double red[16][NV];
  __shared__ int am_last;
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  block_sum<NV>(v, red, tid, nthreads);
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) partials[(size_t)bid * NV + c] = v[c];
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (prev == (unsigned)(nblocks - 1));
  }
  __syncthreads();
  if (!am_last) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double w[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) w[c] = 0.0;
  for (int b = tid; b < nblocks; b += nthreads) {
#pragma unroll
    for (int c = 0; c < NV; ++c)
      w[c] += __hip_atomic_load(&partials[(size_t)b * NV + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum<NV>(w, red, tid, nthreads);
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) result[c] = w[c];
    __hip_atomic_store(counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  return true;
}

// Raw buffer access to one plane: a resource built from a wave-uniform base pointer (scalar
// registers) and a per-lane 32-bit byte offset. This keeps per-lane address arithmetic at 32 bits
// where the loop optimiser would otherwise materialise 64-bit addresses per load. Offsets at or
// beyond `bytes` read 0 and drop stores (the hardware range check), never fault.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const double* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double ld_rs(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}
__device__ __forceinline__ void st_rs(__amdgpu_buffer_rsrc_t r, unsigned byte_off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                       r, (int)byte_off, 0, 0);
}

// Non-temporal variants (cache policy NT): for data a kernel streams exactly once -- inputs read once
// per pass and outputs not read again by the same launch -- so that they do not displace the reused
// halo planes from the caches.
__device__ __forceinline__ double ld_rs_nt(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 2));
}
__device__ __forceinline__ void st_rs_nt(__amdgpu_buffer_rsrc_t r, unsigned byte_off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                       r, (int)byte_off, 0, 2);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float ld_rs_f(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}
__device__ __forceinline__ void st_rs_f(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0, 0);
}
__device__ __forceinline__ float ld_rs_f_nt(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 2));
}
__device__ __forceinline__ void st_rs_f_nt(__amdgpu_buffer_rsrc_t r, unsigned byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0, 2);
}

// Map a launch-order block index to a logical tile index so that each of the 8 XCDs (which
// receive blocks round-robin) works on one contiguous range of tiles and shares halos in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace mr
