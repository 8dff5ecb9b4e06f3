// Streaming kernels that measure the HBM bandwidth this device sustains (the ceiling the
// memory-bound kernels of the solver are judged against). Not part of the method.
//
// kind MR_STREAM_COPY:  c[i] = a[i]            (16 B per element)
// kind MR_STREAM_READ:  sum of a[i]            ( 8 B per element; one partial per block into c)
// kind MR_STREAM_TRIAD: c[i] = a[i] + s b[i]   (24 B per element: the relaxation sweep's two reads
//                                               and one write of FP64 per cell)
// Each lane moves 16-byte vectors; the grid is a fixed multiple of the compute units with a
// grid-stride loop, so every launch keeps all CUs streaming.
#include <hip/hip_runtime.h>

#include "mr.h"
#include "mr_ctx.h"

namespace mr {

template <int KIND, bool NT>
__global__ void __launch_bounds__(256) stream_kernel(const double2* __restrict__ a, const double2* __restrict__ b,
                                                     double2* __restrict__ c, size_t nvec, double s) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvec; i += stride) {
    double2 x;
    if (NT) {
      x.x = __builtin_nontemporal_load(&a[i].x);
      x.y = __builtin_nontemporal_load(&a[i].y);
    } else {
      x = a[i];
    }
    if (KIND == MR_STREAM_READ) {
      acc += x.x + x.y;
      continue;
    }
    if (KIND == MR_STREAM_TRIAD) {
      double2 y;
      if (NT) {
        y.x = __builtin_nontemporal_load(&b[i].x);
        y.y = __builtin_nontemporal_load(&b[i].y);
      } else {
        y = b[i];
      }
      x.x += s * y.x;
      x.y += s * y.y;
    }
    if (NT) {
      __builtin_nontemporal_store(x.x, &c[i].x);
      __builtin_nontemporal_store(x.y, &c[i].y);
    } else {
      c[i] = x;
    }
  }
  if (KIND == MR_STREAM_READ) {
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) reinterpret_cast<double*>(c)[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

}  // namespace mr

using namespace mr;

extern "C" int mr_hbm_stream(int kind, int nontemporal, const double* a, const double* b, double* c, size_t count,
                             int blocks_per_cu, void* hip_stream, float* ms_out) {
  if (!a || !c || (kind == MR_STREAM_TRIAD && !b) || count < 2 || count % 2 != 0 || blocks_per_cu < 1 ||
      blocks_per_cu > 64 || (kind != MR_STREAM_COPY && kind != MR_STREAM_READ && kind != MR_STREAM_TRIAD))
    return fail(MR_EINVAL, "mr_hbm_stream: bad argument");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "mr_hbm_stream");
  const unsigned blocks = (unsigned)(cus * blocks_per_cu);
  if (kind == MR_STREAM_READ && count < blocks) return fail(MR_EINVAL, "mr_hbm_stream: c must hold one value per block");
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (ms_out) {
    e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  }
  const size_t nvec = count / 2;
  const double2* a2 = reinterpret_cast<const double2*>(a);
  const double2* b2 = reinterpret_cast<const double2*>(b);
  double2* c2 = reinterpret_cast<double2*>(c);
#define MR_STREAM_LAUNCH(K)                                                                                  \
  if (kind == K) {                                                                                           \
    if (nontemporal)                                                                                         \
      hipLaunchKernelGGL((stream_kernel<K, true>), dim3(blocks), dim3(256), 0, s, a2, b2, c2, nvec, 0.5);    \
    else                                                                                                     \
      hipLaunchKernelGGL((stream_kernel<K, false>), dim3(blocks), dim3(256), 0, s, a2, b2, c2, nvec, 0.5);   \
  }
  if (e == hipSuccess) {
    MR_STREAM_LAUNCH(MR_STREAM_COPY)
    MR_STREAM_LAUNCH(MR_STREAM_READ)
    MR_STREAM_LAUNCH(MR_STREAM_TRIAD)
    e = hipGetLastError();
  }
#undef MR_STREAM_LAUNCH
  if (ms_out && e == hipSuccess) {
    e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_out, ev[0], ev[1]);
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  return e == hipSuccess ? MR_OK : hip_fail(e, "mr_hbm_stream");
}
