// FP64 momentum reductions over the near-field accelerations.
//
// For equal masses and a symmetric near-field relation the pair forces are
// equal and opposite, so sum_i a_i vanishes in exact arithmetic; with FP32
// forces it measures the accumulated rounding.  Per box this returns
// (sum a_x, sum a_y, sum a_z, sum |a|) reduced in FP64 in a fixed order (wave
// shuffles, then LDS, then a second fixed-order pass over kMomChunks partials
// per box, enough blocks to fill the chip), so the result does not depend on
// scheduling.
#include "nf_internal.h"

namespace anf {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_momentum_partial(const DevBox* __restrict__ boxes,
                                                          const float* __restrict__ acc,
                                                          double* __restrict__ partials) {
  __shared__ double red[4][4];
  const int b = blockIdx.y, chunk = blockIdx.x;
  const int64_t first = boxes[b].first, n = boxes[b].n;
  double sx = 0.0, sy = 0.0, sz = 0.0, sn = 0.0;
  for (int64_t k = (int64_t)chunk * 256 + threadIdx.x; k < n; k += (int64_t)kMomChunks * 256) {
    const int64_t i = first + k;
    const double x = acc[3 * i + 0], y = acc[3 * i + 1], z = acc[3 * i + 2];
    sx += x;
    sy += y;
    sz += z;
    sn += sqrt(x * x + y * y + z * z);
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  sn = wave_sum(sn);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[wv][0] = sx;
    red[wv][1] = sy;
    red[wv][2] = sz;
    red[wv][3] = sn;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    partials[((int64_t)b * kMomChunks + chunk) * 4 + c] =
        ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]));
  }
}

__global__ __launch_bounds__(64) void k_momentum_final(const double* __restrict__ partials,
                                                       double* __restrict__ momentum) {
  static_assert(kMomChunks % 64 == 0, "chunks per lane");
  constexpr int kPerLane = kMomChunks / 64;
  const int b = blockIdx.x, lane = threadIdx.x;
  for (int c = 0; c < 4; ++c) {
    double v = 0.0;
    for (int q = 0; q < kPerLane; ++q)
      v += partials[((int64_t)b * kMomChunks + lane * kPerLane + q) * 4 + c];
    v = wave_sum(v);
    if (lane == 0) momentum[4 * b + c] = v;
  }
}

hipError_t launch_momentum(const DevBox* boxes, int nboxes, int64_t max_box_n, const float* acc,
                           double* partials, double* momentum, hipStream_t s) {
  (void)max_box_n;
  hipLaunchKernelGGL(k_momentum_partial, dim3(kMomChunks, nboxes), dim3(256), 0, s, boxes, acc,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_momentum_final, dim3(nboxes), dim3(64), 0, s, partials, momentum);
  return hipGetLastError();
}

}  // namespace anf
