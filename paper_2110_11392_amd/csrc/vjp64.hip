// FP64 variant of the adjoint pair kernel, the companion of the FP64 forward
// kernel (the "double precision" build option of the paper's code, as a
// run-time entry point).
//
// What it computes: the same vector-Jacobian product as the FP32 adjoint,
//   g_k = sum_{j in NF(k)} [ f(r) (w_j - w_k) + h(r) (d . (w_j - w_k)) d ],
//   h = f'(r)/r, d = x_j - x_k, binning held fixed,
// with f from Eq. 3 (spline inside eps_s, r^-3 outside) or Eq. 2, and every
// operation after the stored FP32 cell offsets in FP64: the separation (an
// FP32 offset minus an integer cell shift, exact), r^2, 1/r from the hardware
// estimate refined by two Newton steps, the pair term written as
// F (v + T d) with F = f and T = h (d.v) / f, and a plain FP64 sum per sink.
// The cotangent is FP64.
//
// How it maps to CDNA4: the FP32 kernels' work items and persistent task
// queue (whole items only), one sink per lane; a source is its FP32 offsets
// (the binned float4) and its FP64 cotangent in sorted order, both read at
// wave-uniform addresses.  MI355X issues FP64 FMAs at the FP32 (non-packed)
// rate, so the longer reciprocal square root and the division inside eps_s
// are the extra cost.
#include "nf_internal.h"

namespace anf {

static __device__ __forceinline__ int uni_v64(int v) { return __builtin_amdgcn_readfirstlane(v); }

static __device__ __forceinline__ int wrap_v64(int v, int K) {
  v += v < 0 ? K : 0;
  v -= v >= K ? K : 0;
  return v;
}

// 1/sqrt(x): hardware estimate, then two Newton steps y <- y (3/2 - x y^2 / 2).
static __device__ __forceinline__ double rsqrt_v64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double t = (x * y) * y;
    y = y * __builtin_fma(-0.5, t, 1.5);
  }
  return y;
}

struct AdjConst64 {
  double c0, c1, c2;  // f(r) = c0 + c1 r + c2 r^2 inside eps (cell units)
  double ha, hb;      // h(r) = ha + hb / r inside eps
  double eps, g;      // eps in cell units; the guard added to r^2
};

// One pair: source offsets (sx, sy, sz) and cotangent (ux, uy, uz) against
// the sink at (qx, qy, qz) (shifted by the source cell's offset) with
// cotangent (wx, wy, wz).  kNear: the pair may lie inside eps.
template <bool kNear>
__device__ __forceinline__ void adjoint64(float sx, float sy, float sz, double ux, double uy,
                                          double uz, double qx, double qy, double qz, double wx,
                                          double wy, double wz, const AdjConst64& k, double& gx,
                                          double& gy, double& gz) {
  const double dx = (double)sx - qx;
  const double dy = (double)sy - qy;
  const double dz = (double)sz - qz;
  const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, k.g)));
  const double rinv = rsqrt_v64(r2);
  const double rinv2 = rinv * rinv;
  const double vx = ux - wx;
  const double vy = uy - wy;
  const double vz = uz - wz;
  const double dv = __builtin_fma(dz, vz, __builtin_fma(dy, vy, dx * vx));
  double F = rinv2 * rinv;
  double T = (-3.0 * rinv2) * dv;
  if (kNear) {
    const double r = r2 * rinv;
    if (r < k.eps) {
      const double fs = __builtin_fma(__builtin_fma(k.c2, r, k.c1), r, k.c0);
      const double hs = __builtin_fma(k.hb, rinv, k.ha);
      F = fs;
      T = (hs * dv) / fs;
    }
  }
  gx = __builtin_fma(F, __builtin_fma(T, dx, vx), gx);
  gy = __builtin_fma(F, __builtin_fma(T, dy, vy), gy);
  gz = __builtin_fma(F, __builtin_fma(T, dz, vz), gz);
}

template <bool kNear>
__device__ __forceinline__ void sum_adjoint64(const float4* __restrict__ rel,
                                              const double* __restrict__ w64, int beg, int end,
                                              double qx, double qy, double qz, double wx,
                                              double wy, double wz, const AdjConst64& k,
                                              double& gx, double& gy, double& gz) {
  for (int j = beg; j < end; ++j) {
    const float4 s = rel[j];
    const double* u = w64 + 3 * (int64_t)j;
    adjoint64<kNear>(s.x, s.y, s.z, u[0], u[1], u[2], qx, qy, qz, wx, wy, wz, k, gx, gy, gz);
  }
}

// The cotangent in sorted order: w64[3 s + c] = w[3 perm[s] + c].
__global__ __launch_bounds__(256) void k_gather_w64(const int32_t* __restrict__ perm,
                                                    const double* __restrict__ w, int64_t n,
                                                    double* __restrict__ w64) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t i = perm[s];
  w64[3 * s + 0] = w[3 * i + 0];
  w64[3 * s + 1] = w[3 * i + 1];
  w64[3 * s + 2] = w[3 * i + 2];
}

__global__ __launch_bounds__(256) void k_pair_vjp_f64(
    const DevBox* __restrict__ boxes, const int4* __restrict__ items,
    const int32_t* __restrict__ tasks, const int32_t* __restrict__ item_cost,
    int32_t* __restrict__ ctrl, const int32_t* __restrict__ off, const float4* __restrict__ rel,
    const double* __restrict__ w64, const int32_t* __restrict__ perm,
    double* __restrict__ grad, int n_static) {
  const int lane = threadIdx.x & 63;
  const int n_tasks = uni_v64(ctrl[kCtrlNTasks]);
  bool first = true;
  while (true) {
    const int t = next_task(&ctrl[kCtrlHead], first, n_static);
    if (t >= n_tasks) break;
    const int item = uni_v64(tasks[t]) >> kTaskShift;
    const int4 it = items[item];
    int left = uni_v64(item_cost[item]);
    set_wave_priority(left);
    const int b = uni_v64(it.x & 0xffff), count = uni_v64(it.x >> 16);
    const int cx = uni_v64(it.y & 0xffff), cy = uni_v64(it.y >> 16);
    const int za = uni_v64(it.z & 0xffff), zb = uni_v64(it.z >> 16);
    const int first_sink = uni_v64(it.w);
    const int K = uni_v64(boxes[b].K), R = uni_v64(boxes[b].R);
    const int cbase = uni_v64(boxes[b].cell_base);
    const int far_mode = uni_v64(boxes[b].far_mode);
    const double e = boxes[b].eps_cells64;
    AdjConst64 kc;
    kc.c0 = 10.0 / (e * e * e);
    kc.c1 = -15.0 / (e * e * e * e);
    kc.c2 = 6.0 / (e * e * e * e * e);
    kc.ha = 2.0 * kc.c2;  // h = f'(r)/r = c1 / r + 2 c2
    kc.hb = kc.c1;
    kc.eps = e;
    // Eq. 2: eps_p^2 added to r^2 (the Newton expressions are then exact);
    // Eq. 3: a guard that keeps 1/r^3 finite for coincident points (their
    // d = 0 and v . d = 0 make the term f (w_j - w_k), which is 0 for the
    // sink itself) and is far below the square of any FP32 separation.
    kc.g = far_mode == kFarAll ? e * e : 1e-200;
    const int pencil0 = cbase + (cx * K + cy) * K;
    const int s = lane < count ? first_sink + lane : -1;
    int lane_z = za;
    for (int z = za; z < zb; ++z)
      if (s >= uni_v64(off[pencil0 + z + 1])) lane_z = z + 1;
    const bool active = s >= 0;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    double wx = 0.0, wy = 0.0, wz = 0.0;
    if (active) {
      p = rel[s];
      wx = w64[3 * (int64_t)s + 0];
      wy = w64[3 * (int64_t)s + 1];
      wz = w64[3 * (int64_t)s + 2];
    }
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int ox = -R; ox <= R; ++ox) {
      const int sx = wrap_v64(cx + ox, K);
      const double qx = (double)p.x - (double)ox;
      for (int oy = -R; oy <= R; ++oy) {
        const int sy = wrap_v64(cy + oy, K);
        const double qy = (double)p.y - (double)oy;
        const int col = cbase + (sx * K + sy) * K;
        const bool col_near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
        for (int zu = za - R; zu <= zb + R; ++zu) {
          const int sz = wrap_v64(zu, K);
          const int beg = uni_v64(off[col + sz]), end = uni_v64(off[col + sz + 1]);
          if (beg == end) continue;
          left -= end - beg;
          set_wave_priority(left);
          const int oz = zu - lane_z;  // lanes accept source cells within +-R of their own
          const bool near = far_mode == kFarNone ||
                            (far_mode == kFarApart && col_near && zu >= za - 1 && zu <= zb + 1);
          if (active && oz >= -R && oz <= R) {
            const double qz = (double)p.z - (double)oz;
            if (near)
              sum_adjoint64<true>(rel, w64, beg, end, qx, qy, qz, wx, wy, wz, kc, gx, gy, gz);
            else
              sum_adjoint64<false>(rel, w64, beg, end, qx, qy, qz, wx, wy, wz, kc, gx, gy, gz);
          }
        }
      }
    }
    if (active) {
      const double cpl = boxes[b].cells_per_len;
      const double iw3 = cpl * cpl * cpl;
      const int64_t i = perm[s];
      grad[3 * i + 0] = gx * iw3;
      grad[3 * i + 1] = gy * iw3;
      grad[3 * i + 2] = gz * iw3;
    }
  }
}

hipError_t launch_vjp_f64(const DevBox* boxes, const PlanWork& w, const int32_t* off,
                          const float* rel, const int32_t* perm, const double* wvec,
                          double* w64, int64_t n_total, double* grad, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_w64, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s,
                     perm, wvec, n_total, w64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const void* fn = reinterpret_cast<const void*>(&k_pair_vjp_f64);
  const int blocks = persistent_blocks(fn, 256);
  hipLaunchKernelGGL(k_pair_vjp_f64, dim3(blocks), dim3(256), 0, s, boxes, w.items, w.tasks,
                     w.item_cost, w.ctrl, off, reinterpret_cast<const float4*>(rel), w64, perm,
                     grad, blocks * 4);
  return hipGetLastError();
}

}  // namespace anf
