// FP64 variant of the forward pair kernel (the "double precision" build option
// of the paper's code, as a run-time entry point).
//
// What it computes: the same near-field sum as the FP32 kernel -- Eq. 3 with
// the min hand-off, or Eq. 2 -- with every operation after the FP32 cell
// offsets in FP64: the separation (exact: an FP32 offset minus an integer
// cell shift), r^2, 1/r from the hardware estimate refined by two Newton
// steps, the force law and a plain FP64 sum per sink.  The result is the
// near field of the stored positions to FP64 rounding.
//
// How it maps to CDNA4: the FP32 kernel's work items, task queue and wave
// structure, with sources still broadcast through SGPRs, as packed records of
// the FP32 offsets widened to FP64 once per call (exact), so no pair converts
// them; MI355X issues FP64 FMAs at the FP32 (non-packed) rate, so the cost is
// the longer reciprocal square root.
#include "nf_internal.h"

namespace anf {

static __device__ __forceinline__ int uni64(int v) { return __builtin_amdgcn_readfirstlane(v); }

static __device__ __forceinline__ int wrap64(int v, int K) {
  v += v < 0 ? K : 0;
  v -= v >= K ? K : 0;
  return v;
}

// 1/sqrt(x): hardware estimate, then two Newton steps y <- y (3/2 - x y^2 / 2).
static __device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double t = (x * y) * y;
    y = y * __builtin_fma(-0.5, t, 1.5);
  }
  return y;
}

struct Const64 {
  double c0, c1, c2, g;
};

template <bool kNear>
__device__ __forceinline__ void interact64(double sx, double sy, double sz, double qx, double qy,
                                           double qz, const Const64& k, double& tx, double& ty,
                                           double& tz) {
  const double dx = sx - qx;
  const double dy = sy - qy;
  const double dz = sz - qz;
  const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, k.g)));
  const double rinv = rsqrt64(r2);
  const double rinv3 = (rinv * rinv) * rinv;
  double f = rinv3;
  if (kNear) {
    const double r = r2 * rinv;
    const double spline = __builtin_fma(__builtin_fma(k.c2, r, k.c1), r, k.c0);
    f = spline < rinv3 ? spline : rinv3;
  }
  tx = __builtin_fma(f, dx, tx);
  ty = __builtin_fma(f, dy, ty);
  tz = __builtin_fma(f, dz, tz);
}

template <bool kNear>
__device__ __forceinline__ void sum64(const double* __restrict__ src3, int beg, int end,
                                      double qx, double qy, double qz, const Const64& k,
                                      double& tx, double& ty, double& tz) {
  int j = beg;
  for (; j + 2 <= end; j += 2) {
    double c[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) c[u] = src3[3 * j + u];
    interact64<kNear>(c[0], c[1], c[2], qx, qy, qz, k, tx, ty, tz);
    interact64<kNear>(c[3], c[4], c[5], qx, qy, qz, k, tx, ty, tz);
  }
  for (; j < end; ++j)
    interact64<kNear>(src3[3 * j], src3[3 * j + 1], src3[3 * j + 2], qx, qy, qz, k, tx, ty, tz);
}

// The two far edge cells of a two-cell item walked together (the forward FP32
// kernel's scheme): per chunk of kChunk positions the wave stages both runs in
// its own LDS slot, then each lane sums its own run's records from there.
__device__ __forceinline__ void sum64_edge_runs(const double* __restrict__ src3,
                                                double* __restrict__ slot, int lane, bool upper,
                                                int bl, int nl, int bh, int nh, double qx,
                                                double qy, double qz, const Const64& k,
                                                double& tx, double& ty, double& tz) {
  const int nmax = nl > nh ? nl : nh;
  const int rn = upper ? nh : nl;
  const double* mine = slot + (upper ? 3 * kChunk : 0);
  const double* __restrict__ runl = src3 + 3 * (int64_t)bl;
  const double* __restrict__ runh = src3 + 3 * (int64_t)bh;
  for (int cb = 0; cb < nmax; cb += kChunk) {
    const int ce = cb + kChunk < nmax ? cb + kChunk : nmax;
    if (cb + lane < nl) {
#pragma unroll
      for (int c = 0; c < 3; ++c) slot[3 * lane + c] = runl[3 * (cb + lane) + c];
    }
    if (cb + lane < nh) {
#pragma unroll
      for (int c = 0; c < 3; ++c) slot[3 * kChunk + 3 * lane + c] = runh[3 * (cb + lane) + c];
    }
    __builtin_amdgcn_wave_barrier();
    const int n = (rn < ce ? rn : ce) - cb;
    for (int j = 0; j < n; ++j)
      interact64<false>(mine[3 * j], mine[3 * j + 1], mine[3 * j + 2], qx, qy, qz, k, tx, ty, tz);
    __builtin_amdgcn_wave_barrier();
  }
}

// Capped at 64 VGPRs and 80 SGPRs (no spills) for 8 resident waves per SIMD
// instead of the compiler's 7.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_pair_forward_f64(
    const DevBox* __restrict__ boxes, const int4* __restrict__ items,
    const int32_t* __restrict__ tasks, const int32_t* __restrict__ item_cost,
    int32_t* __restrict__ ctrl,
    const int32_t* __restrict__ off, const float4* __restrict__ rel,
    const double* __restrict__ src3, const int32_t* __restrict__ perm,
    double* __restrict__ acc_out, int n_static) {
  const int lane = threadIdx.x & 63;
  __shared__ double edge_lds[4][2 * kChunk * 3];  // per wave: two staged runs
  double* const edge_slot = edge_lds[threadIdx.x >> 6];
  const int n_tasks = uni64(ctrl[kCtrlNTasks]);
  bool first = true;
  while (true) {
    const int t = next_task(&ctrl[kCtrlHead], first, n_static);
    if (t >= n_tasks) break;
    const int item = uni64(tasks[t]) >> kTaskShift;
    const int4 it = items[item];
    int left = uni64(item_cost[item]);
    set_wave_priority(left);
    const int b = uni64(it.x & 0xffff), count = uni64(it.x >> 16);
    const int cx = uni64(it.y & 0xffff), cy = uni64(it.y >> 16);
    const int za = uni64(it.z & 0xffff), zb = uni64(it.z >> 16);
    const int first = uni64(it.w);
    const int K = uni64(boxes[b].K), R = uni64(boxes[b].R);
    const int cbase = uni64(boxes[b].cell_base);
    const int far_mode = uni64(boxes[b].far_mode);
    const double e = boxes[b].eps_cells64;
    Const64 kc;
    kc.c0 = 10.0 / (e * e * e);
    kc.c1 = -15.0 / (e * e * e * e);
    kc.c2 = 6.0 / (e * e * e * e * e);
    // Eq. 2: eps_p^2 added to r^2; Eq. 3: a guard that keeps 1/r^3 finite for
    // coincident points (their d = 0 makes the force 0) and is far below the
    // square of any FP32-representable separation.
    kc.g = far_mode == kFarAll ? e * e : 1e-200;
    const int pencil0 = cbase + (cx * K + cy) * K;
    const int s = lane < count ? first + lane : -1;
    int lane_z = za;
    for (int z = za; z < zb; ++z)
      if (s >= uni64(off[pencil0 + z + 1])) lane_z = z + 1;
    const bool active = s >= 0;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) p = rel[s];
    // two-cell items walk their two far edge cells together (sum64_edge_runs)
    const bool pair_edges = zb == za + 1 && R >= 2 && far_mode != kFarNone;
    const bool upper = lane_z == zb;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int ox = -R; ox <= R; ++ox) {
      const int sx = wrap64(cx + ox, K);
      const double qx = (double)p.x - (double)ox;
      for (int oy = -R; oy <= R; ++oy) {
        const int sy = wrap64(cy + oy, K);
        const double qy = (double)p.y - (double)oy;
        const int col = cbase + (sx * K + sy) * K;
        const bool col_near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
        for (int zu = za - R; zu <= zb + R; ++zu) {
          if (pair_edges && (zu == za - R || zu == zb + R)) continue;
          const int sz = wrap64(zu, K);
          const int beg = uni64(off[col + sz]), end = uni64(off[col + sz + 1]);
          if (beg == end) continue;
          left -= end - beg;
          set_wave_priority(left);
          const int oz = zu - lane_z;
          const bool near = far_mode == kFarNone ||
                            (far_mode == kFarApart && col_near && zu >= za - 1 && zu <= zb + 1);
          if (active && oz >= -R && oz <= R) {
            const double qz = (double)p.z - (double)oz;
            if (near)
              sum64<true>(src3 + 3 * (int64_t)beg, 0, end - beg, qx, qy, qz, kc, ax, ay, az);
            else
              sum64<false>(src3 + 3 * (int64_t)beg, 0, end - beg, qx, qy, qz, kc, ax, ay, az);
          }
        }
        if (pair_edges) {
          const int zl = wrap64(za - R, K), zh = wrap64(zb + R, K);
          const int bl = uni64(off[col + zl]), nl = uni64(off[col + zl + 1]) - bl;
          const int bh = uni64(off[col + zh]), nh = uni64(off[col + zh + 1]) - bh;
          if (nl + nh > 0) {
            left -= nl > nh ? nl : nh;
            set_wave_priority(left);
            // every lane takes part (each stages records); inactive lanes'
            // sums are never written
            sum64_edge_runs(src3, edge_slot, lane, upper, bl, nl, bh, nh, qx, qy,
                            (double)p.z - (double)(upper ? R : -R), kc, ax, ay, az);
          }
        }
      }
    }
    if (active) {
      const double cpl = boxes[b].cells_per_len;
      const double iw2 = cpl * cpl;
      const int64_t i = perm[s];
      acc_out[3 * i + 0] = ax * iw2;
      acc_out[3 * i + 1] = ay * iw2;
      acc_out[3 * i + 2] = az * iw2;
    }
  }
}

__global__ __launch_bounds__(256) void k_pack_sources64(const float4* __restrict__ rel, int64_t n,
                                                        double* __restrict__ src3) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float4 r = rel[s];
  src3[3 * s + 0] = r.x;
  src3[3 * s + 1] = r.y;
  src3[3 * s + 2] = r.z;
}

hipError_t launch_forward_f64(const DevBox* boxes, const PlanWork& w, const int32_t* off,
                              const float* rel, const int32_t* perm, double* acc, double* src3,
                              int64_t n_total, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_sources64, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(rel), n_total, src3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const void* fn = reinterpret_cast<const void*>(&k_pair_forward_f64);
  const int blocks = persistent_blocks(fn, 256);
  hipLaunchKernelGGL(k_pair_forward_f64, dim3(blocks), dim3(256), 0, s, boxes, w.items, w.tasks,
                     w.item_cost, w.ctrl, off, reinterpret_cast<const float4*>(rel), src3, perm, acc,
                     blocks * 4);
  return hipGetLastError();
}

}  // namespace anf
