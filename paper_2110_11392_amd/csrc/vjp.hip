// Adjoint (vector-Jacobian product) of the near-field accelerations.
//
// With F(d) = f(r) d (Eq. 3) the Jacobian of one pair is H(d) = f I + h d d^T,
// h = f'(r)/r, symmetric and even in d.  For L = sum_i w_i . a_i and the
// binning held fixed, dL/dx_k = sum_{j in NF(k)} H(d_kj) (w_j - w_k), because
// the near-field relation is symmetric.  In cell units (d in cell widths):
//   r >= eps:  f = r^-3,                 h = -3 r^-5
//   r <  eps:  f = c0 + c1 r + c2 r^2,   h = ha + hb / r   (ha = 12/eps^5, hb = -15/eps^4)
// and the box-unit gradient is the cell-unit sum times 1/w^3.
//
// Same traversal and work items as the forward kernel; each source carries
// (position, cotangent) as two float4s that one wave-uniform 32-byte scalar
// load brings into SGPRs.
#include "nf_internal.h"

namespace anf {

__device__ __forceinline__ float rsq_v(float x) { return __builtin_amdgcn_rsqf(x); }

// kNear: the pair may lie inside eps (select between spline and Newton); else
// every pair of the source cell has r > eps and the Newton branch is exact.
template <bool kNear>
__device__ __forceinline__ void adjoint(const float4 s, const float4 ws, float qx, float qy,
                                        float qz, float wx, float wy, float wz, float c0, float c1,
                                        float c2, float ha, float hb, float eps, float& gx,
                                        float& gy, float& gz) {
  const float dx = s.x - qx;
  const float dy = s.y - qy;
  const float dz = s.z - qz;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, kTinyR2)));
  const float rinv = rsq_v(r2);
  const float rinv2 = rinv * rinv;
  const float rinv3 = rinv2 * rinv;
  float f = rinv3;
  float h = (-3.0f * rinv2) * rinv3;
  if (kNear) {
    const float r = r2 * rinv;
    const bool inner = r < eps;
    f = inner ? __builtin_fmaf(__builtin_fmaf(c2, r, c1), r, c0) : rinv3;
    h = inner ? __builtin_fmaf(hb, rinv, ha) : h;
  }
  const float vx = ws.x - wx;
  const float vy = ws.y - wy;
  const float vz = ws.z - wz;
  const float dv = __builtin_fmaf(dz, vz, __builtin_fmaf(dy, vy, dx * vx));
  const float k = h * dv;
  gx = __builtin_fmaf(k, dx, __builtin_fmaf(f, vx, gx));
  gy = __builtin_fmaf(k, dy, __builtin_fmaf(f, vy, gy));
  gz = __builtin_fmaf(k, dz, __builtin_fmaf(f, vz, gz));
}

__device__ __forceinline__ void two_sum_fold_v(float& a, float& e, float t) {
  const float s = a + t;
  const float bp = s - a;
  const float ap = s - bp;
  e += (a - ap) + (t - bp);
  a = s;
}

__device__ __forceinline__ int wrap1_v(int v, int K) {
  v += v < 0 ? K : 0;
  v -= v >= K ? K : 0;
  return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

struct AdjConst {
  float c0, c1, c2, ha, hb, eps;
};

template <int kU, bool kPipe, bool kNear>
__device__ __forceinline__ void sum_adjoint(const float4* __restrict__ src, int beg, int end,
                                            float qx, float qy, float qz, float wx, float wy,
                                            float wz, const AdjConst& k, float& gx, float& gy,
                                            float& gz) {
  int j = beg;
  if (kPipe && j + kU <= end) {
    float4 cs[kU], cw[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) { cs[u] = src[2 * (j + u)]; cw[u] = src[2 * (j + u) + 1]; }
    for (; j + 2 * kU <= end; j += kU) {
      float4 ns[kU], nw[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) { ns[u] = src[2 * (j + kU + u)]; nw[u] = src[2 * (j + kU + u) + 1]; }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        adjoint<kNear>(cs[u], cw[u], qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, gx, gy, gz);
#pragma unroll
      for (int u = 0; u < kU; ++u) { cs[u] = ns[u]; cw[u] = nw[u]; }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      adjoint<kNear>(cs[u], cw[u], qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, gx, gy, gz);
    j += kU;
  }
  for (; j + kU <= end; j += kU) {
    float4 cs[kU], cw[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) { cs[u] = src[2 * (j + u)]; cw[u] = src[2 * (j + u) + 1]; }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      adjoint<kNear>(cs[u], cw[u], qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, gx, gy, gz);
  }
  for (; j < end; ++j)
    adjoint<kNear>(src[2 * j], src[2 * j + 1], qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb,
            k.eps, gx, gy, gz);
}

// Interleave (rel_s, w_perm[s]) per sorted slot.
__global__ __launch_bounds__(256) void k_gather_src(const float4* __restrict__ rel,
                                                    const int32_t* __restrict__ perm,
                                                    const float* __restrict__ w, int64_t n,
                                                    float4* __restrict__ src) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t i = perm[s];
  src[2 * s] = rel[s];
  src[2 * s + 1] = make_float4(w[3 * i + 0], w[3 * i + 1], w[3 * i + 2], 0.0f);
}

template <int kAcc, int kU, bool kPipe>
__global__ __launch_bounds__(256) void k_pair_vjp(
    const DevBox* __restrict__ boxes, const int4* __restrict__ items,
    const int32_t* __restrict__ queue, const int32_t* __restrict__ n_items_ptr,
    int32_t* __restrict__ head, const int32_t* __restrict__ off, const float4* __restrict__ src,
    const int32_t* __restrict__ perm, float* __restrict__ grad) {
  const int lane = threadIdx.x & 63;
  const int n_items = uni(*n_items_ptr);
  while (true) {
    // Every lane takes part in the atomic (lane 0 adds 1, the others 0) so no
    // divergent branch precedes the wave-uniform exit test below.
    int q = atomicAdd(head, lane == 0 ? 1 : 0);
    q = uni(__shfl(q, 0, 64));
    if (q >= n_items) break;
    const int4 it = items[uni(queue[q])];
    const int b = uni(it.x & 0xffff), count = uni(it.x >> 16);
    const int cx = uni(it.y & 0xffff), cy = uni(it.y >> 16);
    const int za = uni(it.z & 0xffff), zb = uni(it.z >> 16);
    const int first = uni(it.w);
    const int K = uni(boxes[b].K), R = uni(boxes[b].R);
    const int cbase = uni(boxes[b].cell_base);
    AdjConst kc;
    kc.c0 = boxes[b].c0; kc.c1 = boxes[b].c1; kc.c2 = boxes[b].c2;
    kc.ha = boxes[b].ha; kc.hb = boxes[b].hb; kc.eps = boxes[b].eps;
    // c1 and ha each meet another SGPR operand in an FMA; a VALU instruction
    // reads at most one SGPR, so keep them in VGPRs for the whole item.
    asm volatile("" : "+v"(kc.c1), "+v"(kc.ha));
    const int pencil0 = cbase + (cx * K + cy) * K;
    const bool far_ok = uni(boxes[b].far_newton) != 0;

    // lane -> sink: the item's sinks are the contiguous slots [first, first+count)
    const int s = lane < count ? first + lane : -1;
    int lane_z = za;
    for (int z = za; z < zb; ++z)
      if (s >= uni(off[pencil0 + z + 1])) lane_z = z + 1;
    const bool active = s >= 0;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), wk = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) {
      p = src[2 * s];
      wk = src[2 * s + 1];
    }

    float gx = 0.f, gy = 0.f, gz = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
    for (int ox = -R; ox <= R; ++ox) {
      const int sx = wrap1_v(cx + ox, K);
      const float qx = p.x - (float)ox;
      for (int oy = -R; oy <= R; ++oy) {
        const int sy = wrap1_v(cy + oy, K);
        const float qy = p.y - (float)oy;
        const int col = cbase + (sx * K + sy) * K;
        const bool col_near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
        for (int zu = za - R; zu <= zb + R; ++zu) {
          const int sz = wrap1_v(zu, K);
          const int beg = uni(off[col + sz]), end = uni(off[col + sz + 1]);
          if (beg == end) continue;
          const int oz = zu - lane_z;
          const bool near = !far_ok || (col_near && zu >= za - 1 && zu <= zb + 1);
          if (active && oz >= -R && oz <= R) {
            const float qz = p.z - (float)oz;
            if (kAcc == kAccSingle) {
              if (near)
                sum_adjoint<kU, kPipe, true>(src, beg, end, qx, qy, qz, wk.x, wk.y, wk.z, kc, gx,
                                             gy, gz);
              else
                sum_adjoint<kU, kPipe, false>(src, beg, end, qx, qy, qz, wk.x, wk.y, wk.z, kc, gx,
                                              gy, gz);
            } else {
              for (int cb = beg; cb < end; cb += kChunk) {
                const int ce = cb + kChunk < end ? cb + kChunk : end;
                float tx = 0.f, ty = 0.f, tz = 0.f;
                if (near)
                  sum_adjoint<kU, kPipe, true>(src, cb, ce, qx, qy, qz, wk.x, wk.y, wk.z, kc, tx,
                                               ty, tz);
                else
                  sum_adjoint<kU, kPipe, false>(src, cb, ce, qx, qy, qz, wk.x, wk.y, wk.z, kc, tx,
                                                ty, tz);
                if (kAcc == kAccChunked) {
                  gx += tx; gy += ty; gz += tz;
                } else {
                  two_sum_fold_v(gx, ex, tx);
                  two_sum_fold_v(gy, ey, ty);
                  two_sum_fold_v(gz, ez, tz);
                }
              }
            }
          }
        }
      }
    }
    if (active) {
      const float iw3 = boxes[b].inv_w3;
      const int64_t i = perm[s];
      grad[3 * i + 0] = (gx + ex) * iw3;
      grad[3 * i + 1] = (gy + ey) * iw3;
      grad[3 * i + 2] = (gz + ez) * iw3;
    }
  }
}

template <int kAcc, int kU, bool kPipe>
static hipError_t launch_vjp_t(const DevBox* boxes, const PlanWork& w, int64_t pencils,
                               const int32_t* off, const float4* src, const int32_t* perm,
                               float* grad, int grid_mult, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_pair_vjp<kAcc, kU, kPipe>);
  const int blocks = persistent_blocks(fn, 256) * grid_mult;
  hipLaunchKernelGGL((k_pair_vjp<kAcc, kU, kPipe>), dim3(blocks), dim3(256), 0, s, boxes, w.items,
                     w.queue, w.item_base + pencils, plan_head(w), off, src, perm, grad);
  return hipGetLastError();
}

template <int kAcc>
static hipError_t dispatch_vjp(const KernelConfig& cfg, const DevBox* boxes, const PlanWork& w,
                               int64_t pencils, const int32_t* off, const float4* src,
                               const int32_t* perm, float* grad, hipStream_t s) {
  const int g = cfg.grid_mult;
  switch (cfg.unroll * 2 + (cfg.pipeline ? 1 : 0)) {
    case 5: return launch_vjp_t<kAcc, 2, true>(boxes, w, pencils, off, src, perm, grad, g, s);
    case 8: return launch_vjp_t<kAcc, 4, false>(boxes, w, pencils, off, src, perm, grad, g, s);
    case 9: return launch_vjp_t<kAcc, 4, true>(boxes, w, pencils, off, src, perm, grad, g, s);
    default: return launch_vjp_t<kAcc, 2, false>(boxes, w, pencils, off, src, perm, grad, g, s);
  }
}

hipError_t launch_vjp(AccMode mode, const KernelConfig& cfg, const DevBox* boxes,
                      const PlanWork& w, int64_t pencils, const int32_t* off, const float* rel,
                      const int32_t* perm, const float* wvec, float4* src_w, int64_t n_total,
                      float* grad, hipStream_t s) {
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_src, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(rel), perm, wvec, n_total, src_w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (mode) {
    case kAccSingle: return dispatch_vjp<kAccSingle>(cfg, boxes, w, pencils, off, src_w, perm, grad, s);
    case kAccChunked: return dispatch_vjp<kAccChunked>(cfg, boxes, w, pencils, off, src_w, perm, grad, s);
    default: return dispatch_vjp<kAccCompensated>(cfg, boxes, w, pencils, off, src_w, perm, grad, s);
  }
}

}  // namespace anf
