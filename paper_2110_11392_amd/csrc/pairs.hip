// Forward near-field pair kernel (the hot loop).
//
// What it computes (Sec. 3.4.1, Eq. 3): for every sink i, the sum over every
// source j != i in the (2R+1)^3 cells around i's cell of f(r) d, d = x_j - x_i,
// f = min(spline(r), 1/r^3) -- the branch-free hand-off of Sec. 3.4.4; the
// minimum selects the spline exactly when r < eps_s because
// u^3 (10 - 15u + 6u^2) increases monotonically and equals 1 at u = 1.
//
// How it maps to CDNA4:
//   * one work item = 64 sinks, one per lane, held in VGPRs for the whole item;
//   * the item is processed by a single wavefront that walks the (2R+1)^2 source
//     columns and the z-range of source cells; a source cell's particles are a
//     contiguous slice of the cell-sorted arrays, read at wave-uniform addresses
//     so they arrive through the scalar cache into SGPRs and feed every lane's
//     VALU instruction directly -- every lane sees the same source at the same
//     time, so no LDS staging, barrier or broadcast read is needed;
//   * the periodic wrap never reaches the arithmetic: a source cell's integer
//     offset o from the sink's cell is folded into the sink (q = p - o) once per
//     source cell, and d = s - q uses only FP32 cell-relative coordinates;
//   * sums are per-lane registers; a persistent grid pops items from a
//     longest-first queue with one atomic per item.
#include "nf_internal.h"

namespace anf {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// One interaction: t += f(|d|) d with d = s - q (cell units).  kNear: the pair
// may lie inside the softening length, so f = min(spline(r), 1/r^3); otherwise
// the source cell is so far from every sink that r > eps for all its pairs and
// f = 1/r^3 -- exactly the value the minimum would select.
template <bool kNear>
__device__ __forceinline__ void interact(const float4 s, float qx, float qy, float qz, float c0,
                                         float c1, float c2, float& tx, float& ty, float& tz) {
  const float dx = s.x - qx;
  const float dy = s.y - qy;
  const float dz = s.z - qz;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, kTinyR2)));
  const float rinv = rsq(r2);
  const float rinv3 = (rinv * rinv) * rinv;
  float f = rinv3;
  if (kNear) {
    const float r = r2 * rinv;
    const float spline = __builtin_fmaf(__builtin_fmaf(c2, r, c1), r, c0);
    f = __builtin_fminf(spline, rinv3);
  }
  tx = __builtin_fmaf(f, dx, tx);
  ty = __builtin_fmaf(f, dy, ty);
  tz = __builtin_fmaf(f, dz, tz);
}

// Error-free TwoSum of (a, t): a <- fl(a + t), e accumulates the rounding error.
__device__ __forceinline__ void two_sum_fold(float& a, float& e, float t) {
  const float s = a + t;
  const float bp = s - a;
  const float ap = s - bp;
  e += (a - ap) + (t - bp);
  a = s;
}

__device__ __forceinline__ int wrap1(int v, int K) {
  v += v < 0 ? K : 0;
  v -= v >= K ? K : 0;
  return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum the sources [beg, end) into (tx, ty, tz), kU per step.  With kPipe the
// next kU sources are requested before the current ones are used, so the
// scalar-cache latency of one group overlaps the arithmetic of the previous.
template <int kU, bool kPipe, bool kNear>
__device__ __forceinline__ void sum_sources(const float4* __restrict__ rel, int beg, int end,
                                            float qx, float qy, float qz, float c0, float c1,
                                            float c2, float& tx, float& ty, float& tz) {
  int j = beg;
  if (kPipe && j + kU <= end) {
    float4 cur[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) cur[u] = rel[j + u];
    for (; j + 2 * kU <= end; j += kU) {
      float4 nxt[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) nxt[u] = rel[j + kU + u];
#pragma unroll
      for (int u = 0; u < kU; ++u) interact<kNear>(cur[u], qx, qy, qz, c0, c1, c2, tx, ty, tz);
#pragma unroll
      for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) interact<kNear>(cur[u], qx, qy, qz, c0, c1, c2, tx, ty, tz);
    j += kU;
  }
  for (; j + kU <= end; j += kU) {
    float4 cur[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) cur[u] = rel[j + u];
#pragma unroll
    for (int u = 0; u < kU; ++u) interact<kNear>(cur[u], qx, qy, qz, c0, c1, c2, tx, ty, tz);
  }
  for (; j < end; ++j) interact<kNear>(rel[j], qx, qy, qz, c0, c1, c2, tx, ty, tz);
}

template <int kAcc, bool kCount, int kU, bool kPipe>
__global__ __launch_bounds__(256) void k_pair_forward(
    const DevBox* __restrict__ boxes, const int4* __restrict__ items,
    const int32_t* __restrict__ queue, const int32_t* __restrict__ n_items_ptr,
    int32_t* __restrict__ head, const int32_t* __restrict__ off, const float4* __restrict__ rel,
    const int32_t* __restrict__ perm, float* __restrict__ acc_out,
    unsigned long long* __restrict__ pair_count) {
  const int lane = threadIdx.x & 63;
  const int n_items = uniform(*n_items_ptr);
  while (true) {
    // Every lane takes part in the atomic (lane 0 adds 1, the others 0) so no
    // divergent branch precedes the wave-uniform exit test below.
    int q = atomicAdd(head, lane == 0 ? 1 : 0);
    q = uniform(__shfl(q, 0, 64));
    if (q >= n_items) break;
    const int4 it = items[uniform(queue[q])];
    const int b = uniform(it.x & 0xffff), count = uniform(it.x >> 16);
    const int cx = uniform(it.y & 0xffff), cy = uniform(it.y >> 16);
    const int za = uniform(it.z & 0xffff), zb = uniform(it.z >> 16);
    const int first = uniform(it.w);
    const int K = uniform(boxes[b].K), R = uniform(boxes[b].R);
    const int cbase = uniform(boxes[b].cell_base);
    const float c0 = boxes[b].c0, c2 = boxes[b].c2;
    // c1 meets an SGPR operand (c2) in the spline FMA; a VALU instruction reads
    // at most one SGPR, so keep c1 in a VGPR for the whole item.
    float c1 = boxes[b].c1;
    asm volatile("" : "+v"(c1));
    const int pencil0 = cbase + (cx * K + cy) * K;
    // Cells two or more apart on some axis are >= 1 cell width apart, so with
    // eps < 1/2 cell every pair in them is Newtonian (f = 1/r^3).
    const bool far_ok = uniform(boxes[b].far_newton) != 0;

    // ---- which sink this lane owns -------------------------------------
    // lane -> sink: the item's sinks are the contiguous slots [first, first+count)
    const int s = lane < count ? first + lane : -1;
    int lane_z = za;
    for (int z = za; z < zb; ++z)
      if (s >= uniform(off[pencil0 + z + 1])) lane_z = z + 1;
    const bool active = s >= 0;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) p = rel[s];

    float ax = 0.f, ay = 0.f, az = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
    long long npairs = 0;
    for (int ox = -R; ox <= R; ++ox) {
      const int sx = wrap1(cx + ox, K);
      const float qx = p.x - (float)ox;
      for (int oy = -R; oy <= R; ++oy) {
        const int sy = wrap1(cy + oy, K);
        const float qy = p.y - (float)oy;
        const int col = cbase + (sx * K + sy) * K;
        const bool col_near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
        for (int zu = za - R; zu <= zb + R; ++zu) {
          const int sz = wrap1(zu, K);
          const int beg = uniform(off[col + sz]), end = uniform(off[col + sz + 1]);
          if (beg == end) continue;
          const int oz = zu - lane_z;
          // Wave-uniform: can any pair of this source cell fall inside eps?
          const bool near = !far_ok || (col_near && zu >= za - 1 && zu <= zb + 1);
          if (active && oz >= -R && oz <= R) {
            const float qz = p.z - (float)oz;
            if (kCount) npairs += end - beg;
            if (kAcc == kAccSingle) {
              if (near)
                sum_sources<kU, kPipe, true>(rel, beg, end, qx, qy, qz, c0, c1, c2, ax, ay, az);
              else
                sum_sources<kU, kPipe, false>(rel, beg, end, qx, qy, qz, c0, c1, c2, ax, ay, az);
            } else {
              for (int cb = beg; cb < end; cb += kChunk) {
                const int ce = cb + kChunk < end ? cb + kChunk : end;
                float tx = 0.f, ty = 0.f, tz = 0.f;
                if (near)
                  sum_sources<kU, kPipe, true>(rel, cb, ce, qx, qy, qz, c0, c1, c2, tx, ty, tz);
                else
                  sum_sources<kU, kPipe, false>(rel, cb, ce, qx, qy, qz, c0, c1, c2, tx, ty, tz);
                if (kAcc == kAccChunked) {
                  ax += tx; ay += ty; az += tz;
                } else {
                  two_sum_fold(ax, ex, tx);
                  two_sum_fold(ay, ey, ty);
                  two_sum_fold(az, ez, tz);
                }
              }
            }
          }
        }
      }
    }
    if (active) {
      const float iw2 = boxes[b].inv_w2;
      const int64_t i = perm[s];
      acc_out[3 * i + 0] = (ax + ex) * iw2;
      acc_out[3 * i + 1] = (ay + ey) * iw2;
      acc_out[3 * i + 2] = (az + ez) * iw2;
    }
    if (kCount) {
      if (active) npairs -= 1;  // the sink itself sits in its own cell
      for (int d = 32; d >= 1; d >>= 1) npairs += __shfl_xor(npairs, d, 64);
      if (lane == 0) atomicAdd(pair_count, (unsigned long long)npairs);
    }
  }
}

template <int kAcc, bool kCount, int kU, bool kPipe>
static hipError_t launch_forward_t(const DevBox* boxes, const PlanWork& w, int64_t pencils,
                                   const int32_t* off, const float* rel, const int32_t* perm,
                                   float* acc, int64_t* pair_count, int grid_mult, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_pair_forward<kAcc, kCount, kU, kPipe>);
  const int blocks = persistent_blocks(fn, 256) * grid_mult;
  hipLaunchKernelGGL((k_pair_forward<kAcc, kCount, kU, kPipe>), dim3(blocks), dim3(256), 0, s,
                     boxes, w.items, w.queue, w.item_base + pencils, plan_head(w), off,
                     reinterpret_cast<const float4*>(rel), perm, acc,
                     reinterpret_cast<unsigned long long*>(pair_count));
  return hipGetLastError();
}

template <int kAcc, bool kCount>
static hipError_t dispatch_variant(const KernelConfig& cfg, const DevBox* boxes, const PlanWork& w,
                                   int64_t pencils, const int32_t* off, const float* rel,
                                   const int32_t* perm, float* acc, int64_t* pc, hipStream_t s) {
  const int g = cfg.grid_mult;
  switch (cfg.unroll * 2 + (cfg.pipeline ? 1 : 0)) {
    case 4: return launch_forward_t<kAcc, kCount, 2, false>(boxes, w, pencils, off, rel, perm, acc, pc, g, s);
    case 5: return launch_forward_t<kAcc, kCount, 2, true>(boxes, w, pencils, off, rel, perm, acc, pc, g, s);
    case 9: return launch_forward_t<kAcc, kCount, 4, true>(boxes, w, pencils, off, rel, perm, acc, pc, g, s);
    case 16: return launch_forward_t<kAcc, kCount, 8, false>(boxes, w, pencils, off, rel, perm, acc, pc, g, s);
    case 17: return launch_forward_t<kAcc, kCount, 8, true>(boxes, w, pencils, off, rel, perm, acc, pc, g, s);
    default: return launch_forward_t<kAcc, kCount, 4, false>(boxes, w, pencils, off, rel, perm, acc, pc, g, s);
  }
}

hipError_t launch_forward(AccMode mode, bool count_pairs, const KernelConfig& cfg,
                          const DevBox* boxes, const PlanWork& w, int64_t pencils,
                          const int32_t* off, const float* rel, const int32_t* perm, float* acc,
                          int64_t* pair_count, hipStream_t s) {
  if (count_pairs) {
    // The debug counter is a correctness tool: one fixed variant per mode.
    const KernelConfig base = default_config(0);
    switch (mode) {
      case kAccSingle: return dispatch_variant<kAccSingle, true>(base, boxes, w, pencils, off, rel, perm, acc, pair_count, s);
      case kAccChunked: return dispatch_variant<kAccChunked, true>(base, boxes, w, pencils, off, rel, perm, acc, pair_count, s);
      default: return dispatch_variant<kAccCompensated, true>(base, boxes, w, pencils, off, rel, perm, acc, pair_count, s);
    }
  }
  switch (mode) {
    case kAccSingle: return dispatch_variant<kAccSingle, false>(cfg, boxes, w, pencils, off, rel, perm, acc, nullptr, s);
    case kAccChunked: return dispatch_variant<kAccChunked, false>(cfg, boxes, w, pencils, off, rel, perm, acc, nullptr, s);
    default: return dispatch_variant<kAccCompensated, false>(cfg, boxes, w, pencils, off, rel, perm, acc, nullptr, s);
  }
}

}  // namespace anf
