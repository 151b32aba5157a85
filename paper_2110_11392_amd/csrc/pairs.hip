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

// One interaction: t += f(|d|) d with d = s - q (cell units).
__device__ __forceinline__ void interact(const float4 s, float qx, float qy, float qz, float c0,
                                         float c1, float c2, float& tx, float& ty, float& tz) {
  const float dx = s.x - qx;
  const float dy = s.y - qy;
  const float dz = s.z - qz;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, kTinyR2)));
  const float rinv = rsq(r2);
  const float r = r2 * rinv;
  const float spline = __builtin_fmaf(__builtin_fmaf(c2, r, c1), r, c0);
  const float rinv3 = (rinv * rinv) * rinv;
  const float f = __builtin_fminf(spline, rinv3);
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

// Sum the sources [beg, end) into (tx, ty, tz), four per step.
__device__ __forceinline__ void sum_sources(const float4* __restrict__ rel, int beg, int end,
                                            float qx, float qy, float qz, float c0, float c1,
                                            float c2, float& tx, float& ty, float& tz) {
  int j = beg;
  for (; j + 4 <= end; j += 4) {
    const float4 s0 = rel[j + 0];
    const float4 s1 = rel[j + 1];
    const float4 s2 = rel[j + 2];
    const float4 s3 = rel[j + 3];
    interact(s0, qx, qy, qz, c0, c1, c2, tx, ty, tz);
    interact(s1, qx, qy, qz, c0, c1, c2, tx, ty, tz);
    interact(s2, qx, qy, qz, c0, c1, c2, tx, ty, tz);
    interact(s3, qx, qy, qz, c0, c1, c2, tx, ty, tz);
  }
  for (; j < end; ++j) interact(rel[j], qx, qy, qz, c0, c1, c2, tx, ty, tz);
}

template <int kAcc, bool kCount>
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
    const int b = uniform(it.x);
    const int cx = uniform(it.y & 0xffff), cy = uniform(it.y >> 16);
    const int za = uniform(it.z & 0xffff), zb = uniform(it.z >> 16);
    const int tile = uniform(it.w);
    const int K = uniform(boxes[b].K), R = uniform(boxes[b].R);
    const int cbase = uniform(boxes[b].cell_base);
    const float c0 = boxes[b].c0, c1 = boxes[b].c1, c2 = boxes[b].c2;
    const int pencil0 = cbase + (cx * K + cy) * K;

    // ---- which sink this lane owns -------------------------------------
    int s = -1, lane_z = za;
    if (tile >= 0) {
      const int c = pencil0 + za;
      const int beg = uniform(off[c]) + tile * kTile, end = uniform(off[c + 1]);
      if (beg + lane < end) s = beg + lane;
    } else {
      int cum = 0;
      for (int z = za; z <= zb; ++z) {
        const int o0 = uniform(off[pencil0 + z]), o1 = uniform(off[pencil0 + z + 1]);
        const int rem = (o1 - o0) & (kTile - 1);
        if (lane >= cum && lane < cum + rem) {
          s = o1 - rem + (lane - cum);
          lane_z = z;
        }
        cum += rem;
      }
    }
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
        for (int zu = za - R; zu <= zb + R; ++zu) {
          const int sz = wrap1(zu, K);
          const int beg = uniform(off[col + sz]), end = uniform(off[col + sz + 1]);
          if (beg == end) continue;
          const int oz = zu - lane_z;
          if (active && oz >= -R && oz <= R) {
            const float qz = p.z - (float)oz;
            if (kCount) npairs += end - beg;
            if (kAcc == kAccSingle) {
              sum_sources(rel, beg, end, qx, qy, qz, c0, c1, c2, ax, ay, az);
            } else {
              for (int cb = beg; cb < end; cb += kChunk) {
                const int ce = cb + kChunk < end ? cb + kChunk : end;
                float tx = 0.f, ty = 0.f, tz = 0.f;
                sum_sources(rel, cb, ce, qx, qy, qz, c0, c1, c2, tx, ty, tz);
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

template <int kAcc, bool kCount>
static hipError_t launch_forward_t(const DevBox* boxes, const PlanWork& w, int64_t pencils,
                                   const int32_t* off, const float* rel, const int32_t* perm,
                                   float* acc, int64_t* pair_count, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_pair_forward<kAcc, kCount>);
  const int blocks = persistent_blocks(fn, 256);
  hipLaunchKernelGGL((k_pair_forward<kAcc, kCount>), dim3(blocks), dim3(256), 0, s, boxes,
                     w.items, w.queue, w.item_base + pencils, plan_head(w), off,
                     reinterpret_cast<const float4*>(rel), perm, acc,
                     reinterpret_cast<unsigned long long*>(pair_count));
  return hipGetLastError();
}

hipError_t launch_forward(AccMode mode, bool count_pairs, const DevBox* boxes, const PlanWork& w,
                          int64_t pencils, const int32_t* off, const float* rel,
                          const int32_t* perm, float* acc, int64_t* pair_count, hipStream_t s) {
  if (count_pairs) {
    switch (mode) {
      case kAccSingle: return launch_forward_t<kAccSingle, true>(boxes, w, pencils, off, rel, perm, acc, pair_count, s);
      case kAccChunked: return launch_forward_t<kAccChunked, true>(boxes, w, pencils, off, rel, perm, acc, pair_count, s);
      default: return launch_forward_t<kAccCompensated, true>(boxes, w, pencils, off, rel, perm, acc, pair_count, s);
    }
  }
  switch (mode) {
    case kAccSingle: return launch_forward_t<kAccSingle, false>(boxes, w, pencils, off, rel, perm, acc, nullptr, s);
    case kAccChunked: return launch_forward_t<kAccChunked, false>(boxes, w, pencils, off, rel, perm, acc, nullptr, s);
    default: return launch_forward_t<kAccCompensated, false>(boxes, w, pencils, off, rel, perm, acc, nullptr, s);
  }
}

}  // namespace anf
