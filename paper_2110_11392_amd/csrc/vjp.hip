// Adjoint (vector-Jacobian product) of the near-field accelerations.
//
// With F(d) = f(r) d (Eq. 3, or Eq. 2) the Jacobian of one pair is H(d) = f I + h d d^T,
// h = f'(r)/r, symmetric and even in d.  For L = sum_i w_i . a_i and the
// binning held fixed, dL/dx_k = sum_{j in NF(k)} H(d_kj) (w_j - w_k), because
// the near-field relation is symmetric.  In cell units (d in cell widths):
//   r >= eps:  f = r^-3,                 h = -3 r^-5
//   r <  eps:  f = c0 + c1 r + c2 r^2,   h = ha + hb / r   (ha = 12/eps^5, hb = -15/eps^4)
// and for Eq. 2 f = s^-3/2, h = -3 s^-5/2 with s = r^2 + eps_p^2 -- the Newton
// expressions with eps_p^2 as the guard added to r^2.  The box-unit gradient is
// the cell-unit sum times 1/w^3.
//
// Same traversal and work items as the forward kernel; each source carries
// (position, cotangent) as a packed 24-byte record that wave-uniform scalar
// loads bring into SGPRs (and, for the paired edge cells of two-cell items,
// the wave's LDS slot).
#include "nf_internal.h"

namespace anf {

__device__ __forceinline__ float rsq_v(float x) { return __builtin_amdgcn_rsqf(x); }

// One adjoint interaction with the source record s = (x, y, z, w_x, w_y, w_z).
// The pair term f v + h (d.v) d is evaluated as F (v + T d) with F = f and
// T = h (d.v) / f.  On the Newton branch T = -3 r^-2 (d.v), so no division is
// needed there, and the form takes one instruction fewer than forming f v and
// h (d.v) d separately.  Inside eps (kNear) the spline values select F = f and
// T = h (d.v) / f, with f >= 0.625 / eps^3 > 0 (the spline's minimum).
// kNear: the pair may lie inside eps; else every pair of the source cell has
// r > eps and the Newton branch is exact.  Both paths evaluate the Newton
// branch with the same expressions, so a sink's bits do not depend on which
// path a work item takes for a source cell.
template <bool kNear>
__device__ __forceinline__ void adjoint(const float* s, float qx, float qy, float qz, float wx,
                                        float wy, float wz, float c0, float c1, float c2,
                                        float ha, float hb, float eps, float g, float& gx,
                                        float& gy, float& gz) {
  const float dx = s[0] - qx;
  const float dy = s[1] - qy;
  const float dz = s[2] - qz;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, g)));
  const float rinv = rsq_v(r2);
  const float rinv2 = rinv * rinv;
  const float vx = s[3] - wx;
  const float vy = s[4] - wy;
  const float vz = s[5] - wz;
  const float dv = __builtin_fmaf(dz, vz, __builtin_fmaf(dy, vy, dx * vx));
  float F = rinv2 * rinv;
  float T = (-3.0f * rinv2) * dv;
  if (kNear) {
    const float r = r2 * rinv;
    const bool inner = r < eps;
    const float fs = __builtin_fmaf(__builtin_fmaf(c2, r, c1), r, c0);
    const float hs = __builtin_fmaf(hb, rinv, ha);
    F = inner ? fs : F;
    T = inner ? (hs * dv) * __builtin_amdgcn_rcpf(fs) : T;
  }
  const float ex = __builtin_fmaf(T, dx, vx);
  const float ey = __builtin_fmaf(T, dy, vy);
  const float ez = __builtin_fmaf(T, dz, vz);
  gx = __builtin_fmaf(F, ex, gx);
  gy = __builtin_fmaf(F, ey, gy);
  gz = __builtin_fmaf(F, ez, gz);
}

__device__ __forceinline__ int wrap1_v(int v, int K) {
  v += v < 0 ? K : 0;
  v -= v >= K ? K : 0;
  return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

struct AdjConst {
  float c0, c1, c2, ha, hb, eps, g;
  float near2;  // (1.1 eps)^2: beyond it every pair takes the Newton branch
};

// kU adjoint interactions of one source group on a cell that may hold pairs
// inside eps.  Pairs with r > eps take the Newton expressions in adjoint<true>
// as well, so the spline select is needed only when some lane has r^2 below
// (1.1 eps)^2 (a wave-uniform vote); either way the bits equal adjoint<true>.
template <int kU>
__device__ __forceinline__ void adjoint_group_near(const float* c, float qx, float qy, float qz,
                                                   float wx, float wy, float wz,
                                                   const AdjConst& k, float& gx, float& gy,
                                                   float& gz) {
  // Only F and T change inside the branch, so the accumulators are updated
  // once, after it, with the same operations as adjoint<>.
  float dx[kU], dy[kU], dz[kU], vx[kU], vy[kU], vz[kU], r2[kU], rinv[kU], dv[kU], F[kU], T[kU];
  float m = 3.0e38f;
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const float* s = c + 6 * u;
    dx[u] = s[0] - qx;
    dy[u] = s[1] - qy;
    dz[u] = s[2] - qz;
    r2[u] = __builtin_fmaf(dz[u], dz[u], __builtin_fmaf(dy[u], dy[u], __builtin_fmaf(dx[u], dx[u], k.g)));
    m = __builtin_fminf(m, r2[u]);
    rinv[u] = rsq_v(r2[u]);
    const float rinv2 = rinv[u] * rinv[u];
    vx[u] = s[3] - wx;
    vy[u] = s[4] - wy;
    vz[u] = s[5] - wz;
    dv[u] = __builtin_fmaf(dz[u], vz[u], __builtin_fmaf(dy[u], vy[u], dx[u] * vx[u]));
    F[u] = rinv2 * rinv[u];
    T[u] = (-3.0f * rinv2) * dv[u];
  }
  if (__ballot(m < k.near2) != 0) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float r = r2[u] * rinv[u];
      const bool inner = r < k.eps;
      const float fs = __builtin_fmaf(__builtin_fmaf(k.c2, r, k.c1), r, k.c0);
      const float hs = __builtin_fmaf(k.hb, rinv[u], k.ha);
      F[u] = inner ? fs : F[u];
      T[u] = inner ? (hs * dv[u]) * __builtin_amdgcn_rcpf(fs) : T[u];
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const float ex = __builtin_fmaf(T[u], dx[u], vx[u]);
    const float ey = __builtin_fmaf(T[u], dy[u], vy[u]);
    const float ez = __builtin_fmaf(T[u], dz[u], vz[u]);
    gx = __builtin_fmaf(F[u], ex, gx);
    gy = __builtin_fmaf(F[u], ey, gy);
    gz = __builtin_fmaf(F[u], ez, gz);
  }
}

template <int kU, bool kNear>
__device__ __forceinline__ void adjoint_group(const float* c, float qx, float qy, float qz,
                                              float wx, float wy, float wz, const AdjConst& k,
                                              float& gx, float& gy, float& gz) {
  if (kNear) {
    adjoint_group_near<kU>(c, qx, qy, qz, wx, wy, wz, k, gx, gy, gz);
  } else {
#pragma unroll
    for (int u = 0; u < kU; ++u)
      adjoint<false>(c + 6 * u, qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, k.g,
                     gx, gy, gz);
  }
}

// Sum the sources [beg, end) of packed 24-byte records, kU per step (with kPipe
// the next kU records are requested before the current ones are used).
template <int kU, bool kPipe, bool kNear>
__device__ __forceinline__ void sum_adjoint(const float* __restrict__ src6, int beg, int end,
                                            float qx, float qy, float qz, float wx, float wy,
                                            float wz, const AdjConst& k, float& gx, float& gy,
                                            float& gz) {
  int j = beg;
  if (kPipe && j + kU <= end) {
    float cur[6 * kU];
#pragma unroll
    for (int u = 0; u < 6 * kU; ++u) cur[u] = src6[6 * j + u];
    for (; j + 2 * kU <= end; j += kU) {
      float nxt[6 * kU];
#pragma unroll
      for (int u = 0; u < 6 * kU; ++u) nxt[u] = src6[6 * (j + kU) + u];
      adjoint_group<kU, kNear>(cur, qx, qy, qz, wx, wy, wz, k, gx, gy, gz);
#pragma unroll
      for (int u = 0; u < 6 * kU; ++u) cur[u] = nxt[u];
    }
    adjoint_group<kU, kNear>(cur, qx, qy, qz, wx, wy, wz, k, gx, gy, gz);
    j += kU;
  }
  for (; j + kU <= end; j += kU) {
    float cur[6 * kU];
#pragma unroll
    for (int u = 0; u < 6 * kU; ++u) cur[u] = src6[6 * j + u];
    adjoint_group<kU, kNear>(cur, qx, qy, qz, wx, wy, wz, k, gx, gy, gz);
  }
  for (; j < end; ++j) {
    float one[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) one[u] = src6[6 * j + u];
    adjoint<kNear>(one, qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, k.g, gx, gy, gz);
  }
}

// The two edge cells of a two-cell item (za, za + 1): lanes of the lower
// sink cell need the cell R below it and lanes of the upper sink cell the cell
// R above it, and neither set needs the other's.  Both are far cells (every
// pair has r > eps, or the Plummer law), so the wave steps through the two
// runs together and pays the longer run's length instead of the sum of both.
// Per chunk of kChunk positions the wave stages both runs' records in its own
// LDS slot (lane l copies position l of each run, coalesced), then every lane
// reads its own run's records from there: two distinct LDS addresses per read,
// served as broadcasts.  (Per-lane global loads of the same records took the
// L1 address path for 24 cycles per record and wave.)  Lanes of the shorter
// run stop at its end.  The single mode keeps adding every pair to the one
// running accumulator; the chunked and compensated modes fold each chunk's sum
// into it like a cell's.
constexpr int kEdgeRec = 6;

template <int kAcc>
__device__ __forceinline__ void adjoint_edge_runs(const float* __restrict__ src6,
                                                  float* __restrict__ slot, int lane, bool upper,
                                                  int bl, int nl, int bh, int nh, float qx,
                                                  float qy, float qz, float wx, float wy,
                                                  float wz, const AdjConst& k, float& gx,
                                                  float& gy, float& gz, float& ex, float& ey,
                                                  float& ez) {
  const int nmax = nl > nh ? nl : nh;
  const int rn = upper ? nh : nl;
  const float* mine = slot + (upper ? kChunk * kEdgeRec : 0);
  const float* __restrict__ runl = src6 + kEdgeRec * (int64_t)bl;
  const float* __restrict__ runh = src6 + kEdgeRec * (int64_t)bh;
  for (int cb = 0; cb < nmax; cb += kChunk) {
    const int ce = cb + kChunk < nmax ? cb + kChunk : nmax;
    if (cb + lane < nl) {
#pragma unroll
      for (int c = 0; c < kEdgeRec; ++c) slot[kEdgeRec * lane + c] = runl[kEdgeRec * (cb + lane) + c];
    }
    if (cb + lane < nh) {
#pragma unroll
      for (int c = 0; c < kEdgeRec; ++c)
        slot[kChunk * kEdgeRec + kEdgeRec * lane + c] = runh[kEdgeRec * (cb + lane) + c];
    }
    __builtin_amdgcn_wave_barrier();
    const int n = (rn < ce ? rn : ce) - cb;  // this lane's positions in the chunk
    // SINGLE: the running accumulator itself; otherwise a fresh chunk partial
    const bool one = kAcc == kAccSingle;
    float tx = one ? gx : 0.f, ty = one ? gy : 0.f, tz = one ? gz : 0.f;
    int j = 0;
    for (; j + 2 <= n; j += 2) {
      float c2[2 * kEdgeRec];
#pragma unroll
      for (int u = 0; u < 2 * kEdgeRec; ++u) c2[u] = mine[kEdgeRec * j + u];
      adjoint<false>(c2, qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, k.g, tx,
                     ty, tz);
      adjoint<false>(c2 + kEdgeRec, qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps,
                     k.g, tx, ty, tz);
    }
    if (j < n) {
      float c1[kEdgeRec];
#pragma unroll
      for (int u = 0; u < kEdgeRec; ++u) c1[u] = mine[kEdgeRec * j + u];
      adjoint<false>(c1, qx, qy, qz, wx, wy, wz, k.c0, k.c1, k.c2, k.ha, k.hb, k.eps, k.g, tx,
                     ty, tz);
    }
    __builtin_amdgcn_wave_barrier();
    if (kAcc == kAccSingle) {
      gx = tx; gy = ty; gz = tz;
    } else if (n > 0) {
      if (kAcc == kAccChunked) {
        gx += tx; gy += ty; gz += tz;
      } else {
        two_sum_fold(gx, ex, tx);
        two_sum_fold(gy, ey, ty);
        two_sum_fold(gz, ez, tz);
      }
    }
  }
}

// Packed source records (rel_s, w_perm[s]) per sorted slot, 6 floats each.
__global__ __launch_bounds__(256) void k_gather_src(const float4* __restrict__ rel,
                                                    const int32_t* __restrict__ perm,
                                                    const float* __restrict__ w, int64_t n,
                                                    float* __restrict__ src6) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t i = perm[s];
  const float4 r = rel[s];
  src6[6 * s + 0] = r.x;
  src6[6 * s + 1] = r.y;
  src6[6 * s + 2] = r.z;
  src6[6 * s + 3] = w[3 * i + 0];
  src6[6 * s + 4] = w[3 * i + 1];
  src6[6 * s + 5] = w[3 * i + 2];
}

// Register caps for more resident waves: unrolls 2 and 3 fit 8 waves per SIMD,
// unroll 4 fits 7.  Unroll 2 does not spill; unroll 3 spills 56 bytes at task
// and column boundaries, unroll 4 76 bytes, with one reload in the single-record
// tail of an edge-run chunk.  Without the caps the compiler takes 112 SGPRs
// and, at unroll 4, 80 VGPRs: 7 and 6 waves.
template <int kU>
constexpr int vjp_min_waves() { return kU <= 3 ? 8 : (kU == 4 ? 7 : 1); }

template <int kAcc, int kU, bool kPipe>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(vjp_min_waves<kU>(), 8))) void k_pair_vjp(
    const DevBox* __restrict__ boxes, const int4* __restrict__ items,
    const int32_t* __restrict__ tasks, const int32_t* __restrict__ item_cost,
    int32_t* __restrict__ ctrl, const int32_t* __restrict__ off, const float* __restrict__ src6,
    const int32_t* __restrict__ perm, float* __restrict__ grad, float* __restrict__ partial,
    int n_static) {
  const int lane = threadIdx.x & 63;
  // this wave's staging slot for the paired edge runs (two runs of kChunk records)
  __shared__ float edge_lds[4][2 * kChunk * kEdgeRec];
  float* const edge_slot = edge_lds[threadIdx.x >> 6];
  const int n_tasks = uni(ctrl[kCtrlNTasks]);
  const int n_whole = uni(ctrl[kCtrlNWhole]);
  const int n_split = uni(ctrl[kCtrlNSplit]);
  const int slices = uni(ctrl[kCtrlSlices]);
  bool first = true;
  while (true) {
    const int t = next_task(&ctrl[kCtrlHead], first, n_static);
    if (t >= n_tasks) break;
    const int task = uni(tasks[t]);
    const int code = task & kTaskCodeMask;  // 0: whole item; c > 0: x offset c - 1 - R only
    const int4 it = items[task >> kTaskShift];
    const int b = uni(it.x & 0xffff), count = uni(it.x >> 16);
    const int cx = uni(it.y & 0xffff), cy = uni(it.y >> 16);
    const int za = uni(it.z & 0xffff), zb = uni(it.z >> 16);
    const int first = uni(it.w);
    const int K = uni(boxes[b].K), R = uni(boxes[b].R);
    // sources this task visits: the item's cost, or one x offset's share of it
    int left = uni(item_cost[task >> kTaskShift]);
    if (code) left /= 2 * R + 1;
    set_wave_priority(left);
    const int cbase = uni(boxes[b].cell_base);
    AdjConst kc;
    kc.c0 = boxes[b].c0; kc.c1 = boxes[b].c1; kc.c2 = boxes[b].c2;
    kc.ha = boxes[b].ha; kc.hb = boxes[b].hb; kc.eps = boxes[b].eps; kc.g = boxes[b].guard;
    kc.near2 = boxes[b].near2;
    // c1 and ha each meet another SGPR operand in an FMA; a VALU instruction
    // reads at most one SGPR, so keep them in VGPRs for the whole item.
    asm volatile("" : "+v"(kc.c1), "+v"(kc.ha));
    const int pencil0 = cbase + (cx * K + cy) * K;
    const int far_mode = uni(boxes[b].far_mode);
    const int ox_lo = code ? code - 1 - R : -R;
    const int ox_hi = code ? ox_lo : R;

    // lane -> sink: the item's sinks are the contiguous slots [first, first+count)
    const int s = lane < count ? first + lane : -1;
    int lane_z = za;
    for (int z = za; z < zb; ++z)
      if (s >= uni(off[pencil0 + z + 1])) lane_z = z + 1;
    const bool active = s >= 0;
    // Two-cell items take their edge cells as paired runs when those cells
    // are far (R >= 2, no spline; adjoint_edge_runs).
    const bool pair_edges = zb == za + 1 && R >= 2 && far_mode != kFarNone;
    const bool upper = lane_z == zb;
    float px = 0.f, py = 0.f, pz = 0.f, wkx = 0.f, wky = 0.f, wkz = 0.f;
    if (active) {
      const float* __restrict__ mine = src6 + 6 * (int64_t)s;
      px = mine[0];
      py = mine[1];
      pz = mine[2];
      wkx = mine[3];
      wky = mine[4];
      wkz = mine[5];
    }

    // (G, E): the sink's sum; (g, e): the current x-offset slice (SINGLE keeps
    // one running accumulator in g and never folds).
    float Gx = 0.f, Gy = 0.f, Gz = 0.f, Ex = 0.f, Ey = 0.f, Ez = 0.f;
    float gx = 0.f, gy = 0.f, gz = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
    for (int ox = ox_lo; ox <= ox_hi; ++ox) {
      if (kAcc != kAccSingle) gx = gy = gz = ex = ey = ez = 0.f;
      const int sx = wrap1_v(cx + ox, K);
      const float qx = px - (float)ox;
      for (int oy = -R; oy <= R; ++oy) {
        const int sy = wrap1_v(cy + oy, K);
        const float qy = py - (float)oy;
        const int col = cbase + (sx * K + sy) * K;
        const bool col_near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
        for (int zu = za - R; zu <= zb + R; ++zu) {
          if (pair_edges && (zu == za - R || zu == zb + R)) continue;
          const int sz = wrap1_v(zu, K);
          const int beg = uni(off[col + sz]), end = uni(off[col + sz + 1]);
          if (beg == end) continue;
          left -= end - beg;
          set_wave_priority(left);
          const int oz = zu - lane_z;
          const bool near = far_mode == kFarNone ||
                            (far_mode == kFarApart && col_near && zu >= za - 1 && zu <= zb + 1);
          if (active && oz >= -R && oz <= R) {
            const float qz = pz - (float)oz;
            if (kAcc == kAccSingle) {
              if (near)
                sum_adjoint<kU, kPipe, true>(src6 + 6 * (int64_t)beg, 0, end - beg, qx, qy, qz, wkx, wky, wkz, kc, gx,
                                             gy, gz);
              else
                sum_adjoint<kU, kPipe, false>(src6 + 6 * (int64_t)beg, 0, end - beg, qx, qy, qz, wkx, wky, wkz, kc, gx,
                                              gy, gz);
            } else {
              for (int cb = beg; cb < end; cb += kChunk) {
                const int ce = cb + kChunk < end ? cb + kChunk : end;
                float tx = 0.f, ty = 0.f, tz = 0.f;
                if (near)
                  sum_adjoint<kU, kPipe, true>(src6 + 6 * (int64_t)cb, 0, ce - cb, qx, qy, qz, wkx, wky, wkz, kc, tx,
                                               ty, tz);
                else
                  sum_adjoint<kU, kPipe, false>(src6 + 6 * (int64_t)cb, 0, ce - cb, qx, qy, qz, wkx, wky, wkz, kc, tx,
                                                ty, tz);
                if (kAcc == kAccChunked) {
                  gx += tx; gy += ty; gz += tz;
                } else {
                  two_sum_fold(gx, ex, tx);
                  two_sum_fold(gy, ey, ty);
                  two_sum_fold(gz, ez, tz);
                }
              }
            }
          }
        }
        if (pair_edges) {
          const int zl = wrap1_v(za - R, K), zh = wrap1_v(zb + R, K);
          const int bl = uni(off[col + zl]), nl = uni(off[col + zl + 1]) - bl;
          const int bh = uni(off[col + zh]), nh = uni(off[col + zh + 1]) - bh;
          if (nl + nh > 0) {
            left -= nl > nh ? nl : nh;
            set_wave_priority(left);
            // every lane takes part (each stages records); inactive lanes'
            // sums are never written
            adjoint_edge_runs<kAcc>(src6, edge_slot, lane, upper, bl, nl, bh, nh, qx, qy,
                                    pz - (float)(upper ? R : -R), wkx, wky, wkz, kc, gx, gy, gz,
                                    ex, ey, ez);
          }
        }
      }
      if (kAcc != kAccSingle && code == 0) {
        slice_fold<kAcc>(Gx, Ex, gx, ex);
        slice_fold<kAcc>(Gy, Ey, gy, ey);
        slice_fold<kAcc>(Gz, Ez, gz, ez);
      }
    }
    if (kAcc == kAccSingle) {
      Gx = gx; Gy = gy; Gz = gz;
    }
    if (code == 0) {
      if (active) {
        const float iw3 = boxes[b].inv_w3;
        const int64_t i = perm[s];
        grad[3 * i + 0] = (Gx + Ex) * iw3;
        grad[3 * i + 1] = (Gy + Ey) * iw3;
        grad[3 * i + 2] = (Gz + Ez) * iw3;
      }
    } else {
      // a tail item split by x offset: keep this slice for k_combine_slices
      const int slot = (t - n_whole) % n_split;
      float* dst = partial + (int64_t)(slot * slices + (code - 1)) * kPartialStride * kTile + lane;
      dst[0 * kTile] = gx; dst[1 * kTile] = gy; dst[2 * kTile] = gz;
      dst[3 * kTile] = ex; dst[4 * kTile] = ey; dst[5 * kTile] = ez;
    }
  }
}

template <int kAcc, int kU, bool kPipe>
static hipError_t launch_vjp_t(const DevBox* boxes, const PlanWork& w, const int32_t* off,
                               const float* src, const int32_t* perm, float* grad, int grid_mult,
                               hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_pair_vjp<kAcc, kU, kPipe>);
  const int resident = persistent_blocks(fn, 256);
  const int blocks = resident * grid_mult;
  hipLaunchKernelGGL((k_pair_vjp<kAcc, kU, kPipe>), dim3(blocks), dim3(256), 0, s, boxes, w.items,
                     w.tasks, w.item_cost, w.ctrl, off, src, perm, grad, w.partial, resident * 4);
  return hipGetLastError();
}

template <int kAcc>
static hipError_t dispatch_vjp(const KernelConfig& cfg, const DevBox* boxes, const PlanWork& w,
                               const int32_t* off, const float* src, const int32_t* perm,
                               float* grad, hipStream_t s) {
  const int g = cfg.grid_mult;
  switch (cfg.unroll * 2 + (cfg.pipeline ? 1 : 0)) {
    case 5: return launch_vjp_t<kAcc, 2, true>(boxes, w, off, src, perm, grad, g, s);
    case 6: return launch_vjp_t<kAcc, 3, false>(boxes, w, off, src, perm, grad, g, s);
    case 7: return launch_vjp_t<kAcc, 3, true>(boxes, w, off, src, perm, grad, g, s);
    case 8: return launch_vjp_t<kAcc, 4, false>(boxes, w, off, src, perm, grad, g, s);
    case 9: return launch_vjp_t<kAcc, 4, true>(boxes, w, off, src, perm, grad, g, s);
    default: return launch_vjp_t<kAcc, 2, false>(boxes, w, off, src, perm, grad, g, s);
  }
}

hipError_t launch_vjp(AccMode mode, const KernelConfig& cfg, const DevBox* boxes,
                      const PlanWork& w, int64_t pencils, const int32_t* off, const float* rel,
                      const int32_t* perm, const float* wvec, float* src_w, int64_t n_total,
                      float* grad, hipStream_t s) {
  (void)pencils;
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_src, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(rel), perm, wvec, n_total, src_w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (mode) {
    case kAccSingle: e = dispatch_vjp<kAccSingle>(cfg, boxes, w, off, src_w, perm, grad, s); break;
    case kAccChunked: e = dispatch_vjp<kAccChunked>(cfg, boxes, w, off, src_w, perm, grad, s); break;
    default: e = dispatch_vjp<kAccCompensated>(cfg, boxes, w, off, src_w, perm, grad, s); break;
  }
  if (e != hipSuccess) return e;
  return launch_combine(mode, true, boxes, w, perm, grad, nullptr, s);
}

}  // namespace anf
