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
//   * the exception is an item whose sinks lie in two cells: its two far edge
//     cells (each needed by one of the two lane sets) are walked together,
//     staged per 64-position chunk in the wave's own LDS slot;
//   * the periodic wrap never reaches the arithmetic: a source cell's integer
//     offset o from the sink's cell is folded into the sink (q = p - o) once per
//     source cell, and d = s - q uses only FP32 cell-relative coordinates;
//   * sums are per-lane registers; a persistent grid takes items from a
//     longest-first queue (each wave's first item by its grid index, the rest
//     with one atomic each), and each wave's priority follows the sources left
//     in its current item.
#include "nf_internal.h"

namespace anf {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ int wrap1(int v, int K) {
  v += v < 0 ? K : 0;
  v -= v >= K ? K : 0;
  return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-item constants of the pair law: f(r) = c0 + c1 r + c2 r^2 inside eps
// (cell units, Eq. 3) and the squared top-hat radius b2 of the density estimate.
struct PairConst {
  float c0, c1, c2, b2, g;
  float near2;  // (1.1 eps)^2: beyond it the spline exceeds 1/r^3 by more than 1%
};

// One interaction: t += f(|d|) d with d = s - q (cell units) and r^2 taken with
// the guard g added.  kNear: the pair may lie inside the spline's softening
// length, so f = min(spline(r), 1/r^3); otherwise f = (r^2 + g)^(-3/2): for Eq. 3
// the source cell is so far from every sink that r > eps for all its pairs and
// this is exactly the value the minimum would select; for Eq. 2 (g = eps_p^2)
// it is the Plummer law itself.  kDens also adds the apodized top-hat weight
// max(b^2 - r^2, 0) of Sec. 3.4.4 to rho (b2 carries the same guard).
template <bool kNear, bool kDens>
__device__ __forceinline__ void interact(float sx, float sy, float sz, float qx, float qy,
                                         float qz, const PairConst& k, float& tx, float& ty,
                                         float& tz, float& rho) {
  const float dx = sx - qx;
  const float dy = sy - qy;
  const float dz = sz - qz;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, k.g)));
  const float rinv = rsq(r2);
  const float rinv3 = (rinv * rinv) * rinv;
  float f = rinv3;
  if (kNear) {
    const float r = r2 * rinv;
    const float spline = __builtin_fmaf(__builtin_fmaf(k.c2, r, k.c1), r, k.c0);
    f = __builtin_fminf(spline, rinv3);
  }
  tx = __builtin_fmaf(f, dx, tx);
  ty = __builtin_fmaf(f, dy, ty);
  tz = __builtin_fmaf(f, dz, tz);
  if (kDens) rho += __builtin_fmaxf(k.b2 - r2, 0.0f);
}

// kU interactions of one source group on a cell that may hold pairs inside
// eps.  The separations are formed first; only if some lane has r^2 below
// near2 = (1.1 eps)^2 (a wave-uniform vote) does the group take the spline
// select, otherwise every pair is at least 1.1 eps apart, where the spline
// exceeds 1/r^3 by over 1% and the minimum is exactly 1/r^3 -- so both ways
// give the bits of interact<true>.
template <int kU, bool kDens>
__device__ __forceinline__ void interact_group_near(const float* c, float qx, float qy, float qz,
                                                    const PairConst& k, float& tx, float& ty,
                                                    float& tz, float& rho) {
  float dx[kU], dy[kU], dz[kU], r2[kU];
  float m = 3.0e38f;
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    dx[u] = c[3 * u] - qx;
    dy[u] = c[3 * u + 1] - qy;
    dz[u] = c[3 * u + 2] - qz;
    r2[u] = __builtin_fmaf(dz[u], dz[u], __builtin_fmaf(dy[u], dy[u], __builtin_fmaf(dx[u], dx[u], k.g)));
    m = __builtin_fminf(m, r2[u]);
  }
  // The Newton factor for every pair; a group with a lane below near2 then
  // replaces it by the minimum with the spline.  Only f changes inside the
  // branch, so the accumulators are updated once, after it.
  float f[kU], rinv[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    rinv[u] = rsq(r2[u]);
    f[u] = (rinv[u] * rinv[u]) * rinv[u];
  }
  if (__ballot(m < k.near2) != 0) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float r = r2[u] * rinv[u];
      const float spline = __builtin_fmaf(__builtin_fmaf(k.c2, r, k.c1), r, k.c0);
      f[u] = __builtin_fminf(spline, f[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    tx = __builtin_fmaf(f[u], dx[u], tx);
    ty = __builtin_fmaf(f[u], dy[u], ty);
    tz = __builtin_fmaf(f[u], dz[u], tz);
    if (kDens) rho += __builtin_fmaxf(k.b2 - r2[u], 0.0f);
  }
}

template <int kU, bool kNear, bool kDens>
__device__ __forceinline__ void interact_group(const float* c, float qx, float qy, float qz,
                                               const PairConst& k, float& tx, float& ty,
                                               float& tz, float& rho) {
  if (kNear) {
    interact_group_near<kU, kDens>(c, qx, qy, qz, k, tx, ty, tz, rho);
  } else {
#pragma unroll
    for (int u = 0; u < kU; ++u)
      interact<false, kDens>(c[3 * u], c[3 * u + 1], c[3 * u + 2], qx, qy, qz, k, tx, ty, tz, rho);
  }
}

// Sum the sources [beg, end) into (tx, ty, tz) (and rho), kU per step.  Sources
// are packed (x, y, z) records of 12 bytes so that a group of kU sources
// occupies 3 kU SGPRs.  With kPipe the next kU sources are requested before the
// current ones are used, so the scalar-cache latency of one group overlaps the
// arithmetic of the previous.
template <int kU, bool kPipe, bool kNear, bool kDens>
__device__ __forceinline__ void sum_sources(const float* __restrict__ src3, int beg, int end,
                                            float qx, float qy, float qz, const PairConst& k,
                                            float& tx, float& ty, float& tz, float& rho) {
  int j = beg;
  if (kPipe && j + kU <= end) {
    float cur[3 * kU];
#pragma unroll
    for (int u = 0; u < 3 * kU; ++u) cur[u] = src3[3 * j + u];
    for (; j + 2 * kU <= end; j += kU) {
      float nxt[3 * kU];
#pragma unroll
      for (int u = 0; u < 3 * kU; ++u) nxt[u] = src3[3 * (j + kU) + u];
      interact_group<kU, kNear, kDens>(cur, qx, qy, qz, k, tx, ty, tz, rho);
#pragma unroll
      for (int u = 0; u < 3 * kU; ++u) cur[u] = nxt[u];
    }
    interact_group<kU, kNear, kDens>(cur, qx, qy, qz, k, tx, ty, tz, rho);
    j += kU;
  }
  for (; j + kU <= end; j += kU) {
    float cur[3 * kU];
#pragma unroll
    for (int u = 0; u < 3 * kU; ++u) cur[u] = src3[3 * j + u];
    interact_group<kU, kNear, kDens>(cur, qx, qy, qz, k, tx, ty, tz, rho);
  }
  for (; j < end; ++j)
    interact<kNear, kDens>(src3[3 * j], src3[3 * j + 1], src3[3 * j + 2], qx, qy, qz, k, tx, ty,
                           tz, rho);
}

// The two edge cells of a two-cell item (za, za + 1): lanes of the lower
// sink cell need the cell R below it and lanes of the upper sink cell the cell
// R above it, and neither set needs the other's.  Both are far cells
// (Newtonian for Eq. 3, or the Plummer law), so the wave steps through the two
// runs together and pays the longer run's length instead of the sum of both.
// Per chunk of kChunk positions the wave stages both runs' records in its own
// LDS slot (lane l copies position l of each run, coalesced), then every lane
// reads its own run's records from there: two distinct LDS addresses per read,
// served as broadcasts.  (Per-lane global loads of the same records took the
// L1 address path for 16 cycles per record and wave.)  Lanes of the shorter
// run stop at its end.  The single mode keeps adding every pair to the one
// running accumulator; the chunked and compensated modes fold each chunk's sum
// into it like a cell's.
template <int kAcc, int kU>
__device__ __forceinline__ void sum_edge_runs(const float* __restrict__ src3,
                                              float* __restrict__ slot, int lane, bool upper,
                                              int bl, int nl, int bh, int nh, float qx, float qy,
                                              float qz, const PairConst& k, float& ax, float& ay,
                                              float& az, float& ex, float& ey, float& ez) {
  const int nmax = nl > nh ? nl : nh;
  const int rn = upper ? nh : nl;
  const float* mine = slot + (upper ? 3 * kChunk : 0);
  const float* __restrict__ runl = src3 + 3 * (int64_t)bl;
  const float* __restrict__ runh = src3 + 3 * (int64_t)bh;
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
    const int n = (rn < ce ? rn : ce) - cb;  // this lane's positions in the chunk
    // SINGLE: the running accumulator itself; otherwise a fresh chunk partial
    const bool one = kAcc == kAccSingle;
    float tx = one ? ax : 0.f, ty = one ? ay : 0.f, tz = one ? az : 0.f, rho = 0.f;
    int j = 0;
    for (; j + kU <= n; j += kU) {
      float c[3 * kU];
#pragma unroll
      for (int u = 0; u < 3 * kU; ++u) c[u] = mine[3 * j + u];
      interact_group<kU, false, false>(c, qx, qy, qz, k, tx, ty, tz, rho);
    }
    for (; j < n; ++j)
      interact<false, false>(mine[3 * j], mine[3 * j + 1], mine[3 * j + 2], qx, qy, qz, k, tx, ty,
                             tz, rho);
    __builtin_amdgcn_wave_barrier();
    if (kAcc == kAccSingle) {
      ax = tx; ay = ty; az = tz;
    } else if (n > 0) {
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

// Packed 12-byte source records (x, y, z) from the binned float4 offsets.
__global__ __launch_bounds__(256) void k_pack_sources(const float4* __restrict__ rel, int64_t n,
                                                      float* __restrict__ src3) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float4 r = rel[s];
  src3[3 * s + 0] = r.x;
  src3[3 * s + 1] = r.y;
  src3[3 * s + 2] = r.z;
}

// The production shapes (kU <= 4, no pair counter) fit 8 waves per SIMD once
// their scalar registers are capped; without the cap the compiler takes about
// 105 SGPRs and 7 waves.  (With the density estimate at unroll 4, 12 bytes
// spill outside the pair loop.)  The other variants would spill more, so they
// keep the compiler's own choice.
template <int kU, bool kCount, bool kDens>
constexpr int fwd_min_waves() { return kU <= 4 && !kCount ? 8 : 1; }

template <int kAcc, bool kCount, int kU, bool kPipe, bool kDens>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(fwd_min_waves<kU, kCount, kDens>(), 8))) void k_pair_forward(
    const DevBox* __restrict__ boxes, const int4* __restrict__ items,
    const int32_t* __restrict__ tasks, const int32_t* __restrict__ item_cost, int32_t* __restrict__ ctrl,
    const int32_t* __restrict__ off, const float4* __restrict__ rel,
    const float* __restrict__ src3, const int32_t* __restrict__ perm, float* __restrict__ acc_out,
    float* __restrict__ dens_out, float* __restrict__ partial,
    unsigned long long* __restrict__ pair_count, int n_static) {
  const int lane = threadIdx.x & 63;
  // this wave's staging slot for the paired edge runs (two runs of kChunk records)
  __shared__ float edge_lds[4][2 * kChunk * 3];
  float* const edge_slot = edge_lds[threadIdx.x >> 6];
  const int n_tasks = uniform(ctrl[kCtrlNTasks]);
  const int n_whole = uniform(ctrl[kCtrlNWhole]);
  const int n_split = uniform(ctrl[kCtrlNSplit]);
  const int slices = uniform(ctrl[kCtrlSlices]);
  bool first = true;
  while (true) {
    const int t = next_task(&ctrl[kCtrlHead], first, n_static);
    if (t >= n_tasks) break;
    const int task = uniform(tasks[t]);
    const int code = task & kTaskCodeMask;  // 0: whole item; c > 0: x offset c - 1 - R only
    const int4 it = items[task >> kTaskShift];
    const int b = uniform(it.x & 0xffff), count = uniform(it.x >> 16);
    const int cx = uniform(it.y & 0xffff), cy = uniform(it.y >> 16);
    const int za = uniform(it.z & 0xffff), zb = uniform(it.z >> 16);
    const int first = uniform(it.w);
    const int K = uniform(boxes[b].K), R = uniform(boxes[b].R);
    // sources this task visits: the item's cost, or one x offset's share of it
    int left = uniform(item_cost[task >> kTaskShift]);
    if (code) left /= 2 * R + 1;
    set_wave_priority(left);
    const int cbase = uniform(boxes[b].cell_base);
    PairConst kc;
    kc.c0 = boxes[b].c0;
    kc.c1 = boxes[b].c1;
    kc.c2 = boxes[b].c2;
    kc.b2 = boxes[b].b2;
    kc.g = boxes[b].guard;
    kc.near2 = boxes[b].near2;
    // c1 meets an SGPR operand (c2) in the spline FMA; a VALU instruction reads
    // at most one SGPR, so keep c1 in a VGPR for the whole item.  The guard
    // added to every r^2 is kept in a VGPR too: on gfx950 an instruction that
    // reads an SGPR issues only to the first of the two VALU pipes, and the
    // first FMA of every pair reads the guard (forward kernel 2.7% faster).
    asm volatile("" : "+v"(kc.c1), "+v"(kc.g));
    const int pencil0 = cbase + (cx * K + cy) * K;
    // Cells two or more apart on some axis are >= 1 cell width apart, so with
    // eps < 1/2 cell every pair in them is Newtonian (f = 1/r^3), and with
    // b < 1/2 cell none of them is within the density radius.
    const int far_mode = uniform(boxes[b].far_mode);
    const bool dens_far = kDens && uniform(boxes[b].dens_far) != 0;
    const int ox_lo = code ? code - 1 - R : -R;
    const int ox_hi = code ? ox_lo : R;

    // ---- which sink this lane owns -------------------------------------
    // lane -> sink: the item's sinks are the contiguous slots [first, first+count)
    const int s = lane < count ? first + lane : -1;
    int lane_z = za;
    for (int z = za; z < zb; ++z)
      if (s >= uniform(off[pencil0 + z + 1])) lane_z = z + 1;
    const bool active = s >= 0;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) p = rel[s];
    // Two-cell items take their edge cells as paired runs when those cells are
    // far (R >= 2, no spline) and add no density (sum_edge_runs).
    const bool pair_edges = zb == za + 1 && R >= 2 && far_mode != kFarNone &&
                            (!kDens || dens_far);
    const bool upper = lane_z == zb;

    // (A, E): the sink's sum; (a, e): the current x-offset slice (SINGLE keeps
    // one running accumulator in a and never folds).
    float Ax = 0.f, Ay = 0.f, Az = 0.f, Ex = 0.f, Ey = 0.f, Ez = 0.f, Rho = 0.f;
    float ax = 0.f, ay = 0.f, az = 0.f, ex = 0.f, ey = 0.f, ez = 0.f, rho = 0.f;
    long long npairs = 0;
    for (int ox = ox_lo; ox <= ox_hi; ++ox) {
      if (kAcc != kAccSingle) ax = ay = az = ex = ey = ez = rho = 0.f;
      const int sx = wrap1(cx + ox, K);
      const float qx = p.x - (float)ox;
      for (int oy = -R; oy <= R; ++oy) {
        const int sy = wrap1(cy + oy, K);
        const float qy = p.y - (float)oy;
        const int col = cbase + (sx * K + sy) * K;
        const bool col_near = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
        for (int zu = za - R; zu <= zb + R; ++zu) {
          if (pair_edges && (zu == za - R || zu == zb + R)) continue;
          const int sz = wrap1(zu, K);
          const int beg = uniform(off[col + sz]), end = uniform(off[col + sz + 1]);
          if (beg == end) continue;
          left -= end - beg;
          set_wave_priority(left);
          const int oz = zu - lane_z;
          // Wave-uniform: is this source cell within one cell of every sink
          // cell of the item, and can a pair of it fall inside the spline?
          const bool geo_near = col_near && zu >= za - 1 && zu <= zb + 1;
          const bool near = far_mode == kFarNone || (far_mode == kFarApart && geo_near);
          const bool dens_here = kDens && (geo_near || !dens_far);
          if (active && oz >= -R && oz <= R) {
            const float qz = p.z - (float)oz;
            if (kCount) npairs += end - beg;
            if (kAcc == kAccSingle) {
              if (near)
                sum_sources<kU, kPipe, true, kDens>(src3 + 3 * (int64_t)beg, 0, end - beg, qx, qy, qz, kc, ax, ay, az, rho);
              else if (dens_here)
                sum_sources<kU, kPipe, false, kDens>(src3 + 3 * (int64_t)beg, 0, end - beg, qx, qy, qz, kc, ax, ay, az, rho);
              else
                sum_sources<kU, kPipe, false, false>(src3 + 3 * (int64_t)beg, 0, end - beg, qx, qy, qz, kc, ax, ay, az, rho);
            } else {
              for (int cb = beg; cb < end; cb += kChunk) {
                const int ce = cb + kChunk < end ? cb + kChunk : end;
                float tx = 0.f, ty = 0.f, tz = 0.f;
                if (near)
                  sum_sources<kU, kPipe, true, kDens>(src3 + 3 * (int64_t)cb, 0, ce - cb, qx, qy, qz, kc, tx, ty, tz, rho);
                else if (dens_here)
                  sum_sources<kU, kPipe, false, kDens>(src3 + 3 * (int64_t)cb, 0, ce - cb, qx, qy, qz, kc, tx, ty, tz, rho);
                else
                  sum_sources<kU, kPipe, false, false>(src3 + 3 * (int64_t)cb, 0, ce - cb, qx, qy, qz, kc, tx, ty, tz, rho);
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
        if (pair_edges) {
          const int zl = wrap1(za - R, K), zh = wrap1(zb + R, K);
          const int bl = uniform(off[col + zl]), nl = uniform(off[col + zl + 1]) - bl;
          const int bh = uniform(off[col + zh]), nh = uniform(off[col + zh + 1]) - bh;
          if (nl + nh > 0) {
            left -= nl > nh ? nl : nh;
            set_wave_priority(left);
            if (kCount && active) npairs += upper ? nh : nl;
            // every lane takes part (each stages records); inactive lanes'
            // sums are never written
            sum_edge_runs<kAcc, kU>(src3, edge_slot, lane, upper, bl, nl, bh, nh, qx, qy,
                                    p.z - (float)(upper ? R : -R), kc, ax, ay, az, ex, ey, ez);
          }
        }
      }
      if (kAcc != kAccSingle && code == 0) {
        slice_fold<kAcc>(Ax, Ex, ax, ex);
        slice_fold<kAcc>(Ay, Ey, ay, ey);
        slice_fold<kAcc>(Az, Ez, az, ez);
        Rho += rho;
      }
    }
    if (kAcc == kAccSingle) {
      Ax = ax; Ay = ay; Az = az; Rho = rho;
    }
    if (code == 0) {
      if (active) {
        const float iw2 = boxes[b].inv_w2;
        const int64_t i = perm[s];
        acc_out[3 * i + 0] = (Ax + Ex) * iw2;
        acc_out[3 * i + 1] = (Ay + Ey) * iw2;
        acc_out[3 * i + 2] = (Az + Ez) * iw2;
        if (kDens) dens_out[i] = Rho * boxes[b].inv_b2;
      }
    } else {
      // a tail item split by x offset: keep this slice for k_combine_slices
      const int slot = (t - n_whole) % n_split;
      float* dst = partial + (int64_t)(slot * slices + (code - 1)) * kPartialStride * kTile + lane;
      dst[0 * kTile] = ax; dst[1 * kTile] = ay; dst[2 * kTile] = az;
      dst[3 * kTile] = ex; dst[4 * kTile] = ey; dst[5 * kTile] = ez;
      dst[6 * kTile] = rho;
    }
    if (kCount) {
      // the sink itself sits in its own cell, visited by the x offset 0
      if (active && ox_lo <= 0 && ox_hi >= 0) npairs -= 1;
      for (int d = 32; d >= 1; d >>= 1) npairs += __shfl_xor(npairs, d, 64);
      if (lane == 0) atomicAdd(pair_count, (unsigned long long)npairs);
    }
  }
}

template <int kAcc, bool kCount, int kU, bool kPipe, bool kDens>
static hipError_t launch_forward_t(const DevBox* boxes, const PlanWork& w, const int32_t* off,
                                   const float* rel, const float* src3, const int32_t* perm,
                                   float* acc, float* dens, int64_t* pair_count, int grid_mult,
                                   hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_pair_forward<kAcc, kCount, kU, kPipe, kDens>);
  const int resident = persistent_blocks(fn, 256);
  const int blocks = resident * grid_mult;
  hipLaunchKernelGGL((k_pair_forward<kAcc, kCount, kU, kPipe, kDens>), dim3(blocks), dim3(256), 0,
                     s, boxes, w.items, w.tasks, w.item_cost, w.ctrl, off, reinterpret_cast<const float4*>(rel),
                     src3, perm, acc, dens, w.partial,
                     reinterpret_cast<unsigned long long*>(pair_count), resident * 4);
  return hipGetLastError();
}

template <int kAcc, bool kCount, bool kDens>
static hipError_t dispatch_variant(const KernelConfig& cfg, const DevBox* boxes, const PlanWork& w,
                                   const int32_t* off, const float* rel, const float* src3,
                                   const int32_t* perm, float* acc, float* dens, int64_t* pc,
                                   hipStream_t s) {
  const int g = cfg.grid_mult;
  switch (cfg.unroll * 2 + (cfg.pipeline ? 1 : 0)) {
    case 4: return launch_forward_t<kAcc, kCount, 2, false, kDens>(boxes, w, off, rel, src3, perm, acc, dens, pc, g, s);
    case 5: return launch_forward_t<kAcc, kCount, 2, true, kDens>(boxes, w, off, rel, src3, perm, acc, dens, pc, g, s);
    case 9: return launch_forward_t<kAcc, kCount, 4, true, kDens>(boxes, w, off, rel, src3, perm, acc, dens, pc, g, s);
    case 16: return launch_forward_t<kAcc, kCount, 8, false, kDens>(boxes, w, off, rel, src3, perm, acc, dens, pc, g, s);
    case 17: return launch_forward_t<kAcc, kCount, 8, true, kDens>(boxes, w, off, rel, src3, perm, acc, dens, pc, g, s);
    default: return launch_forward_t<kAcc, kCount, 4, false, kDens>(boxes, w, off, rel, src3, perm, acc, dens, pc, g, s);
  }
}

template <int kAcc>
static hipError_t dispatch_mode(bool count_pairs, const KernelConfig& cfg, const DevBox* boxes,
                                const PlanWork& w, const int32_t* off, const float* rel,
                                const float* src3, const int32_t* perm, float* acc, float* dens,
                                int64_t* pc, hipStream_t s) {
  // The debug pair counter is a correctness tool: one fixed kernel variant, no density.
  if (count_pairs)
    return dispatch_variant<kAcc, true, false>(default_config(0), boxes, w, off, rel, src3, perm,
                                               acc, nullptr, pc, s);
  if (dens)
    return dispatch_variant<kAcc, false, true>(cfg, boxes, w, off, rel, src3, perm, acc, dens,
                                               nullptr, s);
  return dispatch_variant<kAcc, false, false>(cfg, boxes, w, off, rel, src3, perm, acc, nullptr,
                                              nullptr, s);
}

hipError_t launch_forward(AccMode mode, bool count_pairs, const KernelConfig& cfg,
                          const DevBox* boxes, const PlanWork& w, int64_t pencils,
                          const int32_t* off, const float* rel, const int32_t* perm, float* acc,
                          float* density, int64_t* pair_count, float* src3, int64_t n_total,
                          hipStream_t s) {
  (void)pencils;
  if (n_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_sources, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(rel), n_total, src3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (mode) {
    case kAccSingle: e = dispatch_mode<kAccSingle>(count_pairs, cfg, boxes, w, off, rel, src3, perm, acc, density, pair_count, s); break;
    case kAccChunked: e = dispatch_mode<kAccChunked>(count_pairs, cfg, boxes, w, off, rel, src3, perm, acc, density, pair_count, s); break;
    default: e = dispatch_mode<kAccCompensated>(count_pairs, cfg, boxes, w, off, rel, src3, perm, acc, density, pair_count, s); break;
  }
  if (e != hipSuccess) return e;
  return launch_combine(mode, false, boxes, w, perm, acc, density, s);
}

}  // namespace anf
