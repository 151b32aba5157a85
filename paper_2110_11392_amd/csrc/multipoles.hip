// Cell multipoles in the complete basis of order p (Eq. 4), and their
// reduction to (p+1)^2 values per cell.
//
// What it computes: for every cell, M^{a,b,c} = sum_q x_q^a y_q^b z_q^c over
// the cell's particles, (x, y, z) the displacement from the cell centre in box
// units, for a + b + c <= p (enumerated a outermost, c innermost).  The sums
// are FP64 (the paper keeps every far-field computation in double precision),
// formed from the stored FP32 cell-relative offsets.
//
// How it maps to CDNA4:
//   * each cell gets L lanes (a power of two, about n/16 of them, at most 64)
//     and each lane sums `per` = ceil(n/L) consecutive particles of the cell;
//   * cells are bucketed by (L, per) with a counting sort, and a work wave
//     takes 64/L cells of one bucket, so all 64 lanes of a wave do the same
//     number of particles -- the balance the paper gets from its "step-down"
//     remainder iterations;
//   * a wave stages its cells' offsets in LDS with straight-line coalesced
//     loads, all in flight together, in particle-row order (particle m of a
//     lane's segment at slot 64 m + lane), and requests the next work wave's
//     cell table before its own arithmetic; cells needing more than 16
//     particles per lane read global memory directly;
//   * a lane keeps its partial moments in FP64 VGPRs (passes of at most 56
//     terms, split by the power of x), then each cell's L lanes are added in
//     registers with DPP moves in a fixed pattern, so results are run-to-run
//     deterministic whatever wave a cell lands in;
//   * the last lane of each cell's block scales the sums by w^(a+b+c) and
//     writes them.
// The reduced basis is a second pass over the complete rows, staged in LDS.
#include "nf_internal.h"

namespace anf {

constexpr int kMpSeg = 16;     // target particles per lane
constexpr bool kMpUseLds = true;  // stage each wave's offsets in LDS
constexpr int kMpStage = kMpUseLds ? 64 * kMpSeg : 1;  // particles a wave stages in LDS
// Buckets: (log2 L, ceil(per / kMpPerStep)) for per <= kMpSeg, then one bucket
// of cells that need 64 lanes and more than kMpSeg particles per lane, then
// the empty cells.
constexpr int kMpPerLevels = 16;
constexpr int kMpPerStep = kMpSeg / kMpPerLevels;
static_assert(kMpSeg % kMpPerLevels == 0, "per-lane levels");
static_assert(!kMpUseLds || kMpPerStep == 1, "LDS staging needs the exact per-lane count");
constexpr int kMpGiant = 7 * (kMpPerLevels + 1);
constexpr int kMpEmpty = kMpGiant + 1;
static_assert(kMpEmpty + 2 <= kMpBuckets && kMpEmpty + 2 <= 256, "bucket arrays and scan");

__host__ __device__ constexpr int mp_terms_a(int p, int a0, int a1) {
  int t = 0;
  for (int a = a0; a <= a1; ++a) t += (p - a + 1) * (p - a + 2) / 2;
  return t;
}

// Passes over a lane's particles: the terms are split by the power of x into
// consecutive ranges of at most mp_max_acc terms (greedy), so the partial sums
// of one pass fit in VGPRs with room for three waves per SIMD and no spills
// (p = 8: 45 + 36 + 49 + 35 terms in four passes).
__host__ __device__ constexpr int mp_max_acc(int p) { return p < 0 ? 0 : 56; }

// First power of x of pass `k` (pass k covers [mp_pass_a0(p, k), mp_pass_a0(p, k+1) - 1]);
// p + 1 once the passes are exhausted.
__host__ __device__ constexpr int mp_pass_a0(int p, int k) {
  int a = 0;
  for (int pass = 0; pass < k && a <= p; ++pass) {
    int t = 0;
    const int start = a;
    while (a <= p && (a == start || t + (p - a + 1) * (p - a + 2) / 2 <= mp_max_acc(p))) {
      t += (p - a + 1) * (p - a + 2) / 2;
      ++a;
    }
  }
  return a;
}

int64_t multipole_terms(int p, bool reduced) {
  if (p < 0) return 0;
  return reduced ? (int64_t)(p + 1) * (p + 1) : (int64_t)mp_terms_a(p, 0, p);
}

// Lanes per cell: the power of two nearest above n / kMpSeg, at most 64.
__device__ __forceinline__ int mp_lanes_log2(int n) {
  const int want = (n + kMpSeg - 1) / kMpSeg;
  int l = 0;
  while (l < 6 && (1 << l) < want) ++l;
  return l;
}

__device__ __forceinline__ int mp_key(int n) {
  if (n <= 0) return kMpEmpty;
  const int l = mp_lanes_log2(n);
  const int per = (n + (1 << l) - 1) >> l;
  return per <= kMpSeg ? l * (kMpPerLevels + 1) + (per + kMpPerStep - 1) / kMpPerStep : kMpGiant;
}

// Lanes per cell of a bucket (the giant and empty buckets: 64 and 1).
__host__ __device__ constexpr int mp_key_lanes_log2(int key) {
  return key == kMpGiant ? 6 : (key == kMpEmpty ? 0 : key / (kMpPerLevels + 1));
}

// ---- planning: counting sort of the cells by bucket --------------------------

// A planning block covers 256 ppt cells (ppt per thread, 1..16, chosen so that
// there are about 256 blocks): the device-wide atomics on the bucket counters
// (one per block and non-empty bucket) stay few while every CU still gets work.
constexpr int kMpPlanPerThread = 16;

__global__ __launch_bounds__(256) void k_mp_classify(const int32_t* __restrict__ off,
                                                     int64_t cells, int ppt,
                                                     int32_t* __restrict__ key_out,
                                                     int32_t* __restrict__ hist) {
  __shared__ int local[kMpEmpty + 1];
  for (int k = threadIdx.x; k <= kMpEmpty; k += blockDim.x) local[k] = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kMpPlanPerThread; ++j) {
    const int64_t c = ((int64_t)blockIdx.x * ppt + j) * 256 + threadIdx.x;
    if (j < ppt && c < cells) {
      const int key = mp_key(off[c + 1] - off[c]);
      key_out[c] = key;
      atomicAdd(&local[key], 1);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= kMpEmpty; k += blockDim.x)
    if (local[k]) atomicAdd(&hist[k], local[k]);
}

// One block of 256 threads: bucket bases, cursors, and the first wave of every
// bucket (64 / L cells per wave), by two exclusive scans in LDS;
// base[kMpEmpty + 1] = cells, waves[kMpEmpty + 1] = total waves.
__global__ __launch_bounds__(256) void k_mp_buckets(const int32_t* __restrict__ hist,
                                                    int32_t* __restrict__ base,
                                                    int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ waves) {
  __shared__ int sc[256], sw[256];
  const int k = threadIdx.x;
  const int h = k <= kMpEmpty ? hist[k] : 0;
  const int per_wave = 64 >> mp_key_lanes_log2(k <= kMpEmpty ? k : 0);
  sc[k] = h;
  sw[k] = (h + per_wave - 1) / per_wave;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scans
    const int a = k >= d ? sc[k - d] : 0, b = k >= d ? sw[k - d] : 0;
    __syncthreads();
    sc[k] += a;
    sw[k] += b;
    __syncthreads();
  }
  if (k <= kMpEmpty + 1) {
    const int cb = k == 0 ? 0 : sc[k - 1], wb = k == 0 ? 0 : sw[k - 1];
    base[k] = cb;
    waves[k] = wb;
    if (k <= kMpEmpty) cursor[k] = cb;
  }
}

// Each block ranks its cells per bucket in LDS and reserves one range per
// bucket with a single global atomic (the order inside a bucket does not
// matter: every cell's sums are independent of its position).
__global__ __launch_bounds__(256) void k_mp_scatter(const int32_t* __restrict__ key_in,
                                                    const int32_t* __restrict__ off,
                                                    int64_t cells, int ppt,
                                                    int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ sorted,
                                                    int2* __restrict__ span) {
  __shared__ int cnt[kMpEmpty + 1], start[kMpEmpty + 1];
  for (int k = threadIdx.x; k <= kMpEmpty; k += blockDim.x) cnt[k] = 0;
  __syncthreads();
  int key[kMpPlanPerThread], rank[kMpPlanPerThread];
#pragma unroll
  for (int j = 0; j < kMpPlanPerThread; ++j) {
    const int64_t c = ((int64_t)blockIdx.x * ppt + j) * 256 + threadIdx.x;
    key[j] = -1;
    rank[j] = 0;
    if (j < ppt && c < cells) {
      key[j] = key_in[c];
      rank[j] = atomicAdd(&cnt[key[j]], 1);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= kMpEmpty; k += blockDim.x)
    start[k] = cnt[k] ? atomicAdd(&cursor[k], cnt[k]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kMpPlanPerThread; ++j) {
    if (key[j] >= 0) {
      const int64_t c = ((int64_t)blockIdx.x * ppt + j) * 256 + threadIdx.x;
      const int at = start[key[j]] + rank[j];
      sorted[at] = (int32_t)c;
      span[at] = make_int2(off[c], off[c + 1] - off[c]);
    }
  }
}

// ---- the moment kernel ----------------------------------------------------

struct MpShared {
  float x[kMpStage], y[kMpStage], z[kMpStage];  // the wave's staged offsets
};

// Add one particle's terms with x power in [A0, A1] to acc.
template <int P, int A0, int A1, int T>
__device__ __forceinline__ void mp_add(const float4 r, double (&acc)[T]) {
  const double x = r.x, y = r.y, z = r.z;
  double zp[P + 1];
  zp[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= P - A0; ++k) zp[k] = zp[k - 1] * z;
  double xa = 1.0;
#pragma unroll
  for (int a = 0; a < A0; ++a) xa *= x;
  int k = 0;
#pragma unroll
  for (int a = A0; a <= A1; ++a) {
    double m = xa;  // x^a y^b, b = 0, 1, ...
#pragma unroll
    for (int b = 0; b <= P - a; ++b) {
#pragma unroll
      for (int c = 0; c <= P - a - b; ++c) {
        acc[k] = c == 0 ? acc[k] + m : __builtin_fma(m, zp[c], acc[k]);
        ++k;
      }
      m *= y;
    }
    xa *= x;
  }
}

// A lane's share of its wave: particles [beg, end) of global cell `cell`
// (cell < 0: none), lane i of the cell's n = L lanes.
struct MpLane {
  int beg, end, cell, i, n;
  int lds;   // first staged slot of [beg, end), or -1 when read from global memory
  double w;  // cell width of the cell's box
};

template <int P, int A0, int A1>
__device__ __forceinline__ void mp_pass(const float4* __restrict__ rel, const MpLane& ln,
                                        MpShared& sh, int lane, int depth,
                                        double* __restrict__ out) {
  const int beg = ln.beg, end = ln.end;
  constexpr int T = mp_terms_a(P, A0, A1);
  constexpr int TT = mp_terms_a(P, 0, P);
  constexpr int base = A0 == 0 ? 0 : mp_terms_a(P, 0, A0 - 1);
  double acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = 0.0;
  // Particles in groups of kG, double-buffered: the loads of the next group
  // are issued before the arithmetic of the current one (scheduling barriers
  // keep the compiler from sinking them), so a group's memory latency hides
  // behind the previous group's arithmetic.  Indices are clamped to the
  // segment; a group past its end is redone by the tail loop.
  constexpr int kG = 2;
  const int last = end - 1;
  float ax[kG], ay[kG], az[kG], bx[kG], by[kG], bz[kG];
  const float* f = reinterpret_cast<const float*>(rel);
  auto load = [&](float (&x)[kG], float (&y)[kG], float (&z)[kG], int at) {
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int64_t q = 4 * (int64_t)(at + g < last ? at + g : last);
      x[g] = f[q];
      y[g] = f[q + 1];
      z[g] = f[q + 2];
    }
  };
  auto add = [&](const float (&x)[kG], const float (&y)[kG], const float (&z)[kG]) {
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      mp_add<P, A0, A1>(make_float4(x[g], y[g], z[g], 0.f), acc);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (kMpUseLds && ln.lds >= 0) {
    // The next particle's offsets are read from LDS before this particle's
    // terms are added, so the LDS latency hides behind the arithmetic.
    const int cnt = end - beg;
    const float* sx = sh.x + ln.lds;
    const float* sy = sh.y + ln.lds;
    const float* sz = sh.z + ln.lds;
    if (cnt > 0) {
      // Particle m of this lane's segment sits in row m: sx[64 m].  Two
      // register sets alternate (no copies, so a wait covers only the older
      // loads: LDS reads complete in order); the index is clamped to the
      // segment, and a load past its end is never used.
      float ax = sx[0], ay = sy[0], az = sz[0];
      int m = 0;
      for (; m + 1 < cnt; m += 2) {
        const float bx = sx[64 * (m + 1)], by = sy[64 * (m + 1)], bz = sz[64 * (m + 1)];
        __builtin_amdgcn_sched_barrier(0);
        mp_add<P, A0, A1>(make_float4(ax, ay, az, 0.f), acc);
        __builtin_amdgcn_sched_barrier(0);
        const int k = m + 2 < cnt ? m + 2 : m + 1;
        ax = sx[64 * k];
        ay = sy[64 * k];
        az = sz[64 * k];
        __builtin_amdgcn_sched_barrier(0);
        mp_add<P, A0, A1>(make_float4(bx, by, bz, 0.f), acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (m < cnt) mp_add<P, A0, A1>(make_float4(ax, ay, az, 0.f), acc);
    }
  } else {
  int j = beg;
  if (j + kG <= end) {
    load(ax, ay, az, j);
    while (true) {
      load(bx, by, bz, j + kG);
      __builtin_amdgcn_sched_barrier(0);
      add(ax, ay, az);
      j += kG;
      if (j + kG > end) break;
      load(ax, ay, az, j + kG);
      __builtin_amdgcn_sched_barrier(0);
      add(bx, by, bz);
      j += kG;
      if (j + kG > end) break;
    }
  }
  for (; j < end; ++j) mp_add<P, A0, A1>(rel[j], acc);
  }
  // Add each cell's L lanes in registers over its aligned block of lanes with
  // DPP moves (no LDS round trips): partner lane i^1, then i^2 (quad
  // permutes), the mirrored half-row and the mirrored row, after which every
  // lane of a block of up to 16 holds the block's sum; for 32 and 64 lanes the
  // row broadcasts add rows 0 and 2 into rows 1 and 3, then rows 0-1 into rows
  // 2-3.  The block's last lane then holds the sum in a fixed order (a + b and
  // b + a round alike, so all holders agree), scales it by w^(a+b+c) and
  // writes the row.  An empty cell's lane writes zeros.
  if (depth >= 1) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += dpp_f64<0xB1, 0xF>(acc[t]);   // quad_perm [1,0,3,2]
  }
  if (depth >= 2) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += dpp_f64<0x4E, 0xF>(acc[t]);   // quad_perm [2,3,0,1]
  }
  if (depth >= 3) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += dpp_f64<0x141, 0xF>(acc[t]);  // row_half_mirror
  }
  if (depth >= 4) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += dpp_f64<0x140, 0xF>(acc[t]);  // row_mirror
  }
  if (depth >= 5) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += dpp_f64<0x142, 0xA>(acc[t]);  // row_bcast:15 -> rows 1, 3
  }
  if (depth >= 6) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] += dpp_f64<0x143, 0xC>(acc[t]);  // row_bcast:31 -> rows 2, 3
  }
  if (ln.cell >= 0 && ln.i == ln.n - 1) {
    double* dst = out + (int64_t)ln.cell * TT + base;
    double wp[P + 1];
    wp[0] = 1.0;
#pragma unroll
    for (int o = 1; o <= P; ++o) wp[o] = wp[o - 1] * ln.w;
    int k = 0;
#pragma unroll
    for (int a = A0; a <= A1; ++a)
#pragma unroll
      for (int b = 0; b <= P - a; ++b)
#pragma unroll
        for (int c = 0; c <= P - a - b; ++c) {
          dst[k] = acc[k] * wp[a + b + c];
          ++k;
        }
  }
}

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_multipoles(
    const DevBox* __restrict__ boxes, int nboxes, const int32_t* __restrict__ bucket_base,
    const int32_t* __restrict__ bucket_waves, const int32_t* __restrict__ sorted,
    const int2* __restrict__ span, const float4* __restrict__ rel, double* __restrict__ out) {
  __shared__ MpShared sh;
  constexpr int S1 = mp_pass_a0(P, 1), S2 = mp_pass_a0(P, 2), S3 = mp_pass_a0(P, 3);
  static_assert(mp_pass_a0(P, 4) > P, "at most four passes");
  static_assert(P <= 8, "order table sized for p <= 8");
  const int lane = threadIdx.x;
  const int n_waves = __builtin_amdgcn_readfirstlane(bucket_waves[kMpEmpty + 1]);
  // A work wave takes the sorted cells [first, first + ncell) of one bucket;
  // lane k < ncell holds cell k's id and (first particle, count).  The next
  // work wave's cells are requested before this one's arithmetic, so their
  // memory latency overlaps it.
  int key = 0, ncell = 0, my_c = -1;
  int2 my_sp = make_int2(0, 0);
  auto fetch = [&](int wv) {
    int lo = 0, hi = kMpEmpty;  // the bucket of wave wv: the last k with bucket_waves[k] <= wv
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (__builtin_amdgcn_readfirstlane(bucket_waves[mid]) <= wv) lo = mid; else hi = mid - 1;
    }
    key = lo;
    const int per_wave = 64 >> mp_key_lanes_log2(key);
    const int first = __builtin_amdgcn_readfirstlane(bucket_base[key]) +
                      (wv - __builtin_amdgcn_readfirstlane(bucket_waves[key])) * per_wave;
    const int lim = __builtin_amdgcn_readfirstlane(bucket_base[key + 1]);
    ncell = lim - first < per_wave ? lim - first : per_wave;
    my_c = -1;
    my_sp = make_int2(0, 0);
    if (lane < ncell) {
      my_c = sorted[first + lane];
      my_sp = span[first + lane];
    }
  };
  if ((int)blockIdx.x < n_waves) fetch(blockIdx.x);
  for (int wv = blockIdx.x; wv < n_waves; wv += gridDim.x) {
    const int cur_key = key, cur_ncell = ncell, cur_c = my_c;
    const int2 cur_sp = my_sp;
    if (wv + (int)gridDim.x < n_waves) fetch(wv + gridDim.x);
    const int l2 = mp_key_lanes_log2(cur_key);
    const int L = 1 << l2;
    const int k = lane >> l2;  // this lane's cell within the wave
    const int c = __shfl(cur_c, k, 64);
    const int cb = __shfl(cur_sp.x, k, 64), cn = __shfl(cur_sp.y, k, 64);
    MpLane ln = {0, 0, -1, lane & (L - 1), L, -1, 0.0};
    if (k < cur_ncell) {
      const int per = (cn + L - 1) >> l2;
      const int ce = cb + cn;
      ln.beg = cb + ln.i * per < ce ? cb + ln.i * per : ce;
      ln.end = ln.beg + per < ce ? ln.beg + per : ce;
      ln.cell = c;
      const int b = nboxes == 1 ? 0 : find_box_by_cell(boxes, nboxes, c);
      ln.w = boxes[b].width;
    }
    if (kMpUseLds && cur_key < kMpGiant) {
      // Stage the wave's cells in LDS, one row of 64 slots per particle index
      // within a segment: particle m of cell k belongs to segment lane
      // k L + m / per, row m % per, slot 64 row + lane, so a lane's reads in
      // the passes walk one column and the 64 lanes read 64 consecutive
      // words (no bank conflicts).  Particle slot + 64 j of the wave's cells
      // (in cell order, cell k starting at k L per) is fetched by lane `lane`
      // in step j; all steps' loads are in flight together.
      const int per = cur_key - l2 * (kMpPerLevels + 1);
      const int stride = L * per;
      // Straight-line code: every step loads (slots past the wave's cells
      // re-read the wave's first particle) and only real slots are stored.
      const int safe = __shfl(cur_sp.x, 0, 64);
      float4 r[kMpSeg];
      int dst[kMpSeg];
      int slot_ok = 0;
#pragma unroll
      for (int j = 0; j < kMpSeg; ++j) {
        const int slot = lane + 64 * j;
        const int kk = slot / stride;
        const int m = slot - kk * stride;
        const int cbk = __shfl(cur_sp.x, kk & 63, 64), nk = __shfl(cur_sp.y, kk & 63, 64);
        const bool ok = j < per && kk < cur_ncell && m < nk;
        r[j] = rel[ok ? cbk + m : safe];
        const int q = m / per;
        dst[j] = 64 * (m - q * per) + kk * L + q;
        slot_ok |= ok ? 1 << j : 0;
      }
#pragma unroll
      for (int j = 0; j < kMpSeg; ++j) {
        if (slot_ok & (1 << j)) {
          sh.x[dst[j]] = r[j].x;
          sh.y[dst[j]] = r[j].y;
          sh.z[dst[j]] = r[j].z;
        }
      }
      if (ln.cell >= 0) ln.lds = lane;
    }
    __syncthreads();
    mp_pass<P, 0, S1 - 1>(rel, ln, sh, lane, l2, out);
    if constexpr (S1 <= P) mp_pass<P, S1, S2 - 1>(rel, ln, sh, lane, l2, out);
    if constexpr (S2 <= P) mp_pass<P, S2, S3 - 1>(rel, ln, sh, lane, l2, out);
    if constexpr (S3 <= P) mp_pass<P, S3, P>(rel, ln, sh, lane, l2, out);
    __syncthreads();  // the next wave's staging overwrites the slots
  }
}

// ---- reduction to (p+1)^2 values -------------------------------------------
// R^{a,b,c0} = sum_{m, i} (-1)^m C(m, i) a! b! c0! / ((a-2i)! (b-2m+2i)! (c0+2m)!)
//              M^{a-2i, b-2m+2i, c0+2m},
// so that the exterior expansion sum (-1)^n M^{abc}/(a!b!c!) D_{abc} keeps its
// value with D_{a,b,c+2} = -D_{a+2,b,c} - D_{a,b+2,c} (1/r is harmonic).

__device__ __forceinline__ int mp_index(int p, int a, int b, int c) {
  // position of (a, b, c) in the complete enumeration (a outermost)
  int k = 0;
  for (int aa = 0; aa < a; ++aa) k += (p - aa + 1) * (p - aa + 2) / 2;
  for (int bb = 0; bb < b; ++bb) k += p - a - bb + 1;
  return k + c;
}

__device__ __forceinline__ double mp_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

// The reduction table: for each reduced term r its sources (complete-basis
// indices) and coefficients, at most 15 each for p <= 8.  One block writes it
// once per call.
constexpr int kMpRedSrc = 16;
constexpr int kMpRedCells = 16;

__global__ __launch_bounds__(128) void k_mp_reduce_table(int p, double* __restrict__ coef,
                                                         int32_t* __restrict__ src,
                                                         int32_t* __restrict__ cnt) {
  __shared__ double fact[2 * kMaxMultipoleOrder + 1];  // n! for n <= 2p (exact in FP64)
  if ((int)threadIdx.x <= 2 * kMaxMultipoleOrder) fact[threadIdx.x] = mp_fact((int)threadIdx.x);
  __syncthreads();
  const int RT = (p + 1) * (p + 1);
  for (int r = threadIdx.x; r < RT; r += blockDim.x) {
    // decode reduced term r -> (a, b, c0), enumerated a, b, then c0 in {0, 1}
    int rr = r, a = 0, b = 0;
    for (a = 0; a <= p; ++a) {
      int here = 0;
      for (int bb = 0; bb <= p - a; ++bb) here += (p - a - bb >= 1) ? 2 : 1;
      if (rr < here) break;
      rr -= here;
    }
    for (b = 0; b <= p - a; ++b) {
      const int here = (p - a - b >= 1) ? 2 : 1;
      if (rr < here) break;
      rr -= here;
    }
    const int c0 = rr;
    int n = 0;
    for (int m = 0; 2 * m <= a + b; ++m)
      for (int i = 0; i <= m; ++i) {
        const int sa = a - 2 * i, sb = b - 2 * (m - i), sc = c0 + 2 * m;
        if (sa < 0 || sb < 0) continue;
        coef[r * kMpRedSrc + n] = ((m & 1) ? -1.0 : 1.0) *
                                  (fact[m] / (fact[i] * fact[m - i])) * fact[a] * fact[b] *
                                  fact[c0] / (fact[sa] * fact[sb] * fact[sc]);
        src[r * kMpRedSrc + n] = mp_index(p, sa, sb, sc);
        ++n;
      }
    cnt[r] = n;
  }
}

// Each thread owns one reduced term r (its table entries in registers) and a
// group of cells; the block walks chunks of kMpRedCells consecutive cells,
// whose complete rows (contiguous in memory) are first copied into LDS with
// coalesced loads.  Threads r = 0..RT-1 of a group write one cell's reduced
// row, consecutive in memory.
__global__ __launch_bounds__(256) void k_mp_reduce(const double* __restrict__ full, int p,
                                                   int64_t cells,
                                                   const double* __restrict__ tab_coef,
                                                   const int32_t* __restrict__ tab_src,
                                                   const int32_t* __restrict__ tab_cnt,
                                                   double* __restrict__ out) {
  __shared__ double rows[kMpRedCells * 165];
  const int RT = (p + 1) * (p + 1);
  const int TT = mp_terms_a(p, 0, p);
  const int groups = (int)blockDim.x / RT;
  const int t = threadIdx.x;
  const int r = t % RT, g = t / RT;
  const bool active = g < groups;
  double cf[kMpRedSrc];
  int sr[kMpRedSrc];
  const int n = active ? tab_cnt[r] : 0;
#pragma unroll
  for (int e = 0; e < kMpRedSrc; ++e) {
    cf[e] = e < n ? tab_coef[r * kMpRedSrc + e] : 0.0;
    sr[e] = e < n ? tab_src[r * kMpRedSrc + e] : 0;
  }
  const int64_t chunks = (cells + kMpRedCells - 1) / kMpRedCells;
  for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
    const int64_t c0 = ch * kMpRedCells;
    const int nc = (int)(cells - c0 < kMpRedCells ? cells - c0 : kMpRedCells);
    __syncthreads();  // the previous chunk's rows are consumed
    const double* in = full + c0 * TT;
    for (int k = t; k < nc * TT; k += blockDim.x) rows[k] = in[k];
    __syncthreads();
    if (active) {
      double* dst = out + c0 * RT;
      for (int cl = g; cl < nc; cl += groups) {
        const double* row = rows + cl * TT;
        double sum = 0.0;
#pragma unroll
        for (int e = 0; e < kMpRedSrc; ++e)
          if (e < n) sum += cf[e] * row[sr[e]];
        dst[cl * RT + r] = sum;
      }
    }
  }
}

// ---- host launch -------------------------------------------------------------

template <int P>
static hipError_t launch_mp_t(const DevBox* boxes, int nboxes, const MpWork& w,
                              const int32_t* off, const float* rel, double* full, hipStream_t s) {
  (void)off;  // the cells' particle ranges come from the planner's span table
  const void* fn = reinterpret_cast<const void*>(&k_multipoles<P>);
  int blocks = persistent_blocks(fn, 64);
  if ((int64_t)blocks > w.cells) blocks = (int)(w.cells > 0 ? w.cells : 1);
  hipLaunchKernelGGL(k_multipoles<P>, dim3(blocks), dim3(64), 0, s, boxes, nboxes, w.bucket_base,
                     w.bucket_waves, w.sorted, w.span, reinterpret_cast<const float4*>(rel), full);
  return hipGetLastError();
}

hipError_t launch_multipoles(const DevBox* boxes, int nboxes, int64_t cells_total, int order,
                             bool reduced, const MpWork& w, const int32_t* off, const float* rel,
                             double* out, hipStream_t s) {
  if (cells_total <= 0) return hipSuccess;
  hipError_t e = fill_i32(w.hist, 0, kMpBuckets, s);
  if (e != hipSuccess) return e;
  int64_t ppt = cells_total / (256 * 256);
  ppt = ppt < 1 ? 1 : (ppt > kMpPlanPerThread ? kMpPlanPerThread : ppt);
  const unsigned cg = (unsigned)((cells_total + 256 * ppt - 1) / (256 * ppt));
  hipLaunchKernelGGL(k_mp_classify, dim3(cg), dim3(256), 0, s, off, cells_total, (int)ppt, w.keys,
                     w.hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mp_buckets, dim3(1), dim3(256), 0, s, w.hist, w.bucket_base, w.cursor,
                     w.bucket_waves);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mp_scatter, dim3(cg), dim3(256), 0, s, w.keys, off, cells_total, (int)ppt,
                     w.cursor, w.sorted, w.span);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double* full = reduced ? w.full : out;
  switch (order) {
    case 0: e = launch_mp_t<0>(boxes, nboxes, w, off, rel, full, s); break;
    case 1: e = launch_mp_t<1>(boxes, nboxes, w, off, rel, full, s); break;
    case 2: e = launch_mp_t<2>(boxes, nboxes, w, off, rel, full, s); break;
    case 3: e = launch_mp_t<3>(boxes, nboxes, w, off, rel, full, s); break;
    case 4: e = launch_mp_t<4>(boxes, nboxes, w, off, rel, full, s); break;
    case 5: e = launch_mp_t<5>(boxes, nboxes, w, off, rel, full, s); break;
    case 6: e = launch_mp_t<6>(boxes, nboxes, w, off, rel, full, s); break;
    case 7: e = launch_mp_t<7>(boxes, nboxes, w, off, rel, full, s); break;
    default: e = launch_mp_t<8>(boxes, nboxes, w, off, rel, full, s); break;
  }
  if (e != hipSuccess || !reduced) return e;
  hipLaunchKernelGGL(k_mp_reduce_table, dim3(1), dim3(128), 0, s, order, w.red_coef, w.red_src,
                     w.red_cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t blocks = (cells_total + kMpRedCells - 1) / kMpRedCells;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_mp_reduce, dim3((unsigned)blocks), dim3(256), 0, s, w.full, order,
                     cells_total, w.red_coef, w.red_src, w.red_cnt, out);
  return hipGetLastError();
}

}  // namespace anf
