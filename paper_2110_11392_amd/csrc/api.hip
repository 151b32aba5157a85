// C ABI of libabacus_nf: argument validation, parameter resolution, workspace
// layout, launch sequencing and the measurement hooks.  No device memory is
// allocated here; every call enqueues work on the caller's stream.
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nf_internal.h"

using namespace anf;

namespace {

thread_local std::string g_last_hip_error;

constexpr int64_t kMaxIndex = (int64_t(1) << 31) - 1;
constexpr int kMaxBoxes = 65535;
// Sec. 3.2: the spline softening length is 2.16 times the Plummer-equivalent one.
constexpr double kSplineOverPlummer = 2.16;

int hip_fail(hipError_t e, const char* what) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
  g_last_hip_error = buf;
  return ABACUS_NF_EHIP;
}

#define ANF_HIP(call, what)                           \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, what);  \
  } while (0)

struct Resolved {
  std::vector<DevBox> boxes;
  int64_t n_total = 0, cells_total = 0, pencils_total = 0, max_box_n = 0;
  // 2R+1 when every box shares one near-field radius R <= 3 (tail items can be
  // split into one task per x offset), else 1.
  int split_slices = 1;
  // every box carries a density radius, so the density estimate can be asked for
  bool density_ok = true;
  bool plummer = false;  // Eq. 2 instead of Eq. 3
  int64_t kdk_chunks = 0;  // statistics chunks over all boxes
};

// Step a1: validate every box and derive the kernel constants.
int resolve(const abacus_nf_box* in, int nboxes, Resolved* out, bool plummer = false) {
  if (!in || nboxes < 1 || nboxes > kMaxBoxes) return ABACUS_NF_EINVAL;
  out->boxes.resize(nboxes);
  out->plummer = plummer;
  int64_t n_total = 0, cells_total = 0, pencils_total = 0, max_n = 0;
  for (int b = 0; b < nboxes; ++b) {
    const abacus_nf_box& x = in[b];
    if (x.n < 0) return ABACUS_NF_EINVAL;
    if (!(x.box > 0.0) || !std::isfinite(x.box)) return ABACUS_NF_EINVAL;
    if (x.radius < 0 || x.cpd < 2 * (int64_t)x.radius + 1) return ABACUS_NF_EINVAL;
    if (!(x.eps_plummer > 0.0) || !std::isfinite(x.eps_plummer)) return ABACUS_NF_EINVAL;
    const int64_t K = x.cpd;
    if (K > kMaxCellsPerDim) return ABACUS_NF_ERANGE;
    const int64_t cells = K * K * K;
    const double cpl = (double)K / x.box;
    const double eps_s = kSplineOverPlummer * x.eps_plummer;
    const double e = eps_s * cpl;  // softening in cell widths
    if (!(e >= 1e-6) || !(e <= 1e6)) return ABACUS_NF_EINVAL;
    const double iw2 = cpl * cpl, iw3 = cpl * cpl * cpl;
    if (!std::isfinite(cpl) || !(iw3 < (double)FLT_MAX) || !(iw2 > (double)FLT_MIN))
      return ABACUS_NF_EINVAL;
    DevBox& d = out->boxes[b];
    std::memset(&d, 0, sizeof(d));
    d.first = n_total;
    d.n = x.n;
    d.sink_x0 = 0;
    d.sink_x1 = (int32_t)K;
    d.cell_base = (int32_t)cells_total;
    d.K = (int32_t)K;
    d.R = x.radius;
    d.pencil_base = (int32_t)pencils_total;
    d.cells_per_len = cpl;
    d.width = x.box / (double)K;
    d.box_len = x.box;
    d.chunk_base = (int32_t)out->kdk_chunks;
    out->kdk_chunks += (cells + kKdkChunk - 1) / kKdkChunk;
    d.inv_w2 = (float)iw2;
    d.inv_w3 = (float)iw3;
    d.c0 = (float)(10.0 / (e * e * e));
    d.c1 = (float)(-15.0 / (e * e * e * e));
    d.c2 = (float)(6.0 / (e * e * e * e * e));
    d.eps = (float)e;
    d.near2 = (float)(1.21 * e * e);
    d.ha = (float)(12.0 / (e * e * e * e * e));
    d.hb = (float)(-15.0 / (e * e * e * e));
    if (plummer) {
      // Eq. 2: f = (r^2 + eps_p^2)^(-3/2) for every pair, eps_p as given
      const double ep = x.eps_plummer * cpl;
      d.far_mode = kFarAll;
      d.guard = (float)(ep * ep);
      d.eps_cells64 = ep;
    } else {
      d.eps_cells64 = e;
      // Points of cells two apart on an axis are >= 1 cell apart; with eps below
      // half a cell no rounding can bring such a pair inside eps.
      d.far_mode = e < 0.5 ? kFarApart : kFarNone;
      d.guard = kTinyR2;
    }
    // Optional density radius b: 0 < b <= R cell widths, so that every pair
    // within b is a near-field pair.
    if (x.density_radius != 0.0) {
      const double bh = x.density_radius * cpl;
      if (!(x.density_radius > 0.0) || !std::isfinite(x.density_radius) ||
          !(bh <= (double)x.radius) || !(bh * bh >= 1e-30))
        return ABACUS_NF_EINVAL;
      d.b2 = (float)(bh * bh + (double)d.guard);
      d.inv_b2 = (float)(1.0 / (bh * bh));
      d.dens_far = bh < 0.5 ? 1 : 0;
    } else {
      out->density_ok = false;
    }
    n_total += x.n;
    cells_total += cells;
    pencils_total += K * K;
    if (x.n > max_n) max_n = x.n;
    if (n_total > kMaxIndex || cells_total >= kMaxIndex) return ABACUS_NF_ERANGE;
  }
  int split_slices = 2 * in[0].radius + 1;
  for (int b = 1; b < nboxes; ++b)
    if (in[b].radius != in[0].radius) split_slices = 1;
  out->split_slices = split_slices <= kMaxSlices ? split_slices : 1;
  // Work items are queued as item << kTaskShift | code in an int32.
  if (plan_max_items(n_total, cells_total, pencils_total) >= ((int64_t)1 << (31 - kTaskShift)))
    return ABACUS_NF_ERANGE;
  out->n_total = n_total;
  out->cells_total = cells_total;
  out->pencils_total = pencils_total;
  out->max_box_n = max_n;
  return ABACUS_NF_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Tail items split per launch of abacus_nf_forces_noalloc (their slice
// partials take 9 MB of its scratch at 2R + 1 = 5 slices).
constexpr int64_t kNoAllocMaxSplit = 1024;

struct Layout {
  // shared
  size_t boxtab;
  // binning region
  size_t keys0, keys1, vals0, vals1, hist, hist_scan, bin_scan;
  // force / adjoint region (overlaps the binning region)
  size_t pencil_counts, item_base, items, item_bucket, item_slot, item_cost, tasks, ctrl, plan_scan,
      partial, mom,
      src_w;
  size_t total;
  int64_t max_items, max_tasks, max_split;
};

// Workspace layout.  `forward_only` lays out just what abacus_nf_forces needs
// (no binning region, 12-byte source records) for the static scratch of
// abacus_nf_forces_noalloc.
Layout layout(const Resolved& r, bool forward_only = false) {
  Layout L;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + (bytes ? bytes : 1));
    return at;
  };
  L.boxtab = take(sizeof(DevBox) * r.boxes.size());
  const size_t region = o;
  const int64_t n = r.n_total, c = r.cells_total;
  L.keys0 = L.keys1 = L.vals0 = L.vals1 = L.hist = L.hist_scan = L.bin_scan = 0;
  if (!forward_only) {
    const int64_t rb = radix_blocks(n);
    L.keys0 = take(4 * (size_t)n);
    L.keys1 = take(4 * (size_t)n);
    L.vals0 = take(4 * (size_t)n);
    L.vals1 = take(4 * (size_t)n);
    L.hist = take(4 * (size_t)(256 * rb));
    L.hist_scan = take(4 * (size_t)(256 * rb + 1));
    int64_t scan_n = c > 256 * rb ? c : 256 * rb;
    L.bin_scan = take(4 * (size_t)scan_tmp_ints(scan_n));
  }
  const size_t bin_end = o;
  o = region;
  L.max_items = plan_max_items(n, c, r.pencils_total);
  L.pencil_counts = take(4 * (size_t)r.pencils_total);
  L.item_base = take(4 * (size_t)(r.pencils_total + 1));
  L.items = take(sizeof(int4) * (size_t)L.max_items);
  L.item_bucket = take(4 * (size_t)L.max_items);
  L.item_slot = take(4 * (size_t)L.max_items);
  L.item_cost = take(4 * (size_t)L.max_items);
  // (the forward-only layout keeps room for fewer split tail items: splitting
  // changes which task sums a slice, never the result)
  L.max_split = r.split_slices > 1
                    ? std::min<int64_t>(forward_only ? kNoAllocMaxSplit : kMaxSplit, L.max_items)
                    : 0;
  L.max_tasks = plan_max_tasks(L.max_items, L.max_split);
  L.tasks = take(4 * (size_t)L.max_tasks);
  L.ctrl = take(4 * (size_t)kCtrlInts);
  L.partial = take(sizeof(float) * kPartialStride * kTile * (size_t)(L.max_split * r.split_slices));
  L.plan_scan = take(4 * (size_t)scan_tmp_ints(r.pencils_total));
  L.mom = take(sizeof(double) * 4 * kMomChunks * r.boxes.size());
  // packed source records: 6 floats for the adjoint, 3 for the forward kernel
  L.src_w = take((forward_only ? 3 : 6) * sizeof(float) * (size_t)n);
  const size_t force_end = o;
  L.total = bin_end > force_end ? bin_end : force_end;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

int check_ws(void* ws, size_t ws_bytes, const Layout& L) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0 || ws_bytes < L.total)
    return ABACUS_NF_EWORKSPACE;
  return ABACUS_NF_OK;
}

int acc_mode(uint32_t flags, AccMode* mode) {
  const uint32_t known = ABACUS_NF_SINGLE_ACC | ABACUS_NF_CHUNKED | ABACUS_NF_COMPENSATED |
                         ABACUS_NF_COUNT_PAIRS | ABACUS_NF_PLUMMER;
  if (flags & ~known) return ABACUS_NF_EINVAL;
  const uint32_t acc = flags & (ABACUS_NF_SINGLE_ACC | ABACUS_NF_CHUNKED | ABACUS_NF_COMPENSATED);
  if (acc == 0 || acc == ABACUS_NF_COMPENSATED) *mode = kAccCompensated;
  else if (acc == ABACUS_NF_CHUNKED) *mode = kAccChunked;
  else if (acc == ABACUS_NF_SINGLE_ACC) *mode = kAccSingle;
  else return ABACUS_NF_EINVAL;
  return ABACUS_NF_OK;
}

TuneKey tune_key(const abacus_nf_box* boxes, int nboxes, const Resolved& r, AccMode mode,
                 int kernel) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  for (int b = 0; b < nboxes; ++b) {
    mix(&boxes[b].n, sizeof(boxes[b].n));
    mix(&boxes[b].box, sizeof(boxes[b].box));
    mix(&boxes[b].cpd, sizeof(boxes[b].cpd));
    mix(&boxes[b].radius, sizeof(boxes[b].radius));
    mix(&boxes[b].eps_plummer, sizeof(boxes[b].eps_plummer));
  }
  TuneKey k;
  k.kernel = kernel;
  k.mode = (uint32_t)mode | (r.plummer ? 0x100u : 0u);
  k.nboxes = nboxes;
  k.n_total = r.n_total;
  k.cells_total = r.cells_total;
  k.shape_hash = h;
  return k;
}

// ---- measurement hooks ----------------------------------------------------
struct TimedLaunch {
  int kernel;
  hipEvent_t start, stop;
};
std::mutex g_timing_mu;
bool g_timing = false;
std::vector<TimedLaunch> g_pending;
constexpr int kTimerSlots = 6;  // forward, adjoint, bin, plan, multipoles, kick-drift
double g_ms[kTimerSlots] = {};
int64_t g_launches[kTimerSlots] = {};

struct Timer {
  int kernel;
  hipStream_t stream;
  hipEvent_t start = nullptr, stop = nullptr;
  bool on = false;
  Timer(int k, hipStream_t s) : kernel(k), stream(s) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (!g_timing) return;
    if (hipEventCreate(&start) != hipSuccess || hipEventCreate(&stop) != hipSuccess) return;
    on = hipEventRecord(start, stream) == hipSuccess;
  }
  void done() {
    if (!on) return;
    if (hipEventRecord(stop, stream) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    g_pending.push_back({kernel, start, stop});
    on = false;
  }
};

void drain_timing() {
  for (auto& t : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.stop) == hipSuccess &&
        hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
      g_ms[t.kernel] += ms;
      g_launches[t.kernel] += 1;
    }
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  g_pending.clear();
}

// Tail items to split for this launch: about one per resident wave.
int64_t split_items_for(const KernelConfig& c, AccMode mode, const Resolved& r, const Layout& L) {
  if (!c.split || mode == kAccSingle || r.split_slices < 2) return 0;
  return std::min<int64_t>(L.max_split, resident_wave_capacity());
}

PlanWork plan_work(void* ws, const Layout& L) {
  PlanWork w;
  w.pencil_counts = at<int32_t>(ws, L.pencil_counts);
  w.item_base = at<int32_t>(ws, L.item_base);
  w.items = at<int4>(ws, L.items);
  w.item_bucket = at<int32_t>(ws, L.item_bucket);
  w.item_slot = at<int32_t>(ws, L.item_slot);
  w.item_cost = at<int32_t>(ws, L.item_cost);
  w.tasks = at<int32_t>(ws, L.tasks);
  w.ctrl = at<int32_t>(ws, L.ctrl);
  w.partial = at<float>(ws, L.partial);
  w.scan_tmp = at<int32_t>(ws, L.plan_scan);
  w.max_items = L.max_items;
  w.max_tasks = L.max_tasks;
  w.max_split = L.max_split;
  w.split_items = 0;
  return w;
}

// The per-particle arrays may be NULL when there are no particles.
bool binned_ok(const abacus_nf_binned* b, int64_t n_total) {
  return b && b->cell_offsets && b->status && (n_total == 0 || (b->perm && b->rel));
}

int forces_args(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                const float* acc, const float* density, const int64_t* pair_count,
                uint32_t flags, Resolved* r, AccMode* mode);
int forces_launch(const abacus_nf_box* boxes, int nboxes, const Resolved& r, AccMode mode,
                  bool count, const abacus_nf_binned* b, float* acc, float* density,
                  double* momentum, int64_t* pair_count, void* ws, const Layout& L,
                  hipStream_t s);
int vjp_call(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b, bool slab,
             int32_t x0, int32_t x1, const float* wv, float* grad, uint32_t flags, void* ws,
             size_t ws_bytes, void* stream);
int set_sink_slabs(Resolved* r, int32_t x0, int32_t x1);

// ---- the static scratch of abacus_nf_forces_noalloc -----------------------
// Every GPU the library runs on holds its own copy of this array until the
// process ends.  Host code never uses the array's name as an address (on the
// host it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// that pointer is what the kernels receive.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> device address of `scratch`

int noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  const auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return ABACUS_NF_OK;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
    g_last_hip_error = "hipGetSymbolAddress(scratch): null or misaligned address";
    return ABACUS_NF_EHIP;
  }
  g_scratch_ptr[dev] = p;
  *out = p;
  return ABACUS_NF_OK;
}

}  // namespace

extern "C" {

int abacus_nf_layout(const abacus_nf_box* boxes, int nboxes, int64_t* n_total,
                     int64_t* cells_total) {
  Resolved r;
  const int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  if (n_total) *n_total = r.n_total;
  if (cells_total) *cells_total = r.cells_total;
  return ABACUS_NF_OK;
}

int abacus_nf_workspace_bytes(const abacus_nf_box* boxes, int nboxes, size_t* bytes) {
  if (!bytes) return ABACUS_NF_EINVAL;
  Resolved r;
  const int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  *bytes = layout(r).total;
  return ABACUS_NF_OK;
}

int abacus_nf_bin(const abacus_nf_box* boxes, int nboxes, const float* pos,
                  const abacus_nf_binned* out, void* ws, size_t ws_bytes, void* stream) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  if (!binned_ok(out, r.n_total) || (r.n_total > 0 && !pos)) return ABACUS_NF_EINVAL;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  BinWork w;
  w.keys[0] = at<int32_t>(ws, L.keys0);
  w.keys[1] = at<int32_t>(ws, L.keys1);
  w.vals[0] = at<int32_t>(ws, L.vals0);
  w.vals[1] = at<int32_t>(ws, L.vals1);
  w.hist = at<int32_t>(ws, L.hist);
  w.hist_scan = at<int32_t>(ws, L.hist_scan);
  w.scan_tmp = at<int32_t>(ws, L.bin_scan);
  Timer t(2, s);
  ANF_HIP(launch_bin(dboxes, nboxes, r.n_total, r.cells_total, pos, out, w, s), "binning");
  t.done();
  return ABACUS_NF_OK;
}

int abacus_nf_forces(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                     float* acc, float* density, double* momentum, int64_t* pair_count,
                     uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  Resolved r;
  AccMode mode;
  int rc = forces_args(boxes, nboxes, b, acc, density, pair_count, flags, &r, &mode);
  if (rc) return rc;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  return forces_launch(boxes, nboxes, r, mode, (flags & ABACUS_NF_COUNT_PAIRS) != 0, b, acc,
                       density, momentum, pair_count, ws, L, static_cast<hipStream_t>(stream));
}

int abacus_nf_forces_noalloc(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                             float* acc, float* density, double* momentum, int64_t* pair_count,
                             uint32_t flags, void* stream) {
  Resolved r;
  AccMode mode;
  int rc = forces_args(boxes, nboxes, b, acc, density, pair_count, flags, &r, &mode);
  if (rc) return rc;
  const Layout L = layout(r, true);
  if (L.total > kNoAllocScratchBytes) return ABACUS_NF_ESCRATCH;
  void* ws = nullptr;
  if ((rc = noalloc_scratch(&ws))) return rc;
  return forces_launch(boxes, nboxes, r, mode, (flags & ABACUS_NF_COUNT_PAIRS) != 0, b, acc,
                       density, momentum, pair_count, ws, L, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

int forces_args(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                const float* acc, const float* density, const int64_t* pair_count,
                uint32_t flags, Resolved* r, AccMode* mode) {
  int rc = resolve(boxes, nboxes, r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  if ((rc = acc_mode(flags, mode))) return rc;
  const bool count = (flags & ABACUS_NF_COUNT_PAIRS) != 0;
  if (!binned_ok(b, r->n_total) || (r->n_total > 0 && !acc) || (count && !pair_count))
    return ABACUS_NF_EINVAL;
  if (density && (count || !r->density_ok)) return ABACUS_NF_EINVAL;
  return ABACUS_NF_OK;
}

// Plan, forward pair kernel and momentum reduction of one abacus_nf_forces
// call, with every temporary in `ws` laid out as L.
int forces_launch(const abacus_nf_box* boxes, int nboxes, const Resolved& r, AccMode mode,
                  bool count, const abacus_nf_binned* b, float* acc, float* density,
                  double* momentum, int64_t* pair_count, void* ws, const Layout& L,
                  hipStream_t s) {
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  if (count) ANF_HIP(fill_i64(pair_count, 0, 1, s), "pair counter");
  PlanWork w = plan_work(ws, L);
  const KernelConfig cfg = lookup_config(tune_key(boxes, nboxes, r, mode, 0));
  w.split_items = split_items_for(cfg, mode, r, L);
  {
    Timer t(3, s);
    ANF_HIP(launch_plan(dboxes, nboxes, r.pencils_total, b->cell_offsets, b->status, cfg.span,
                        r.split_slices, w, s),
            "work plan");
    t.done();
  }
  if (r.n_total > 0) {
    Timer t(0, s);
    ANF_HIP(launch_forward(mode, count, cfg, dboxes, w, r.pencils_total, b->cell_offsets, b->rel,
                           b->perm, acc, r.n_total > 0 ? density : nullptr, pair_count,
                           at<float>(ws, L.src_w), r.n_total, s),
            "forward pair kernel");
    t.done();
  }
  if (momentum)
    ANF_HIP(launch_momentum(dboxes, nboxes, r.max_box_n, acc, at<double>(ws, L.mom), momentum, s),
            "momentum reduction");
  return ABACUS_NF_OK;
}

}  // namespace

extern "C" {

int abacus_nf_forces_f64(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                         double* acc, uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (flags & ~ABACUS_NF_PLUMMER) return ABACUS_NF_EINVAL;
  Resolved r;
  int rc = resolve(boxes, nboxes, &r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  if (!binned_ok(b, r.n_total) || (r.n_total > 0 && !acc)) return ABACUS_NF_EINVAL;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  PlanWork w = plan_work(ws, L);
  // The FP64 kernel takes whole items only, in the default span.
  KernelConfig cfg = default_config(0);
  cfg.split = 0;
  w.split_items = 0;
  ANF_HIP(launch_plan(dboxes, nboxes, r.pencils_total, b->cell_offsets, b->status, cfg.span, 1, w,
                      s),
          "work plan");
  if (r.n_total > 0) {
    Timer t(0, s);
    ANF_HIP(launch_forward_f64(dboxes, w, b->cell_offsets, b->rel, b->perm, acc,
                               at<double>(ws, L.src_w), r.n_total, s),
            "FP64 forward pair kernel");
    t.done();
  }
  return ABACUS_NF_OK;
}

int abacus_nf_forces_vjp_f64(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                             const double* wv, double* grad, uint32_t flags, void* ws,
                             size_t ws_bytes, void* stream) {
  if (flags & ~ABACUS_NF_PLUMMER) return ABACUS_NF_EINVAL;
  Resolved r;
  int rc = resolve(boxes, nboxes, &r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  if (!binned_ok(b, r.n_total) || (r.n_total > 0 && (!wv || !grad))) return ABACUS_NF_EINVAL;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  PlanWork w = plan_work(ws, L);
  // Like the FP64 forward kernel: whole items only, in the default span.
  KernelConfig cfg = default_config(1);
  cfg.split = 0;
  w.split_items = 0;
  ANF_HIP(launch_plan(dboxes, nboxes, r.pencils_total, b->cell_offsets, b->status, cfg.span, 1, w,
                      s),
          "work plan");
  if (r.n_total > 0) {
    Timer t(1, s);
    // the sorted FP64 cotangents take the adjoint's 24-byte source-record region
    ANF_HIP(launch_vjp_f64(dboxes, w, b->cell_offsets, b->rel, b->perm, wv,
                           at<double>(ws, L.src_w), r.n_total, grad, s),
            "FP64 adjoint pair kernel");
    t.done();
  }
  return ABACUS_NF_OK;
}

int abacus_nf_forces_vjp(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                         const float* wv, float* grad, uint32_t flags, void* ws, size_t ws_bytes,
                         void* stream) {
  return vjp_call(boxes, nboxes, b, false, 0, 0, wv, grad, flags, ws, ws_bytes, stream);
}

int abacus_nf_forces_slab(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                          int32_t x_begin, int32_t x_end, float* acc, uint32_t flags, void* ws,
                          size_t ws_bytes, void* stream) {
  if (flags & ABACUS_NF_COUNT_PAIRS) return ABACUS_NF_EINVAL;
  Resolved r;
  AccMode mode;
  int rc = forces_args(boxes, nboxes, b, acc, nullptr, nullptr, flags, &r, &mode);
  if (rc) return rc;
  if ((rc = set_sink_slabs(&r, x_begin, x_end))) return rc;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  return forces_launch(boxes, nboxes, r, mode, false, b, acc, nullptr, nullptr, nullptr, ws, L,
                       static_cast<hipStream_t>(stream));
}

int abacus_nf_forces_vjp_slab(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                              int32_t x_begin, int32_t x_end, const float* wv, float* grad,
                              uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  return vjp_call(boxes, nboxes, b, true, x_begin, x_end, wv, grad, flags, ws, ws_bytes, stream);
}

}  // extern "C"

namespace {

// abacus_nf_forces_vjp, or with `slab` its variant for the sink slabs
// [x0, x1) of every box.
int vjp_call(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b, bool slab,
             int32_t x0, int32_t x1, const float* wv, float* grad, uint32_t flags, void* ws,
             size_t ws_bytes, void* stream) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  AccMode mode;
  if ((rc = acc_mode(flags, &mode))) return rc;
  if (flags & ABACUS_NF_COUNT_PAIRS) return ABACUS_NF_EINVAL;
  if (!binned_ok(b, r.n_total) || (r.n_total > 0 && (!wv || !grad))) return ABACUS_NF_EINVAL;
  if (slab && (rc = set_sink_slabs(&r, x0, x1))) return rc;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  PlanWork w = plan_work(ws, L);
  const KernelConfig cfg = lookup_config(tune_key(boxes, nboxes, r, mode, 1));
  w.split_items = split_items_for(cfg, mode, r, L);
  {
    Timer t(3, s);
    ANF_HIP(launch_plan(dboxes, nboxes, r.pencils_total, b->cell_offsets, b->status, cfg.span,
                        r.split_slices, w, s),
            "work plan");
    t.done();
  }
  if (r.n_total > 0) {
    Timer t(1, s);
    ANF_HIP(launch_vjp(mode, cfg, dboxes, w, r.pencils_total, b->cell_offsets, b->rel, b->perm, wv,
                       at<float>(ws, L.src_w), r.n_total, grad, s),
            "adjoint pair kernel");
    t.done();
  }
  return ABACUS_NF_OK;
}

// The sink slabs [x0, x1) of every box (0 <= x0 <= x1 <= K): the work plan
// then takes only the pencils of those slabs.
int set_sink_slabs(Resolved* r, int32_t x0, int32_t x1) {
  for (DevBox& d : r->boxes) {
    if (x0 < 0 || x0 > x1 || x1 > d.K) return ABACUS_NF_EINVAL;
    d.sink_x0 = x0;
    d.sink_x1 = x1;
  }
  return ABACUS_NF_OK;
}

}  // namespace

extern "C" {

static abacus_nf_tuning to_public(const KernelConfig& c) {
  abacus_nf_tuning t;
  t.unroll = c.unroll;
  t.pipeline = c.pipeline;
  t.span = c.span;
  t.grid_mult = c.grid_mult;
  t.split = c.split;
  return t;
}

static KernelConfig from_public(const abacus_nf_tuning& t) {
  KernelConfig c;
  c.unroll = t.unroll;
  c.pipeline = t.pipeline;
  c.span = t.span;
  c.grid_mult = t.grid_mult;
  c.split = t.split;
  return c;
}

int abacus_nf_get_tuning(const abacus_nf_box* boxes, int nboxes, uint32_t flags, int kernel,
                         abacus_nf_tuning* out) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  AccMode mode;
  if ((rc = acc_mode(flags & ~ABACUS_NF_COUNT_PAIRS, &mode))) return rc;
  if (!out || (kernel != 0 && kernel != 1)) return ABACUS_NF_EINVAL;
  *out = to_public(lookup_config(tune_key(boxes, nboxes, r, mode, kernel)));
  return ABACUS_NF_OK;
}

int abacus_nf_set_tuning(const abacus_nf_box* boxes, int nboxes, uint32_t flags, int kernel,
                         const abacus_nf_tuning* t) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  AccMode mode;
  if ((rc = acc_mode(flags & ~ABACUS_NF_COUNT_PAIRS, &mode))) return rc;
  if (kernel != 0 && kernel != 1) return ABACUS_NF_EINVAL;
  const TuneKey key = tune_key(boxes, nboxes, r, mode, kernel);
  if (!t) {
    clear_config(key);
    return ABACUS_NF_OK;
  }
  const KernelConfig c = from_public(*t);
  if (!config_valid(kernel, c)) return ABACUS_NF_EINVAL;
  store_config(key, c, false);
  return ABACUS_NF_OK;
}

int abacus_nf_autotune(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                       float* scratch, uint32_t flags, void* ws, size_t ws_bytes, void* stream,
                       abacus_nf_tuning* forward_out, abacus_nf_tuning* adjoint_out) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r, (flags & ABACUS_NF_PLUMMER) != 0);
  if (rc) return rc;
  AccMode mode;
  if ((rc = acc_mode(flags, &mode))) return rc;
  if (flags & ABACUS_NF_COUNT_PAIRS) return ABACUS_NF_EINVAL;
  if (!binned_ok(b, r.n_total) || (r.n_total > 0 && !scratch)) return ABACUS_NF_EINVAL;
  const Layout L = layout(r);
  if ((rc = check_ws(ws, ws_bytes, L))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const TuneKey kf = tune_key(boxes, nboxes, r, mode, 0), ka = tune_key(boxes, nboxes, r, mode, 1);
  KernelConfig best[2] = {default_config(0), default_config(1)};
  if (r.n_total > 0) {
    DevBox* dboxes = at<DevBox>(ws, L.boxtab);
    ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
    PlanWork w = plan_work(ws, L);
    hipEvent_t e0, e1;
    ANF_HIP(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return hip_fail(hipErrorOutOfMemory, "event");
    }
    hipError_t err = hipSuccess;
    // Time plan + kernel: one warm-up, then the best of three (run-to-run
    // spread is 1-2%, about the gap between neighbouring shapes).
    auto run = [&](int kernel, const KernelConfig& c) -> float {
      float best_ms = 3.0e38f;
      for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
        err = hipEventRecord(e0, s);
        w.split_items = split_items_for(c, mode, r, L);
        if (err == hipSuccess)
          err = launch_plan(dboxes, nboxes, r.pencils_total, b->cell_offsets, b->status, c.span,
                            r.split_slices, w, s);
        if (err == hipSuccess) {
          if (kernel == 0)
            err = launch_forward(mode, false, c, dboxes, w, r.pencils_total, b->cell_offsets,
                                 b->rel, b->perm, scratch, nullptr, nullptr, at<float>(ws, L.src_w),
                                 r.n_total, s);
          else  // any finite cotangent times the same: read the offsets as w
            err = launch_vjp(mode, c, dboxes, w, r.pencils_total, b->cell_offsets, b->rel,
                             b->perm, b->rel, at<float>(ws, L.src_w), r.n_total, scratch, s);
        }
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < best_ms) best_ms = ms;
      }
      return best_ms;
    };
    for (int kernel = 0; kernel < 2 && err == hipSuccess; ++kernel) {
      KernelConfig cur = default_config(kernel);
      float t_cur = run(kernel, cur);
      auto try_cfg = [&](const KernelConfig& c) {
        if (!config_valid(kernel, c) || err != hipSuccess) return;
        const float t = run(kernel, c);
        if (t < t_cur) {
          t_cur = t;
          cur = c;
        }
      };
      for (int span = 1; span <= kMaxSpan; ++span) {
        KernelConfig c = cur;
        c.span = span;
        try_cfg(c);
      }
      const KernelConfig base = cur;
      for (int u : {2, 3, 4, 8})
        for (int pipe = 0; pipe < 2; ++pipe) {
          KernelConfig c = base;
          c.unroll = u;
          c.pipeline = pipe;
          try_cfg(c);
        }
      {
        KernelConfig c = cur;
        c.grid_mult = 3 - cur.grid_mult;
        try_cfg(c);
      }
      {
        KernelConfig c = cur;
        c.split = 1 - cur.split;
        try_cfg(c);
      }
      best[kernel] = cur;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "autotune");
  }
  store_config(kf, best[0], true);
  store_config(ka, best[1], true);
  if (forward_out) *forward_out = to_public(best[0]);
  if (adjoint_out) *adjoint_out = to_public(best[1]);
  return ABACUS_NF_OK;
}

// ---- cell multipoles ---------------------------------------------------------

struct MpLayout {
  size_t boxtab, keys, hist, base, cursor, waves, sorted, span, full, red_coef, red_src, red_cnt,
      total;
};

MpLayout mp_layout(const Resolved& r, int order, bool reduced) {
  MpLayout L;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + (bytes ? bytes : 1));
    return at;
  };
  L.boxtab = take(sizeof(DevBox) * r.boxes.size());
  L.keys = take(4 * (size_t)r.cells_total);
  L.hist = take(4 * (size_t)kMpBuckets);
  L.base = take(4 * (size_t)kMpBuckets);
  L.cursor = take(4 * (size_t)kMpBuckets);
  L.waves = take(4 * (size_t)kMpBuckets);
  L.sorted = take(4 * (size_t)r.cells_total);
  L.span = take(8 * (size_t)r.cells_total);
  L.full = reduced ? take(sizeof(double) * (size_t)multipole_terms(order, false) *
                          (size_t)r.cells_total)
                   : 0;
  L.red_coef = reduced ? take(sizeof(double) * 81 * 16) : 0;
  L.red_src = reduced ? take(4 * 81 * 16) : 0;
  L.red_cnt = reduced ? take(4 * 81) : 0;
  L.total = o;
  return L;
}

struct KdkLayout {
  size_t boxtab, sumsq, amax, part, tile_part, mode, rec, total;
  int64_t tiles;
};

KdkLayout kdk_layout(const Resolved& r) {
  KdkLayout L;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + (bytes ? bytes : 1));
    return at;
  };
  L.boxtab = take(sizeof(DevBox) * r.boxes.size());
  L.sumsq = take(sizeof(double) * (size_t)r.cells_total);
  L.amax = take(sizeof(double) * (size_t)r.cells_total);
  L.part = take(sizeof(double) * 3 * (size_t)r.kdk_chunks);
  L.tiles = (r.n_total + kKdkTile - 1) / kKdkTile;
  L.tile_part = take(sizeof(double) * 4 * (size_t)L.tiles);
  L.mode = take(sizeof(int32_t));
  L.rec = take(sizeof(KdkRec) * (size_t)r.n_total);
  L.total = o;
  return L;
}

int mp_args(int order, uint32_t flags, bool* reduced) {
  if (order < 0 || order > kMaxMultipoleOrder) return ABACUS_NF_EINVAL;
  if (flags & ~ABACUS_NF_REDUCED) return ABACUS_NF_EINVAL;
  *reduced = (flags & ABACUS_NF_REDUCED) != 0;
  return ABACUS_NF_OK;
}

const char* abacus_nf_strerror(int code) {
  switch (code) {
    case ABACUS_NF_OK: return "ok";
    case ABACUS_NF_EINVAL: return "invalid argument";
    case ABACUS_NF_ERANGE: return "size out of range (particles or cells reach 2^31)";
    case ABACUS_NF_EWORKSPACE: return "workspace missing, misaligned or too small";
    case ABACUS_NF_ESCRATCH:
      return "problem too large for the 64 MiB static scratch of abacus_nf_forces_noalloc";
    case ABACUS_NF_EHIP: {
      thread_local std::string msg;
      msg = "HIP error: " + g_last_hip_error;
      return msg.c_str();
    }
    default: return "unknown error code";
  }
}

int abacus_nf_multipole_terms(int order, uint32_t flags, int64_t* terms) {
  bool reduced = false;
  int rc = mp_args(order, flags, &reduced);
  if (rc) return rc;
  if (!terms) return ABACUS_NF_EINVAL;
  *terms = multipole_terms(order, reduced);
  return ABACUS_NF_OK;
}

int abacus_nf_multipoles_workspace_bytes(const abacus_nf_box* boxes, int nboxes, int order,
                                         uint32_t flags, size_t* bytes) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  bool reduced = false;
  if ((rc = mp_args(order, flags, &reduced))) return rc;
  if (!bytes) return ABACUS_NF_EINVAL;
  *bytes = mp_layout(r, order, reduced).total;
  return ABACUS_NF_OK;
}

int abacus_nf_multipoles(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                         int order, uint32_t flags, double* out, void* ws, size_t ws_bytes,
                         void* stream) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  bool reduced = false;
  if ((rc = mp_args(order, flags, &reduced))) return rc;
  if (!binned_ok(b, r.n_total) || !out) return ABACUS_NF_EINVAL;
  const MpLayout L = mp_layout(r, order, reduced);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0 || ws_bytes < L.total)
    return ABACUS_NF_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  MpWork w;
  w.cells = r.cells_total;
  w.keys = at<int32_t>(ws, L.keys);
  w.hist = at<int32_t>(ws, L.hist);
  w.bucket_base = at<int32_t>(ws, L.base);
  w.cursor = at<int32_t>(ws, L.cursor);
  w.bucket_waves = at<int32_t>(ws, L.waves);
  w.sorted = at<int32_t>(ws, L.sorted);
  w.span = at<int2>(ws, L.span);
  w.full = reduced ? at<double>(ws, L.full) : nullptr;
  w.red_coef = reduced ? at<double>(ws, L.red_coef) : nullptr;
  w.red_src = reduced ? at<int32_t>(ws, L.red_src) : nullptr;
  w.red_cnt = reduced ? at<int32_t>(ws, L.red_cnt) : nullptr;
  Timer t(4, s);
  ANF_HIP(launch_multipoles(dboxes, nboxes, r.cells_total, order, reduced, w, b->cell_offsets,
                            b->rel, out, s),
          "multipoles");
  t.done();
  return ABACUS_NF_OK;
}

int abacus_nf_kick_drift_workspace_bytes(const abacus_nf_box* boxes, int nboxes,
                                         size_t* bytes) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  if (!bytes) return ABACUS_NF_EINVAL;
  *bytes = kdk_layout(r).total;
  return ABACUS_NF_OK;
}

int abacus_nf_kick_drift(const abacus_nf_box* boxes, int nboxes, const abacus_nf_binned* b,
                         const double* kick, const double* drift, float* pos, float* vel,
                         const float* acc, double* cell_stats, double* box_stats, void* ws,
                         size_t ws_bytes, void* stream) {
  Resolved r;
  int rc = resolve(boxes, nboxes, &r);
  if (rc) return rc;
  if (!binned_ok(b, r.n_total) || !kick || !drift) return ABACUS_NF_EINVAL;
  if (r.n_total > 0 && (!pos || !vel || !acc)) return ABACUS_NF_EINVAL;
  for (int i = 0; i < nboxes; ++i) {
    if (!std::isfinite(kick[i]) || !std::isfinite(drift[i])) return ABACUS_NF_EINVAL;
    r.boxes[i].kick = kick[i];
    r.boxes[i].drift = drift[i];
  }
  const KdkLayout L = kdk_layout(r);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0 || ws_bytes < L.total)
    return ABACUS_NF_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBox* dboxes = at<DevBox>(ws, L.boxtab);
  ANF_HIP(write_box_table(r.boxes.data(), nboxes, dboxes, s), "box table");
  KdkWork w;
  w.cell_sumsq = at<double>(ws, L.sumsq);
  w.cell_amax = at<double>(ws, L.amax);
  w.chunk_part = at<double>(ws, L.part);
  w.tile_part = at<double>(ws, L.tile_part);
  w.mode = at<int32_t>(ws, L.mode);
  w.rec = at<KdkRec>(ws, L.rec);
  w.chunks = r.kdk_chunks;
  w.tiles = L.tiles;
  Timer t(5, s);
  ANF_HIP(launch_kick_drift(dboxes, nboxes, r.n_total, r.cells_total, w, b->cell_offsets, b->perm,
                            pos, vel,
                            acc, cell_stats, box_stats, s),
          "kick-drift");
  t.done();
  return ABACUS_NF_OK;
}

double abacus_nf_timestep(const double* box_stats, double a, double H, double eta_acc,
                          double eta_H) {
  if (!box_stats) return NAN;
  const double global = box_stats[2] > 0.0 ? box_stats[1] / box_stats[2] : INFINITY;
  const double ratio = box_stats[0] > global ? box_stats[0] : global;
  const double acc_step = eta_acc * a * H * ratio;
  const double hubble_step = eta_H * a;
  return acc_step < hubble_step ? acc_step : hubble_step;
}

int abacus_nf_timing_enable(int enable) {
  std::lock_guard<std::mutex> lock(g_timing_mu);
  g_timing = enable != 0;
  return ABACUS_NF_OK;
}

int abacus_nf_timing_read(int kernel, double* ms, int64_t* launches) {
  if (kernel < 0 || kernel >= kTimerSlots) return ABACUS_NF_EINVAL;
  std::lock_guard<std::mutex> lock(g_timing_mu);
  drain_timing();
  if (ms) *ms = g_ms[kernel];
  if (launches) *launches = g_launches[kernel];
  return ABACUS_NF_OK;
}

int abacus_nf_timing_reset(void) {
  std::lock_guard<std::mutex> lock(g_timing_mu);
  drain_timing();
  for (int k = 0; k < kTimerSlots; ++k) {
    g_ms[k] = 0.0;
    g_launches[k] = 0;
  }
  return ABACUS_NF_OK;
}

}  // extern "C"
