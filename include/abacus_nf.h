/*
 * abacus_nf.h -- C ABI of the MI355X near-field force library.
 *
 * The near field of the Abacus method (Garrison et al. 2021): particles are
 * binned into a periodic K^3 grid of cells (Sec. 2.2) and every particle
 * receives the exact, direct, softened 1/r^2 force of every other particle in
 * the (2R+1)^3 cells around its own cell (Sec. 3.4.1), using the periodic image
 * that lies in the neighbouring cell (Sec. 3.4.2).  The force law is the
 * spline softening of Eq. 3 with eps_s = 2.16 eps_p (Sec. 3.2).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers on the current HIP device,
 *     allocated and owned by the caller.  Nothing is allocated, freed or
 *     synchronised by the library; every call only enqueues work on `stream`
 *     (a hipStream_t passed as void*, NULL = the null stream) and returns.  The
 *     enqueued work can be captured into a HIP graph.
 *   - `boxes` / `nboxes` is a HOST array.  Several independent periodic boxes
 *     can be processed by one call: their particles are concatenated in box
 *     order (box b owns particles [first_b, first_b + n_b), first_b = sum of the
 *     n of earlier boxes) and so are their cells (box b owns global cell ids
 *     [cell_base_b, cell_base_b + K_b^3), cell_base_b = sum of earlier K^3).
 *   - Units: G*m = 1 for every particle (equal unit masses).  Accelerations
 *     are attractive, in box-length units: a_i = sum_j F(x_j - x_i).
 *   - Return value: ABACUS_NF_OK (0) or a negative error code.  Argument
 *     errors are detected on the host before anything is enqueued (outputs are
 *     untouched).  Problems only visible in the data (non-finite positions) set
 *     bits in the device status word of the binned arrays; outputs for such a
 *     call are unspecified.
 *   - A workspace (`ws`, `ws_bytes`, device memory, 256-byte aligned) holds
 *     all temporaries; size it with abacus_nf_workspace_bytes.  Calls that
 *     share a workspace must be ordered on one stream.
 */
#ifndef ABACUS_NF_H
#define ABACUS_NF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define ABACUS_NF_OK          0
#define ABACUS_NF_EINVAL     (-1)  /* bad argument (null pointer, box, K, R, softening, flags) */
#define ABACUS_NF_ERANGE     (-2)  /* sizes beyond the int32 index space of the kernels */
#define ABACUS_NF_EWORKSPACE (-3)  /* workspace missing, misaligned or too small */
#define ABACUS_NF_EHIP       (-4)  /* a HIP runtime call failed; see abacus_nf_strerror */
#define ABACUS_NF_ESCRATCH   (-5)  /* too large for abacus_nf_forces_noalloc's static scratch */

/* ---- device status bits (int32 written by abacus_nf_bin) ---------------- */
#define ABACUS_NF_STATUS_BADPOS 0x1  /* a coordinate was non-finite or |x K / L| >= 2^30 */
/* A cell holds more than 2^28 particles: beyond the kernels' 32-bit offsets
 * inside one cell.  Every call that runs the pair kernels on these binned
 * arrays (abacus_nf_forces, abacus_nf_forces_vjp and their FP64, slab and
 * no-allocation variants) then evaluates no pair: accelerations and gradients
 * are not written, and momentum sums add whatever the acceleration array held.
 * Nothing faults; the sizes a call accepts are otherwise unchanged. */
#define ABACUS_NF_STATUS_CELLFULL 0x2

/* ---- flags for abacus_nf_forces / abacus_nf_forces_vjp ----------------- */
/* Accumulation of each sink's sum (exactly one of the three; default COMPENSATED):
 *   SINGLE_ACC   one FP32 accumulator per sink, every pair added in turn (the
 *                register accumulation of the paper's kernel, Sec. 3.4.2);
 *   CHUNKED      FP32 partial sums over chunks of at most 64 sources of one
 *                cell, added to the accumulator (the "intermediate
 *                accumulators" remedy named in Sec. 3.5.4);
 *   COMPENSATED  the same chunk partials folded into an FP32 (sum, error) pair
 *                with an error-free TwoSum (the Kahan-style remedy of
 *                Sec. 3.5.4). */
#define ABACUS_NF_SINGLE_ACC   0x1u
#define ABACUS_NF_CHUNKED      0x2u
#define ABACUS_NF_COMPENSATED  0x4u
/* Debug: count every evaluated (sink, source) pair, self excluded, into the
 * int64 at `pair_count` (abacus_nf_forces only).  Costs one atomic per work item. */
#define ABACUS_NF_COUNT_PAIRS  0x10u
/* Force law: Plummer softening of Eq. 2, F = d / (r^2 + eps_p^2)^(3/2), with the
 * box's eps_plummer used as given, in place of the default spline of Eq. 3.
 * Accepted by abacus_nf_forces, abacus_nf_forces_vjp and the tuning calls (the
 * two laws keep separate launch shapes).  Every pair then takes the same plain
 * branch; the validation of eps_plummer is unchanged. */
#define ABACUS_NF_PLUMMER      0x20u
/* abacus_nf_multipoles: return the (p+1)^2 reduced basis instead of the
 * complete one. */
#define ABACUS_NF_REDUCED      0x40u

/* ---- data types --------------------------------------------------------- */

/* One periodic box (Sec. 2.2 grid; Sec. 3.4.1 near-field radius; Sec. 3.2
 * softening; Sec. 3.4.4 density estimate).  Requirements: n >= 0; box > 0 and
 * finite; radius >= 0; cpd >= 2*radius + 1 (so the (2R+1)^3 stencil never wraps
 * onto itself); eps_plummer > 0 and finite with
 * 1e-6 <= 2.16*eps_plummer*cpd/box <= 1e6; density_radius is 0 (no density
 * estimate) or finite with 0 < density_radius*cpd/box <= radius and
 * (density_radius*cpd/box)^2 >= 1e-30. */
typedef struct {
    int64_t n;             /* number of particles in this box */
    double  box;           /* side L of the periodic cube */
    int32_t cpd;           /* cells per dimension K */
    int32_t radius;        /* near-field radius R in cells (the paper uses 2) */
    double  eps_plummer;   /* Plummer-equivalent softening; eps_s = 2.16 eps_p */
    double  density_radius;/* top-hat radius b of the density estimate (box units), or 0 */
} abacus_nf_box;

/* Binned particles: the output of abacus_nf_bin, input of the force calls.
 * Sorted order is by global cell id (box, then x slowest, z fastest), and by
 * ascending original index inside a cell (a stable counting sort). */
typedef struct {
    int32_t *cell_offsets; /* cells_total + 1: first sorted slot of each global cell;
                              cell_offsets[cells_total] = n_total */
    int32_t *perm;         /* n_total: sorted slot -> original (global) particle index */
    float   *rel;          /* n_total x 4: in sorted order, (x, y, z) offset from the
                              cell centre in cell-width units, in [-1/2, 1/2); 4th = 0 */
    int32_t *status;       /* 1 int: ABACUS_NF_STATUS_* bits, written by abacus_nf_bin */
} abacus_nf_binned;

/* ---- entry points ------------------------------------------------------- */

/* Totals of a box list: *n_total = sum n, *cells_total = sum K^3.
 * EINVAL on a bad box, ERANGE if either total reaches 2^31 or the pair
 * kernels' work plan could exceed 2^28 items (n/64 + cells + 2 K^2 summed
 * over the boxes reaches 2^28, i.e. more than about 2.7e8 cells). */
int abacus_nf_layout(const abacus_nf_box *boxes, int nboxes, int64_t *n_total,
                     int64_t *cells_total);

/* Bytes of workspace that abacus_nf_bin, abacus_nf_forces and
 * abacus_nf_forces_vjp need for this box list (one workspace serves all three). */
int abacus_nf_workspace_bytes(const abacus_nf_box *boxes, int nboxes, size_t *bytes);

/*
 * abacus_nf_bin -- cell assignment and stable counting sort by cell.
 * Follows Sec. 2.2 (grid of K^3 cells, slabs along x, pencils along z) and
 * Sec. 3.5.1 (positions kept as FP32 offsets from cell centres).
 *   pos  n_total x 3 FP32, global coordinates, row-major.  Any finite value is
 *        taken as its periodic image: with t = x * (K/L) in FP64, the cell is
 *        floor(t) mod K and the offset is t - (floor(t) + 1/2) rounded once to
 *        FP32 (a coordinate on a face belongs to the higher cell).
 *   out  caller-allocated arrays (sizes in abacus_nf_binned); all are written.
 *        With no particles at all, pos, perm and rel may be NULL (here and in
 *        every entry point taking a binned set) and every offset is 0.
 * The status word is cleared and then set if any coordinate is non-finite or
 * |t| >= 2^30.
 */
int abacus_nf_bin(const abacus_nf_box *boxes, int nboxes, const float *pos,
                  const abacus_nf_binned *out, void *ws, size_t ws_bytes, void *stream);

/*
 * abacus_nf_forces -- near-field accelerations.
 * a_i = sum over j != i in the (2R+1)^3 cells around i's cell of F(x_j - x_i)
 * with F of Eq. 3 (spline softening, eps_s = 2.16 eps_p, Sec. 3.2), the image of
 * x_j being the one in the neighbouring cell (Sec. 3.4.1-3.4.2).  Arithmetic is
 * FP32 on cell-relative coordinates; the accumulation follows `flags`.
 *   b          binned arrays from abacus_nf_bin for the same boxes.
 *   acc        n_total x 3 FP32 output in ORIGINAL particle order, box units.
 *   density    NULL, or n_total FP32 outputs in original order: the apodized
 *              top-hat estimate of Sec. 3.4.4, rho_i = sum over the same
 *              near-field points j (i itself included) with r_ij < b of
 *              1 - r_ij^2/b^2, b = density_radius, accumulated as b^2 - r^2 in
 *              cell units in the same pass as the forces (plain FP32 sums per
 *              x offset, whatever the accumulation flag) and divided by b^2.
 *              EINVAL if a box has density_radius 0 or with COUNT_PAIRS.
 *   momentum   NULL, or 4*nboxes FP64 outputs: per box (sum a_x, sum a_y,
 *              sum a_z, sum |a|), reduced in FP64 in a fixed order.  Pair
 *              antisymmetry makes the first three vanish up to rounding.
 *   pair_count NULL, or one int64 that receives the number of evaluated pairs
 *              when ABACUS_NF_COUNT_PAIRS is set.
 */
int abacus_nf_forces(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                     float *acc, float *density, double *momentum, int64_t *pair_count,
                     uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/*
 * abacus_nf_forces_noalloc -- abacus_nf_forces for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments without the workspace,
 * the same kernels and the same results bit for bit.
 *   Temporaries live in a static 64 MiB device array of the library (one per
 *   GPU, held until the process ends); its address is looked up once per
 *   device, on the first call with that device current.  `stream` must belong
 *   to the current device.  Nothing is allocated or freed.
 *   Limit: the work plan, the packed 12-byte source records and the momentum
 *   partials must fit the 64 MiB -- about 4 M particles at 64 per cell --
 *   else ABACUS_NF_ESCRATCH is returned before anything is enqueued.
 *   Every call on one GPU uses that GPU's one array, and the array keeps the
 *   last call's contents (each call clears what it needs cleared): calls that
 *   overlap in time on one GPU (different streams, different threads) race and
 *   must be ordered by the caller.
 */
int abacus_nf_forces_noalloc(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                             float *acc, float *density, double *momentum,
                             int64_t *pair_count, uint32_t flags, void *stream);

/*
 * abacus_nf_forces_f64 -- the same near-field accelerations with every
 * operation after the stored FP32 cell offsets done in FP64 (the paper's
 * double-precision build option): separations, r^2, 1/r (hardware estimate
 * plus two Newton steps), Eq. 3 with the min hand-off or, with
 * ABACUS_NF_PLUMMER, Eq. 2, and a plain FP64 sum per sink.  The result is the
 * near field of the stored positions to FP64 rounding.
 *   acc    n_total x 3 FP64 output in ORIGINAL particle order, box units.
 *   flags  0 or ABACUS_NF_PLUMMER (no accumulation modes, density or pair
 *          counting).  Same workspace as abacus_nf_forces.
 */
int abacus_nf_forces_f64(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                         double *acc, uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/*
 * abacus_nf_forces_vjp_f64 -- the adjoint of abacus_nf_forces_f64, every
 * operation after the stored FP32 cell offsets in FP64: for a cotangent w,
 *   grad_k = sum_{j in NF(k)} [ f(r)(w_j - w_k) + (f'(r)/r)(d.(w_j - w_k)) d ]
 * with d = x_j - x_k and f from Eq. 3 (Sec. 3.2) or, with ABACUS_NF_PLUMMER,
 * Eq. 2; the binning is held fixed (the derivative on the piecewise-smooth
 * branch), a plain FP64 sum per particle.
 *   w      n_total x 3 FP64 cotangent in ORIGINAL particle order.
 *   grad   n_total x 3 FP64 output in ORIGINAL particle order, box units.
 *   flags  0 or ABACUS_NF_PLUMMER.  Same workspace as abacus_nf_forces.
 * Errors as abacus_nf_forces_f64.  Results are run-to-run deterministic.
 */
int abacus_nf_forces_vjp_f64(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                             const double *w, double *grad, uint32_t flags, void *ws,
                             size_t ws_bytes, void *stream);

/*
 * abacus_nf_forces_vjp -- vector-Jacobian product of the accelerations.
 * For a cotangent w (n_total x 3 FP32, original order) returns
 *   grad_k = d/dx_k sum_i w_i . a_i
 *          = sum_{j in NF(k)} [ f(r) (w_j - w_k) + h(r) (d . (w_j - w_k)) d ],
 * d = x_j - x_k, f(r) d = F(d) of Eq. 3 and h = f'(r)/r, with the binning held
 * fixed (the near field is piecewise smooth; this is the derivative inside a
 * piece).  grad is n_total x 3 FP32 in original order (units of a per length).
 * Same traversal and accumulation flags as abacus_nf_forces.
 */
int abacus_nf_forces_vjp(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                         const float *w, float *grad, uint32_t flags, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * abacus_nf_forces_slab / abacus_nf_forces_vjp_slab -- abacus_nf_forces and
 * abacus_nf_forces_vjp for the sinks of the slabs x in [x_begin, x_end) of
 * every box only.  The near field is evaluated one sink slab at a time, with
 * the R source slabs on either side resident (Sec. 3.4.1), and a node of a
 * parallel run holds a range of slabs (Sec. 4.4): this is one such share.
 * Sources still come from every cell of each sink's stencil, so those
 * slabs' outputs are bit-identical to the whole-box call's; the entries of
 * acc / grad for particles outside the slabs are not written.
 *   x_begin, x_end  0 <= x_begin <= x_end <= K of every box (else EINVAL);
 *                   x_begin == x_end computes nothing.
 *   flags           accumulation flags and ABACUS_NF_PLUMMER (COUNT_PAIRS:
 *                   EINVAL).  Same binned arrays and workspace as the
 *                   whole-box calls; other arguments and errors as those.
 */
int abacus_nf_forces_slab(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                          int32_t x_begin, int32_t x_end, float *acc, uint32_t flags, void *ws,
                          size_t ws_bytes, void *stream);
int abacus_nf_forces_vjp_slab(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                              int32_t x_begin, int32_t x_end, const float *w, float *grad,
                              uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* Human-readable text for an error code; for ABACUS_NF_EHIP it includes the
 * message of the last failing HIP call on this thread. */
const char *abacus_nf_strerror(int code);

/* ---- tuning of the pair kernels (a9: tile shapes chosen by measurement) --- */

/* Launch shape of one pair kernel.  Every shape computes the same sums in the
 * same order per sink: the choice changes speed, never results. */
typedef struct {
    int32_t unroll;     /* sources per inner-loop step: 2, 4 or 8 (adjoint: 2, 3 or 4) */
    int32_t pipeline;   /* 1: request the next step's sources before using the current ones */
    int32_t span;       /* most cells one 64-sink work item spans along its pencil: 1, 2 or 3 */
    int32_t grid_mult;  /* persistent workgroups per resident slot: 1 or 2 */
    int32_t split;      /* 1: split the cheapest work items at the end of the queue into one
                           task per x offset (shorter tail; same results); 0: never */
} abacus_nf_tuning;

#define ABACUS_NF_KERNEL_FORWARD 0
#define ABACUS_NF_KERNEL_ADJOINT 1

/*
 * abacus_nf_autotune -- time candidate shapes of the forward and adjoint pair
 * kernels on this binned input and keep the fastest for this problem shape
 * (box list, accumulation flags, device) in a process-wide table that later
 * abacus_nf_forces / abacus_nf_forces_vjp calls use.  The search is a
 * coordinate descent (span, then unroll/pipeline, then grid, then split) with two timed
 * runs per candidate.  `scratch` is n_total x 3 FP32 device memory whose
 * contents are overwritten.  Unlike the other entry points this call
 * SYNCHRONISES `stream`; do not call it while capturing a graph.  If the
 * environment variable ABACUS_NF_TUNE_CACHE names a file, results are appended
 * to it and read back by later processes.  Either output pointer may be NULL.
 */
int abacus_nf_autotune(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                       float *scratch, uint32_t flags, void *ws, size_t ws_bytes, void *stream,
                       abacus_nf_tuning *forward_out, abacus_nf_tuning *adjoint_out);

/* Read or override the shape used for (boxes, flags, kernel); t == NULL in
 * abacus_nf_set_tuning restores the built-in default.  EINVAL on shapes
 * outside the ranges above. */
int abacus_nf_get_tuning(const abacus_nf_box *boxes, int nboxes, uint32_t flags, int kernel,
                         abacus_nf_tuning *out);
int abacus_nf_set_tuning(const abacus_nf_box *boxes, int nboxes, uint32_t flags, int kernel,
                         const abacus_nf_tuning *t);

/* ---- cell multipoles (Eq. 4, Sec. 3.3.2) --------------------------------- */

/* Terms per cell for multipole order p (0 <= p <= 8): (p+3)(p+2)(p+1)/6 in the
 * complete basis, (p+1)^2 with ABACUS_NF_REDUCED.  EINVAL for another order or
 * flag, or a NULL result pointer. */
int abacus_nf_multipole_terms(int order, uint32_t flags, int64_t *terms);

/* Workspace bytes of abacus_nf_multipoles for this box list, order and flags
 * (a separate, usually smaller, size from abacus_nf_workspace_bytes; the
 * reduced basis also keeps the complete rows there: 8 B x cells x terms). */
int abacus_nf_multipoles_workspace_bytes(const abacus_nf_box *boxes, int nboxes, int order,
                                         uint32_t flags, size_t *bytes);

/*
 * abacus_nf_multipoles -- the cell multipoles of every cell of every box.
 * Complete basis (Eq. 4): M^{a,b,c} = sum over the particles q of the cell of
 * x_q^a y_q^b z_q^c, (x, y, z) the particle's displacement from the cell centre
 * in box units -- its stored FP32 cell-relative offset (b->rel) times w = L/K --
 * for a + b + c <= order, enumerated with a outermost and c innermost
 * (a = 0..p, b = 0..p-a, c = 0..p-a-b).  Sums are formed in FP64.
 * With ABACUS_NF_REDUCED, (p+1)^2 values per cell: for c0 in {0, 1} and
 * a + b + c0 <= p (same enumeration, c restricted to {0, 1}),
 *   R^{a,b,c0} = sum_{m>=0} sum_{i=0..m} (-1)^m C(m,i) a! b! c0! /
 *                ((a-2i)! (b-2m+2i)! (c0+2m)!) M^{a-2i, b-2m+2i, c0+2m}
 * (terms with a negative index omitted): the far-field expansion
 * sum (-1)^n M^{abc}/(a!b!c!) d^{abc}(1/r) keeps its value when the complete
 * values are replaced by these, because 1/r is harmonic (the trace-free
 * property the paper uses to store (p+1)^2 values).
 *   b      binned arrays from abacus_nf_bin for the same boxes.
 *   out    cells_total x terms FP64, cell-major in global cell order (box by
 *          box, x slowest, z fastest); every cell is written, empty ones 0.
 * Errors: EINVAL for a bad box, order outside [0, 8], an unknown flag or a
 * NULL pointer; EWORKSPACE if ws is NULL, not 256-byte aligned or smaller
 * than abacus_nf_multipoles_workspace_bytes.  Results are run-to-run
 * deterministic.
 */
int abacus_nf_multipoles(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                         int order, uint32_t flags, double *out, void *ws, size_t ws_bytes,
                         void *stream);

/* ---- kick, drift and the time step (Sec. 3.1, Eq. 1) --------------------- */

/* Workspace bytes of abacus_nf_kick_drift (32 B per particle, 16 B per cell, a little more). */
int abacus_nf_kick_drift_workspace_bytes(const abacus_nf_box *boxes, int nboxes,
                                         size_t *bytes);

/*
 * abacus_nf_kick_drift -- one leapfrog kick and drift, in place, with the
 * statistics of the time-step criterion.  For every particle i (FP32 state,
 * each update formed in FP64 with a separate multiply and add and rounded once
 * to FP32; same arithmetic as a plain C program compiled without contraction):
 *   vel_i <- vel_i + kick[box] * acc_i          (a full step between half steps)
 *   pos_i <- wrap(pos_i + drift[box] * vel_i)   (with the kicked velocity)
 * wrap(t) = t - L floor(t / L) in FP64, brought into [0, L), rounded to FP32,
 * and a value that rounds up to L set to 0.
 *   b          binned arrays of the same positions (before this call): the
 *              cells of the statistics are the cells of the binning.
 *   kick, drift  host arrays of nboxes finite factors (the cosmology's
 *              integrals over the step are the caller's).
 *   pos, vel   n_total x 3 FP32, original order, updated in place.
 *   acc        n_total x 3 FP32, original order (e.g. from abacus_nf_forces).
 *   cell_stats NULL, or cells_total x 2 FP64: per cell v_rms = sqrt(sum |v|^2 / n)
 *              over the kicked velocities (mean not subtracted, as the paper
 *              does) and a_max = max |a|; 0 for an empty cell.
 *   box_stats  NULL, or nboxes x 4 FP64: min over cells with n > 0 and
 *              a_max > 0 of v_rms/a_max (+inf if none), the box's global
 *              v_rms, global a_max and N -- the inputs of abacus_nf_timestep.
 * The particles may be stored in any order; the call checks a sample of the
 * permutation on the device and, unless they are mostly in the binning's cell
 * order, updates them in their own order first (the same bits either way);
 * storing them in cell order makes it fastest.
 * Results are run-to-run deterministic.  Errors: EINVAL for a bad box, a NULL
 * or non-finite factor, or NULL state arrays; EWORKSPACE as elsewhere.
 */
int abacus_nf_kick_drift(const abacus_nf_box *boxes, int nboxes, const abacus_nf_binned *b,
                         const double *kick, const double *drift, float *pos, float *vel,
                         const float *acc, double *cell_stats, double *box_stats, void *ws,
                         size_t ws_bytes, void *stream);

/* Eq. 1 for one box (host only):
 *   da = min(eta_H a, eta_acc a H max(min_c [v_rms/a_max]_c, v_rms/a_max global))
 * from the four box_stats values of abacus_nf_kick_drift; a global a_max of 0
 * counts as an infinite ratio.  NaN if box_stats is NULL. */
double abacus_nf_timestep(const double *box_stats, double a, double H, double eta_acc,
                          double eta_H);

/* ---- measurement hooks (not needed for computing) ------------------------ */
/* When enabled, the library records HIP events around its pair kernels on the
 * caller's stream; abacus_nf_timing_read returns the summed milliseconds and
 * launch count per kernel (0 = forward pair kernel, 1 = adjoint pair kernel,
 * 2 = binning, 3 = work plan, 4 = multipoles, 5 = kick-drift) since the last
 * reset, synchronising on the events; EINVAL for another id.
 * Do not enable while capturing a graph. */
int abacus_nf_timing_enable(int enable);
int abacus_nf_timing_read(int kernel, double *ms, int64_t *launches);
int abacus_nf_timing_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* ABACUS_NF_H */
