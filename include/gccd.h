/*
 * gccd.h -- C ABI of the MI355X (gfx950) charge-transport hot path.
 *
 * Implements the time step of N. E. Avalos and M. Sofo Haro, "G-CoReCCD: a
 * GPU-based simulator of the charge transport in fully-depleted CCDs"
 * (arXiv 2203.11043): holes created in the bulk of a thick, fully depleted
 * CCD drift in the linear depletion field (Sec. II.A, Eq. (1)) at the
 * field-dependent mobility (Eq. (2)), diffuse (Sec. II.B, Eqs. (3)-(4)) and
 * repel each other through the softened all-pairs Coulomb field (Sec. III.B,
 * Eq. (6)) until they reach the potential well at the front surface, where
 * they are binned into pixels (Sec. V.A).
 *
 * Conventions
 *   - Units: lengths in micrometres, z measured from the collection plane
 *     (z = 0 at the front surface, +z into the bulk); fields in V/cm;
 *     mobility in cm^2/(V s); the time step in picoseconds.
 *   - Every function returns GCCD_OK (0) or a negative GCCD_E_* status and
 *     never throws.  gccd_strerror names a status; gccd_last_error gives the
 *     detail of the last failure on a context.
 *   - Array arguments are device pointers (HIP global memory) owned by the
 *     caller, read or written only during the call, in stream order on the
 *     context's stream.  The context owns its internal buffers.
 *   - Calls are asynchronous on the context's stream unless a description
 *     says it synchronises.  A context is not thread safe; different
 *     contexts are independent.
 *   - Carrier state lives in device memory as structure-of-arrays FP64
 *     positions plus an int32 collection step per carrier.
 */
#ifndef GCCD_H
#define GCCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCCD_ABI_VERSION 4u

enum {
    GCCD_OK = 0,
    GCCD_E_INVALID = -1,    /* an argument is out of range, NULL or non-finite  */
    GCCD_E_STATE = -2,      /* call out of order (e.g. run before load)         */
    GCCD_E_DEVICE = -3,     /* a HIP call failed; see gccd_last_error           */
    GCCD_E_NOMEM = -4,      /* device allocation failed                         */
    GCCD_E_NONFINITE = -5   /* a position became non-finite during a run        */
};

typedef struct gccd_ctx gccd_ctx;   /* opaque; owned by the library */

/* Device and physics settings.  The user inputs listed in Sec. III.B of the
 * paper (thickness, a1, a2 of Eq. (1), depth of the potential well, the
 * Coulomb switch) plus the temperature of Eqs. (2) and (4), the permittivity
 * and softening length of Eq. (6) and the random-number seed. */
typedef struct {
    uint32_t abi_version;      /* must equal GCCD_ABI_VERSION                         */
    uint32_t reserved0;        /* must be 0                                           */
    double thickness_um;       /* bulk thickness, > 0; z beyond it is mirrored back   */
    double a1_Vcm_per_um;      /* Eq. (1) slope: E_z(z) = a1 z - a2                   */
    double a2_Vcm;             /* Eq. (1) offset                                      */
    double well_z_um;          /* a hole with z <= well_z is collected; < thickness   */
    double temperature_K;      /* T of Eqs. (2) and (4), > 0                          */
    double eps_r;              /* relative permittivity in K = q/(4 pi eps0 eps_r), >0*/
    double softening_um;       /* epsilon of Eq. (6), > 0                             */
    int32_t coulomb;           /* 1: include Eq. (6); 0: drift and diffusion only     */
    int32_t diffusion;         /* 1: add the Brownian step of Sec. II.B               */
    int32_t mobility_model;    /* 0: Eq. (2); 1: constant low-field value of Eq. (2)  */
    int32_t collected_are_sources; /* 1: collected holes keep repelling (default)    */
    uint64_t seed;             /* Philox4x32-10 key (low word, high word)             */
    uint32_t event;            /* third word of every Philox counter                  */
    uint32_t reserved1;        /* must be 0                                           */
} gccd_params;

/* Counters kept by a context since its last gccd_load. */
typedef struct {
    int64_t step;              /* global step index of the next step                 */
    int64_t n_carriers;        /* N loaded                                            */
    int64_t n_active;          /* carriers still travelling                           */
    uint64_t carrier_steps;    /* sum over steps of the active carriers moved         */
    uint64_t pair_interactions;/* sum over steps of targets x sources of Eq. (6)      */
    double field_ms;           /* device time in the Eq. (6) kernel (timing on only)  */
    int64_t field_launches;    /* launches of that kernel while timing was on        */
    int32_t targets_per_thread;/* launch shape of the Eq. (6) launches               */
    int32_t source_chunks;     /* source chunks of event 0's field sum               */
    int64_t n_events;          /* events loaded                                       */
    int64_t max_source_chunks; /* largest source split over all events               */
    int64_t closure_steps;     /* steps whose Coulomb field came from the closure     */
    int64_t near_chunks;       /* source chunks of the closure's near sum (last run)  */
    int64_t graph_replays;     /* 32-step HIP graphs replayed by gccd_run (schedule GRAPH) */
    int32_t schedule;          /* the GCCD_SCHEDULE_* in force                        */
    int32_t graph_usable;      /* 0 once a capture for this load was refused          */
    int32_t tile_sources;      /* sources per staged tile of the Eq. (6) launches     */
    int32_t reserved;          /* 0                                                   */
} gccd_stats_t;

/* Creates a context bound to the current HIP device and to hip_stream (a
 * hipStream_t; NULL means the null stream).  Validates every field of *p
 * before touching the device: GCCD_E_INVALID for a wrong abi_version,
 * non-finite values, thickness, temperature, eps_r or softening <= 0,
 * well_z >= thickness, or switches outside {0, 1}.  GCCD_E_DEVICE when no
 * GPU is usable.  On success *out owns no carrier buffers yet. */
int gccd_init(const gccd_params* p, void* hip_stream, gccd_ctx** out);

/* Loads n carriers (Sec. III.B: the step loop starts from hole positions
 * that are already resident in device memory): x, y, z are device arrays of n FP64
 * positions in um, copied into the context.  A z beyond the back surface is
 * mirrored back; a z at or below the well is collected at step 0.  Resets the
 * step counter and every statistic.  Synchronises the stream.
 * GCCD_E_INVALID for n <= 0, n > 2^27 or a NULL pointer; GCCD_E_NOMEM if buffers cannot be allocated.  Non-finite
 * input positions make the next gccd_run return GCCD_E_NONFINITE. */
int gccd_load(gccd_ctx* c, int64_t n, const double* x, const double* y, const double* z);

/* Loads n_events independent events (each a separate cloud or track whose
 * holes repel only each other): offsets is a HOST array of n_events + 1
 * carrier offsets (offsets[0] = 0, strictly increasing, every event at least
 * one carrier); x, y, z are device arrays of offsets[n_events] FP64
 * positions, event e occupying [offsets[e], offsets[e+1]).  Event e draws
 * its diffusion steps with Philox counter (carrier index within the event,
 * step, params.event + e, 0), so each event evolves exactly as if it were
 * loaded alone with params.event + e.  Otherwise as gccd_load, which is the
 * one-event case.  GCCD_E_INVALID for bad offsets, more than 2^31-1 carriers
 * in total, or when the event count times the largest event exceeds 2^27. */
int gccd_load_events(gccd_ctx* c, int32_t n_events, const int64_t* offsets, const double* x,
                     const double* y, const double* z);

/* Advances the simulation (Sec. III.B, Fig. 2) by up to max_steps time steps
 * of dt_ps picoseconds.  Each step computes, for every travelling hole, the
 * static field of Eq. (1), the Coulomb field of Eq. (6) from the positions at
 * the start of the step, the mobility of Eq. (2) at the magnitude of their
 * sum, the drift mu E dt and the diffusion step of Eqs. (3)-(4) (Philox4x32-10
 * counter (carrier, step, event, 0), Box-Muller), then moves it in FP64 and
 * collects it when z <= well_z.  Stops early when no hole travels.  Runs are
 * cumulative: run(a) then run(b) equals run(a+b) bit for bit.  Synchronises
 * the stream every few steps and at return.  *steps_done (may be NULL) gets
 * the steps that had travelling holes, *n_active (may be NULL) the holes still
 * travelling; running out of steps is not an error.  GCCD_E_INVALID for
 * dt_ps <= 0 or max_steps < 0, GCCD_E_STATE before gccd_load,
 * GCCD_E_NONFINITE if a position became NaN or infinite (the context then
 * needs a new gccd_load before the next run, field or image). */
int gccd_run(gccd_ctx* c, double dt_ps, int64_t max_steps, int64_t* steps_done,
             int64_t* n_active);

/* Image of the collected holes (Sec. V.A: a 2D histogram of the final
 * positions, bin size equal to the pixel width).  Pixel (ix, iy) covers
 * [x0 + ix p, x0 + (ix+1) p) x [y0 + iy p, y0 + (iy+1) p), with the index
 * floor((x - x0) / p) computed in IEEE FP64.  counts is a device array of
 * ny*nx uint32, row-major (iy major), overwritten; *n_outside is a device
 * uint64 that receives the collected holes outside the grid.  Holes still
 * travelling are not counted.  GCCD_E_INVALID for pitch <= 0, nx or ny <= 0,
 * nx*ny > 2^31, non-finite origin, NULL pointers; GCCD_E_STATE before load. */
int gccd_image(gccd_ctx* c, double x0_um, double y0_um, double pitch_um, int32_t nx,
               int32_t ny, uint32_t* counts, uint64_t* n_outside);

/* As gccd_image, with one grid per event: counts is a device array of
 * n_events*ny*nx uint32 (event major), n_outside a device array of n_events
 * uint64. */
int gccd_image_events(gccd_ctx* c, double x0_um, double y0_um, double pitch_um, int32_t nx,
                      int32_t ny, uint32_t* counts, uint64_t* n_outside);

/* The Coulomb field of Eq. (6), in V/cm, at every loaded carrier from the
 * current sources of its own event (all its carriers, or only travelling ones
 * when collected_are_sources is 0), computed by the same kernel and source
 * split as gccd_run.  ex, ey, ez are device arrays of n FP64 values.
 * Synchronises the stream.  GCCD_E_STATE before load, GCCD_E_INVALID for
 * NULL pointers. */
int gccd_field(gccd_ctx* c, double* ex, double* ey, double* ez);

/* Copies the current FP64 positions and collection steps (-1 while a hole
 * travels, else the step count at which it arrived; 0 for holes loaded at or
 * below the well) into device arrays of n elements.  Any pointer may be NULL
 * to skip it.  GCCD_E_STATE before load. */
int gccd_positions(gccd_ctx* c, double* x, double* y, double* z, int32_t* collect_step);

/* Fills *out with the counters above; synchronises the stream. */
int gccd_stats(gccd_ctx* c, gccd_stats_t* out);

/* Fixes the launch shape of the Eq. (6) kernel: targets per thread (1, 2 or
 * 4) and the number of source chunks each target's sum is split into (1-64,
 * the same for every event, at most the event's tile count of 256 sources).
 * 0 for either means "choose automatically" (the default): one target per
 * thread, and per event a chunk count near the one that gives about 64
 * workgroups per compute unit, picked so that the event's tiles split into
 * chunks as nearly equal as possible.  With one target per thread in the
 * default precision, source tiles farther than the targets' box half-diagonal
 * are summed in the expanded-square form (see gccd_set_precision).  The
 * split changes the FP32 summation order; the targets per thread change the
 * workgroups' origins and so the rounding of the pair differences.  Applies
 * to the current load and later ones; synchronises the stream.
 * GCCD_E_INVALID outside those ranges. */
int gccd_set_launch(gccd_ctx* c, int32_t targets_per_thread, int32_t source_chunks);

/* Sources per tile of the Eq. (6) work split (the paper's Sec. III.B
 * kernel stages the sources through shared memory in blocks; here a work
 * item sums its target block against a run of such tiles): 64, 128 or 256,
 * or 0 for the automatic choice, which takes 64 when the load's work items
 * at that size still fit in one round of workgroups (a small cloud: more,
 * shorter items) and 256 otherwise.  Smaller tiles exist for one target per
 * thread in the default precision; other shapes and precisions use 256
 * whatever is set.  The tile size changes which tiles share a partial sum
 * and so the FP32 summation order.  Applies to the current load and later
 * ones; synchronises the stream.  GCCD_E_INVALID for any other value. */
int gccd_set_tile(gccd_ctx* c, int32_t sources);

/* Picks the launch shape of gccd_set_launch and gccd_set_tile by
 * measurement: times the Eq. (6) launch of the loaded state (its travelling
 * holes against their sources) for (targets per thread, tile sources) in
 * (1, 64), (1, 128), (1, 256), (2, 256), (4, 256) (the first two in the
 * default precision only) and source chunks 0 (automatic), 4, 8, 12, 16,
 * 20, 24, 28, 32, 36, 40, 48, 56, 64 (capped per event at its tile count),
 * the median of three launches each after one untimed, and keeps the
 * fastest for this load and later ones, as those calls would.  About 280
 * launches: call it once per workload.  The shape changes the FP32
 * summation order, so results are reproducible across processes only for
 * a fixed shape: the chosen values (any pointer may be NULL; the tile size
 * is gccd_stats' tile_sources) can be passed to gccd_set_launch and
 * gccd_set_tile.  Without Coulomb repulsion or travelling holes nothing is
 * timed and the current shape stays.  Synchronises the stream.
 * GCCD_E_STATE before load. */
int gccd_autotune(gccd_ctx* c, int32_t* targets_per_thread, int32_t* source_chunks,
                  double* ms_per_launch);

/* Arithmetic of the Eq. (6) pair sum.  The paper keeps positions as single
 * precision floats and gives no error analysis; these modes measure what
 * each design choice costs and buys.  Every FP32 mode forms pair
 * differences, r^2, r^-3 (hardware reciprocal square root, cubed) and the
 * per-tile sums in FP32; they differ in the origin the coordinates are
 * rounded relative to and in how the difference of a pair is formed.
 *   DEFAULT   origin at the centre of each workgroup's targets; pairs closer
 *             than a quarter of the target's distance from that origin
 *             (at most a quarter of the targets' half-diagonal rho)
 *             recomputed from the residuals of the coordinates (the fast,
 *             bounded mode).  With one target per thread, source tiles whose box is
 *             farther than rho from the targets' box take r^2 + eps^2 as
 *             (|s|^2 + eps^2) + |t|^2 - 2 t.s and the sum as t sum w - sum s w
 *             (one VALU operation fewer per pair; at most about 5e-6
 *             relative error per term there); and in a load whose work
 *             items fit in one round of workgroups (a small cloud), tiles
 *             within rho/4 take the compensated difference in every pair
 *             instead of the per-pair check
 *   BLOCK     the same origins, no close-pair recomputation
 *   EVENT     one origin per event (the centre of its sources' bounding
 *             box), no recomputation
 *   ABSOLUTE  no origin: FP32 absolute coordinates, as the paper stores them
 *   COMPENSATED  workgroup origins; every pair's difference formed from the
 *             coordinates and their residuals (double-single differences)
 *   FP64      every pair in FP64 (difference, r^2, r^-3 = 1/(q sqrt q)) and
 *             FP64 sums; reference quality, several times slower */
enum {
    GCCD_PRECISION_DEFAULT = 0,
    GCCD_PRECISION_BLOCK = 1,
    GCCD_PRECISION_EVENT = 2,
    GCCD_PRECISION_ABSOLUTE = 3,
    GCCD_PRECISION_COMPENSATED = 4,
    GCCD_PRECISION_FP64 = 5
};

/* Selects the arithmetic of the Eq. (6) kernel (GCCD_PRECISION_*) for gccd_run
 * and gccd_field.  The FP64 mode keeps each chunk's sum as two FP32 partial
 * groups and so splits a target's sum into at most 32 source chunks (a
 * larger gccd_set_launch value is clamped).  Applies to the current load and
 * later ones; synchronises the stream.  GCCD_E_INVALID for an unknown mode. */
int gccd_set_precision(gccd_ctx* c, int32_t mode);

/* How gccd_run issues the time steps of the exact path (Coulomb on, no
 * closure), the batched-events row of the work: thousands of events of
 * uneven size in one launch per step, over a list of work items (event,
 * target block, source chunk) ordered by cost, largest first.
 *   GRID   one workgroup per work item; each launch is sized to the items
 *   QUEUE  a persistent launch: as many workgroups as the GPU holds at once,
 *          each taking the next work item from a counter in device memory
 *          until the list is exhausted
 *   GRAPH  one workgroup per item of the load's item capacity (those past
 *          the item count, kept in device memory, leave at once), and each
 *          run of 32 consecutive steps (the stretch between two reads of the
 *          counts by the host) captured once as a HIP graph and replayed;
 *          the work items are rebuilt in place between replays, so one
 *          capture serves the whole run
 * QUEUE and GRAPH apply to one target per thread in the default precision;
 * other shapes use GRID.  A capture that fails, or that would hold a
 * memory-set node (the library's own steps issue none), is dropped: that
 * load's steps are then issued one by one.  Every schedule runs the
 * same item body on the same items, so results are bit-identical.
 * Per-launch timing (gccd_set_timing) needs events around each field
 * launch, which graph replays do not provide: with timing on, GRAPH issues
 * its steps one by one.  Default: GRAPH, the fastest measured on MI355X:
 * replays save the launch gaps of the short steps of small loads (0.037
 * against 0.044 ms per step at 1000 holes, 0.047 against 0.054 at 3000)
 * and are level with GRID at 1e5 holes and at the 4096-cloud batch; the
 * queue costs a reset launch and an atomic per item and is never faster.
 * Synchronises the
 * stream.  GCCD_E_INVALID for an unknown mode. */
enum {
    GCCD_SCHEDULE_GRID = 0,
    GCCD_SCHEDULE_QUEUE = 1,
    GCCD_SCHEDULE_GRAPH = 2
};
int gccd_set_schedule(gccd_ctx* c, int32_t mode);

/* Far-field closure.  The Eq. (6) sum is split at a distance a: sources
 * closer than a are summed exactly, pair by pair, as in the exact path; the
 * rest is read from a grid.  Every carrier (travelling or collected) deposits
 * its charge with trilinear weights on a 32^3 grid of spacing h centred on
 * the charges' centroid, h = max(0.5 s, d_max / 14) with s the rms width per
 * axis and d_max the largest offset of a charge from the centroid on any
 * axis; a = 0.8 h.  A linear U-Net maps the grid charge to the far field at
 * the nodes in units of K / h^2 (K of Eq. (6)), evaluated in bf16 on the
 * matrix cores with FP32 accumulation, and Catmull-Rom interpolation carries
 * it to the carriers.  The paper computes the full O(N^2) sum; the closure is
 * an approximation for large single clouds, trained on exact fields.
 *
 * The network: convolutions without bias, PyTorch Conv3d weight layout
 * (c_out, c_in, kz, ky, kx), in this order (name: c_in -> c_out, grid):
 *   e0a 1->16, e0b 16->16 (32^3); 2x2x2 mean; e1a 16->32, e1b 32->32 (16^3);
 *   mean; e2a 32->32, e2b 32->32 (8^3); mean; b3a 32->32, b3b 32->32 (4^3);
 *   x2 linear upsampling of b3b, joined with e2b -> d2 64->32 (8^3);
 *   upsampled d2 with e1b -> d1 64->32 (16^3); upsampled d1 with e0b ->
 *   d0 48->16 (32^3); head 16->3, 1x1x1 (32^3).  3x3x3 kernels with zero
 *   padding except the head; the joined tensors hold the upsampled channels
 *   first.  GCCD_CLOSURE_WEIGHTS floats in all. */
#define GCCD_CLOSURE_WEIGHTS 290784

/* Enables the closure for gccd_run and gccd_field when the load is a single
 * event of at least min_carriers holes with Coulomb repulsion on and
 * collected holes kept as sources; any other load uses the exact path (the
 * fallback).  weights is a HOST array of n_weights = GCCD_CLOSURE_WEIGHTS
 * FP32 values (copied and rounded to bf16); NULL disables the closure.
 * Synchronises the stream.  GCCD_E_INVALID for a wrong count, a negative
 * min_carriers or non-finite weights; GCCD_E_NOMEM if the grid buffers
 * cannot be allocated. */
int gccd_set_closure(gccd_ctx* c, const float* weights, int64_t n_weights,
                     int64_t min_carriers);

/* The closure's two parts at every loaded carrier, from the current
 * positions, whether or not the closure is enabled: near_* receives the exact
 * sum over the sources closer than a and far_* the interpolated far field
 * (zero when no weights are set), both in V/cm, carrier order, device arrays
 * of n doubles; rho (device, 32^3 floats, index (z * 32 + y) * 32 + x) the
 * deposited charge per node; grid (device, 4 doubles) the position of node 0
 * and the spacing h in um.  Uses the single event of the load.  Synchronises
 * the stream.  GCCD_E_STATE before load or with more than one event,
 * GCCD_E_INVALID for NULL pointers. */
int gccd_closure_parts(gccd_ctx* c, double* near_x, double* near_y, double* near_z,
                       double* far_x, double* far_y, double* far_z, float* rho, double* grid);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.
 *
 * The Eq. (6) field of n holes of one event, as gccd_init(p) + gccd_load(n,
 * x, y, z) + gccd_field + gccd_destroy return it in the default launch shape
 * and precision (the same kernels, work items and summation order: the same
 * values bit for bit), without allocating: every intermediate buffer lives in
 * one static device array of about 29 MB, which each GPU the library runs on
 * holds until the process ends.  x, y, z are device arrays of n FP64
 * positions in um (read only: the load-time mirror and collection are applied
 * to internal copies); ex, ey, ez device arrays of n FP64 values in V/cm,
 * carrier order.  Asynchronous on hip_stream (NULL: the null stream); no
 * host synchronisation, no memory-set commands.  Every call on a GPU uses
 * that GPU's one array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  GCCD_E_INVALID for
 * invalid parameters (as gccd_init), n < 1, n > GCCD_NOALLOC_MAX_CARRIERS or
 * NULL pointers; GCCD_E_DEVICE when a launch or copy fails. */
#define GCCD_NOALLOC_MAX_CARRIERS 32768
int gccd_field_noalloc(const gccd_params* p, int64_t n, const double* x, const double* y,
                       const double* z, double* ex, double* ey, double* ez, void* hip_stream);

/* on = 1 times every Eq. (6) launch with HIP events on the context's stream
 * (reported by gccd_stats); on = 0 stops timing. */
int gccd_set_timing(gccd_ctx* c, int32_t on);

const char* gccd_strerror(int status);
const char* gccd_last_error(const gccd_ctx* c);

/* Frees the context and its device buffers.  NULL is ignored. */
void gccd_destroy(gccd_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
