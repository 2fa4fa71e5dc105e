// Internal declarations shared by the host ABI and the kernels of libgccd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gccd {

constexpr int kFieldThreads = 256;   // threads per Eq. (6) workgroup (4 wave64)
constexpr int kTile = 256;           // sources staged in LDS per tile
constexpr int kMaxChunks = 64;       // largest source split of one target's sum
constexpr int kBoxRows = 126;        // per source tile: its box (rows 0-5), its four 64-slot
                                     // quarters' boxes (row 6 + 4 k + q for bound k of quarter
                                     // q), its sixteen 16-slot groups' boxes (row 30 + 16 k + g)
constexpr int kStepThreads = 256;
constexpr int kFusedList = 2048;     // largest load whose step kernel rebuilds the list itself
constexpr int kFusedTiles = 16;      // ... in at most this many source tiles

// Carrier lists hold one 64-bit key per carrier:
//   [event | collected | 36-bit Hilbert index of the 0.25 um cell | local index]
// with the local index (within its event) in the low lbits bits and the
// event in the top ebits bits (ebits + lbits <= 27).  Keys are unique, so
// sorting them is deterministic; the sorted list is one segment per event,
// in event order, each holding its travelling holes first and each part in
// spatial order, so nearby holes share workgroups and source tiles.
constexpr double kCellPerUm = 4.0;     // cells of 0.25 um along the curve
constexpr int kCurveBits = 36;         // 12 bits per axis (wraps every 1024 um)
constexpr int kMaxKeyPayload = 27;     // ebits + lbits

struct KeyLayout {
    uint32_t lbits;   // local index bits
    uint32_t ebits;   // event bits
};

// One work item of the Eq. (6) launch (one workgroup, or one turn of a
// persistent workgroup): targets [blk * 256 * TPT, ...) of the event's target
// slots, that is target block blk of an event against the event's source
// tiles first, first + step, first + 2 step, ... below min(end, the event's
// current tile count), summed into partial-sum group `group` of the event's
// `groups` (the FP64 mode writes its lo parts to group groups + group).
struct FieldItem {
    uint32_t event;
    uint32_t blk;
    uint32_t group;
    uint32_t groups;
    uint32_t first;
    uint32_t end;
    uint32_t step;
    uint32_t pad;
};
constexpr uint32_t kTilesToEnd = 0xFFFFFFFFu;  // FieldItem::end: up to the last tile

struct FieldArgs {
    const FieldItem* items;
    const uint32_t* ev_off;     // [E+1] first slot (and carrier) of each event
    const uint32_t* ev_active;  // [E] travelling holes of each event (first in its segment)
    const uint32_t* ev_tile;    // [E+1] first source tile of each event
    uint32_t one_event_n;       // > 0: a single event of this many carriers (slot 0,
                                // tile 0), whose offsets the expanded kernel need not read
    int32_t targets_all;        // 1: every carrier of the event is a target
    int32_t sources_all;        // 1: every carrier is a source, else the travelling ones
    const double* px;           // positions in list-slot order (gathered)
    const double* py;
    const double* pz;
    const double* tile_box;     // [kBoxRows][tile_stride] boxes of the source tiles
    uint32_t tile_stride;
    float eps2;                 // softening length squared, um^2
    double eps2d;               // the same in FP64 (FP64 mode)
    float* part;                // [group][3][pstride] FP32 partial sums by slot; the FP64
                                // mode writes group g's sum as hi in group g, lo in G + g
    uint32_t pstride;
    const uint32_t* n_items;    // persistent launch: the item count, in device memory
    uint32_t* queue;            // persistent launch: [0] next item (zero before the launch)
    int32_t near_compensated;   // one target per thread, default precision: tiles within
                                // rho/4 take the compensated difference (small launches)
    int32_t count_items;        // 1: the launch is sized to the item capacity and a
                                // workgroup past *n_items leaves at once (graph schedule)
    int32_t unit;               // sources per staged tile of the one-target-per-thread
                                // default kernel: kTile, kTile / 2 or kTile / 4 (the
                                // items count tiles of that size; other kernels: kTile)
    // Close pairs summed exactly (default precision): a pair with r^2 + eps^2 below
    // acc2 has its term formed in FP64 and added, in fixed point, to the target's
    // slot of `close` ([3][pstride] 64-bit integers, zero before the launch; the
    // consumer of the field reads and clears it); its FP32 term is dropped.
    float acc2;                 // (kExactRadius^2 + 1) eps^2
    double acc_box2;            // (kExactRadius eps)^2: a tile box at least this far from
                                // the targets' box holds no such pair
    double acc_scale;           // fixed-point units per um^-2
    unsigned long long* close;
};

// Pairs closer than kExactRadius softening lengths are summed exactly (see
// FieldArgs::close); the fixed-point unit is 2^-kExactShift / eps^2, so the
// largest term of Eq. (6), 0.385 / eps^2, takes 2^38.6 units.
constexpr double kExactRadius = 64.0;
constexpr int kExactShift = 40;

// Everything the per-carrier update of one step needs.
struct StepArgs {
    double* x;
    double* y;
    double* z;
    int32_t* cstep;
    int32_t list_mode;         // 1: slots of the sorted list (Coulomb on); 0: carriers
    const uint64_t* keys_in;   // the list this step runs over (list mode; its segments
                               // may be one step old: a hole travels while cstep < 0)
    uint64_t* keys_out;        // every slot's new key, before sorting (list mode)
    int32_t sort_runs;         // list mode: keys_out as sorted runs of kStepThreads slots
                               // (each workgroup turn sorts its own), for a sort that
                               // then only merges them
    const uint32_t* ev_off;    // [E+1]
    const uint32_t* ev_active; // [E] travelling holes of each event in keys_in (list mode)
    int32_t sources_all;       // sources of a target's Eq. (6) sum: its whole event, or
                               // (0) the ev_active travelling holes
    const int32_t* ev_chunks;  // [E] chunks of each event's field sum (list mode)
    const uint32_t* ev_of;     // [n] event of each carrier (carrier mode)
    int32_t one_event;         // 1: a single event (offset 0, every carrier), whose
                               // offsets and carrier events need not be read
    KeyLayout kl;
    const float* part;
    uint32_t pstride;
    uint32_t n_all;
    int32_t coulomb;
    int32_t diffusion;
    int32_t mobility_model;
    double K;                 // V um^2 / cm
    double a1, a2;            // Eq. (1)
    double thickness, z_well;
    double mu0, log_ec, beta, inv_beta;   // Eq. (2) at the context's T (log_ec = log Ec)
    double dt_s;              // time step, s
    double vt;                // k_B T / q, V
    uint32_t step;             // the step index, or its offset from *step_base
    const uint32_t* step_base; // list mode: device word added to step (a graph replays
                               // the same arguments at a new base)
    uint32_t event0;          // Philox event word of event 0
    uint32_t key0, key1;
    uint32_t* cnt_ring;       // [3] travelling holes at the start of step s in [s % 3]
    unsigned long long* close;  // list mode: the exactly summed close terms by slot
                                // ([3][pstride]); read and cleared
    double close_unit;          // um^-2 per fixed-point unit of close
    unsigned long long* stats;  // [0] carrier-steps, [1] pair interactions
    int32_t* misc;              // [0] non-finite flag, [1] step after the last busy one
    // A load of at most kFusedList carriers in at most kFusedTiles source
    // tiles (list mode): with arrive set, the
    // last workgroup of the step sorts keys_out into keys_sorted, writes each
    // event's travelling holes to ev_active_out and gathers the positions and
    // boxes of the n_tiles source tiles into px, py, pz, tile_box (what
    // sort_keys, count_active and gather_tiles do for larger loads).
    uint32_t* arrive;           // workgroups arrived ([1], zero between launches)
    uint64_t* keys_sorted;
    uint32_t* ev_active_out;
    uint32_t n_events;
    const uint32_t* ev_tile;
    const uint32_t* tile_event;
    uint32_t n_tiles;
    double* px;
    double* py;
    double* pz;
    double* tile_box;
    uint32_t box_stride;
};

// precision: a GCCD_PRECISION_* mode
int field_slots_per_cu(int tpt, int precision);
int field_queue_slots_per_cu();
// queue_grid > 0: the persistent launch of that many workgroups (one target
// per thread, default precision), after clearing the counter a.queue[0]
// grid_cap > 0 (one target per thread, default precision): grid_cap
// workgroups, those past the device-side item count *a.n_items leaving at
// once, so that one captured launch serves every item count up to the cap.
hipError_t launch_field(const FieldArgs& a, int tpt, int precision, uint32_t n_items,
                        uint32_t queue_grid, hipStream_t s, uint32_t grid_cap = 0);
hipError_t launch_step(const StepArgs& a, uint32_t n_slots, hipStream_t s);
hipError_t launch_load(double* z, int32_t* cstep, const uint32_t* ev_off, uint32_t* ev_of,
                       uint32_t n_events, uint32_t n, double thickness, double z_well,
                       uint32_t* cnt, hipStream_t s);
hipError_t launch_make_keys(const double* x, const double* y, const double* z,
                            const int32_t* cstep, const uint32_t* ev_of, const uint32_t* ev_off,
                            uint32_t n, KeyLayout kl, uint64_t* keys, hipStream_t s);
// launch_gather and launch_count in one launch (every hole a source).
hipError_t launch_gather_count(const uint64_t* keys, const uint32_t* ev_off,
                               const uint32_t* ev_tile, const uint32_t* tile_event,
                               uint32_t n_events, uint32_t n_tiles, KeyLayout kl, const double* x,
                               const double* y, const double* z, double* px, double* py,
                               double* pz, double* box, uint32_t stride, uint32_t* ev_active,
                               hipStream_t s);
hipError_t launch_gather(const uint64_t* keys, const uint32_t* ev_off, const uint32_t* ev_tile,
                         const uint32_t* tile_event, const uint32_t* ev_active, int sources_all,
                         uint32_t n_tiles, KeyLayout kl, const double* x, const double* y,
                         const double* z, double* px, double* py, double* pz, double* box,
                         uint32_t stride, hipStream_t s);
hipError_t launch_count(const uint64_t* keys, const uint32_t* ev_off, uint32_t n_events,
                        KeyLayout kl, uint32_t* ev_active, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// Sums the partial groups [g0, g0 + ev_chunks[e]) (or [g0, g0 + groups) when
// groups > 0) of every slot and writes K times the sum in carrier order.
// close (may be NULL): the exactly summed close terms by slot, added in and
// cleared (close_unit um^-2 per unit).
hipError_t launch_field_finish(const float* part, uint32_t pstride, const int32_t* ev_chunks,
                               int g0, int groups, const uint64_t* keys, const uint32_t* ev_off,
                               KeyLayout kl, uint32_t n, double K, unsigned long long* close,
                               double close_unit, double* ex, double* ey, double* ez,
                               hipStream_t s);
// gccd_field_noalloc: event tables, zeroed words and close sums, work items.
hipError_t launch_noalloc_setup(uint32_t n, uint32_t tiles, int32_t g, int32_t tail,
                                uint32_t split, uint32_t blocks, uint32_t* ev_off,
                                uint32_t* ev_tile, int32_t* ev_chunks, uint32_t* tile_event,
                                uint32_t* words, uint32_t n_words, FieldItem* items,
                                unsigned long long* close, hipStream_t s);
hipError_t launch_image(const double* x, const double* y, const int32_t* cstep,
                        const uint32_t* ev_of, uint32_t n, int per_event, double x0, double y0,
                        double pitch, int32_t nx, int32_t ny, uint32_t* counts,
                        unsigned long long* n_out, hipStream_t s);

// ---------------------------------------------------------------------------
// Far-field closure: the Eq. (6) sum split at a distance a into an exact
// near part (near_tiles) and a far part read from a 32^3 grid through a
// linear U-Net (bf16 MFMA convolutions) and Catmull-Rom interpolation.
// ---------------------------------------------------------------------------
constexpr int kGrid = 32;                    // nodes per axis
constexpr int kGridNodes = kGrid * kGrid * kGrid;
constexpr double kSigmaCells = 0.5;          // h = 0.5 x rms width per axis
constexpr double kMaxDevCells = 14.0;        // no charge farther than 14 h from the centroid
constexpr double kNearCells = 0.8;           // a = 0.8 h
constexpr int kMomBlocks = 512;              // fixed partition of the placement reduction

// Written on the device each time the closure field is computed.
struct GridParams {
    double origin[3];   // node 0 on each axis, um (node k at origin + k h)
    double h;           // node spacing, um
    double inv_h;
    double a2;          // a^2, um^2: source tiles farther than a are skipped
    double cut2;        // a^2 + eps^2: a pair counts while r^2 + eps^2 < cut2
    double inv_h2;      // 1 / h^2: the network's field unit K / h^2, over K
};

// One convolution of the network: out = W * in over a cubic grid of n^3
// nodes, channels last.  The input is channels [in_off, in_off + cin) of
// rows of in_stride bf16; the output goes to channels [out_off, out_off +
// cout) of rows of out_stride bf16, or to rows of 4 floats (the field).
struct ConvArgs {
    const uint16_t* in;
    int32_t in_stride, in_off, cin;
    const uint16_t* wpk;    // weights packed per 32-deep K slice and 16-wide N tile
    int32_t nslice, ntile, taps, n;
    uint16_t* out;          // bf16 output, or NULL
    float* outf;            // FP32 output [n^3][4], or NULL
    int32_t out_stride, out_off, cout;
};

hipError_t launch_near(const FieldArgs& a, const GridParams* gp, uint32_t n_items,
                       hipStream_t s);
hipError_t launch_moments(const double* x, const double* y, const double* z, uint32_t n,
                          double* part, hipStream_t s);
hipError_t launch_grid_params(const double* part, const double* x, const double* y,
                              const double* z, uint32_t n, double eps2, GridParams* gp,
                              hipStream_t s);
hipError_t launch_deposit(const double* px, const double* py, const double* pz, uint32_t n,
                          const GridParams* gp, unsigned long long* acc, hipStream_t s);
hipError_t launch_rho(const unsigned long long* acc, uint16_t* rho_bf16, float* rho_f32,
                      hipStream_t s);
hipError_t launch_conv(const ConvArgs& a, hipStream_t s);
hipError_t launch_pool(const uint16_t* in, int in_stride, int in_off, int c, int n_fine,
                       uint16_t* out, hipStream_t s);
hipError_t launch_upsample(const uint16_t* in, int c, int m, uint16_t* out, int out_stride,
                           int out_off, hipStream_t s);
hipError_t launch_far(const float* F, const GridParams* gp, const double* px, const double* py,
                      const double* pz, uint32_t nt, float* ox, float* oy, float* oz,
                      hipStream_t s);

// Sorts the n keys of `keys` into `out` (merge sort, gccd_sort.hip); `keys`
// is used as the other buffer of the merge levels and left in no useful order.
// run0 > 0: keys[0, n) already consists of sorted runs of run0 keys (a power
// of two from kSortItems to the block-sort tile), which are only merged.
hipError_t sort_keys(uint64_t* keys, uint64_t* out, uint32_t n, hipStream_t s,
                     uint32_t run0 = 0);

}  // namespace gccd
