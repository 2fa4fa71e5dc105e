// Host side of the C ABI declared in include/gccd.h: parameter validation,
// device buffers, the step loop of Sec. III.B (Fig. 2), the spatially sorted
// carrier list and the work items of the Eq. (6) launch.
#include "gccd.h"
#include "gccd_internal.h"

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace gccd;

namespace {

// CODATA 2018 (SI): elementary charge, Boltzmann constant, vacuum permittivity.
constexpr double kQ = 1.602176634e-19;
constexpr double kKB = 1.380649e-23;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

constexpr int kPoll = 32;                       // steps between host reads of the counts
// Pair interactions per step from which the exact path pipelines its list
// (sorts the next step's keys on a second stream while the field runs).
// Below it the field launch is too short to hide the sort, and the sort's
// workgroups, which fit beside the field kernel's on no compute unit, wait
// for them and stretch the field launch's tail instead (measured on the muon
// track: 0.69 against 0.42 ms per step over its run).
constexpr double kPipeMinPairs = 5e9;
constexpr int64_t kMaxCarriers = 2147483647LL;  // slots are 32-bit

// Device block of counters (32-bit words): a ring of three travelling-hole
// counts by step mod 3, the non-finite flag, the step after the last step
// with travelling holes and two uint64 statistics.
enum : int {
    kMetaCount = 0,
    kMetaFlag = 3,
    kMetaLast = 4,
    kMetaStats = 8,
    kMetaWords = 16
};
// words of the schedule buffer (device, and a pinned host copy to upload from)
enum : int {
    kSchedQueue = 0,  // persistent launch: next work item
    kSchedItems = 1,  // persistent launch: work items in the list
    kSchedStep = 2,   // list mode: step index of the first step of the current stretch
    kSchedArrive = 3, // a small load's step kernel: its workgroups arrived (zero between)
    kSchedWords = 4
};

}  // namespace

struct gccd_ctx {
    gccd_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 256;

    // derived constants
    double K = 0, mu0 = 0, ec = 0, beta = 0, inv_beta = 0, vt = 0;

    // the loaded carriers
    bool loaded = false;
    bool list_mode = false;  // Coulomb on: the sorted list drives every step
    int64_t n = 0;
    uint32_t n_events = 0;
    KeyLayout kl{1, 0};
    std::vector<uint32_t> off_h;   // [E+1] first carrier of each event
    std::vector<uint32_t> tile_h;  // [E+1] first source tile of each event
    std::vector<int32_t> chunks_h; // [E] chunks of each event's field sum
    std::vector<int32_t> groups_h; // [E] partial-sum groups (2x chunks in the FP64 mode)
    std::vector<int32_t> tail_h;   // [E] chunks of the tail layer (0: one layer)
    std::vector<uint32_t> split_h; // [E] first tile of the tail layer
    std::vector<uint32_t> order_h; // events by decreasing size (work-item order)
    uint32_t n_tiles = 0;
    int max_chunks = 1;
    int max_groups = 1;

    double* x = nullptr;
    double* y = nullptr;
    double* z = nullptr;
    int32_t* cstep = nullptr;
    uint32_t* ev_of = nullptr;
    // The sorted lists.  keys[cur] is the list the next step runs over;
    // the step kernel writes every slot's new key into ukeys[u], which is
    // sorted into a list.  Steps of the exact path with every hole a source
    // are pipelined: the sort of the keys of step s+1's positions runs on the
    // side stream while step s+1 runs over the list of step s (the list only
    // orders the work; the travelling holes are told by their collection
    // step), and is used from step s+2 on.  Other steps sort before the next
    // step (the list then holds the positions it runs over).
    uint64_t* keys[2] = {nullptr, nullptr};
    uint64_t* ukeys[2] = {nullptr, nullptr};
    int cur = 0;
    int u = 0;
    bool sorting = false;            // the side stream sorts into keys[cur ^ 1]
    hipStream_t side = nullptr;      // default priority, like every stream here
    hipEvent_t ev_keys = nullptr;    // the step kernel has written ukeys
    hipEvent_t ev_list = nullptr;    // the side stream's list and counts are done
    double* ps[3] = {nullptr, nullptr, nullptr};
    double* tile_box = nullptr;
    float* part = nullptr;
    unsigned long long* close = nullptr;  // [3][n] fixed-point sums of exactly summed close pairs
    uint32_t* ev_off_d = nullptr;
    uint32_t* ev_tile_d = nullptr;
    uint32_t* tile_event_d = nullptr;
    uint32_t* ev_active_d[2] = {nullptr, nullptr};  // travelling holes per event, by list
    int32_t* ev_chunks_d = nullptr;
    FieldItem* items_d = nullptr;
    size_t items_cap = 0;
    uint32_t n_items = 0;
    uint32_t* meta = nullptr;
    uint32_t* host_meta = nullptr;    // pinned
    uint32_t* host_active = nullptr;  // pinned [E]
    FieldItem* host_items = nullptr;  // pinned [items_cap]

    int64_t step = 0;
    int64_t n_active = 0;

    int tpt_fixed = 0, chunks_fixed = 0;
    int tpt = 1;
    int unit = kTile;       // sources per staged tile of the Eq. (6) launch (choose_unit)
    int pipe_mode = -1;     // the list pipelined (1) or not (0); decided at load and
                            // at every step that is a multiple of kPoll
    int unit_fixed = 0;     // gccd_set_tile: 0 automatic
    int precision = GCCD_PRECISION_DEFAULT;

    // far-field closure (load-independent buffers)
    bool closure_on = false;
    int64_t closure_min = 0;
    uint16_t* wpk = nullptr;           // packed bf16 weights of every layer
    std::vector<size_t> wpk_off;       // offset of each layer in wpk (elements)
    uint16_t* act = nullptr;           // every bf16 activation buffer of the network
    float* fgrid = nullptr;            // far field at the nodes [32^3][4]
    float* rho_f32 = nullptr;          // deposited charge [32^3]
    unsigned long long* acc = nullptr; // fixed-point deposit [32^3]
    GridParams* gp = nullptr;
    double* mom = nullptr;             // [kMomBlocks][10]
    int part_groups = 0;               // capacity of part, in groups
    int near_chunks = 1;
    int groups_mode = 0;               // what ev_chunks_d holds: 0 exact groups, 1 closure
    int32_t closure_groups = 1;        // host copy of the closure's group count
    int64_t closure_steps = 0;

    // how gccd_run issues the steps (GCCD_SCHEDULE_*), and the captured graph
    int schedule = GCCD_SCHEDULE_GRAPH;
    uint32_t* sched = nullptr;       // [kSchedWords]
    uint32_t* host_sched = nullptr;  // pinned [kSchedWords]
    int queue_slots = 0;             // workgroups of the persistent launch per CU (0: not yet asked)
    bool near_compensated = false;   // the load's items fit in one round of workgroup slots
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr; // captures are recorded here (the context's stream
                                      // may be the null stream, which cannot capture)
    bool graph_refused = false;      // a capture for this load failed or held a memset node
    int graph_cur = -1, graph_u = -1;  // the list buffers the captured steps start from
    int graph_pipe = -1;               // ... and whether they pipeline the list
    int64_t graph_replays = 0;

    bool timing = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    double field_ms = 0;
    int64_t field_launches = 0;

    std::string err;
};

namespace {

int fail(gccd_ctx* c, int status, const char* what, hipError_t e = hipSuccess) {
    if (c) {
        char buf[512];
        if (e != hipSuccess)
            snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        else
            snprintf(buf, sizeof buf, "%s", what);
        c->err = buf;
    }
    return status;
}

#define GCCD_HIP(ctx, call)                                                  \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return fail((ctx), GCCD_E_DEVICE, #call, e_); \
    } while (0)

bool is_finite(double v) { return std::isfinite(v); }

int validate(const gccd_params* p) {
    if (!p) return GCCD_E_INVALID;
    if (p->abi_version != GCCD_ABI_VERSION || p->reserved0 != 0 || p->reserved1 != 0)
        return GCCD_E_INVALID;
    if (!is_finite(p->thickness_um) || !(p->thickness_um > 0)) return GCCD_E_INVALID;
    if (!is_finite(p->a1_Vcm_per_um) || !is_finite(p->a2_Vcm)) return GCCD_E_INVALID;
    if (!is_finite(p->well_z_um) || !(p->well_z_um < p->thickness_um)) return GCCD_E_INVALID;
    if (!is_finite(p->temperature_K) || !(p->temperature_K > 0)) return GCCD_E_INVALID;
    if (!is_finite(p->eps_r) || !(p->eps_r > 0)) return GCCD_E_INVALID;
    if (!is_finite(p->softening_um) || !(p->softening_um > 0)) return GCCD_E_INVALID;
    if ((p->coulomb | 1) != 1 || (p->diffusion | 1) != 1 || (p->mobility_model | 1) != 1 ||
        (p->collected_are_sources | 1) != 1)
        return GCCD_E_INVALID;
    return GCCD_OK;
}

template <typename T>
void dfree(T*& ptr) {
    (void)hipFree(ptr);
    ptr = nullptr;
}

template <typename T>
void hfree(T*& ptr) {
    (void)hipHostFree(ptr);
    ptr = nullptr;
}

// The captured steps refer to the load's buffers and launch shape: any change
// of those drops the graph (the next gccd_run captures again).
void drop_graph(gccd_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

void free_buffers(gccd_ctx* c) {
    if (c->side) (void)hipStreamSynchronize(c->side);  // a list may still be sorting
    drop_graph(c);
    c->graph_refused = false;
    c->sorting = false;
    dfree(c->x);
    dfree(c->y);
    dfree(c->z);
    dfree(c->cstep);
    dfree(c->ev_of);
    dfree(c->keys[0]);
    dfree(c->keys[1]);
    dfree(c->ukeys[0]);
    dfree(c->ukeys[1]);
    for (auto& q : c->ps) dfree(q);
    dfree(c->tile_box);
    dfree(c->part);
    dfree(c->close);
    dfree(c->ev_off_d);
    dfree(c->ev_tile_d);
    dfree(c->tile_event_d);
    dfree(c->ev_active_d[0]);
    dfree(c->ev_active_d[1]);
    dfree(c->ev_chunks_d);
    dfree(c->items_d);
    hfree(c->host_active);
    hfree(c->host_items);
    c->items_cap = 0;
    c->part_groups = 0;
    c->loaded = false;
}

void free_closure(gccd_ctx* c) {
    dfree(c->wpk);
    dfree(c->act);
    dfree(c->fgrid);
    dfree(c->rho_f32);
    dfree(c->acc);
    dfree(c->gp);
    dfree(c->mom);
    c->closure_on = false;
}

uint32_t bits_for(uint64_t count) {  // smallest b with 2^b >= count (0 for count <= 1)
    uint32_t b = 0;
    while ((1ull << b) < count) ++b;
    return b;
}

// Source chunks of each event's sum.  The split fixes the FP32 summation
// order, so it depends on the loaded sizes only, never on how many holes
// still travel: every step of a load, and gccd_field, sum in the same order.
// Enough workgroups to fill the chip (about 48 waves per SIMD in total,
// which also evens out workgroups that meet more close pairs), at most 3072
// sources per chunk, and at least one tile per chunk (a small cloud is
// latency-bound: it gains from every extra workgroup).  The FP64 mode stores
// each chunk's sum in two groups and so takes at most kMaxChunks / 2 chunks.
// An event's item length is set by its largest chunk, ceil(T/s) tiles of T;
// the mean is T/s.  Near the chunk count s0 that fills the GPU, take the count
// whose largest chunk is least above the mean (ties: the one nearest s0), so
// that no few chunks carry one tile more than all the others.
uint64_t balance_chunks(uint64_t tiles, uint64_t s0, uint64_t cap) {
    if (tiles <= s0) return s0;
    const uint64_t lo = std::max<uint64_t>(1, s0 * 9 / 10);
    const uint64_t hi = std::min<uint64_t>(std::min<uint64_t>(cap, tiles), s0 * 5 / 4);
    auto evenness = [tiles](uint64_t s) {
        return (double)tiles / (double)(s * ((tiles + s - 1) / s));
    };
    uint64_t best = s0;
    double best_e = evenness(s0);
    for (uint64_t s = lo; s <= hi; ++s) {
        const double e = evenness(s);
        const uint64_t d = s > s0 ? s - s0 : s0 - s, bd = best > s0 ? best - s0 : s0 - best;
        if (e > best_e + 1e-3 || (e > best_e - 1e-3 && d < bd)) {
            best = s;
            best_e = e;
        }
    }
    return best;
}

// The tail layer.  Work items of equal length end raggedly: once the list
// is dispatched, the compute units finish their last items over the span of
// one item, with fewer and fewer workgroups resident.  In a launch of only a
// few rounds of items that span is a sizeable share of the whole (measured:
// a 1e5-hole cloud, 8-tile items, kept its slots 89 % busy).  So, with the
// automatic choice, the largest events get a second layer: each of their last
// T2 tiles is a chunk of its own, listed after every first-layer item, T2
// chosen so that the tail work is about half a first-layer item per
// workgroup slot.  The first T1 = T - T2 tiles keep the balanced round-robin
// split.  The layers change which tiles share a partial sum, not the pairs
// summed.
// The tail layer of one event of `tiles` source tiles, `blocks` target
// blocks and s first-layer chunks, given the tile-units of tail work still
// wanted: fills chunks (both layers), tail (its chunks) and split (its first
// tile) and returns the work it takes, or 0 when the event gets no tail.
int64_t event_tail(uint64_t tiles, uint64_t blocks, uint64_t s, uint64_t cap, int64_t need,
                   int32_t* chunks, int32_t* tail, uint32_t* split) {
    uint64_t t2 = std::min<uint64_t>(tiles / 4, ((uint64_t)need + blocks - 1) / blocks);
    t2 = std::max<uint64_t>(t2, 1);
    const uint64_t s2 = t2;  // one tile per tail chunk
    if (s2 + 1 > cap) return 0;
    const uint64_t t1 = tiles - t2;
    const uint64_t s1 = balance_chunks(t1, std::min<uint64_t>({s, cap - s2, t1}), cap - s2);
    *chunks = (int32_t)(s1 + s2);
    *tail = (int32_t)s2;
    *split = (uint32_t)t1;
    return (int64_t)(blocks * t2);
}

void plan_tail(gccd_ctx* c, uint64_t cap) {
    c->tail_h.assign(c->n_events, 0);
    c->split_h.assign(c->n_events, 0);
    if (c->chunks_fixed) return;
    const uint64_t per = (uint64_t)kFieldThreads * (uint64_t)c->tpt;
    const uint64_t slots =
        (uint64_t)c->n_cu * (uint64_t)field_slots_per_cu(c->tpt, c->precision);
    uint64_t items = 0, big = 0;
    for (uint32_t e = 0; e < c->n_events; ++e) {
        const uint64_t ne = c->off_h[e + 1] - c->off_h[e];
        const uint64_t tiles = (ne + c->unit - 1) / c->unit, s = (uint64_t)c->chunks_h[e];
        items += (ne + per - 1) / per * s;
        big = std::max<uint64_t>(big, (tiles + s - 1) / s);
    }
    if (items >= 32 * slots || big < 4) return;  // many rounds, or items already short
    int64_t need = (int64_t)(slots * big / 2);    // tile-units of tail work wanted
    for (uint32_t e : c->order_h) {
        if (need <= 0) break;
        const uint64_t ne = c->off_h[e + 1] - c->off_h[e];
        const uint64_t tiles = (ne + c->unit - 1) / c->unit, blocks = (ne + per - 1) / per;
        const uint64_t s = (uint64_t)c->chunks_h[e];
        if ((tiles + s - 1) / s < 4) break;  // smaller events have short items already
        need -= event_tail(tiles, blocks, s, cap, need, &c->chunks_h[e], &c->tail_h[e],
                           &c->split_h[e]);
    }
}

// The automatic first-layer chunk count of an event of ne holes in tiles of
// `unit` sources when the load has tblocks target blocks in all.
uint64_t auto_chunks(uint64_t ne, uint64_t unit, uint64_t tblocks, int n_cu, uint64_t cap) {
    const uint64_t tiles = (ne + unit - 1) / unit;
    const uint64_t want = (uint64_t)n_cu * 64;
    uint64_t s = std::max<uint64_t>((ne + 3071) / 3072, (want + tblocks - 1) / tblocks);
    s = std::min<uint64_t>(s, std::max<uint64_t>(1, tiles));
    s = std::max<uint64_t>(s, 1);
    return balance_chunks(tiles, std::min<uint64_t>(s, cap), cap);
}

// Sources per staged tile of the one-target-per-thread default kernel:
// automatically kTile / 4 when even one such tile per chunk gives every
// target block's items a single round of workgroup slots (a small load,
// whose time is the length of one item), else kTile; other shapes and
// precisions always kTile.
uint64_t auto_unit(uint64_t items_at_quarter_tiles, int n_cu, int slots_per_cu) {
    return items_at_quarter_tiles <= (uint64_t)n_cu * (uint64_t)slots_per_cu ? kTile / 4 : kTile;
}

void choose_unit(gccd_ctx* c) {
    if (c->tpt != 1 || c->precision != GCCD_PRECISION_DEFAULT) {
        c->unit = kTile;
        return;
    }
    if (c->unit_fixed) {
        c->unit = c->unit_fixed;
        return;
    }
    uint64_t items = 0;
    for (uint32_t e = 0; e < c->n_events; ++e) {
        const uint64_t ne = c->off_h[e + 1] - c->off_h[e];
        items += (ne + kFieldThreads - 1) / kFieldThreads * ((ne + kTile / 4 - 1) / (kTile / 4));
    }
    c->unit = (int)auto_unit(items, c->n_cu, field_slots_per_cu(1, GCCD_PRECISION_DEFAULT));
}

void choose_chunks(gccd_ctx* c) {
    choose_unit(c);
    uint64_t tblocks = 0;
    for (uint32_t e = 0; e < c->n_events; ++e)
        tblocks += (c->off_h[e + 1] - c->off_h[e] + kFieldThreads * c->tpt - 1) /
                   (kFieldThreads * c->tpt);
    c->chunks_h.assign(c->n_events, 1);
    c->groups_h.assign(c->n_events, 1);
    c->max_chunks = 1;
    c->max_groups = 1;
    const bool split = c->precision == GCCD_PRECISION_FP64;
    const uint64_t cap = split ? kMaxChunks / 2 : kMaxChunks;
    for (uint32_t e = 0; e < c->n_events; ++e) {
        const uint64_t ne = c->off_h[e + 1] - c->off_h[e];
        const uint64_t tiles = (ne + c->unit - 1) / c->unit;
        uint64_t s;
        if (c->chunks_fixed) {
            // at most one chunk per tile: small events of a batch get no empty chunks
            s = std::min<uint64_t>((uint64_t)c->chunks_fixed, std::max<uint64_t>(1, tiles));
        } else {
            s = auto_chunks(ne, (uint64_t)c->unit, tblocks, c->n_cu, cap);
        }
        s = std::min<uint64_t>(s, cap);
        c->chunks_h[e] = (int32_t)s;
    }
    plan_tail(c, cap);
    for (uint32_t e = 0; e < c->n_events; ++e) {
        const int s = c->chunks_h[e];
        c->groups_h[e] = split ? 2 * s : s;
        c->max_chunks = std::max(c->max_chunks, s);
        c->max_groups = std::max(c->max_groups, c->groups_h[e]);
    }
}

// Work items for targets bound[e] of each event: largest events first, so the
// longest workgroups start early.  Within a target block the chunks are
// listed from chunk b mod S on: when S does not divide the tile count, the
// first chunks carry one tile more, and the rotation keeps those longer
// items from landing on the same compute units block after block (the
// dispatcher deals workgroups to the XCDs and their CUs in launch order).
// Only the launch order changes; each item's sums do not.
// The tail layers of all events follow all first layers.
int build_items(gccd_ctx* c, const uint32_t* bound) {
    const uint32_t per = (uint32_t)(kFieldThreads * c->tpt);
    size_t k = 0;
    for (int layer = 0; layer < 2; ++layer)
        for (uint32_t e : c->order_h) {
            const uint32_t blocks = (bound[e] + per - 1) / per;
            const uint32_t g = (uint32_t)c->chunks_h[e], s2 = (uint32_t)c->tail_h[e];
            if (layer == 1 && s2 == 0) continue;
            const uint32_t s = layer == 0 ? g - s2 : s2;       // chunks of this layer
            const uint32_t g0 = layer == 0 ? 0u : g - s2;      // its first group
            const uint32_t t0 = layer == 0 ? 0u : c->split_h[e];  // its first tile
            const uint32_t end = (layer == 0 && s2) ? c->split_h[e] : kTilesToEnd;
            for (uint32_t b = 0; b < blocks; ++b)
                for (uint32_t j = 0; j < s; ++j) {
                    if (k >= c->items_cap) return fail(c, GCCD_E_DEVICE, "work item overflow");
                    const uint32_t q = (j + b) % s;
                    c->host_items[k++] = FieldItem{e, b, g0 + q, g, t0 + q, end, s, 0};
                }
        }
    c->n_items = (uint32_t)k;
    if (k) {
        GCCD_HIP(c, hipMemcpyAsync(c->items_d, c->host_items, k * sizeof(FieldItem),
                                   hipMemcpyHostToDevice, c->stream));
    }
    // the persistent launch reads the count on the device (the host copy is
    // not written again before the stream has been synchronised)
    c->host_sched[kSchedItems] = (uint32_t)k;
    GCCD_HIP(c, hipMemcpyAsync(c->sched + kSchedItems, c->host_sched + kSchedItems,
                               sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    return GCCD_OK;
}

// Partial-sum buffer and work-item capacity for the current chunk choice.
int size_chunk_buffers(gccd_ctx* c) {
    drop_graph(c);
    dfree(c->part);
    dfree(c->items_d);
    hfree(c->host_items);
    size_t items = 0;
    for (uint32_t e = 0; e < c->n_events; ++e) {
        const uint64_t ne = c->off_h[e + 1] - c->off_h[e];
        items += (size_t)((ne + kFieldThreads - 1) / kFieldThreads) * (size_t)c->chunks_h[e];
    }
    c->items_cap = std::max<size_t>(items, 1);
    // a load whose items fit in one round of workgroup slots is latency-bound:
    // its close tiles take the branch-free compensated difference
    c->near_compensated =
        c->items_cap <= (size_t)c->n_cu * (size_t)field_slots_per_cu(1, GCCD_PRECISION_DEFAULT);
    c->groups_mode = 0;
    // the partial sums are only needed with repulsion on (a field call on a
    // load without it allocates them then: ensure_part)
    c->part_groups = c->p.coulomb ? c->max_groups : 0;
    if ((c->p.coulomb &&
         hipMalloc(&c->part, (size_t)c->max_groups * 3 * (size_t)c->n * sizeof(float)) !=
             hipSuccess) ||
        hipMalloc(&c->items_d, c->items_cap * sizeof(FieldItem)) != hipSuccess ||
        hipHostMalloc((void**)&c->host_items, c->items_cap * sizeof(FieldItem)) != hipSuccess)
        return fail(c, GCCD_E_NOMEM, "device allocation of the field buffers failed");
    GCCD_HIP(c, hipMemcpyAsync(c->ev_chunks_d, c->groups_h.data(), c->n_events * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    return GCCD_OK;
}

// The close-pair sums of the default precision: allocated with the partial
// sums, zero between launches (every consumer of a field launch clears the
// slots it reads).
int ensure_close(gccd_ctx* c) {
    if (c->close) return GCCD_OK;
    const size_t words = 3 * (size_t)c->n;
    if (hipMalloc(&c->close, words * sizeof(unsigned long long)) != hipSuccess)
        return fail(c, GCCD_E_NOMEM, "close-pair sum allocation failed");
    GCCD_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(c->close), 2 * words, 0u, c->stream));
    return GCCD_OK;
}

int ensure_part(gccd_ctx* c) {
    if (int r = ensure_close(c); r != GCCD_OK) return r;
    if (c->part_groups >= c->max_groups) return GCCD_OK;
    drop_graph(c);
    dfree(c->part);
    if (hipMalloc(&c->part, (size_t)c->max_groups * 3 * (size_t)c->n * sizeof(float)) !=
        hipSuccess)
        return fail(c, GCCD_E_NOMEM, "partial-sum allocation failed");
    c->part_groups = c->max_groups;
    return GCCD_OK;
}

int record_field_start(gccd_ctx* c, hipEvent_t** pair) {
    *pair = nullptr;
    if (!c->timing) return GCCD_OK;
    if (c->ev_used * 2 + 2 > (int)c->ev.size()) {
        for (int i = 0; i < 2 * kPoll; ++i) {
            hipEvent_t e;
            GCCD_HIP(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    *pair = &c->ev[c->ev_used * 2];
    ++c->ev_used;
    GCCD_HIP(c, hipEventRecord((*pair)[0], c->stream));
    return GCCD_OK;
}

// Called after the stream has been synchronised.
int collect_timing(gccd_ctx* c) {
    for (int i = 0; i < c->ev_used; ++i) {
        float ms = 0;
        GCCD_HIP(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        c->field_ms += ms;
        ++c->field_launches;
    }
    c->ev_used = 0;
    return GCCD_OK;
}

uint64_t meta64(const gccd_ctx* c, int word) {
    uint64_t v;
    memcpy(&v, c->host_meta + word, sizeof v);
    return v;
}

FieldArgs field_args(const gccd_ctx* c, bool targets_all) {
    FieldArgs fa{};
    fa.items = c->items_d;
    fa.ev_off = c->ev_off_d;
    fa.ev_active = c->ev_active_d[c->cur];
    fa.ev_tile = c->ev_tile_d;
    fa.one_event_n = c->n_events == 1 ? (uint32_t)c->n : 0u;
    fa.targets_all = targets_all ? 1 : 0;
    fa.sources_all = c->p.collected_are_sources;
    fa.px = c->ps[0];
    fa.py = c->ps[1];
    fa.pz = c->ps[2];
    fa.tile_box = c->tile_box;
    fa.tile_stride = std::max<uint32_t>(c->n_tiles, 1);
    fa.eps2 = (float)(c->p.softening_um * c->p.softening_um);
    fa.eps2d = c->p.softening_um * c->p.softening_um;
    fa.part = c->part;
    fa.pstride = (uint32_t)c->n;
    fa.n_items = c->sched + kSchedItems;
    fa.queue = c->sched + kSchedQueue;
    fa.near_compensated = c->near_compensated ? 1 : 0;
    fa.unit = c->unit;
    const double eps2 = c->p.softening_um * c->p.softening_um;
    fa.acc2 = (float)((kExactRadius * kExactRadius + 1.0) * eps2);
    fa.acc_box2 = kExactRadius * kExactRadius * eps2;
    fa.acc_scale = std::ldexp(eps2, kExactShift);
    fa.close = c->close;
    return fa;
}

// Workgroups of the persistent launch (the queue schedule), or 0.
uint32_t queue_grid(gccd_ctx* c) {
    if (c->schedule != GCCD_SCHEDULE_QUEUE || c->tpt != 1 ||
        c->precision != GCCD_PRECISION_DEFAULT)
        return 0;
    if (c->queue_slots == 0) c->queue_slots = field_queue_slots_per_cu();
    // no more workgroups than the load can ever have items (fixed per load,
    // so a captured graph stays valid as the items shrink)
    const size_t slots = (size_t)c->n_cu * (size_t)c->queue_slots;
    return (uint32_t)std::max<size_t>(1, std::min(slots, c->items_cap));
}

// The graph schedule's launch: one workgroup per item of the load's item
// capacity, those past the item count in device memory leaving at once
// (fixed per load, so a captured graph stays valid as the items shrink);
// 0 for the other schedules and shapes.
uint32_t graph_cap(const gccd_ctx* c) {
    if (c->schedule != GCCD_SCHEDULE_GRAPH || c->tpt != 1 ||
        c->precision != GCCD_PRECISION_DEFAULT)
        return 0;
    return (uint32_t)std::max<size_t>(1, c->items_cap);
}

// The current positions in the slot order of keys[cur], and the boxes of
// its source tiles.
int gather(gccd_ctx* c) {
    GCCD_HIP(c, launch_gather(c->keys[c->cur], c->ev_off_d, c->ev_tile_d, c->tile_event_d,
                              c->ev_active_d[c->cur], c->p.collected_are_sources, c->n_tiles,
                              c->kl, c->x, c->y, c->z, c->ps[0], c->ps[1], c->ps[2], c->tile_box,
                              std::max<uint32_t>(c->n_tiles, 1), c->stream));
    return GCCD_OK;
}

// The sorted list from the keys in `unsorted` (clobbered; with run0 > 0 it
// holds sorted runs of run0 keys): sort into keys[cur], count each event's
// travelling holes, gather the positions.
int finish_list(gccd_ctx* c, uint64_t* unsorted, uint32_t run0 = 0) {
    const uint32_t n = (uint32_t)c->n;
    GCCD_HIP(c, sort_keys(unsorted, c->keys[c->cur], n, c->stream, run0));
    if (c->p.collected_are_sources) {  // the gather needs no count: one launch
        GCCD_HIP(c, launch_gather_count(c->keys[c->cur], c->ev_off_d, c->ev_tile_d,
                                        c->tile_event_d, c->n_events, c->n_tiles, c->kl, c->x,
                                        c->y, c->z, c->ps[0], c->ps[1], c->ps[2], c->tile_box,
                                        std::max<uint32_t>(c->n_tiles, 1),
                                        c->ev_active_d[c->cur], c->stream));
        return GCCD_OK;
    }
    GCCD_HIP(c, launch_count(c->keys[c->cur], c->ev_off_d, c->n_events, c->kl,
                             c->ev_active_d[c->cur], c->stream));
    return gather(c);
}

// Leaves the pipelined state: the list being sorted on the side stream (the
// one of the current positions) becomes the current list.
int settle(gccd_ctx* c) {
    if (!c->sorting) return GCCD_OK;
    GCCD_HIP(c, hipStreamWaitEvent(c->stream, c->ev_list, 0));
    c->cur ^= 1;
    c->sorting = false;
    return gather(c);
}

int read_counts(gccd_ctx* c) {
    GCCD_HIP(c, hipMemcpyAsync(c->host_meta, c->meta, kMetaWords * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, c->stream));
    if (c->list_mode)
        GCCD_HIP(c, hipMemcpyAsync(c->host_active, c->ev_active_d[c->cur],
                                   c->n_events * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                   c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    return GCCD_OK;
}

// ---------------------------------------------------------------------------
// Far-field closure: network description, buffers, the field sequence.
// ---------------------------------------------------------------------------
struct LayerDesc {
    int cin, cout, taps;
};
// in the order of the weight array (the header lists the names)
constexpr LayerDesc kLayers[12] = {{1, 16, 27},  {16, 16, 27}, {16, 32, 27}, {32, 32, 27},
                                   {32, 32, 27}, {32, 32, 27}, {32, 32, 27}, {32, 32, 27},
                                   {64, 32, 27}, {64, 32, 27}, {48, 16, 27}, {16, 3, 1}};
enum : int { kE0a, kE0b, kE1a, kE1b, kE2a, kE2b, kB3a, kB3b, kD2, kD1, kD0, kHead };

// bf16 activation tensors, channels last: (nodes per axis, channels)
enum : int { kX0, kT0, kD0b, kP1, kT1, kD1b, kP2, kT2, kD2b, kP3, kT3, kB3, kE2, kE1, kE0, kNumAct };
constexpr int kActN[kNumAct] = {32, 32, 32, 16, 16, 16, 8, 8, 8, 4, 4, 4, 8, 16, 32};
constexpr int kActC[kNumAct] = {1, 16, 48, 16, 32, 64, 32, 32, 64, 32, 32, 32, 32, 32, 16};

size_t act_offset(int t) {
    size_t o = 0;
    for (int i = 0; i < t; ++i) o += (size_t)kActN[i] * kActN[i] * kActN[i] * kActC[i];
    return o;
}

uint16_t host_bf16(float f) {  // round to nearest, ties to even
    uint32_t b;
    memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

int ensure_closure_buffers(gccd_ctx* c) {
    if (c->act) return GCCD_OK;
    const size_t act = act_offset(kNumAct);
    if (hipMalloc(&c->act, act * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&c->fgrid, (size_t)kGridNodes * 4 * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->rho_f32, (size_t)kGridNodes * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->acc, (size_t)kGridNodes * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->gp, sizeof(GridParams)) != hipSuccess ||
        hipMalloc(&c->mom, (size_t)kMomBlocks * 10 * sizeof(double)) != hipSuccess) {
        free_closure(c);
        return fail(c, GCCD_E_NOMEM, "closure buffer allocation failed");
    }
    GCCD_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(c->fgrid), (uint64_t)kGridNodes * 4,
                                0u, c->stream));
    return GCCD_OK;
}

bool closure_applies(const gccd_ctx* c) {
    return c->closure_on && c->loaded && c->list_mode && c->n_events == 1 &&
           c->p.collected_are_sources && c->n >= c->closure_min;
}

// Source chunks of the near sum: as many as allowed (at least 4 candidate
// tiles per chunk, at most 32).  The near work of a target block varies by
// orders of magnitude (dense centre against sparse edge, and blocks whose
// box spans a jump of the spatial order see most tiles as near), so the
// split is chosen for the longest blocks, not to fill the chip: a chunk
// that finds no tile near costs only the scan of its candidates.
void choose_near_chunks(gccd_ctx* c) {
    const uint64_t tiles = ((uint64_t)c->n + kTile - 1) / kTile;
    const uint64_t s = std::min<uint64_t>(32, std::max<uint64_t>(1, tiles / 4));
    c->near_chunks = (int)s;
}

// part holds the near chunks plus one group for the far field; the item
// buffers hold every (target block, chunk) pair.
int ensure_closure_capacity(gccd_ctx* c) {
    const int groups = c->near_chunks + 1;
    if (groups > c->part_groups) {
        drop_graph(c);  // the captured steps name the old buffers
        dfree(c->part);
        if (hipMalloc(&c->part, (size_t)groups * 3 * (size_t)c->n * sizeof(float)) != hipSuccess)
            return fail(c, GCCD_E_NOMEM, "closure partial-sum allocation failed");
        c->part_groups = groups;
    }
    const size_t items = (((size_t)c->n + kFieldThreads - 1) / kFieldThreads) * c->near_chunks;
    if (items > c->items_cap) {
        drop_graph(c);
        dfree(c->items_d);
        hfree(c->host_items);
        if (hipMalloc(&c->items_d, items * sizeof(FieldItem)) != hipSuccess ||
            hipHostMalloc((void**)&c->host_items, items * sizeof(FieldItem)) != hipSuccess)
            return fail(c, GCCD_E_NOMEM, "closure work-item allocation failed");
        c->items_cap = items;
    }
    return GCCD_OK;
}

int build_near_items(gccd_ctx* c, uint32_t bound) {
    const uint32_t blocks = (bound + kFieldThreads - 1) / kFieldThreads;
    const uint32_t s = (uint32_t)c->near_chunks;
    size_t k = 0;
    for (uint32_t b = 0; b < blocks; ++b)
        for (uint32_t j = 0; j < s; ++j) {  // rotated as in build_items
            if (k >= c->items_cap) return fail(c, GCCD_E_DEVICE, "work item overflow");
            c->host_items[k++] = FieldItem{0, b, (j + b) % s, s, (j + b) % s, kTilesToEnd, s, 0};
        }
    c->n_items = (uint32_t)k;
    if (k) {
        GCCD_HIP(c, hipMemcpyAsync(c->items_d, c->host_items, k * sizeof(FieldItem),
                                   hipMemcpyHostToDevice, c->stream));
    }
    return GCCD_OK;
}

// What the step kernel and gccd_field sum per event: the exact path's groups,
// or the closure's near chunks plus the far group (single event).
int set_groups(gccd_ctx* c, int mode) {
    if (mode == c->groups_mode) return GCCD_OK;
    if (mode == 1) {
        c->closure_groups = c->near_chunks + 1;
        GCCD_HIP(c, hipMemcpyAsync(c->ev_chunks_d, &c->closure_groups, sizeof(int32_t),
                                   hipMemcpyHostToDevice, c->stream));
    } else {
        GCCD_HIP(c, hipMemcpyAsync(c->ev_chunks_d, c->groups_h.data(),
                                   c->n_events * sizeof(int32_t), hipMemcpyHostToDevice,
                                   c->stream));
    }
    GCCD_HIP(c, hipStreamSynchronize(c->stream));  // the host source may change next
    c->groups_mode = mode;
    return GCCD_OK;
}

int run_network(gccd_ctx* c) {
    uint16_t* A = c->act;
    auto T = [&](int t) { return A + act_offset(t); };
    auto conv = [&](int layer, int in, int in_off, int out, int out_off) -> hipError_t {
        const LayerDesc& L = kLayers[layer];
        ConvArgs a{};
        a.in = T(in);
        a.in_stride = kActC[in];
        a.in_off = in_off;
        a.cin = L.cin;
        a.wpk = c->wpk + c->wpk_off[layer];
        a.nslice = (L.taps * L.cin + 31) / 32;
        a.ntile = (L.cout + 15) / 16;
        a.taps = L.taps;
        a.n = kActN[in];
        a.cout = L.cout;
        if (out < 0) {
            a.outf = c->fgrid;
        } else {
            a.out = T(out);
            a.out_stride = kActC[out];
            a.out_off = out_off;
        }
        return launch_conv(a, c->stream);
    };
    hipStream_t st = c->stream;
    GCCD_HIP(c, conv(kE0a, kX0, 0, kT0, 0));
    GCCD_HIP(c, conv(kE0b, kT0, 0, kD0b, 32));            // skip 0 -> channels 32..47
    GCCD_HIP(c, launch_pool(T(kD0b), 48, 32, 16, 32, T(kP1), st));
    GCCD_HIP(c, conv(kE1a, kP1, 0, kT1, 0));
    GCCD_HIP(c, conv(kE1b, kT1, 0, kD1b, 32));            // skip 1 -> channels 32..63
    GCCD_HIP(c, launch_pool(T(kD1b), 64, 32, 32, 16, T(kP2), st));
    GCCD_HIP(c, conv(kE2a, kP2, 0, kT2, 0));
    GCCD_HIP(c, conv(kE2b, kT2, 0, kD2b, 32));            // skip 2 -> channels 32..63
    GCCD_HIP(c, launch_pool(T(kD2b), 64, 32, 32, 8, T(kP3), st));
    GCCD_HIP(c, conv(kB3a, kP3, 0, kT3, 0));
    GCCD_HIP(c, conv(kB3b, kT3, 0, kB3, 0));
    GCCD_HIP(c, launch_upsample(T(kB3), 32, 4, T(kD2b), 64, 0, st));
    GCCD_HIP(c, conv(kD2, kD2b, 0, kE2, 0));
    GCCD_HIP(c, launch_upsample(T(kE2), 32, 8, T(kD1b), 64, 0, st));
    GCCD_HIP(c, conv(kD1, kD1b, 0, kE1, 0));
    GCCD_HIP(c, launch_upsample(T(kE1), 32, 16, T(kD0b), 48, 0, st));
    GCCD_HIP(c, conv(kD0, kD0b, 0, kE0, 0));
    GCCD_HIP(c, conv(kHead, kE0, 0, -1, 0));
    return GCCD_OK;
}

// The closure's field of the current sorted list: near chunks into groups
// [0, S), the far field of target slots [0, nt) into group S.
int closure_field(gccd_ctx* c, bool targets_all, uint32_t nt, bool with_net) {
    const uint32_t n = (uint32_t)c->n;
    const double eps2 = c->p.softening_um * c->p.softening_um;
    hipStream_t st = c->stream;
    GCCD_HIP(c, launch_moments(c->ps[0], c->ps[1], c->ps[2], n, c->mom, st));
    GCCD_HIP(c, launch_grid_params(c->mom, c->ps[0], c->ps[1], c->ps[2], n, eps2, c->gp, st));
    GCCD_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(c->acc), 2ull * kGridNodes, 0u, st));
    GCCD_HIP(c, launch_deposit(c->ps[0], c->ps[1], c->ps[2], n, c->gp, c->acc, st));
    GCCD_HIP(c, launch_rho(c->acc, c->act + act_offset(kX0), c->rho_f32, st));
    if (with_net) {
        int r = run_network(c);
        if (r != GCCD_OK) return r;
    }
    FieldArgs fa = field_args(c, targets_all);
    GCCD_HIP(c, launch_near(fa, c->gp, c->n_items, st));
    float* far = c->part + (size_t)c->near_chunks * 3 * n;
    if (with_net)
        GCCD_HIP(c, launch_far(c->fgrid, c->gp, c->ps[0], c->ps[1], c->ps[2], nt, far, far + n,
                               far + 2 * (size_t)n, st));
    else
        GCCD_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(far), 3ull * n, 0u, st));
    return GCCD_OK;
}

}  // namespace

namespace {

// Captures kPoll steps issued by `issue` (step offsets 0 .. kPoll-1) as a
// graph, recorded on a stream of the context's own and replayed later on the
// caller's stream.  A capture that fails, or that holds a memory-set node
// (replays of such nodes are not trusted here), is dropped and the load
// marked: its steps are then issued one by one.  Nothing runs while
// capturing.
template <typename Issue>
int capture_steps(gccd_ctx* c, Issue& issue) {
    drop_graph(c);
    // issuing advances the list state; nothing runs while capturing, so it is
    // put back (a full stretch leaves it as it was; a refused one need not)
    const int cur0 = c->cur, u0 = c->u;
    const bool sorting0 = c->sorting;
    if (!c->cap_stream) GCCD_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    c->ev_used = 0;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    int r = GCCD_OK;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (uint32_t i = 0; i < (uint32_t)kPoll && r == GCCD_OK; ++i) r = issue(i, 0u);
        e = hipStreamEndCapture(c->stream, &g);
    }
    c->stream = user;
    c->ev_used = 0;
    c->cur = cur0;
    c->u = u0;
    c->sorting = sorting0;
    bool ok = r == GCCD_OK && e == hipSuccess && g != nullptr;
    if (ok) {
        size_t nn = 0;
        ok = hipGraphGetNodes(g, nullptr, &nn) == hipSuccess;
        std::vector<hipGraphNode_t> nodes(nn);
        if (ok && nn) ok = hipGraphGetNodes(g, nodes.data(), &nn) == hipSuccess;
        for (size_t i = 0; ok && i < nn; ++i) {
            hipGraphNodeType t;
            ok = hipGraphNodeGetType(nodes[i], &t) == hipSuccess && t != hipGraphNodeTypeMemset;
        }
    }
    if (ok) ok = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->err.clear();
        c->graph_refused = true;
        return GCCD_OK;
    }
    c->graph = g;
    return GCCD_OK;
}

}  // namespace

extern "C" {

const char* gccd_strerror(int status) {
    switch (status) {
        case GCCD_OK: return "ok";
        case GCCD_E_INVALID: return "invalid argument";
        case GCCD_E_STATE: return "call out of order";
        case GCCD_E_DEVICE: return "HIP device error";
        case GCCD_E_NOMEM: return "device out of memory";
        case GCCD_E_NONFINITE: return "non-finite carrier position";
        default: return "unknown status";
    }
}

const char* gccd_last_error(const gccd_ctx* c) { return c ? c->err.c_str() : ""; }

int gccd_init(const gccd_params* p, void* hip_stream, gccd_ctx** out) {
    if (!out) return GCCD_E_INVALID;
    *out = nullptr;
    int v = validate(p);
    if (v != GCCD_OK) return v;

    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return GCCD_E_DEVICE;
    gccd_ctx* c = new (std::nothrow) gccd_ctx;
    if (!c) return GCCD_E_NOMEM;
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return GCCD_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;

    // Eq. (6): K = q / (4 pi eps0 eps_r) in V m, times 1e12 um^2/m^2 and
    // 1e-2 (V/cm)/(V/m) gives V um^2 / cm.
    c->K = kQ / (4.0 * kPi * kEps0 * p->eps_r) * 1e12 * 1e-2;
    // Eq. (2) at temperature T.
    const double T = p->temperature_K;
    c->mu0 = 1.31e8 * pow(T, -2.2);
    c->ec = 1.24 * pow(T, 1.68);
    c->beta = 0.46 * pow(T, 0.17);
    c->inv_beta = 1.0 / c->beta;
    // Eq. (4): D = (k_B T / q) mu.
    c->vt = kKB * T / kQ;

    if (hipMalloc(&c->meta, kMetaWords * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&c->host_meta, kMetaWords * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->sched, kSchedWords * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&c->host_sched, kSchedWords * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(c->meta);
        (void)hipHostFree(c->host_meta);
        (void)hipFree(c->sched);
        delete c;
        return GCCD_E_NOMEM;
    }
    memset(c->host_sched, 0, kSchedWords * sizeof(uint32_t));
    if (hipMemcpy(c->sched, c->host_sched, kSchedWords * sizeof(uint32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->meta);
        (void)hipHostFree(c->host_meta);
        (void)hipFree(c->sched);
        (void)hipHostFree(c->host_sched);
        delete c;
        return GCCD_E_DEVICE;
    }
    *out = c;
    return GCCD_OK;
}

void gccd_destroy(gccd_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_buffers(c);
    free_closure(c);
    (void)hipFree(c->meta);
    (void)hipHostFree(c->host_meta);
    (void)hipFree(c->sched);
    (void)hipHostFree(c->host_sched);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_keys) (void)hipEventDestroy(c->ev_keys);
    if (c->ev_list) (void)hipEventDestroy(c->ev_list);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

int gccd_load_events(gccd_ctx* c, int32_t n_events, const int64_t* offsets, const double* x,
                     const double* y, const double* z) {
    if (!c) return GCCD_E_INVALID;
    if (n_events < 1 || !offsets || !x || !y || !z)
        return fail(c, GCCD_E_INVALID, "gccd_load_events: no events or NULL pointer");
    if (offsets[0] != 0) return fail(c, GCCD_E_INVALID, "gccd_load_events: offsets[0] != 0");
    int64_t max_ne = 0;
    for (int32_t e = 0; e < n_events; ++e) {
        const int64_t ne = offsets[e + 1] - offsets[e];
        if (ne < 1) return fail(c, GCCD_E_INVALID, "gccd_load_events: an event has no carrier");
        max_ne = std::max(max_ne, ne);
    }
    const int64_t n = offsets[n_events];
    if (n > kMaxCarriers) return fail(c, GCCD_E_INVALID, "gccd_load_events: too many carriers");
    const KeyLayout kl{std::max<uint32_t>(1, bits_for((uint64_t)max_ne)),
                       bits_for((uint64_t)n_events)};
    if (kl.lbits + kl.ebits > (uint32_t)kMaxKeyPayload)
        return fail(c, GCCD_E_INVALID,
                    "gccd_load_events: events x largest event exceed 2^27 key space");

    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    free_buffers(c);
    c->n = n;
    c->n_events = (uint32_t)n_events;
    c->kl = kl;
    c->tpt = c->tpt_fixed ? c->tpt_fixed : 1;
    c->off_h.resize(n_events + 1);
    c->tile_h.resize(n_events + 1);
    c->tile_h[0] = 0;
    for (int32_t e = 0; e <= n_events; ++e) c->off_h[e] = (uint32_t)offsets[e];
    for (int32_t e = 0; e < n_events; ++e)
        c->tile_h[e + 1] = c->tile_h[e] + (c->off_h[e + 1] - c->off_h[e] + kTile - 1) / kTile;
    c->n_tiles = c->tile_h[n_events];
    std::vector<uint32_t> tile_event(std::max<uint32_t>(c->n_tiles, 1), 0);
    for (int32_t e = 0; e < n_events; ++e)
        for (uint32_t t = c->tile_h[e]; t < c->tile_h[e + 1]; ++t) tile_event[t] = (uint32_t)e;
    c->order_h.resize(n_events);
    std::iota(c->order_h.begin(), c->order_h.end(), 0u);
    std::stable_sort(c->order_h.begin(), c->order_h.end(), [&](uint32_t a, uint32_t b) {
        return c->off_h[a + 1] - c->off_h[a] > c->off_h[b + 1] - c->off_h[b];
    });
    choose_chunks(c);

    const size_t d = (size_t)n * sizeof(double);
    const size_t E = (size_t)n_events;
    bool ok = hipMalloc(&c->x, d) == hipSuccess && hipMalloc(&c->y, d) == hipSuccess &&
              hipMalloc(&c->z, d) == hipSuccess &&
              hipMalloc(&c->cstep, (size_t)n * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&c->ev_of, (size_t)n * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->keys[0], (size_t)n * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&c->keys[1], (size_t)n * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&c->ukeys[0], (size_t)n * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&c->ukeys[1], (size_t)n * sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&c->ps[0], d) == hipSuccess && hipMalloc(&c->ps[1], d) == hipSuccess &&
              hipMalloc(&c->ps[2], d) == hipSuccess &&
              hipMalloc(&c->tile_box, kBoxRows * sizeof(double) * tile_event.size()) ==
                  hipSuccess &&
              hipMalloc(&c->ev_off_d, (E + 1) * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->ev_tile_d, (E + 1) * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->tile_event_d, tile_event.size() * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->ev_active_d[0], E * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->ev_active_d[1], E * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->ev_chunks_d, E * sizeof(int32_t)) == hipSuccess &&
              hipHostMalloc((void**)&c->host_active, E * sizeof(uint32_t)) == hipSuccess;
    if (!ok) {
        free_buffers(c);
        return fail(c, GCCD_E_NOMEM, "gccd_load_events: device allocation failed");
    }
    GCCD_HIP(c, hipMemcpyAsync(c->ev_off_d, c->off_h.data(), (E + 1) * sizeof(uint32_t),
                               hipMemcpyHostToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(c->ev_tile_d, c->tile_h.data(), (E + 1) * sizeof(uint32_t),
                               hipMemcpyHostToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(c->tile_event_d, tile_event.data(),
                               tile_event.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                               c->stream));
    {
        int r = c->p.coulomb ? ensure_close(c) : GCCD_OK;
        if (r == GCCD_OK) r = size_chunk_buffers(c);  // synchronises: tile_event may go out of scope
        if (r != GCCD_OK) {
            free_buffers(c);
            return r;
        }
    }

    GCCD_HIP(c, hipMemcpyAsync(c->x, x, d, hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(c->y, y, d, hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(c->z, z, d, hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, launch_fill_u32(c->meta, kMetaWords, 0u, c->stream));
    GCCD_HIP(c, launch_load(c->z, c->cstep, c->ev_off_d, c->ev_of, c->n_events, (uint32_t)n,
                            c->p.thickness_um, c->p.well_z_um, c->meta + kMetaCount, c->stream));
    c->list_mode = c->p.coulomb != 0;
    c->cur = 0;
    c->u = 0;
    c->pipe_mode = -1;
    if (c->list_mode) {
        GCCD_HIP(c, launch_make_keys(c->x, c->y, c->z, c->cstep, c->ev_of, c->ev_off_d,
                                     (uint32_t)n, c->kl, c->ukeys[0], c->stream));
        int r = finish_list(c, c->ukeys[0]);
        if (r != GCCD_OK) return r;
    }
    {
        int r = read_counts(c);
        if (r != GCCD_OK) return r;
    }
    c->n_active = c->host_meta[kMetaCount];
    c->step = 0;
    c->loaded = true;
    c->field_ms = 0;
    c->field_launches = 0;
    c->ev_used = 0;
    c->closure_steps = 0;
    return GCCD_OK;
}

int gccd_load(gccd_ctx* c, int64_t n, const double* x, const double* y, const double* z) {
    if (!c) return GCCD_E_INVALID;
    if (n <= 0 || n > (1ll << kMaxKeyPayload))
        return fail(c, GCCD_E_INVALID, "gccd_load: n out of range");
    const int64_t off[2] = {0, n};
    return gccd_load_events(c, 1, off, x, y, z);
}

int gccd_set_launch(gccd_ctx* c, int32_t tpt, int32_t chunks) {
    if (!c) return GCCD_E_INVALID;
    if (!(tpt == 0 || tpt == 1 || tpt == 2 || tpt == 4) || chunks < 0 || chunks > kMaxChunks)
        return fail(c, GCCD_E_INVALID, "gccd_set_launch: shape out of range");
    c->tpt_fixed = tpt;
    c->chunks_fixed = chunks;
    if (c->loaded) {
        GCCD_HIP(c, hipStreamSynchronize(c->stream));
        c->tpt = tpt ? tpt : 1;
        choose_chunks(c);
        int r = size_chunk_buffers(c);
        if (r != GCCD_OK) {
            free_buffers(c);
            return r;
        }
    }
    return GCCD_OK;
}

int gccd_set_tile(gccd_ctx* c, int32_t sources) {
    if (!c) return GCCD_E_INVALID;
    if (!(sources == 0 || sources == kTile / 4 || sources == kTile / 2 || sources == kTile))
        return fail(c, GCCD_E_INVALID, "gccd_set_tile: sources must be 0, 64, 128 or 256");
    c->unit_fixed = sources;
    if (c->loaded) {
        GCCD_HIP(c, hipStreamSynchronize(c->stream));
        choose_chunks(c);
        int r = size_chunk_buffers(c);
        if (r != GCCD_OK) {
            free_buffers(c);
            return r;
        }
    }
    return GCCD_OK;
}

int gccd_set_precision(gccd_ctx* c, int32_t mode) {
    if (!c) return GCCD_E_INVALID;
    if (mode < GCCD_PRECISION_DEFAULT || mode > GCCD_PRECISION_FP64)
        return fail(c, GCCD_E_INVALID, "gccd_set_precision: unknown mode");
    c->precision = mode;
    if (c->loaded) {
        GCCD_HIP(c, hipStreamSynchronize(c->stream));
        choose_chunks(c);
        int r = size_chunk_buffers(c);
        if (r != GCCD_OK) {
            free_buffers(c);
            return r;
        }
    }
    return GCCD_OK;
}

int gccd_set_schedule(gccd_ctx* c, int32_t mode) {
    if (!c) return GCCD_E_INVALID;
    if (mode < GCCD_SCHEDULE_GRID || mode > GCCD_SCHEDULE_GRAPH)
        return fail(c, GCCD_E_INVALID, "gccd_set_schedule: unknown mode");
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->graph_refused = false;
    c->schedule = mode;
    return GCCD_OK;
}

int gccd_set_closure(gccd_ctx* c, const float* weights, int64_t n_weights,
                     int64_t min_carriers) {
    if (!c) return GCCD_E_INVALID;
    if (weights && (n_weights != GCCD_CLOSURE_WEIGHTS || min_carriers < 0))
        return fail(c, GCCD_E_INVALID, "gccd_set_closure: wrong weight count or min_carriers");
    if (weights) {
        for (int64_t i = 0; i < n_weights; ++i)
            if (!std::isfinite(weights[i]))
                return fail(c, GCCD_E_INVALID, "gccd_set_closure: non-finite weight");
    }
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    dfree(c->wpk);
    c->closure_on = false;
    if (!weights) return GCCD_OK;

    // pack every layer in the B-operand order of the MFMA convolution
    std::vector<uint16_t> packed;
    c->wpk_off.clear();
    size_t src = 0;
    for (const LayerDesc& L : kLayers) {
        const int kmax = L.taps * L.cin;
        const int nslice = (kmax + 31) / 32, ntile = (L.cout + 15) / 16;
        c->wpk_off.push_back(packed.size());
        for (int s = 0; s < nslice; ++s)
            for (int t = 0; t < ntile; ++t)
                for (int l = 0; l < 64; ++l)
                    for (int i = 0; i < 8; ++i) {
                        const int k = s * 32 + (l >> 4) * 8 + i, co = t * 16 + (l & 15);
                        float v = 0.0f;
                        if (k < kmax && co < L.cout) {
                            const int tap = k / L.cin, ci = k % L.cin;
                            v = weights[src + ((size_t)co * L.cin + ci) * L.taps + tap];
                        }
                        packed.push_back(host_bf16(v));
                    }
        src += (size_t)L.cout * L.cin * L.taps;
    }
    if (src != (size_t)GCCD_CLOSURE_WEIGHTS)
        return fail(c, GCCD_E_INVALID, "gccd_set_closure: layer table and weight count differ");
    int r = ensure_closure_buffers(c);
    if (r != GCCD_OK) return r;
    if (hipMalloc(&c->wpk, packed.size() * sizeof(uint16_t)) != hipSuccess)
        return fail(c, GCCD_E_NOMEM, "gccd_set_closure: weight allocation failed");
    GCCD_HIP(c, hipMemcpyAsync(c->wpk, packed.data(), packed.size() * sizeof(uint16_t),
                               hipMemcpyHostToDevice, c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));  // packed goes out of scope
    c->closure_on = true;
    c->closure_min = min_carriers;
    return GCCD_OK;
}

int gccd_closure_parts(gccd_ctx* c, double* near_x, double* near_y, double* near_z,
                       double* far_x, double* far_y, double* far_z, float* rho, double* grid) {
    if (!c) return GCCD_E_INVALID;
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_closure_parts before gccd_load");
    if (c->n_events != 1)
        return fail(c, GCCD_E_STATE, "gccd_closure_parts: the load has more than one event");
    if (!near_x || !near_y || !near_z || !far_x || !far_y || !far_z || !rho || !grid)
        return fail(c, GCCD_E_INVALID, "gccd_closure_parts: NULL pointer");
    const uint32_t n = (uint32_t)c->n;
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    int r = ensure_closure_buffers(c);
    if (r != GCCD_OK) return r;
    if (!c->list_mode) {
        GCCD_HIP(c, launch_make_keys(c->x, c->y, c->z, c->cstep, c->ev_of, c->ev_off_d, n, c->kl,
                                     c->ukeys[0], c->stream));
        r = finish_list(c, c->ukeys[0]);
    } else {
        r = gather(c);  // the current positions in the order of the current list
    }
    if (r != GCCD_OK) return r;
    choose_near_chunks(c);
    r = ensure_closure_capacity(c);
    if (r == GCCD_OK) r = build_near_items(c, n);
    if (r == GCCD_OK) r = closure_field(c, true, n, c->wpk != nullptr);
    if (r != GCCD_OK) return r;
    const int S = c->near_chunks;
    GCCD_HIP(c, launch_field_finish(c->part, n, c->ev_chunks_d, 0, S, c->keys[c->cur], c->ev_off_d,
                                    c->kl, n, c->K, nullptr, 0.0, near_x, near_y, near_z,
                                    c->stream));
    GCCD_HIP(c, launch_field_finish(c->part, n, c->ev_chunks_d, S, 1, c->keys[c->cur], c->ev_off_d,
                                    c->kl, n, c->K, nullptr, 0.0, far_x, far_y, far_z, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(rho, c->rho_f32, (size_t)kGridNodes * sizeof(float),
                               hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(grid, c->gp, 4 * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    return GCCD_OK;
}

int gccd_autotune(gccd_ctx* c, int32_t* targets_per_thread, int32_t* source_chunks,
                  double* ms_per_launch) {
    if (!c) return GCCD_E_INVALID;
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_autotune before gccd_load");
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    double best_ms = -1.0;
    int best_t = c->tpt_fixed, best_s = c->chunks_fixed, best_u = c->unit_fixed;
    if (c->list_mode && c->n_active > 0) {
        hipEvent_t e0, e1;
        GCCD_HIP(c, hipEventCreate(&e0));
        GCCD_HIP(c, hipEventCreate(&e1));
        // (targets per thread, tile sources): smaller tiles exist for the
        // one-target-per-thread default kernel only
        static const int kTU[5][2] = {{1, kTile / 4}, {1, kTile / 2}, {1, kTile}, {2, kTile},
                                      {4, kTile}};
        static const int kS[14] = {0, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 48, 56, 64};
        int r = GCCD_OK;
        for (int ti = 0; ti < 5 && r == GCCD_OK; ++ti) {
            const int tpt = kTU[ti][0], unit = kTU[ti][1];
            if (c->precision != GCCD_PRECISION_DEFAULT && unit != kTile) continue;
            for (int si = 0; si < 14 && r == GCCD_OK; ++si) {
                c->tpt_fixed = tpt;
                c->chunks_fixed = kS[si];
                c->unit_fixed = unit;
                c->tpt = tpt;
                choose_chunks(c);
                r = size_chunk_buffers(c);
                if (r == GCCD_OK) r = build_items(c, c->host_active);
                if (r != GCCD_OK) break;
                FieldArgs fa = field_args(c, false);
                float t[3];
                for (int rep = 0; rep < 4 && r == GCCD_OK; ++rep) {  // one untimed, three timed
                    if (hipEventRecord(e0, c->stream) != hipSuccess ||
                        launch_field(fa, c->tpt, c->precision, c->n_items, queue_grid(c), c->stream,
                                     graph_cap(c)) !=
                            hipSuccess ||
                        hipEventRecord(e1, c->stream) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess)
                        r = fail(c, GCCD_E_DEVICE, "gccd_autotune: timed launch failed");
                    else if (rep > 0 && hipEventElapsedTime(&t[rep - 1], e0, e1) != hipSuccess)
                        r = fail(c, GCCD_E_DEVICE, "gccd_autotune: event timing failed");
                }
                if (r != GCCD_OK) break;
                std::sort(t, t + 3);
                if (best_ms < 0.0 || t[1] < best_ms) {
                    best_ms = t[1];
                    best_t = tpt;
                    best_s = kS[si];
                    best_u = unit;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // the timed launches left close-pair sums that nothing consumed
        if (r == GCCD_OK && c->close &&
            launch_fill_u32(reinterpret_cast<uint32_t*>(c->close), 6 * (uint64_t)c->n, 0u,
                            c->stream) != hipSuccess)
            r = fail(c, GCCD_E_DEVICE, "gccd_autotune: clearing the close-pair sums failed");
        if (r != GCCD_OK) {
            free_buffers(c);
            return r;
        }
    }
    // keep the fastest shape for this load and later ones
    c->tpt_fixed = best_t;
    c->chunks_fixed = best_s;
    c->unit_fixed = best_u;
    c->tpt = best_t ? best_t : 1;
    choose_chunks(c);
    int r = size_chunk_buffers(c);
    if (r != GCCD_OK) {
        free_buffers(c);
        return r;
    }
    if (targets_per_thread) *targets_per_thread = c->tpt;
    if (source_chunks) *source_chunks = best_s;
    if (ms_per_launch) *ms_per_launch = best_ms;
    return GCCD_OK;
}

int gccd_set_timing(gccd_ctx* c, int32_t on) {
    if (!c || (on | 1) != 1) return GCCD_E_INVALID;
    c->timing = on != 0;
    return GCCD_OK;
}

int gccd_run(gccd_ctx* c, double dt_ps, int64_t max_steps, int64_t* steps_done,
             int64_t* n_active) {
    if (!c) return GCCD_E_INVALID;
    if (!is_finite(dt_ps) || !(dt_ps > 0) || max_steps < 0)
        return fail(c, GCCD_E_INVALID, "gccd_run: dt_ps must be > 0 and max_steps >= 0");
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_run before gccd_load");
    if (c->step + max_steps > 4294967295LL)
        return fail(c, GCCD_E_INVALID, "gccd_run: step counter would exceed 2^32-1");

    const int64_t step0 = c->step;
    const uint32_t n = (uint32_t)c->n;
    int64_t bound = c->n_active;
    GCCD_HIP(c, hipStreamSynchronize(c->stream));  // the item staging buffer is free
    const bool use_closure = closure_applies(c);
    if (use_closure) {
        choose_near_chunks(c);
        int r = ensure_closure_capacity(c);
        if (r == GCCD_OK) r = set_groups(c, 1);
        if (r != GCCD_OK) return r;
    } else if (c->list_mode) {
        int r = set_groups(c, 0);
        if (r != GCCD_OK) return r;
    }
    auto rebuild = [&]() -> int {
        return use_closure ? build_near_items(c, (uint32_t)bound) : build_items(c, c->host_active);
    };
    if (c->list_mode && bound > 0) {
        int r = rebuild();
        if (r != GCCD_OK) return r;
    }

    StepArgs sa{};
    sa.x = c->x;
    sa.y = c->y;
    sa.z = c->z;
    sa.cstep = c->cstep;
    sa.list_mode = c->list_mode ? 1 : 0;
    sa.ev_off = c->ev_off_d;
    sa.sources_all = c->p.collected_are_sources;
    sa.ev_chunks = c->ev_chunks_d;
    sa.ev_of = c->ev_of;
    sa.one_event = c->n_events == 1 ? 1 : 0;
    sa.kl = c->kl;
    sa.part = c->part;
    sa.pstride = n;
    sa.n_all = n;
    sa.coulomb = c->p.coulomb;
    sa.diffusion = c->p.diffusion;
    sa.mobility_model = c->p.mobility_model;
    sa.K = c->K;
    sa.a1 = c->p.a1_Vcm_per_um;
    sa.a2 = c->p.a2_Vcm;
    sa.thickness = c->p.thickness_um;
    sa.z_well = c->p.well_z_um;
    sa.mu0 = c->mu0;
    sa.log_ec = std::log(c->ec);
    sa.beta = c->beta;
    sa.inv_beta = c->inv_beta;
    sa.dt_s = dt_ps * 1e-12;
    sa.vt = c->vt;
    sa.event0 = c->p.event;
    sa.key0 = (uint32_t)c->p.seed;
    sa.key1 = (uint32_t)(c->p.seed >> 32);
    sa.close = c->list_mode ? c->close : nullptr;
    sa.close_unit = std::ldexp(1.0 / (c->p.softening_um * c->p.softening_um), -kExactShift);
    sa.cnt_ring = c->meta + kMetaCount;
    sa.stats = reinterpret_cast<unsigned long long*>(c->meta + kMetaStats);
    sa.misc = reinterpret_cast<int32_t*>(c->meta + kMetaFlag);

    // A small load's step kernel rebuilds the list itself (its last
    // workgroup sorts, counts and gathers: two launches per step).  Other
    // exact steps with every hole a source are pipelined (see gccd_ctx::keys)
    // while their pair work hides the sort (kPipeMinPairs); the others need
    // the list of the positions they run over.  The choice is made at load
    // and at every step that is a multiple of kPoll (the polls are aligned to
    // those steps), from the counts there, so a run gives the same bits however
    // it is split into calls.
    const bool fused = c->list_mode && !use_closure && n <= (uint32_t)kFusedList &&
                       c->n_tiles <= (uint32_t)kFusedTiles;
    const bool pipe_ok = !fused && c->list_mode && !use_closure && c->p.collected_are_sources;
    auto decide_pipe = [&]() -> int {
        if (!pipe_ok) return 0;
        double pairs = 0.0;
        for (uint32_t e = 0; e < c->n_events; ++e) {
            const double a = (double)c->host_active[e];
            pairs += a * (c->p.collected_are_sources ? (double)(c->off_h[e + 1] - c->off_h[e]) : a);
        }
        return pairs >= kPipeMinPairs ? 1 : 0;
    };
    if (!pipe_ok)
        c->pipe_mode = 0;
    else if (c->pipe_mode < 0 || step0 % kPoll == 0)
        c->pipe_mode = decide_pipe();
    bool pipelined = c->pipe_mode == 1;
    if (fused) {
        sa.arrive = c->sched + kSchedArrive;
        sa.n_events = c->n_events;
        sa.ev_tile = c->ev_tile_d;
        sa.tile_event = c->tile_event_d;
        sa.n_tiles = c->n_tiles;
        sa.px = c->ps[0];
        sa.py = c->ps[1];
        sa.pz = c->ps[2];
        sa.tile_box = c->tile_box;
        sa.box_stride = std::max<uint32_t>(c->n_tiles, 1);
    }
    // Puts the list state in line with `pipelined`.
    auto enter_mode = [&]() -> int {
        if (c->list_mode && !pipelined) {
            int r = settle(c);
            if (r != GCCD_OK) return r;
        }
        if (pipelined && !c->side) {
            GCCD_HIP(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
            GCCD_HIP(c, hipEventCreateWithFlags(&c->ev_keys, hipEventDisableTiming));
            GCCD_HIP(c, hipEventCreateWithFlags(&c->ev_list, hipEventDisableTiming));
        }
        if (pipelined && !c->sorting && bound > 0) {
            // Enter the steady state: the next step's list (the current one) also
            // stands in keys[cur ^ 1] as if the side stream had sorted it.  The
            // next two steps run over the same list either way, so results do not
            // change; every stretch then starts alike and can be captured.
            const size_t kb = (size_t)c->n * sizeof(uint64_t);
            GCCD_HIP(c, hipMemcpyAsync(c->keys[c->cur ^ 1], c->keys[c->cur], kb,
                                       hipMemcpyDeviceToDevice, c->stream));
            GCCD_HIP(c, hipMemcpyAsync(c->ev_active_d[c->cur ^ 1], c->ev_active_d[c->cur],
                                       c->n_events * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                       c->stream));
            GCCD_HIP(c, hipEventRecord(c->ev_list, c->stream));
            c->sorting = true;
        }
        return GCCD_OK;
    };
    {
        int r = enter_mode();
        if (r != GCCD_OK) return r;
    }
    int64_t stretch = 0;  // steps of the stretch being issued

    // One time step: in list mode step i of the current stretch (its index is
    // the base in sched[kSchedStep] plus i), else absolute step s.
    if (c->list_mode) sa.step_base = c->sched + kSchedStep;
    auto issue = [&](uint32_t i, uint32_t s) -> int {
        if (c->list_mode) {
            sa.step = i;
            if (pipelined) {
                int r = gather(c);  // this step's positions in the order of keys[cur]
                if (r != GCCD_OK) return r;
            }
            hipEvent_t* evp = nullptr;
            int r = record_field_start(c, &evp);
            if (r != GCCD_OK) return r;
            if (use_closure) {
                r = closure_field(c, false, (uint32_t)bound, true);
                if (r != GCCD_OK) return r;
            } else {
                FieldArgs fa = field_args(c, false);
                GCCD_HIP(c, launch_field(fa, c->tpt, c->precision, c->n_items, queue_grid(c),
                                         c->stream, graph_cap(c)));
            }
            if (evp) GCCD_HIP(c, hipEventRecord(evp[1], c->stream));
            sa.keys_in = c->keys[c->cur];
            sa.keys_out = c->ukeys[c->u];
            // a serial list: the step kernel's workgroups sort their slots'
            // keys into runs, so the sort only merges them (the side stream's
            // sort of a pipelined list overlaps the field and gains nothing)
            sa.sort_runs = (!fused && !pipelined) ? 1 : 0;
            sa.ev_active = c->ev_active_d[c->cur];
            if (fused) {  // the kernel leaves the next step's list in place of this one's
                sa.keys_sorted = c->keys[c->cur];
                sa.ev_active_out = c->ev_active_d[c->cur];
            }
            GCCD_HIP(c, launch_step(sa, n, c->stream));
            if (fused) return GCCD_OK;
            if (!pipelined)  // the next step's list, from the runs the step kernel sorted
                return finish_list(c, c->ukeys[c->u], kStepThreads);
            // The list of the new positions is sorted on the side stream while
            // the next step runs over the one the side stream finished last
            // (the first step of a stretch follows the join of the last one).
            GCCD_HIP(c, hipEventRecord(c->ev_keys, c->stream));
            if (c->sorting) {
                if (i != 0) GCCD_HIP(c, hipStreamWaitEvent(c->stream, c->ev_list, 0));
                c->cur ^= 1;
            }
            const int dst = c->cur ^ 1;  // the list the step just finished used, or a free one
            GCCD_HIP(c, hipStreamWaitEvent(c->side, c->ev_keys, 0));
            GCCD_HIP(c, sort_keys(c->ukeys[c->u], c->keys[dst], n, c->side));
            GCCD_HIP(c, launch_count(c->keys[dst], c->ev_off_d, c->n_events, c->kl,
                                     c->ev_active_d[dst], c->side));
            GCCD_HIP(c, hipEventRecord(c->ev_list, c->side));
            c->sorting = true;
            c->u ^= 1;
            if ((int64_t)i + 1 == stretch)  // join: the stretch ends with its last sort done
                GCCD_HIP(c, hipStreamWaitEvent(c->stream, c->ev_list, 0));
            return GCCD_OK;
        }
        sa.step = s;
        GCCD_HIP(c, launch_step(sa, n, c->stream));
        return GCCD_OK;
    };
    // per-launch timing events cannot be read back from graph replays here:
    // with timing on, the steps are issued one by one
    const bool graphable = c->list_mode && !use_closure && !c->timing &&
                           graph_cap(c) > 0;

    int64_t k = 0;
    while (k < max_steps && bound > 0) {
        // stretches end at multiples of kPoll (a call that starts between
        // them first runs up to the next)
        const int64_t to_poll = kPoll - (step0 + k) % kPoll;
        const int64_t chunk_steps = (max_steps - k < to_poll) ? (max_steps - k) : to_poll;
        if (c->list_mode) {
            // the host copy is free: the stream was synchronised at the last poll
            c->host_sched[kSchedStep] = (uint32_t)(step0 + k);
            GCCD_HIP(c, hipMemcpyAsync(c->sched + kSchedStep, c->host_sched + kSchedStep,
                                       sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
        }
        stretch = chunk_steps;
        bool replayed = false;
        // a pipelined stretch is replayed from the list buffers it was
        // captured from (an even stretch leaves them as it found them)
        if (graphable && chunk_steps == kPoll && !c->graph_refused) {
            if (c->graph_exec && (c->graph_cur != c->cur || c->graph_u != c->u ||
                                  c->graph_pipe != (pipelined ? 1 : 0)))
                drop_graph(c);
            if (!c->graph_exec) {
                int r = capture_steps(c, issue);
                if (r != GCCD_OK) return r;
                c->graph_cur = c->cur;
                c->graph_u = c->u;
                c->graph_pipe = pipelined ? 1 : 0;
            }
            if (c->graph_exec) {
                GCCD_HIP(c, hipGraphLaunch(c->graph_exec, c->stream));
                ++c->graph_replays;
                replayed = true;
            }
        }
        if (!replayed) {
            for (int64_t i = 0; i < chunk_steps; ++i) {
                int r = issue((uint32_t)i, (uint32_t)(step0 + k + i));
                if (r != GCCD_OK) return r;
            }
        }
        k += chunk_steps;
        int r = read_counts(c);
        if (r != GCCD_OK) return r;
        if (c->timing) {
            r = collect_timing(c);
            if (r != GCCD_OK) return r;
        }
        bound = c->host_meta[kMetaCount + (uint32_t)(step0 + k) % 3u];
        if (c->host_meta[kMetaFlag] != 0) {
            c->step = (int64_t)(uint32_t)c->host_meta[kMetaLast];
            c->n_active = bound;
            c->loaded = false;
            return fail(c, GCCD_E_NONFINITE,
                        "gccd_run: a carrier position became non-finite; reload to continue");
        }
        if (pipe_ok && (step0 + k) % kPoll == 0) {
            // the list pipelined or not for the next stretch
            c->pipe_mode = decide_pipe();
            if ((c->pipe_mode == 1) != pipelined && bound > 0 && k < max_steps) {
                pipelined = c->pipe_mode == 1;
                r = enter_mode();
                if (r != GCCD_OK) return r;
            }
        }
        if (c->list_mode && bound > 0 && k < max_steps) {
            r = rebuild();  // counts only shrink: fewer items
            if (r != GCCD_OK) return r;
        }
    }
    // The step after the last one that moved a hole: later steps found no hole
    // travelling and left the state unchanged.
    const int64_t last = (k > 0) ? (int64_t)(uint32_t)c->host_meta[kMetaLast] : step0;
    c->step = (last > step0) ? last : step0;
    c->n_active = bound;
    if (use_closure) c->closure_steps += c->step - step0;
    if (steps_done) *steps_done = c->step - step0;
    if (n_active) *n_active = c->n_active;
    return GCCD_OK;
}

int gccd_field(gccd_ctx* c, double* ex, double* ey, double* ez) {
    if (!c) return GCCD_E_INVALID;
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_field before gccd_load");
    if (!ex || !ey || !ez) return fail(c, GCCD_E_INVALID, "gccd_field: NULL pointer");
    const uint32_t n = (uint32_t)c->n;
    GCCD_HIP(c, hipStreamSynchronize(c->stream));  // the item staging buffer is free
    {
        int r;
        if (!c->list_mode) {
            // no list is kept without Coulomb repulsion: build one for this call
            GCCD_HIP(c, launch_make_keys(c->x, c->y, c->z, c->cstep, c->ev_of, c->ev_off_d, n,
                                         c->kl, c->ukeys[0], c->stream));
            r = finish_list(c, c->ukeys[0]);
        } else {
            r = gather(c);  // the current positions in the order of the current list
        }
        if (r != GCCD_OK) return r;
    }
    if (closure_applies(c)) {
        choose_near_chunks(c);
        int r = ensure_closure_capacity(c);
        if (r == GCCD_OK) r = set_groups(c, 1);
        if (r == GCCD_OK) r = build_near_items(c, n);
        if (r == GCCD_OK) r = closure_field(c, true, n, true);
        if (r != GCCD_OK) return r;
    } else {
        int r = ensure_part(c);
        if (r == GCCD_OK) r = set_groups(c, 0);
        if (r != GCCD_OK) return r;
        std::vector<uint32_t> all(c->n_events);
        for (uint32_t e = 0; e < c->n_events; ++e) all[e] = c->off_h[e + 1] - c->off_h[e];
        r = build_items(c, all.data());
        if (r != GCCD_OK) return r;
        FieldArgs fa = field_args(c, true);
        GCCD_HIP(c, launch_field(fa, c->tpt, c->precision, c->n_items, queue_grid(c), c->stream,
                                 graph_cap(c)));
    }
    GCCD_HIP(c, launch_field_finish(
                    c->part, n, c->ev_chunks_d, 0, 0, c->keys[c->cur], c->ev_off_d, c->kl, n, c->K,
                    c->close, std::ldexp(1.0 / (c->p.softening_um * c->p.softening_um), -kExactShift),
                    ex, ey, ez, c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));  // host_items may be rebuilt next
    return GCCD_OK;
}

int gccd_positions(gccd_ctx* c, double* x, double* y, double* z, int32_t* collect_step) {
    if (!c) return GCCD_E_INVALID;
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_positions before gccd_load");
    const size_t d = (size_t)c->n * sizeof(double);
    if (x) GCCD_HIP(c, hipMemcpyAsync(x, c->x, d, hipMemcpyDeviceToDevice, c->stream));
    if (y) GCCD_HIP(c, hipMemcpyAsync(y, c->y, d, hipMemcpyDeviceToDevice, c->stream));
    if (z) GCCD_HIP(c, hipMemcpyAsync(z, c->z, d, hipMemcpyDeviceToDevice, c->stream));
    if (collect_step)
        GCCD_HIP(c, hipMemcpyAsync(collect_step, c->cstep, (size_t)c->n * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, c->stream));
    return GCCD_OK;
}

static int image_common(gccd_ctx* c, double x0, double y0, double pitch, int32_t nx, int32_t ny,
                        uint32_t* counts, uint64_t* n_outside, bool per_event) {
    if (!c) return GCCD_E_INVALID;
    if (!is_finite(x0) || !is_finite(y0) || !is_finite(pitch) || !(pitch > 0) || nx <= 0 ||
        ny <= 0 || (int64_t)nx * (int64_t)ny > 2147483648LL || !counts || !n_outside)
        return fail(c, GCCD_E_INVALID, "gccd_image: bad grid or NULL pointer");
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_image before gccd_load");
    const uint64_t grids = per_event ? c->n_events : 1;
    GCCD_HIP(c, launch_fill_u32(counts, grids * (uint64_t)nx * (uint64_t)ny, 0u, c->stream));
    GCCD_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(n_outside), 2 * grids, 0u, c->stream));
    GCCD_HIP(c, launch_image(c->x, c->y, c->cstep, c->ev_of, (uint32_t)c->n, per_event ? 1 : 0,
                             x0, y0, pitch, nx, ny, counts,
                             reinterpret_cast<unsigned long long*>(n_outside), c->stream));
    return GCCD_OK;
}

int gccd_image(gccd_ctx* c, double x0, double y0, double pitch, int32_t nx, int32_t ny,
               uint32_t* counts, uint64_t* n_outside) {
    return image_common(c, x0, y0, pitch, nx, ny, counts, n_outside, false);
}

int gccd_image_events(gccd_ctx* c, double x0, double y0, double pitch, int32_t nx, int32_t ny,
                      uint32_t* counts, uint64_t* n_outside) {
    return image_common(c, x0, y0, pitch, nx, ny, counts, n_outside, true);
}

int gccd_stats(gccd_ctx* c, gccd_stats_t* out) {
    if (!c || !out) return GCCD_E_INVALID;
    memset(out, 0, sizeof *out);
    out->targets_per_thread = c->tpt;
    out->source_chunks = c->loaded ? c->chunks_h[0] : 0;
    out->tile_sources = c->loaded ? c->unit : 0;
    out->field_ms = c->field_ms;
    out->field_launches = c->field_launches;
    out->graph_replays = c->graph_replays;
    out->schedule = c->schedule;
    out->graph_usable = c->graph_refused ? 0 : 1;
    if (!c->loaded) return GCCD_OK;
    GCCD_HIP(c, hipMemcpyAsync(c->host_meta, c->meta, kMetaWords * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    out->step = c->step;
    out->n_carriers = c->n;
    out->n_active = c->n_active;
    out->carrier_steps = meta64(c, kMetaStats);
    out->pair_interactions = meta64(c, kMetaStats + 2);
    out->n_events = c->n_events;
    out->max_source_chunks = c->max_chunks;
    out->closure_steps = c->closure_steps;
    out->near_chunks = c->near_chunks;
    return GCCD_OK;
}


// ---------------------------------------------------------------------------
// gccd_field_noalloc: gccd_init + gccd_load + gccd_field + gccd_destroy of one
// event in the default launch shape and precision, on buffers carved from a
// static device array instead of allocated ones.
// ---------------------------------------------------------------------------
namespace {

// Regions of the scratch array, in bytes, for at most GCCD_NOALLOC_MAX_CARRIERS
// holes (each 256-byte aligned).
constexpr size_t kNaN = GCCD_NOALLOC_MAX_CARRIERS;
constexpr size_t kNaTiles = (kNaN + kTile - 1) / kTile;
constexpr size_t kNaBlocks = (kNaN + kFieldThreads - 1) / kFieldThreads;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaPos = align256(kNaN * sizeof(double));        // x, y, z, px, py, pz
constexpr size_t kNaI32 = align256(kNaN * sizeof(uint32_t));      // cstep, ev_of
constexpr size_t kNaKeys = align256(kNaN * sizeof(uint64_t));     // keys[0], keys[1]
constexpr size_t kNaClose = align256(3 * kNaN * sizeof(unsigned long long));
constexpr size_t kNaPart = align256((size_t)kMaxChunks * 3 * kNaN * sizeof(float));
constexpr size_t kNaBox = align256((size_t)kBoxRows * kNaTiles * sizeof(double));
constexpr size_t kNaItems = align256(kNaBlocks * kMaxChunks * sizeof(FieldItem));
constexpr size_t kNaSmall = align256((8 + kNaTiles + kMetaWords + kSchedWords) * sizeof(uint32_t));
constexpr size_t kNaBytes =
    6 * kNaPos + 2 * kNaI32 + 2 * kNaKeys + kNaClose + kNaPart + kNaBox + kNaItems + kNaSmall;

__device__ __align__(256) unsigned char scratch[kNaBytes];

// Per device: the address of that device's copy of `scratch` (host code may
// not use the array's name as a device address) and the launch facts the
// chunk choice depends on.
constexpr int kNaDevices = 64;
struct NoAllocDevice {
    unsigned char* ptr = nullptr;
    int n_cu = 0;
    int slots = 0;  // workgroups of the default Eq. (6) kernel per compute unit
};
std::mutex g_na_mutex;
NoAllocDevice g_na[kNaDevices];

int noalloc_device(int dev, NoAllocDevice* out) {
    if (dev < 0 || dev >= kNaDevices) return GCCD_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    NoAllocDevice& d = g_na[dev];
    if (!d.ptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return GCCD_E_DEVICE;
        }
        int n_cu = 0;
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            n_cu <= 0)
            n_cu = 256;
        d.n_cu = n_cu;
        d.slots = field_slots_per_cu(1, GCCD_PRECISION_DEFAULT);
        d.ptr = static_cast<unsigned char*>(p);
    }
    *out = d;
    return GCCD_OK;
}

}  // namespace

int gccd_field_noalloc(const gccd_params* p, int64_t n, const double* x, const double* y,
                       const double* z, double* ex, double* ey, double* ez, void* hip_stream) {
    if (validate(p) != GCCD_OK || n < 1 || n > GCCD_NOALLOC_MAX_CARRIERS || !x || !y || !z ||
        !ex || !ey || !ez)
        return GCCD_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GCCD_E_DEVICE;
    NoAllocDevice d;
    if (int r = noalloc_device(dev, &d); r != GCCD_OK) return r;
    hipStream_t st = (hipStream_t)hip_stream;
    const uint32_t nn = (uint32_t)n;

    // the tile size and chunk plan of choose_unit and choose_chunks for one
    // event, one target per thread; `tiles` counts the 256-source tiles whose
    // boxes gather_tiles writes, `utiles` the tiles of the chosen size
    const uint64_t tiles = ((uint64_t)nn + kTile - 1) / kTile;
    const uint64_t blocks = ((uint64_t)nn + kFieldThreads - 1) / kFieldThreads;
    const uint64_t unit =
        auto_unit(blocks * (((uint64_t)nn + kTile / 4 - 1) / (kTile / 4)), d.n_cu, d.slots);
    const uint64_t utiles = ((uint64_t)nn + unit - 1) / unit;
    const uint64_t cap = kMaxChunks;
    int32_t g = (int32_t)std::min<uint64_t>(auto_chunks(nn, unit, blocks, d.n_cu, cap), cap);
    int32_t tail = 0;
    uint32_t split = 0;
    {
        const uint64_t slots = (uint64_t)d.n_cu * (uint64_t)d.slots;
        const uint64_t big = (utiles + g - 1) / (uint64_t)g;
        if (blocks * (uint64_t)g < 32 * slots && big >= 4)
            (void)event_tail(utiles, blocks, (uint64_t)g, cap, (int64_t)(slots * big / 2), &g,
                             &tail, &split);
    }
    const uint32_t n_items = (uint32_t)(blocks * (uint64_t)g);

    // carve the regions
    unsigned char* q = d.ptr;
    auto take = [&](size_t bytes) {
        unsigned char* r = q;
        q += bytes;
        return r;
    };
    double* cx = reinterpret_cast<double*>(take(kNaPos));
    double* cy = reinterpret_cast<double*>(take(kNaPos));
    double* cz = reinterpret_cast<double*>(take(kNaPos));
    double* px = reinterpret_cast<double*>(take(kNaPos));
    double* py = reinterpret_cast<double*>(take(kNaPos));
    double* pz = reinterpret_cast<double*>(take(kNaPos));
    int32_t* cstep = reinterpret_cast<int32_t*>(take(kNaI32));
    uint32_t* ev_of = reinterpret_cast<uint32_t*>(take(kNaI32));
    uint64_t* keys0 = reinterpret_cast<uint64_t*>(take(kNaKeys));
    uint64_t* keys1 = reinterpret_cast<uint64_t*>(take(kNaKeys));
    unsigned long long* close = reinterpret_cast<unsigned long long*>(take(kNaClose));
    float* part = reinterpret_cast<float*>(take(kNaPart));
    double* box = reinterpret_cast<double*>(take(kNaBox));
    FieldItem* items = reinterpret_cast<FieldItem*>(take(kNaItems));
    uint32_t* small = reinterpret_cast<uint32_t*>(take(kNaSmall));
    uint32_t* ev_off = small;          // [2]
    uint32_t* ev_tile = small + 2;     // [2]
    uint32_t* ev_active = small + 4;   // [1]
    int32_t* ev_chunks = reinterpret_cast<int32_t*>(small + 5);  // [1]
    uint32_t* meta = small + 8;        // [kMetaWords]
    uint32_t* sched = meta + kMetaWords;
    uint32_t* tile_event = sched + kSchedWords;  // [tiles]

    const KeyLayout kl{std::max<uint32_t>(1, bits_for((uint64_t)nn)), 0u};
    const size_t dbytes = (size_t)nn * sizeof(double);
#define NA_HIP(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) {                    \
            (void)hipGetLastError();                   \
            return GCCD_E_DEVICE;                      \
        }                                              \
    } while (0)
    // meta and sched are contiguous: both zeroed
    NA_HIP(launch_noalloc_setup(nn, (uint32_t)tiles, g, tail, split, (uint32_t)blocks, ev_off,
                                ev_tile, ev_chunks, tile_event, meta, kMetaWords + kSchedWords,
                                items, close, st));
    NA_HIP(hipMemcpyAsync(cx, x, dbytes, hipMemcpyDeviceToDevice, st));
    NA_HIP(hipMemcpyAsync(cy, y, dbytes, hipMemcpyDeviceToDevice, st));
    NA_HIP(hipMemcpyAsync(cz, z, dbytes, hipMemcpyDeviceToDevice, st));
    NA_HIP(launch_load(cz, cstep, ev_off, ev_of, 1u, nn, p->thickness_um, p->well_z_um,
                       meta + kMetaCount, st));
    NA_HIP(launch_make_keys(cx, cy, cz, cstep, ev_of, ev_off, nn, kl, keys1, st));
    NA_HIP(sort_keys(keys1, keys0, nn, st));
    NA_HIP(launch_count(keys0, ev_off, 1u, kl, ev_active, st));
    NA_HIP(launch_gather(keys0, ev_off, ev_tile, tile_event, ev_active, p->collected_are_sources,
                         (uint32_t)tiles, kl, cx, cy, cz, px, py, pz, box, (uint32_t)tiles, st));
    FieldArgs fa{};
    fa.items = items;
    fa.ev_off = ev_off;
    fa.ev_active = ev_active;
    fa.ev_tile = ev_tile;
    fa.one_event_n = nn;
    fa.targets_all = 1;
    fa.sources_all = p->collected_are_sources;
    fa.px = px;
    fa.py = py;
    fa.pz = pz;
    fa.tile_box = box;
    fa.tile_stride = (uint32_t)tiles;
    const double eps2 = p->softening_um * p->softening_um;
    fa.eps2 = (float)eps2;
    fa.eps2d = eps2;
    fa.part = part;
    fa.pstride = nn;
    fa.n_items = sched + kSchedItems;
    fa.queue = sched + kSchedQueue;
    fa.near_compensated = n_items <= (uint64_t)d.n_cu * (uint64_t)d.slots ? 1 : 0;
    fa.acc2 = (float)((kExactRadius * kExactRadius + 1.0) * eps2);
    fa.acc_box2 = kExactRadius * kExactRadius * eps2;
    fa.acc_scale = std::ldexp(eps2, kExactShift);
    fa.close = close;
    fa.unit = (int32_t)unit;
    NA_HIP(launch_field(fa, 1, GCCD_PRECISION_DEFAULT, n_items, 0u, st));
    const double K = kQ / (4.0 * kPi * kEps0 * p->eps_r) * 1e12 * 1e-2;
    NA_HIP(launch_field_finish(part, nn, ev_chunks, 0, 0, keys0, ev_off, kl, nn, K, close,
                               std::ldexp(1.0 / eps2, -kExactShift), ex, ey, ez, st));
#undef NA_HIP
    return GCCD_OK;
}

}  // extern "C"
