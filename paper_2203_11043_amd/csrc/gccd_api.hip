// Host side of the C ABI declared in include/gccd.h: parameter validation,
// device buffers, the step loop of Sec. III.B (Fig. 2) and its launch shapes.
#include "gccd.h"
#include "gccd_internal.h"

#include <cmath>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

using namespace gccd;

namespace {

// CODATA 2018 (SI): elementary charge, Boltzmann constant, vacuum permittivity.
constexpr double kQ = 1.602176634e-19;
constexpr double kKB = 1.380649e-23;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

constexpr int kPoll = 32;  // steps between host reads of the active count
constexpr int64_t kMaxCarriers = 1ll << 27;  // carrier index fits the low key bits

// Small device block of counters: [0..2] active counts (ring of three, by step
// mod 3), [3] non-finite flag, [4] step after the last step with travelling
// holes, [8..11] two uint64 statistics.
constexpr int kMetaWords = 16;

}  // namespace

struct gccd_ctx {
    gccd_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 256;

    // derived constants
    double K = 0, mu0 = 0, ec = 0, beta = 0, inv_beta = 0, vt = 0;

    int64_t n = 0, cap = 0;
    double* x = nullptr;
    double* y = nullptr;
    double* z = nullptr;
    int32_t* cstep = nullptr;
    // key lists: keys[cur] holds this step's travelling holes (sorted when
    // Coulomb is on), keys[cur ^ 1] receives the next step's, keys[2] is
    // scratch for gccd_field
    uint64_t* keys[3] = {nullptr, nullptr, nullptr};
    int cur = 0;
    uint32_t idx_bits = 1;
    void* sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    // lists hold all n carriers (Coulomb on, collected holes are sources) or
    // only the travelling ones
    bool full_list = false;
    double* tile_box = nullptr;  // [6][tile_stride] source-tile bounding boxes
    uint32_t tile_stride = 0;
    // positions gathered into list-slot order: set 0 for the run's list (the
    // Eq. (6) sources, and its targets), set 1 for gccd_field's targets
    double* ps[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    float* part = nullptr;
    uint32_t* meta = nullptr;
    uint32_t* host_meta = nullptr;  // pinned

    bool loaded = false;
    int64_t step = 0;
    int64_t n_active = 0;

    int tpt_fixed = 0, chunks_fixed = 0;
    int last_tpt = 0, last_chunks = 0;

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

#define GCCD_HIP(ctx, call)                                              \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
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

void free_buffers(gccd_ctx* c) {
    (void)hipFree(c->x);
    (void)hipFree(c->y);
    (void)hipFree(c->z);
    (void)hipFree(c->cstep);
    for (int i = 0; i < 3; ++i) (void)hipFree(c->keys[i]);
    (void)hipFree(c->sort_tmp);
    (void)hipFree(c->tile_box);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            (void)hipFree(c->ps[a][b]);
            c->ps[a][b] = nullptr;
        }
    (void)hipFree(c->part);
    c->x = c->y = c->z = nullptr;
    c->cstep = nullptr;
    c->keys[0] = c->keys[1] = c->keys[2] = nullptr;
    c->sort_tmp = nullptr;
    c->sort_tmp_bytes = 0;
    c->tile_box = nullptr;
    c->tile_stride = 0;
    c->part = nullptr;
    c->cap = 0;
}

// Launch shape of Eq. (6) for up to nt targets and ns sources: enough
// workgroups to give every CU several of them (splitting the sources into
// chunks when the targets alone are too few), and at least a few LDS tiles per
// chunk.  The split fixes the FP32 summation order, so it is chosen from the
// loaded carrier count only -- never from how many are still travelling --
// and every step of a load, and gccd_field, sums in the same order.
void choose_shape(const gccd_ctx* c, uint32_t nt, uint32_t ns, int* tpt, int* chunks) {
    // One target per lane: the smallest workgroup box, hence the fewest
    // close pairs taking the exact-difference branch, and 62 VGPRs (eight
    // waves per SIMD).  Measured faster than two or four per lane.
    int t = c->tpt_fixed ? c->tpt_fixed : 1;
    int s = c->chunks_fixed;
    if (s == 0) {
        const uint64_t per_block = (uint64_t)kFieldThreads * t;
        const uint64_t tblocks = (nt + per_block - 1) / per_block;
        // about 48 waves per SIMD in total (6 rounds of 8 resident), which
        // evens out workgroups whose boxes see more close pairs
        const uint64_t want = (uint64_t)c->n_cu * 48;
        uint64_t k = tblocks ? (want + tblocks - 1) / tblocks : 1;
        const uint64_t by_tiles = ns / (4u * kTile);  // keep >= 4 tiles per chunk
        if (k > by_tiles) k = by_tiles;
        if (k < 1) k = 1;
        if (k > (uint64_t)kMaxChunks) k = kMaxChunks;
        s = (int)k;
    }
    *tpt = t;
    *chunks = s;
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
        hipHostMalloc((void**)&c->host_meta, kMetaWords * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(c->meta);
        delete c;
        return GCCD_E_NOMEM;
    }
    *out = c;
    return GCCD_OK;
}

void gccd_destroy(gccd_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_buffers(c);
    (void)hipFree(c->meta);
    (void)hipHostFree(c->host_meta);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

int gccd_load(gccd_ctx* c, int64_t n, const double* x, const double* y, const double* z) {
    if (!c) return GCCD_E_INVALID;
    if (n <= 0 || n > kMaxCarriers || !x || !y || !z)
        return fail(c, GCCD_E_INVALID, "gccd_load: n out of range or NULL pointer");
    uint32_t bits = 1;
    while ((1ll << bits) < n) ++bits;
    if (n > c->cap) {
        GCCD_HIP(c, hipStreamSynchronize(c->stream));
        free_buffers(c);
        const size_t d = (size_t)n * sizeof(double);
        const size_t i = (size_t)n * sizeof(int32_t);
        const size_t k = (size_t)n * sizeof(uint64_t);
        bool ok = hipMalloc(&c->x, d) == hipSuccess && hipMalloc(&c->y, d) == hipSuccess &&
                  hipMalloc(&c->z, d) == hipSuccess && hipMalloc(&c->cstep, i) == hipSuccess &&
                  hipMalloc(&c->keys[0], k) == hipSuccess &&
                  hipMalloc(&c->keys[1], k) == hipSuccess &&
                  hipMalloc(&c->keys[2], k) == hipSuccess &&
                  hipMalloc(&c->tile_box, 6 * sizeof(double) * (size_t)((n + kTile - 1) / kTile)) ==
                      hipSuccess &&
                  hipMalloc(&c->ps[0][0], d) == hipSuccess && hipMalloc(&c->ps[0][1], d) == hipSuccess &&
                  hipMalloc(&c->ps[0][2], d) == hipSuccess && hipMalloc(&c->ps[1][0], d) == hipSuccess &&
                  hipMalloc(&c->ps[1][1], d) == hipSuccess && hipMalloc(&c->ps[1][2], d) == hipSuccess &&
                  hipMalloc(&c->part, (size_t)kMaxChunks * 3 * (size_t)n * sizeof(float)) ==
                      hipSuccess;
        if (!ok) {
            free_buffers(c);
            c->loaded = false;
            return fail(c, GCCD_E_NOMEM, "gccd_load: device allocation failed");
        }
        c->cap = n;
        c->tile_stride = (uint32_t)((n + kTile - 1) / kTile);
    }
    size_t need = 0;
    GCCD_HIP(c, sort_keys_storage((uint32_t)n, kMortonBits + 1u + bits, &need));
    if (need > c->sort_tmp_bytes) {
        (void)hipFree(c->sort_tmp);
        c->sort_tmp = nullptr;
        c->sort_tmp_bytes = 0;
        if (hipMalloc(&c->sort_tmp, need) != hipSuccess) {
            free_buffers(c);
            c->loaded = false;
            return fail(c, GCCD_E_NOMEM, "gccd_load: sort storage allocation failed");
        }
        c->sort_tmp_bytes = need;
    }
    c->idx_bits = bits;
    const size_t bytes = (size_t)n * sizeof(double);
    GCCD_HIP(c, hipMemcpyAsync(c->x, x, bytes, hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(c->y, y, bytes, hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, hipMemcpyAsync(c->z, z, bytes, hipMemcpyDeviceToDevice, c->stream));
    GCCD_HIP(c, launch_fill_u32(c->meta, kMetaWords, 0u, c->stream));
    c->full_list = c->p.coulomb && c->p.collected_are_sources;
    if (!c->full_list) GCCD_HIP(c, launch_fill_u64(c->keys[1], (uint64_t)n, kNoKey, c->stream));
    GCCD_HIP(c, launch_load(c->z, c->cstep, c->keys[1], c->meta + 0, c->x, c->y, (uint32_t)n,
                            bits, c->full_list ? 1 : 0, c->p.thickness_um, c->p.well_z_um,
                            c->stream));
    GCCD_HIP(c, sort_keys(c->sort_tmp, c->sort_tmp_bytes, c->keys[1], c->keys[0], (uint32_t)n,
                          kMortonBits + 1u + bits, c->stream));
    c->cur = 0;
    GCCD_HIP(c, hipMemcpyAsync(c->host_meta, c->meta, kMetaWords * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    c->n = n;
    c->step = 0;
    c->n_active = c->host_meta[0];
    c->loaded = true;
    c->field_ms = 0;
    c->field_launches = 0;
    c->ev_used = 0;
    return GCCD_OK;
}

int gccd_set_launch(gccd_ctx* c, int32_t tpt, int32_t chunks) {
    if (!c) return GCCD_E_INVALID;
    if (!(tpt == 0 || tpt == 1 || tpt == 2 || tpt == 4) || chunks < 0 || chunks > kMaxChunks)
        return fail(c, GCCD_E_INVALID, "gccd_set_launch: shape out of range");
    c->tpt_fixed = tpt;
    c->chunks_fixed = chunks;
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
    uint32_t bound = (uint32_t)c->n_active;

    StepArgs sa{};
    sa.x = c->x;
    sa.y = c->y;
    sa.z = c->z;
    sa.cstep = c->cstep;
    sa.part = c->part;
    sa.pstride = n;
    sa.coulomb = c->p.coulomb;
    sa.diffusion = c->p.diffusion;
    sa.mobility_model = c->p.mobility_model;
    sa.src_all = c->p.collected_are_sources;
    sa.n_all = n;
    sa.idx_bits = c->idx_bits;
    sa.K = c->K;
    sa.a1 = c->p.a1_Vcm_per_um;
    sa.a2 = c->p.a2_Vcm;
    sa.thickness = c->p.thickness_um;
    sa.z_well = c->p.well_z_um;
    sa.mu0 = c->mu0;
    sa.ec = c->ec;
    sa.beta = c->beta;
    sa.inv_beta = c->inv_beta;
    sa.dt_s = dt_ps * 1e-12;
    sa.vt = c->vt;
    sa.event = c->p.event;
    sa.key0 = (uint32_t)c->p.seed;
    sa.key1 = (uint32_t)(c->p.seed >> 32);
    sa.stats = reinterpret_cast<unsigned long long*>(c->meta + 8);
    sa.misc = reinterpret_cast<int32_t*>(c->meta + 3);

    const uint64_t idx_mask = (1ull << c->idx_bits) - 1ull;
    FieldArgs fa{};
    fa.tx = fa.sx = c->ps[0][0];
    fa.ty = fa.sy = c->ps[0][1];
    fa.tz = fa.sz = c->ps[0][2];
    fa.tile_box = c->tile_box;
    fa.tile_stride = c->tile_stride;
    fa.eps2 = (float)(c->p.softening_um * c->p.softening_um);
    fa.part = c->part;
    fa.pstride = n;
    int tpt, chunks;
    choose_shape(c, n, n, &tpt, &chunks);
    const uint32_t end_bit = kMortonBits + 1u + c->idx_bits;
    sa.full_list = c->full_list ? 1 : 0;

    int64_t k = 0;
    while (k < max_steps && bound > 0) {
        const int64_t chunk_steps = (max_steps - k < kPoll) ? (max_steps - k) : kPoll;
        for (int64_t i = 0; i < chunk_steps; ++i) {
            const uint32_t s = (uint32_t)(step0 + k + i);
            uint64_t* kin = c->keys[c->cur];
            uint64_t* kout = c->keys[c->cur ^ 1];
            uint32_t* cin = c->meta + (s % 3u);
            if (c->p.coulomb) {
                // targets: the travelling holes, first in the list; sources:
                // the whole list (full) or the same travelling holes; both
                // read from the slot-ordered copy gathered here
                fa.tcount = cin;
                fa.nt = bound;
                fa.scount = c->full_list ? nullptr : cin;
                fa.ns = c->full_list ? n : bound;
                fa.nchunk = chunks;
                c->last_tpt = tpt;
                c->last_chunks = chunks;
                GCCD_HIP(c, launch_gather(kin, fa.scount, fa.ns, fa.ns, idx_mask, n, c->x, c->y,
                                          c->z, c->ps[0][0], c->ps[0][1], c->ps[0][2],
                                          c->tile_box, c->tile_stride, c->stream));
                hipEvent_t* evp = nullptr;
                int r = record_field_start(c, &evp);
                if (r != GCCD_OK) return r;
                GCCD_HIP(c, launch_field(fa, tpt, bound, c->stream));
                if (evp) GCCD_HIP(c, hipEventRecord(evp[1], c->stream));
                sa.nchunk = chunks;
            } else {
                sa.nchunk = 0;
            }
            if (!c->full_list) GCCD_HIP(c, launch_fill_u64(kout, bound, kNoKey, c->stream));
            sa.keys_in = kin;
            sa.cnt_in = cin;
            sa.keys_out = kout;
            sa.cnt_out = c->meta + ((s + 1u) % 3u);
            sa.cnt_clear = c->meta + ((s + 2u) % 3u);
            sa.step = s;
            GCCD_HIP(c, launch_step(sa, bound, c->stream));
            if (c->p.coulomb) {
                // next step's list in spatial order, travelling holes first
                // (the unused tail of a travelling-only list holds kNoKey)
                GCCD_HIP(c, sort_keys(c->sort_tmp, c->sort_tmp_bytes, kout, kin,
                                      c->full_list ? n : bound, end_bit, c->stream));
            } else {
                c->cur ^= 1;
            }
        }
        k += chunk_steps;
        GCCD_HIP(c, hipMemcpyAsync(c->host_meta, c->meta, kMetaWords * sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, c->stream));
        GCCD_HIP(c, hipStreamSynchronize(c->stream));
        if (c->timing) {
            int r = collect_timing(c);
            if (r != GCCD_OK) return r;
        }
        const uint32_t s_next = (uint32_t)(step0 + k);
        bound = c->host_meta[s_next % 3u];
        if (c->host_meta[3] != 0) {
            // The active-list ring may now be ahead of the step counter: the
            // state is unusable until the next gccd_load.
            c->step = (int64_t)(uint32_t)c->host_meta[4];
            c->n_active = bound;
            c->loaded = false;
            return fail(c, GCCD_E_NONFINITE,
                        "gccd_run: a carrier position became non-finite; reload to continue");
        }
    }
    // The step after the last one that moved a hole: later steps found no hole
    // travelling and left the state (and the counter ring, all zero) unchanged.
    const int64_t last = (k > 0) ? (int64_t)(uint32_t)c->host_meta[4] : step0;
    c->step = (last > step0) ? last : step0;
    c->n_active = bound;
    if (steps_done) *steps_done = c->step - step0;
    if (n_active) *n_active = c->n_active;
    return GCCD_OK;
}

int gccd_field(gccd_ctx* c, double* ex, double* ey, double* ez) {
    if (!c) return GCCD_E_INVALID;
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_field before gccd_load");
    if (!ex || !ey || !ez) return fail(c, GCCD_E_INVALID, "gccd_field: NULL pointer");
    const uint32_t n = (uint32_t)c->n;
    const uint32_t s = (uint32_t)c->step;
    const uint32_t end_bit = kMortonBits + 1u + c->idx_bits;
    const uint64_t idx_mask = (1ull << c->idx_bits) - 1ull;
    FieldArgs fa{};
    fa.tile_box = c->tile_box;
    fa.tile_stride = c->tile_stride;
    fa.eps2 = (float)(c->p.softening_um * c->p.softening_um);
    fa.part = c->part;
    fa.pstride = n;
    fa.nt = n;
    fa.tcount = nullptr;
    fa.sx = c->ps[0][0];
    fa.sy = c->ps[0][1];
    fa.sz = c->ps[0][2];
    const uint64_t* tkeys = nullptr;
    if (c->full_list || c->p.collected_are_sources) {
        // every carrier is both a target and a source: the run's list when it
        // holds all of them, else all keys sorted into the unused list
        const uint64_t* all = c->keys[c->cur];
        if (!c->full_list) {
            uint64_t* tk = c->keys[c->cur ^ 1];
            GCCD_HIP(c, launch_keys_all(c->x, c->y, c->z, n, c->idx_bits, c->keys[2], c->stream));
            GCCD_HIP(c, sort_keys(c->sort_tmp, c->sort_tmp_bytes, c->keys[2], tk, n, end_bit,
                                  c->stream));
            all = tk;
        }
        GCCD_HIP(c, launch_gather(all, nullptr, n, n, idx_mask, n, c->x, c->y, c->z, c->ps[0][0],
                                  c->ps[0][1], c->ps[0][2], c->tile_box, c->tile_stride,
                                  c->stream));
        fa.tx = c->ps[0][0];
        fa.ty = c->ps[0][1];
        fa.tz = c->ps[0][2];
        fa.scount = nullptr;
        fa.ns = n;
        tkeys = all;
    } else {
        // sources: the travelling holes (the run's list); targets: every
        // carrier, sorted into the unused list
        uint32_t* cnt = c->meta + (s % 3u);
        const uint32_t na = (uint32_t)c->n_active;
        GCCD_HIP(c, launch_gather(c->keys[c->cur], cnt, na, na, idx_mask, n, c->x, c->y, c->z,
                                  c->ps[0][0], c->ps[0][1], c->ps[0][2], c->tile_box,
                                  c->tile_stride, c->stream));
        uint64_t* tk = c->keys[c->cur ^ 1];
        GCCD_HIP(c, launch_keys_all(c->x, c->y, c->z, n, c->idx_bits, c->keys[2], c->stream));
        GCCD_HIP(c, sort_keys(c->sort_tmp, c->sort_tmp_bytes, c->keys[2], tk, n, end_bit,
                              c->stream));
        GCCD_HIP(c, launch_gather(tk, nullptr, n, n, idx_mask, n, c->x, c->y, c->z, c->ps[1][0],
                                  c->ps[1][1], c->ps[1][2], nullptr, 0, c->stream));
        fa.tx = c->ps[1][0];
        fa.ty = c->ps[1][1];
        fa.tz = c->ps[1][2];
        fa.scount = cnt;
        fa.ns = na;
        tkeys = tk;
    }
    int tpt, chunks;
    choose_shape(c, n, n, &tpt, &chunks);
    fa.nchunk = chunks;
    c->last_tpt = tpt;
    c->last_chunks = chunks;
    GCCD_HIP(c, launch_field(fa, tpt, n, c->stream));
    GCCD_HIP(c, launch_field_finish(c->part, n, chunks, tkeys, idx_mask, n, c->K, ex, ey, ez,
                                    c->stream));
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

int gccd_image(gccd_ctx* c, double x0, double y0, double pitch, int32_t nx, int32_t ny,
               uint32_t* counts, uint64_t* n_outside) {
    if (!c) return GCCD_E_INVALID;
    if (!is_finite(x0) || !is_finite(y0) || !is_finite(pitch) || !(pitch > 0) || nx <= 0 || ny <= 0 ||
        (int64_t)nx * (int64_t)ny > 2147483648LL || !counts || !n_outside)
        return fail(c, GCCD_E_INVALID, "gccd_image: bad grid or NULL pointer");
    if (!c->loaded) return fail(c, GCCD_E_STATE, "gccd_image before gccd_load");
    GCCD_HIP(c, launch_fill_u32(counts, (uint64_t)nx * (uint64_t)ny, 0u, c->stream));
    GCCD_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(n_outside), 2, 0u, c->stream));
    GCCD_HIP(c, launch_image(c->x, c->y, c->cstep, (uint32_t)c->n, x0, y0, pitch, nx, ny, counts,
                             reinterpret_cast<unsigned long long*>(n_outside), c->stream));
    return GCCD_OK;
}

int gccd_stats(gccd_ctx* c, gccd_stats_t* out) {
    if (!c || !out) return GCCD_E_INVALID;
    memset(out, 0, sizeof *out);
    out->targets_per_thread = c->last_tpt;
    out->source_chunks = c->last_chunks;
    out->field_ms = c->field_ms;
    out->field_launches = c->field_launches;
    if (!c->loaded) return GCCD_OK;
    GCCD_HIP(c, hipMemcpyAsync(c->host_meta, c->meta, kMetaWords * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, c->stream));
    GCCD_HIP(c, hipStreamSynchronize(c->stream));
    uint64_t st[2];
    memcpy(st, c->host_meta + 8, sizeof st);
    out->step = c->step;
    out->n_carriers = c->n;
    out->n_active = c->n_active;
    out->carrier_steps = st[0];
    out->pair_interactions = st[1];
    return GCCD_OK;
}

}  // extern "C"
