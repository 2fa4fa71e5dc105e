// HIP kernels (gfx950 / CDNA4) of the charge-transport hot path of
// Avalos & Sofo Haro, arXiv 2203.11043:
//   field_tiles   -- Eq. (6), softened all-pairs Coulomb field (the O(N^2) part)
//   step_update   -- Eqs. (1)-(4) and the z check of Sec. III.B, fused per carrier
//   load_prepare  -- load-time boundary handling
//   make_keys, count_active, gather_tiles -- the spatially sorted carrier list
//   image_bin     -- 2D histogram of collected holes (Sec. V.A)
// Several independent events (clouds) can share one launch; every kernel
// keeps them apart through the per-event slot offsets.
#include "gccd.h"
#include "gccd_fp64.h"
#include "gccd_internal.h"
#include "gccd_sort_dev.h"

#include <math.h>

namespace gccd {

// ---------------------------------------------------------------------------
// Keys.  A hole's 0.25 um cell (12 bits per axis, wrapping every 1024 um) is
// mapped to its 36-bit index along a 3D Hilbert curve, which visits
// face-adjacent cells one after the other: a run of consecutive keys is a
// compact region with no jumps, so source tiles and target blocks have small
// bounding boxes.  The index follows Skilling's transposition (J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707, 381 (2004)): undo
// the excess work axis by axis from the top bit down, Gray-encode, and
// interleave the bits of the transposed coordinates (x first in each triple).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell12(double v) {
    if (!isfinite(v)) return 0u;
    return (uint32_t)(int64_t)floor(v * kCellPerUm) & 0xFFFu;
}

__device__ __forceinline__ uint64_t hilbert36(uint32_t cx, uint32_t cy, uint32_t cz) {
    uint32_t X[3] = {cx, cy, cz};
#pragma unroll
    for (uint32_t Q = 1u << 11; Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const bool set = (X[i] & Q) != 0u;
            const uint32_t t = set ? 0u : ((X[0] ^ X[i]) & P);  // exchange low bits
            X[0] ^= (set ? P : 0u) ^ t;                          // or invert them
            X[i] ^= t;
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0u;
#pragma unroll
    for (uint32_t Q = 1u << 11; Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
    uint64_t key = 0;
#pragma unroll
    for (int j = 11; j >= 0; --j) {
#pragma unroll
        for (int i = 0; i < 3; ++i) key = (key << 1) | (uint64_t)((X[i] >> j) & 1u);
    }
    return key;
}

__device__ __forceinline__ uint64_t make_key(uint32_t event, bool collected, double x, double y,
                                             double z, uint32_t local, KeyLayout kl) {
    uint64_t k = (uint64_t)local;
    k |= hilbert36(cell12(x), cell12(y), cell12(z)) << kl.lbits;
    if (collected) k |= 1ull << (kl.lbits + kCurveBits);
    k |= (uint64_t)event << (kl.lbits + kCurveBits + 1);
    return k;
}

__device__ __forceinline__ uint32_t key_local(uint64_t k, KeyLayout kl) {
    return (uint32_t)(k & ((1ull << kl.lbits) - 1ull));
}

__device__ __forceinline__ uint32_t key_event(uint64_t k, KeyLayout kl) {
    return (uint32_t)(k >> (kl.lbits + kCurveBits + 1));
}

__device__ __forceinline__ bool key_collected(uint64_t k, KeyLayout kl) {
    return ((k >> (kl.lbits + kCurveBits)) & 1ull) != 0ull;
}

// event of carrier i: the last e with ev_off[e] <= i (binary search)
__device__ __forceinline__ uint32_t event_of(const uint32_t* ev_off, uint32_t n_events,
                                             uint32_t i) {
    uint32_t lo = 0, hi = n_events;  // invariant: ev_off[lo] <= i < ev_off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ev_off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// A value every lane of the wave holds identically, moved to scalar
// registers (the compiler cannot prove uniformity after a shuffle reduction).
__device__ __forceinline__ double uniform(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m));
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    return v;
}

// Pairs closer than kExactRadius softening lengths are summed exactly.  The
// pair loop only records them (exact_push: the target's index in the item's
// block and the source's slot in its event, in an LDS list of the work item)
// and drops their FP32 terms; at the end of the item exact_flush forms each
// recorded term in FP64 from the FP64 positions, as Eq. (6) defines it, and
// adds it in fixed point to the target's slot of the close sums.  Integer
// addition is associative, so the sums do not depend on the order in which
// work items finish.  Keeping the FP64 work out of the pair loop keeps its
// registers (and the kernel's occupancy) as they are.  A pair that finds the
// list full keeps its FP32 term.
constexpr int kExactCap = 512;

struct ExactList {
    uint32_t n;
    uint32_t tgt[kExactCap];
    uint32_t src[kExactCap];
};

__device__ __forceinline__ bool exact_push(ExactList& L, uint32_t tgt, uint32_t src) {
    const uint32_t i = atomicAdd(&L.n, 1u);
    if (i >= (uint32_t)kExactCap) return false;
    L.tgt[i] = tgt;
    L.src[i] = src;
    return true;
}

// Called by every lane of the workgroup after the item's last barrier;
// targets of the item are slots off + tbase + tgt, sources slots off + src.
// Leaves the list empty for the next item (whose first barrier orders the
// clearing before any push).
__device__ __forceinline__ void exact_flush(const FieldArgs& a, ExactList& L, uint32_t off,
                                            uint32_t tbase) {
    const uint32_t cnt = min(L.n, (uint32_t)kExactCap);
    if (cnt == 0) return;  // uniform: every lane reads L.n after the same barrier
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const uint32_t t = off + tbase + L.tgt[i], s = off + L.src[i];
        const double dx = a.px[t] - a.px[s], dy = a.py[t] - a.py[s], dz = a.pz[t] - a.pz[s];
        double q = fma(dx, dx, a.eps2d);
        q = fma(dy, dy, q);
        q = fma(dz, dz, q);
        const double w = a.acc_scale / (q * sqrt(q));
        unsigned long long* c = a.close + t;
        atomicAdd(c, (unsigned long long)__double2ll_rn(dx * w));
        atomicAdd(c + a.pstride, (unsigned long long)__double2ll_rn(dy * w));
        atomicAdd(c + 2 * (size_t)a.pstride, (unsigned long long)__double2ll_rn(dz * w));
    }
    __syncthreads();
    if (threadIdx.x == 0) L.n = 0;
}

// ---------------------------------------------------------------------------
// Eq. (6):  E_j = K sum_i r_ij / (|r_ij|^2 + eps^2)^{3/2},  r_ij = r_j - r_i,
// summed over the sources of the target's own event.
//
// One workgroup takes one work item: kFieldThreads*TPT consecutive target
// slots of one event's spatially sorted segment (a compact region of the
// cloud) and one chunk of that event's source tiles, dealt round-robin
// (first, first + S, ... below the item's end).  Sources are staged
// through LDS in tiles of kTile (double buffered: the next tile's global
// loads are in flight while the current one is consumed); every lane of
// every wave reads the same LDS words, so the reads are bank-conflict-free
// broadcasts.  Each lane keeps TPT targets in registers.
//
// Precision.  The workgroup takes the centre o of its targets' bounding box
// (half-diagonal rho) as origin and holds every coordinate, targets and
// staged sources alike, as the FP32 pair hi = fl32(x - o), lo = fl32(x - o -
// hi).  A pair difference d is first formed from the hi parts alone; its
// error is at most 2u (rho + |d|), and since the Jacobian of d/|d|^3 has norm
// 2/|d|^3 the term's relative error is at most 4u (1 + |t - o|/|d|) <= 4u (1 +
// rho/|d|).  Pairs closer than a quarter of the target's distance |t - o|
// from the origin -- rare, found with one compare per pair, or ruled out for
// a whole source tile whose bounding box is rho/4 or more from the targets'
// box -- are recomputed with the lo parts added, which makes their
// difference accurate to about u |d|.
// Every term therefore carries at most 20u (1.2e-6) relative error from the
// coordinates, plus about 8u from r^2, the hardware reciprocal square root
// (cubed for r^-3) and the products, so each carrier's field is within about
// 2e-6 of the sum of its term magnitudes plus the FP32 summation error.
// Each tile's contributions are summed separately and then added to the
// running sum (blocked summation).
//
// Pairs closer than kExactRadius eps (64 nm at eps = 1 nm) are the one case
// where that relative bound is not enough: their terms reach 0.385 / eps^2,
// tens to hundreds of times the rms field of a cloud, and an FP32 term and the
// FP32 additions that follow it would carry about 10u of that into the
// target's field.  They are summed exactly instead (exact_push): the close-pair
// radius is at least that distance, so these pairs always take the checked
// path, and tiles that can hold them are never summed in the unchecked or the
// expanded form.
//
// The other GCCD_PRECISION_* modes change the origin (one per event, or
// none: absolute coordinates) or the difference formation (hi parts only,
// or hi and lo for every pair); they exist to measure those choices.
// ---------------------------------------------------------------------------
// How the difference of a pair is formed from the FP32 parts hi, lo of the
// origin-relative coordinates.
enum : int {
    kDiffHi = 0,    // hi parts only
    kDiffNear = 1,  // hi parts; pairs closer than rc recomputed with the lo parts added
    kDiffAll = 2    // hi and lo parts for every pair (double-single differences)
};

// CUT: the term counts only when r^2 + eps^2 < cut2 (the near part of a
// near/far split); 2 more VALU per pair.  EXACT (with kDiffNear): pairs with
// r^2 + eps^2 below ap->acc2 are recorded in *xl (target t of the lane is
// tgt0 + t * kFieldThreads of the item's block, the source src of the event).
template <int TPT, int DIFF, bool CUT = false, bool EXACT = false>
__device__ __forceinline__ void pair_terms(const float* __restrict__ lxp,
                                           const float* __restrict__ lyp,
                                           const float* __restrict__ lzp, uint32_t k, float shx,
                                           float shy, float shz, float slx, float sly, float slz,
                                           const float (&thx)[TPT], const float (&thy)[TPT],
                                           const float (&thz)[TPT], const float (&tlx)[TPT],
                                           const float (&tly)[TPT], const float (&tlz)[TPT],
                                           float eps2, const float (&rc2)[TPT], float (&ax)[TPT],
                                           float (&ay)[TPT], float (&az)[TPT],
                                           float cut2 = 0.0f, const FieldArgs* ap = nullptr,
                                           ExactList* xl = nullptr, uint32_t tgt0 = 0u,
                                           uint32_t src = 0u) {
    float dx[TPT], dy[TPT], dz[TPT], r2[TPT];
    bool near = false;
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        dx[t] = thx[t] - shx;
        dy[t] = thy[t] - shy;
        dz[t] = thz[t] - shz;
        if (DIFF == kDiffAll) {
            dx[t] += tlx[t] - slx;
            dy[t] += tly[t] - sly;
            dz[t] += tlz[t] - slz;
        }
        r2[t] = __builtin_fmaf(dx[t], dx[t], eps2);
        r2[t] = __builtin_fmaf(dy[t], dy[t], r2[t]);
        r2[t] = __builtin_fmaf(dz[t], dz[t], r2[t]);
        if (DIFF == kDiffNear) near |= r2[t] < rc2[t];
    }
    if (DIFF == kDiffNear && __builtin_expect(__ballot(near) != 0ull, 0)) {
        // wave-uniform branch, taken only when some lane of the wave has a
        // close pair: add the lo parts to the differences of those pairs
        const float nlx = lxp[k], nly = lyp[k], nlz = lzp[k];
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            if (r2[t] < rc2[t]) {
                dx[t] += tlx[t] - nlx;
                dy[t] += tly[t] - nly;
                dz[t] += tlz[t] - nlz;
                r2[t] = __builtin_fmaf(dx[t], dx[t], eps2);
                r2[t] = __builtin_fmaf(dy[t], dy[t], r2[t]);
                r2[t] = __builtin_fmaf(dz[t], dz[t], r2[t]);
            }
        }
        if (EXACT) {
            // rc2 is at least acc2 for a target and 0 for a padding slot; a pair
            // at distance 0 has a zero term and stays in the FP32 sum
#pragma unroll
            for (int t = 0; t < TPT; ++t) {
                if (r2[t] < fminf(ap->acc2, rc2[t]) && r2[t] > eps2 &&
                    exact_push(*xl, tgt0 + (uint32_t)(t * kFieldThreads), src))
                    dx[t] = dy[t] = dz[t] = 0.0f;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        // r^-3 as rsq^3: one transcendental and two multiplies measured
        // faster on gfx950 than rsq * rcp (two transcendentals, one multiply)
        const float inv = __builtin_amdgcn_rsqf(r2[t]);
        float w = inv * inv * inv;
        if (CUT) w = r2[t] < cut2 ? w : 0.0f;
        ax[t] = __builtin_fmaf(dx[t], w, ax[t]);
        ay[t] = __builtin_fmaf(dy[t], w, ay[t]);
        az[t] = __builtin_fmaf(dz[t], w, az[t]);
    }
}

// All pairs of one staged tile (cnt sources) with the lane's TPT targets.
template <int TPT, int DIFF, bool CUT = false, bool EXACT = false>
__device__ __forceinline__ void tile_terms(const float* __restrict__ hxp,
                                           const float* __restrict__ hyp,
                                           const float* __restrict__ hzp,
                                           const float* __restrict__ lxp,
                                           const float* __restrict__ lyp,
                                           const float* __restrict__ lzp, uint32_t cnt,
                                           const float (&thx)[TPT], const float (&thy)[TPT],
                                           const float (&thz)[TPT], const float (&tlx)[TPT],
                                           const float (&tly)[TPT], const float (&tlz)[TPT],
                                           float eps2, const float (&rc2)[TPT], float (&bx)[TPT],
                                           float (&by)[TPT], float (&bz)[TPT],
                                           float cut2 = 0.0f, const FieldArgs* ap = nullptr,
                                           ExactList* xl = nullptr, uint32_t tgt0 = 0u,
                                           uint32_t src0 = 0u) {
    uint32_t k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const float4 hx4 = *reinterpret_cast<const float4*>(hxp + k);
        const float4 hy4 = *reinterpret_cast<const float4*>(hyp + k);
        const float4 hz4 = *reinterpret_cast<const float4*>(hzp + k);
        float4 lx4 = make_float4(0.f, 0.f, 0.f, 0.f), ly4 = lx4, lz4 = lx4;
        if (DIFF == kDiffAll) {
            lx4 = *reinterpret_cast<const float4*>(lxp + k);
            ly4 = *reinterpret_cast<const float4*>(lyp + k);
            lz4 = *reinterpret_cast<const float4*>(lzp + k);
        }
        pair_terms<TPT, DIFF, CUT, EXACT>(lxp, lyp, lzp, k + 0, hx4.x, hy4.x, hz4.x, lx4.x, ly4.x, lz4.x, thx,
                              thy, thz, tlx, tly, tlz, eps2, rc2, bx, by, bz,
                                   cut2, ap, xl, tgt0, src0 + k + 0);
        pair_terms<TPT, DIFF, CUT, EXACT>(lxp, lyp, lzp, k + 1, hx4.y, hy4.y, hz4.y, lx4.y, ly4.y, lz4.y, thx,
                              thy, thz, tlx, tly, tlz, eps2, rc2, bx, by, bz,
                                   cut2, ap, xl, tgt0, src0 + k + 1);
        pair_terms<TPT, DIFF, CUT, EXACT>(lxp, lyp, lzp, k + 2, hx4.z, hy4.z, hz4.z, lx4.z, ly4.z, lz4.z, thx,
                              thy, thz, tlx, tly, tlz, eps2, rc2, bx, by, bz,
                                   cut2, ap, xl, tgt0, src0 + k + 2);
        pair_terms<TPT, DIFF, CUT, EXACT>(lxp, lyp, lzp, k + 3, hx4.w, hy4.w, hz4.w, lx4.w, ly4.w, lz4.w, thx,
                              thy, thz, tlx, tly, tlz, eps2, rc2, bx, by, bz,
                                   cut2, ap, xl, tgt0, src0 + k + 3);
    }
    for (; k < cnt; ++k) {
        pair_terms<TPT, DIFF, CUT, EXACT>(lxp, lyp, lzp, k, hxp[k], hyp[k], hzp[k], lxp[k], lyp[k], lzp[k],
                                   thx, thy, thz, tlx, tly, tlz, eps2, rc2, bx, by, bz, cut2, ap, xl, tgt0, src0 + k);
    }
}

template <int TPT, int PREC>
__global__ __launch_bounds__(kFieldThreads) void field_tiles(FieldArgs a) {
    __shared__ __align__(16) float sh[2][6][kTile];
    __shared__ double box[6][kFieldThreads / 64];
    __shared__ double ebox[6][kFieldThreads / 64];  // EVENT mode: the event's source box
    __shared__ double tbox[2][6];  // bounding box of the staged source tile
    __shared__ ExactList xl;       // default precision: close pairs of the item

    const FieldItem it = a.items[blockIdx.x];
    const uint32_t off = a.ev_off[it.event];
    const uint32_t ne = a.ev_off[it.event + 1] - off;
    const uint32_t na = a.ev_active[it.event];
    const uint32_t nt = a.targets_all ? ne : na;
    const uint32_t ns = a.sources_all ? ne : na;
    const uint32_t tbase = it.blk * (uint32_t)(kFieldThreads * TPT);
    if (tbase >= nt) return;  // the whole workgroup leaves before any barrier

    // The item takes the event's source tiles first, first + S, first + 2S,
    // ... below its end.  Each tile is a compact region (the segment is
    // spatially sorted) whose bounding box is precomputed; dealing them
    // round-robin gives every chunk a sample of the whole cloud, so the
    // close pairs -- the costlier ones -- spread evenly over the workgroups.
    const uint32_t ntiles = (ns + kTile - 1) / kTile;
    const uint32_t tile0 = a.ev_tile[it.event];
    const uint32_t chunk = it.group;  // partial-sum group written
    const uint32_t step_t = it.step;
    const uint32_t t_first = it.first;
    const uint32_t t_end = min(it.end, ntiles);
    const int tid = threadIdx.x;
    if (tid == 0) xl.n = 0;  // ordered before any push by the barrier below

    // targets and their bounding box
    double px[TPT], py[TPT], pz[TPT];
    double lo_x = INFINITY, lo_y = INFINITY, lo_z = INFINITY;
    double hi_x = -INFINITY, hi_y = -INFINITY, hi_z = -INFINITY;
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const uint32_t ts = tbase + (uint32_t)(t * kFieldThreads + tid);
        px[t] = py[t] = pz[t] = 0.0;
        if (ts < nt) {
            px[t] = a.px[off + ts];
            py[t] = a.py[off + ts];
            pz[t] = a.pz[off + ts];
            lo_x = fmin(lo_x, px[t]);
            lo_y = fmin(lo_y, py[t]);
            lo_z = fmin(lo_z, pz[t]);
            hi_x = fmax(hi_x, px[t]);
            hi_y = fmax(hi_y, py[t]);
            hi_z = fmax(hi_z, pz[t]);
        }
    }
    {
        const int wave = tid >> 6, lane = tid & 63;
        lo_x = wave_min(lo_x);
        lo_y = wave_min(lo_y);
        lo_z = wave_min(lo_z);
        hi_x = wave_max(hi_x);
        hi_y = wave_max(hi_y);
        hi_z = wave_max(hi_z);
        if (lane == 0) {
            box[0][wave] = lo_x;
            box[1][wave] = lo_y;
            box[2][wave] = lo_z;
            box[3][wave] = hi_x;
            box[4][wave] = hi_y;
            box[5][wave] = hi_z;
        }
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kFieldThreads / 64; ++w) {
        lo_x = fmin(lo_x, box[0][w]);
        lo_y = fmin(lo_y, box[1][w]);
        lo_z = fmin(lo_z, box[2][w]);
        hi_x = fmax(hi_x, box[3][w]);
        hi_y = fmax(hi_y, box[4][w]);
        hi_z = fmax(hi_z, box[5][w]);
    }
    lo_x = uniform(lo_x);
    lo_y = uniform(lo_y);
    lo_z = uniform(lo_z);
    hi_x = uniform(hi_x);
    hi_y = uniform(hi_y);
    hi_z = uniform(hi_z);
    // Every lane now holds the same box.  A box of non-finite positions
    // gives a NaN origin; the field is then NaN, and the step kernel flags it.
    double ox = 0.5 * (lo_x + hi_x), oy = 0.5 * (lo_y + hi_y), oz = 0.5 * (lo_z + hi_z);
    if (PREC == GCCD_PRECISION_ABSOLUTE) {
        ox = oy = oz = 0.0;
    } else if (PREC == GCCD_PRECISION_EVENT) {
        // centre of the union of the event's source-tile boxes
        double e[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (uint32_t t = (uint32_t)tid; t < ntiles; t += kFieldThreads) {
            const size_t g = (size_t)tile0 + t;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                e[d] = fmin(e[d], a.tile_box[(size_t)d * a.tile_stride + g]);
                e[d + 3] = fmax(e[d + 3], a.tile_box[(size_t)(d + 3) * a.tile_stride + g]);
            }
        }
        const int wave = tid >> 6;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            e[d] = wave_min(e[d]);
            e[d + 3] = wave_max(e[d + 3]);
        }
        if ((tid & 63) == 0) {
#pragma unroll
            for (int d = 0; d < 6; ++d) ebox[d][wave] = e[d];
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kFieldThreads / 64; ++w) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                e[d] = fmin(e[d], ebox[d][w]);
                e[d + 3] = fmax(e[d + 3], ebox[d + 3][w]);
            }
        }
        ox = uniform(0.5 * (e[0] + e[3]));
        oy = uniform(0.5 * (e[1] + e[4]));
        oz = uniform(0.5 * (e[2] + e[5]));
    }
    const double hx = 0.5 * (hi_x - lo_x), hy = 0.5 * (hi_y - lo_y), hz = 0.5 * (hi_z - lo_z);
    const double rc2d = 0.0625 * (hx * hx + hy * hy + hz * hz);  // (rho / 4)^2

    // rc2[t]: the close-pair radius squared of target t, a quarter of its own
    // distance from the origin (the error bound 4u (1 + |t - o| / |d|) holds
    // for every target; a lane-wise radius takes the branch less often than
    // the workgroup's rho / 4); 0 for slots past the last target
    float thx[TPT], thy[TPT], thz[TPT], tlx[TPT], tly[TPT], tlz[TPT], rc2[TPT];
    float ax[TPT], ay[TPT], az[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const double rx = px[t] - ox, ry = py[t] - oy, rz = pz[t] - oz;
        thx[t] = (float)rx;
        thy[t] = (float)ry;
        thz[t] = (float)rz;
        tlx[t] = (float)(rx - (double)thx[t]);
        tly[t] = (float)(ry - (double)thy[t]);
        tlz[t] = (float)(rz - (double)thz[t]);
        const uint32_t ts = tbase + (uint32_t)(t * kFieldThreads + tid);
        rc2[t] = ts < nt ? 0.0625f * (float)((double)thx[t] * thx[t] + (double)thy[t] * thy[t] +
                                             (double)thz[t] * thz[t])
                         : 0.0f;
        if (PREC == GCCD_PRECISION_DEFAULT && ts < nt) rc2[t] = fmaxf(rc2[t], a.acc2);
        ax[t] = 0.0f;
        ay[t] = 0.0f;
        az[t] = 0.0f;
    }

    double qx = 0.0, qy = 0.0, qz = 0.0;  // this lane's source of the next tile
    double qb = 0.0;                      // lanes 0-5: one bound of that tile's box
    auto fetch = [&](uint32_t t) {
        const uint32_t i = t * kTile + (uint32_t)tid;
        qx = ox;
        qy = oy;
        qz = oz;
        if (i < ns) {
            qx = a.px[off + i];
            qy = a.py[off + i];
            qz = a.pz[off + i];
        }
        if (tid < 6) qb = a.tile_box[(size_t)tid * a.tile_stride + tile0 + t];
    };
    auto stage = [&](int b) {
        if (tid < 6) tbox[b][tid] = qb;
        const double rx = qx - ox, ry = qy - oy, rz = qz - oz;
        const float fx = (float)rx, fy = (float)ry, fz = (float)rz;
        sh[b][0][tid] = fx;
        sh[b][1][tid] = fy;
        sh[b][2][tid] = fz;
        sh[b][3][tid] = (float)(rx - (double)fx);
        sh[b][4][tid] = (float)(ry - (double)fy);
        sh[b][5][tid] = (float)(rz - (double)fz);
    };

    int buf = 0;
    if (t_first < t_end) {
        fetch(t_first);
        stage(0);
    }
    __syncthreads();
    for (uint32_t t = t_first; t < t_end; t += step_t) {
        const uint32_t next = t + step_t;
        if (next < t_end) fetch(next);
        const uint32_t cnt = min((uint32_t)kTile, ns - t * kTile);

        float bx[TPT], by[TPT], bz[TPT];
#pragma unroll
        for (int u = 0; u < TPT; ++u) bx[u] = by[u] = bz[u] = 0.0f;

        const float* hxp = sh[buf][0];
        const float* hyp = sh[buf][1];
        const float* hzp = sh[buf][2];
        const float* lxp = sh[buf][3];
        const float* lyp = sh[buf][4];
        const float* lzp = sh[buf][5];
        // A tile whose bounding box is at least rho/4 from the targets' box
        // cannot hold a close pair: its pairs skip the per-pair check.
        const double* tb = tbox[buf];
        const double gx = fmax(0.0, fmax(tb[0] - hi_x, lo_x - tb[3]));
        const double gy = fmax(0.0, fmax(tb[1] - hi_y, lo_y - tb[4]));
        const double gz = fmax(0.0, fmax(tb[2] - hi_z, lo_z - tb[5]));
        const bool far_tile = gx * gx + gy * gy + gz * gz >= fmax(rc2d, a.acc_box2);
        if (PREC == GCCD_PRECISION_COMPENSATED) {
            tile_terms<TPT, kDiffAll>(hxp, hyp, hzp, lxp, lyp, lzp, cnt, thx, thy, thz, tlx, tly,
                                      tlz, a.eps2, rc2, bx, by, bz);
        } else if (PREC != GCCD_PRECISION_DEFAULT || far_tile) {
            tile_terms<TPT, kDiffHi>(hxp, hyp, hzp, lxp, lyp, lzp, cnt, thx, thy, thz, tlx, tly,
                                     tlz, a.eps2, rc2, bx, by, bz);
        } else {
            tile_terms<TPT, kDiffNear, false, true>(hxp, hyp, hzp, lxp, lyp, lzp, cnt, thx, thy,
                                                    thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz,
                                                    0.0f, &a, &xl, (uint32_t)tid, t * kTile);
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            ax[u] += bx[u];
            ay[u] += by[u];
            az[u] += bz[u];
        }
        if (next < t_end) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    if (PREC == GCCD_PRECISION_DEFAULT) exact_flush(a, xl, off, tbase);
    float* outx = a.part + (size_t)(chunk * 3 + 0) * a.pstride + off;
    float* outy = a.part + (size_t)(chunk * 3 + 1) * a.pstride + off;
    float* outz = a.part + (size_t)(chunk * 3 + 2) * a.pstride + off;
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const uint32_t ts = tbase + (uint32_t)(t * kFieldThreads + tid);
        if (ts < nt) {
            outx[ts] = ax[t];
            outy[ts] = ay[t];
            outz[ts] = az[t];
        }
    }
}

// Default precision, one target per lane: the far tiles in the expanded form.
//
// For a source tile whose bounding box lies more than rho from the box of
// the wave's targets (rho: the half-diagonal of the workgroup's targets, whose
// centre is the origin), every pair has |d| > rho, and the pair sum is taken
// from
//     |d|^2 + eps^2 = (|s|^2 + eps^2) + |t|^2 - 2 t.s,
//     sum d w = t sum w - sum s w,          w = (|d|^2 + eps^2)^{-3/2},
// with s and t the hi parts relative to the workgroup origin.  The staged
// tile holds -2 s and S = |s|^2 + eps^2 (rounded once from FP64), so a pair
// costs an add, three FMAs for r^2, the reciprocal square root cubed and
// four accumulations -- 11 VALU against 12 for the difference form.  The
// expansion loses accuracy to cancellation: the partial results of r^2 are
// bounded by (|s| + |t|)^2 <= (2 rho + |d|)^2 <= 9 |d|^2, so r^2 carries at
// most 45u relative error and the term about 68u, plus the 8u of the dropped
// lo parts (as for the difference form at |d| > rho): below 5e-6 in all.
// The final t sum w - sum s w cancels by at most (|t| + |s|)/|d| <= 3, which
// scales the FP32 summation error of those tiles by that factor.  It is
// formed in FP64 from the FP32 sums.
//
// Tiles within rho of the wave's box take the difference form exactly as
// field_tiles<1, DEFAULT> does (the sources' hi parts recovered from -2 s by
// an exact halving inside the FMA), with the same close-pair rule (tiles
// within rho/4 of the wave's box checked pair by pair against a quarter of
// each target's distance from the origin; a tile farther than that holds no
// close pair of the wave, so the unchecked sum is the same), so in a launch
// that fills the GPU
// the close pairs -- and whole small events, which have no far tiles -- are
// summed bit for bit as by that kernel.  Small loads differ on purpose: see
// COMP below.
// CHECK: pairs closer than the lane's radius (rc2, at least acc2 for a target,
// 0 for a padding lane) are recomputed with the lo parts, and those below acc2
// (source slot src of the event) are recorded for exact summation.
template <bool CHECK>
__device__ __forceinline__ void diff_pair(const FieldArgs& a, ExactList& xl, uint32_t src,
                                          const float* __restrict__ lxp,
                                          const float* __restrict__ lyp,
                                          const float* __restrict__ lzp, uint32_t k, float m2x,
                                          float m2y, float m2z, float thx, float thy, float thz,
                                          float tlx, float tly, float tlz, float eps2, float rc2,
                                          float& bx, float& by, float& bz) {
    // thx + 0.5 (-2 s_x) rounds once, to the same value as thx - s_x
    float dx = __builtin_fmaf(m2x, 0.5f, thx);
    float dy = __builtin_fmaf(m2y, 0.5f, thy);
    float dz = __builtin_fmaf(m2z, 0.5f, thz);
    float r2 = __builtin_fmaf(dx, dx, eps2);
    r2 = __builtin_fmaf(dy, dy, r2);
    r2 = __builtin_fmaf(dz, dz, r2);
    if (CHECK && __builtin_expect(__ballot(r2 < rc2) != 0ull, 0)) {
        const float nlx = lxp[k], nly = lyp[k], nlz = lzp[k];
        if (r2 < rc2) {
            dx += tlx - nlx;
            dy += tly - nly;
            dz += tlz - nlz;
            r2 = __builtin_fmaf(dx, dx, eps2);
            r2 = __builtin_fmaf(dy, dy, r2);
            r2 = __builtin_fmaf(dz, dz, r2);
        }
        if (r2 < fminf(a.acc2, rc2) && r2 > eps2 && exact_push(xl, threadIdx.x, src))
            dx = dy = dz = 0.0f;
    }
    const float inv = __builtin_amdgcn_rsqf(r2);
    const float w = inv * inv * inv;
    bx = __builtin_fmaf(dx, w, bx);
    by = __builtin_fmaf(dy, w, by);
    bz = __builtin_fmaf(dz, w, bz);
}

// Difference form with the lo parts in every pair (the compensated
// difference of the COMPENSATED mode); pairs below acc2 are recorded for
// exact summation.
__device__ __forceinline__ void comp_pair(const FieldArgs& a, ExactList& xl, uint32_t src,
                                          float m2x, float m2y,
                                          float m2z, float lx, float ly, float lz, float thx,
                                          float thy, float thz, float tlx, float tly, float tlz,
                                          float eps2, float rc2, float& bx, float& by,
                                          float& bz) {
    float dx = __builtin_fmaf(m2x, 0.5f, thx) + (tlx - lx);
    float dy = __builtin_fmaf(m2y, 0.5f, thy) + (tly - ly);
    float dz = __builtin_fmaf(m2z, 0.5f, thz) + (tlz - lz);
    float r2 = __builtin_fmaf(dx, dx, eps2);
    r2 = __builtin_fmaf(dy, dy, r2);
    r2 = __builtin_fmaf(dz, dz, r2);
    if (__builtin_expect(__ballot(r2 < fminf(a.acc2, rc2)) != 0ull, 0)) {
        if (r2 < fminf(a.acc2, rc2) && r2 > eps2 && exact_push(xl, threadIdx.x, src))
            dx = dy = dz = 0.0f;
    }
    const float inv = __builtin_amdgcn_rsqf(r2);
    const float w = inv * inv * inv;
    bx = __builtin_fmaf(dx, w, bx);
    by = __builtin_fmaf(dy, w, by);
    bz = __builtin_fmaf(dz, w, bz);
}

__device__ __forceinline__ void comp_tile(const FieldArgs& a, ExactList& xl, uint32_t src0,
                                          const float* __restrict__ mxp, const float* __restrict__ myp,
                                          const float* __restrict__ mzp, const float* __restrict__ lxp,
                                          const float* __restrict__ lyp, const float* __restrict__ lzp,
                                          uint32_t cnt, float thx, float thy, float thz, float tlx,
                                          float tly, float tlz, float eps2, float rc2, float& bx,
                                          float& by, float& bz) {
    uint32_t k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const float4 x4 = *reinterpret_cast<const float4*>(mxp + k);
        const float4 y4 = *reinterpret_cast<const float4*>(myp + k);
        const float4 z4 = *reinterpret_cast<const float4*>(mzp + k);
        const float4 a4 = *reinterpret_cast<const float4*>(lxp + k);
        const float4 b4 = *reinterpret_cast<const float4*>(lyp + k);
        const float4 c4 = *reinterpret_cast<const float4*>(lzp + k);
        comp_pair(a, xl, src0 + k + 0, x4.x, y4.x, z4.x, a4.x, b4.x, c4.x, thx, thy, thz, tlx, tly, tlz, eps2,
                  rc2, bx, by, bz);
        comp_pair(a, xl, src0 + k + 1, x4.y, y4.y, z4.y, a4.y, b4.y, c4.y, thx, thy, thz, tlx, tly, tlz, eps2,
                  rc2, bx, by, bz);
        comp_pair(a, xl, src0 + k + 2, x4.z, y4.z, z4.z, a4.z, b4.z, c4.z, thx, thy, thz, tlx, tly, tlz, eps2,
                  rc2, bx, by, bz);
        comp_pair(a, xl, src0 + k + 3, x4.w, y4.w, z4.w, a4.w, b4.w, c4.w, thx, thy, thz, tlx, tly, tlz, eps2,
                  rc2, bx, by, bz);
    }
    for (; k < cnt; ++k)
        comp_pair(a, xl, src0 + k, mxp[k], myp[k], mzp[k], lxp[k], lyp[k], lzp[k], thx, thy, thz,
                  tlx, tly, tlz, eps2, rc2, bx, by, bz);
}

template <bool CHECK>
__device__ __forceinline__ void diff_tile(const FieldArgs& a, ExactList& xl, uint32_t src0,
                                          const float* __restrict__ mxp,
                                          const float* __restrict__ myp,
                                          const float* __restrict__ mzp,
                                          const float* __restrict__ lxp,
                                          const float* __restrict__ lyp,
                                          const float* __restrict__ lzp, uint32_t cnt, float thx,
                                          float thy, float thz, float tlx, float tly, float tlz,
                                          float eps2, float rc2, float& bx, float& by,
                                          float& bz) {
    uint32_t k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const float4 x4 = *reinterpret_cast<const float4*>(mxp + k);
        const float4 y4 = *reinterpret_cast<const float4*>(myp + k);
        const float4 z4 = *reinterpret_cast<const float4*>(mzp + k);
        diff_pair<CHECK>(a, xl, src0 + k + 0, lxp, lyp, lzp, k + 0, x4.x, y4.x, z4.x, thx, thy, thz, tlx, tly, tlz,
                         eps2, rc2, bx, by, bz);
        diff_pair<CHECK>(a, xl, src0 + k + 1, lxp, lyp, lzp, k + 1, x4.y, y4.y, z4.y, thx, thy, thz, tlx, tly, tlz,
                         eps2, rc2, bx, by, bz);
        diff_pair<CHECK>(a, xl, src0 + k + 2, lxp, lyp, lzp, k + 2, x4.z, y4.z, z4.z, thx, thy, thz, tlx, tly, tlz,
                         eps2, rc2, bx, by, bz);
        diff_pair<CHECK>(a, xl, src0 + k + 3, lxp, lyp, lzp, k + 3, x4.w, y4.w, z4.w, thx, thy, thz, tlx, tly, tlz,
                         eps2, rc2, bx, by, bz);
    }
    for (; k < cnt; ++k)
        diff_pair<CHECK>(a, xl, src0 + k, lxp, lyp, lzp, k, mxp[k], myp[k], mzp[k], thx, thy, thz, tlx, tly, tlz,
                         eps2, rc2, bx, by, bz);
}

__device__ __forceinline__ void expanded_pair(float m2x, float m2y, float m2z, float S, float T,
                                              float thx, float thy, float thz, float& sw,
                                              float& sx, float& sy, float& sz) {
    float r2 = S + T;
    r2 = __builtin_fmaf(thz, m2z, r2);
    r2 = __builtin_fmaf(thy, m2y, r2);
    r2 = __builtin_fmaf(thx, m2x, r2);
    const float inv = __builtin_amdgcn_rsqf(r2);
    const float w = inv * inv * inv;
    sw += w;
    sx = __builtin_fmaf(m2x, w, sx);
    sy = __builtin_fmaf(m2y, w, sy);
    sz = __builtin_fmaf(m2z, w, sz);
}

// One work item.  Every lane of the workgroup calls it with the same item;
// it returns early only for an item without targets, before any barrier, and
// otherwise ends after a barrier, so the LDS can take the next item at once.
struct ExpandedLds {
    float sh[2][7][kTile];  // staged: -2 s_x, -2 s_y, -2 s_z, |s|^2 + eps^2, lo_x, lo_y, lo_z
    double box[6][kFieldThreads / 64];
    double tbox[2][6];      // bounding box of the staged source tile
    ExactList xl;           // close pairs of the item
};

// COMP: tiles closer than rho/4 to the targets take the compensated
// difference in every pair instead of the per-pair check and its branch.
// In a launch of at most one round of workgroups (a small cloud) nearly
// every wave finds a close pair in such tiles, the branch is taken almost
// always, and the branch-free form halves the launch; in a full GPU the
// check is cheaper per pair.
// The box bound k (0-2 low x, y, z; 3-5 high) of source tile t of UNIT
// sources of the event whose 256-source tiles start at tile0: a 256-source
// tile's own box, a 64-source quarter's, or the union of two quarters'.
template <int UNIT>
__device__ __forceinline__ double unit_bound(const FieldArgs& a, uint32_t tile0, uint32_t t,
                                             int k) {
    const size_t st = a.tile_stride;
    if (UNIT == kTile) return a.tile_box[(size_t)k * st + tile0 + t];
    if (UNIT == kTile / 4)
        return a.tile_box[(size_t)(6 + 4 * k + (int)(t & 3u)) * st + tile0 + (t >> 2)];
    const int q = 2 * (int)(t & 1u);
    const double v0 = a.tile_box[(size_t)(6 + 4 * k + q) * st + tile0 + (t >> 1)];
    const double v1 = a.tile_box[(size_t)(6 + 4 * k + q + 1) * st + tile0 + (t >> 1)];
    return k < 3 ? fmin(v0, v1) : fmax(v0, v1);
}

// UNIT: sources per staged tile (256, 128 or 64; the work item's first,
// step and end count such tiles).  Smaller tiles give a small cloud more
// work items of fewer sources each; the LDS layout is the same.
template <bool COMP, int UNIT>
__device__ __forceinline__ void expanded_item(const FieldArgs& a, const FieldItem it,
                                              ExpandedLds& L, uint32_t na0) {
    auto& sh = L.sh;
    auto& box = L.box;
    auto& tbox = L.tbox;
    // a single event (na0: its travelling holes, read with the item) needs
    // no lookups before the targets' loads
    const bool one = a.one_event_n != 0u;
    const uint32_t off = one ? 0u : a.ev_off[it.event];
    const uint32_t ne = one ? a.one_event_n : a.ev_off[it.event + 1] - off;
    const uint32_t na = one ? na0 : a.ev_active[it.event];
    const uint32_t nt = a.targets_all ? ne : na;
    const uint32_t ns = a.sources_all ? ne : na;
    const uint32_t tbase = it.blk * (uint32_t)kFieldThreads;
    if (tbase >= nt) return;  // the whole workgroup leaves before any barrier
    const uint32_t ntiles = (ns + UNIT - 1) / UNIT;
    const uint32_t tile0 = one ? 0u : a.ev_tile[it.event];
    const uint32_t chunk = it.group;  // partial-sum group written
    const uint32_t step_t = it.step;
    const uint32_t t_first = it.first;
    const uint32_t t_end = min(it.end, ntiles);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;

    const uint32_t ts = tbase + (uint32_t)tid;
    double px = 0.0, py = 0.0, pz = 0.0;
    double lo_x = INFINITY, lo_y = INFINITY, lo_z = INFINITY;
    double hi_x = -INFINITY, hi_y = -INFINITY, hi_z = -INFINITY;
    if (ts < nt) {
        px = a.px[off + ts];
        py = a.py[off + ts];
        pz = a.pz[off + ts];
        lo_x = hi_x = px;
        lo_y = hi_y = py;
        lo_z = hi_z = pz;
    }
    lo_x = wave_min(lo_x);
    lo_y = wave_min(lo_y);
    lo_z = wave_min(lo_z);
    hi_x = wave_max(hi_x);
    hi_y = wave_max(hi_y);
    hi_z = wave_max(hi_z);
    // this wave's own 64 targets: each wave classifies the source tiles by
    // their distance from its own box (at least their distance from the
    // workgroup's), so a tile near only the other waves' targets is far here
    const double wl_x = uniform(lo_x), wl_y = uniform(lo_y), wl_z = uniform(lo_z);
    const double wh_x = uniform(hi_x), wh_y = uniform(hi_y), wh_z = uniform(hi_z);
    if (lane == 0) {
        box[0][wave] = lo_x;
        box[1][wave] = lo_y;
        box[2][wave] = lo_z;
        box[3][wave] = hi_x;
        box[4][wave] = hi_y;
        box[5][wave] = hi_z;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kFieldThreads / 64; ++w) {
        lo_x = fmin(lo_x, box[0][w]);
        lo_y = fmin(lo_y, box[1][w]);
        lo_z = fmin(lo_z, box[2][w]);
        hi_x = fmax(hi_x, box[3][w]);
        hi_y = fmax(hi_y, box[4][w]);
        hi_z = fmax(hi_z, box[5][w]);
    }
    lo_x = uniform(lo_x);
    lo_y = uniform(lo_y);
    lo_z = uniform(lo_z);
    hi_x = uniform(hi_x);
    hi_y = uniform(hi_y);
    hi_z = uniform(hi_z);
    const double ox = 0.5 * (lo_x + hi_x), oy = 0.5 * (lo_y + hi_y), oz = 0.5 * (lo_z + hi_z);
    const double hx = 0.5 * (hi_x - lo_x), hy = 0.5 * (hi_y - lo_y), hz = 0.5 * (hi_z - lo_z);
    // no expanded or unchecked tile may hold a pair closer than kExactRadius eps
    const double rho2 = fmax(hx * hx + hy * hy + hz * hz, a.acc_box2);
    const double rc2d = fmax(0.0625 * (hx * hx + hy * hy + hz * hz), a.acc_box2);  // (rho/4)^2
    const double eps2d = (double)a.eps2;

    float thx, thy, thz, tlx, tly, tlz, T;
    {
        // lanes past the last target sit at the origin (their sums are unused)
        const double rx = (ts < nt ? px : ox) - ox, ry = (ts < nt ? py : oy) - oy,
                     rz = (ts < nt ? pz : oz) - oz;
        thx = (float)rx;
        thy = (float)ry;
        thz = (float)rz;
        tlx = (float)(rx - (double)thx);
        tly = (float)(ry - (double)thy);
        tlz = (float)(rz - (double)thz);
        T = (float)((double)thx * thx + (double)thy * thy + (double)thz * thz);
    }
    // this lane's close-pair radius squared: a quarter of its target's
    // distance from the origin, as in field_tiles, and at least the exact-sum
    // radius (0 for the padding lanes)
    const float rc2 = ts < nt ? fmaxf(0.0625f * T, a.acc2) : 0.0f;
    float sw = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;  // far tiles
    float ex = 0.0f, ey = 0.0f, ez = 0.0f;              // near tiles

    double qx = 0.0, qy = 0.0, qz = 0.0;  // this lane's source of the next tile
    double qb = 0.0;                      // lanes 0-5: one bound of that tile's box
    auto fetch = [&](uint32_t t) {
        const uint32_t i = t * UNIT + (uint32_t)tid;
        qx = ox;
        qy = oy;
        qz = oz;
        if (tid < UNIT && i < ns) {
            qx = a.px[off + i];
            qy = a.py[off + i];
            qz = a.pz[off + i];
        }
        if (tid < 6) qb = unit_bound<UNIT>(a, tile0, t, tid);
    };
    auto stage = [&](int b) {
        if (tid < 6) tbox[b][tid] = qb;
        const double rx = qx - ox, ry = qy - oy, rz = qz - oz;
        const float fx = (float)rx, fy = (float)ry, fz = (float)rz;
        sh[b][0][tid] = -2.0f * fx;
        sh[b][1][tid] = -2.0f * fy;
        sh[b][2][tid] = -2.0f * fz;
        sh[b][3][tid] = (float)((double)fx * fx + (double)fy * fy + (double)fz * fz + eps2d);
        sh[b][4][tid] = (float)(rx - (double)fx);
        sh[b][5][tid] = (float)(ry - (double)fy);
        sh[b][6][tid] = (float)(rz - (double)fz);
    };

    int buf = 0;
    if (t_first < t_end) {
        fetch(t_first);
        stage(0);
    }
    __syncthreads();
    for (uint32_t t = t_first; t < t_end; t += step_t) {
        const uint32_t next = t + step_t;
        if (next < t_end) fetch(next);
        const uint32_t cnt = min((uint32_t)UNIT, ns - t * UNIT);
        const float* mxp = sh[buf][0];
        const float* myp = sh[buf][1];
        const float* mzp = sh[buf][2];
        const double* tb = tbox[buf];
        const double gx = fmax(0.0, fmax(tb[0] - wh_x, wl_x - tb[3]));
        const double gy = fmax(0.0, fmax(tb[1] - wh_y, wl_y - tb[4]));
        const double gz = fmax(0.0, fmax(tb[2] - wh_z, wl_z - tb[5]));
        const double g2 = gx * gx + gy * gy + gz * gz;  // wave-uniform
        if (g2 > rho2) {
            const float* Sp = sh[buf][3];
            float bw = 0.0f, bx = 0.0f, by = 0.0f, bz = 0.0f;
            uint32_t k = 0;
            for (; k + 4 <= cnt; k += 4) {
                const float4 x4 = *reinterpret_cast<const float4*>(mxp + k);
                const float4 y4 = *reinterpret_cast<const float4*>(myp + k);
                const float4 z4 = *reinterpret_cast<const float4*>(mzp + k);
                const float4 s4 = *reinterpret_cast<const float4*>(Sp + k);
                expanded_pair(x4.x, y4.x, z4.x, s4.x, T, thx, thy, thz, bw, bx, by, bz);
                expanded_pair(x4.y, y4.y, z4.y, s4.y, T, thx, thy, thz, bw, bx, by, bz);
                expanded_pair(x4.z, y4.z, z4.z, s4.z, T, thx, thy, thz, bw, bx, by, bz);
                expanded_pair(x4.w, y4.w, z4.w, s4.w, T, thx, thy, thz, bw, bx, by, bz);
            }
            for (; k < cnt; ++k)
                expanded_pair(mxp[k], myp[k], mzp[k], Sp[k], T, thx, thy, thz, bw, bx, by, bz);
            sw += bw;
            sx += bx;
            sy += by;
            sz += bz;
        } else {
            float bx = 0.0f, by = 0.0f, bz = 0.0f;
            if (g2 >= rc2d)
                diff_tile<false>(a, L.xl, t * UNIT, mxp, myp, mzp, sh[buf][4], sh[buf][5], sh[buf][6], cnt,
                                 thx, thy, thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz);
            else if (COMP)
                comp_tile(a, L.xl, t * UNIT, mxp, myp, mzp, sh[buf][4], sh[buf][5], sh[buf][6], cnt, thx,
                          thy, thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz);
            else
                diff_tile<true>(a, L.xl, t * UNIT, mxp, myp, mzp, sh[buf][4], sh[buf][5], sh[buf][6], cnt,
                                thx, thy, thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz);
            ex += bx;
            ey += by;
            ez += bz;
        }
        if (next < t_end) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    exact_flush(a, L.xl, off, tbase);

    if (ts < nt) {
        // t sum w - sum s w, the second held as -2 sum s w
        const float fx = (float)((double)thx * sw + 0.5 * (double)sx) + ex;
        const float fy = (float)((double)thy * sw + 0.5 * (double)sy) + ey;
        const float fz = (float)((double)thz * sw + 0.5 * (double)sz) + ez;
        a.part[(size_t)(chunk * 3 + 0) * a.pstride + off + ts] = fx;
        a.part[(size_t)(chunk * 3 + 1) * a.pstride + off + ts] = fy;
        a.part[(size_t)(chunk * 3 + 2) * a.pstride + off + ts] = fz;
    }
}

// One workgroup per work item.
template <bool COMP, int UNIT>
__global__ __launch_bounds__(kFieldThreads) void field_tiles_expanded(FieldArgs a) {
    // the item, the count and event 0's travelling holes are read together
    // (the grid never exceeds the item capacity, so the item is in bounds)
    const FieldItem it = a.items[blockIdx.x];
    const uint32_t na0 = a.ev_active[0];
    if (a.count_items && blockIdx.x >= *a.n_items) return;  // the whole workgroup
    __shared__ __align__(16) ExpandedLds L;
    if (threadIdx.x == 0) L.xl.n = 0;  // ordered before any push by the item's first barrier
    expanded_item<COMP, UNIT>(a, it, L, na0);
}

// Persistent form: a fixed grid of workgroups takes the items in list order
// from a counter (queue[0], zero before the launch) until *n_items are taken.
// Every workgroup leaves once the counter has passed the end, so the grid
// drains whatever the item count; the grid and the arguments stay the same
// when the items are rebuilt, which lets a captured graph be replayed.
template <bool COMP, int UNIT>
__global__ __launch_bounds__(kFieldThreads) __attribute__((amdgpu_waves_per_eu(7)))
void field_queue_expanded(FieldArgs a) {
    __shared__ __align__(16) ExpandedLds L;
    __shared__ uint32_t next;
    const uint32_t n_items = *a.n_items;
    const uint32_t na0 = a.ev_active[0];
    if (threadIdx.x == 0) L.xl.n = 0;  // ordered before any push by the barriers below
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t i = next;
        __syncthreads();  // every lane has read `next` before lane 0 writes it again
        if (i >= n_items) break;
        expanded_item<COMP, UNIT>(a, a.items[i], L, na0);
    }
}

// Eq. (6) entirely in FP64: the difference, r^2 + eps^2, r^-3 = 1/(q sqrt q)
// with IEEE square root and division, and the sums.  Same work items, tiles
// and source dealing as field_tiles; the FP64 sum of group g is written as
// the FP32 pair hi (group g) and lo (group G + g, G the event's groups),
// which the FP64 reduction of the groups adds back exactly.
template <int TPT>
__global__ __launch_bounds__(kFieldThreads) void field_tiles_f64(FieldArgs a) {
    __shared__ double sh[2][3][kTile];

    const FieldItem it = a.items[blockIdx.x];
    const uint32_t off = a.ev_off[it.event];
    const uint32_t ne = a.ev_off[it.event + 1] - off;
    const uint32_t na = a.ev_active[it.event];
    const uint32_t nt = a.targets_all ? ne : na;
    const uint32_t ns = a.sources_all ? ne : na;
    const uint32_t tbase = it.blk * (uint32_t)(kFieldThreads * TPT);
    if (tbase >= nt) return;
    const uint32_t ntiles = (ns + kTile - 1) / kTile;
    const uint32_t chunk = it.group;  // partial-sum group written
    const uint32_t step_t = it.step;
    const uint32_t t_first = it.first;
    const uint32_t t_end = min(it.end, ntiles);
    const int tid = threadIdx.x;
    const double eps2 = a.eps2d;

    double px[TPT], py[TPT], pz[TPT], ax[TPT], ay[TPT], az[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const uint32_t ts = tbase + (uint32_t)(t * kFieldThreads + tid);
        px[t] = py[t] = pz[t] = 0.0;
        if (ts < nt) {
            px[t] = a.px[off + ts];
            py[t] = a.py[off + ts];
            pz[t] = a.pz[off + ts];
        }
        ax[t] = ay[t] = az[t] = 0.0;
    }

    double qx = 0.0, qy = 0.0, qz = 0.0;
    auto fetch = [&](uint32_t t) {
        const uint32_t i = t * kTile + (uint32_t)tid;
        qx = qy = qz = 0.0;
        if (i < ns) {
            qx = a.px[off + i];
            qy = a.py[off + i];
            qz = a.pz[off + i];
        }
    };
    auto stage = [&](int b) {
        sh[b][0][tid] = qx;
        sh[b][1][tid] = qy;
        sh[b][2][tid] = qz;
    };

    int buf = 0;
    if (t_first < t_end) {
        fetch(t_first);
        stage(0);
    }
    __syncthreads();
    for (uint32_t t = t_first; t < t_end; t += step_t) {
        const uint32_t next = t + step_t;
        if (next < t_end) fetch(next);
        const uint32_t cnt = min((uint32_t)kTile, ns - t * kTile);
        for (uint32_t k = 0; k < cnt; ++k) {
            const double sx = sh[buf][0][k], sy = sh[buf][1][k], sz = sh[buf][2][k];
#pragma unroll
            for (int u = 0; u < TPT; ++u) {
                const double dx = px[u] - sx, dy = py[u] - sy, dz = pz[u] - sz;
                double q = fma(dx, dx, eps2);
                q = fma(dy, dy, q);
                q = fma(dz, dz, q);
                const double w = 1.0 / (q * sqrt(q));
                ax[u] = fma(dx, w, ax[u]);
                ay[u] = fma(dy, w, ay[u]);
                az[u] = fma(dz, w, az[u]);
            }
        }
        if (next < t_end) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const uint32_t ts = tbase + (uint32_t)(t * kFieldThreads + tid);
        if (ts >= nt) continue;
        const double v[3] = {ax[t], ay[t], az[t]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float hi = (float)v[d];
            const float lo = (float)(v[d] - (double)hi);
            a.part[(size_t)(chunk * 3 + d) * a.pstride + off + ts] = hi;
            a.part[(size_t)((it.groups + chunk) * 3 + d) * a.pstride + off + ts] = lo;
        }
    }
}

// ---------------------------------------------------------------------------
// Near part of the closure's split of Eq. (6): the same sum over the
// sources closer than a only (r^2 + eps^2 < a^2 + eps^2).  Work items,
// origins, hi/lo staging and the close-pair recomputation are those of
// field_tiles; the difference is which tiles are visited.  The item's
// candidate tiles (first, first + S, ...) are tested 256 at a time against
// the targets' box, the ones within a are compacted into an LDS list, and
// only those are staged and summed, each wave taking only the 16-source
// groups of a staged tile that come within a of its own 64 targets.  A
// group entirely within a of every target of the wave skips the per-pair
// cutoff.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFieldThreads) void near_tiles(FieldArgs a, const GridParams* gp) {
    __shared__ __align__(16) float sh[2][6][kTile];
    __shared__ double box[6][kFieldThreads / 64];
    __shared__ double tbox[2][kBoxRows];  // the staged tile's boxes (tile, quarters, groups)
    __shared__ uint32_t list[kFieldThreads];
    __shared__ uint32_t wcount[kFieldThreads / 64];

    const FieldItem it = a.items[blockIdx.x];
    const uint32_t off = a.ev_off[it.event];
    const uint32_t ne = a.ev_off[it.event + 1] - off;
    const uint32_t na = a.ev_active[it.event];
    const uint32_t nt = a.targets_all ? ne : na;
    const uint32_t ns = a.sources_all ? ne : na;
    const uint32_t tbase = it.blk * (uint32_t)kFieldThreads;
    if (tbase >= nt) return;
    const uint32_t ntiles = (ns + kTile - 1) / kTile;
    const uint32_t tile0 = a.ev_tile[it.event];
    const uint32_t chunk = it.group;  // partial-sum group written
    const uint32_t step_t = it.step;
    const uint32_t t_first = it.first;
    const uint32_t t_end = min(it.end, ntiles);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;

    const uint32_t ts = tbase + (uint32_t)tid;
    double px = 0.0, py = 0.0, pz = 0.0;
    double lo_x = INFINITY, lo_y = INFINITY, lo_z = INFINITY;
    double hi_x = -INFINITY, hi_y = -INFINITY, hi_z = -INFINITY;
    if (ts < nt) {
        px = a.px[off + ts];
        py = a.py[off + ts];
        pz = a.pz[off + ts];
        lo_x = hi_x = px;
        lo_y = hi_y = py;
        lo_z = hi_z = pz;
    }
    lo_x = wave_min(lo_x);
    lo_y = wave_min(lo_y);
    lo_z = wave_min(lo_z);
    hi_x = wave_max(hi_x);
    hi_y = wave_max(hi_y);
    hi_z = wave_max(hi_z);
    // this wave's own 64 targets, for culling source quarters
    const double wl_x = uniform(lo_x), wl_y = uniform(lo_y), wl_z = uniform(lo_z);
    const double wh_x = uniform(hi_x), wh_y = uniform(hi_y), wh_z = uniform(hi_z);
    if (lane == 0) {
        box[0][wave] = lo_x;
        box[1][wave] = lo_y;
        box[2][wave] = lo_z;
        box[3][wave] = hi_x;
        box[4][wave] = hi_y;
        box[5][wave] = hi_z;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kFieldThreads / 64; ++w) {
        lo_x = fmin(lo_x, box[0][w]);
        lo_y = fmin(lo_y, box[1][w]);
        lo_z = fmin(lo_z, box[2][w]);
        hi_x = fmax(hi_x, box[3][w]);
        hi_y = fmax(hi_y, box[4][w]);
        hi_z = fmax(hi_z, box[5][w]);
    }
    lo_x = uniform(lo_x);
    lo_y = uniform(lo_y);
    lo_z = uniform(lo_z);
    hi_x = uniform(hi_x);
    hi_y = uniform(hi_y);
    hi_z = uniform(hi_z);
    const double ox = 0.5 * (lo_x + hi_x), oy = 0.5 * (lo_y + hi_y), oz = 0.5 * (lo_z + hi_z);
    const double hx = 0.5 * (hi_x - lo_x), hy = 0.5 * (hi_y - lo_y), hz = 0.5 * (hi_z - lo_z);
    const double rc2d = 0.0625 * (hx * hx + hy * hy + hz * hz);
    const double a2 = uniform(gp->a2);
    const float cut2 = uniform((float)gp->cut2);

    float thx[1], thy[1], thz[1], tlx[1], tly[1], tlz[1], ax[1], ay[1], az[1], rc2[1];
    {
        const double rx = px - ox, ry = py - oy, rz = pz - oz;
        thx[0] = (float)rx;
        thy[0] = (float)ry;
        thz[0] = (float)rz;
        tlx[0] = (float)(rx - (double)thx[0]);
        tly[0] = (float)(ry - (double)thy[0]);
        tlz[0] = (float)(rz - (double)thz[0]);
        ax[0] = ay[0] = az[0] = 0.0f;
        // close-pair radius of this target, as in field_tiles
        rc2[0] = ts < nt ? 0.0625f * (float)((double)thx[0] * thx[0] + (double)thy[0] * thy[0] +
                                             (double)thz[0] * thz[0])
                         : 0.0f;
    }

    double qx = 0.0, qy = 0.0, qz = 0.0, qb = 0.0;
    auto fetch = [&](uint32_t t) {
        const uint32_t i = t * kTile + (uint32_t)tid;
        qx = ox;
        qy = oy;
        qz = oz;
        if (i < ns) {
            qx = a.px[off + i];
            qy = a.py[off + i];
            qz = a.pz[off + i];
        }
        if (tid < kBoxRows) qb = a.tile_box[(size_t)tid * a.tile_stride + tile0 + t];
    };
    auto stage = [&](int b) {
        if (tid < kBoxRows) tbox[b][tid] = qb;
        const double rx = qx - ox, ry = qy - oy, rz = qz - oz;
        const float fx = (float)rx, fy = (float)ry, fz = (float)rz;
        sh[b][0][tid] = fx;
        sh[b][1][tid] = fy;
        sh[b][2][tid] = fz;
        sh[b][3][tid] = (float)(rx - (double)fx);
        sh[b][4][tid] = (float)(ry - (double)fy);
        sh[b][5][tid] = (float)(rz - (double)fz);
    };

    const uint32_t ncand = t_first < t_end ? (t_end - t_first + step_t - 1) / step_t : 0u;
    for (uint32_t base = 0; base < ncand; base += kFieldThreads) {
        // 1. which of the next 256 candidate tiles come within a of the targets
        const uint32_t m = base + (uint32_t)tid;
        bool keep = false;
        uint32_t t = 0;
        if (m < ncand) {
            t = t_first + m * step_t;
            const size_t g = (size_t)tile0 + t;
            const double* tb = a.tile_box;
            const size_t st = a.tile_stride;
            const double gx = fmax(0.0, fmax(tb[0 * st + g] - hi_x, lo_x - tb[3 * st + g]));
            const double gy = fmax(0.0, fmax(tb[1 * st + g] - hi_y, lo_y - tb[4 * st + g]));
            const double gz = fmax(0.0, fmax(tb[2 * st + g] - hi_z, lo_z - tb[5 * st + g]));
            keep = gx * gx + gy * gy + gz * gz < a2;
        }
        // 2. compact them, in candidate order, into the LDS list
        const uint64_t bal = __ballot(keep);
        if (lane == 0) wcount[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kFieldThreads / 64; ++w) {
            const uint32_t cw = wcount[w];
            if (w < wave) before += cw;
            total += cw;
        }
        if (keep) list[before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = t;
        __syncthreads();
        // 3. the kept tiles, double buffered as in field_tiles
        int buf = 0;
        if (total > 0) {
            fetch(list[0]);
            stage(0);
        }
        __syncthreads();
        for (uint32_t q = 0; q < total; ++q) {
            const uint32_t tt = list[q];
            const bool more = q + 1 < total;
            if (more) fetch(list[q + 1]);
            const uint32_t cnt = min((uint32_t)kTile, ns - tt * kTile);
            float bx[1] = {0.0f}, by[1] = {0.0f}, bz[1] = {0.0f};
            const double* tb = tbox[buf];
            // each wave takes the 16-source groups of the tile within a of its
            // own targets: lane l tests group l % 16 (three ballots collect the
            // answers), then the wave sums the groups that pass, one by one
            uint32_t cand, in_m, far_m;
            {
                const int grp = lane & 15;
                const double* gb = tb + 30 + grp;  // bound k of the group at gb[16 k]
                const double gx = fmax(0.0, fmax(gb[0] - wh_x, wl_x - gb[48]));
                const double gy = fmax(0.0, fmax(gb[16] - wh_y, wl_y - gb[64]));
                const double gz = fmax(0.0, fmax(gb[32] - wh_z, wl_z - gb[80]));
                const double gap2 = gx * gx + gy * gy + gz * gz;
                // largest distance between the boxes: every pair well inside a
                // (a margin far above the FP32 error of r^2) needs no per-pair test
                const double mx = fmax(gb[48] - wl_x, wh_x - gb[0]);
                const double my = fmax(gb[64] - wl_y, wh_y - gb[16]);
                const double mz = fmax(gb[80] - wl_z, wh_z - gb[32]);
                const bool valid = (uint32_t)grp * 16u < cnt;
                cand = (uint32_t)__ballot(valid && gap2 < a2) & 0xFFFFu;
                in_m = (uint32_t)__ballot(mx * mx + my * my + mz * mz < 0.9999 * a2) & 0xFFFFu;
                far_m = (uint32_t)__ballot(gap2 >= rc2d) & 0xFFFFu;
            }
            while (cand) {
                const int grp = __builtin_ctz(cand);
                cand &= cand - 1u;
                const uint32_t k0 = (uint32_t)grp * 16u;
                const uint32_t kn = min(16u, cnt - k0);
                const bool inside = (in_m >> grp) & 1u;
                const bool far_q = (far_m >> grp) & 1u;
                const float* hxp = sh[buf][0] + k0;
                const float* hyp = sh[buf][1] + k0;
                const float* hzp = sh[buf][2] + k0;
                const float* lxp = sh[buf][3] + k0;
                const float* lyp = sh[buf][4] + k0;
                const float* lzp = sh[buf][5] + k0;
                if (inside) {
                    if (far_q)
                        tile_terms<1, kDiffHi, false>(hxp, hyp, hzp, lxp, lyp, lzp, kn, thx, thy,
                                                      thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz);
                    else
                        tile_terms<1, kDiffNear, false>(hxp, hyp, hzp, lxp, lyp, lzp, kn, thx, thy,
                                                        thz, tlx, tly, tlz, a.eps2, rc2, bx, by,
                                                        bz);
                } else {
                    if (far_q)
                        tile_terms<1, kDiffHi, true>(hxp, hyp, hzp, lxp, lyp, lzp, kn, thx, thy,
                                                     thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz,
                                                     cut2);
                    else
                        tile_terms<1, kDiffNear, true>(hxp, hyp, hzp, lxp, lyp, lzp, kn, thx, thy,
                                                       thz, tlx, tly, tlz, a.eps2, rc2, bx, by, bz,
                                                       cut2);
                }
            }
            ax[0] += bx[0];
            ay[0] += by[0];
            az[0] += bz[0];
            if (more) stage(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    if (ts < nt) {
        a.part[(size_t)(chunk * 3 + 0) * a.pstride + off + ts] = ax[0];
        a.part[(size_t)(chunk * 3 + 1) * a.pstride + off + ts] = ay[0];
        a.part[(size_t)(chunk * 3 + 2) * a.pstride + off + ts] = az[0];
    }
}

hipError_t launch_near(const FieldArgs& a, const GridParams* gp, uint32_t n_items,
                       hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    near_tiles<<<n_items, kFieldThreads, 0, s>>>(a, gp);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_field_prec(const FieldArgs& a, int tpt, uint32_t n_items,
                                    hipStream_t s) {
    switch (tpt) {
        case 1: field_tiles<1, PREC><<<n_items, kFieldThreads, 0, s>>>(a); break;
        case 2: field_tiles<2, PREC><<<n_items, kFieldThreads, 0, s>>>(a); break;
        case 4: field_tiles<4, PREC><<<n_items, kFieldThreads, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Workgroups of the Eq. (6) kernel that one compute unit holds at once for
// this shape (registers and LDS permitting); 1 if the runtime cannot say.
int field_queue_slots_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(field_queue_expanded<false, kTile>), kFieldThreads,
            0) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

int field_slots_per_cu(int tpt, int precision) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (precision == GCCD_PRECISION_FP64) {
        if (tpt == 1)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void*>(field_tiles_f64<1>), kFieldThreads, 0);
        else if (tpt == 2)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void*>(field_tiles_f64<2>), kFieldThreads, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void*>(field_tiles_f64<4>), kFieldThreads, 0);
    } else if (tpt == 1 && precision == GCCD_PRECISION_DEFAULT) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(field_tiles_expanded<false, kTile>), kFieldThreads, 0);
    } else if (tpt == 1) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(field_tiles<1, GCCD_PRECISION_BLOCK>),
            kFieldThreads, 0);
    } else if (tpt == 2) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(field_tiles<2, GCCD_PRECISION_DEFAULT>),
            kFieldThreads, 0);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(field_tiles<4, GCCD_PRECISION_DEFAULT>),
            kFieldThreads, 0);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

hipError_t launch_field(const FieldArgs& a, int tpt, int precision, uint32_t n_items,
                        uint32_t queue_grid, hipStream_t s, uint32_t grid_cap) {
    if (grid_cap > 0) {
        if (tpt != 1 || precision != GCCD_PRECISION_DEFAULT || n_items > grid_cap)
            return hipErrorInvalidValue;
        FieldArgs b = a;
        b.count_items = 1;
        const bool c = b.near_compensated != 0;
        switch (b.unit) {
            case kTile / 4:
                if (c) field_tiles_expanded<true, kTile / 4><<<grid_cap, kFieldThreads, 0, s>>>(b);
                else field_tiles_expanded<false, kTile / 4><<<grid_cap, kFieldThreads, 0, s>>>(b);
                break;
            case kTile / 2:
                if (c) field_tiles_expanded<true, kTile / 2><<<grid_cap, kFieldThreads, 0, s>>>(b);
                else field_tiles_expanded<false, kTile / 2><<<grid_cap, kFieldThreads, 0, s>>>(b);
                break;
            case kTile:
                if (c) field_tiles_expanded<true, kTile><<<grid_cap, kFieldThreads, 0, s>>>(b);
                else field_tiles_expanded<false, kTile><<<grid_cap, kFieldThreads, 0, s>>>(b);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (queue_grid > 0 && tpt == 1 && precision == GCCD_PRECISION_DEFAULT) {
        // the item count is read on the device: launched even with none
        const hipError_t e = launch_fill_u32(a.queue, 1u, 0u, s);
        if (e != hipSuccess) return e;
        const bool c = a.near_compensated != 0;
        switch (a.unit) {
            case kTile / 4:
                if (c) field_queue_expanded<true, kTile / 4><<<queue_grid, kFieldThreads, 0, s>>>(a);
                else field_queue_expanded<false, kTile / 4><<<queue_grid, kFieldThreads, 0, s>>>(a);
                break;
            case kTile / 2:
                if (c) field_queue_expanded<true, kTile / 2><<<queue_grid, kFieldThreads, 0, s>>>(a);
                else field_queue_expanded<false, kTile / 2><<<queue_grid, kFieldThreads, 0, s>>>(a);
                break;
            case kTile:
                if (c) field_queue_expanded<true, kTile><<<queue_grid, kFieldThreads, 0, s>>>(a);
                else field_queue_expanded<false, kTile><<<queue_grid, kFieldThreads, 0, s>>>(a);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (n_items == 0) return hipSuccess;
    // only the one-target-per-lane default kernel takes smaller tiles
    if (a.unit != kTile && !(tpt == 1 && precision == GCCD_PRECISION_DEFAULT))
        return hipErrorInvalidValue;
    switch (precision) {
        case GCCD_PRECISION_DEFAULT:
            if (tpt == 1) {
                const bool c = a.near_compensated != 0;
                switch (a.unit) {
                    case kTile / 4:
                        if (c) field_tiles_expanded<true, kTile / 4><<<n_items, kFieldThreads, 0, s>>>(a);
                        else field_tiles_expanded<false, kTile / 4><<<n_items, kFieldThreads, 0, s>>>(a);
                        break;
                    case kTile / 2:
                        if (c) field_tiles_expanded<true, kTile / 2><<<n_items, kFieldThreads, 0, s>>>(a);
                        else field_tiles_expanded<false, kTile / 2><<<n_items, kFieldThreads, 0, s>>>(a);
                        break;
                    case kTile:
                        if (c) field_tiles_expanded<true, kTile><<<n_items, kFieldThreads, 0, s>>>(a);
                        else field_tiles_expanded<false, kTile><<<n_items, kFieldThreads, 0, s>>>(a);
                        break;
                    default: return hipErrorInvalidValue;
                }
                return hipGetLastError();
            }
            return launch_field_prec<GCCD_PRECISION_DEFAULT>(a, tpt, n_items, s);
        case GCCD_PRECISION_BLOCK:
            return launch_field_prec<GCCD_PRECISION_BLOCK>(a, tpt, n_items, s);
        case GCCD_PRECISION_EVENT:
            return launch_field_prec<GCCD_PRECISION_EVENT>(a, tpt, n_items, s);
        case GCCD_PRECISION_ABSOLUTE:
            return launch_field_prec<GCCD_PRECISION_ABSOLUTE>(a, tpt, n_items, s);
        case GCCD_PRECISION_COMPENSATED:
            return launch_field_prec<GCCD_PRECISION_COMPENSATED>(a, tpt, n_items, s);
        case GCCD_PRECISION_FP64:
            switch (tpt) {
                case 1: field_tiles_f64<1><<<n_items, kFieldThreads, 0, s>>>(a); break;
                case 2: field_tiles_f64<2><<<n_items, kFieldThreads, 0, s>>>(a); break;
                case 4: field_tiles_f64<4><<<n_items, kFieldThreads, 0, s>>>(a); break;
                default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        default: return hipErrorInvalidValue;
    }
}

static uint32_t grid_for(uint64_t n, int threads, uint32_t cap) {
    uint64_t g = (n + (uint64_t)threads - 1) / (uint64_t)threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

// ---------------------------------------------------------------------------
// The sorted list.  make_keys writes every carrier's key (carrier order);
// after the sort, count_active finds in each event's segment the first
// collected key (the segment holds its travelling holes first) and records
// the step's holes and pair interactions; gather_tiles copies the positions
// into slot order and takes the bounding box of every source tile.
// ---------------------------------------------------------------------------
__global__ void make_keys(const double* x, const double* y, const double* z,
                          const int32_t* cstep, const uint32_t* ev_of, const uint32_t* ev_off,
                          uint32_t n, KeyLayout kl, uint64_t* keys) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const uint32_t e = ev_of[j];
        keys[j] = make_key(e, cstep[j] >= 0, x[j], y[j], z[j], j - ev_off[e], kl);
    }
}

hipError_t launch_make_keys(const double* x, const double* y, const double* z,
                            const int32_t* cstep, const uint32_t* ev_of, const uint32_t* ev_off,
                            uint32_t n, KeyLayout kl, uint64_t* keys, hipStream_t s) {
    make_keys<<<grid_for(n, 256, 8192), 256, 0, s>>>(x, y, z, cstep, ev_of, ev_off, n, kl, keys);
    return hipGetLastError();
}

// The travelling holes of each event: the first collected key of its
// segment (travelling holes come first), by binary search.
constexpr int kCountThreads = 256;

__global__ __launch_bounds__(kCountThreads) void count_active(const uint64_t* keys,
                                                              const uint32_t* ev_off,
                                                              uint32_t n_events, KeyLayout kl,
                                                              uint32_t* ev_active) {
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_events;
         e += gridDim.x * blockDim.x) {
        const uint32_t off = ev_off[e], ne = ev_off[e + 1] - off;
        uint32_t lo = 0, hi = ne;  // first collected key of the segment in [lo, hi]
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (key_collected(keys[off + mid], kl))
                hi = mid;
            else
                lo = mid + 1;
        }
        ev_active[e] = lo;
    }
}

hipError_t launch_count(const uint64_t* keys, const uint32_t* ev_off, uint32_t n_events,
                        KeyLayout kl, uint32_t* ev_active, hipStream_t s) {
    count_active<<<grid_for(n_events, kCountThreads, 1024), kCountThreads, 0, s>>>(
        keys, ev_off, n_events, kl, ev_active);
    return hipGetLastError();
}

// Source tile g of event e = tile_event[g] (local tile t = g - ev_tile[e]),
// by one workgroup of kTile threads: positions of every slot of the tile
// (key_at(slot) gives the slot's key; ns_or_active is the event's travelling
// holes, the sources unless sources_all), bounding box of
// the slots that are sources (rows 0-5 of box: low x, y, z, high x, y, z),
// and the same for each 64-slot quarter of the tile (row 6 + 4 k + q for
// bound k of quarter q) and each 16-slot group (row 30 + 16 k + g), which
// the near-field kernel culls by.  The group boxes are the first four steps
// of the lane reduction that gives the quarter boxes.
template <class KeyAt>
__device__ __forceinline__ void gather_tile(uint32_t g, KeyAt key_at, const uint32_t* ev_off,
                                            const uint32_t* ev_tile, const uint32_t* tile_event,
                                            uint32_t ns_or_active, int sources_all, KeyLayout kl,
                                            const double* x, const double* y, const double* z,
                                            double* px, double* py, double* pz, double* box,
                                            uint32_t stride, double (*red)[kTile / 64]) {
    const uint32_t e = tile_event[g];
    const uint32_t t = g - ev_tile[e];
    const uint32_t off = ev_off[e], ne = ev_off[e + 1] - off;
    const uint32_t ns = sources_all ? ne : ns_or_active;
    const uint32_t i = t * kTile + threadIdx.x;
    double lx = INFINITY, ly = INFINITY, lz = INFINITY;
    double hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    if (i < ne) {
        // a slot of event e holds a key of event e; the clamp keeps every
        // load inside the event regardless
        const uint32_t c = off + min(key_local(key_at(off + i), kl), ne - 1u);
        const double vx = x[c], vy = y[c], vz = z[c];
        px[off + i] = vx;
        py[off + i] = vy;
        pz[off + i] = vz;
        if (i < ns) {
            lx = hx = vx;
            ly = hy = vy;
            lz = hz = vz;
        }
    }
    // butterfly over lanes: after the strides 1..8 every lane holds its
    // 16-slot group's box, after 16 and 32 its quarter's
#pragma unroll
    for (int m = 1; m <= 8; m <<= 1) {
        lx = fmin(lx, __shfl_xor(lx, m));
        ly = fmin(ly, __shfl_xor(ly, m));
        lz = fmin(lz, __shfl_xor(lz, m));
        hx = fmax(hx, __shfl_xor(hx, m));
        hy = fmax(hy, __shfl_xor(hy, m));
        hz = fmax(hz, __shfl_xor(hz, m));
    }
    if ((threadIdx.x & 15) == 0) {
        const int grp = threadIdx.x >> 4;  // 0 .. 15
        const double v[6] = {lx, ly, lz, hx, hy, hz};
#pragma unroll
        for (int k = 0; k < 6; ++k) box[(size_t)(30 + 16 * k + grp) * stride + g] = v[k];
    }
#pragma unroll
    for (int m = 16; m <= 32; m <<= 1) {
        lx = fmin(lx, __shfl_xor(lx, m));
        ly = fmin(ly, __shfl_xor(ly, m));
        lz = fmin(lz, __shfl_xor(lz, m));
        hx = fmax(hx, __shfl_xor(hx, m));
        hy = fmax(hy, __shfl_xor(hy, m));
        hz = fmax(hz, __shfl_xor(hz, m));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = lx;
        red[1][wave] = ly;
        red[2][wave] = lz;
        red[3][wave] = hx;
        red[4][wave] = hy;
        red[5][wave] = hz;
        const double v[6] = {lx, ly, lz, hx, hy, hz};
#pragma unroll
        for (int k = 0; k < 6; ++k) box[(size_t)(6 + 4 * k + wave) * stride + g] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = red[k][0];
        for (int w = 1; w < kTile / 64; ++w) v = (k < 3) ? fmin(v, red[k][w]) : fmax(v, red[k][w]);
        box[(size_t)k * stride + g] = v;
    }
}

__global__ __launch_bounds__(kTile) void gather_tiles(
    const uint64_t* keys, const uint32_t* ev_off, const uint32_t* ev_tile,
    const uint32_t* tile_event, const uint32_t* ev_active, int sources_all, KeyLayout kl,
    const double* x, const double* y, const double* z, double* px, double* py, double* pz,
    double* box, uint32_t stride) {
    __shared__ double red[6][kTile / 64];
    const uint32_t g = blockIdx.x;
    gather_tile(
        g, [&](uint32_t slot) { return keys[slot]; }, ev_off, ev_tile, tile_event,
        sources_all ? 0u : ev_active[tile_event[g]], sources_all, kl, x, y, z, px, py, pz, box,
        stride, red);
}

// gather_tiles and count_active in one launch, for lists whose sources are
// every hole (the gather then needs no count): tile g also finds whether the
// event's first collected key -- its travelling count, the keys of a
// segment being ordered travelling before collected -- lies in its slots.
// Exactly one workgroup writes each event's count: the one whose tile holds
// the first collected key (the slot before the tile travelling, or the tile
// first in its event), or the event's last tile if no key is collected;
// workgroup 0 writes 0 for the events with no holes (and no tiles).
__global__ __launch_bounds__(kTile) void gather_count_tiles(
    const uint64_t* keys, const uint32_t* ev_off, const uint32_t* ev_tile,
    const uint32_t* tile_event, uint32_t n_events, KeyLayout kl, const double* x,
    const double* y, const double* z, double* px, double* py, double* pz, double* box,
    uint32_t stride, uint32_t* ev_active) {
    __shared__ double red[6][kTile / 64];
    __shared__ uint32_t first_col[kTile / 64];
    const uint32_t g = blockIdx.x;
    if (g == 0) {
        for (uint32_t e = threadIdx.x; e < n_events; e += kTile)
            if (ev_off[e + 1] == ev_off[e]) ev_active[e] = 0u;
    }
    gather_tile(
        g, [&](uint32_t slot) { return keys[slot]; }, ev_off, ev_tile, tile_event, 0u, 1, kl,
        x, y, z, px, py, pz, box, stride, red);
    const uint32_t e = tile_event[g];
    const uint32_t t0 = (g - ev_tile[e]) * kTile;
    const uint32_t off = ev_off[e], ne = ev_off[e + 1] - off;
    const uint32_t i = t0 + threadIdx.x;
    const bool col = i < ne && key_collected(keys[off + i], kl);
    const uint64_t bal = __ballot(col);
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0)
        first_col[wave] = bal ? wave * 64u + (uint32_t)__builtin_ctzll(bal) : (uint32_t)kTile;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t p = (uint32_t)kTile;  // first collected slot of the tile, from its start
        for (uint32_t w = 0; w < kTile / 64; ++w) p = min(p, first_col[w]);
        if (p < (uint32_t)kTile) {
            if (t0 == 0u || !key_collected(keys[off + t0 - 1u], kl)) ev_active[e] = t0 + p;
        } else if (t0 + (uint32_t)kTile >= ne) {
            ev_active[e] = ne;  // the event's last tile, and no key collected
        }
    }
}

hipError_t launch_gather_count(const uint64_t* keys, const uint32_t* ev_off,
                               const uint32_t* ev_tile, const uint32_t* tile_event,
                               uint32_t n_events, uint32_t n_tiles, KeyLayout kl, const double* x,
                               const double* y, const double* z, double* px, double* py,
                               double* pz, double* box, uint32_t stride, uint32_t* ev_active,
                               hipStream_t s) {
    if (n_tiles == 0) return launch_count(keys, ev_off, n_events, kl, ev_active, s);
    gather_count_tiles<<<n_tiles, kTile, 0, s>>>(keys, ev_off, ev_tile, tile_event, n_events, kl,
                                                 x, y, z, px, py, pz, box, stride, ev_active);
    return hipGetLastError();
}

hipError_t launch_gather(const uint64_t* keys, const uint32_t* ev_off, const uint32_t* ev_tile,
                         const uint32_t* tile_event, const uint32_t* ev_active, int sources_all,
                         uint32_t n_tiles, KeyLayout kl, const double* x, const double* y,
                         const double* z, double* px, double* py, double* pz, double* box,
                         uint32_t stride, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    gather_tiles<<<n_tiles, kTile, 0, s>>>(keys, ev_off, ev_tile, tile_event, ev_active,
                                           sources_all, kl, x, y, z, px, py, pz, box, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Random diffusion vectors: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// ten rounds of two 32x32->64 multiplies whose high halves are XORed into the
// other words together with the round key; the key advances by two Weyl
// constants between rounds.  Counter = (carrier within its event, step,
// event, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply-add instruction gives both halves
        const uint64_t pA = (uint64_t)kMulA * c0, pB = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pB >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pA >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)pB;
        c2 = n2;
        c3 = (uint32_t)pA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
}

__device__ __forceinline__ double unit_open(uint32_t w) {
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

// ---------------------------------------------------------------------------
// One time step for every travelling hole (Sec. III.B, Fig. 2): static field
// (Eq. (1)) + Coulomb field (the chunk partials of field_tiles, summed in
// FP64 in chunk order), |E|, mobility (Eq. (2)), drift mu E dt, diffusion
// (Eqs. (3)-(4), Box-Muller on one Philox block), FP64 position update,
// mirror at the back surface, collection at the well.
//   list mode (Coulomb on): one thread per slot of the sorted list; every
//     carrier keeps its slot in the next (unsorted) list with its new key,
//     collected holes copying theirs through; the next sort restores order.
//   carrier mode: one thread per carrier; travelling holes are counted, one
//     atomic per wave.
// ---------------------------------------------------------------------------
// The list of a load of at most kFusedList carriers in at most kFusedTiles
// source tiles, rebuilt by the last workgroup of its step: the new keys,
// which each workgroup of the step left as a sorted run of its slots
// (sort_block_keys), merged in LDS (merge_sorted_runs), each event's
// travelling holes (its first collected key, by binary search in LDS), and
// the positions and boxes of every source tile in slot order -- the same
// list, counts, slots and boxes as sort_keys, count_active and
// gather_tiles.  The positions are gathered four slots per thread with all
// their loads in flight and kept in LDS; the boxes are then reduced by one
// thread per 16-slot group, per 64-slot quarter and per tile.
__device__ __forceinline__ void build_small_list(const StepArgs& a) {
    __shared__ uint64_t s[kFusedList + kFusedList / kSortItems];
    __shared__ uint32_t act[kFusedList];
    const uint32_t n = a.n_all;
    // the step's workgroups left sorted runs of kStepThreads keys
    if (n <= (uint32_t)kFusedList / 2)
        merge_sorted_runs<kFusedList / 2 / kSortItems>(a.keys_out, n, s, kStepThreads);
    else
        merge_sorted_runs<kFusedList / kSortItems>(a.keys_out, n, s, kStepThreads);
    for (uint32_t i = threadIdx.x; i < n; i += kStepThreads) a.keys_sorted[i] = s[lds_slot(i)];
    for (uint32_t e = threadIdx.x; e < a.n_events; e += kStepThreads) {
        const uint32_t off = a.one_event ? 0u : a.ev_off[e];
        const uint32_t ne = a.one_event ? n : a.ev_off[e + 1] - off;
        uint32_t lo = 0, hi = ne;  // first collected key of the segment in [lo, hi]
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (key_collected(s[lds_slot(off + mid)], a.kl))
                hi = mid;
            else
                lo = mid + 1;
        }
        act[e] = lo;
        a.ev_active_out[e] = lo;
    }
    __syncthreads();
    // positions of every tile slot (tile g, slot w at g kTile + w), gathered
    // four per thread with all loads in flight, kept in LDS with a flag for
    // the slots that are sources
    __shared__ double gp[3][kFusedTiles * kTile];
    __shared__ uint8_t gsrc[kFusedTiles * kTile];
    __shared__ double gbox[kFusedTiles * (kTile / 16)][6];
    const uint32_t nq = a.n_tiles * (uint32_t)kTile;
    constexpr uint32_t kBatch = 4;
    for (uint32_t q0 = threadIdx.x; q0 < nq; q0 += kBatch * kStepThreads) {
        double v[kBatch][3];
        bool src[kBatch], in[kBatch];
        uint32_t dst[kBatch];
#pragma unroll
        for (uint32_t b = 0; b < kBatch; ++b) {
            const uint32_t q = q0 + b * kStepThreads;
            v[b][0] = v[b][1] = v[b][2] = 0.0;
            src[b] = in[b] = false;
            dst[b] = 0;
            if (q < nq) {
                const uint32_t g = q / kTile, w = q % kTile;
                // a single event's tiles start at slot 0 (no lookups)
                const uint32_t e = a.one_event ? 0u : a.tile_event[g];
                const uint32_t off = a.one_event ? 0u : a.ev_off[e];
                const uint32_t ne = a.one_event ? n : a.ev_off[e + 1] - off;
                const uint32_t ns = a.sources_all ? ne : act[e];
                const uint32_t i = (a.one_event ? g : g - a.ev_tile[e]) * kTile + w;
                if (i < ne) {
                    const uint32_t c = off + min(key_local(s[lds_slot(off + i)], a.kl), ne - 1u);
                    v[b][0] = a.x[c];
                    v[b][1] = a.y[c];
                    v[b][2] = a.z[c];
                    in[b] = true;
                    src[b] = i < ns;
                    dst[b] = off + i;
                }
            }
        }
#pragma unroll
        for (uint32_t b = 0; b < kBatch; ++b) {
            const uint32_t q = q0 + b * kStepThreads;
            if (q >= nq) break;
            if (in[b]) {
                a.px[dst[b]] = v[b][0];
                a.py[dst[b]] = v[b][1];
                a.pz[dst[b]] = v[b][2];
            }
            gp[0][q] = v[b][0];
            gp[1][q] = v[b][1];
            gp[2][q] = v[b][2];
            gsrc[q] = src[b] ? 1 : 0;
        }
    }
    __syncthreads();
    // the boxes of the sources: one thread per 16-slot group, then one per
    // 64-slot quarter (four groups), then one per tile (four quarters)
    const size_t st = a.box_stride;
    const uint32_t ng = a.n_tiles * (uint32_t)(kTile / 16);
    for (uint32_t t = threadIdx.x; t < ng; t += kStepThreads) {
        double b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll 4
        for (uint32_t w = t * 16u; w < t * 16u + 16u; ++w) {
            if (!gsrc[w]) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                b[k] = fmin(b[k], gp[k][w]);
                b[3 + k] = fmax(b[3 + k], gp[k][w]);
            }
        }
        const uint32_t g = t / (kTile / 16), grp = t % (kTile / 16);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            gbox[t][k] = b[k];
            a.tile_box[(size_t)(30 + 16 * k + grp) * st + g] = b[k];
        }
    }
    __syncthreads();
    __shared__ double qbox[kFusedTiles * 4][6];
    for (uint32_t t = threadIdx.x; t < a.n_tiles * 4u; t += kStepThreads) {
        const uint32_t g = t / 4u, qw = t % 4u;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double m = gbox[t * 4u][k];
#pragma unroll
            for (uint32_t j = 1; j < 4; ++j)
                m = k < 3 ? fmin(m, gbox[t * 4u + j][k]) : fmax(m, gbox[t * 4u + j][k]);
            qbox[t][k] = m;
            a.tile_box[(size_t)(6 + 4 * k + qw) * st + g] = m;
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < a.n_tiles; t += kStepThreads) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double m = qbox[t * 4u][k];
#pragma unroll
            for (uint32_t j = 1; j < 4; ++j)
                m = k < 3 ? fmin(m, qbox[t * 4u + j][k]) : fmax(m, qbox[t * 4u + j][k]);
            a.tile_box[(size_t)k * st + t] = m;
        }
    }
}

// The FP64 functions of the step (gccd_fp64.h).  Carrier mode (no
// repulsion) is bound by VALU issue and takes the three-operand Horner steps
// (one instruction fewer per step, at the cost of registers); list mode,
// which streams the partial sums, the compiler's own form, which needs
// fewer registers.
template <bool LIST>
__device__ __forceinline__ double exp_fin_s(double x) {
    return fp64::exp_fin<!LIST>(x);
}
template <bool LIST>
__device__ __forceinline__ double log_pos_s(double x) {
    return fp64::log_pos<!LIST>(x);
}
template <bool LIST>
__device__ __forceinline__ double log1p_fin_s(double x) {
    return fp64::log1p_fin<!LIST>(x);
}
template <bool LIST>
__device__ __forceinline__ void sincospi_s(double x, double* s, double* c) {
    fp64::sincospi<!LIST>(x, s, c);
}

// LIST: list mode (a.list_mode, Coulomb on); carrier mode is a kernel of
// its own (drift_update), without the list code, for the step without
// repulsion.
template <bool FUSE, bool LIST>
__device__ __forceinline__ void step_body(const StepArgs& a) {
    const uint32_t step = a.step + (a.step_base ? *a.step_base : 0u);
    // travelling holes at the start of this step, of the next one, and the
    // counter of the step after next (cleared now; nobody reads it)
    const uint32_t* cnt_in = a.cnt_ring + step % 3u;
    uint32_t* cnt_out = a.cnt_ring + (step + 1u) % 3u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long holes = *cnt_in;
        a.cnt_ring[(step + 2u) % 3u] = 0u;
        if (holes > 0) {
            atomicAdd(&a.stats[0], holes);
            a.misc[1] = (int32_t)(step + 1u);
        }
    }
    const int lane = threadIdx.x & 63;
    uint32_t kept = 0;  // this wave's holes still travelling (wave-uniform)
    unsigned long long pairs = 0;  // this lane's pair interactions of Eq. (6)
    // FUSE, or a.sort_runs: each turn's kStepThreads slots leave their new
    // keys as one sorted run (sort_block_keys), which the next sort only
    // merges; else every slot leaves its key in place
    const bool runs = FUSE || (LIST && a.sort_runs != 0);
    __shared__ uint64_t sk[kStepThreads];
    for (uint32_t base = blockIdx.x * kStepThreads; base < a.n_all;
         base += gridDim.x * kStepThreads) {
        const uint32_t slot = base + threadIdx.x;
        uint64_t run_key = ~0ull;  // this slot's new key, when the keys form runs
        bool keep = false;
        if (slot < a.n_all) {
            uint32_t e, j, local, src = 0u;
            bool active;
            uint64_t key = 0;
            if (LIST) {
                // the list may be one step old (its travelling segment then
                // still holds the holes collected in the last step): the
                // carrier's own collection step decides
                key = a.keys_in[slot];
                uint32_t off, ne;
                if (a.one_event) {
                    e = 0u;
                    off = 0u;
                    ne = a.n_all;
                } else {
                    e = key_event(key, a.kl);
                    off = a.ev_off[e];
                    ne = a.ev_off[e + 1] - off;
                }
                local = min(key_local(key, a.kl), ne - 1u);
                j = off + local;
                active = a.cstep[j] < 0;
                if (active) {
                    src = a.sources_all ? ne : a.ev_active[e];
                } else if (a.close && slot - off < a.ev_active[e]) {
                    // a target of the field launch collected in the last step:
                    // its close-pair sums are not consumed, so cleared here
                    const size_t ps = a.pstride;
                    a.close[slot] = 0ull;
                    a.close[slot + ps] = 0ull;
                    a.close[slot + 2 * ps] = 0ull;
                }
            } else {
                j = slot;
                if (a.one_event) {
                    e = 0u;
                    local = j;
                } else {
                    e = a.ev_of[j];
                    local = j - a.ev_off[e];
                }
                active = a.cstep[j] < 0;
            }
            if (active) {
                pairs += src;  // sources of the Eq. (6) sum at this target
                double ecx = 0.0, ecy = 0.0, ecz = 0.0;
                if (LIST && a.coulomb) {
                    double sx = 0.0, sy = 0.0, sz = 0.0;
                    const int nchunk = a.ev_chunks[e];
                    const float* pp = a.part + slot;
                    const size_t ps = a.pstride;
                    int c = 0;
                    // eight (a small load, latency-bound: sixteen), then four
                    // groups' loads in flight ahead of their adds (the adds in
                    // group order)
                    constexpr int kW = FUSE ? 16 : 8;
                    for (; c + kW <= nchunk; c += kW) {
                        float v[kW][3];
#pragma unroll
                        for (int u = 0; u < kW; ++u)
#pragma unroll
                            for (int d = 0; d < 3; ++d) v[u][d] = pp[(size_t)((c + u) * 3 + d) * ps];
#pragma unroll
                        for (int u = 0; u < kW; ++u) {
                            sx += (double)v[u][0];
                            sy += (double)v[u][1];
                            sz += (double)v[u][2];
                        }
                    }
                    if (FUSE && c + 8 <= nchunk) {
                        float v[8][3];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
#pragma unroll
                            for (int d = 0; d < 3; ++d) v[u][d] = pp[(size_t)((c + u) * 3 + d) * ps];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            sx += (double)v[u][0];
                            sy += (double)v[u][1];
                            sz += (double)v[u][2];
                        }
                        c += 8;
                    }
                    for (; c + 4 <= nchunk; c += 4) {
                        float v[4][3];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int d = 0; d < 3; ++d) v[u][d] = pp[(size_t)((c + u) * 3 + d) * ps];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            sx += (double)v[u][0];
                            sy += (double)v[u][1];
                            sz += (double)v[u][2];
                        }
                    }
                    for (; c < nchunk; ++c) {
                        sx += (double)pp[(size_t)(c * 3 + 0) * ps];
                        sy += (double)pp[(size_t)(c * 3 + 1) * ps];
                        sz += (double)pp[(size_t)(c * 3 + 2) * ps];
                    }
                    if (a.close) {
                        // the exactly summed close pairs, cleared for the next launch
                        unsigned long long* cp = a.close + slot;
                        const long long cx = (long long)cp[0], cy = (long long)cp[ps],
                                        cz = (long long)cp[2 * ps];
                        if ((cx | cy | cz) != 0ll) {
                            sx += (double)cx * a.close_unit;
                            sy += (double)cy * a.close_unit;
                            sz += (double)cz * a.close_unit;
                            cp[0] = 0ull;
                            cp[ps] = 0ull;
                            cp[2 * ps] = 0ull;
                        }
                    }
                    ecx = a.K * sx;
                    ecy = a.K * sy;
                    ecz = a.K * sz;
                }
                const double x0 = a.x[j], y0 = a.y[j], z0 = a.z[j];
                const double es = a.a1 * z0 - a.a2;
                const double ex = ecx, ey = ecy, ez = LIST ? ecz + es : es;
                double mu = a.mu0;
                if (a.mobility_model == 0) {
                    // Eq. (2), mu0 / (1 + (|E|/Ec)^beta)^(1/beta), as
                    // mu0 exp(-log1p(y) / beta) with y = exp(beta (log|E|^2 / 2
                    // - log Ec)): four transcendentals instead of two general
                    // powers and a square root.  The arguments are held in the
                    // functions' finite ranges, so no special case is tested:
                    // |E|^2 at or above 2^-1000 (|E| = 0 then gives a y far
                    // below the rounding of 1 + y, so mu = mu0 exactly, as
                    // y = 0 would), the exponents within [-745, 709]
                    const double e2 = fmax(ex * ex + ey * ey + ez * ez, 0x1p-1000);
                    const double ly = a.beta * (0.5 * log_pos_s<LIST>(e2) - a.log_ec);
                    const double y = exp_fin_s<LIST>(fmin(fmax(ly, -745.0), 709.0));
                    mu = a.mu0 * exp_fin_s<LIST>(fmax(-a.inv_beta * log1p_fin_s<LIST>(y), -745.0));
                }
                // v = mu E in cm/s; v dt in cm; 1 cm = 1e4 um.  Without
                // repulsion the field is the static one, along z only: no
                // lateral drift (mu 0 dt = +0 exactly)
                double dx = LIST ? mu * ex * a.dt_s * 1e4 : 0.0;
                double dy = LIST ? mu * ey * a.dt_s * 1e4 : 0.0;
                double dz = mu * ez * a.dt_s * 1e4;
                if (a.diffusion) {
                    uint32_t w0 = local, w1 = step, w2 = a.event0 + e, w3 = 0u;
                    philox4x32_10(w0, w1, w2, w3, a.key0, a.key1);
                    // -2 ln u > 2^-33 for u on the open grid (w + 1/2) 2^-32
                    const double r01 = fp64::sqrt_pos(-2.0 * log_pos_s<LIST>(unit_open(w0)));
                    const double r23 = fp64::sqrt_pos(-2.0 * log_pos_s<LIST>(unit_open(w2)));
                    // the angles 2 pi u in half-turns: 2 u is exact, and one
                    // argument reduction serves both sine and cosine
                    double s1, c1, s3, c3;
                    sincospi_s<LIST>(2.0 * unit_open(w1), &s1, &c1);
                    sincospi_s<LIST>(2.0 * unit_open(w3), &s3, &c3);
                    (void)s3;
                    const double D = a.vt * mu;                        // Eq. (4), cm^2/s
                    // Eq. (3), um; 2 D dt > 0 (T > 0, dt > 0), held at or
                    // above 2^-1000 so that the square root's estimate stays
                    // in range even for a dt that underflows it
                    const double s2 = fmax(2.0 * D * a.dt_s, 0x1p-1000);
                    const double sigma = fp64::sqrt_pos(s2) * 1e4;
                    dx += sigma * (r01 * c1);
                    dy += sigma * (r01 * s1);
                    dz += sigma * (r23 * c3);
                }
                const double xn = x0 + dx, yn = y0 + dy;
                double zn = z0 + dz;
                if (zn > a.thickness) zn = 2.0 * a.thickness - zn;
                a.x[j] = xn;
                a.y[j] = yn;
                a.z[j] = zn;
                if (!isfinite(xn) || !isfinite(yn) || !isfinite(zn)) atomicOr(&a.misc[0], 1);
                const bool collected = zn <= a.z_well;
                if (collected) a.cstep[j] = (int32_t)(step + 1u);
                keep = !collected;
                if (LIST) key = make_key(e, collected, xn, yn, zn, local, a.kl);
            }
            if (runs)
                run_key = key;
            else if (LIST)
                a.keys_out[slot] = key;
        }
        kept += (uint32_t)__popcll(__ballot(keep));
        if (runs) {  // uniform: every thread of the workgroup takes each turn
            const uint32_t m = min((uint32_t)kStepThreads, a.n_all - base);
            const uint64_t sorted = sort_block_keys(run_key, m, sk);
            if (threadIdx.x < m) a.keys_out[base + threadIdx.x] = sorted;
        }
    }
    // one atomic per workgroup for each count: a counter taking one per wave
    // and grid-stride turn (2.6e5 at 2^24 holes) serialised the whole step
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) pairs += __shfl_xor(pairs, m);
    __shared__ uint32_t wave_kept[kStepThreads / 64];
    __shared__ unsigned long long wave_pairs[kStepThreads / 64];
    if (lane == 0) {
        wave_kept[threadIdx.x >> 6] = kept;
        wave_pairs[threadIdx.x >> 6] = pairs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        unsigned long long pr = 0;
        for (int w = 0; w < kStepThreads / 64; ++w) {
            t += wave_kept[w];
            pr += wave_pairs[w];
        }
        if (t) atomicAdd(cnt_out, t);
        if (pr && a.coulomb) atomicAdd(&a.stats[1], pr);
    }
    if constexpr (FUSE) {
        // the last workgroup to arrive rebuilds the list (merging the runs
        // the workgroups left): each thread's
        // stores of the step are made visible at device scope before its
        // workgroup arrives, and the last one sees every workgroup's
        __shared__ uint32_t last;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(a.arrive, 1u) == gridDim.x - 1u ? 1u : 0u;
        __syncthreads();
        if (last) {
            __threadfence();
            if (threadIdx.x == 0) atomicExch(a.arrive, 0u);  // zero for the next launch
            build_small_list(a);
        }
    }
}

template <bool FUSE>
__global__ __launch_bounds__(kStepThreads) void step_update(StepArgs a) {
    step_body<FUSE, true>(a);
}

__global__ __launch_bounds__(kStepThreads) void drift_update(StepArgs a) {
    step_body<false, false>(a);
}

hipError_t launch_step(const StepArgs& a, uint32_t n_slots, hipStream_t s) {
    if (a.arrive) {
        // the rebuilt list needs every slot and tile in one workgroup's LDS
        if (!a.list_mode || n_slots != a.n_all || n_slots > (uint32_t)kFusedList ||
            a.n_tiles > (uint32_t)kFusedTiles)
            return hipErrorInvalidValue;
        // one slot per thread: workgroup b's keys are slots [b, b + 1) kStepThreads
        step_update<true><<<(n_slots + kStepThreads - 1) / kStepThreads, kStepThreads, 0, s>>>(a);
    } else if (a.list_mode) {
        step_update<false><<<grid_for(n_slots, kStepThreads, 16384), kStepThreads, 0, s>>>(a);
    } else {
        drift_update<<<grid_for(n_slots, kStepThreads, 16384), kStepThreads, 0, s>>>(a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Load-time boundary handling: mirror z beyond the back surface, collect
// holes at or below the well (collection step 0), record each carrier's
// event, count the travelling ones.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kStepThreads) void load_prepare(double* z, int32_t* cstep,
                                                             const uint32_t* ev_off,
                                                             uint32_t* ev_of, uint32_t n_events,
                                                             uint32_t n, double thickness,
                                                             double z_well, uint32_t* cnt) {
    const int lane = threadIdx.x & 63;
    uint32_t kept = 0;  // this wave's travelling holes (wave-uniform)
    for (uint32_t base = blockIdx.x * kStepThreads; base < n; base += gridDim.x * kStepThreads) {
        const uint32_t j = base + threadIdx.x;
        bool keep = false;
        if (j < n) {
            double zz = z[j];
            if (zz > thickness) zz = 2.0 * thickness - zz;
            z[j] = zz;
            const bool collected = zz <= z_well;
            cstep[j] = collected ? 0 : -1;
            keep = !collected;
            ev_of[j] = event_of(ev_off, n_events, j);
        }
        kept += (uint32_t)__popcll(__ballot(keep));
    }
    // one atomic per workgroup, as in step_update
    __shared__ uint32_t wave_kept[kStepThreads / 64];
    if (lane == 0) wave_kept[threadIdx.x >> 6] = kept;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kStepThreads / 64; ++w) t += wave_kept[w];
        if (t) atomicAdd(cnt, t);
    }
}

hipError_t launch_load(double* z, int32_t* cstep, const uint32_t* ev_off, uint32_t* ev_of,
                       uint32_t n_events, uint32_t n, double thickness, double z_well,
                       uint32_t* cnt, hipStream_t s) {
    load_prepare<<<grid_for(n, kStepThreads, 8192), kStepThreads, 0, s>>>(
        z, cstep, ev_off, ev_of, n_events, n, thickness, z_well, cnt);
    return hipGetLastError();
}

__global__ void fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    fill_u32<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// Coulomb field of every carrier for gccd_field: chunk partials summed in
// FP64 in chunk order, times K (same reduction as step_update), written back
// to the carrier each slot holds.
__global__ void field_finish(const float* part, uint32_t pstride, const int32_t* ev_chunks,
                             int g0, int groups, const uint64_t* keys, const uint32_t* ev_off,
                             KeyLayout kl, uint32_t n, double K, unsigned long long* close,
                             double close_unit, double* ex, double* ey, double* ez) {
    for (uint32_t slot = blockIdx.x * blockDim.x + threadIdx.x; slot < n;
         slot += gridDim.x * blockDim.x) {
        const uint64_t key = keys[slot];
        const uint32_t e = key_event(key, kl);
        const uint32_t off = ev_off[e], ne = ev_off[e + 1] - off;
        const uint32_t j = off + min(key_local(key, kl), ne - 1u);
        double sx = 0.0, sy = 0.0, sz = 0.0;
        const int g1 = g0 + (groups > 0 ? groups : ev_chunks[e]);
        for (int c = g0; c < g1; ++c) {
            sx += (double)part[(size_t)(c * 3 + 0) * pstride + slot];
            sy += (double)part[(size_t)(c * 3 + 1) * pstride + slot];
            sz += (double)part[(size_t)(c * 3 + 2) * pstride + slot];
        }
        if (close) {
            unsigned long long* cp = close + slot;
            const long long cx = (long long)cp[0], cy = (long long)cp[pstride],
                            cz = (long long)cp[2 * (size_t)pstride];
            if ((cx | cy | cz) != 0ll) {
                sx += (double)cx * close_unit;
                sy += (double)cy * close_unit;
                sz += (double)cz * close_unit;
                cp[0] = 0ull;
                cp[pstride] = 0ull;
                cp[2 * (size_t)pstride] = 0ull;
            }
        }
        ex[j] = K * sx;
        ey[j] = K * sy;
        ez[j] = K * sz;
    }
}

hipError_t launch_field_finish(const float* part, uint32_t pstride, const int32_t* ev_chunks,
                               int g0, int groups, const uint64_t* keys, const uint32_t* ev_off,
                               KeyLayout kl, uint32_t n, double K, unsigned long long* close,
                               double close_unit, double* ex, double* ey, double* ez,
                               hipStream_t s) {
    field_finish<<<grid_for(n, 256, 8192), 256, 0, s>>>(part, pstride, ev_chunks, g0, groups, keys,
                                                         ev_off, kl, n, K, close, close_unit, ex,
                                                         ey, ez);
    return hipGetLastError();
}

// The per-call state of gccd_field_noalloc (one event of n holes, t tiles,
// `blocks` target blocks, g chunks of which the last `tail` form the tail
// layer from tile `split`), written in its scratch memory: event tables,
// zeroed counters and close-pair sums, and the work items in the order the
// context's item builder lists them for one event.
__global__ void noalloc_setup(uint32_t n, uint32_t tiles, int32_t g, int32_t tail, uint32_t split,
                              uint32_t blocks, uint32_t* ev_off, uint32_t* ev_tile,
                              int32_t* ev_chunks, uint32_t* tile_event, uint32_t* words,
                              uint32_t n_words, FieldItem* items, unsigned long long* close) {
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (i0 == 0) {
        ev_off[0] = 0u;
        ev_off[1] = n;
        ev_tile[0] = 0u;
        ev_tile[1] = tiles;
        ev_chunks[0] = g;
    }
    for (uint64_t i = i0; i < n_words; i += stride) words[i] = 0u;
    for (uint64_t i = i0; i < tiles; i += stride) tile_event[i] = 0u;
    for (uint64_t i = i0; i < 3ull * n; i += stride) close[i] = 0ull;
    const uint32_t s1 = (uint32_t)(g - tail), s2 = (uint32_t)tail;
    const uint64_t first = (uint64_t)blocks * s1, total = first + (uint64_t)blocks * s2;
    for (uint64_t k = i0; k < total; k += stride) {
        FieldItem it;
        it.event = 0u;
        it.groups = (uint32_t)g;
        it.pad = 0u;
        if (k < first) {
            const uint32_t b = (uint32_t)(k / s1), q = (uint32_t)((k % s1 + b) % s1);
            it.blk = b;
            it.group = q;
            it.first = q;
            it.end = s2 ? split : kTilesToEnd;
            it.step = s1;
        } else {
            const uint64_t kk = k - first;
            const uint32_t b = (uint32_t)(kk / s2), q = (uint32_t)((kk % s2 + b) % s2);
            it.blk = b;
            it.group = s1 + q;
            it.first = split + q;
            it.end = kTilesToEnd;
            it.step = s2;
        }
        items[k] = it;
    }
}

hipError_t launch_noalloc_setup(uint32_t n, uint32_t tiles, int32_t g, int32_t tail,
                                uint32_t split, uint32_t blocks, uint32_t* ev_off,
                                uint32_t* ev_tile, int32_t* ev_chunks, uint32_t* tile_event,
                                uint32_t* words, uint32_t n_words, FieldItem* items,
                                unsigned long long* close, hipStream_t s) {
    noalloc_setup<<<grid_for(3ull * n, 256, 1024), 256, 0, s>>>(
        n, tiles, g, tail, split, blocks, ev_off, ev_tile, ev_chunks, tile_event, words, n_words,
        items, close);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sec. V.A image: half-open pixels, index floor((x - x0) / pitch) in IEEE
// FP64 (correctly rounded division), integer atomics into the caller's grid:
// one grid for all events, or one per event (per_event).
// ---------------------------------------------------------------------------
__global__ void image_bin(const double* x, const double* y, const int32_t* cstep,
                          const uint32_t* ev_of, uint32_t n, int per_event, double x0, double y0,
                          double pitch, int32_t nx, int32_t ny, uint32_t* counts,
                          unsigned long long* n_out) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        if (cstep[j] < 0) continue;
        const uint64_t e = per_event ? (uint64_t)ev_of[j] : 0ull;
        const double fx = floor((x[j] - x0) / pitch);
        const double fy = floor((y[j] - y0) / pitch);
        if (fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny) {
            atomicAdd(&counts[e * (uint64_t)nx * (uint64_t)ny + (uint64_t)fy * nx + (uint64_t)fx],
                      1u);
        } else {
            atomicAdd(&n_out[e], 1ull);
        }
    }
}

hipError_t launch_image(const double* x, const double* y, const int32_t* cstep,
                        const uint32_t* ev_of, uint32_t n, int per_event, double x0, double y0,
                        double pitch, int32_t nx, int32_t ny, uint32_t* counts,
                        unsigned long long* n_out, hipStream_t s) {
    image_bin<<<grid_for(n, 256, 8192), 256, 0, s>>>(x, y, cstep, ev_of, n, per_event, x0, y0,
                                                      pitch, nx, ny, counts, n_out);
    return hipGetLastError();
}

}  // namespace gccd
