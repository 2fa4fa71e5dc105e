// Sorting of the 64-bit carrier keys that order the Eq. (6) targets
// spatially (the keys are unique, so every correct sort gives the same
// list).  A merge sort written for this list:
//   block_sort  -- each workgroup sorts a tile of up to kSortTile keys
//                  (register sorts of kSortItems keys, then merge levels in
//                  LDS), giving sorted runs of kSortTile (a list that fits
//                  one tile is sorted by one workgroup sized to it);
//   merge_runs  -- one launch per level doubles the run length: each
//                  workgroup writes kSortTile consecutive outputs of one
//                  merged pair of runs, locating its share of both runs by a
//                  64-way search (one wave per end of its output range) and
//                  merging it out of LDS, kSortItems outputs per thread.
// A list of up to kSortTile keys takes one launch; 1e5 keys take one plus
// five levels.  The kernels only read and write the two key buffers (no
// memory-set commands, no temporary storage, no host synchronisation), so a
// sequence of steps that sorts can be captured in a HIP graph.
#include "gccd_sort_dev.h"

namespace gccd {

constexpr int kSortThreads = 512;
constexpr uint32_t kSortTile = kSortThreads * kSortItems;  // 4096

// One tile of T = THREADS * kSortItems keys per workgroup, sorted in LDS
// (block_sort_lds; with run0 > 0 the tile's runs of run0 keys are already
// sorted and only merged, merge_sorted_runs); loads and stores of global
// memory are coalesced.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void block_sort(const uint64_t* in, uint64_t* out,
                                                      uint32_t n, uint32_t run0) {
    constexpr uint32_t T = (uint32_t)THREADS * kSortItems;
    __shared__ uint64_t s[T + T / kSortItems];
    const uint32_t b0 = blockIdx.x * T;
    const uint32_t cnt = min(T, n - b0);
    if (run0 != 0u)
        merge_sorted_runs<THREADS>(in + b0, cnt, s, min(run0, T));
    else
        block_sort_lds<THREADS>(in + b0, cnt, s);
    for (uint32_t i = threadIdx.x; i < cnt; i += THREADS) out[b0 + i] = s[lds_slot(i)];
}

// Of the first k outputs of merging A[0, la) and B[0, lb) (sorted, no key in
// both), the number taken from A: the least i in [max(0, k - lb), min(k, la)]
// with i == min(k, la) or A[i] > B[k - 1 - i].  Every lane of the wave calls
// it with the same arguments and gets the same answer; each round tests 64
// candidates (two loads per lane) and keeps the interval between the last
// that fails and the first that holds.
__device__ uint32_t merge_split(const uint64_t* A, uint32_t la, const uint64_t* B, uint32_t lb,
                                uint32_t k) {
    uint32_t lo = k > lb ? k - lb : 0u;
    uint32_t hi = min(k, la);
    const uint32_t lane = threadIdx.x & 63u;
    while (hi > lo) {
        const uint32_t span = hi - lo;
        uint32_t m;
        bool valid;
        if (span <= 64u) {
            m = lo + lane;
            valid = lane < span;
        } else {
            m = lo + (uint32_t)(((uint64_t)span * (lane + 1u)) / 65u);
            valid = true;
        }
        // m < hi <= la and k - 1 - m < lb for every valid candidate
        const bool holds = valid && A[m] > B[k - 1u - m];
        const uint64_t bal = __ballot(holds);
        if (span <= 64u) {
            lo = bal ? lo + (uint32_t)__builtin_ctzll(bal) : hi;
            break;
        }
        const uint32_t f = bal ? (uint32_t)__builtin_ctzll(bal) : 64u;
        const uint32_t mf = __shfl(m, (int)min(f, 63u));
        const uint32_t mb = __shfl(m, (int)(f > 0u ? f - 1u : 0u));
        if (f < 64u) hi = mf;
        if (f > 0u) lo = mb + 1u;
    }
    return lo;
}

// One merge level: runs of width w in `in` become runs of 2 w in `out`.
__global__ __launch_bounds__(kSortThreads) void merge_runs(const uint64_t* in, uint64_t* out,
                                                          uint32_t n, uint32_t w) {
    __shared__ uint64_t buf[kSortTile + kSortTile / kSortItems];
    __shared__ uint32_t cut[2];
    const uint64_t o0 = (uint64_t)blockIdx.x * kSortTile;  // first output of the workgroup
    const uint64_t base = o0 / (2ull * w) * (2ull * w);    // its pair of runs starts here
    const uint32_t la = (uint32_t)min<uint64_t>(w, n - base);
    const uint32_t lb = n - base > w ? (uint32_t)min<uint64_t>(w, n - base - w) : 0u;
    const uint64_t* A = in + base;
    const uint64_t* B = A + la;
    const uint32_t k0 = (uint32_t)(o0 - base);
    const uint32_t k1 = min(k0 + kSortTile, la + lb);
    const uint32_t wave = threadIdx.x >> 6;
    if (wave < 2) {
        const uint32_t k = wave == 0 ? k0 : k1;
        const uint32_t i = merge_split(A, la, B, lb, k);
        if ((threadIdx.x & 63u) == 0) cut[wave] = i;
    }
    __syncthreads();
    const uint32_t i0 = cut[0], i1 = cut[1];
    const uint32_t na = i1 - i0, nb = (k1 - i1) - (k0 - i0);
    for (uint32_t t = threadIdx.x; t < na + nb; t += kSortThreads)
        buf[t] = t < na ? A[i0 + t] : B[k0 - i0 + (t - na)];
    __syncthreads();
    // outputs [kt, kt + kSortItems) of this workgroup's share, merged into
    // registers, then stored through LDS so that the global stores coalesce
    const uint32_t kt = threadIdx.x * kSortItems;
    const uint32_t nk = na + nb;
    uint64_t v[kSortItems];
    if (kt < nk) {
        const uint64_t* a = buf;
        const uint64_t* b = buf + na;
        uint32_t lo = kt > nb ? kt - nb : 0u, hi = min(kt, na);
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a[mid] > b[kt - 1u - mid])
                hi = mid;
            else
                lo = mid + 1u;
        }
        uint32_t ia = lo, ib = kt - lo;
#pragma unroll
        for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e) {
            if (kt + e < nk) {
                const bool take_a = ib >= nb || (ia < na && a[ia] < b[ib]);
                v[e] = take_a ? a[ia++] : b[ib++];
            }
        }
    }
    __syncthreads();  // every read of buf is done
    if (kt < nk) {
#pragma unroll
        for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e)
            if (kt + e < nk) buf[lds_slot(kt + e)] = v[e];
    }
    __syncthreads();
    uint64_t* o = out + base + k0;
    for (uint32_t t = threadIdx.x; t < nk; t += kSortThreads) o[t] = buf[lds_slot(t)];
}

// Sorts keys[0, n) (clobbered) into out[0, n).
hipError_t sort_keys(uint64_t* keys, uint64_t* out, uint32_t n, hipStream_t s, uint32_t run0) {
    if (n == 0) return hipSuccess;
    if (run0 != 0u && (run0 < (uint32_t)kSortItems || (run0 & (run0 - 1u)) != 0u))
        return hipErrorInvalidValue;
    const uint32_t tiles = (n + kSortTile - 1) / kSortTile;
    int levels = 0;
    for (uint64_t r = kSortTile; r < n; r <<= 1) ++levels;
    // the block sort writes where `levels` merges, alternating, end in out
    uint64_t* src = (levels & 1) ? keys : out;
    if (n <= 32u * kSortItems)
        block_sort<32><<<1, 32, 0, s>>>(keys, src, n, run0);
    else if (n <= 64u * kSortItems)
        block_sort<64><<<1, 64, 0, s>>>(keys, src, n, run0);
    else if (n <= 128u * kSortItems)
        block_sort<128><<<1, 128, 0, s>>>(keys, src, n, run0);
    else if (n <= 256u * kSortItems)
        block_sort<256><<<1, 256, 0, s>>>(keys, src, n, run0);
    else
        block_sort<kSortThreads><<<tiles, kSortThreads, 0, s>>>(keys, src, n, run0);
    hipError_t e = hipGetLastError();
    uint64_t w = kSortTile;
    for (int l = 0; l < levels && e == hipSuccess; ++l, w <<= 1) {
        uint64_t* dst = src == keys ? out : keys;
        merge_runs<<<tiles, kSortThreads, 0, s>>>(src, dst, n, (uint32_t)w);
        e = hipGetLastError();
        src = dst;
    }
    return e;
}

}  // namespace gccd
