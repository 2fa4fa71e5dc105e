// Device code of the one-workgroup sort of carrier keys, shared by the
// per-step sort (gccd_sort.hip) and the step kernel that rebuilds the list of
// a small load itself (gccd_kernels.hip).
#pragma once

#include "gccd_internal.h"

namespace gccd {

constexpr int kSortItems = 8;  // keys per lane

__device__ __forceinline__ void compare_exchange(uint64_t& a, uint64_t& b, bool up) {
    if ((a > b) == up) {
        const uint64_t t = a;
        a = b;
        b = t;
    }
}

// LDS slot of position i of a tile: one pad word after every kSortItems
// keys, so that the kSortItems consecutive keys of each lane (a stride of
// kSortItems + 1 words between lanes) spread over the banks.
__device__ __forceinline__ uint32_t lds_slot(uint32_t i) { return i + i / kSortItems; }

// Ascending sort of a lane's kSortItems keys in registers (bitonic network).
__device__ __forceinline__ void register_sort(uint64_t (&v)[kSortItems]) {
#pragma unroll
    for (uint32_t k = 2; k <= (uint32_t)kSortItems; k <<= 1)
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e)
                if ((e & j) == 0u) compare_exchange(v[e], v[e | j], (e & k) == 0u);
}

// The merge levels of block_sort_lds from sorted runs of w0 keys (a power
// of two, at least kSortItems): lane t of the first THREADS holds positions
// t kSortItems .. t kSortItems + kSortItems - 1 in v; the sorted T keys end
// in s[lds_slot(i)], followed by a barrier.
template <int THREADS>
__device__ __forceinline__ void merge_levels(uint64_t (&v)[kSortItems], uint64_t* s, uint32_t w0) {
    constexpr uint32_t T = (uint32_t)THREADS * kSortItems;
    const bool on = threadIdx.x < (uint32_t)THREADS;
    const uint32_t first = threadIdx.x * kSortItems;
    for (uint32_t w = w0; w < T; w <<= 1) {
        __syncthreads();  // every read of s is done before it is written again
        if (on) {
#pragma unroll
            for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e) s[lds_slot(first + e)] = v[e];
        }
        __syncthreads();
        if (on) {
            // outputs [k, k + kSortItems) of the merge of runs A = [base, base + w)
            // and B = [base + w, base + 2 w) (both full: T is a power of two)
            const uint32_t base = first / (2 * w) * (2 * w);
            const uint32_t k = first - base, A = base, B = base + w;
            uint32_t lo = k > w ? k - w : 0u, hi = min(k, w);
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s[lds_slot(A + mid)] > s[lds_slot(B + k - 1u - mid)])
                    hi = mid;
                else
                    lo = mid + 1u;
            }
            uint32_t ia = lo, ib = k - lo;
            uint64_t a = ia < w ? s[lds_slot(A + ia)] : ~0ull;
            uint64_t b = ib < w ? s[lds_slot(B + ib)] : ~0ull;
#pragma unroll
            for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e) {
                if (ib >= w || (ia < w && a < b)) {
                    v[e] = a;
                    ++ia;
                    a = ia < w ? s[lds_slot(A + ia)] : ~0ull;
                } else {
                    v[e] = b;
                    ++ib;
                    b = ib < w ? s[lds_slot(B + ib)] : ~0ull;
                }
            }
        }
    }
    __syncthreads();
    if (on) {
#pragma unroll
        for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e) s[lds_slot(first + e)] = v[e];
    }
    __syncthreads();
}

// Sorts in[0, cnt) (cnt <= T = THREADS * kSortItems) into s[lds_slot(i)],
// i < T, padded with ~0 (a key equal to the padding value is the same
// value).  Each of the first THREADS lanes sorts kSortItems consecutive keys
// in registers, then log2(T / kSortItems) levels merge pairs of sorted runs
// in LDS, each lane writing kSortItems consecutive outputs of its pair
// (found by a binary search on the merge path, then a sequential merge).
// Every level moves each key once through LDS.  Every thread of the
// workgroup calls it (lanes from THREADS on only pass the barriers); s holds
// T + T / kSortItems words; it ends with a barrier.
template <int THREADS>
__device__ __forceinline__ void block_sort_lds(const uint64_t* in, uint32_t cnt, uint64_t* s) {
    constexpr uint32_t T = (uint32_t)THREADS * kSortItems;
    const bool on = threadIdx.x < (uint32_t)THREADS;
    const uint32_t first = threadIdx.x * kSortItems;
    for (uint32_t i = threadIdx.x; i < T; i += blockDim.x) s[lds_slot(i)] = i < cnt ? in[i] : ~0ull;
    __syncthreads();
    uint64_t v[kSortItems];
    if (on) {
#pragma unroll
        for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e) v[e] = s[lds_slot(first + e)];
        register_sort(v);
    }
    merge_levels<THREADS>(v, s, kSortItems);
}

// Merge of in[0, cnt) (cnt <= T = THREADS * kSortItems), whose runs of w0
// keys (the last one possibly shorter) are each sorted, into s[lds_slot(i)],
// i < T, padded with ~0.  Every thread of the workgroup calls it; it ends
// with a barrier.
template <int THREADS>
__device__ __forceinline__ void merge_sorted_runs(const uint64_t* in, uint32_t cnt, uint64_t* s,
                                                  uint32_t w0) {
    constexpr uint32_t T = (uint32_t)THREADS * kSortItems;
    const uint32_t first = threadIdx.x * kSortItems;
    for (uint32_t i = threadIdx.x; i < T; i += blockDim.x) s[lds_slot(i)] = i < cnt ? in[i] : ~0ull;
    __syncthreads();
    uint64_t v[kSortItems];
    if (threadIdx.x < (uint32_t)THREADS) {
#pragma unroll
        for (uint32_t e = 0; e < (uint32_t)kSortItems; ++e) v[e] = s[lds_slot(first + e)];
    }
    merge_levels<THREADS>(v, s, w0);
}

// Sort of one key per thread over the workgroup by rank: thread t < m holds
// one of m distinct keys and counts the keys below its own (m broadcast LDS
// reads, two VALU each, no dependent chain), then writes it at that rank;
// threads from m on (no key) keep their places after every key.  Returns
// the key at sorted position threadIdx.x (~0 from m on).  For a few hundred
// keys this is several times faster than a bitonic network, whose stages
// each wait on a lane exchange.  s holds blockDim.x words; every thread
// calls it.
__device__ __forceinline__ uint64_t sort_block_keys(uint64_t v, uint32_t m, uint64_t* s) {
    const uint32_t t = threadIdx.x;
    if (t >= m) v = ~0ull;
    s[t] = v;
    __syncthreads();
    uint32_t r = t;
    if (t < m) {
        r = 0;
        for (uint32_t u = 0; u < m; ++u) r += s[u] < v ? 1u : 0u;
    }
    __syncthreads();
    s[r] = v;
    __syncthreads();
    return s[t];
}

}  // namespace gccd
