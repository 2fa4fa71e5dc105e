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
    for (uint32_t w = kSortItems; w < T; w <<= 1) {
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

// 64-bit value of lane (this lane ^ m) of the wave: two LDS-crossbar
// permutes with the byte index computed once.
__device__ __forceinline__ uint64_t lane_xor(uint64_t v, uint32_t m) {
    const int idx = (int)((__lane_id() ^ m) << 2);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(idx, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(idx, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Compare-exchange stage of a bitonic network at distance J < K inside each
// lane's K keys (element i = lane_base + r ascends where (i & k) == 0).
template <int K, int J>
__device__ __forceinline__ void lane_stage(uint64_t (&v)[K], uint32_t base, uint32_t k) {
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)K; ++r)
        if ((r & (uint32_t)J) == 0u) compare_exchange(v[r], v[r | J], ((base + r) & k) == 0u);
}

// Bitonic sort of in[0, n) (n <= T = blockDim.x * K, blockDim.x a multiple
// of 64, T a power of two) into s[lds_slot(i)], i < T, padded with ~0, for
// lists small enough that the latency of the network, not its work, sets
// the time.  Lane t holds elements t K .. t K + K - 1 in registers: stages
// at distance j < K stay in the lane, stages at K <= j < 64 K exchange with
// lane t ^ (j / K) of the same wave (no barrier), and only the stages at
// 64 K and beyond pass through LDS.  Every thread of the workgroup calls
// it; it ends with a barrier.
template <int K>
__device__ __forceinline__ void bitonic_sort_lanes(const uint64_t* in, uint32_t n, uint64_t* s) {
    static_assert(K == 4 || K == 8, "keys per lane");
    const uint32_t T = blockDim.x * (uint32_t)K;
    const uint32_t t = threadIdx.x, base = t * (uint32_t)K;
    uint64_t v[K];
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)K; ++r) v[r] = base + r < n ? in[base + r] : ~0ull;
    for (uint32_t k = 2; k <= T; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (j < (uint32_t)K) {
                if (j == 1u)
                    lane_stage<K, 1>(v, base, k);
                else if (j == 2u)
                    lane_stage<K, 2>(v, base, k);
                else
                    lane_stage<K, (K > 4 ? 4 : 1)>(v, base, k);
                continue;
            }
            // k > j >= K: bit k of every element of the lane is bit k of base
            const uint32_t m = j / (uint32_t)K;
            const bool keep_min = ((t & m) == 0u) == ((base & k) == 0u);
            if (m < 64u) {
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)K; ++r) {
                    const uint64_t o = lane_xor(v[r], m);
                    v[r] = ((o < v[r]) == keep_min) ? o : v[r];
                }
            } else {
                __syncthreads();  // the last exchange's reads are done
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)K; ++r) s[lds_slot(base + r)] = v[r];
                __syncthreads();
                const uint32_t pb = (t ^ m) * (uint32_t)K;
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)K; ++r) {
                    const uint64_t o = s[lds_slot(pb + r)];
                    v[r] = ((o < v[r]) == keep_min) ? o : v[r];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)K; ++r) s[lds_slot(base + r)] = v[r];
    __syncthreads();
}


}  // namespace gccd
