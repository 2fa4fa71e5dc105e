// Internal declarations shared by the host ABI and the kernels of libgccd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gccd {

constexpr int kFieldThreads = 256;   // threads per Eq. (6) workgroup (4 wave64)
constexpr int kTile = 256;           // sources staged in LDS per tile
constexpr int kMaxChunks = 64;       // largest source split of one target's sum
constexpr int kStepThreads = 256;

// Carrier lists hold 64-bit keys: the carrier index in the low idx_bits
// bits, a 36-bit Morton code of the hole's 0.25 um cell above it, and above
// that a bit set for collected holes.  Keys are unique, so sorting them is
// deterministic; the sorted order puts travelling holes first and groups
// nearby holes into the same workgroup and the same source tile.
constexpr double kCellPerUm = 4.0;     // Morton cells of 0.25 um
constexpr int kMortonBits = 36;        // 12 bits per axis (wraps every 1024 um)
constexpr uint64_t kNoKey = ~0ull;     // sorts after every real key

// Targets and sources of one Eq. (6) launch, as FP64 positions already laid
// out in list-slot order (gathered from the carrier arrays after each sort),
// so that every read of the field kernel is coalesced.
struct FieldArgs {
    const double* tx;
    const double* ty;
    const double* tz;
    const uint32_t* tcount;   // device count of targets; NULL: use nt
    uint32_t nt;
    const double* sx;
    const double* sy;
    const double* sz;
    const uint32_t* scount;   // device count of sources; NULL: use ns
    uint32_t ns;
    const double* tile_box;   // [6][tile_stride] boxes of the source tiles, or NULL
    uint32_t tile_stride;
    int32_t nchunk;           // source chunks (partials per target)
    float eps2;               // softening length squared, um^2
    float* part;              // [nchunk][3][pstride] FP32 partial sums
    uint32_t pstride;
};

// Everything the per-carrier update of one step needs.
struct StepArgs {
    double* x;
    double* y;
    double* z;
    int32_t* cstep;
    const uint64_t* keys_in;  // this step's list; its first *cnt_in keys travel
    const uint32_t* cnt_in;
    uint64_t* keys_out;       // next step's list, before sorting
    int32_t full_list;        // 1: lists hold all n carriers, else travelling ones only
    uint32_t* cnt_out;
    uint32_t* cnt_clear;
    const float* part;
    uint32_t pstride;
    int32_t nchunk;
    int32_t coulomb;
    int32_t diffusion;
    int32_t mobility_model;
    int32_t src_all;          // 1: sources are all n carriers
    uint32_t n_all;
    uint32_t idx_bits;        // low key bits holding the carrier index
    double K;                 // V um^2 / cm
    double a1, a2;            // Eq. (1)
    double thickness, z_well;
    double mu0, ec, beta, inv_beta;   // Eq. (2) at the context's T
    double dt_s;              // time step, s
    double vt;                // k_B T / q, V
    uint32_t step;
    uint32_t event;
    uint32_t key0, key1;
    unsigned long long* stats;  // [0] carrier-steps, [1] pair interactions
    int32_t* misc;              // [0] non-finite flag, [1] step after the last busy one
};

hipError_t launch_field(const FieldArgs& a, int tpt, uint32_t nt_bound, hipStream_t s);
hipError_t launch_step(const StepArgs& a, uint32_t n_bound, hipStream_t s);
hipError_t launch_load(double* z, int32_t* cstep, uint64_t* keys, uint32_t* cnt,
                       const double* x, const double* y, uint32_t n, uint32_t idx_bits,
                       int full_list, double thickness, double z_well, hipStream_t s);
// Gathers the positions of the first *count (or count_c) keys of a list into
// slot order and, if box is not NULL, the bounding box of every tile of kTile
// slots.
hipError_t launch_gather(const uint64_t* keys, const uint32_t* count, uint32_t count_c,
                         uint32_t bound, uint64_t idx_mask, uint32_t n_all, const double* x,
                         const double* y, const double* z, double* px, double* py, double* pz,
                         double* box, uint32_t stride, hipStream_t s);
hipError_t launch_keys_all(const double* x, const double* y, const double* z, uint32_t n,
                           uint32_t idx_bits, uint64_t* keys, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_field_finish(const float* part, uint32_t pstride, int nchunk,
                               const uint64_t* tkeys, uint64_t idx_mask, uint32_t n, double K,
                               double* ex, double* ey, double* ez, hipStream_t s);
hipError_t launch_image(const double* x, const double* y, const int32_t* cstep, uint32_t n,
                        double x0, double y0, double pitch, int32_t nx, int32_t ny,
                        uint32_t* counts, unsigned long long* n_out, hipStream_t s);

// Sorting of key lists (rocPRIM radix sort; storage provided by the caller).
hipError_t sort_keys_storage(uint32_t n, uint32_t end_bit, size_t* bytes);
hipError_t sort_keys(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out,
                     uint32_t n, uint32_t end_bit, hipStream_t s);

}  // namespace gccd
