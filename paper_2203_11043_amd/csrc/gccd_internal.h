// Internal declarations shared by the host ABI and the kernels of libgccd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gccd {

constexpr int kFieldThreads = 256;   // threads per Eq. (6) workgroup (4 wave64)
constexpr int kTile = 256;           // sources staged in LDS per tile
constexpr int kMaxChunks = 32;       // largest source split of one target's sum
constexpr int kStepThreads = 256;

// Which carriers are the targets and the sources of one Eq. (6) launch.
struct FieldArgs {
    const double* x;
    const double* y;
    const double* z;
    const int32_t* tlist;     // target carrier of each slot; NULL: slot = carrier
    const uint32_t* tcount;   // device count of targets; NULL: use nt
    uint32_t nt;
    const int32_t* slist;     // source carrier of each source slot; NULL: identity
    const uint32_t* scount;   // device count of sources; NULL: use ns
    uint32_t ns;
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
    const int32_t* list_in;
    const uint32_t* cnt_in;
    int32_t* list_out;
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
hipError_t launch_load(double* z, int32_t* cstep, int32_t* list, uint32_t* cnt,
                       uint32_t n, double thickness, double z_well, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_field_finish(const float* part, uint32_t pstride, int nchunk, uint32_t n,
                               double K, double* ex, double* ey, double* ez, hipStream_t s);
hipError_t launch_image(const double* x, const double* y, const int32_t* cstep, uint32_t n,
                        double x0, double y0, double pitch, int32_t nx, int32_t ny,
                        uint32_t* counts, unsigned long long* n_out, hipStream_t s);

}  // namespace gccd
