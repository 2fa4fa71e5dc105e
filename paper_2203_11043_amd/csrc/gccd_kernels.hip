// HIP kernels (gfx950 / CDNA4) of the charge-transport hot path of
// Avalos & Sofo Haro, arXiv 2203.11043:
//   field_tiles   -- Eq. (6), softened all-pairs Coulomb field (the O(N^2) part)
//   step_update   -- Eqs. (1)-(4) and the z check of Sec. III.B, fused per carrier
//   load_prepare  -- load-time boundary handling and first active list
//   image_bin     -- 2D histogram of collected holes (Sec. V.A)
#include "gccd_internal.h"

#include <math.h>

namespace gccd {

// ---------------------------------------------------------------------------
// Eq. (6):  E_j = K sum_i r_ij / (|r_ij|^2 + eps^2)^{3/2},  r_ij = r_j - r_i.
//
// One workgroup owns kFieldThreads*TPT target slots and one chunk of the
// sources.  Sources are staged through LDS in tiles of kTile (double
// buffered: the next tile's global loads are in flight while the current one
// is consumed); every lane of every wave reads the same LDS word, so the
// reads are bank-conflict-free broadcasts.  Each lane keeps TPT targets in
// registers for independent dependency chains.
//
// Precision: positions are FP64.  Each coordinate is carried as an FP32 pair
// hi = fl32(x), lo = fl32(x - hi), so x - x' = (hi - hi') + (lo - lo'); the
// hi difference is exact whenever the two points are close, and the pair
// difference keeps about 48 bits without FP64 arithmetic in the loop.  The
// rest of the pair math is FP32 with the hardware reciprocal square root.
// Each tile's contributions are summed separately and then added to the
// running sum (blocked summation), which keeps the FP32 rounding growth at
// O(sqrt(tile) + sqrt(sources/tile)) instead of O(sqrt(sources)).
// ---------------------------------------------------------------------------
template <int TPT>
__device__ __forceinline__ void pair_terms(float shx, float shy, float shz, float slx,
                                           float sly, float slz, const float (&thx)[TPT],
                                           const float (&thy)[TPT], const float (&thz)[TPT],
                                           const float (&tlx)[TPT], const float (&tly)[TPT],
                                           const float (&tlz)[TPT], float eps2,
                                           float (&ax)[TPT], float (&ay)[TPT],
                                           float (&az)[TPT]) {
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        float dx = (thx[t] - shx) + (tlx[t] - slx);
        float dy = (thy[t] - shy) + (tly[t] - sly);
        float dz = (thz[t] - shz) + (tlz[t] - slz);
        float r2 = __builtin_fmaf(dx, dx, eps2);
        r2 = __builtin_fmaf(dy, dy, r2);
        r2 = __builtin_fmaf(dz, dz, r2);
        float inv = __builtin_amdgcn_rsqf(r2);
        float w = inv * inv * inv;
        ax[t] = __builtin_fmaf(dx, w, ax[t]);
        ay[t] = __builtin_fmaf(dy, w, ay[t]);
        az[t] = __builtin_fmaf(dz, w, az[t]);
    }
}

template <int TPT>
__global__ __launch_bounds__(kFieldThreads) void field_tiles(FieldArgs a) {
    __shared__ __align__(16) float sh[2][6][kTile];

    const uint32_t nt = a.tcount ? *a.tcount : a.nt;
    const uint32_t ns = a.scount ? *a.scount : a.ns;
    const int chunk = (int)(blockIdx.x % (uint32_t)a.nchunk);
    const uint32_t tbase = (blockIdx.x / (uint32_t)a.nchunk) * (uint32_t)(kFieldThreads * TPT);
    if (tbase >= nt) return;  // the whole workgroup leaves before any barrier

    const uint32_t s_begin = (uint32_t)(((uint64_t)ns * (uint64_t)chunk) / (uint64_t)a.nchunk);
    const uint32_t s_end = (uint32_t)(((uint64_t)ns * (uint64_t)(chunk + 1)) / (uint64_t)a.nchunk);
    const int tid = threadIdx.x;

    float thx[TPT], thy[TPT], thz[TPT], tlx[TPT], tly[TPT], tlz[TPT];
    float ax[TPT], ay[TPT], az[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        uint32_t slot = tbase + (uint32_t)(t * kFieldThreads + tid);
        double px = 0.0, py = 0.0, pz = 0.0;
        if (slot < nt) {
            uint32_t j = a.tlist ? (uint32_t)a.tlist[slot] : slot;
            px = a.x[j];
            py = a.y[j];
            pz = a.z[j];
        }
        thx[t] = (float)px;
        thy[t] = (float)py;
        thz[t] = (float)pz;
        tlx[t] = (float)(px - (double)thx[t]);
        tly[t] = (float)(py - (double)thy[t]);
        tlz[t] = (float)(pz - (double)thz[t]);
        ax[t] = 0.0f;
        ay[t] = 0.0f;
        az[t] = 0.0f;
    }

    double qx = 0.0, qy = 0.0, qz = 0.0;  // this lane's source of the next tile
    auto fetch = [&](uint32_t tile) {
        uint32_t i = tile + (uint32_t)tid;
        qx = qy = qz = 0.0;
        if (i < s_end) {
            uint32_t c = a.slist ? (uint32_t)a.slist[i] : i;
            qx = a.x[c];
            qy = a.y[c];
            qz = a.z[c];
        }
    };
    auto stage = [&](int b) {
        float hx = (float)qx, hy = (float)qy, hz = (float)qz;
        sh[b][0][tid] = hx;
        sh[b][1][tid] = hy;
        sh[b][2][tid] = hz;
        sh[b][3][tid] = (float)(qx - (double)hx);
        sh[b][4][tid] = (float)(qy - (double)hy);
        sh[b][5][tid] = (float)(qz - (double)hz);
    };

    int buf = 0;
    if (s_begin < s_end) {
        fetch(s_begin);
        stage(0);
    }
    __syncthreads();
    for (uint32_t tile = s_begin; tile < s_end; tile += kTile) {
        const uint32_t next = tile + kTile;
        if (next < s_end) fetch(next);
        const uint32_t cnt = min((uint32_t)kTile, s_end - tile);

        float bx[TPT], by[TPT], bz[TPT];
#pragma unroll
        for (int t = 0; t < TPT; ++t) bx[t] = by[t] = bz[t] = 0.0f;

        const float* hxp = sh[buf][0];
        const float* hyp = sh[buf][1];
        const float* hzp = sh[buf][2];
        const float* lxp = sh[buf][3];
        const float* lyp = sh[buf][4];
        const float* lzp = sh[buf][5];
        uint32_t k = 0;
        for (; k + 4 <= cnt; k += 4) {
            float4 hx = *reinterpret_cast<const float4*>(hxp + k);
            float4 hy = *reinterpret_cast<const float4*>(hyp + k);
            float4 hz = *reinterpret_cast<const float4*>(hzp + k);
            float4 lx = *reinterpret_cast<const float4*>(lxp + k);
            float4 ly = *reinterpret_cast<const float4*>(lyp + k);
            float4 lz = *reinterpret_cast<const float4*>(lzp + k);
            pair_terms<TPT>(hx.x, hy.x, hz.x, lx.x, ly.x, lz.x, thx, thy, thz, tlx, tly, tlz,
                            a.eps2, bx, by, bz);
            pair_terms<TPT>(hx.y, hy.y, hz.y, lx.y, ly.y, lz.y, thx, thy, thz, tlx, tly, tlz,
                            a.eps2, bx, by, bz);
            pair_terms<TPT>(hx.z, hy.z, hz.z, lx.z, ly.z, lz.z, thx, thy, thz, tlx, tly, tlz,
                            a.eps2, bx, by, bz);
            pair_terms<TPT>(hx.w, hy.w, hz.w, lx.w, ly.w, lz.w, thx, thy, thz, tlx, tly, tlz,
                            a.eps2, bx, by, bz);
        }
        for (; k < cnt; ++k) {
            pair_terms<TPT>(hxp[k], hyp[k], hzp[k], lxp[k], lyp[k], lzp[k], thx, thy, thz, tlx,
                            tly, tlz, a.eps2, bx, by, bz);
        }
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            ax[t] += bx[t];
            ay[t] += by[t];
            az[t] += bz[t];
        }
        if (next < s_end) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    float* px = a.part + (size_t)(chunk * 3 + 0) * a.pstride;
    float* py = a.part + (size_t)(chunk * 3 + 1) * a.pstride;
    float* pz = a.part + (size_t)(chunk * 3 + 2) * a.pstride;
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        uint32_t slot = tbase + (uint32_t)(t * kFieldThreads + tid);
        if (slot < nt) {
            px[slot] = ax[t];
            py[slot] = ay[t];
            pz[slot] = az[t];
        }
    }
}

hipError_t launch_field(const FieldArgs& a, int tpt, uint32_t nt_bound, hipStream_t s) {
    const uint32_t per_block = (uint32_t)(kFieldThreads * tpt);
    const uint64_t tblocks = ((uint64_t)nt_bound + per_block - 1) / per_block;
    if (tblocks == 0) return hipSuccess;
    const dim3 grid((uint32_t)(tblocks * (uint64_t)a.nchunk));
    switch (tpt) {
        case 1: field_tiles<1><<<grid, kFieldThreads, 0, s>>>(a); break;
        case 2: field_tiles<2><<<grid, kFieldThreads, 0, s>>>(a); break;
        case 4: field_tiles<4><<<grid, kFieldThreads, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Random diffusion vectors: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// ten rounds of two 32x32->64 multiplies whose high halves are XORed into the
// other words together with the round key; the key advances by two Weyl
// constants between rounds.  Counter = (carrier, step, event, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
        const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
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
// mirror at the back surface, collection at the well.  Holes that keep
// travelling are appended to the next active list, one atomic per wave.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kStepThreads) void step_update(StepArgs a) {
    const uint32_t n_in = *a.cnt_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.cnt_clear = 0u;  // counter of the step after next; nobody reads it now
        if (n_in > 0) {
            atomicAdd(&a.stats[0], (unsigned long long)n_in);
            if (a.coulomb) {
                unsigned long long nsrc = a.src_all ? a.n_all : n_in;
                atomicAdd(&a.stats[1], (unsigned long long)n_in * nsrc);
            }
            a.misc[1] = (int32_t)(a.step + 1u);
        }
    }
    const int lane = threadIdx.x & 63;
    const double two_pi = 6.283185307179586476925286766559;
    for (uint32_t base = blockIdx.x * kStepThreads; base < n_in;
         base += gridDim.x * kStepThreads) {
        const uint32_t slot = base + threadIdx.x;
        bool keep = false;
        int32_t j = 0;
        if (slot < n_in) {
            j = a.list_in[slot];
            double ecx = 0.0, ecy = 0.0, ecz = 0.0;
            if (a.coulomb) {
                double sx = 0.0, sy = 0.0, sz = 0.0;
                for (int c = 0; c < a.nchunk; ++c) {
                    sx += (double)a.part[(size_t)(c * 3 + 0) * a.pstride + slot];
                    sy += (double)a.part[(size_t)(c * 3 + 1) * a.pstride + slot];
                    sz += (double)a.part[(size_t)(c * 3 + 2) * a.pstride + slot];
                }
                ecx = a.K * sx;
                ecy = a.K * sy;
                ecz = a.K * sz;
            }
            const double x0 = a.x[j], y0 = a.y[j], z0 = a.z[j];
            const double es = a.a1 * z0 - a.a2;
            const double ex = ecx, ey = ecy, ez = ecz + es;
            const double em = sqrt(ex * ex + ey * ey + ez * ez);
            double mu = a.mu0;
            if (a.mobility_model == 0) mu = a.mu0 / pow(1.0 + pow(em / a.ec, a.beta), a.inv_beta);
            // v = mu E in cm/s; v dt in cm; 1 cm = 1e4 um
            double dx = mu * ex * a.dt_s * 1e4;
            double dy = mu * ey * a.dt_s * 1e4;
            double dz = mu * ez * a.dt_s * 1e4;
            if (a.diffusion) {
                uint32_t w0 = (uint32_t)j, w1 = a.step, w2 = a.event, w3 = 0u;
                philox4x32_10(w0, w1, w2, w3, a.key0, a.key1);
                const double r01 = sqrt(-2.0 * log(unit_open(w0)));
                const double r23 = sqrt(-2.0 * log(unit_open(w2)));
                const double ang1 = two_pi * unit_open(w1);
                const double ang3 = two_pi * unit_open(w3);
                const double D = a.vt * mu;                        // Eq. (4), cm^2/s
                const double sigma = sqrt(2.0 * D * a.dt_s) * 1e4;  // Eq. (3), um
                dx += sigma * (r01 * cos(ang1));
                dy += sigma * (r01 * sin(ang1));
                dz += sigma * (r23 * cos(ang3));
            }
            const double xn = x0 + dx, yn = y0 + dy;
            double zn = z0 + dz;
            if (zn > a.thickness) zn = 2.0 * a.thickness - zn;
            a.x[j] = xn;
            a.y[j] = yn;
            a.z[j] = zn;
            if (!isfinite(xn) || !isfinite(yn) || !isfinite(zn)) atomicOr(&a.misc[0], 1);
            if (zn <= a.z_well) {
                a.cstep[j] = (int32_t)(a.step + 1u);
            } else {
                keep = true;
            }
        }
        const unsigned long long m = __ballot(keep);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t wbase = 0;
            if (lane == leader) wbase = atomicAdd(a.cnt_out, (uint32_t)__popcll(m));
            wbase = __shfl(wbase, leader);
            if (keep) {
                const unsigned long long below = (lane == 0) ? 0ull : (m << (64 - lane));
                a.list_out[wbase + (uint32_t)__popcll(below)] = j;
            }
        }
    }
}

static uint32_t grid_for(uint64_t n, int threads, uint32_t cap) {
    uint64_t g = (n + (uint64_t)threads - 1) / (uint64_t)threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t launch_step(const StepArgs& a, uint32_t n_bound, hipStream_t s) {
    step_update<<<grid_for(n_bound, kStepThreads, 8192), kStepThreads, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Load-time boundary handling: mirror z beyond the back surface, collect
// holes at or below the well (collection step 0), list the others.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kStepThreads) void load_prepare(double* z, int32_t* cstep,
                                                             int32_t* list, uint32_t* cnt,
                                                             uint32_t n, double thickness,
                                                             double z_well) {
    const int lane = threadIdx.x & 63;
    for (uint32_t base = blockIdx.x * kStepThreads; base < n; base += gridDim.x * kStepThreads) {
        const uint32_t j = base + threadIdx.x;
        bool keep = false;
        if (j < n) {
            double zz = z[j];
            if (zz > thickness) zz = 2.0 * thickness - zz;
            z[j] = zz;
            if (zz <= z_well) {
                cstep[j] = 0;
            } else {
                cstep[j] = -1;
                keep = true;
            }
        }
        const unsigned long long m = __ballot(keep);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t wbase = 0;
            if (lane == leader) wbase = atomicAdd(cnt, (uint32_t)__popcll(m));
            wbase = __shfl(wbase, leader);
            if (keep) {
                const unsigned long long below = (lane == 0) ? 0ull : (m << (64 - lane));
                list[wbase + (uint32_t)__popcll(below)] = (int32_t)j;
            }
        }
    }
}

hipError_t launch_load(double* z, int32_t* cstep, int32_t* list, uint32_t* cnt, uint32_t n,
                       double thickness, double z_well, hipStream_t s) {
    load_prepare<<<grid_for(n, kStepThreads, 8192), kStepThreads, 0, s>>>(z, cstep, list, cnt, n,
                                                                          thickness, z_well);
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
// FP64 in chunk order, times K (same reduction as step_update).
__global__ void field_finish(const float* part, uint32_t pstride, int nchunk, uint32_t n,
                             double K, double* ex, double* ey, double* ez) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            sx += (double)part[(size_t)(c * 3 + 0) * pstride + j];
            sy += (double)part[(size_t)(c * 3 + 1) * pstride + j];
            sz += (double)part[(size_t)(c * 3 + 2) * pstride + j];
        }
        ex[j] = K * sx;
        ey[j] = K * sy;
        ez[j] = K * sz;
    }
}

hipError_t launch_field_finish(const float* part, uint32_t pstride, int nchunk, uint32_t n,
                               double K, double* ex, double* ey, double* ez, hipStream_t s) {
    field_finish<<<grid_for(n, 256, 8192), 256, 0, s>>>(part, pstride, nchunk, n, K, ex, ey, ez);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sec. V.A image: half-open pixels, index floor((x - x0) / pitch) in IEEE
// FP64 (correctly rounded division), integer atomics into the caller's grid.
// ---------------------------------------------------------------------------
__global__ void image_bin(const double* x, const double* y, const int32_t* cstep, uint32_t n,
                          double x0, double y0, double pitch, int32_t nx, int32_t ny,
                          uint32_t* counts, unsigned long long* n_out) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        if (cstep[j] < 0) continue;
        const double fx = floor((x[j] - x0) / pitch);
        const double fy = floor((y[j] - y0) / pitch);
        if (fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny) {
            atomicAdd(&counts[(int64_t)fy * nx + (int64_t)fx], 1u);
        } else {
            atomicAdd(n_out, 1ull);
        }
    }
}

hipError_t launch_image(const double* x, const double* y, const int32_t* cstep, uint32_t n,
                        double x0, double y0, double pitch, int32_t nx, int32_t ny,
                        uint32_t* counts, unsigned long long* n_out, hipStream_t s) {
    image_bin<<<grid_for(n, 256, 8192), 256, 0, s>>>(x, y, cstep, n, x0, y0, pitch, nx, ny,
                                                      counts, n_out);
    return hipGetLastError();
}

}  // namespace gccd
