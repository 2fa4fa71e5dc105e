/*
 * gccd_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, FP64 CPU reference ("the oracle") for the charge-transport
 * time step of N. E. Avalos and M. Sofo Haro, "G-CoReCCD: a GPU-based
 * simulator of the charge transport in fully-depleted CCDs" (arXiv
 * 2203.11043).  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, constant or
 * helper with the GPU library: everything here is written out again from the
 * paper and from the published definitions it relies on.
 *
 * Units: lengths in micrometres (z measured from the collection plane, z = 0
 * at the front surface, +z into the bulk), fields in V/cm, mobility in
 * cm^2/(V s), time in seconds.
 */
#ifndef GCCD_ORACLE_H
#define GCCD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double thickness_um;   /* bulk thickness (Sec. III.B, list of user inputs) */
    double a1;             /* Eq. (1) slope, (V/cm)/um                         */
    double a2;             /* Eq. (1) offset, V/cm                             */
    double z_well_um;      /* depth of the potential well (Sec. III.B)         */
    double temperature_K;  /* T in Eqs. (2) and (4)                            */
    double eps_r;          /* relative permittivity of silicon, Eq. (6)        */
    double softening_um;   /* epsilon of Eq. (6)                               */
    int32_t coulomb;       /* 1: include Eq. (6) (Sec. III.B: user switch)     */
    int32_t diffusion;     /* 1: include the Brownian step of Sec. II.B        */
    int32_t mobility_model;/* 0: Eq. (2); 1: constant low-field mobility       */
    int32_t collected_are_sources; /* 1: collected holes keep repelling        */
    uint64_t seed;         /* Philox key                                       */
    uint32_t event;        /* third Philox counter word                        */
    uint32_t pad_;
} orc_params;

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Three N(0,1) draws for carrier j at step s (Box-Muller on one Philox block). */
void orc_normals(uint64_t seed, uint32_t j, uint32_t s, uint32_t event, double n[3]);

/* Eq. (2): hole mobility in cm^2/(V s) at field magnitude E (V/cm), T (K). */
double orc_mobility(double E, double T, int32_t model);

/* K = q / (4 pi eps0 eps_r), expressed in V um^2 / cm. */
double orc_coulomb_constant(double eps_r);

/* k_B T / q in volts. */
double orc_thermal_voltage(double T);

/* Eq. (6): softened Coulomb field (V/cm) at nt target points from ns source
 * charges, summed over sources in index order.  If amag is not NULL it gets
 * K * sum_i |r_ij| / (r_ij^2 + eps^2)^{3/2}, the sum of term magnitudes. */
void orc_field(int64_t nt, const double* tx, const double* ty, const double* tz,
               int64_t ns, const double* sx, const double* sy, const double* sz,
               double softening_um, double K,
               double* ex, double* ey, double* ez, double* amag);

/* Eq. (6) over the sources at distance r_lo <= |r_ij| < r_hi from each target
 * (r_hi may be INFINITY).  Used to check a near-field/far-field split. */
void orc_field_window(int64_t nt, const double* tx, const double* ty, const double* tz,
                      int64_t ns, const double* sx, const double* sy, const double* sz,
                      double softening_um, double K, double r_lo, double r_hi,
                      double* ex, double* ey, double* ez);

/* Load-time boundary handling: z above the back surface is mirrored back into
 * the bulk; z at or below the well is collected at step 0 (cstep = 0); every
 * other carrier is active (cstep = -1).  Returns the number of active ones. */
int64_t orc_prepare(const orc_params* p, int64_t n, double* x, double* y, double* z,
                    int32_t* cstep);

/* Runs time steps step0, step0+1, ... until no carrier is active or max_steps
 * steps were taken.  Positions and cstep are updated in place.  Returns 0, or
 * -1 on invalid arguments, -2 if a position became non-finite. */
int orc_run(const orc_params* p, double dt_s, int64_t n,
            double* x, double* y, double* z, int32_t* cstep,
            int64_t step0, int64_t max_steps,
            int64_t* steps_done, int64_t* n_active);

/* 2D histogram of collected carriers (Sec. V.A): half-open bins of width
 * pitch starting at (x0, y0).  counts is ny*nx row-major and is overwritten. */
void orc_image(int64_t n, const double* x, const double* y, const int32_t* cstep,
               double x0, double y0, double pitch, int32_t nx, int32_t ny,
               uint32_t* counts, uint64_t* n_outside);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
