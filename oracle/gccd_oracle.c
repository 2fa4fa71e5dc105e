/*
 * gccd_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain FP64 CPU reference for one time step of the G-CoReCCD charge
 * transport (Avalos & Sofo Haro, arXiv 2203.11043).  It follows the paper's
 * order of operations (Sec. III.B, Fig. 2): static field, Coulomb field, their
 * sum, its magnitude, the mobility, the drift velocity, the random diffusion
 * vector, the total displacement, and finally the check of every z position.
 * No blocking, no fusion, no reordering: every carrier's field is a plain sum
 * over the sources in index order, in double precision.
 *
 * Readings of the paper where it is silent (each is listed with its reason in
 * the project's design notes):
 *   - eps_Si in Eq. (5) is the relative permittivity; K = q/(4 pi eps0 eps_r).
 *   - Eq. (1) is the z component of the static field, z measured from the
 *     collection plane; holes move along +mu*E.
 *   - the same local mobility mu(|E_total|) sets drift and diffusion.
 *   - forward Euler, all fields from the positions at the start of the step.
 *   - each Cartesian coordinate receives variance 2 D dt (Eq. (3)).
 *   - a carrier whose z falls to the well depth or below is collected and
 *     frozen; collected carriers stay Coulomb sources unless told otherwise.
 *   - a z beyond the back surface is mirrored back into the bulk.
 *   - the random vectors come from Philox4x32-10 with counter
 *     (carrier, step, event, 0) and key (seed low, seed high), turned into
 *     normals by the Box-Muller transform; the fourth word's partner is unused.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include "gccd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants (CODATA 2018, SI) ------------------------------- */
static const double ORC_Q    = 1.602176634e-19;   /* elementary charge, C   */
static const double ORC_KB   = 1.380649e-23;      /* Boltzmann, J/K         */
static const double ORC_EPS0 = 8.8541878128e-12;  /* vacuum permittivity    */
static const double ORC_PI   = 3.14159265358979323846;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- Philox4x32-10 --------------------------------------------------------
 * Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", SC'11:
 * a 4-word counter is mixed by ten rounds.  Each round multiplies words 0
 * and 2 by two fixed odd constants, keeps both halves of the 64-bit
 * products, and XORs the high halves with the other two words and the round
 * key; the key advances by two Weyl increments between rounds. */
static void orc_mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   /* key increments    */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint32_t hi0, lo0, hi1, lo1;
        orc_mulhilo32(M0, c0, &hi0, &lo0);
        orc_mulhilo32(M1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u in (0,1): the 32-bit word plus one half, scaled by 2^-32, so that log(u)
 * is always finite. */
static double orc_unit(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

void orc_normals(uint64_t seed, uint32_t j, uint32_t s, uint32_t event, double n[3]) {
    uint32_t ctr[4] = { j, s, event, 0u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u0 = orc_unit(w[0]), u1 = orc_unit(w[1]);
    double u2 = orc_unit(w[2]), u3 = orc_unit(w[3]);
    /* Box & Muller (1958): radius from one uniform, angle from the other. */
    double r01 = sqrt(-2.0 * log(u0));
    double r23 = sqrt(-2.0 * log(u2));
    n[0] = r01 * cos(2.0 * ORC_PI * u1);
    n[1] = r01 * sin(2.0 * ORC_PI * u1);
    n[2] = r23 * cos(2.0 * ORC_PI * u3);
}

/* ---- Eq. (2): hole mobility ------------------------------------------------ */
double orc_mobility(double E, double T, int32_t model) {
    double low_field = 1.31e8 * pow(T, -2.2);
    if (model == 1) return low_field;
    double expo = 0.46 * pow(T, 0.17);
    double critical = 1.24 * pow(T, 1.68);
    double ratio = E / critical;
    return low_field / pow(1.0 + pow(ratio, expo), 1.0 / expo);
}

/* K of Eq. (6) in V um^2/cm: q/(4 pi eps0 eps_r) is in V m; a distance in um
 * contributes 1e12 um^2 per m^2, and 1 V/m is 1e-2 V/cm. */
double orc_coulomb_constant(double eps_r) {
    return ORC_Q / (4.0 * ORC_PI * ORC_EPS0 * eps_r) * 1e12 * 1e-2;
}

/* Eq. (4) without the mobility: k_B T / q in volts. */
double orc_thermal_voltage(double T) { return ORC_KB * T / ORC_Q; }

/* ---- Eq. (6): softened all-pairs field ------------------------------------ */
void orc_field(int64_t nt, const double* tx, const double* ty, const double* tz,
               int64_t ns, const double* sx, const double* sy, const double* sz,
               double softening_um, double K,
               double* ex, double* ey, double* ez, double* amag) {
    double e2 = softening_um * softening_um;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nt; ++j) {
        double fx = 0.0, fy = 0.0, fz = 0.0, fa = 0.0;
        for (int64_t i = 0; i < ns; ++i) {
            /* r_ij = r_j - r_i points from the source to the target. */
            double dx = tx[j] - sx[i];
            double dy = ty[j] - sy[i];
            double dz = tz[j] - sz[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            /* (r^2 + eps^2)^{3/2}, written as the product with its root */
            double q = r2 + e2;
            double w = 1.0 / (q * sqrt(q));
            fx += dx * w;
            fy += dy * w;
            fz += dz * w;
            if (amag) fa += sqrt(r2) * w;
        }
        ex[j] = K * fx;
        ey[j] = K * fy;
        ez[j] = K * fz;
        if (amag) amag[j] = K * fa;
    }
}

/* Eq. (6) restricted to the sources whose distance r = |r_ij| from the target
 * lies in [r_lo, r_hi): the split of the sum that a near-field/far-field
 * scheme uses.  Same term as orc_field; distances compared unsoftened. */
void orc_field_window(int64_t nt, const double* tx, const double* ty, const double* tz,
                      int64_t ns, const double* sx, const double* sy, const double* sz,
                      double softening_um, double K, double r_lo, double r_hi,
                      double* ex, double* ey, double* ez) {
    double soft2 = softening_um * softening_um;
    double lo2 = r_lo * r_lo, hi2 = r_hi * r_hi;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nt; ++j) {
        double acc_x = 0.0, acc_y = 0.0, acc_z = 0.0;
        for (int64_t i = 0; i < ns; ++i) {
            double ux = tx[j] - sx[i], uy = ty[j] - sy[i], uz = tz[j] - sz[i];
            double dist2 = ux * ux + uy * uy + uz * uz;
            if (dist2 < lo2 || !(dist2 < hi2)) continue;
            double s = dist2 + soft2;
            double inv3 = 1.0 / (s * sqrt(s));
            acc_x += ux * inv3;
            acc_y += uy * inv3;
            acc_z += uz * inv3;
        }
        ex[j] = K * acc_x;
        ey[j] = K * acc_y;
        ez[j] = K * acc_z;
    }
}

/* ---- load-time boundary handling ------------------------------------------ */
int64_t orc_prepare(const orc_params* p, int64_t n, double* x, double* y, double* z,
                    int32_t* cstep) {
    (void)x; (void)y;
    int64_t active = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (z[j] > p->thickness_um) z[j] = 2.0 * p->thickness_um - z[j];
        if (z[j] <= p->z_well_um) {
            cstep[j] = 0;
        } else {
            cstep[j] = -1;
            ++active;
        }
    }
    return active;
}

/* ---- the time-step loop (Sec. III.B, Fig. 2) ------------------------------- */
int orc_run(const orc_params* p, double dt_s, int64_t n,
            double* x, double* y, double* z, int32_t* cstep,
            int64_t step0, int64_t max_steps,
            int64_t* steps_done, int64_t* n_active) {
    if (!p || n < 0 || max_steps < 0 || !(dt_s > 0.0) || step0 < 0) return -1;
    const double T = p->temperature_K;
    const double K = orc_coulomb_constant(p->eps_r);
    const double vt = orc_thermal_voltage(T);

    int64_t* act = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double* sx = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* sy = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* sz = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ax = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ay = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* az = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ecx = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ecy = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ecz = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* nx_ = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ny_ = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* nz_ = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int rc = 0;
    int64_t done = 0, na = 0;

    for (int64_t k = 0; k < max_steps; ++k) {
        int64_t s = step0 + k;
        /* which carriers are still travelling */
        na = 0;
        for (int64_t j = 0; j < n; ++j)
            if (cstep[j] < 0) act[na++] = j;
        if (na == 0) break;  /* every charge has arrived: leave the loop */

        /* Coulomb field at every active carrier from the positions at the
         * start of this step (Eq. (6)). */
        if (p->coulomb) {
            int64_t ns = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (p->collected_are_sources || cstep[i] < 0) {
                    sx[ns] = x[i]; sy[ns] = y[i]; sz[ns] = z[i]; ++ns;
                }
            }
            for (int64_t a = 0; a < na; ++a) {
                ax[a] = x[act[a]]; ay[a] = y[act[a]]; az[a] = z[act[a]];
            }
            orc_field(na, ax, ay, az, ns, sx, sy, sz, p->softening_um, K,
                      ecx, ecy, ecz, NULL);
        } else {
            for (int64_t a = 0; a < na; ++a) { ecx[a] = 0.0; ecy[a] = 0.0; ecz[a] = 0.0; }
        }

        /* per-carrier transport, written to new positions (Jacobi order) */
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < na; ++a) {
            int64_t j = act[a];
            double Es = p->a1 * z[j] - p->a2;                 /* Eq. (1)  */
            double Ex = ecx[a], Ey = ecy[a], Ez = ecz[a] + Es; /* sum      */
            double Em = sqrt(Ex * Ex + Ey * Ey + Ez * Ez);     /* |E|      */
            double mu = orc_mobility(Em, T, p->mobility_model);/* Eq. (2)  */
            /* v = mu E in cm/s; times dt gives cm; 1 cm = 1e4 um */
            double vx = mu * Ex, vy = mu * Ey, vz = mu * Ez;
            double dx = vx * dt_s * 1e4, dy = vy * dt_s * 1e4, dz = vz * dt_s * 1e4;
            if (p->diffusion) {
                double D = vt * mu;                            /* Eq. (4), cm^2/s */
                double sigma = sqrt(2.0 * D * dt_s) * 1e4;     /* Eq. (3), um     */
                double g[3];
                orc_normals(p->seed, (uint32_t)j, (uint32_t)s, p->event, g);
                dx += sigma * g[0];
                dy += sigma * g[1];
                dz += sigma * g[2];
            }
            nx_[a] = x[j] + dx;
            ny_[a] = y[j] + dy;
            nz_[a] = z[j] + dz;
        }

        /* move, then check every z position */
        for (int64_t a = 0; a < na; ++a) {
            int64_t j = act[a];
            double zn = nz_[a];
            if (zn > p->thickness_um) zn = 2.0 * p->thickness_um - zn;
            x[j] = nx_[a];
            y[j] = ny_[a];
            z[j] = zn;
            if (!isfinite(x[j]) || !isfinite(y[j]) || !isfinite(z[j])) rc = -2;
            if (zn <= p->z_well_um) cstep[j] = (int32_t)(s + 1);
        }
        ++done;
        if (rc) break;
    }
    na = 0;
    for (int64_t j = 0; j < n; ++j)
        if (cstep[j] < 0) ++na;
    if (steps_done) *steps_done = done;
    if (n_active) *n_active = na;

    free(act); free(sx); free(sy); free(sz); free(ax); free(ay); free(az);
    free(ecx); free(ecy); free(ecz); free(nx_); free(ny_); free(nz_);
    return rc;
}

/* ---- image: 2D histogram of collected positions ----------------------------- */
void orc_image(int64_t n, const double* x, const double* y, const int32_t* cstep,
               double x0, double y0, double pitch, int32_t nx, int32_t ny,
               uint32_t* counts, uint64_t* n_outside) {
    memset(counts, 0, sizeof(uint32_t) * (size_t)nx * (size_t)ny);
    uint64_t out = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (cstep[j] < 0) continue;  /* still travelling: not in the image */
        double fx = floor((x[j] - x0) / pitch);
        double fy = floor((y[j] - y0) / pitch);
        if (fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny) {
            counts[(int64_t)fy * nx + (int64_t)fx] += 1u;
        } else {
            ++out;
        }
    }
    *n_outside = out;
}
