// FP64 elementary functions of the time step (Eq. (2) mobility and the
// Box-Muller transform of the diffusion step, Eqs. (3)-(4)): exp after
// reduction by powers of two, log from 2 atanh((m - 1)/(m + 1)), log1p from
// log(1 + y) corrected for the rounding of 1 + y, sin/cos of pi r after
// reduction by half turns, each with a near-minimax polynomial on the
// reduced interval (coefficients printed by fp64_coefficients.py from
// 40-digit Chebyshev fits), and the reciprocal and square root by Newton
// steps from a hardware estimate.  Each is accurate to 2 units in the last
// place over the arguments the step gives them and their whole ranges
// (checked against 40-digit references on the host); the general-purpose
// library versions spend about twice the instructions on guarantees the step
// does not need (correct rounding of every argument, scaling for subnormal
// inputs), and the step without repulsion is bound by instruction issue.
//
// Only fma, frexp, ldexp, rint, IEEE comparison and the two estimates are
// used; the host build takes its estimates from single precision and then
// the same Newton steps, so the tests measure the same algorithm.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define GCCD_HD __host__ __device__
#else
#define GCCD_HD
#endif

namespace gccd {
namespace fp64 {

// One Horner step p r + c.  F3: on the device a single three-operand FMA
// with the coefficient in a register.  The compiler's own choice keeps each
// hoisted coefficient live and copies it into the accumulator of the
// two-operand form first, one more instruction per step; F3 saves it at the
// cost of the registers that hold the coefficients (for a kernel bound by
// instruction issue, not by occupancy).  The host build computes the same
// IEEE fma either way.
template <bool F3>
GCCD_HD inline double horner(double p, double r, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (F3) {
        double d;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(p), "v"(r), "v"(c));
        return d;
    }
#endif
    return fma(p, r, c);
}

// 1/x for finite x > 0 with a normal reciprocal: two Newton steps
// y <- y + y (1 - x y) from an estimate good to about 2^-22 (the hardware's
// on the device, single precision on the host), each squaring the error.
GCCD_HD inline double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(x);
#else
    double y = (double)(1.0f / (float)x);
#endif
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// sqrt(x) for finite normal x > 0: from an estimate y of 1/sqrt(x), one
// coupled Newton step on g = x y (towards sqrt x) and h = y / 2, then a
// final correction of g by its residual x - g^2.
GCCD_HD inline double sqrt_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
#else
    const double y = (double)(1.0f / sqrtf((float)x));
#endif
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    return fma(h, fma(-g, g, x), g);
}

// ln 2 split for exact products k * kLn2Hi with |k| < 2^11 (kLn2Hi has 42
// significant bits); kLn2Lo = ln 2 - kLn2Hi rounded.
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
constexpr double kLog2E = 1.4426950408889634;  // 1 / ln 2
constexpr double kSqrtHalf = 0.7071067811865476;

// e^x for x in [-745.2, 709.8] (no special cases).  x = k ln 2 + r,
// |r| <= ln 2 / 2 (Cody-Waite reduction with the split ln 2; the first
// product is exact), e^r by a degree-11 polynomial (relative error 1.7e-17
// on the interval), times 2^k.
template <bool F3 = false>
GCCD_HD inline double exp_fin(double x) {
    const double k = rint(x * kLog2E);
    const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
    double p = 2.5110037721946562e-08;
    p = horner<F3>(p, r, 2.7632639789868395e-07);
    p = horner<F3>(p, r, 2.7557240918265525e-06);
    p = horner<F3>(p, r, 2.480148548192088e-05);
    p = horner<F3>(p, r, 0.00019841269890047406);
    p = horner<F3>(p, r, 0.0013888888952315155);
    p = horner<F3>(p, r, 0.008333333333319601);
    p = horner<F3>(p, r, 0.04166666666648809);
    p = horner<F3>(p, r, 0.1666666666666668);
    p = horner<F3>(p, r, 0.5000000000000019);
    p = horner<F3>(p, r, 1.0);
    p = horner<F3>(p, r, 1.0);
    return ldexp(p, (int)k);
}

// e^x with the special values: NaN for NaN, +inf above 709.8, 0 below
// -745.2.
template <bool F3 = false>
GCCD_HD inline double exp(double x) {
    if (x != x) return x;
    if (x > 709.8) return INFINITY;
    if (x < -745.2) return 0.0;
    return exp_fin<F3>(x);
}

// ln x for finite x > 0.  x = 2^e m with m in [sqrt(1/2), sqrt(2));
// ln m = 2 atanh(f), f = (m - 1)/(m + 1), |f| <= 0.1716, taken as
// 2 f + f s q(s), s = f^2, with q a degree-6 polynomial (relative error
// 4.7e-16 in a term below 1 % of the sum); ln x = e ln 2 + ln m.  f is
// carried as f + f_lo (the residual of the division, with m + 1 split
// exactly into its rounded value and error), so that 2 f, the leading term,
// is nearly exact.
template <bool F3 = false>
GCCD_HD inline double log_pos(double x) {
    int e;
    double m = frexp(x, &e);  // m in [1/2, 1)
    if (m < kSqrtHalf) {
        m *= 2.0;
        e -= 1;
    }
    const double num = m - 1.0;             // exact
    const double den = m + 1.0;             // rounded
    const double den_lo = m - (den - 1.0);  // m + 1 - den, exact
    const double y = recip(den);
    const double f = num * y;
    const double f_lo = (fma(-f, den, num) - f * den_lo) * y;
    const double s = f * f;
    double q = 0.14616451042434167;
    q = horner<F3>(q, s, 0.15331721490738642);
    q = horner<F3>(q, s, 0.18182889128565508);
    q = horner<F3>(q, s, 0.22222211134749734);
    q = horner<F3>(q, s, 0.28571428625975764);
    q = horner<F3>(q, s, 0.39999999999899505);
    q = horner<F3>(q, s, 0.666666666666667);
    const double de = (double)e;
    const double lo = fma(de, kLn2Lo, fma(f * s, q, 2.0 * f_lo));
    return fma(de, kLn2Hi, 2.0 * f) + lo;
}

// ln x with the special values: -inf at 0, NaN below 0 and for NaN, +inf
// at +inf.
template <bool F3 = false>
GCCD_HD inline double log(double x) {
    if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;  // also NaN for NaN
    if (x == INFINITY) return x;
    return log_pos<F3>(x);
}

// ln(1 + y) for finite y > -1 with 1 + y finite (no special cases): u = 1 + y
// rounded, d = y - (u - 1) its rounding error (exact), ln(1 + y) =
// ln u + d / u to first order in d / u.  Where u rounds to 1, ln u is 0 and
// the result is y.
template <bool F3 = false>
GCCD_HD inline double log1p_fin(double y) {
    const double u = 1.0 + y;
    const double d = y - (u - 1.0);
    return log_pos<F3>(u) + d * recip(u);
}

// ln(1 + y), y >= -1, with the special values (-inf at -1, +inf at +inf,
// NaN for NaN).
template <bool F3 = false>
GCCD_HD inline double log1p(double y) {
    const double u = 1.0 + y;
    if (u == 1.0) return y;
    if (u == INFINITY || u != u) return u;
    const double d = y - (u - 1.0);
    return log<F3>(u) + d * recip(u);
}

// sin(pi x) and cos(pi x) for finite x with |x| < 2^51: x = n/2 + r
// (exact), |r| <= 1/4, sin(pi r) = r P(r^2) and cos(pi r) = C(r^2) with
// near-minimax P and C of degrees 6 and 7 in r^2 (relative errors 3.9e-17
// and 2.1e-17), then the quadrant n mod 4.
template <bool F3 = false>
GCCD_HD inline void sincospi(double x, double* sp, double* cp) {
    const double n = rint(2.0 * x);
    const double r = fma(-0.5, n, x);
    const double z = r * r;
    double ps = 0.000461531855383581;
    ps = horner<F3>(ps, z, -0.007370021586907771);
    ps = horner<F3>(ps, z, 0.08214586918000175);
    ps = horner<F3>(ps, z, -0.5992645289396449);
    ps = horner<F3>(ps, z, 2.5501640398733763);
    ps = horner<F3>(ps, z, -5.167712780049954);
    ps = horner<F3>(ps, z, 3.141592653589793);
    const double s = r * ps;
    double pc = -0.00010356747255199479;
    pc = horner<F3>(pc, z, 0.0019294657440800042);
    pc = horner<F3>(pc, z, -0.025806885652951306);
    pc = horner<F3>(pc, z, 0.23533063019088787);
    pc = horner<F3>(pc, z, -1.3352627688519174);
    pc = horner<F3>(pc, z, 4.058712126416747);
    pc = horner<F3>(pc, z, -4.934802200544679);
    const double c = fma(pc, z, 1.0);
    const int q = (int)((int64_t)n & 3);
    const double a = (q & 1) ? c : s;  // sin(pi x) up to sign
    const double b = (q & 1) ? s : c;  // cos(pi x) up to sign
    *sp = (q & 2) ? -a : a;
    *cp = (q == 1 || q == 2) ? -b : b;
}

}  // namespace fp64
}  // namespace gccd
