// FP64 elementary functions of the time step (Eq. (2) mobility and the
// Box-Muller transform of the diffusion step, Eqs. (3)-(4)), written from
// their series: exp from its Taylor series after reduction by powers of two,
// log from the series of 2 atanh((m - 1)/(m + 1)), log1p from log(1 + y)
// corrected for the rounding of 1 + y, and sin/cos of pi r from their Taylor
// series after reduction by half turns.  Each is accurate to 2 units in the
// last place over the arguments the step gives them and their whole ranges
// (checked against 40-digit references on the host); the general-purpose
// library versions spend about
// twice the instructions on guarantees the step does not need (correct
// rounding of every argument, extended internal precision), and the step
// without repulsion is bound by instruction issue.
//
// Only fma, frexp, ldexp, rint and IEEE division and comparison are used,
// so the same code compiles for the host, where the tests measure its error.
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

// ln 2 split for exact products k * kLn2Hi with |k| < 2^11 (kLn2Hi has 42
// significant bits); kLn2Lo = ln 2 - kLn2Hi rounded.
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
constexpr double kLog2E = 1.4426950408889634;  // 1 / ln 2
constexpr double kSqrtHalf = 0.7071067811865476;

// e^x.  x = k ln 2 + r, |r| <= ln 2 / 2 (Cody-Waite reduction with the
// split ln 2; the first product is exact), e^r by its Taylor series to r^13
// (the first omitted term is below 5e-18 of the sum), times 2^k.
template <bool F3 = false>
GCCD_HD inline double exp(double x) {
    if (x != x) return x;
    if (x > 709.8) return INFINITY;
    if (x < -745.2) return 0.0;
    const double k = rint(x * kLog2E);
    const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
    double p = 1.6059043836821613e-10;  // 1/13!
    p = horner<F3>(p, r, 2.08767569878681e-09);
    p = horner<F3>(p, r, 2.505210838544172e-08);
    p = horner<F3>(p, r, 2.755731922398589e-07);
    p = horner<F3>(p, r, 2.7557319223985893e-06);
    p = horner<F3>(p, r, 2.48015873015873e-05);
    p = horner<F3>(p, r, 0.0001984126984126984);
    p = horner<F3>(p, r, 0.001388888888888889);
    p = horner<F3>(p, r, 0.008333333333333333);
    p = horner<F3>(p, r, 0.041666666666666664);
    p = horner<F3>(p, r, 0.16666666666666666);
    p = horner<F3>(p, r, 0.5);
    p = horner<F3>(p, r, 1.0);
    p = horner<F3>(p, r, 1.0);
    return ldexp(p, (int)k);
}

// ln x.  x = 2^e m with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(f),
// f = (m - 1)/(m + 1), |f| <= 0.1716, by its series to f^23 (the first
// omitted term is below 1e-18 of the sum); ln x = e ln 2 + ln m.  f is
// carried as f + f_lo (the residual of the division, with m + 1 split
// exactly into its rounded value and error), so that 2 f, the leading term,
// is nearly exact.
template <bool F3 = false>
GCCD_HD inline double log(double x) {
    if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;  // also NaN for NaN
    if (x == INFINITY) return x;
    int e;
    double m = frexp(x, &e);  // m in [1/2, 1)
    if (m < kSqrtHalf) {
        m *= 2.0;
        e -= 1;
    }
    const double num = m - 1.0;             // exact
    const double den = m + 1.0;             // rounded
    const double den_lo = m - (den - 1.0);  // m + 1 - den, exact
    const double y = 1.0 / den;
    const double f = num * y;
    const double f_lo = (fma(-f, den, num) - f * den_lo) * y;
    const double s = f * f;
    double q = 0.08695652173913043;  // 2/23
    q = horner<F3>(q, s, 0.09523809523809523);
    q = horner<F3>(q, s, 0.10526315789473684);
    q = horner<F3>(q, s, 0.11764705882352941);
    q = horner<F3>(q, s, 0.13333333333333333);
    q = horner<F3>(q, s, 0.15384615384615385);
    q = horner<F3>(q, s, 0.18181818181818182);
    q = horner<F3>(q, s, 0.2222222222222222);
    q = horner<F3>(q, s, 0.2857142857142857);
    q = horner<F3>(q, s, 0.4);
    q = horner<F3>(q, s, 0.6666666666666666);  // 2/3
    const double de = (double)e;
    const double lo = fma(de, kLn2Lo, fma(f * s, q, 2.0 * f_lo));
    return fma(de, kLn2Hi, 2.0 * f) + lo;
}

// ln(1 + y), y >= -1: u = 1 + y rounded, d = y - (u - 1) its rounding error
// (exact), ln(1 + y) = ln u + d / u to first order in d / u.
template <bool F3 = false>
GCCD_HD inline double log1p(double y) {
    const double u = 1.0 + y;
    if (u == 1.0) return y;
    if (u == INFINITY || u != u) return u;
    const double d = y - (u - 1.0);
    return log<F3>(u) + d / u;
}

// sin(pi x) and cos(pi x) for finite x with |x| < 2^51: x = n/2 + r
// (exact), |r| <= 1/4, the series of sin(pi r) to r^17 and cos(pi r) to
// r^16, then the quadrant n mod 4.
template <bool F3 = false>
GCCD_HD inline void sincospi(double x, double* sp, double* cp) {
    const double n = rint(2.0 * x);
    const double r = fma(-0.5, n, x);
    const double z = r * r;
    double ps = 7.952054001475513e-07;  // pi^17/17!
    ps = horner<F3>(ps, z, -2.1915353447830217e-05);
    ps = horner<F3>(ps, z, 0.00046630280576761255);
    ps = horner<F3>(ps, z, -0.0073704309457143504);
    ps = horner<F3>(ps, z, 0.08214588661112823);
    ps = horner<F3>(ps, z, -0.5992645293207921);
    ps = horner<F3>(ps, z, 2.5501640398773455);
    ps = horner<F3>(ps, z, -5.16771278004997);
    ps = horner<F3>(ps, z, 3.141592653589793);
    const double s = r * ps;
    double pc = 4.303069587032947e-06;  // pi^16/16!
    pc = horner<F3>(pc, z, -0.0001046381049248457);
    pc = horner<F3>(pc, z, 0.0019295743094039231);
    pc = horner<F3>(pc, z, -0.02580689139001406);
    pc = horner<F3>(pc, z, 0.2353306303588932);
    pc = horner<F3>(pc, z, -1.3352627688545895);
    pc = horner<F3>(pc, z, 4.0587121264167685);
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
