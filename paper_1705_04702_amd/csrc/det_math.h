// det_math.h -- FP64 elementary functions with a fixed operation sequence,
// used by the FP64 validation instantiation so that its results do not depend
// on the device math library (the same specification is implemented on the
// reference side; together with contraction disabled, the validation kernel
// then rounds exactly like an FP64 reference).
//
// Method: Cody & Waite additive argument reduction ("Software Manual for the
// Elementary Functions", 1980) and truncated Taylor series in Horner form;
// log through 2 atanh(s), s = (m-1)/(m+1), m in [sqrt(1/2), sqrt(2)];
// log1p through Goldberg's correction log(u) x / (u - 1), u = 1 + x
// ("What every computer scientist should know about floating-point
// arithmetic", 1991, Theorem 4); atanh |x| = log1p(2|x|/(1-|x|))/2 with odd
// symmetry; sin/cos by quadrant reduction with pi/2 split in three parts.
// The includer defines MCRT_HD.
#pragma once

#include <stdint.h>

namespace mcrt {
namespace dm {

// constants as exact hexadecimal literals
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;   // ln 2 to 32 significant bits
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;  // ln 2 - kLn2Hi
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
constexpr double kPio2a = 0x1.921fb54400000p+0;   // pi/2 to 33 bits
constexpr double kPio2b = 0x1.0b4611a600000p-34;  // next 33 bits
constexpr double kPio2c = 0x1.3198a2e037073p-69;  // remainder
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;

// c(j) = 1/j!
MCRT_HD double inv_fact(int j)
{
    constexpr double t[23] = {
        1.0, 1.0, 0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5,
        0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16,
        0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29,
        0x1.6124613a86d09p-33, 0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-41, 0x1.ae7f3e733b81fp-45,
        0x1.952c77030ad4ap-49, 0x1.6827863b97d97p-53, 0x1.2f49b46814157p-57, 0x1.e542ba4020225p-62,
        0x1.71b8ef6dcf572p-66, 0x1.0ce396db7f853p-70};
    return t[j];
}

// 1/(2j+1)
MCRT_HD double inv_odd(int j)
{
    constexpr double t[12] = {
        1.0, 0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3, 0x1.c71c71c71c71cp-4,
        0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4, 0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5,
        0x1.af286bca1af28p-5, 0x1.8618618618618p-5, 0x1.642c8590b2164p-5};
    return t[j];
}

MCRT_HD double bits_to_double(uint64_t b)
{
    double d;
    __builtin_memcpy(&d, &b, sizeof d);
    return d;
}

MCRT_HD uint64_t double_to_bits(double d)
{
    uint64_t b;
    __builtin_memcpy(&b, &d, sizeof b);
    return b;
}

MCRT_HD double two_to(int j) { return bits_to_double((uint64_t)(j + 1023) << 52); }

// p 2^k, rounding at most once (into the subnormal range)
MCRT_HD double ldexp_exact(double p, int k)
{
    if (k > 1023) return p * two_to(1023) * two_to(k - 1023);
    if (k < -1022) return p * two_to(-1022) * two_to(k + 1022);
    return p * two_to(k);
}

MCRT_HD double exp(double x)
{
    if (x != x) return x;
    if (x > 709.782712893384) return __builtin_huge_val();
    if (x < -745.2) return 0.0;
    const double k = floor(x * kInvLn2 + 0.5);
    const double r = (x - k * kLn2Hi) - k * kLn2Lo;
    double p = inv_fact(13);
#pragma unroll
    for (int j = 12; j >= 0; --j) p = p * r + inv_fact(j);
    return ldexp_exact(p, (int)k);
}

MCRT_HD double expm1(double x)
{
    if (x != x) return x;
    if (fabs(x) < 1.0) {
        double p = inv_fact(22);
#pragma unroll
        for (int j = 21; j >= 1; --j) p = p * x + inv_fact(j);
        return x * p;
    }
    return exp(x) - 1.0;
}

MCRT_HD double log(double x)
{
    if (x != x || x < 0.0) return __builtin_nan("");
    if (x == 0.0) return -__builtin_huge_val();
    if (x == __builtin_huge_val()) return x;
    int e = 0;
    if (x < 0x1p-1022) {
        x = x * 0x1p54;
        e = -54;
    }
    uint64_t b = double_to_bits(x);
    e += (int)((b >> 52) & 0x7ff) - 1023;
    double m = bits_to_double((b & 0x000fffffffffffffull) | (0x3ffull << 52));
    if (m > kSqrt2) {
        m = m * 0.5;
        e += 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double s2 = s * s;
    double q = inv_odd(11);
#pragma unroll
    for (int j = 10; j >= 0; --j) q = q * s2 + inv_odd(j);
    const double lm = 2.0 * s * q;
    const double de = (double)e;
    return de * kLn2Hi + (de * kLn2Lo + lm);
}

MCRT_HD double log1p(double x)
{
    if (x != x) return x;
    if (x == -1.0) return -__builtin_huge_val();
    if (x < -1.0) return __builtin_nan("");
    const double u = 1.0 + x;
    if (u == 1.0) return x;
    return log(u) * (x / (u - 1.0));
}

MCRT_HD double atanh(double x)
{
    const double ax = fabs(x);
    const double h = 0.5 * log1p((2.0 * ax) / (1.0 - ax));
    return x < 0.0 ? -h : h;
}

MCRT_HD void sincos(double x, double &sn, double &cs)
{
    const double q = floor(x * kTwoOverPi + 0.5);
    const double r = ((x - q * kPio2a) - q * kPio2b) - q * kPio2c;
    const double r2 = r * r;
    double ps = -inv_fact(19);
#pragma unroll
    for (int j = 8; j >= 0; --j) ps = ((j & 1) ? -inv_fact(2 * j + 1) : inv_fact(2 * j + 1)) + r2 * ps;
    double pc = inv_fact(20);
#pragma unroll
    for (int j = 9; j >= 0; --j) pc = ((j & 1) ? -inv_fact(2 * j) : inv_fact(2 * j)) + r2 * pc;
    const double sr = r * ps, cr = pc;
    const long long n = (long long)q;
    const int quad = (int)(((n % 4) + 4) % 4);
    if (quad == 0) {
        sn = sr;
        cs = cr;
    } else if (quad == 1) {
        sn = cr;
        cs = -sr;
    } else if (quad == 2) {
        sn = -sr;
        cs = -cr;
    } else {
        sn = -cr;
        cs = sr;
    }
}

} // namespace dm
} // namespace mcrt
