// phase.hpp -- unit phases exp(-i x) for arbitrary real x in fp64 on gfx950
// and sign flips, shared by the pass kernels and the sector kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "hubvqe.hpp"

namespace hv {

// x with its sign bit flipped when bit (0 or 1) is set: a Jordan-Wigner sign
// applied without a select.
__device__ __forceinline__ double flip_sign(double x, uint32_t bit)
{
    return __longlong_as_double(__double_as_longlong(x) ^ ((long long)bit << 63));
}

// exp(-i x) for the general diagonal: x = k h + r with h = 2 pi / 2^kCisBits
// (Cody-Waite reduction with a two-part h whose leading part has 36
// significant bits, exact for |k| < 2^17), the phase of k h from the LDS
// table cis[k mod 2^kCisBits] = (cos kh, sin kh), and cos r, sin r by their
// Taylor series (|r| <= pi / 2^kCisBits, truncation below 1e-19).
__device__ __forceinline__ double2 cis_neg(double x, const double2 *cis)
{
    constexpr double kInvH = 0x1.45f306dc9c883p+5;    // 2^kCisBits / (2 pi), kCisBits = 8
    constexpr double kHHi = 0x1.921fb54440000p-6;     // 2 pi / 2^kCisBits, leading part
    constexpr double kHLo = 0x1.68c234c4c6629p-45;    // remainder
    const double k = rint(x * kInvH);
    double r = fma(-k, kHHi, x);
    r = fma(-k, kHLo, r);
    const double2 t = cis[(int)k & ((1 << kCisBits) - 1)];
    const double r2 = r * r;
    const double c = fma(r2, fma(r2, fma(r2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    const double sr = r * fma(r2, fma(r2, fma(r2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
    // cos x = cos kh cos r - sin kh sin r, sin x = sin kh cos r + cos kh sin r
    return make_double2(t.x * c - t.y * sr, -(t.y * c + t.x * sr));
}

// The table cis[m] = (cos, sin)(2 pi m / 2^kCisBits) that cis_neg reads,
// built by the threads of a workgroup (tid, T).
__device__ __forceinline__ void build_cis(double2 *cis, int tid, int T)
{
    for (int m = tid; m < (1 << kCisBits); m += T) {
        double s, c;
        sincospi((double)m / (double)(1 << (kCisBits - 1)), &s, &c);
        cis[m] = make_double2(c, s);
    }
}

}  // namespace hv
