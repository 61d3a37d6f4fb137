// recipdiv.hpp -- RN(y / u) by a precomputed reciprocal, for divisors known
// ahead of the dividends (the diagonal of the triangular solve): the same
// bits as div_rn (mp_arith.hpp), the long division only near a rounding
// midpoint.
#pragma once

#include "mp_arith.hpp"

namespace mpg {

// Exact product P (LA + LB limbs) of an LA-limb and an LB-limb mantissa,
// by columns.
template <int LA, int LB>
__device__ __forceinline__ void mul_full2(const uint32_t* a, const uint32_t* b, uint32_t* P)
{
    uint64_t acc = 0;
    uint32_t c2 = 0;
#pragma unroll
    for (int t = 0; t <= LA + LB - 2; t++) {
#pragma unroll
        for (int i = 0; i < LA; i++) {
            const int j = t - i;
            if (j >= 0 && j < LB) mac(acc, c2, a[i], b[j]);
        }
        P[t] = (uint32_t)acc;
        acc = (acc >> 32) | ((uint64_t)c2 << 32);
        c2 = 0;
    }
    P[LA + LB - 1] = (uint32_t)acc;
}

// RN_{p+64}(1 / u) for nonzero u: the correctly rounded reciprocal with two
// more limbs (u's value extended by two zero limbs, 1 = 2^(p+63) 2^(1-(p+64)))
template <int L>
__device__ __forceinline__ MP<L + 2> recip_ext(const MP<L>& u)
{
    MP<L + 2> one, ue;
#pragma unroll
    for (int q = 0; q < L + 1; q++) one.m[q] = 0u;
    one.m[L + 1] = 0x80000000u;
    one.e = 1;
    one.s = 0u;
    ue.m[0] = 0u;
    ue.m[1] = 0u;
#pragma unroll
    for (int q = 0; q < L; q++) ue.m[q + 2] = u.m[q];
    ue.e = u.e;
    ue.s = u.s;
    return div_rn<L + 2>(one, ue);
}

// RN(y / u), the same value as div_rn(y, u), from R = recip_ext(u) when the
// divisor is known ahead (the diagonal of a triangular solve).  The exact
// product Z = M_y M_R (2L + 2 limbs, in [2^(2p+62), 2^(2p+64))) differs from
// the true quotient, scaled alike, by less than |Z| 2^-(p+63) (R's relative
// rounding error is at most 2^-(p+64)): less than 2^-63 of the unit of the
// p-bit result.  So when the round bit and the 59 bits below it (down to
// 2^-60 of the unit) are neither 1 then all zeros nor 0 then all ones, the
// quotient lies on the same side of the rounding midpoint as Z, at least
// 2^-60 - 2^-63 of the unit away from it: RN(quotient) = RN(Z), the round
// bit alone deciding (no tie is possible).  Otherwise (about 2^-58 of the
// cases), and for a zero operand, the long division decides.
template <int L>
__device__ __forceinline__ MP<L> div_by_recip(const MP<L>& y, const MP<L>& u, const MP<L + 2>& R)
{
    if (is_zero(y) || is_zero(u)) return div_rn<L>(y, u);
    uint32_t P[2 * L + 2];
    mul_full2<L, L + 2>(y.m, R.m, P);
    const bool n1 = (P[2 * L + 1] >> 31) != 0;      // Z >= 2^(2p+63): keep limbs L+2 .. 2L+1
    // round bit; W: the bits of limb L+1 below it; V: limb L down to 2^-60 of the unit
    const uint32_t rb = n1 ? (P[L + 1] >> 31) : ((P[L + 1] >> 30) & 1u);
    const uint32_t wmask = n1 ? 0x7fffffffu : 0x3fffffffu;
    const uint32_t W = P[L + 1] & wmask;
    const uint32_t V = n1 ? (P[L] >> 4) : (P[L] >> 3);
    const uint32_t vmask = n1 ? 0x0fffffffu : 0x1fffffffu;
    const bool near = rb ? (W == 0u && V == 0u) : (W == wmask && V == vmask);
    if (near) return div_rn<L>(y, u);
    MP<L> r;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = n1 ? P[k + L + 2] : funnel(P[k + L + 2], P[k + L + 1], 31);
    uint32_t c = rb;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = addc(r.m[k], 0, c, &c);
    if (c) r.m[L - 1] = 0x80000000u;                // rounded up to 2^p
    r.e = y.e + R.e - (n1 ? 0 : 1) + (int32_t)c;
    r.s = y.s ^ u.s;
    return r;
}

}  // namespace mpg
