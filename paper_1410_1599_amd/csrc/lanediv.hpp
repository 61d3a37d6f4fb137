// lanediv.hpp -- RN(x / y) computed by a whole wavefront for the narrow
// precisions (L = 4 .. 32 limbs), one limb per lane.
//
// The one-lane div_rn (mp_arith.hpp) runs L + 2 serial digit steps, each an
// L-limb multiply-subtract with its carries and borrows passed limb to limb:
// at 512 bits one division takes about 6 us of a single lane, which is on the
// critical path of every LU column (the multipliers l_ic = a_ic / a_cc).
// Here lane t holds limb t of the
// running remainder and of the divisor (lanes t >= L hold zeros), so a digit
// step is one multiply per lane; what a lane owes the next one (the high
// product word and its borrow) moves up by one DPP lane shift, and the
// remaining one-bit borrows travel by a ballot lookahead over the lanes.
//
// The digit estimate, its corrections and the rounding are those of div_rn
// (Knuth's Algorithm D in radix 2^32, the digit from the remainder's top
// three limbs and the divisor's top two in double precision, then at most
// two add-backs or two further subtractions), so the quotient, the round bit
// and the sticky bit, and with them the result, are the same bits.
//
// Every routine must be called by all 64 lanes of the wave (uniform control
// flow); values in the lane layout are one uint32 per lane, exponent and sign
// are wave-uniform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mp_arith.hpp"

namespace mpg {

template <int L>
__device__ __forceinline__ uint64_t lane_mask()
{
    static_assert(L >= 3 && L <= 62, "one limb per lane, with room above");
    return (uint64_t(1) << L) - 1;
}

// lane t gets lane t - 1's value (lane 0 gets 0): DPP wave_shr:1
__device__ __forceinline__ uint32_t lane_up(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}

// lane t gets lane t + 1's value (lane 63 gets 0): DPP wave_shl:1
__device__ __forceinline__ uint32_t lane_down(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}

// limb k as a wave-uniform value (0 outside [0, L))
template <int L>
__device__ __forceinline__ uint32_t lane_limb(uint32_t v, int k)
{
    return (k >= 0 && k < L) ? __builtin_amdgcn_readlane(v, k) : 0u;
}

// z = x + y + cin over the L limbs (cin 0 or 1, uniform); returns the carry
// out of limb L - 1.  Carry into lane t: bit t of (G|P) + G + cin, xor G|P,
// xor G, with G the lanes whose own addition carried and P those whose sum is
// all ones.
template <int L>
__device__ __forceinline__ uint32_t lane_add(uint32_t x, uint32_t y, uint32_t cin, uint32_t& z)
{
    const uint64_t M = lane_mask<L>();
    const int t = (int)__lane_id();
    uint32_t c;
    z = addc(x, y, 0u, &c);
    const uint64_t G = __builtin_amdgcn_ballot_w64(c != 0u) & M;
    const uint64_t P = __builtin_amdgcn_ballot_w64(z == 0xffffffffu) & M;
    const uint64_t GP = G | P;
    const uint64_t cv = (GP + G + (uint64_t)cin) ^ GP ^ G;      // bit t: carry into lane t
    const uint32_t ci = t < L ? (uint32_t)((cv >> t) & 1u) : 0u;
    z += ci;
    return (uint32_t)((cv >> L) & 1u);
}

// R := R - q * Y over the L limbs of R and its top limb rh (q uniform, below
// 2^32); returns 1 when the result is negative (a borrow out of rh).
template <int L>
__device__ __forceinline__ uint32_t lane_sub_mul(uint32_t& R, uint32_t& rh, uint32_t q, uint32_t y)
{
    const uint64_t M = lane_mask<L>();
    const int t = (int)__lane_id();
    const uint64_t pr = (uint64_t)q * y;
    const uint32_t pc = (uint32_t)(pr >> 32);
    uint32_t bw;
    R = subb(R, (uint32_t)pr, 0u, &bw);
    // what lane t - 1 owes: its high product word and its borrow (lanes from
    // L on take nothing: lane L - 1's debt goes to rh below)
    uint32_t in_pc = lane_up(pc), in_bw = lane_up(bw);
    in_pc = t < L ? in_pc : 0u;
    in_bw = t < L ? in_bw : 0u;
    uint32_t b;
    R = subb(R, in_pc, in_bw, &b);
    const uint64_t G = __builtin_amdgcn_ballot_w64(b != 0u) & M;
    const uint64_t P = __builtin_amdgcn_ballot_w64(R == 0u) & M;
    const uint64_t GP = G | P;
    const uint64_t bv = (GP + G) ^ GP ^ G;                       // bit t: borrow into lane t
    const uint32_t bi = t < L ? (uint32_t)((bv >> t) & 1u) : 0u;
    R -= bi;
    const uint32_t top_b = (uint32_t)((bv >> L) & 1u);
    uint32_t b1, b2;
    rh = subb(rh, lane_limb<L>(pc, L - 1), lane_limb<L>(bw, L - 1), &b1);
    rh = subb(rh, 0u, top_b, &b2);
    return b1 | b2;
}

// RN(x / y) with y nonzero, x and y in the lane layout (xm, ym: this lane's
// limb; exponents and signs uniform).  Returns this lane's limb of the
// quotient's mantissa (0 for lanes >= L); *re and *rs get its exponent and
// sign.  The same steps and bits as div_rn.
template <int L>
__device__ __forceinline__ uint32_t lane_div_rn(uint32_t xm, int32_t xe, uint32_t xs, uint32_t ym, int32_t ye,
                                                uint32_t ys, int32_t* re, uint32_t* rs)
{
    const int t = (int)__lane_id();
    if (lane_limb<L>(xm, L - 1) == 0u) {      // x = 0
        *re = 0;
        *rs = 0u;
        return 0u;
    }
    const double D = (double)lane_limb<L>(ym, L - 1) * 4294967296.0 + (double)lane_limb<L>(ym, L - 2);
    const double invD = 1.0 / D;
    const uint32_t ny = t < L ? ~ym : 0u;
    uint32_t R = t < L ? xm : 0u;
    uint32_t rh = 0u, Qw = 0u, q_top = 0u, q_last = 0u;
    for (int step = 0; step < L + 2; step++) {
        const double N = ((double)rh * 4294967296.0 + (double)lane_limb<L>(R, L - 1)) * 4294967296.0 +
                         (double)lane_limb<L>(R, L - 2);
        double qd = floor(N * invD);
        qd = qd > 4294967295.0 ? 4294967295.0 : qd;
        uint32_t qh = __builtin_amdgcn_readfirstlane((uint32_t)qd);
        uint32_t neg = lane_sub_mul<L>(R, rh, qh, t < L ? ym : 0u);
        // negative: add the divisor back (a carry out of the top limb ends it)
#pragma unroll
        for (int it = 0; it < 2; it++) {
            if (neg) {
                const uint32_t c = lane_add<L>(R, t < L ? ym : 0u, 0u, R);
                uint32_t c2;
                rh = addc(rh, 0u, c, &c2);
                qh -= 1;
                neg = c2 ? 0u : 1u;
            }
        }
        // still >= the divisor: subtract once more (a second time only if the
        // first went through).  With no top limb left and R's top limb below
        // the divisor's, R is below it: no test subtraction needed.
#pragma unroll
        for (int it = 0; it < 2; it++) {
            if (rh == 0u && lane_limb<L>(R, L - 1) < lane_limb<L>(ym, L - 1)) break;
            uint32_t T;
            const uint32_t c = lane_add<L>(R, ny, 1u, T);          // carry out: no borrow from the L limbs
            uint32_t b2;
            const uint32_t th = subb(rh, 0u, c ? 0u : 1u, &b2);
            if (b2) break;
            R = t < L ? T : 0u;
            rh = th;
            qh += 1;
        }
        // digit `step` is quotient limb L + 1 - step: the top one, the L
        // mantissa-window limbs (limb k + 1 in lane k), the last one
        if (step == 0) q_top = qh;
        else if (step <= L) Qw = (t == L - step) ? qh : Qw;
        else q_last = qh;
        // next window: the remainder (now below the divisor) times 2^32
        rh = lane_limb<L>(R, L - 1);
        const uint32_t up = lane_up(R);
        R = t < L ? up : 0u;
    }
    const bool rem = __builtin_amdgcn_ballot_w64(R != 0u) != 0 || rh != 0u;
    const bool big = q_top != 0u;                 // M_x >= M_y: p + 33 bits
    uint32_t M, rb, st;
    if (big) {
        uint32_t up = lane_down(Qw);
        up = (t == L - 1) ? q_top : up;
        M = t < L ? funnel(up, Qw, 1u) : 0u;
        rb = lane_limb<L>(Qw, 0) & 1u;
        st = (q_last != 0u || rem) ? 1u : 0u;
    } else {
        M = Qw;
        rb = q_last >> 31;
        st = ((q_last & 0x7fffffffu) != 0u || rem) ? 1u : 0u;
    }
    int32_t e = xe - ye + (big ? 1 : 0);
    const uint32_t lsb = lane_limb<L>(M, 0) & 1u;
    const uint32_t cu = rb & (st | lsb);
    const uint32_t cout = lane_add<L>(M, 0u, cu, M);
    if (cout) {                                   // rounded up to 2^p
        M = (t == L - 1) ? 0x80000000u : 0u;
        e += 1;
    }
    *re = e;
    *rs = xs ^ ys;
    return M;
}

}  // namespace mpg
