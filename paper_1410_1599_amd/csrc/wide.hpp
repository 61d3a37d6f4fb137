// wide.hpp -- p-bit binary floating point held by a whole wavefront, for
// p = 2048, 4096, 8192, 10240 (the paper's high precisions, Sections 3 and 4): the
// same number format and rounding as mp_arith.hpp, one correctly rounded
// result (to nearest, ties to even) per operation.
//
// A value is WMP<L> (L = 64 R limbs): lane t holds limbs R t .. R t + R - 1 of
// the mantissa (limb 0 least significant, so lane 63 holds the top); the
// exponent and sign are the same in every lane.  Every routine here must be
// called by all 64 lanes of a wave with the same arguments' uniform parts:
// lanes talk through ds_bpermute, readlane and ballots only (no LDS, no
// memory), and every branch on data is on a wave-uniform value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mp_arith.hpp"

namespace mpg {

template <int L>
struct WMP {
    static constexpr int R = L / 64;
    uint32_t m[L / 64];
    int32_t e;
    uint32_t s;
};

template <int L>
constexpr bool is_wide() { return L >= 64; }

__device__ __forceinline__ int wlane() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t wballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }
__device__ __forceinline__ uint32_t wuni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t wread(uint32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
// value v of lane src (src in [0, 63]); every lane must be active (a
// disabled source lane reads as 0), so it is never called under a condition
// that differs between lanes
__device__ __forceinline__ uint32_t wperm(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ int top_bit64(uint64_t x) { return 63 - __builtin_clzll(x); }

// register k (k the same in every lane) of an R-register set
template <int R>
__device__ __forceinline__ uint32_t pick(const uint32_t (&m)[R], int k)
{
    uint32_t v = m[0];
#pragma unroll
    for (int q = 1; q < R; q++) v = (k == q) ? m[q] : v;
    return v;
}

template <int L>
__device__ __forceinline__ WMP<L> wzero()
{
    WMP<L> r;
#pragma unroll
    for (int k = 0; k < L / 64; k++) r.m[k] = 0;
    r.e = 0;
    r.s = 0;
    return r;
}

// limb g (g the same in every lane) as a wave-uniform value; 0 outside [0, L)
template <int L>
__device__ __forceinline__ uint32_t wlimb(const uint32_t (&m)[L / 64], int g)
{
    constexpr int R = L / 64;
    if (g < 0 || g >= L) return 0u;
    return wread(pick<R>(m, g % R), g / R);
}

// out[r] = limb R t + r + off of m in lane t (off the same in every lane),
// 0 outside [0, L)
template <int L>
__device__ __forceinline__ void wshift_limbs(const uint32_t (&m)[L / 64], int off, uint32_t (&out)[L / 64])
{
    constexpr int R = L / 64;
    const int t = wlane();
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int g = R * t + r + off;
        const int sr = (((r + off) % R) + R) % R;   // source register: the same in every lane
        const int sl = (g - sr) / R;                  // source lane (exact division)
        const uint32_t v = wperm(pick<R>(m, sr), sl & 63);
        out[r] = (g >= 0 && g < L) ? v : 0u;
    }
}

template <int L>
__device__ __forceinline__ bool wis_zero(const WMP<L>& x)
{
    return wlimb<L>(x.m, L - 1) == 0u;
}

// x + y + cin over L limbs (cin 0 or 1, the same in every lane); returns the
// carry out of the top limb.  Each lane adds its own limbs; the carries
// between lanes come from one 64-bit addition of the lanes' generate and
// propagate masks (carry into lane t = bit t of (G|P) + G + cin, xor G|P, xor G).
template <int L>
__device__ __forceinline__ uint32_t wadd(const uint32_t (&x)[L / 64], const uint32_t (&y)[L / 64], uint32_t cin,
                                         uint32_t (&z)[L / 64])
{
    constexpr int R = L / 64;
    uint32_t c = 0;
    bool ones = true;
#pragma unroll
    for (int r = 0; r < R; r++) {
        z[r] = addc(x[r], y[r], c, &c);
        ones = ones && (z[r] == 0xffffffffu);
    }
    const uint64_t G = wballot(c != 0), P = wballot(ones);
    const uint64_t GP = G | P;
    const uint64_t u = GP + G;
    const uint64_t s = u + (uint64_t)cin;
    const uint32_t cout = (u < GP || s < u) ? 1u : 0u;
    uint32_t ci = (uint32_t)(((s ^ GP ^ G) >> wlane()) & 1u);
#pragma unroll
    for (int r = 0; r < R; r++) z[r] = addc(z[r], 0u, ci, &ci);
    return cout;
}

// sign of M_a - M_b
template <int L>
__device__ __forceinline__ int wcmp_mant(const uint32_t (&a)[L / 64], const uint32_t (&b)[L / 64])
{
    constexpr int R = L / 64;
    bool diff = false, gt = false;
#pragma unroll
    for (int r = R - 1; r >= 0; r--) {
        if (!diff && a[r] != b[r]) {
            diff = true;
            gt = a[r] > b[r];
        }
    }
    const uint64_t dm = wballot(diff);
    if (dm == 0) return 0;
    const int tl = top_bit64(dm);
    return ((wballot(gt) >> tl) & 1u) ? 1 : -1;
}

// sign of |x| - |y|
template <int L>
__device__ __forceinline__ int cmp_abs(const WMP<L>& x, const WMP<L>& y)
{
    const bool zx = wis_zero<L>(x), zy = wis_zero<L>(y);
    if (zx || zy) return zx ? (zy ? 0 : -1) : 1;
    if (x.e != y.e) return x.e > y.e ? 1 : -1;
    return wcmp_mant<L>(x.m, y.m);
}

// m := m + cu at limb 0 (cu 0 or 1); a carry out of the top (m was all ones)
// leaves 2^(p-1) and adds one to e
template <int L>
__device__ __forceinline__ void wround_up(uint32_t (&m)[L / 64], uint32_t cu, int32_t& e)
{
    constexpr int R = L / 64;
    if (!cu) return;
    uint32_t zero[R];
#pragma unroll
    for (int r = 0; r < R; r++) zero[r] = 0u;
    if (wadd<L>(m, zero, 1u, m)) {
        if (wlane() == 63) m[R - 1] = 0x80000000u;   // the other limbs wrapped to zero
        e += 1;
    }
}

// RN(x + y).  Y (the smaller magnitude) is aligned below X with a 64-bit
// guard held as two wave-uniform words and every lower bit of Y folded into
// the guard's lowest bit (a nonzero tail sits at least 62 bits below the
// rounding position after the at most one-bit normalisation that can follow
// an inexact alignment, so it only acts as the sticky bit); gaps of at most
// one bit are exact.  A gap of p + 2 or more leaves X: |Y| < ulp(X) / 4.
template <int L>
__device__ __forceinline__ WMP<L> add_rn(const WMP<L>& x, const WMP<L>& y)
{
    constexpr int R = L / 64;
    constexpr uint32_t p = 32u * L;
    const int t = wlane();
    const bool zx = wis_zero<L>(x), zy = wis_zero<L>(y);
    if (zy) return zx ? wzero<L>() : x;
    if (zx) return y;
    const bool ygt = (y.e > x.e) || (y.e == x.e && wcmp_mant<L>(y.m, x.m) > 0);
    WMP<L> X, Y;
#pragma unroll
    for (int r = 0; r < R; r++) {
        X.m[r] = ygt ? y.m[r] : x.m[r];
        Y.m[r] = ygt ? x.m[r] : y.m[r];
    }
    X.e = ygt ? y.e : x.e;
    Y.e = ygt ? x.e : y.e;
    X.s = ygt ? y.s : x.s;
    Y.s = ygt ? x.s : y.s;
    const uint32_t d = (uint32_t)(X.e - Y.e);
    if (d >= p + 2u) return X;
    const bool subt = X.s != Y.s;
    const int q = (int)(d >> 5);
    const uint32_t sh = d & 31u;

    // T = Y >> d: limb j = (Y[j+q+1] : Y[j+q]) >> sh
    uint32_t y0[R], y1[R], T[R];
    wshift_limbs<L>(Y.m, q, y0);
    wshift_limbs<L>(Y.m, q + 1, y1);
#pragma unroll
    for (int r = 0; r < R; r++) T[r] = funnel(y1[r], y0[r], sh);
    // guard limbs -1 and -2 of Y >> d, and the sticky OR of Y's bits below d - 64
    const uint32_t yq = wlimb<L>(Y.m, q), yq1 = wlimb<L>(Y.m, q - 1), yq2 = wlimb<L>(Y.m, q - 2);
    const uint32_t gh = funnel(yq, yq1, sh);
    uint32_t gl = funnel(yq1, yq2, sh);
    bool st = false;
    if (d > 64u) {
        const uint32_t s0 = d - 64u;
        const int kq = (int)(s0 >> 5);
        const uint32_t kb = s0 & 31u;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int g = R * t + r;
            if (g < kq) st = st || (Y.m[r] != 0u);
            else if (g == kq && kb) st = st || ((Y.m[r] & ((1u << kb) - 1u)) != 0u);
        }
    }
    if (wballot(st) != 0) gl |= 1u;

    uint32_t M[R];
    uint32_t grh, grl, cout = 0;
    if (!subt) {
        cout = wadd<L>(X.m, T, 0u, M);
        grh = gh;
        grl = gl;
    } else {
        // X 2^64 - (T 2^64 + G): the guard part first, then X - T - borrow
        const uint64_t G = ((uint64_t)gh << 32) | gl;
        const uint64_t Gn = (uint64_t)0 - G;
        grh = (uint32_t)(Gn >> 32);
        grl = (uint32_t)Gn;
        uint32_t Tn[R];
#pragma unroll
        for (int r = 0; r < R; r++) Tn[r] = ~T[r];
        wadd<L>(X.m, Tn, G != 0 ? 0u : 1u, M);
    }
    int32_t e = X.e;
    if (cout) {
        // (1 : M : guard) >> 1, the bit leaving the guard kept as sticky
        uint32_t up[R];
        wshift_limbs<L>(M, 1, up);
        const uint32_t m0 = wlimb<L>(M, 0);
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t hi = (R * t + r == L - 1) ? 1u : up[r];
            M[r] = funnel(hi, M[r], 1u);
        }
        const uint32_t lost = grl & 1u;
        grl = funnel(grh, grl, 1u) | lost;
        grh = funnel(m0, grh, 1u);
        e += 1;
    } else if (subt) {
        // leading zeros of (M : guard); a shift of two or more bits only
        // follows a gap of at most one bit, where nothing was dropped
        bool nzl = false;
        int topr = 0;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (M[r] != 0u) {
                nzl = true;
                topr = r;
            }
        const uint64_t nz = wballot(nzl);
        uint32_t z;
        if (nz != 0) {
            const int tl = top_bit64(nz);
            const int tr = (int)wread((uint32_t)topr, tl);
            const uint32_t tv = wlimb<L>(M, R * tl + tr);
            z = 32u * (uint32_t)(L - 1 - (R * tl + tr)) + (uint32_t)__builtin_clz(tv);
        } else if (grh != 0u) {
            z = 32u * L + (uint32_t)__builtin_clz(grh);
        } else if (grl != 0u) {
            z = 32u * L + 32u + (uint32_t)__builtin_clz(grl);
        } else {
            return wzero<L>();                      // exact cancellation: +0
        }
        if (z > 0) {
            const int qz = (int)(z >> 5);
            const uint32_t bz = z & 31u;
            uint32_t a0[R], a1[R];
            wshift_limbs<L>(M, -qz, a0);
            wshift_limbs<L>(M, -qz - 1, a1);
            // limbs below M are the guard (index -1, -2), then zeros
            auto below = [&](int idx) -> uint32_t { return idx == -1 ? grh : (idx == -2 ? grl : 0u); };
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int ia = R * t + r - qz;
                const uint32_t va = ia >= 0 ? a0[r] : below(ia);
                const uint32_t vb = ia - 1 >= 0 ? a1[r] : below(ia - 1);
                M[r] = bz ? funnel(va, vb, 32u - bz) : va;
            }
            const uint32_t h1 = below(-1 - qz), h2 = below(-2 - qz), h3 = below(-3 - qz);
            const uint32_t ngh = bz ? funnel(h1, h2, 32u - bz) : h1;
            const uint32_t ngl = bz ? funnel(h2, h3, 32u - bz) : h2;
            grh = ngh;
            grl = ngl;
            e -= (int32_t)z;
        }
    }
    // round to nearest even at the guard
    const uint32_t rb = grh >> 31;
    const bool sticky = ((grh & 0x7fffffffu) | grl) != 0u;
    const uint32_t lsb = wlimb<L>(M, 0) & 1u;
    wround_up<L>(M, rb & ((sticky ? 1u : 0u) | lsb), e);
    WMP<L> res;
#pragma unroll
    for (int r = 0; r < R; r++) res.m[r] = M[r];
    res.e = e;
    res.s = X.s;
    return res;
}

template <int L>
__device__ __forceinline__ WMP<L> neg(const WMP<L>& x)
{
    WMP<L> r = x;
    r.s = wis_zero<L>(x) ? 0u : (x.s ^ 1u);
    return r;
}

template <int L>
__device__ __forceinline__ WMP<L> sub_rn(const WMP<L>& x, const WMP<L>& y)
{
    return add_rn<L>(x, neg<L>(y));
}

// RN(a b).  Lane t forms the low product columns R t + k and the high ones
// L + R t + k (k < R), column c = sum_i a_i b_(c-i) in 96-bit accumulators.
// At step s column k of the lane takes a_(s+k) (a wave-uniform value, read
// from its lane) times b_((R t - s) mod L), the same b limb for all k (one
// ds_bpermute per step): for s <= R t that is a term of the low column, for
// s > R t of the high one, so every lane does exactly L R limb products and
// switches its accumulators once, at s = R t + 1, which is a block boundary
// of the R-step blocks below.  The columns are then carried into 2L limbs (a
// lane's carry-out goes to the next lane of its half, the low half's last lane
// feeds the high half's first, and the one-bit carries that remain travel by
// a 128-lane ballot lookahead): the high half is already the mantissa's lane
// layout, and its top p bits are rounded.
template <int L>
__device__ __forceinline__ WMP<L> mul_rn(const WMP<L>& a, const WMP<L>& b)
{
    constexpr int R = L / 64;
    constexpr int NB = (L + R - 1 + R - 1) / R;       // blocks covering s = 1 - R .. L - 1
    const int t = wlane();
    if (wis_zero<L>(a) || wis_zero<L>(b)) return wzero<L>();
    uint64_t acc[R], accl[R];
    uint32_t c2[R], c2l[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        acc[k] = 0;
        c2[k] = 0;
        accl[k] = 0;
        c2l[k] = 0;
    }
    uint32_t bnext[R];
#pragma unroll
    for (int u = 0; u < R; u++) bnext[u] = wperm(b.m[R - 1 - u], t & 63);
    for (int q = 0; q < NB; q++) {
        // block q: s = R (q - 1) + 1 + u, u < R; lane q - 1 leaves its low columns
        if (t == q - 1) {
#pragma unroll
            for (int k = 0; k < R; k++) {
                accl[k] = acc[k];
                c2l[k] = c2[k];
                acc[k] = 0;
                c2[k] = 0;
            }
        }
        // a_(s+k) for this block: limbs R (q - 1) + 1 + v, v < 2R - 1
        uint32_t aw[2 * R - 1];
#pragma unroll
        for (int v = 0; v < 2 * R - 1; v++) {
            const int g = R * (q - 1) + 1 + v;
            const uint32_t x = wread(a.m[(1 + v) % R], (q - 1 + (1 + v) / R) & 63);
            aw[v] = (g >= 0 && g < L) ? x : 0u;
        }
        // b_((R t - s) mod L) = limb R ((t - q) mod 64) + R - 1 - u, fetched
        // one block ahead so the permute latency hides under the products
        uint32_t bw[R];
#pragma unroll
        for (int u = 0; u < R; u++) bw[u] = bnext[u];
        {
            const int src = (t - q - 1) & 63;
#pragma unroll
            for (int u = 0; u < R; u++) bnext[u] = wperm(b.m[R - 1 - u], src);
        }
#pragma unroll
        for (int u = 0; u < R; u++) {
            uint64_t cy[R];
#pragma unroll
            for (int k = 0; k < R; k++)
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "=s"(cy[k]) : "v"(aw[u + k]), "v"(bw[u]));
#pragma unroll
            for (int k = 0; k < R; k++) {
                uint64_t unused;
                asm volatile("v_addc_co_u32_e64 %0, %1, %0, 0, %2" : "+v"(c2[k]), "=s"(unused) : "s"(cy[k]));
            }
        }
    }
    if (t >= NB - 1) {                                 // lanes whose switch lies past the last block
#pragma unroll
        for (int k = 0; k < R; k++) {
            accl[k] = acc[k];
            c2l[k] = c2[k];
            acc[k] = 0;
            c2[k] = 0;
        }
    }
    // columns -> limbs, low half PL and high half PH, and each lane's carry-out (< 2^43)
    uint32_t PL[R], PH[R];
    uint64_t cyl = 0, cyh = 0;
#pragma unroll
    for (int k = 0; k < R; k++) {
        uint64_t lo = accl[k] + cyl;
        uint32_t hi = c2l[k] + (lo < cyl ? 1u : 0u);
        PL[k] = (uint32_t)lo;
        cyl = (lo >> 32) | ((uint64_t)hi << 32);
        lo = acc[k] + cyh;
        hi = c2[k] + (lo < cyh ? 1u : 0u);
        PH[k] = (uint32_t)lo;
        cyh = (lo >> 32) | ((uint64_t)hi << 32);
    }
    const int prev = (t - 1) & 63;
    const uint32_t l0 = wperm((uint32_t)cyl, prev), l1 = wperm((uint32_t)(cyl >> 32), prev);
    const uint32_t h0 = wperm((uint32_t)cyh, prev), h1 = wperm((uint32_t)(cyh >> 32), prev);
    const uint64_t inl = t > 0 ? (((uint64_t)l1 << 32) | l0) : 0u;
    const uint64_t inh = t > 0 ? (((uint64_t)h1 << 32) | h0) : (((uint64_t)l1 << 32) | l0);   // lane 0: low lane 63
    uint32_t gl = 0, gh = 0;
    bool onesl = true, onesh = true;
    if constexpr (R == 1) {
        // one limb per lane: the incoming carry (< 2^43) leaves up to 2^11
        // over, which goes one lane further before only one-bit carries remain
        const uint64_t vl = (uint64_t)PL[0] + inl, vh = (uint64_t)PH[0] + inh;
        PL[0] = (uint32_t)vl;
        PH[0] = (uint32_t)vh;
        const uint32_t ol = (uint32_t)(vl >> 32), oh = (uint32_t)(vh >> 32);
        const uint32_t pol = wperm(ol, prev), poh = wperm(oh, prev);
        const uint32_t il = t > 0 ? pol : 0u, ih = t > 0 ? poh : pol;
        PL[0] = addc(PL[0], il, 0u, &gl);
        PH[0] = addc(PH[0], ih, 0u, &gh);
        onesl = PL[0] == 0xffffffffu;
        onesh = PH[0] == 0xffffffffu;
    } else {
        PL[0] = addc(PL[0], (uint32_t)inl, 0u, &gl);
        PH[0] = addc(PH[0], (uint32_t)inh, 0u, &gh);
        PL[1] = addc(PL[1], (uint32_t)(inl >> 32), gl, &gl);
        PH[1] = addc(PH[1], (uint32_t)(inh >> 32), gh, &gh);
#pragma unroll
        for (int k = 2; k < R; k++) {
            PL[k] = addc(PL[k], 0u, gl, &gl);
            PH[k] = addc(PH[k], 0u, gh, &gh);
        }
#pragma unroll
        for (int k = 0; k < R; k++) {
            onesl = onesl && (PL[k] == 0xffffffffu);
            onesh = onesh && (PH[k] == 0xffffffffu);
        }
    }
    {
        // 128-lane lookahead: low lanes then high lanes
        const uint64_t Gl = wballot(gl != 0), Pl = wballot(onesl), Gh = wballot(gh != 0), Ph = wballot(onesh);
        const uint64_t GPl = Gl | Pl, GPh = Gh | Ph;
        const uint64_t lo = GPl + Gl;
        const uint64_t hi = GPh + Gh + (lo < GPl ? 1u : 0u);
        uint32_t cl = (uint32_t)(((lo ^ GPl ^ Gl) >> t) & 1u);
        uint32_t ch = (uint32_t)(((hi ^ GPh ^ Gh) >> t) & 1u);
#pragma unroll
        for (int k = 0; k < R; k++) {
            PL[k] = addc(PL[k], 0u, cl, &cl);
            PH[k] = addc(PH[k], 0u, ch, &ch);
        }
    }
    const uint32_t ptop = wread(PH[R - 1], 63);
    const uint32_t pl1 = wread(PL[R - 1], 63);           // product limb L - 1
    const bool n1 = (ptop >> 31) != 0;
    bool lowl = false;                                     // product limbs 0 .. L - 2
#pragma unroll
    for (int k = 0; k < R; k++)
        if (R * t + k <= L - 2) lowl = lowl || (PL[k] != 0u);
    const bool low = wballot(lowl) != 0;
    uint32_t M[R];
    uint32_t rb, st;
    if (n1) {
#pragma unroll
        for (int r = 0; r < R; r++) M[r] = PH[r];
        rb = pl1 >> 31;
        st = (pl1 & 0x7fffffffu) != 0u || low;
    } else {
        uint32_t Hd[R];
        wshift_limbs<L>(PH, -1, Hd);
#pragma unroll
        for (int r = 0; r < R; r++) M[r] = funnel(PH[r], (R * t + r == 0) ? pl1 : Hd[r], 31u);
        rb = (pl1 >> 30) & 1u;
        st = (pl1 & 0x3fffffffu) != 0u || low;
    }
    int32_t e = a.e + b.e - (n1 ? 0 : 1);
    const uint32_t lsb = wlimb<L>(M, 0) & 1u;
    wround_up<L>(M, rb & (st | lsb), e);
    WMP<L> res;
#pragma unroll
    for (int r = 0; r < R; r++) res.m[r] = M[r];
    res.e = e;
    res.s = a.s ^ b.s;
    return res;
}

// R := R - q M_y over the L lane-layout limbs of R and its top limb rh (q <
// 2^32, the same in every lane); returns 1 if the result is negative (a
// borrow out of rh).  Each lane runs its own multiply-subtract chain; what
// it owes the next lane (the high product word and the borrow, at most 2^32)
// is passed on by ds_bpermute and subtracted there, and the one-bit borrows
// that remain travel by the ballot lookahead.
template <int L>
__device__ __forceinline__ uint32_t wsub_mul(uint32_t (&Rl)[L / 64], uint32_t& rh, uint32_t q,
                                             const uint32_t (&v)[L / 64])
{
    constexpr int R = L / 64;
    const int t = wlane();
    uint32_t pc = 0, bw = 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint64_t pr = (uint64_t)q * v[r] + pc;
        pc = (uint32_t)(pr >> 32);
        Rl[r] = subb(Rl[r], (uint32_t)pr, bw, &bw);
    }
    // permute with every lane active (an inactive source lane reads as 0),
    // then drop lane 0's wrapped-around value
    const uint32_t pp = wperm(pc, (t - 1) & 63), pb = wperm(bw, (t - 1) & 63);
    const uint32_t in_pc = t > 0 ? pp : 0u;
    const uint32_t in_bw = t > 0 ? pb : 0u;
    uint32_t b = 0;
    Rl[0] = subb(Rl[0], in_pc, in_bw, &b);
    bool zeros = Rl[0] == 0u;
#pragma unroll
    for (int r = 1; r < R; r++) {
        Rl[r] = subb(Rl[r], 0u, b, &b);
        zeros = zeros && (Rl[r] == 0u);
    }
    const uint64_t G = wballot(b != 0), P = wballot(zeros);
    const uint64_t GP = G | P;
    const uint64_t u = GP + G;
    const uint32_t top_b = u < GP ? 1u : 0u;
    uint32_t bi = (uint32_t)(((u ^ GP ^ G) >> t) & 1u);
#pragma unroll
    for (int r = 0; r < R; r++) Rl[r] = subb(Rl[r], 0u, bi, &bi);
    const uint32_t top_pc = wread(pc, 63), top_bw = wread(bw, 63);
    uint32_t b1, b2;
    rh = subb(rh, top_pc, top_bw, &b1);
    rh = subb(rh, 0u, top_b, &b2);
    return b1 | b2;
}

// RN(x / y), y nonzero: radix-2^32 long division (Knuth D) of
// M_x 2^(32(L+1)) by M_y, the same steps and digit estimate as the one-lane
// div_rn (mp_arith.hpp): the digit from the remainder's top three limbs and
// M_y's top two in double precision is the true digit or one off either way,
// corrected by adding M_y back or subtracting it once more.  The quotient
// has p + 32 or p + 33 bits, so the round bit is exact and the rest plus the
// remainder is the sticky bit.  True division, never a reciprocal multiply.
template <int L>
__device__ __forceinline__ WMP<L> div_rn(const WMP<L>& x, const WMP<L>& y)
{
    constexpr int R = L / 64;
    const int t = wlane();
    if (wis_zero<L>(x)) return wzero<L>();
    const double D = (double)wlimb<L>(y.m, L - 1) * 4294967296.0 + (double)wlimb<L>(y.m, L - 2);
    const double invD = 1.0 / D;
    uint32_t Rl[R], Qw[R], nv[R];
    uint32_t rh = 0, q_top = 0, q_last = 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        Rl[r] = x.m[r];
        Qw[r] = 0u;
        nv[r] = ~y.m[r];
    }
    for (int step = 0; step < L + 2; step++) {
        const double N = ((double)rh * 4294967296.0 + (double)wlimb<L>(Rl, L - 1)) * 4294967296.0 +
                         (double)wlimb<L>(Rl, L - 2);
        double qd = floor(N * invD);
        qd = qd > 4294967295.0 ? 4294967295.0 : qd;
        uint32_t qh = wuni((uint32_t)qd);
        uint32_t neg = wsub_mul<L>(Rl, rh, qh, y.m);
        // negative: add M_y back (a carry out of the top limb ends it)
#pragma unroll
        for (int it = 0; it < 2; it++) {
            if (neg) {
                const uint32_t c = wadd<L>(Rl, y.m, 0u, Rl);
                uint32_t c2;
                rh = addc(rh, 0u, c, &c2);
                qh -= 1;
                neg = c2 ? 0u : 1u;
            }
        }
        // still >= M_y: subtract once more (a second time only if the first went through)
#pragma unroll
        for (int it = 0; it < 2; it++) {
            uint32_t T[R];
            const uint32_t c = wadd<L>(Rl, nv, 1u, T);    // carry out: no borrow from the L limbs
            uint32_t b2;
            const uint32_t th = subb(rh, 0u, c ? 0u : 1u, &b2);
            if (b2) break;
#pragma unroll
            for (int r = 0; r < R; r++) Rl[r] = T[r];
            rh = th;
            qh += 1;
        }
        // digit `step` is quotient limb L + 1 - step: the top one, the L
        // mantissa-window limbs (lane layout), the last one
        if (step == 0) {
            q_top = qh;
        } else if (step <= L) {
            const int k = L - step;
            if (t == k / R) {
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (r == k % R) Qw[r] = qh;
            }
        } else {
            q_last = qh;
        }
        // next window: the remainder (now < M_y) times 2^32
        rh = wlimb<L>(Rl, L - 1);
        uint32_t sh[R];
        wshift_limbs<L>(Rl, -1, sh);
#pragma unroll
        for (int r = 0; r < R; r++) Rl[r] = sh[r];
    }
    bool reml = false;
#pragma unroll
    for (int r = 0; r < R; r++) reml = reml || (Rl[r] != 0u);
    const bool rem = wballot(reml) != 0 || rh != 0u;
    const bool big = q_top != 0u;                 // M_x >= M_y: p + 33 bits
    uint32_t M[R], rb, st;
    if (big) {
        uint32_t up[R];
        wshift_limbs<L>(Qw, 1, up);
#pragma unroll
        for (int r = 0; r < R; r++) M[r] = funnel((R * t + r == L - 1) ? q_top : up[r], Qw[r], 1u);
        rb = wlimb<L>(Qw, 0) & 1u;
        st = (q_last != 0u || rem) ? 1u : 0u;
    } else {
#pragma unroll
        for (int r = 0; r < R; r++) M[r] = Qw[r];
        rb = q_last >> 31;
        st = ((q_last & 0x7fffffffu) != 0u || rem) ? 1u : 0u;
    }
    int32_t e = x.e - y.e + (big ? 1 : 0);
    const uint32_t lsb = wlimb<L>(M, 0) & 1u;
    wround_up<L>(M, rb & (st | lsb), e);
    WMP<L> res;
#pragma unroll
    for (int r = 0; r < R; r++) res.m[r] = M[r];
    res.e = e;
    res.s = x.s ^ y.s;
    return res;
}

// ------------------------------------------------------------------ memory

// element idx of a matrix in the plane layout: lane t loads limbs R t .. R t + R - 1
template <int L>
__device__ __forceinline__ WMP<L> wload(const uint32_t* __restrict__ base, int64_t ps, int64_t idx)
{
    constexpr int R = L / 64;
    const int t = wlane();
    WMP<L> x;
#pragma unroll
    for (int r = 0; r < R; r++) x.m[r] = base[(int64_t)(R * t + r) * ps + idx];
    x.e = (int32_t)wuni(base[(int64_t)L * ps + idx]);
    x.s = wuni(base[(int64_t)(L + 1) * ps + idx]);
    return x;
}

template <int L>
__device__ __forceinline__ void wstore(uint32_t* __restrict__ base, int64_t ps, int64_t idx, const WMP<L>& x)
{
    constexpr int R = L / 64;
    const int t = wlane();
#pragma unroll
    for (int r = 0; r < R; r++) base[(int64_t)(R * t + r) * ps + idx] = x.m[r];
    if (t == 0) {
        base[(int64_t)L * ps + idx] = (uint32_t)x.e;
        base[(int64_t)(L + 1) * ps + idx] = x.s;
    }
}

}  // namespace mpg
