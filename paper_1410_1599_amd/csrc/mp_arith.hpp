// mp_arith.hpp -- p-bit binary floating point on one GPU lane, round to
// nearest with ties to even after every operation (the paper's MPFR
// arithmetic, Section 3).
//
// A number is MP<L>: L = p/32 uint32 limbs (limb 0 least significant), an
// int32 exponent and a sign word.  value = (-1)^s * M * 2^(e - p) with
// 2^(p-1) <= M < 2^p; zero is M = 0, e = 0, s = 0 (one zero, +0).  A nonzero
// value always has the top bit of limb L-1 set, so "top limb == 0" is the zero
// test.
//
// Exponents: the operations add or subtract exponents in int32; inputs with
// |e| < 2^29 keep every product and quotient exponent of a GEMM or LU in
// range (the library states this as a precondition).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

template <int L>
struct MP {
    uint32_t m[L];
    int32_t e;
    uint32_t s;
};

// ------------------------------------------------------------------ limbs

__device__ __forceinline__ uint32_t addc(uint32_t a, uint32_t b, uint32_t cin, uint32_t* cout)
{
    unsigned int c;
    uint32_t r = __builtin_addc(a, b, cin, &c);
    *cout = c;
    return r;
}

__device__ __forceinline__ uint32_t subb(uint32_t a, uint32_t b, uint32_t bin, uint32_t* bout)
{
    unsigned int c;
    uint32_t r = __builtin_subc(a, b, bin, &c);
    *bout = c;
    return r;
}

// ((hi:lo) >> s)[31:0] for s in [0, 31]
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

__device__ __forceinline__ uint32_t clz32(uint32_t x)
{
    return x ? (uint32_t)__builtin_clz(x) : 32u;
}

// 96-bit column accumulator (acc64 : c2) += a * b.  v_mad_u64_u32 returns
// the carry out of its 64-bit sum in a lane mask, which v_addc adds into c2:
// two VALU instructions per limb product (the compiler's own lowering
// recomputes the carry with a 64-bit compare).  Register operands only.
__device__ __forceinline__ void mac(uint64_t& acc, uint32_t& c2, uint32_t a, uint32_t b)
{
    uint64_t cy, unused;
    asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(cy) : "v"(a), "v"(b));
    asm volatile("v_addc_co_u32_e64 %0, %1, %0, 0, %2" : "+v"(c2), "=s"(unused) : "s"(cy));
}

// the first product of a column: c2 starts from the carry of this product
__device__ __forceinline__ void mac_first(uint64_t& acc, uint32_t& c2, uint32_t a, uint32_t b)
{
    uint64_t cy, unused;
    asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(cy) : "v"(a), "v"(b));
    asm volatile("v_addc_co_u32_e64 %0, %1, 0, 0, %2" : "=v"(c2), "=s"(unused) : "s"(cy));
}

// acc = a * b (no carry out)
__device__ __forceinline__ void mac_init(uint64_t& acc, uint32_t a, uint32_t b)
{
    uint64_t unused;
    asm volatile("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(acc), "=s"(unused) : "v"(a), "v"(b));
}

// M_a < M_b for L-limb mantissas: one subtract-with-borrow chain whose final
// borrow is the answer (the compiler's own lowering of the unused differences
// is a compare per limb and a scalar mask chain)
template <int L>
__device__ __forceinline__ bool mant_less(const uint32_t* a, const uint32_t* b)
{
    uint64_t bw;
    uint32_t d;
    asm volatile("v_sub_co_u32_e64 %0, %1, %2, %3" : "=v"(d), "=s"(bw) : "v"(a[0]), "v"(b[0]));
#pragma unroll
    for (int k = 1; k < L; k++)
        asm volatile("v_subb_co_u32_e64 %0, %1, %2, %3, %1" : "=v"(d), "+s"(bw) : "v"(a[k]), "v"(b[k]));
    (void)d;
    uint32_t r;                               // this lane's bit of the borrow mask
    asm volatile("v_cndmask_b32_e64 %0, 0, 1, %1" : "=v"(r) : "s"(bw));
    return r != 0;
}

template <int L>
__device__ __forceinline__ MP<L> mp_zero()
{
    MP<L> r;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = 0;
    r.e = 0;
    r.s = 0;
    return r;
}

template <int L>
__device__ __forceinline__ bool is_zero(const MP<L>& x)
{
    return x.m[L - 1] == 0;
}

template <int L>
__device__ __forceinline__ MP<L> select(bool c, const MP<L>& a, const MP<L>& b)
{
    MP<L> r;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = c ? a.m[k] : b.m[k];
    r.e = c ? a.e : b.e;
    r.s = c ? a.s : b.s;
    return r;
}

// ------------------------------------------------------------------ plane layout

// element idx of a matrix whose limb k sits at base[k * ps + idx], exponent at
// base[L * ps + idx], sign at base[(L + 1) * ps + idx]
template <int L>
__device__ __forceinline__ MP<L> load(const uint32_t* __restrict__ base, int64_t ps, int64_t idx)
{
    MP<L> x;
#pragma unroll
    for (int k = 0; k < L; k++) x.m[k] = base[k * ps + idx];
    x.e = (int32_t)base[L * ps + idx];
    x.s = base[(L + 1) * ps + idx];
    return x;
}

template <int L>
__device__ __forceinline__ void store(uint32_t* __restrict__ base, int64_t ps, int64_t idx, const MP<L>& x)
{
#pragma unroll
    for (int k = 0; k < L; k++) base[k * ps + idx] = x.m[k];
    base[L * ps + idx] = (uint32_t)x.e;
    base[(L + 1) * ps + idx] = x.s;
}

// ------------------------------------------------------------------ multiply

// Exact 2L-limb product P of two L-limb mantissas, by columns.
template <int L>
__device__ __forceinline__ void mul_full(const uint32_t* a, const uint32_t* b, uint32_t* P)
{
    uint64_t acc = 0;
    uint32_t c2 = 0;
#pragma unroll
    for (int t = 0; t <= 2 * L - 2; t++) {
#pragma unroll
        for (int i = 0; i < L; i++) {
            const int j = t - i;
            if (j >= 0 && j < L) mac(acc, c2, a[i], b[j]);
        }
        P[t] = (uint32_t)acc;
        acc = (acc >> 32) | ((uint64_t)c2 << 32);
        c2 = 0;
    }
    P[2 * L - 1] = (uint32_t)acc;
}

// RN(a * b).
//
// Fast path: only the columns t >= L-2 of the product are formed (the
// products a_i b_j with i + j >= L-2).  The columns left out add less than
// L-1 units of limb L-1 and the fraction held in limb L-2 less than one more,
// so the true value of the product's limb L-1 and below lies in
// [h, h + L) in units of limb L-1, h being the computed limb.  When that
// whole interval is on one side of the rounding midpoint and cannot carry into
// the kept limbs, the rounding is decided; otherwise (probability about
// 2L / 2^31 per product) the exact product is formed and rounded from it.
template <int L>
__device__ __forceinline__ MP<L> mul_rn(const MP<L>& a, const MP<L>& b)
{
    static_assert(L >= 3, "the truncated product needs L >= 3");
    uint32_t H[L + 2];                       // H[k] = column L-2+k
    {
        uint64_t acc = 0;
        uint32_t c2 = 0;
#pragma unroll
        for (int t = L - 2; t <= 2 * L - 2; t++) {
            bool first = true;
#pragma unroll
            for (int i = 0; i < L; i++) {
                const int j = t - i;
                if (j < 0 || j >= L) continue;
                if (first && t == L - 2) mac_init(acc, a.m[i], b.m[j]);
                else if (first) mac_first(acc, c2, a.m[i], b.m[j]);
                else mac(acc, c2, a.m[i], b.m[j]);
                first = false;
            }
            H[t - (L - 2)] = (uint32_t)acc;
            acc = (acc >> 32) | ((uint64_t)c2 << 32);
            c2 = 0;
        }
        H[L + 1] = (uint32_t)acc;
    }
    bool n1 = (H[L + 1] >> 31) != 0;         // product in [2^(2p-1), 2^(2p))
    const uint32_t h = n1 ? H[1] : (H[1] & 0x7fffffffu);
    const uint32_t half = n1 ? 0x80000000u : 0x40000000u;
    const uint32_t top = n1 ? 0xffffffffu : 0x7fffffffu;
    const bool down = h <= half - (uint32_t)L;
    const bool upq = (h > half) && (h <= top - (uint32_t)L + 1u);
    uint32_t up = upq ? 1u : 0u;
    if (!(down || upq)) {
        uint32_t P[2 * L];
        mul_full<L>(a.m, b.m, P);
#pragma unroll
        for (int k = 0; k < L + 2; k++) H[k] = P[L - 2 + k];
        n1 = (P[2 * L - 1] >> 31) != 0;
        uint32_t low = 0;
#pragma unroll
        for (int k = 0; k < L - 1; k++) low |= P[k];
        const uint32_t rb = n1 ? (P[L - 1] >> 31) : ((P[L - 1] >> 30) & 1u);
        const uint32_t st = (n1 ? (P[L - 1] & 0x7fffffffu) : (P[L - 1] & 0x3fffffffu)) | low;
        const uint32_t lsb = n1 ? (P[L] & 1u) : (P[L - 1] >> 31);
        up = rb & ((st != 0) | lsb);
    }
    MP<L> r;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = n1 ? H[k + 2] : funnel(H[k + 2], H[k + 1], 31);
    uint32_t c = up;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = addc(r.m[k], 0, c, &c);
    if (c) r.m[L - 1] = 0x80000000u;         // 2^p: the others are already 0
    // a zero factor makes H zero, so the mantissa is already zero: only the
    // exponent and sign need the canonical zero
    const bool z = is_zero(a) || is_zero(b);
    r.e = z ? 0 : a.e + b.e - (n1 ? 0 : 1) + (int32_t)c;
    r.s = z ? 0u : (a.s ^ b.s);
    return r;
}

// ------------------------------------------------------------------ add

// T[0..L] = (M * 2^32) >> r for r in [0, 31] (exact: nothing leaves the
// bottom of the guard limb)
template <int L>
__device__ __forceinline__ void align_bits(const uint32_t* m, uint32_t r, uint32_t* T)
{
    T[0] = funnel(m[0], 0u, r);
#pragma unroll
    for (int k = 1; k < L; k++) T[k] = funnel(m[k], m[k - 1], r);
    T[L] = m[L - 1] >> r;
}

// (X * 2^32 + (T ^ mk) + (mk & 1)): the guard-limb sum or difference,
// carry out in c
template <int L>
__device__ __forceinline__ void add_window(const uint32_t* xm, const uint32_t* T, uint32_t mk, uint32_t* R,
                                           uint32_t& c)
{
    c = mk & 1u;
    R[0] = addc(0u, T[0] ^ mk, c, &c);
#pragma unroll
    for (int k = 1; k <= L; k++) R[k] = addc(xm[k - 1], T[k] ^ mk, c, &c);
}

// any of the low s bits of the L-limb mantissa m set (s < 32 L)
template <int L>
__device__ __forceinline__ bool lost_bits(const uint32_t* m, uint32_t s)
{
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < L; k++) {
        const uint32_t lo = 32u * k;
        const uint32_t mask = s >= lo + 32u ? 0xffffffffu : (s > lo ? (1u << (s - lo)) - 1u : 0u);
        acc |= m[k] & mask;
    }
    return acc != 0;
}

// RN(x + y).  Works on an (L+1)-limb extension R = |X| * 2^32 of the larger
// operand: a guard limb under the mantissa.  The smaller operand Y is shifted
// right by the exponent gap d.  A gap below 32 shifts nothing out of the
// guard limb (the common case, a funnel shift per limb); when any lane of the
// wave has a larger gap, the whole wave takes a whole-limb shift in binary
// stages (two stages while every gap is below 128, all of them otherwise).
// The bits of Y that fall below the guard limb are not carried along: they
// can only decide an exact tie in R, which the rounding step detects and
// resolves from Y directly.
template <int L>
__device__ __forceinline__ MP<L> add_rn(const MP<L>& x, const MP<L>& y)
{
    const bool zx = is_zero(x), zy = is_zero(y);
    // |y| > |x| for nonzero operands: the exponents, then the top limbs, and
    // the whole mantissas only when some lane of the wave has both equal
    const bool eqe = y.e == x.e;
    bool mlt = x.m[L - 1] < y.m[L - 1];
    const bool tie = eqe && (x.m[L - 1] == y.m[L - 1]);
    if (__builtin_amdgcn_ballot_w64(tie) != 0) {
        const bool full = mant_less<L>(x.m, y.m);
        mlt = tie ? full : mlt;
    }
    const bool ygt = (y.e > x.e) || (eqe && mlt);
    const bool sw = zy ? false : (zx ? true : ygt);
    const MP<L> X = select(sw, y, x);
    const MP<L> Y = select(sw, x, y);
    const bool yz = sw ? zx : zy;
    const uint32_t d = yz ? 0u : (uint32_t)(X.e - Y.e);
    const bool subt = X.s != Y.s;

    // T = Y * 2^(32 - d): Y aligned below X's guard limb.  For d < 32 this
    // is exact.  For larger d the bits of Y below the window are dropped
    // here; see the rounding step for where they count.
    uint32_t T[L + 1];
    if (__builtin_amdgcn_ballot_w64(d >= 32u) == 0) {
        align_bits<L>(Y.m, d, T);
    } else if (__builtin_amdgcn_ballot_w64(d >= 128u) == 0) {
        // gaps below 128: whole-limb shifts by q = d/32 <= 3, two stages
        const uint32_t q = d >> 5;
        align_bits<L>(Y.m, d & 31u, T);
#pragma unroll
        for (int b = 1; b <= 2; b <<= 1) {
            const bool on = (q & (uint32_t)b) != 0;
#pragma unroll
            for (int k = 0; k <= L; k++) T[k] = on ? ((k + b <= L) ? T[k + b] : 0u) : T[k];
        }
    } else {                                  // whole-limb shift by q = d/32, in binary stages
        const uint32_t dc = d < 32u * (L + 1) ? d : 32u * (L + 1);
        const uint32_t q = dc >> 5;
        align_bits<L>(Y.m, dc & 31u, T);
#pragma unroll
        for (int b = 1; b <= L + 1; b <<= 1) {
            const bool on = (q & (uint32_t)b) != 0;
#pragma unroll
            for (int k = 0; k <= L; k++) T[k] = on ? ((k + b <= L) ? T[k + b] : 0u) : T[k];
        }
        if (d >= 32u * (L + 1)) T[0] = 1u;    // Y entirely below the window: a sticky bit
    }

    // R = X*2^32 +- T
    const uint32_t mk = subt ? 0xffffffffu : 0u;
    uint32_t R[L + 1];
    uint32_t c;
    add_window<L>(X.m, T, mk, R, c);
    int32_t e = X.e;
    if (!subt && c) {                         // sum reached 2^(p+32): shift right once
        const uint32_t lost = R[0] & 1u;
#pragma unroll
        for (int k = 0; k < L; k++) R[k] = funnel(R[k + 1], R[k], 1);
        R[L] = 0x80000000u | (R[L] >> 1);
        R[0] |= lost;
        e += 1;
    }
    const bool deep = subt && (R[L] == 0);    // cancellation of a whole limb or more (rare)
    if (__builtin_expect(deep, 0)) {
        uint32_t q = 0;
        bool still = true;
#pragma unroll
        for (int k = L; k >= 0; k--) {
            still = still && (R[k] == 0);
            q += still ? 1u : 0u;
        }
#pragma unroll
        for (int b = 1; b <= L + 1; b <<= 1) {
            if (q & (uint32_t)b) {
#pragma unroll
                for (int k = L; k >= 0; k--) R[k] = (k - b >= 0) ? R[k - b] : 0u;
            }
        }
        e -= (int32_t)(32u * q);
    }
    const uint32_t z = clz32(R[L]) & 31u;     // R[L] == 0 only for an exact zero
    if (z) {
#pragma unroll
        for (int k = L; k >= 1; k--) R[k] = funnel(R[k], R[k - 1], 32u - z);
        R[0] <<= z;
    }
    e -= (int32_t)z;

    // round to the p bits R[1..L].  When 32 <= d < 32(L+1) the exact sum
    // differs from R by the dropped bits of Y, less than one unit of R's
    // bit 0 (added, or taken away for a difference); at most one bit has
    // cancelled, so the rounding position is bit 30 or above and the dropped
    // bits decide only an exact tie in R: above it for a sum (round up),
    // below it for a difference (round down).
    const uint32_t rb = R[0] >> 31;
    const uint32_t st = (R[0] & 0x7fffffffu) ? 1u : 0u;
    uint32_t cu = rb & (st | (R[1] & 1u));
    if (rb && !st && d >= 32u && d < 32u * (L + 1)) {
        if (lost_bits<L>(Y.m, d - 32u)) cu = subt ? 0u : 1u;
    }
    MP<L> r;
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = addc(R[k + 1], 0, cu, &cu);
    if (cu) {
        r.m[L - 1] = 0x80000000u;
        e += 1;
    }
    // an exact zero (cancellation, or both operands zero) leaves every limb
    // zero; give it the canonical exponent and sign (+0)
    const bool rz = r.m[L - 1] == 0;
    r.e = rz ? 0 : e;
    r.s = rz ? 0u : X.s;
    return r;
}

template <int L>
__device__ __forceinline__ MP<L> neg(const MP<L>& x)
{
    MP<L> r = x;
    r.s = is_zero(x) ? 0u : (x.s ^ 1u);
    return r;
}

template <int L>
__device__ __forceinline__ MP<L> sub_rn(const MP<L>& x, const MP<L>& y)
{
    return add_rn<L>(x, neg<L>(y));
}

// ------------------------------------------------------------------ compare, divide

// |x| compared with |y|: -1, 0, 1
template <int L>
__device__ __forceinline__ int cmp_abs(const MP<L>& x, const MP<L>& y)
{
    const bool zx = is_zero(x), zy = is_zero(y);
    if (zx || zy) return (int)(!zx) - (int)(!zy);
    if (x.e != y.e) return x.e > y.e ? 1 : -1;
#pragma unroll
    for (int k = L - 1; k >= 0; k--)
        if (x.m[k] != y.m[k]) return x.m[k] > y.m[k] ? 1 : -1;
    return 0;
}

// RN(x / y), y nonzero: true division, not a reciprocal.
//
// Long division in radix 2^32 (Knuth's Algorithm D) of Mx * 2^(32(L+1)) by
// My, which is already normalised (top bit set): L+2 quotient digits
// Q = floor(Mx 2^(32(L+1)) / My) and a remainder.  Q has p+32 or p+33 bits,
// so after keeping p bits the round bit is known and everything below it,
// with the remainder, is the sticky bit.
//
// Digit estimate: with R the (L+1)-limb window of the running remainder
// (R < 2^32 My) and N, D its top three and My's top two limbs, the true digit
// floor(R / My) and N / D differ by less than 2^-30 plus an integer step,
// and N / D evaluated in double precision as N * (1 / D) is off by less than
// 2^-18 (five roundings of values below 2^96 and 2^64, relative 2^-53 each,
// on a quotient below 2^33).  So the floor of the double estimate is the digit
// or one off either way; the multiply-subtract is corrected by adding My back
// or subtracting it once more (two rounds of each are allowed).
template <int L>
__device__ __forceinline__ MP<L> div_rn(const MP<L>& x, const MP<L>& y)
{
    static_assert(L >= 3, "the digit estimate needs L >= 3");
    const uint32_t* v = y.m;
    const double D = (double)v[L - 1] * 4294967296.0 + (double)v[L - 2];
    const double invD = 1.0 / D;
    uint32_t R[L + 1], Q[L + 2];
#pragma unroll
    for (int k = 0; k < L; k++) R[k] = x.m[k];
    R[L] = 0;
#pragma unroll
    for (int k = 0; k < L + 2; k++) Q[k] = 0;
#pragma unroll
    for (int step = 0; step < L + 2; step++) {
        const double N = ((double)R[L] * 4294967296.0 + (double)R[L - 1]) * 4294967296.0 + (double)R[L - 2];
        double qd = floor(N * invD);
        qd = qd > 4294967295.0 ? 4294967295.0 : qd;
        uint32_t qh = (uint32_t)qd;
        // R -= qh * My
        uint32_t bw = 0, pc = 0;
#pragma unroll
        for (int k = 0; k < L; k++) {
            const uint64_t pr = (uint64_t)qh * v[k] + pc;
            pc = (uint32_t)(pr >> 32);
            R[k] = subb(R[k], (uint32_t)pr, bw, &bw);
        }
        R[L] = subb(R[L], pc, bw, &bw);
        // negative: add My back (a carry out of the top limb ends it)
#pragma unroll
        for (int it = 0; it < 2; it++) {
            if (bw) {
                uint32_t c = 0;
#pragma unroll
                for (int k = 0; k < L; k++) R[k] = addc(R[k], v[k], c, &c);
                R[L] = addc(R[L], 0u, c, &c);
                qh -= 1;
                bw = c ? 0u : 1u;
            }
        }
        // still >= My: subtract once more (a second time only if the first
        // went through)
#pragma unroll
        for (int it = 0; it < 2; it++) {
            uint32_t b2 = 0, T[L + 1];
#pragma unroll
            for (int k = 0; k < L; k++) T[k] = subb(R[k], v[k], b2, &b2);
            T[L] = subb(R[L], 0u, b2, &b2);
            if (b2) break;
#pragma unroll
            for (int k = 0; k <= L; k++) R[k] = T[k];
            qh += 1;
        }
#pragma unroll
        for (int k = L + 1; k >= 1; k--) Q[k] = Q[k - 1];
        Q[0] = qh;
        // next window: R (now < My) times 2^32, bringing in a zero limb
#pragma unroll
        for (int k = L; k >= 1; k--) R[k] = R[k - 1];
        R[0] = 0;
    }
    // the last shift above multiplied the remainder by 2^32; it is only tested
    // for zero
    uint32_t rem = 0;
#pragma unroll
    for (int k = 0; k <= L; k++) rem |= R[k];
    const bool big = Q[L + 1] != 0;           // Mx >= My: p+33 bits
    MP<L> r;
    uint32_t rb, st;
    if (big) {
#pragma unroll
        for (int k = 0; k < L; k++) r.m[k] = funnel(Q[k + 2], Q[k + 1], 1);
        rb = Q[1] & 1u;
        st = Q[0] | rem;
    } else {
#pragma unroll
        for (int k = 0; k < L; k++) r.m[k] = Q[k + 1];
        rb = Q[0] >> 31;
        st = (Q[0] & 0x7fffffffu) | rem;
    }
    uint32_t cu = rb & ((st != 0) | (r.m[0] & 1u));
#pragma unroll
    for (int k = 0; k < L; k++) r.m[k] = addc(r.m[k], 0, cu, &cu);
    int32_t e = x.e - y.e + (big ? 1 : 0);
    if (cu) {
        r.m[L - 1] = 0x80000000u;
        e += 1;
    }
    r.e = e;
    r.s = x.s ^ y.s;
    if (is_zero(x)) r = mp_zero<L>();
    return r;
}

}  // namespace mpg
