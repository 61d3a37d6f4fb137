/*
 * mpref.c -- CPU oracle for p-bit MP matrix products and LU (plain C, OpenMP).
 *
 * TEST INFRASTRUCTURE ONLY.  The library never links or calls this file; only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
 * shares no code with the GPU path.
 *
 * It performs the same sequence of correctly rounded scalar operations as the
 * Python oracle (oracle/mpnum.py, oracle/gemm.py, oracle/lu.py), for sizes the
 * Python oracle cannot reach, and it is cross-checked against that oracle on
 * small shapes.  Every operation forms its exact result as a multi-limb
 * integer and rounds it once (round_pack).  Nothing is tuned.
 *
 * Number model (the paper's MPFR arithmetic, Section 3): a value is
 * (-1)^neg * M * 2^(e - p) with 2^(p-1) <= M < 2^p, or zero (M = 0, e = 0,
 * neg = 0).  p is a multiple of 32 here, L = p / 32 limbs, limb 0 least
 * significant.
 *
 * Matrix interface: the plane layout of include/mpgemm.h, read and written by
 * this file's own loaders: element (i, j) of a matrix with leading dimension
 * ld and plane stride ps keeps limb k at w[k*ps + i*ld + j], the exponent
 * (int32) at w[L*ps + i*ld + j] and the sign (0/1) at w[(L+1)*ps + i*ld + j].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifndef MAXL
#define MAXL 48              /* up to 1536 bits (the residual runs at 2p+64); the wide build sets 656 */
#endif
#define WIDE (2 * MAXL + 8)

typedef struct {
    int neg;
    int64_t e;
    uint32_t m[MAXL];
} mpv;

/* ------------------------------------------------------------------ scalar */

static int is_zero(const mpv *x, int L)
{
    for (int k = 0; k < L; k++)
        if (x->m[k]) return 0;
    return 1;
}

static void set_zero(mpv *x)
{
    memset(x, 0, sizeof *x);
}

/* bit length of the nw-limb integer w (0 for w = 0) */
static int64_t bitlen(const uint32_t *w, int nw)
{
    for (int k = nw - 1; k >= 0; k--)
        if (w[k]) {
            int b = 32;
            uint32_t t = w[k];
            while (!(t & 0x80000000u)) { t <<= 1; b--; }
            return (int64_t)k * 32 + b;
        }
    return 0;
}

static int get_bit(const uint32_t *w, int nw, int64_t i)
{
    if (i < 0 || i >= (int64_t)nw * 32) return 0;
    return (w[i >> 5] >> (i & 31)) & 1;
}

/* out[0..no) = floor(w / 2^s) restricted to no limbs */
static void shr(uint32_t *out, int no, const uint32_t *w, int nw, int64_t s)
{
    int64_t q = s >> 5;
    int r = (int)(s & 31);
    for (int k = 0; k < no; k++) {
        int64_t a = k + q;
        uint64_t lo = (a < nw) ? w[a] : 0;
        uint64_t hi = (a + 1 < nw) ? w[a + 1] : 0;
        out[k] = (uint32_t)(((hi << 32) | lo) >> r);
    }
}

/* out[0..no) = w * 2^s (s >= 0), truncated to no limbs */
static void shl(uint32_t *out, int no, const uint32_t *w, int nw, int64_t s)
{
    int64_t q = s >> 5;
    int r = (int)(s & 31);
    for (int k = no - 1; k >= 0; k--) {
        int64_t a = k - q;
        uint64_t hi = (a >= 0 && a < nw) ? w[a] : 0;
        uint64_t lo = (a - 1 >= 0 && a - 1 < nw) ? w[a - 1] : 0;
        out[k] = (uint32_t)((((hi << 32) | lo) << r) >> 32);
    }
}

/* any bit of w below bit position s set? */
static int sticky_below(const uint32_t *w, int nw, int64_t s)
{
    int64_t full = s >> 5;                       /* whole limbs below s */
    for (int64_t k = 0; k < full && k < nw; k++)
        if (w[k]) return 1;
    if (full < nw && (s & 31))
        if (w[full] & ((1u << (s & 31)) - 1u)) return 1;
    return 0;
}

/*
 * r := RN_p((-1)^neg * W * 2^f), W the nw-limb integer w.
 * Keep the top p bits, round to nearest with ties to the even mantissa.
 */
static void round_pack(mpv *r, const uint32_t *w, int nw, int neg, int64_t f, int L)
{
    int p = 32 * L;
    int64_t b = bitlen(w, nw);
    if (b == 0) { set_zero(r); return; }
    uint32_t q[MAXL + 1];
    if (b > p) {
        int64_t s = b - p;
        shr(q, L + 1, w, nw, s);                 /* p kept bits (+ an empty limb) */
        int rb = get_bit(w, nw, s - 1);
        int st = sticky_below(w, nw, s - 1);
        if (rb && (st || (q[0] & 1))) {
            uint64_t c = 1;
            for (int k = 0; k < L + 1; k++) {
                c += q[k];
                q[k] = (uint32_t)c;
                c >>= 32;
            }
            if (bitlen(q, L + 1) > p) {          /* reached 2^p */
                shr(q, L + 1, q, L + 1, 1);
                s += 1;
            }
        }
        f += s;
    } else {
        shl(q, L + 1, w, nw, p - b);
        f -= (p - b);
    }
    memcpy(r->m, q, sizeof(uint32_t) * L);
    for (int k = L; k < MAXL; k++) r->m[k] = 0;
    r->e = f + p;
    r->neg = neg;
}

static void mp_mul(mpv *r, const mpv *x, const mpv *y, int L)
{
    if (is_zero(x, L) || is_zero(y, L)) { set_zero(r); return; }
    uint32_t w[2 * MAXL];
    memset(w, 0, sizeof(uint32_t) * 2 * L);
    for (int i = 0; i < L; i++) {                /* schoolbook, exact */
        uint64_t c = 0;
        for (int j = 0; j < L; j++) {
            uint64_t t = (uint64_t)x->m[i] * y->m[j] + w[i + j] + c;
            w[i + j] = (uint32_t)t;
            c = t >> 32;
        }
        w[i + L] = (uint32_t)c;
    }
    int p = 32 * L;
    round_pack(r, w, 2 * L, x->neg ^ y->neg, (x->e - p) + (y->e - p), L);
}

/* compare nw-limb magnitudes */
static int cmp_w(const uint32_t *a, const uint32_t *b, int nw)
{
    for (int k = nw - 1; k >= 0; k--)
        if (a[k] != b[k]) return a[k] > b[k] ? 1 : -1;
    return 0;
}

/* r := RN(x + (-1)^negy * |y|) (negy flips y's sign for subtraction) */
static void mp_addsigned(mpv *r, const mpv *x, const mpv *y, int flip, int L)
{
    int p = 32 * L;
    mpv yy = *y;
    if (flip && !is_zero(&yy, L)) yy.neg ^= 1;
    if (is_zero(x, L)) { *r = yy; return; }
    if (is_zero(&yy, L)) { *r = *x; return; }
    /* gap of p+3 or more: the smaller operand is under a quarter ulp */
    if (x->e - yy.e >= p + 3) { *r = *x; return; }
    if (yy.e - x->e >= p + 3) { *r = yy; return; }
    int64_t e0 = x->e < yy.e ? x->e : yy.e;
    int nw = L + (p + 3) / 32 + 3;
    uint32_t X[WIDE], Y[WIDE], S[WIDE];
    shl(X, nw, x->m, L, x->e - e0);              /* exact alignment */
    shl(Y, nw, yy.m, L, yy.e - e0);
    int neg;
    if (x->neg == yy.neg) {
        uint64_t c = 0;
        for (int k = 0; k < nw; k++) {
            c += (uint64_t)X[k] + Y[k];
            S[k] = (uint32_t)c;
            c >>= 32;
        }
        neg = x->neg;
    } else {
        int cm = cmp_w(X, Y, nw);
        if (cm == 0) { set_zero(r); return; }
        const uint32_t *big = cm > 0 ? X : Y, *sml = cm > 0 ? Y : X;
        int64_t br = 0;
        for (int k = 0; k < nw; k++) {
            int64_t t = (int64_t)big[k] - sml[k] - br;
            br = t < 0;
            S[k] = (uint32_t)(t + (br << 32));
        }
        neg = cm > 0 ? x->neg : yy.neg;
    }
    round_pack(r, S, nw, neg, e0 - p, L);
}

static void mp_add(mpv *r, const mpv *x, const mpv *y, int L) { mp_addsigned(r, x, y, 0, L); }
static void mp_sub(mpv *r, const mpv *x, const mpv *y, int L) { mp_addsigned(r, x, y, 1, L); }

/* r := RN(x / y), y != 0: restoring long division, then one rounding */
static void mp_div(mpv *r, const mpv *x, const mpv *y, int L)
{
    int p = 32 * L;
    if (is_zero(x, L)) { set_zero(r); return; }
    int k = p + 3;
    int nw = 2 * L + 2;
    uint32_t N[WIDE], Q[WIDE], R[WIDE], D[WIDE];
    memset(N, 0, sizeof N); memset(Q, 0, sizeof Q); memset(R, 0, sizeof R); memset(D, 0, sizeof D);
    shl(N, nw, x->m, L, k);                      /* N = Mx * 2^k */
    memcpy(D, y->m, sizeof(uint32_t) * L);
    int64_t nb = bitlen(N, nw);
    for (int64_t i = nb - 1; i >= 0; i--) {      /* one quotient bit per step */
        shl(R, nw, R, nw, 1);
        R[0] |= (uint32_t)get_bit(N, nw, i);
        if (cmp_w(R, D, nw) >= 0) {
            int64_t br = 0;
            for (int t = 0; t < nw; t++) {
                int64_t v = (int64_t)R[t] - D[t] - br;
                br = v < 0;
                R[t] = (uint32_t)(v + (br << 32));
            }
            Q[i >> 5] |= 1u << (i & 31);
        }
    }
    int st = 0;
    for (int t = 0; t < nw; t++) if (R[t]) st = 1;
    /* value = (Q + st/2) * 2^(ex - ey - k): append the sticky bit below Q */
    uint32_t Q2[WIDE];
    shl(Q2, nw + 1, Q, nw, 1);
    Q2[0] |= (uint32_t)st;
    round_pack(r, Q2, nw + 1, x->neg ^ y->neg, x->e - y->e - k - 1, L);
}

/* |x| vs |y| */
static int mp_cmpabs(const mpv *x, const mpv *y, int L)
{
    int zx = is_zero(x, L), zy = is_zero(y, L);
    if (zx || zy) return (!zx) - (!zy);
    if (x->e != y->e) return x->e > y->e ? 1 : -1;
    return cmp_w(x->m, y->m, L);
}

/* ------------------------------------------------------------------ matrices */

/* a matrix held by the oracle: row-major array of mpv */
typedef struct {
    mpv *v;
    int64_t rows, cols, ld;
} mat;

#define AT(M, i, j) ((M).v[(int64_t)(i) * (M).ld + (j)])

static mat mat_new(int64_t rows, int64_t cols)
{
    mat M;
    M.rows = rows; M.cols = cols; M.ld = cols > 0 ? cols : 1;
    M.v = (mpv *)calloc((size_t)(rows > 0 ? rows : 1) * M.ld, sizeof(mpv));
    return M;
}

static mat mat_view(mat M, int64_t r0, int64_t c0, int64_t rows, int64_t cols)
{
    mat V = M;
    V.v = M.v + r0 * M.ld + c0;
    V.rows = rows; V.cols = cols;
    return V;
}

static void mat_free(mat M) { free(M.v); }

static void load(mat M, const uint32_t *w, int64_t ld, int64_t ps, int L)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M.rows; i++)
        for (int64_t j = 0; j < M.cols; j++) {
            mpv *x = &AT(M, i, j);
            int64_t idx = i * ld + j;
            memset(x, 0, sizeof *x);
            for (int k = 0; k < L; k++) x->m[k] = w[k * ps + idx];
            x->e = (int32_t)w[L * ps + idx];
            x->neg = w[(L + 1) * ps + idx] ? 1 : 0;
            if (is_zero(x, L)) set_zero(x);
        }
}

static int store(mat M, uint32_t *w, int64_t ld, int64_t ps, int L)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t i = 0; i < M.rows; i++)
        for (int64_t j = 0; j < M.cols; j++) {
            const mpv *x = &AT(M, i, j);
            int64_t idx = i * ld + j;
            for (int k = 0; k < L; k++) w[k * ps + idx] = x->m[k];
            if (x->e > INT32_MAX || x->e < INT32_MIN) bad = 1;
            w[L * ps + idx] = (uint32_t)(int32_t)x->e;
            w[(L + 1) * ps + idx] = (uint32_t)x->neg;
        }
    return bad ? -6 : 0;
}

enum { ALG_SIMPLE = 0, ALG_BLOCK = 1, ALG_STRASSEN = 2, ALG_WINOGRAD = 3 };
enum { POL_PEEL = 0, POL_PAD = 1, POL_MIXED = 2 };

/* eq. (1): c_ij = sum_k a_ik b_kj, k ascending, from exact zero */
static void simple(mat C, mat A, mat B, int L)
{
    int64_t m = C.rows, n = C.cols, l = A.cols;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) {
            mpv c, t;
            set_zero(&c);
            for (int64_t k = 0; k < l; k++) {
                mp_mul(&t, &AT(A, i, k), &AT(B, k, j), L);
                mp_add(&c, &c, &t, L);
            }
            AT(C, i, j) = c;
        }
}

/* eq. (2): block loops; each product goes straight into c_ij (== Simple) */
static void block(mat C, mat A, mat B, int L, int64_t bs)
{
    int64_t m = C.rows, n = C.cols, l = A.cols;
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) set_zero(&AT(C, i, j));
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int64_t i0 = 0; i0 < m; i0 += bs)
        for (int64_t j0 = 0; j0 < n; j0 += bs)
            for (int64_t k0 = 0; k0 < l; k0 += bs)
                for (int64_t i = i0; i < i0 + bs && i < m; i++)
                    for (int64_t j = j0; j < j0 + bs && j < n; j++) {
                        mpv c = AT(C, i, j), t;
                        for (int64_t k = k0; k < k0 + bs && k < l; k++) {
                            mp_mul(&t, &AT(A, i, k), &AT(B, k, j), L);
                            mp_add(&c, &c, &t, L);
                        }
                        AT(C, i, j) = c;
                    }
}

/* Z := X op Y elementwise (op 0 add, 1 sub) */
static void ew(mat Z, mat X, mat Y, int op, int L)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < Z.rows; i++)
        for (int64_t j = 0; j < Z.cols; j++) {
            mpv r;
            if (op) mp_sub(&r, &AT(X, i, j), &AT(Y, i, j), L);
            else mp_add(&r, &AT(X, i, j), &AT(Y, i, j), L);
            AT(Z, i, j) = r;
        }
}

static void copy_into(mat Z, mat X)
{
    for (int64_t i = 0; i < Z.rows; i++)
        for (int64_t j = 0; j < Z.cols; j++) AT(Z, i, j) = AT(X, i, j);
}

static void recursive(mat C, mat A, mat B, int algo, int64_t cutoff, int policy, int L);

/* one Strassen level on even sizes (Section 2, P1..P7 and the quadrants) */
static void strassen_level(mat C, mat A, mat B, int64_t cutoff, int policy, int L)
{
    int64_t h = C.rows / 2, g = A.cols / 2, w = C.cols / 2;
    mat A11 = mat_view(A, 0, 0, h, g), A12 = mat_view(A, 0, g, h, g);
    mat A21 = mat_view(A, h, 0, h, g), A22 = mat_view(A, h, g, h, g);
    mat B11 = mat_view(B, 0, 0, g, w), B12 = mat_view(B, 0, w, g, w);
    mat B21 = mat_view(B, g, 0, g, w), B22 = mat_view(B, g, w, g, w);
    mat SA = mat_new(h, g), SB = mat_new(g, w), P[8];
    for (int i = 1; i <= 7; i++) P[i] = mat_new(h, w);
    ew(SA, A11, A22, 0, L); ew(SB, B11, B22, 0, L); recursive(P[1], SA, SB, 2, cutoff, policy, L);
    ew(SA, A21, A22, 0, L);                         recursive(P[2], SA, B11, 2, cutoff, policy, L);
    ew(SB, B12, B22, 1, L);                         recursive(P[3], A11, SB, 2, cutoff, policy, L);
    ew(SB, B21, B11, 1, L);                         recursive(P[4], A22, SB, 2, cutoff, policy, L);
    ew(SA, A11, A12, 0, L);                         recursive(P[5], SA, B22, 2, cutoff, policy, L);
    ew(SA, A21, A11, 1, L); ew(SB, B11, B12, 0, L); recursive(P[6], SA, SB, 2, cutoff, policy, L);
    ew(SA, A12, A22, 1, L); ew(SB, B21, B22, 0, L); recursive(P[7], SA, SB, 2, cutoff, policy, L);
    mat C11 = mat_view(C, 0, 0, h, w), C12 = mat_view(C, 0, w, h, w);
    mat C21 = mat_view(C, h, 0, h, w), C22 = mat_view(C, h, w, h, w);
    ew(C11, P[1], P[4], 0, L); ew(C11, C11, P[5], 1, L); ew(C11, C11, P[7], 0, L);
    ew(C12, P[3], P[5], 0, L);
    ew(C21, P[2], P[4], 0, L);
    ew(C22, P[1], P[3], 0, L); ew(C22, C22, P[2], 1, L); ew(C22, C22, P[6], 0, L);
    mat_free(SA); mat_free(SB);
    for (int i = 1; i <= 7; i++) mat_free(P[i]);
}

/* one level of Winograd's variant on even sizes (S1..S8, M1..M7, T1, T2) */
static void winograd_level(mat C, mat A, mat B, int64_t cutoff, int policy, int L)
{
    int64_t h = C.rows / 2, g = A.cols / 2, w = C.cols / 2;
    mat A11 = mat_view(A, 0, 0, h, g), A12 = mat_view(A, 0, g, h, g);
    mat A21 = mat_view(A, h, 0, h, g), A22 = mat_view(A, h, g, h, g);
    mat B11 = mat_view(B, 0, 0, g, w), B12 = mat_view(B, 0, w, g, w);
    mat B21 = mat_view(B, g, 0, g, w), B22 = mat_view(B, g, w, g, w);
    mat S[9], M[8];
    for (int i = 1; i <= 4; i++) S[i] = mat_new(h, g);
    for (int i = 5; i <= 8; i++) S[i] = mat_new(g, w);
    for (int i = 1; i <= 7; i++) M[i] = mat_new(h, w);
    ew(S[1], A21, A22, 0, L);
    ew(S[2], S[1], A11, 1, L);
    ew(S[3], A11, A21, 1, L);
    ew(S[4], A12, S[2], 1, L);
    ew(S[5], B12, B11, 1, L);
    ew(S[6], B22, S[5], 1, L);
    ew(S[7], B22, B12, 1, L);
    ew(S[8], S[6], B21, 1, L);
    recursive(M[1], S[2], S[6], 3, cutoff, policy, L);
    recursive(M[2], A11, B11, 3, cutoff, policy, L);
    recursive(M[3], A12, B21, 3, cutoff, policy, L);
    recursive(M[4], S[3], S[7], 3, cutoff, policy, L);
    recursive(M[5], S[1], S[5], 3, cutoff, policy, L);
    recursive(M[6], S[4], B22, 3, cutoff, policy, L);
    recursive(M[7], A22, S[8], 3, cutoff, policy, L);
    mat T1 = mat_new(h, w), T2 = mat_new(h, w);
    ew(T1, M[1], M[2], 0, L);
    ew(T2, T1, M[4], 0, L);
    mat C11 = mat_view(C, 0, 0, h, w), C12 = mat_view(C, 0, w, h, w);
    mat C21 = mat_view(C, h, 0, h, w), C22 = mat_view(C, h, w, h, w);
    ew(C11, M[2], M[3], 0, L);
    ew(C12, T1, M[5], 0, L); ew(C12, C12, M[6], 0, L);
    ew(C21, T2, M[7], 1, L);
    ew(C22, T2, M[5], 0, L);
    for (int i = 1; i <= 8; i++) mat_free(S[i]);
    for (int i = 1; i <= 7; i++) mat_free(M[i]);
    mat_free(T1); mat_free(T2);
}

/* 0 even, 1 peel, 2 pad */
static int odd_action(int64_t d, int policy)
{
    if (d % 2 == 0) return 0;
    if (policy == POL_PEEL) return 1;
    if (policy == POL_PAD) return 2;
    return (d % 4 == 3) ? 2 : 1;
}

static int64_t core_size(int64_t d, int act)
{
    return act == 2 ? d + 1 : (act == 1 ? d - 1 : d);
}

/* R(A, B): recurse iff min(m, l, n) > cutoff; odd sizes peeled or padded */
static void recursive(mat C, mat A, mat B, int algo, int64_t cutoff, int policy, int L)
{
    int64_t m = C.rows, n = C.cols, l = A.cols;
    if (m == 0 || n == 0) return;
    int64_t mn = m < l ? m : l;
    mn = mn < n ? mn : n;
    if (mn <= cutoff) { simple(C, A, B, L); return; }
    int am = odd_action(m, policy), al = odd_action(l, policy), an = odd_action(n, policy);
    int64_t me = core_size(m, am), le = core_size(l, al), ne = core_size(n, an);
    mat Ae = mat_new(me, le), Be = mat_new(le, ne), Ce = mat_new(me, ne);
    for (int64_t i = 0; i < me; i++)
        for (int64_t k = 0; k < le; k++)
            if (i < m && k < l) AT(Ae, i, k) = AT(A, i, k);     /* else exact zero */
    for (int64_t k = 0; k < le; k++)
        for (int64_t j = 0; j < ne; j++)
            if (k < l && j < n) AT(Be, k, j) = AT(B, k, j);
    if (algo == ALG_STRASSEN) strassen_level(Ce, Ae, Be, cutoff, policy, L);
    else winograd_level(Ce, Ae, Be, cutoff, policy, L);
    int64_t mi = m < me ? m : me, ni = n < ne ? n : ne;
    copy_into(mat_view(C, 0, 0, mi, ni), Ce);
    if (al == 1) {                               /* peeled inner index l-1 */
        int64_t k = l - 1;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < mi; i++)
            for (int64_t j = 0; j < ni; j++) {
                mpv t;
                mp_mul(&t, &AT(A, i, k), &AT(B, k, j), L);
                mp_add(&AT(C, i, j), &AT(C, i, j), &t, L);
            }
    }
    if (an == 1)                                 /* peeled column n-1 */
        simple(mat_view(C, 0, n - 1, mi, 1), mat_view(A, 0, 0, mi, l), mat_view(B, 0, n - 1, l, 1), L);
    if (am == 1)                                 /* peeled row m-1 */
        simple(mat_view(C, m - 1, 0, 1, n), mat_view(A, m - 1, 0, 1, l), B, L);
    mat_free(Ae); mat_free(Be); mat_free(Ce);
}

static void gemm_any(mat C, mat A, mat B, int algo, int64_t cutoff, int policy, int64_t bs, int L)
{
    if (algo == ALG_SIMPLE) simple(C, A, B, L);
    else if (algo == ALG_BLOCK) block(C, A, B, L, bs);
    else recursive(C, A, B, algo, cutoff, policy, L);
}

/* ------------------------------------------------------------------ C entry points */

int ref_gemm(int64_t m, int64_t l, int64_t n, int p, int algo, int64_t cutoff, int policy, int64_t bs,
             const uint32_t *A, int64_t lda, int64_t psa,
             const uint32_t *B, int64_t ldb, int64_t psb,
             uint32_t *C, int64_t ldc, int64_t psc)
{
    if (p % 32 || p <= 0 || p / 32 > MAXL) return -2;
    int L = p / 32;
    mat a = mat_new(m, l), b = mat_new(l, n), c = mat_new(m, n);
    load(a, A, lda, psa, L);
    load(b, B, ldb, psb, L);
    gemm_any(c, a, b, algo, cutoff, policy, bs, L);
    int rc = store(c, C, ldc, psc, L);
    mat_free(a); mat_free(b); mat_free(c);
    return rc;
}

/* scalar op for cross-checks: 0 mul, 1 add, 2 sub, 3 div; x, y, r in (L+2)-word records */
int ref_scalar(int op, int p, const uint32_t *x, const uint32_t *y, uint32_t *r)
{
    if (p % 32 || p <= 0 || p / 32 > MAXL) return -2;
    int L = p / 32;
    mpv a, b, c;
    mat ma = {&a, 1, 1, 1}, mb = {&b, 1, 1, 1}, mc = {&c, 1, 1, 1};
    load(ma, x, 1, 1, L);
    load(mb, y, 1, 1, L);
    if (op == 0) mp_mul(&c, &a, &b, L);
    else if (op == 1) mp_add(&c, &a, &b, L);
    else if (op == 2) mp_sub(&c, &a, &b, L);
    else {
        if (is_zero(&b, L)) return -1;
        mp_div(&c, &a, &b, L);
    }
    return store(mc, r, 1, 1, L);
}

/* Section 4 blocked LU, with partial pivoting (pivot != 0) or, as in the
   paper, without (pivot == 0: every pivot is the diagonal entry); see
   oracle/lu.py for the readings */
static int lu(mat a, int32_t *piv, int64_t panel, int algo, int64_t cutoff, int policy, int pivot, int L)
{
    int64_t n = a.rows;
    int info = 0;
    for (int64_t j0 = 0; j0 < n; j0 += panel) {
        int64_t kb = panel < n - j0 ? panel : n - j0, je = j0 + kb;
        for (int64_t c = j0; c < je; c++) {
            int64_t r = c;
            for (int64_t i = c + 1; pivot && i < n; i++)
                if (mp_cmpabs(&AT(a, i, c), &AT(a, r, c), L) > 0) r = i;
            piv[c] = (int32_t)r;
            if (r != c)
                for (int64_t j = 0; j < n; j++) {
                    mpv t = AT(a, c, j);
                    AT(a, c, j) = AT(a, r, j);
                    AT(a, r, j) = t;
                }
            if (is_zero(&AT(a, c, c), L)) {
                if (!info) info = (int)(c + 1);
                continue;
            }
#pragma omp parallel for schedule(static)
            for (int64_t i = c + 1; i < n; i++) {
                mp_div(&AT(a, i, c), &AT(a, i, c), &AT(a, c, c), L);
                for (int64_t j = c + 1; j < je; j++) {
                    mpv t;
                    mp_mul(&t, &AT(a, i, c), &AT(a, c, j), L);
                    mp_sub(&AT(a, i, j), &AT(a, i, j), &t, L);
                }
            }
        }
        if (je >= n) break;
#pragma omp parallel for schedule(static)
        for (int64_t j = je; j < n; j++)
            for (int64_t t = 0; t < kb; t++)
                for (int64_t r = t + 1; r < kb; r++) {
                    mpv u;
                    mp_mul(&u, &AT(a, j0 + r, j0 + t), &AT(a, j0 + t, j), L);
                    mp_sub(&AT(a, j0 + r, j), &AT(a, j0 + r, j), &u, L);
                }
        mat P = mat_new(n - je, n - je);
        gemm_any(P, mat_view(a, je, j0, n - je, kb), mat_view(a, j0, je, kb, n - je), algo, cutoff, policy, 16, L);
        ew(mat_view(a, je, je, n - je, n - je), mat_view(a, je, je, n - je, n - je), P, 1, L);
        mat_free(P);
    }
    return info;
}

int ref_lu_ex(int64_t n, int p, int64_t panel, int algo, int64_t cutoff, int policy, int pivot,
              uint32_t *A, int64_t lda, int64_t psa, int32_t *piv, int32_t *info)
{
    if (p % 32 || p <= 0 || p / 32 > MAXL) return -2;
    int L = p / 32;
    mat a = mat_new(n, n);
    load(a, A, lda, psa, L);
    *info = lu(a, piv, panel, algo, cutoff, policy, pivot, L);
    int rc = store(a, A, lda, psa, L);
    mat_free(a);
    return rc;
}

int ref_lu(int64_t n, int p, int64_t panel, int algo, int64_t cutoff, int policy,
           uint32_t *A, int64_t lda, int64_t psa, int32_t *piv, int32_t *info)
{
    return ref_lu_ex(n, p, panel, algo, cutoff, policy, 1, A, lda, psa, piv, info);
}

/* x := solve with the factors (swaps, unit-lower forward, upper backward) */
int ref_lu_solve(int64_t n, int p, const uint32_t *LU, int64_t ld, int64_t ps, const int32_t *piv,
                 uint32_t *b, int64_t psb)
{
    if (p % 32 || p <= 0 || p / 32 > MAXL) return -2;
    int L = p / 32;
    mat a = mat_new(n, n), y = mat_new(n, 1), x = mat_new(n, 1);
    load(a, LU, ld, ps, L);
    load(y, b, 1, psb, L);
    for (int64_t k = 0; k < n; k++)
        if (piv[k] != k) {
            mpv t = AT(y, k, 0);
            AT(y, k, 0) = AT(y, piv[k], 0);
            AT(y, piv[k], 0) = t;
        }
    for (int64_t t = 0; t < n; t++)
        for (int64_t r = t + 1; r < n; r++) {
            mpv u;
            mp_mul(&u, &AT(a, r, t), &AT(y, t, 0), L);
            mp_sub(&AT(y, r, 0), &AT(y, r, 0), &u, L);
        }
    for (int64_t t = n - 1; t >= 0; t--) {
        if (is_zero(&AT(a, t, t), L)) { mat_free(a); mat_free(y); mat_free(x); return -1; }
        mp_div(&AT(x, t, 0), &AT(y, t, 0), &AT(a, t, t), L);
        for (int64_t r = 0; r < t; r++) {
            mpv u;
            mp_mul(&u, &AT(a, r, t), &AT(x, t, 0), L);
            mp_sub(&AT(y, r, 0), &AT(y, r, 0), &u, L);
        }
    }
    int rc = store(x, b, 1, psb, L);
    mat_free(a); mat_free(y); mat_free(x);
    return rc;
}

/* widen x (L limbs) to the L2-limb format exactly */
static void widen(mpv *r, const mpv *x, int L, int L2)
{
    *r = *x;
    if (is_zero(x, L)) { set_zero(r); return; }
    uint32_t t[MAXL];
    memset(t, 0, sizeof t);
    for (int k = 0; k < L; k++) t[k + (L2 - L)] = x->m[k];
    memcpy(r->m, t, sizeof t);
}

/* log2-scaled double of |x|: returns d and sets *e so that |x| ~ d * 2^e */
static double to_dbl(const mpv *x, int L, int64_t *e)
{
    if (is_zero(x, L)) { *e = 0; return 0.0; }
    double d = (double)x->m[L - 1] / 4294967296.0 + (L > 1 ? (double)x->m[L - 2] / 18446744073709551616.0 : 0.0);
    *e = x->e;
    return d;
}

/*
 * ||PA - LU||_inf / ||A||_inf and max_i |x_i - 1|, evaluated in (2p + 64)-bit
 * arithmetic: every product l_ik u_kj of two p-bit numbers is exact there and
 * each of the n roundings of a row sum costs at most 2^-(2p+63) relative, far
 * below any residual of a p-bit factorisation.  Results as (mantissa, exp2).
 */
int ref_lu_residual(int64_t n, int p, const uint32_t *A0, int64_t lda, int64_t psa,
                    const uint32_t *LU, int64_t ldl, int64_t psl, const int32_t *piv,
                    double *res_m, int64_t *res_e)
{
    if (p % 32 || p <= 0 || 2 * (p / 32) + 2 > MAXL) return -2;
    int L = p / 32, L2 = 2 * L + 2;
    mat a = mat_new(n, n), f = mat_new(n, n);
    load(a, A0, lda, psa, L);
    load(f, LU, ldl, psl, L);
    for (int64_t k = 0; k < n; k++)                     /* P A */
        if (piv[k] != k)
            for (int64_t j = 0; j < n; j++) {
                mpv t = AT(a, k, j);
                AT(a, k, j) = AT(a, piv[k], j);
                AT(a, piv[k], j) = t;
            }
    mpv *rown = (mpv *)calloc((size_t)n, sizeof(mpv)), *rowa = (mpv *)calloc((size_t)n, sizeof(mpv));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; i++) {
        mpv sr, sa;
        set_zero(&sr); set_zero(&sa);
        for (int64_t j = 0; j < n; j++) {
            mpv s, t, x, y, z;
            set_zero(&s);
            int64_t kmax = i < j ? i : j;
            for (int64_t k = 0; k <= kmax; k++) {
                widen(&y, &AT(f, k, j), L, L2);
                if (k == i) t = y;                       /* unit diagonal of L */
                else {
                    widen(&x, &AT(f, i, k), L, L2);
                    mp_mul(&t, &x, &y, L2);
                }
                mp_add(&s, &s, &t, L2);
            }
            widen(&z, &AT(a, i, j), L, L2);
            mp_sub(&s, &z, &s, L2);
            s.neg = 0;
            mp_add(&sr, &sr, &s, L2);
            z.neg = 0;
            mp_add(&sa, &sa, &z, L2);
        }
        rown[i] = sr;
        rowa[i] = sa;
    }
    mpv mr, ma;
    set_zero(&mr); set_zero(&ma);
    for (int64_t i = 0; i < n; i++) {
        if (mp_cmpabs(&rown[i], &mr, L2) > 0) mr = rown[i];
        if (mp_cmpabs(&rowa[i], &ma, L2) > 0) ma = rowa[i];
    }
    int64_t er, ea;
    double dr = to_dbl(&mr, L2, &er), da = to_dbl(&ma, L2, &ea);
    *res_m = da > 0 ? dr / da : 0.0;
    *res_e = er - ea;
    free(rown); free(rowa);
    mat_free(a); mat_free(f);
    return 0;
}

/* limit the OpenMP thread count (0 = leave as is); returns the count in use */
#include <omp.h>
int ref_threads(int t)
{
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
}
