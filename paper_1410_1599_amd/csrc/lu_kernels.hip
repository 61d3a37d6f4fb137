// lu_kernels.hip -- the steps of blocked LU with partial pivoting (Section 4)
// and of the triangular solves.  The matrix is one MatRef; every element
// update is c := sub_rn(c, mul_rn(l, u)), so each element sees the same
// sequence of correctly rounded operations as the CPU oracle.
#include "lanediv.hpp"
#include "launch.hpp"
#include "mp_arith.hpp"
#include "recipdiv.hpp"

namespace mpg {

namespace {

template <int L>
__device__ __forceinline__ MP<L> ldm(const Bases& bs, const MatRef& r, int64_t i, int64_t j)
{
    return load<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j);
}

template <int L>
__device__ __forceinline__ void stm(const Bases& bs, const MatRef& r, int64_t i, int64_t j, const MP<L>& v)
{
    store<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j, v);
}

constexpr int PIV_THREADS = 256;

// The pivot of column c is the first row index r >= c of the largest |a_rc|
// (exact comparison; ties to the smaller index).  Each of the NT threads of a
// workgroup brings its best (index, value) over a share of the rows, visited
// in ascending order (best = -1: no rows).  The candidates are reduced without
// a comparison tree: one LDS atomic max over a 64-bit key (exponent, top limb)
// finds the largest key, the threads holding it list themselves, and one
// thread settles that short list (usually one entry) by full comparison, ties
// to the smaller index.  Writes piv[c] = r and info = c + 1 for the first
// exactly zero pivot; returns r in every thread.
template <int L, int NT>
__device__ int64_t settle_pivot(int32_t best, const MP<L>& bv, int64_t c, int32_t* piv, int32_t* info)
{
    __shared__ uint32_t sv[L + 2][NT];
    __shared__ int32_t sidx[NT];
    __shared__ unsigned long long skey;
    __shared__ int32_t scount, sbest;
    __shared__ int32_t scand[NT];
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < L; q++) sv[q][tid] = bv.m[q];
    sv[L][tid] = (uint32_t)bv.e;
    sv[L + 1][tid] = bv.s;
    sidx[tid] = best;
    if (tid == 0) {
        skey = 0;
        scount = 0;
    }
    __syncthreads();
    // |x| grows with (exponent, top limb) among nonzero values (|e| < 2^29);
    // zero has key 0
    const unsigned long long key =
        is_zero<L>(bv) ? 0ull : (((unsigned long long)(uint32_t)(bv.e + (1 << 30)) << 32) | bv.m[L - 1]);
    if (best >= 0) atomicMax(&skey, key);
    __syncthreads();
    if (best >= 0 && key == skey) scand[atomicAdd(&scount, 1)] = tid;
    __syncthreads();
    if (tid == 0) {
        int32_t bi = -1;
        MP<L> bx = mp_zero<L>();
        for (int q = 0; q < scount; q++) {
            const int u = scand[q];
            MP<L> x;
#pragma unroll
            for (int w = 0; w < L; w++) x.m[w] = sv[w][u];
            x.e = (int32_t)sv[L][u];
            x.s = sv[L + 1][u];
            const int32_t iu = sidx[u];
            const int cm = bi < 0 ? 1 : cmp_abs<L>(x, bx);
            if (cm > 0 || (cm == 0 && iu < bi)) {
                bi = iu;
                bx = x;
            }
        }
        sbest = bi;
        piv[c] = bi;
        if (is_zero<L>(bx) && info[0] == 0) info[0] = (int32_t)(c + 1);
    }
    __syncthreads();
    return sbest;
}

// Exchange rows c and r (r != c) over the panel columns [j0, je), every
// plane: a thread takes whole columns, loading both rows' words before it
// stores any (the two rows never overlap).
template <int L, int NT>
__device__ void swap_rows(const Bases& bs, const MatRef& a, int64_t c, int64_t r, int64_t j0, int64_t je)
{
    for (int64_t j = j0 + threadIdx.x; j < je; j += NT) {
        const MP<L> x = ldm<L>(bs, a, c, j), y = ldm<L>(bs, a, r, j);
        stm<L>(bs, a, c, j, y);
        stm<L>(bs, a, r, j, x);
    }
}

// pivot search of column c over the rows [c, n) (each thread a strided
// share), then the swap of rows c and r over the panel columns [j0, je)
template <int L, int NT>
__device__ void pivot_and_swap(const Bases& bs, const MatRef& a, int64_t n, int64_t c, int64_t j0, int64_t je,
                               int32_t* piv, int32_t* info)
{
    const int tid = threadIdx.x;
    int32_t best = -1;
    MP<L> bv = mp_zero<L>();
    for (int64_t i = c + tid; i < n; i += NT) {
        const MP<L> v = ldm<L>(bs, a, i, c);
        if (best < 0 || cmp_abs<L>(v, bv) > 0) {
            best = (int32_t)i;
            bv = v;
        }
    }
    const int64_t r = settle_pivot<L, NT>(best, bv, c, piv, info);
    if (r != c) swap_rows<L, NT>(bs, a, c, r, j0, je);
}

// search == 0: the paper's LU without row exchanges: the pivot is a_cc
template <int L>
__global__ void __launch_bounds__(PIV_THREADS)
k_lu_pivot_swap(Bases bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je, int32_t* piv, int32_t* info,
                int search)
{
    if (search) {
        pivot_and_swap<L, PIV_THREADS>(bs, a, n, c, j0, je, piv, info);
    } else if (threadIdx.x == 0) {
        piv[c] = (int32_t)c;
        if (is_zero<L>(ldm<L>(bs, a, c, c)) && info[0] == 0) info[0] = (int32_t)(c + 1);
    }
}

// Wave-wide reductions (one-wave workgroups)
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ long long wave_min_i64(long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const long long w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

constexpr int ELIM_ROWS = 4;      // rows (one wave each) per workgroup of a column step

// Several rows hold the largest key km (the first is row first): compare
// their values from the copy in full, ascending, first index on ties.
template <int L>
__device__ long long settle_equal_keys(const PanelCopy& pc, int64_t n, int64_t c, int64_t j0,
                                       unsigned long long km, long long first)
{
    long long bi = -1;
    MP<L> bx = mp_zero<L>();
    for (int64_t k = first; k < n; k++) {
        if (pc.keys_in[k] != km) continue;
        const MP<L> v = load<L>(pc.cand_in, pc.cps, k * pc.cld + (c - j0));
        if (bi < 0 || cmp_abs<L>(v, bx) > 0) {
            bi = k;
            bx = v;
        }
    }
    return bi;
}

// The pivot of column c from the copy the step of column c - 1 left
// (PanelCopy), found by the calling wave alone (every lane gets it): the
// largest key over the rows [c, n), from the groups of ELIM_ROWS rows (each
// group's largest key, the first of its rows holding it, and whether another
// does); when one row holds it (one group, and one row of that group), that
// row (a nonzero key is a nonzero value); when several do, their values
// (from the copy) are compared in full, ascending, first index on ties; a
// zero column gives the first row and *zero.  The same choice as the full
// search of pivot_and_swap, from one round of loads of the group records.
template <int L>
__device__ int64_t find_pivot(const PanelCopy& pc, int64_t n, int64_t c, int64_t j0, bool* zero)
{
    const int lane = threadIdx.x & 63;
    const int64_t ng = (n - c + ELIM_ROWS - 1) / ELIM_ROWS;
    // this lane's groups g = lane, lane + 64, ...: the largest key, how many
    // of them hold it, and the first one's record
    constexpr long long NONE = 0x7fffffffffffffffll;
    unsigned long long km = 0, finfo = 0;
    long long fg = NONE;
    int hold = 0;
    for (int64_t g = lane; g < ng; g += 64) {
        const unsigned long long v = pc.cmax_in[2 * g], f = pc.cmax_in[2 * g + 1];
        if (fg == NONE || v > km) {
            km = v;
            fg = g;
            finfo = f;
            hold = 1;
        } else if (v == km) {
            hold++;
        }
    }
    const unsigned long long kmax = wave_max_u64(km);
    *zero = kmax == 0;
    if (kmax == 0) return c;
    if (km != kmax) {
        fg = NONE;
        hold = 0;
    }
    hold = wave_sum(hold);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const long long og = __shfl_xor(fg, o);
        const unsigned long long oi = __shfl_xor(finfo, o);
        if (og < fg) {
            fg = og;
            finfo = oi;
        }
    }
    const long long first = (long long)(finfo & 0x7fffffffffffffffull);
    if (hold == 1 && (finfo >> 63) == 0) return first;
    long long bi = 0;
    if (lane == 0) bi = settle_equal_keys<L>(pc, n, c, j0, kmax, first);
    return __shfl(bi, 0);
}

// The pivot step of column c as a launch of its own (the precisions whose
// column step has no registers to spare for the search): the pivot from the
// copy (find_pivot), then rows c and r exchanged over the panel columns
// [j0, je).
template <int L>
__global__ void __launch_bounds__(64)
k_lu_pivot_copy(Bases bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je, int32_t* piv, int32_t* info,
                PanelCopy pc)
{
    bool zero_col;
    const int64_t r = find_pivot<L>(pc, n, c, j0, &zero_col);
    if (threadIdx.x == 0) {
        piv[c] = (int32_t)r;
        if (zero_col && info[0] == 0) info[0] = (int32_t)(c + 1);
    }
    if (r != c) swap_rows<L, 64>(bs, a, c, r, j0, je);
}

// The step of column c: one wave per row position pos in (c, n), ELIM_ROWS
// of them per workgroup: l = a_pos,c / a_cc by the whole wave, one limb per
// lane (lanediv.hpp; the same bits as div_rn), its limbs then read out of the
// lanes, and a_pos,j := a_pos,j - l a_cj for the panel columns j in (c, je);
// a zero pivot skips the column (no quotient, no update).
//
// FUSED (row exchanges, a step after the panel's first): the pivot search of
// column c runs in the same launch.  Every wave finds the pivot row r from
// the keys of the copy (find_pivot) and works as if rows c and r were
// already exchanged: the pivot row (old row r) is read from the copy, never
// from A, and the row at position r is old row c.  The wave of position r
// also performs the exchange over the panel columns [j0, je): it is the only
// one that touches positions c and r, so no wave reads what another writes.
// Workgroup 0 records piv[c] and a zero pivot in info.
//
// next == ELIM_NEXT_KEYS (c + 1 < je): each wave stores its row's new
// a_pos,c+1 key (exponent, top limb; 0 for zero) in keys_out[pos] and its
// row's panel columns (c, je) in cand_out, and each workgroup the largest
// key of its rows in cmax_out[blockIdx.x] (one plain store: an atomic
// maximum over the workgroups sharing a word serialises in memory), for the
// step of column c + 1.
//
// next == ELIM_NEXT_DIAG (no row exchanges): the owner of row c + 1 checks its
// new a_c+1,c+1 for zero (info) and sets piv[c + 1] = c + 1.
constexpr int ELIM_THREADS = 64 * ELIM_ROWS;
constexpr int ELIM_PLAIN = 0, ELIM_NEXT_KEYS = 1, ELIM_NEXT_DIAG = 2;

template <int L, bool FUSED>
__global__ void __launch_bounds__(ELIM_THREADS)
k_lu_eliminate(Bases bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je, int32_t* piv, int32_t* info,
               PanelCopy pc, int next)
{
    __shared__ unsigned long long skey[ELIM_ROWS];
    const int tid = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t pos = c + 1 + (int64_t)blockIdx.x * ELIM_ROWS + w;
    const bool keep = next == ELIM_NEXT_KEYS;
    unsigned long long key = 0;
    int64_t r = c;
    if (FUSED) {
        bool zero_col;
        r = find_pivot<L>(pc, n, c, j0, &zero_col);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            piv[c] = (int32_t)r;
            if (zero_col && info[0] == 0) info[0] = (int32_t)(c + 1);
        }
    }
    if (pos < n) {
        const bool swap = FUSED && pos == r;      // this row's content sits at position c
        const int64_t src = swap ? c : pos;
        uint32_t* pa = base_ptr(bs, a.base) + a.off;
        // the pivot row: from the copy (FUSED) or row c of A
        const uint32_t* pu = FUSED ? pc.cand_in : pa;
        const int64_t ups = FUSED ? pc.cps : a.ps;
        const int64_t u0 = FUSED ? r * pc.cld - j0 : c * a.ld;    // + j: element (pivot row, j)
        // this lane's first pair of operands is loaded while the wave divides
        const int64_t jf = c + 1 + tid;
        const bool has = jf < je;
        MP<L> xf = has ? ldm<L>(bs, a, src, jf) : mp_zero<L>();
        const MP<L> uf = has ? load<L>(pu, ups, u0 + jf) : mp_zero<L>();
        // the pivot and a_src,c in the lane layout: lane t holds limb t
        const int64_t idd = u0 + c, idx = src * a.ld + c;
        const uint32_t dm = tid < L ? pu[tid * ups + idd] : 0u;
        const uint32_t xm = tid < L ? pa[tid * a.ps + idx] : 0u;
        const int32_t de = (int32_t)pu[L * ups + idd], xe = (int32_t)pa[L * a.ps + idx];
        const uint32_t dsg = pu[(L + 1) * ups + idd], xsg = pa[(L + 1) * a.ps + idx];
        const bool skip = lane_limb<L>(dm, L - 1) == 0u;        // a zero pivot (uniform)
        MP<L> l = mp_zero<L>();
        if (!skip) {
            int32_t le;
            uint32_t ls;
            const uint32_t lm = lane_div_rn<L>(xm, xe, xsg, dm, de, dsg, &le, &ls);
            const int64_t idp = pos * a.ld + c;
            if (tid < L) pa[tid * a.ps + idp] = lm;
            if (tid == 0) {
                pa[L * a.ps + idp] = (uint32_t)le;
                pa[(L + 1) * a.ps + idp] = ls;
            }
#pragma unroll
            for (int q = 0; q < L; q++) l.m[q] = __builtin_amdgcn_readlane(lm, q);
            l.e = le;
            l.s = ls;
        }
        const int64_t co = pos * pc.cld - j0;                    // + j: this row in cand_out
        // a_pos,j from x (the row's content) and u (the pivot row's)
        auto update = [&](const MP<L>& x, const MP<L>& u, int64_t j) __attribute__((always_inline)) -> MP<L> {
            if (swap) stm<L>(bs, a, c, j, u);                    // row c := old row r (x is read)
            const MP<L> y = skip ? x : sub_rn<L>(x, mul_rn<L>(l, u));
            if (!skip || swap) stm<L>(bs, a, pos, j, y);
            if (keep) store<L>(pc.cand_out, pc.cps, co + j, y);
            return y;
        };
        if (has) xf = update(xf, uf, jf);
        for (int64_t j = jf + 64; j < je; j += 64) update(ldm<L>(bs, a, src, j), load<L>(pu, ups, u0 + j), j);
        if (swap) {
            // the rest of the exchange: columns [j0, c) both ways, and the pivot
            // into a_cc (a_rc got the quotient above)
            for (int64_t j = j0 + tid; j < c; j += 64) {
                const MP<L> x = ldm<L>(bs, a, c, j), v = ldm<L>(bs, a, r, j);
                stm<L>(bs, a, c, j, v);
                stm<L>(bs, a, r, j, x);
            }
            const int64_t idc = c * a.ld + c;
            if (tid < L) pa[tid * a.ps + idc] = dm;
            if (tid == 0) {
                pa[L * a.ps + idc] = (uint32_t)de;
                pa[(L + 1) * a.ps + idc] = dsg;
            }
        }
        // lane 0 now holds the row's final a_pos,c+1 in xf (column c+1 < je)
        if (next == ELIM_NEXT_DIAG && tid == 0 && pos == c + 1) {
            piv[c + 1] = (int32_t)(c + 1);
            if (is_zero<L>(xf) && info[0] == 0) info[0] = (int32_t)(c + 2);
        }
        if (keep && tid == 0) {
            key = is_zero<L>(xf) ? 0ull
                                 : (((unsigned long long)(uint32_t)(xf.e + (1 << 30)) << 32) | xf.m[L - 1]);
            pc.keys_out[pos] = key;
        }
    }
    if (keep) {
        // the group record: the largest key of the workgroup's rows (0 for
        // rows past n), the first row holding it, and whether another does
        if (tid == 0) skey[w] = key;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long m = 0;
#pragma unroll
            for (int k = 0; k < ELIM_ROWS; k++) m = skey[k] > m ? skey[k] : m;
            int kf = -1, nh = 0;
#pragma unroll
            for (int k = 0; k < ELIM_ROWS; k++)
                if (skey[k] == m) {
                    kf = kf < 0 ? k : kf;
                    nh++;
                }
            pc.cmax_out[2 * blockIdx.x] = m;
            pc.cmax_out[2 * blockIdx.x + 1] =
                (unsigned long long)(c + 1 + (int64_t)blockIdx.x * ELIM_ROWS + kf) | (nh > 1 ? (1ull << 63) : 0ull);
        }
    }
}

// U12 := L11^-1 A12: one workgroup per column j >= je, one lane per panel row;
// step t updates rows r > t with row t, which step t-1 finished.  For panels
// of up to 64 rows the column stays in registers (lane r holds row r; the
// finished row t is broadcast through LDS); wider panels go through memory.
template <int L>
__global__ void __launch_bounds__(64)
k_lu_u12(Bases bs, MatRef a, int64_t j0, int64_t kb, int64_t je)
{
    const int64_t j = je + blockIdx.x;
    if (kb <= 64) {
        __shared__ uint32_t su[L + 2];
        const int r = threadIdx.x;
        MP<L> x = r < kb ? ldm<L>(bs, a, j0 + r, j) : mp_zero<L>();
        // l_r,t+1 is loaded while step t computes
        MP<L> ln = (r > 0 && r < kb) ? ldm<L>(bs, a, j0 + r, j0) : mp_zero<L>();
        for (int64_t t = 0; t < kb - 1; t++) {
            if (r == t) {
#pragma unroll
                for (int q = 0; q < L; q++) su[q] = x.m[q];
                su[L] = (uint32_t)x.e;
                su[L + 1] = x.s;
            }
            __syncthreads();
            const MP<L> lc = ln;
            ln = (r > t + 1 && r < kb) ? ldm<L>(bs, a, j0 + r, j0 + t + 1) : mp_zero<L>();
            if (r > t && r < kb) {
                MP<L> u;
#pragma unroll
                for (int q = 0; q < L; q++) u.m[q] = su[q];
                u.e = (int32_t)su[L];
                u.s = su[L + 1];
                x = sub_rn<L>(x, mul_rn<L>(lc, u));
            }
            __syncthreads();
        }
        if (r < kb) stm<L>(bs, a, j0 + r, j, x);
        return;
    }
    for (int64_t t = 0; t < kb - 1; t++) {
        const MP<L> u = ldm<L>(bs, a, j0 + t, j);
        for (int64_t r = t + 1 + threadIdx.x; r < kb; r += 64)
            stm<L>(bs, a, j0 + r, j, sub_rn<L>(ldm<L>(bs, a, j0 + r, j), mul_rn<L>(ldm<L>(bs, a, j0 + r, j0 + t), u)));
        __syncthreads();
    }
}

// Apply the swaps piv[k0 .. k1) in order (k1 - k0 <= LASWP_MAXK) to the
// columns [c0, c1) and [c2, c3).  The swaps only move the rows k0 .. k1 - 1
// and the rows they name, so they form one permutation of at most
// 2 (k1 - k0) "slots": slot t < kb is row k0 + t, slot kb + t the row piv[k0 +
// t] when it lies past k1 and swap t is the first to name it (else unused).
// Each thread works out src[s] (the slot whose old content ends in slot s)
// for its slots by itself, following the swaps backwards from the slot's
// row; then each workgroup moves the changed slots of one plane and
// LASWP_CW columns through LDS (all reads before all writes).
constexpr int LASWP_MAXK = 256, LASWP_MAXS = 2 * LASWP_MAXK, LASWP_CW = 16, LASWP_THREADS = 256;

template <int L>
__global__ void __launch_bounds__(LASWP_THREADS)
k_lu_laswp(Bases bs, MatRef a, const int32_t* piv, int64_t k0, int64_t k1, int64_t c0, int64_t c1, int64_t c2,
           int64_t c3)
{
    __shared__ int32_t rowof[LASWP_MAXS], src[LASWP_MAXS], pv[LASWP_MAXK];
    __shared__ uint32_t tile[LASWP_MAXS][LASWP_CW];
    const int kb = (int)(k1 - k0);
    const int ns = 2 * kb;
    for (int t = threadIdx.x; t < kb; t += LASWP_THREADS) pv[t] = piv[k0 + t];   // pv[t] >= k0 + t
    __syncthreads();
    for (int sl = threadIdx.x; sl < ns; sl += LASWP_THREADS) {
        int32_t row = -1;
        if (sl < kb) {
            row = (int32_t)(k0 + sl);
        } else {
            const int t = sl - kb;
            const int32_t r = pv[t];
            bool first = r >= k1;
            for (int u = 0; u < t && first; u++) first = pv[u] != r;
            if (first) row = r;
        }
        int sv = sl;
        if (row >= 0) {
            int64_t x = row;                  // the old row whose content ends in this slot
            for (int t = kb - 1; t >= 0; t--) {
                if (x == k0 + t) x = pv[t];
                else if (x == pv[t]) x = k0 + t;
            }
            if (x < k1) {
                sv = (int)(x - k0);
            } else {
                int u = 0;
                while (pv[u] != x) u++;       // x is named by some swap
                sv = kb + u;
            }
        }
        rowof[sl] = row;
        src[sl] = sv;
    }
    __syncthreads();
    const int64_t n1 = c1 - c0, nc = n1 + (c3 - c2);
    const int64_t cb = (int64_t)blockIdx.x * LASWP_CW;
    uint32_t* P = base_ptr(bs, a.base) + a.off + (int64_t)blockIdx.y * a.ps;
    for (int e = threadIdx.x; e < ns * LASWP_CW; e += LASWP_THREADS) {
        const int sl = e / LASWP_CW, jj = e % LASWP_CW;
        const int64_t ci = cb + jj;
        if (ci < nc && rowof[sl] >= 0 && src[sl] != sl) {
            const int64_t j = ci < n1 ? c0 + ci : c2 + (ci - n1);
            tile[sl][jj] = P[(int64_t)rowof[src[sl]] * a.ld + j];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ns * LASWP_CW; e += LASWP_THREADS) {
        const int sl = e / LASWP_CW, jj = e % LASWP_CW;
        const int64_t ci = cb + jj;
        if (ci < nc && rowof[sl] >= 0 && src[sl] != sl) {
            const int64_t j = ci < n1 ? c0 + ci : c2 + (ci - n1);
            P[(int64_t)rowof[sl] * a.ld + j] = tile[sl][jj];
        }
    }
}

// x := U^-1 L^-1 P b in one workgroup (the vector lives in global memory and
// every step is separated by a workgroup barrier)
constexpr int SOLVE_THREADS = 1024;

template <int L>
__global__ void __launch_bounds__(SOLVE_THREADS)
k_lu_solve(Bases bs, MatRef lu, MatRef x, const int32_t* piv, int64_t n)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        for (int64_t k = 0; k < n; k++) {
            const int64_t r = piv[k];
            if (r == k) continue;
            const MP<L> u = ldm<L>(bs, x, k, 0), v = ldm<L>(bs, x, r, 0);
            stm<L>(bs, x, k, 0, v);
            stm<L>(bs, x, r, 0, u);
        }
    }
    __syncthreads();
    for (int64_t t = 0; t < n; t++) {                 // L y = P b, unit diagonal
        const MP<L> yt = ldm<L>(bs, x, t, 0);
        for (int64_t r = t + 1 + tid; r < n; r += SOLVE_THREADS)
            stm<L>(bs, x, r, 0, sub_rn<L>(ldm<L>(bs, x, r, 0), mul_rn<L>(ldm<L>(bs, lu, r, t), yt)));
        __syncthreads();
    }
    for (int64_t t = n - 1; t >= 0; t--) {            // U x = y
        if (tid == 0) stm<L>(bs, x, t, 0, div_rn<L>(ldm<L>(bs, x, t, 0), ldm<L>(bs, lu, t, t)));
        __syncthreads();
        const MP<L> xt = ldm<L>(bs, x, t, 0);
        for (int64_t r = tid; r < t; r += SOLVE_THREADS)
            stm<L>(bs, x, r, 0, sub_rn<L>(ldm<L>(bs, x, r, 0), mul_rn<L>(ldm<L>(bs, lu, r, t), xt)));
        __syncthreads();
    }
}

unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

}  // namespace

// T := A^T for an n x n matrix, every plane: planes of T are n x n with
// leading dimension n.  16 x 16 blocks go through LDS so that both the reads
// and the writes of a wave are row segments.  Grid (blocks of columns, blocks
// of rows, planes).
__global__ void __launch_bounds__(256)
k_lu_transpose(const uint32_t* __restrict__ A, int64_t lda, int64_t psa, uint32_t* __restrict__ T, int64_t n)
{
    __shared__ uint32_t tile[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t i0 = (int64_t)blockIdx.y * 16, j0 = (int64_t)blockIdx.x * 16, q = blockIdx.z;
    if (i0 + ty < n && j0 + tx < n) tile[ty][tx] = A[q * psa + (i0 + ty) * lda + j0 + tx];
    __syncthreads();
    if (j0 + ty < n && i0 + tx < n) T[q * n * n + (j0 + ty) * n + i0 + tx] = tile[tx][ty];
}

// The same solve with the vector in registers: thread t owns rows t + k * 512
// (k < RPT, n <= 512 RPT; 512 threads leave 256 registers per lane).  The
// factors are read from their transpose luT (luT(j, i) = lu(i, j)), so the
// column of L or U that a step needs is a run of consecutive words of every
// plane: one workgroup streams the factors once, coalesced.  The row swaps are first composed into one
// permutation in LDS; at every step the owner of the finished entry publishes
// it through LDS (two alternating slots, one barrier per step) and every
// other row applies its update in the same order as above.
constexpr int SOLVE_REG_THREADS = 512;

template <int L, int RPT>
__global__ void __launch_bounds__(SOLVE_REG_THREADS)
k_lu_solve_reg(Bases bs, MatRef luT, MatRef x, const int32_t* piv, int64_t n)
{
    __shared__ int32_t perm[SOLVE_REG_THREADS * RPT];
    __shared__ uint32_t sx[2][L + 2];
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int r = tid + k * SOLVE_REG_THREADS;
        if (r < n) perm[r] = r;
    }
    __syncthreads();
    if (tid == 0) {
        for (int t = 0; t < (int)n; t++) {
            const int p = piv[t];
            const int w = perm[t];
            perm[t] = perm[p];
            perm[p] = w;
        }
    }
    __syncthreads();
    MP<L> v[RPT];
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int r = tid + k * SOLVE_REG_THREADS;
        v[k] = r < n ? ldm<L>(bs, x, perm[r], 0) : mp_zero<L>();
    }
    auto publish = [&](int t, const MP<L>& y) {
        uint32_t* d = sx[t & 1];
#pragma unroll
        for (int q = 0; q < L; q++) d[q] = y.m[q];
        d[L] = (uint32_t)y.e;
        d[L + 1] = y.s;
    };
    auto fetch = [&](int t) {
        const uint32_t* d = sx[t & 1];
        MP<L> y;
#pragma unroll
        for (int q = 0; q < L; q++) y.m[q] = d[q];
        y.e = (int32_t)d[L];
        y.s = d[L + 1];
        return y;
    };
    // the factor entries of step t + 1 are loaded while step t computes
    MP<L> fc[RPT];
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int r = tid + k * SOLVE_REG_THREADS;
        fc[k] = (r > 0 && r < n) ? ldm<L>(bs, luT, 0, r) : mp_zero<L>();
    }
    for (int t = 0; t < (int)n; t++) {              // L y = P b, unit diagonal
        if (tid == t % SOLVE_REG_THREADS) {
#pragma unroll
            for (int k = 0; k < RPT; k++)
                if (k == t / SOLVE_REG_THREADS) publish(t, v[k]);
        }
        __syncthreads();
        const MP<L> yt = fetch(t);
        MP<L> fn[RPT];
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            const int r = tid + k * SOLVE_REG_THREADS;
            fn[k] = (r > t + 1 && r < n) ? ldm<L>(bs, luT, t + 1, r) : mp_zero<L>();
        }
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            const int r = tid + k * SOLVE_REG_THREADS;
            if (r > t && r < n) v[k] = sub_rn<L>(v[k], mul_rn<L>(fc[k], yt));
            fc[k] = fn[k];
        }
    }
    // up to 512 bits, and up to 32 limbs of rows per thread (beyond that the
    // registers spill), each thread first forms the reciprocals of its rows'
    // diagonal entries (recip_ext, all rows at once), so that the division on
    // each backward step's critical path becomes a product and a rounding
    // check (div_by_recip: the same bits as div_rn)
    constexpr bool RECIP = L <= 16 && L * RPT <= 32;
    MP<L + 2> rinv[RECIP ? RPT : 1];
    if constexpr (RECIP) {
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            const int r = tid + k * SOLVE_REG_THREADS;
            const MP<L> d = r < n ? ldm<L>(bs, luT, r, r) : mp_zero<L>();
            rinv[k] = is_zero<L>(d) ? mp_zero<L + 2>() : recip_ext<L>(d);
        }
    }
    // column n - 1 of U (its diagonal entry for the owner of row n - 1)
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int r = tid + k * SOLVE_REG_THREADS;
        fc[k] = r < n ? ldm<L>(bs, luT, n - 1, r) : mp_zero<L>();
    }
    for (int t = (int)n - 1; t >= 0; t--) {         // U x = y
        if (tid == t % SOLVE_REG_THREADS) {
#pragma unroll
            for (int k = 0; k < RPT; k++)
                if (k == t / SOLVE_REG_THREADS) {
                    if constexpr (RECIP) v[k] = div_by_recip<L>(v[k], fc[k], rinv[k]);
                    else v[k] = div_rn<L>(v[k], fc[k]);
                    publish(t, v[k]);
                }
        }
        __syncthreads();
        const MP<L> xt = fetch(t);
        MP<L> fn[RPT];
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            const int r = tid + k * SOLVE_REG_THREADS;
            fn[k] = (t >= 1 && r <= t - 1) ? ldm<L>(bs, luT, t - 1, r) : mp_zero<L>();
        }
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            const int r = tid + k * SOLVE_REG_THREADS;
            if (r < t) v[k] = sub_rn<L>(v[k], mul_rn<L>(fc[k], xt));
            fc[k] = fn[k];
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int r = tid + k * SOLVE_REG_THREADS;
        if (r < n) stm<L>(bs, x, r, 0, v[k]);
    }
}

#define MPG_DISPATCH_L(L_, CALL)           \
    switch (L_) {                          \
    case 4: { constexpr int LL = 4; CALL; break; }   \
    case 8: { constexpr int LL = 8; CALL; break; }   \
    case 16: { constexpr int LL = 16; CALL; break; } \
    case 32: { constexpr int LL = 32; CALL; break; } \
    default: return hipErrorInvalidValue;  \
    }

hipError_t launch_lu_pivot_swap(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                int32_t* piv, int32_t* info, int search, hipStream_t s)
{
    if (L >= 64) return launch_lu_pivot_swap_wide(L, bs, a, n, c, j0, je, piv, info, search, s);
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_pivot_swap<LL>), dim3(1), dim3(PIV_THREADS), 0, s, bs, a, n, c, j0, je,
                                         piv, info, search));
    return hipGetLastError();
}

hipError_t launch_lu_eliminate(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                               int32_t* piv, int32_t* info, const PanelCopy& pc, int next, int fused, hipStream_t s)
{
    if (c < j0 || c >= je || je > n) return hipErrorInvalidValue;
    if (next != ELIM_PLAIN && c + 1 >= je) return hipErrorInvalidValue;
    const int64_t nch = (n + ELIM_ROWS - 1) / ELIM_ROWS;
    if (next == ELIM_NEXT_KEYS && (!pc.keys_out || !pc.cand_out || !pc.cmax_out || pc.cld < je - j0 ||
                                   pc.nch != nch))
        return hipErrorInvalidValue;
    if (fused && (c == j0 || !pc.keys_in || !pc.cand_in || !pc.cmax_in || pc.cld < je - j0 || pc.nch != nch ||
                  next == ELIM_NEXT_DIAG))
        return hipErrorInvalidValue;
    if (L >= 64) {
        if (next != ELIM_PLAIN || fused) return hipErrorInvalidValue;
        if (n - c - 1 <= 0) return hipSuccess;
        return launch_lu_eliminate_wide(L, bs, a, n, c, je, s);
    }
    const int64_t rows = n - c - 1, ng = (rows + ELIM_ROWS - 1) / ELIM_ROWS;
    if (fused) {
        // one workgroup at least: it records the pivot of the last column
        // (up to 512 bits: at 1024 the step has no registers to spare for
        // the search, and launch_lu_pivot_copy runs it)
        const dim3 g((unsigned)(ng > 0 ? ng : 1)), b(ELIM_THREADS);
        switch (L) {
        case 4: hipLaunchKernelGGL((k_lu_eliminate<4, true>), g, b, 0, s, bs, a, n, c, j0, je, piv, info, pc, next); break;
        case 8: hipLaunchKernelGGL((k_lu_eliminate<8, true>), g, b, 0, s, bs, a, n, c, j0, je, piv, info, pc, next); break;
        case 16:
            hipLaunchKernelGGL((k_lu_eliminate<16, true>), g, b, 0, s, bs, a, n, c, j0, je, piv, info, pc, next);
            break;
        default: return hipErrorInvalidValue;
        }
    } else {
        if (rows <= 0) return hipSuccess;
        MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_eliminate<LL, false>), dim3((unsigned)ng), dim3(ELIM_THREADS), 0,
                                             s, bs, a, n, c, j0, je, piv, info, pc, next));
    }
    return hipGetLastError();
}

hipError_t launch_lu_pivot_copy(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                int32_t* piv, int32_t* info, const PanelCopy& pc, hipStream_t s)
{
    if (L >= 64 || c <= j0 || c >= je || je > n || !pc.keys_in || !pc.cand_in || !pc.cmax_in ||
        pc.cld < je - j0 || pc.nch != (n + ELIM_ROWS - 1) / ELIM_ROWS)
        return hipErrorInvalidValue;
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_pivot_copy<LL>), dim3(1), dim3(64), 0, s, bs, a, n, c, j0, je, piv,
                                         info, pc));
    return hipGetLastError();
}

hipError_t launch_lu_u12(int L, const Bases& bs, MatRef a, int64_t j0, int64_t kb, int64_t je, int64_t n,
                         hipStream_t s)
{
    if (n - je <= 0 || kb <= 1) return hipSuccess;
    if (L >= 64) return launch_lu_u12_wide(L, bs, a, j0, kb, je, n, s);
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_u12<LL>), dim3((unsigned)(n - je)), dim3(64), 0, s, bs, a, j0, kb, je));
    return hipGetLastError();
}

hipError_t launch_lu_laswp(int L, const Bases& bs, MatRef a, const int32_t* piv, int64_t k0, int64_t k1,
                           int64_t c0, int64_t c1, int64_t c2, int64_t c3, hipStream_t s)
{
    const int64_t nc = (c1 - c0) + (c3 - c2);
    if (nc <= 0 || k1 <= k0) return hipSuccess;
    const dim3 g((unsigned)((nc + LASWP_CW - 1) / LASWP_CW), (unsigned)(L + 2));
    for (int64_t k = k0; k < k1; k += LASWP_MAXK) {
        const int64_t ke = k + LASWP_MAXK < k1 ? k + LASWP_MAXK : k1;
        if (L >= 64) {   // the permutation moves words of every plane alike: any L
            hipLaunchKernelGGL((k_lu_laswp<4>), g, dim3(LASWP_THREADS), 0, s, bs, a, piv, k, ke, c0, c1, c2, c3);
            continue;
        }
        MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_laswp<LL>), g, dim3(LASWP_THREADS), 0, s, bs, a, piv, k, ke, c0,
                                             c1, c2, c3));
    }
    return hipGetLastError();
}

hipError_t launch_lu_solve(int L, const Bases& bs, MatRef lu, MatRef x, const int32_t* piv, int64_t n, uint32_t* luT,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (L >= 64) return launch_lu_solve_wide(L, bs, lu, x, piv, n, s);
    if (n <= 8 * SOLVE_REG_THREADS) {
        if (!luT) return hipErrorInvalidValue;
        const unsigned nb = (unsigned)((n + 15) / 16);
        hipLaunchKernelGGL(k_lu_transpose, dim3(nb, nb, (unsigned)(L + 2)), dim3(256), 0, s,
                           base_ptr(bs, lu.base) + lu.off, lu.ld, lu.ps, luT, n);
        Bases bt = bs;
        bt.p[BASE_C] = luT;
        const MatRef t{BASE_C, 0, 0, n, n * n};
        const dim3 g(1), b(SOLVE_REG_THREADS);
        if (n <= SOLVE_REG_THREADS) {
            MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_solve_reg<LL, 1>), g, b, 0, s, bt, t, x, piv, n));
        } else if (n <= 2 * SOLVE_REG_THREADS) {
            MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_solve_reg<LL, 2>), g, b, 0, s, bt, t, x, piv, n));
        } else if (n <= 4 * SOLVE_REG_THREADS) {
            MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_solve_reg<LL, 4>), g, b, 0, s, bt, t, x, piv, n));
        } else {
            MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_solve_reg<LL, 8>), g, b, 0, s, bt, t, x, piv, n));
        }
        return hipGetLastError();
    }
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_solve<LL>), dim3(1), dim3(SOLVE_THREADS), 0, s, bs, lu, x, piv, n));
    return hipGetLastError();
}

}  // namespace mpg
