// slice_kernels.hip -- the INT8-slice product: MP matrices cut into signed
// 8-bit digit planes under per-row (A) and per-column (B) exponent scaling,
// exact INT8 x INT8 -> INT32 products on the matrix cores, recombination in
// wide integers and one rounding to p bits per entry.
//
// With e_i the largest exponent in row i of A and W_A the window width, each
// a_ik becomes the integer alpha_ik = trunc(a_ik 2^(W_A - e_i)) (exact when
// e_i - exp(a_ik) <= W_A - p); likewise beta_kj for B with column maxima
// f_j.  alpha is written in balanced base 256, digits in [-128, 127]:
// alpha = sum_s d_s 256^s.  Then
//     sum_k alpha_ik beta_kj = sum_u 256^u G_u,   G_u = sum_{s+t=u} sum_k dA_s dB_t,
// every G_u is one INT8 GEMM with INT32 accumulation over the concatenated
// inner index (exact while (pairs x l) 2^14 < 2^31; longer diagonals are
// split), and c_ij = RN_p(2^(e_i + f_j - W_A - W_B) sum_u 256^u G_u).
#include "mp_arith.hpp"
#include "slice.hpp"

namespace mpg {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ exponent scan

// Largest and smallest exponent of the nonzero entries of every row (A) or
// column (B); a zero row or column reports max = min = INT32_MIN.
//
// Rows: one workgroup per row, threads across the row (coalesced), LDS tree.
// Columns: a workgroup takes 256 consecutive columns and a chunk of SCAN_ROWS
// rows (coalesced across threads) and writes a partial result per chunk; a
// second small pass folds the chunks.
constexpr int SCAN_ROWS = 64;

__device__ __forceinline__ void fold(int32_t& hi, int32_t& lo, int32_t h2, int32_t l2)
{
    hi = h2 > hi ? h2 : hi;
    lo = l2 < lo ? l2 : lo;
}

template <int L>
__global__ void __launch_bounds__(256)
k_slice_scan_rows(const uint32_t* __restrict__ X, int64_t ld, int64_t ps, int64_t inner, int32_t* __restrict__ emax,
                  int32_t* __restrict__ emin)
{
    __shared__ int32_t sh[256], sl[256];
    const int64_t o = blockIdx.x;
    int32_t hi = INT32_MIN, lo = INT32_MAX;
    for (int64_t q = threadIdx.x; q < inner; q += 256) {
        const int64_t idx = o * ld + q;
        if (X[(L - 1) * ps + idx] == 0) continue;
        const int32_t e = (int32_t)X[L * ps + idx];
        fold(hi, lo, e, e);
    }
    sh[threadIdx.x] = hi;
    sl[threadIdx.x] = lo;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            int32_t h = sh[threadIdx.x], l = sl[threadIdx.x];
            fold(h, l, sh[threadIdx.x + s], sl[threadIdx.x + s]);
            sh[threadIdx.x] = h;
            sl[threadIdx.x] = l;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        emax[o] = sh[0];
        emin[o] = sh[0] == INT32_MIN ? INT32_MIN : sl[0];
    }
}

template <int L>
__global__ void __launch_bounds__(256)
k_slice_scan_cols(const uint32_t* __restrict__ X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
                  int32_t* __restrict__ phi, int32_t* __restrict__ plo)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (o >= outer) return;
    int32_t hi = INT32_MIN, lo = INT32_MAX;
    const int64_t q1 = (chunk + 1) * SCAN_ROWS < inner ? (chunk + 1) * SCAN_ROWS : inner;
    for (int64_t q = chunk * SCAN_ROWS; q < q1; q++) {
        const int64_t idx = q * ld + o;
        if (X[(L - 1) * ps + idx] == 0) continue;
        const int32_t e = (int32_t)X[L * ps + idx];
        fold(hi, lo, e, e);
    }
    phi[chunk * outer + o] = hi;
    plo[chunk * outer + o] = lo;
}

__global__ void __launch_bounds__(256)
k_slice_scan_fold(const int32_t* __restrict__ phi, const int32_t* __restrict__ plo, int64_t outer, int64_t nchunks,
                  int32_t* __restrict__ emax, int32_t* __restrict__ emin)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= outer) return;
    int32_t hi = INT32_MIN, lo = INT32_MAX;
    for (int64_t c = 0; c < nchunks; c++) fold(hi, lo, phi[c * outer + o], plo[c * outer + o]);
    emax[o] = hi;
    emin[o] = hi == INT32_MIN ? INT32_MIN : lo;
}

// ------------------------------------------------------------------ slicing

// word w (bits 32w .. 32w+31) of M * 2^sh, M the L-limb mantissa, sh of any
// sign (bits shifted below 0 are dropped: truncation toward zero)
template <int L>
__device__ __forceinline__ uint32_t shifted_word(const uint32_t* m, int32_t sh, int w)
{
    const int32_t pos = 32 * w - sh;                 // bit of M at bit 32w of the result
    const int32_t q = pos >> 5;                      // arithmetic: floor
    const uint32_t r = (uint32_t)pos & 31u;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < L; k++) {
        lo = (q == k) ? m[k] : lo;
        hi = (q + 1 == k) ? m[k] : hi;
    }
    return r ? funnel(hi, lo, r) : lo;
}

// balanced base-256 digits of 4 consecutive inner indices k = 4g .. 4g+3 of
// one outer index o (row of A / column of B), 4 digits per word; zeros
// outside the matrix (the padding of the digit planes)
template <int L, int NW>
__device__ __forceinline__ void slice_digits_of(const uint32_t* __restrict__ X, int64_t ld, int64_t ps, int64_t outer,
                                                int64_t inner, int by_cols, const int32_t* __restrict__ emax,
                                                int32_t W, int64_t o, int64_t g, uint32_t (&dig)[4][NW])
{
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int64_t k = 4 * g + e;
        uint32_t m[L];
        uint32_t sgn = 0;
        int32_t ex = 0;
        bool nz = false;
        if (o < outer && k < inner) {
            const int64_t idx = by_cols ? k * ld + o : o * ld + k;
#pragma unroll
            for (int q = 0; q < L; q++) m[q] = X[q * ps + idx];
            ex = (int32_t)X[L * ps + idx];
            sgn = X[(L + 1) * ps + idx];
            nz = m[L - 1] != 0;
        }
        if (!nz) {
#pragma unroll
            for (int q = 0; q < L; q++) m[q] = 0;
            sgn = 0;
        }
        // alpha = M * 2^(e - p) * 2^(W - emax) = M * 2^sh
        const int32_t sh = nz ? (W - 32 * L - (emax[o] - ex)) : 0;
        // two's complement of +-alpha, word by word, then balanced base-256 recoding
        uint32_t neg_c = sgn;                        // +1 of the negation
        int32_t rc = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            uint32_t a = shifted_word<L>(m, sh, w);
            if (sgn) a = addc(~a, 0u, neg_c, &neg_c);
            uint32_t out = 0;
#pragma unroll
            for (int b = 0; b < 4; b++) {
                int32_t v = (int32_t)((a >> (8 * b)) & 0xffu) + rc;
                rc = v >= 128 ? 1 : 0;
                v -= rc ? 256 : 0;
                out |= ((uint32_t)v & 0xffu) << (8 * b);
            }
            dig[e][w] = out;
        }
    }
}

// digit s of the 4 indices as one dword (4 consecutive k)
template <int NW>
__device__ __forceinline__ uint32_t plane_word(const uint32_t (&dig)[4][NW], int s)
{
    const int w = s >> 2, b = s & 3;
    uint32_t v = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        uint32_t x = 0;
#pragma unroll
        for (int q = 0; q < NW; q++) x = (q == w) ? dig[e][q] : x;
        v |= ((x >> (8 * b)) & 0xffu) << (8 * e);
    }
    return v;
}

// rows of A: one thread per 4 consecutive k of one row (consecutive threads,
// consecutive k: the reads and the digit-plane writes coalesce); writes digit
// plane s at D[s * dps + o * kpad + k]
template <int L, int NW>
__global__ void __launch_bounds__(256)
k_slice_digits(const uint32_t* __restrict__ X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
               const int32_t* __restrict__ emax, int32_t W, int32_t S, int8_t* __restrict__ D, int64_t dps,
               int64_t outer_pad, int64_t kpad)
{
    const int64_t gidx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ngroups = kpad >> 2;
    const int64_t g = gidx % ngroups, o = gidx / ngroups;
    if (o >= outer_pad) return;
    uint32_t dig[4][NW];
    slice_digits_of<L, NW>(X, ld, ps, outer, inner, 0, emax, W, o, g, dig);
    for (int s = 0; s < S; s++) *(uint32_t*)(D + (int64_t)s * dps + o * kpad + 4 * g) = plane_word<NW>(dig, s);
}

// columns of B: a workgroup takes 32 columns x 64 k.  Consecutive threads take
// consecutive columns (the reads of B coalesce); each digit plane goes out
// through an LDS tile so that every column's 64 digits are written as one
// 64-byte row segment of the k-contiguous plane.
constexpr int DC_COLS = 32, DC_GROUPS = 16, DC_THREADS = DC_COLS * DC_GROUPS;

template <int L, int NW>
__global__ void __launch_bounds__(DC_THREADS)
k_slice_digits_cols(const uint32_t* __restrict__ X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
                    const int32_t* __restrict__ emax, int32_t W, int32_t S, int8_t* __restrict__ D, int64_t dps,
                    int64_t kpad)
{
    __shared__ uint32_t tile[DC_COLS][DC_GROUPS + 1];
    const int tid = threadIdx.x;
    const int ol = tid % DC_COLS, gl = tid / DC_COLS;
    const int64_t o0 = (int64_t)blockIdx.x * DC_COLS, g0 = (int64_t)blockIdx.y * DC_GROUPS;
    uint32_t dig[4][NW];
    slice_digits_of<L, NW>(X, ld, ps, outer, inner, 1, emax, W, o0 + ol, g0 + gl, dig);
    const int r = tid / DC_GROUPS, c = tid % DC_GROUPS;
    for (int s = 0; s < S; s++) {
        tile[ol][gl] = plane_word<NW>(dig, s);
        __syncthreads();
        *(uint32_t*)(D + (int64_t)s * dps + (o0 + r) * kpad + 4 * (g0 + c)) = tile[r][c];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ INT8 products

constexpr int TM = SLICE_TILE_M, TN = SLICE_TILE_N, TKK = SLICE_KSTEP;
constexpr int GT = 512;                            // 8 waves: 2 (rows) x 4 (columns) of 128 x 64
constexpr int WM = 128, WN = 64;                   // wave tile
constexpr int FA = WM / 32, FB = WN / 32;          // 32 x 32 MFMA blocks per wave: FA x FB
constexpr int NST = 4;                             // LDS stages in flight
static_assert(2 * WM == TM && 4 * WN == TN, "wave grid 2 x 4");
static_assert(TKK == 64 && TM == 256 && TN == 256 && FA == 4 && FB == 2,
              "the load map and the fragment reads below assume these shapes");

// vmcnt(n), n < 64, with the other counters left alone (gfx9 encoding: vmcnt
// bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
#define SLICE_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x0F70 | ((n) & 15) | (((n) >> 4) << 14))

// LDS holds a stage as 64-byte rows of 4 chunks of 16 bytes; chunk g of row r
// sits at position g ^ ((r >> 2) & 3), so the 16 rows one MFMA fragment read
// touches at a time cover all 64 banks.

// LDS byte address of a shared-memory pointer
__device__ __forceinline__ uint32_t lds_addr(const int8_t* p)
{
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) int8_t*)p;
}

// global_load_lds_dwordx4: each lane's 16 bytes at src go to LDS at
// lds + 16 * lane.  Issued through asm so that the compiler, which would make
// every later LDS read wait for all such loads, leaves the waiting to the
// kernel's explicit vmcnt waits (the instruction has no register result).
__device__ __forceinline__ void lds_dma16(const int8_t* src, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %1\n\t"
                 "s_nop 0\n\t"
                 "global_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(lds)
                 : "m0", "memory");
}

// One workgroup: a 256 x 256 tile of G_slot = sum_{s = s0}^{s1 - 1} A8_s B8_{u-s}^T.
// The inner loop walks (pair, 64-wide k step).  Operands go from global memory
// straight into LDS (global_load_lds_dwordx4: lane l of a wave writes the 16
// bytes at wave base + 16 l), NST - 1 steps ahead of the matrix cores; one
// barrier per step.  A wave's 128 x 64 block is 4 x 2 MFMA blocks of
// 32 x 32 x 32 (on gfx950 the 32 x 32 x 32 INT8 form issues twice the MACs per
// cycle of 16 x 16 x 64); it reads 12 KB of LDS per step (1/43 byte per MAC).
__global__ void __launch_bounds__(GT)
k_slice_gemm(const SliceTask* __restrict__ tasks, const int8_t* __restrict__ A8, const int8_t* __restrict__ B8,
             int32_t* __restrict__ G, int64_t a_plane, int64_t b_plane, int64_t g_plane, int32_t kpad,
             int32_t npad, const int32_t* __restrict__ flags, int32_t tj_n)
{
    __shared__ __attribute__((aligned(16))) int8_t sA[NST][TM * TKK];
    __shared__ __attribute__((aligned(16))) int8_t sB[NST][TN * TKK];
    const SliceTask T = tasks[blockIdx.x];
    // second pass of the certified early stop: only tiles that hold an entry
    // whose rounding the first pass could not decide
    if (flags != nullptr && flags[T.ti * tj_n + T.tj] == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 2, wx = wave & 3;
    v16i acc[FA][FB];
#pragma unroll
    for (int a = 0; a < FA; a++)
#pragma unroll
        for (int b = 0; b < FB; b++)
#pragma unroll
            for (int e = 0; e < 16; e++) acc[a][b][e] = 0;
    const int64_t i0 = (int64_t)T.ti * TM, j0 = (int64_t)T.tj * TN;
    const int ksteps = kpad / TKK;
    const int nsteps = (T.s1 - T.s0) * ksteps;
    // wave w loads tile rows 32 w .. 32 w + 31 of A and of B, 16 rows per
    // instruction; lane l brings row l / 4 of the 16, the chunk that belongs
    // at its LDS position l % 4
    const int lrow = lane >> 2;
    const int lchunk = (lane & 3) ^ ((lane >> 4) & 3);
    auto issue = [&](int step) {
        const int s = T.s0 + step / ksteps;
        const int k0 = (step % ksteps) * TKK;
        const int buf = step % NST;
        const int8_t* Ab = A8 + (int64_t)s * a_plane + (i0 + 32 * wave) * kpad + k0;
        const int8_t* Bb = B8 + (int64_t)(T.u - s) * b_plane + (j0 + 32 * wave) * kpad + k0;
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int64_t off = (int64_t)(16 * b + lrow) * kpad + 16 * lchunk;
            lds_dma16(Ab + off, __builtin_amdgcn_readfirstlane(lds_addr(&sA[buf][(32 * wave + 16 * b) * TKK])));
            lds_dma16(Bb + off, __builtin_amdgcn_readfirstlane(lds_addr(&sB[buf][(32 * wave + 16 * b) * TKK])));
        }
    };
    // this lane's fragment rows: A rows wy * 128 + 32 t + (l % 32), B rows
    // wx * 64 + 32 t + (l % 32); the swizzled chunk depends on l only
    const int frow = lane & 31;
    auto compute = [&](int buf) {
        // all fragments of the step first (48 registers), then its 16 MFMAs
        v4i af[TKK / 32][FA], bf[TKK / 32][FB];
#pragma unroll
        for (int h = 0; h < TKK / 32; h++) {         // 32-deep MFMA slices of the step
            // lane l holds row (col) l % 32 of the block, bytes 16 (l / 32) .. +16 of the slice
            const int pos = 16 * ((2 * h + (lane >> 5)) ^ ((lane >> 2) & 3));
#pragma unroll
            for (int t = 0; t < FA; t++) af[h][t] = *(const v4i*)&sA[buf][(wy * WM + 32 * t + frow) * TKK + pos];
#pragma unroll
            for (int t = 0; t < FB; t++) bf[h][t] = *(const v4i*)&sB[buf][(wx * WN + 32 * t + frow) * TKK + pos];
        }
        __builtin_amdgcn_sched_barrier(0);           // keep the reads ahead of the MFMAs
#pragma unroll
        for (int h = 0; h < TKK / 32; h++)
#pragma unroll
            for (int a = 0; a < FA; a++)
#pragma unroll
                for (int b = 0; b < FB; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[h][a], bf[h][b], acc[a][b], 0, 0, 0);
    };
    // 4 load instructions per wave and step: step t may proceed once at most
    // 4 min(NST - 2, nsteps - 1 - t) of this wave's loads are outstanding.
    // The barrier is a bare s_barrier (asm, so no memory access moves across
    // it): every wave has waited for its own loads, and its reads of stage
    // t - 1 have completed (the matrix cores consumed them), so after it
    // stage t is in LDS and stage t - 1 may be overwritten.
    for (int st = 0; st < NST - 1 && st < nsteps; st++) issue(st);
    for (int step = 0; step < nsteps; step++) {
        const int later = nsteps - 1 - step;
        if (later >= 2) SLICE_WAIT_VM(8);
        else if (later == 1) SLICE_WAIT_VM(4);
        else SLICE_WAIT_VM(0);
        asm volatile("s_barrier" ::: "memory");
        if (step + NST - 1 < nsteps) issue(step + NST - 1);
        compute(step % NST);
    }
    int32_t* Gp = G + (int64_t)T.slot * g_plane;
    // output register e of a block is row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
#pragma unroll
    for (int a = 0; a < FA; a++)
#pragma unroll
        for (int b = 0; b < FB; b++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int64_t row = i0 + wy * WM + a * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int64_t col = j0 + wx * WN + b * 32 + (lane & 31);
                Gp[row * npad + col] = acc[a][b][e];
            }
}

// ------------------------------------------------------------------ recombination

// c_ij = RN_p(2^(e_i + f_j - W_A - W_B) * Z), Z = sum_u 256^u G_u,ij.
// slot_begin[u] .. slot_begin[u+1] are the G slots of diagonal u.  The sum is
// kept as signed 64-bit partial sums per 32-bit position, carried once: the
// partial sum of position q takes diagonals 4q .. 4q+3, each at most
// min(S_A, S_B) l 2^14 in magnitude, shifted by at most 24 bits, so it stays
// below min(S_A, S_B) l 2^38 (1 + 2^-8 + 2^-16 + 2^-24) < 2^63 for
// min(S_A, S_B) l < 2^25, which the host guarantees (l <= 131008, S <= 137).
//
// mode 0: every diagonal.  mode 1: only the diagonals u >= ulo (the first pass
// of the certified early stop); the omitted part is below 2^D in magnitude, so
// Z lies within 2^D of the partial sum V.  With sh the position of V's last
// kept bit, RN(Z) = RN(V) when sh - 1 > D and the bits D .. sh-2 of |V| are
// neither all zero nor all one: then V's tail below the kept bits stays more
// than 2^D away from zero, from the midpoint and from a full unit, so neither
// the kept bits, the round bit, nor a tie can change (nor the bit length or
// the sign, since |V| >= 2^(p-1+sh) > 2^D).  Such an entry is written; any
// other marks its tile in flags.  mode 2: every diagonal, only for the
// entries of flagged tiles.
template <int L, int NWZ>
__global__ void __launch_bounds__(256)
k_slice_combine(const int32_t* __restrict__ G, int64_t g_plane, int32_t npad, const int32_t* __restrict__ slot_begin,
                int32_t ndiag, const int32_t* __restrict__ ea, const int32_t* __restrict__ fb, int32_t WA, int32_t WB,
                uint32_t* __restrict__ C, int64_t ldc, int64_t psc, int64_t m, int64_t n, int32_t mode, int32_t ulo,
                int32_t D, int32_t* __restrict__ flags, int32_t tj_n)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m * n) return;
    const int64_t i = e / n, j = e % n;
    const int64_t tile = (i / SLICE_TILE_M) * tj_n + j / SLICE_TILE_N;
    if (mode == 2 && flags[tile] == 0) return;
    const int32_t u_from = mode == 1 ? ulo : 0;
    int64_t acc[NWZ];
#pragma unroll
    for (int q = 0; q < NWZ; q++) acc[q] = 0;
#pragma unroll
    for (int q = 0; q < NWZ; q++) {
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int u = 4 * q + b;
            if (u >= ndiag) break;
            if (u < u_from) continue;
            for (int sl = slot_begin[u]; sl < slot_begin[u + 1]; sl++)
                acc[q] += (int64_t)G[(int64_t)sl * g_plane + i * npad + j] * ((int64_t)1 << (8 * b));
        }
    }
    // carry into two's complement limbs
    uint32_t Z[NWZ];
    int64_t cy = 0;
#pragma unroll
    for (int q = 0; q < NWZ; q++) {
        const int64_t t = acc[q] + cy;
        Z[q] = (uint32_t)t;
        cy = t >> 32;
    }
    const bool neg = cy < 0;
    if (neg) {
        uint32_t c = 1;
#pragma unroll
        for (int q = 0; q < NWZ; q++) Z[q] = addc(~Z[q], 0u, c, &c);
    }
    // bit length
    int32_t top = -1;
#pragma unroll
    for (int q = 0; q < NWZ; q++) top = Z[q] ? q : top;
    MP<L> r = mp_zero<L>();
    int32_t b = 0;
    if (top >= 0) {
        uint32_t tw = 0;
#pragma unroll
        for (int q = 0; q < NWZ; q++) tw = (q == top) ? Z[q] : tw;
        b = 32 * top + 32 - (int32_t)__builtin_clz(tw);    // bit length of |Z|
    }
    // keep bits [b - p, b): shift right by sh = b - p (may be negative)
    const int32_t sh = b - 32 * L;
    if (mode == 1) {
        bool certain = false;
        if (top >= 0 && sh - 1 > D) {
            uint32_t any1 = 0, any0 = 0;
#pragma unroll
            for (int t = 0; t < NWZ; t++) {
                const int32_t lo = 32 * t;
                const int32_t a = D > lo ? D : lo;
                const int32_t z = (sh - 1) < lo + 32 ? (sh - 1) : lo + 32;
                if (a < z) {
                    const uint32_t w = (uint32_t)(z - a);
                    const uint32_t mask = (w >= 32u ? 0xffffffffu : ((1u << w) - 1u)) << (uint32_t)(a - lo);
                    any1 |= Z[t] & mask;
                    any0 |= ~Z[t] & mask;
                }
            }
            certain = any1 != 0 && any0 != 0;
        }
        if (!certain) {
            flags[tile] = 1;
            return;
        }
    }
    if (top >= 0) {
        uint32_t M[L];
#pragma unroll
        for (int k = 0; k < L; k++) {
            const int32_t pos = sh + 32 * k;
            const int32_t q = pos >> 5;
            const uint32_t rr = (uint32_t)pos & 31u;
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int t = 0; t < NWZ; t++) {
                lo = (q == t) ? Z[t] : lo;
                hi = (q + 1 == t) ? Z[t] : hi;
            }
            M[k] = rr ? funnel(hi, lo, rr) : lo;
        }
        uint32_t rb = 0, st = 0;
        if (sh > 0) {
            const int32_t rpos = sh - 1;             // round bit position in Z
#pragma unroll
            for (int t = 0; t < NWZ; t++) {
                const int32_t base = 32 * t;
                if (rpos >= base && rpos < base + 32) {
                    rb = (Z[t] >> (rpos - base)) & 1u;
                    st |= Z[t] & ((1u << (rpos - base)) - 1u);
                } else if (base + 32 <= rpos) {
                    st |= Z[t];
                }
            }
        }
        uint32_t cu = rb & ((st != 0) | (M[0] & 1u));
#pragma unroll
        for (int k = 0; k < L; k++) r.m[k] = addc(M[k], 0u, cu, &cu);
        int32_t ex = b + (ea[i] + fb[j] - WA - WB);
        if (cu) {
            r.m[L - 1] = 0x80000000u;
            ex += 1;
        }
        r.e = ex;
        r.s = neg ? 1u : 0u;
    }
    store<L>(C, psc, i * ldc + j, r);
}

__global__ void __launch_bounds__(256) k_slice_fill(int32_t* __restrict__ p, int64_t count, int32_t v)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < count) p[e] = v;
}

}  // namespace

hipError_t launch_slice_scan(int L, const uint32_t* X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
                             int by_cols, int32_t* emax, int32_t* emin, int32_t* tmp, hipStream_t s)
{
    if (outer <= 0) return hipSuccess;
    if (!by_cols) {
        const dim3 g((unsigned)outer);
        switch (L) {
        case 4: hipLaunchKernelGGL((k_slice_scan_rows<4>), g, dim3(256), 0, s, X, ld, ps, inner, emax, emin); break;
        case 8: hipLaunchKernelGGL((k_slice_scan_rows<8>), g, dim3(256), 0, s, X, ld, ps, inner, emax, emin); break;
        case 16: hipLaunchKernelGGL((k_slice_scan_rows<16>), g, dim3(256), 0, s, X, ld, ps, inner, emax, emin); break;
        case 32: hipLaunchKernelGGL((k_slice_scan_rows<32>), g, dim3(256), 0, s, X, ld, ps, inner, emax, emin); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int64_t nchunks = inner > 0 ? (inner + SCAN_ROWS - 1) / SCAN_ROWS : 1;
    int32_t* phi = tmp;
    int32_t* plo = tmp + nchunks * outer;
    const dim3 g((unsigned)((outer + 255) / 256), (unsigned)nchunks);
    switch (L) {
    case 4: hipLaunchKernelGGL((k_slice_scan_cols<4>), g, dim3(256), 0, s, X, ld, ps, outer, inner, phi, plo); break;
    case 8: hipLaunchKernelGGL((k_slice_scan_cols<8>), g, dim3(256), 0, s, X, ld, ps, outer, inner, phi, plo); break;
    case 16: hipLaunchKernelGGL((k_slice_scan_cols<16>), g, dim3(256), 0, s, X, ld, ps, outer, inner, phi, plo); break;
    case 32: hipLaunchKernelGGL((k_slice_scan_cols<32>), g, dim3(256), 0, s, X, ld, ps, outer, inner, phi, plo); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_slice_scan_fold, dim3((unsigned)((outer + 255) / 256)), dim3(256), 0, s, phi, plo, outer,
                       nchunks, emax, emin);
    return hipGetLastError();
}

hipError_t launch_slice_digits(int L, const uint32_t* X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
                               int by_cols, const int32_t* emax, int32_t W, int32_t S, int8_t* D, int64_t dps,
                               int64_t outer_pad, int64_t kpad, hipStream_t s)
{
    // NW = words of the W-bit window plus the recoding headroom, per precision
    if (by_cols) {
        // outer_pad is a multiple of the 256-row tile, kpad of the 64-deep k step
        if (outer_pad % DC_COLS || (kpad / 4) % DC_GROUPS) return hipErrorInvalidValue;
        const dim3 g((unsigned)(outer_pad / DC_COLS), (unsigned)(kpad / 4 / DC_GROUPS)), b(DC_THREADS);
        switch (L) {
        case 4: hipLaunchKernelGGL((k_slice_digits_cols<4, SLICE_NW4>), g, b, 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, kpad); break;
        case 8: hipLaunchKernelGGL((k_slice_digits_cols<8, SLICE_NW8>), g, b, 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, kpad); break;
        case 16: hipLaunchKernelGGL((k_slice_digits_cols<16, SLICE_NW16>), g, b, 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, kpad); break;
        case 32: hipLaunchKernelGGL((k_slice_digits_cols<32, SLICE_NW32>), g, b, 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, kpad); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int64_t threads = outer_pad * (kpad / 4);
    const dim3 g((unsigned)((threads + 255) / 256));
    switch (L) {
    case 4: hipLaunchKernelGGL((k_slice_digits<4, SLICE_NW4>), g, dim3(256), 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, outer_pad, kpad); break;
    case 8: hipLaunchKernelGGL((k_slice_digits<8, SLICE_NW8>), g, dim3(256), 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, outer_pad, kpad); break;
    case 16: hipLaunchKernelGGL((k_slice_digits<16, SLICE_NW16>), g, dim3(256), 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, outer_pad, kpad); break;
    case 32: hipLaunchKernelGGL((k_slice_digits<32, SLICE_NW32>), g, dim3(256), 0, s, X, ld, ps, outer, inner, emax, W, S, D, dps, outer_pad, kpad); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_slice_gemm(const SliceTask* tasks, int64_t ntasks, const int8_t* A8, const int8_t* B8, int32_t* G,
                             int64_t a_plane, int64_t b_plane, int64_t g_plane, int32_t kpad, int32_t npad,
                             const int32_t* flags, int32_t tj_n, hipStream_t s)
{
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_gemm, dim3((unsigned)ntasks), dim3(GT), 0, s, tasks, A8, B8, G, a_plane, b_plane,
                       g_plane, kpad, npad, flags, tj_n);
    return hipGetLastError();
}

hipError_t launch_slice_fill(int32_t* p, int64_t count, int32_t v, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_slice_combine(int L, const int32_t* G, int64_t g_plane, int32_t npad, const int32_t* slot_begin,
                                int32_t ndiag, const int32_t* ea, const int32_t* fb, int32_t WA, int32_t WB,
                                uint32_t* C, int64_t ldc, int64_t psc, int64_t m, int64_t n, int32_t mode,
                                int32_t ulo, int32_t D, int32_t* flags, int32_t tj_n, hipStream_t s)
{
    const dim3 g((unsigned)((m * n + 255) / 256));
    switch (L) {
    case 4: hipLaunchKernelGGL((k_slice_combine<4, SLICE_NWZ4>), g, dim3(256), 0, s, G, g_plane, npad, slot_begin, ndiag, ea, fb, WA, WB, C, ldc, psc, m, n, mode, ulo, D, flags, tj_n); break;
    case 8: hipLaunchKernelGGL((k_slice_combine<8, SLICE_NWZ8>), g, dim3(256), 0, s, G, g_plane, npad, slot_begin, ndiag, ea, fb, WA, WB, C, ldc, psc, m, n, mode, ulo, D, flags, tj_n); break;
    case 16: hipLaunchKernelGGL((k_slice_combine<16, SLICE_NWZ16>), g, dim3(256), 0, s, G, g_plane, npad, slot_begin, ndiag, ea, fb, WA, WB, C, ldc, psc, m, n, mode, ulo, D, flags, tj_n); break;
    case 32: hipLaunchKernelGGL((k_slice_combine<32, SLICE_NWZ32>), g, dim3(256), 0, s, G, g_plane, npad, slot_begin, ndiag, ea, fb, WA, WB, C, ldc, psc, m, n, mode, ulo, D, flags, tj_n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mpg
