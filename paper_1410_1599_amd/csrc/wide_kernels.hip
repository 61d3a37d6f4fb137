// wide_kernels.hip -- the kernels of the product and of LU for p = 2048, 4096,
// 8192 and 10240 bits, one value per wavefront (wide.hpp).  They run the same
// scalar operations in the same order as the one-value-per-lane kernels
// (gemm_kernels.hip, lu_kernels.hip), so the results are the same correctly
// rounded sequence the CPU oracle forms; a workgroup of four waves walks the
// same tiles, each wave taking every fourth element of a tile.
#include <algorithm>

#include "launch.hpp"
#include "node_ops.hpp"
#include "wide.hpp"

namespace mpg {

namespace {

constexpr int WT = 256;                // threads per workgroup: four waves
constexpr int WW = WT / 64;
// A tile (256 elements of a leaf product or node pass) is split over SPLIT
// workgroups, so every element gets its own wave: enough waves per SIMD to
// hide the latency of the long dependent carry chains of one value.
constexpr int SPLIT = 16, PER = 256 / SPLIT;

template <int L>
__device__ __forceinline__ WMP<L> wld(const Bases& bs, const MatRef& r, int64_t i, int64_t j)
{
    return wload<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j);
}

template <int L>
__device__ __forceinline__ void wst(const Bases& bs, const MatRef& r, int64_t i, int64_t j, const WMP<L>& v)
{
    wstore<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j, v);
}

__device__ __forceinline__ int wave_id() { return (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ------------------------------------------------------------------ leaf products

// Simple (eq. (1)), and Block, which has the same per-element order: c :=
// add_rn(c, mul_rn(a_ik, b_kj)) for k ascending from exact zero (or from C
// for an accumulating task).  A tile is the same 256-element block the
// one-value-per-lane kernel gives a workgroup.
template <int L>
__global__ void __launch_bounds__(WT)
k_gemm_w(const GemmTask* __restrict__ tasks, const int32_t* __restrict__ tile_task, int64_t ntiles, Bases bs)
{
    const int w = wave_id();
    static_assert(64 * GEMM_TM == 256, "a leaf tile holds 256 elements");
    for (int64_t vb = blockIdx.x; vb < ntiles * SPLIT; vb += gridDim.x) {
        const int64_t t = vb / SPLIT;
        const int part = (int)(vb % SPLIT);
        const GemmTask T = tasks[tile_task[t]];
        const int64_t lt = t - T.tile0;
        const int tc = 1 << T.tcl;
        const int tr = (64 * GEMM_TM) >> T.tcl;
        const int tn = (T.n + tc - 1) >> T.tcl;
        for (int el = part * PER + w; el < (part + 1) * PER; el += WW) {
            const int64_t i = (lt / tn) * tr + (el >> T.tcl);
            const int64_t j = (lt % tn) * tc + (el & (tc - 1));
            if (i >= T.m || j >= T.n) continue;
            WMP<L> c = T.accum ? wld<L>(bs, T.C, i, j) : wzero<L>();
            for (int k = 0; k < T.l; k++) {
                const WMP<L> a = T.at ? wld<L>(bs, T.A, k, i) : wld<L>(bs, T.A, i, k);   // a transposed copy, or not
                c = add_rn<L>(c, mul_rn<L>(a, wld<L>(bs, T.B, k, j)));
            }
            wst<L>(bs, T.C, i, j, c);
        }
    }
}

// ------------------------------------------------------------------ node passes

template <int L, int OP>
__global__ void __launch_bounds__(WT)
k_node_w(const NodeTask* __restrict__ tasks, const int32_t* __restrict__ tile_task, int64_t ntiles, Bases bs)
{
    const int w = wave_id();
    static_assert(NODE_TILE == 256, "a node tile holds 256 elements");
    for (int64_t vb = blockIdx.x; vb < ntiles * SPLIT; vb += gridDim.x) {
        const int64_t t = vb / SPLIT;
        const int part = (int)(vb % SPLIT);
        const NodeTask& T = tasks[tile_task[t]];
        const int64_t total = (int64_t)T.rows * T.cols;
        for (int el = part * PER + w; el < (part + 1) * PER; el += WW) {
            const int64_t e = (t - T.tile0) * NODE_TILE + el;
            if (e >= total) break;
            node_apply<WMP<L>, L, OP>(bs, T, e / T.cols, e % T.cols);
        }
    }
}

// ------------------------------------------------------------------ LU (Section 4)

// Pivot of column c: the first row index r >= c of the largest |a_rc| (each
// wave scans every WW-th row, then wave 0 compares the WW candidates through
// LDS in index order, ties to the smaller index); piv[c] = r, info = c + 1 for
// the first exactly zero pivot; then rows c and r are swapped over the panel
// columns [j0, je).  search == 0: no exchange, the pivot is a_cc.
template <int L>
__global__ void __launch_bounds__(WT)
k_lu_pivot_swap_w(Bases bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je, int32_t* piv, int32_t* info,
                  int search)
{
    constexpr int R = L / 64;
    __shared__ uint32_t sm[WW][L + 2];
    __shared__ int32_t sidx[WW];
    __shared__ int32_t s_r;
    const int w = wave_id(), t = wlane();
    if (!search) {
        if (w == 0) {
            const bool z = wis_zero<L>(wld<L>(bs, a, c, c));
            if (t == 0) {
                piv[c] = (int32_t)c;
                if (z && info[0] == 0) info[0] = (int32_t)(c + 1);
            }
        }
        return;
    }
    int64_t best = -1;
    WMP<L> bv = wzero<L>();
    for (int64_t i = c + w; i < n; i += WW) {
        const WMP<L> v = wld<L>(bs, a, i, c);
        if (best < 0 || cmp_abs<L>(v, bv) > 0) {
            best = i;
            bv = v;
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) sm[w][R * t + r] = bv.m[r];
    if (t == 0) {
        sm[w][L] = (uint32_t)bv.e;
        sm[w][L + 1] = bv.s;
        sidx[w] = (int32_t)best;
    }
    __syncthreads();
    if (w == 0) {
        int32_t bi = -1;
        WMP<L> bx = wzero<L>();
        for (int q = 0; q < WW; q++) {
            const int32_t iq = sidx[q];
            if (iq < 0) continue;
            WMP<L> x;
#pragma unroll
            for (int r = 0; r < R; r++) x.m[r] = sm[q][R * t + r];
            x.e = (int32_t)sm[q][L];
            x.s = sm[q][L + 1];
            const int cm = bi < 0 ? 1 : cmp_abs<L>(x, bx);
            if (cm > 0 || (cm == 0 && iq < bi)) {
                bi = iq;
                bx = x;
            }
        }
        const bool z = wis_zero<L>(bx);
        if (t == 0) {
            s_r = bi;
            piv[c] = bi;
            if (z && info[0] == 0) info[0] = (int32_t)(c + 1);
        }
    }
    __syncthreads();
    const int64_t r = s_r;
    if (r != c) {
        // words e = q wd + (j - j0) of the two rows, SW per thread per round,
        // all loads of a round before any store (the rows never overlap)
        constexpr int SW = 16;
        uint32_t* p = base_ptr(bs, a.base) + a.off;
        const uint32_t wd = (uint32_t)(je - j0), tot = wd * (uint32_t)(L + 2);
        uint32_t* rc = p + c * a.ld + j0;
        uint32_t* rr = p + r * a.ld + j0;
        for (uint32_t e0 = 0; e0 < tot; e0 += SW * WT) {
            uint32_t xv[SW], yv[SW];
            int64_t off[SW];
#pragma unroll
            for (int u = 0; u < SW; u++) {
                const uint32_t e = e0 + (uint32_t)(u * WT) + threadIdx.x;
                off[u] = e < tot ? (int64_t)(e / wd) * a.ps + (e % wd) : -1;
                if (off[u] >= 0) {
                    xv[u] = rc[off[u]];
                    yv[u] = rr[off[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < SW; u++) {
                if (off[u] >= 0) {
                    rc[off[u]] = yv[u];
                    rr[off[u]] = xv[u];
                }
            }
        }
    }
}

// one wave per row i in (c, n): the multiplier l_i = a_ic / a_cc replaces a_ic;
// a zero pivot skips the column (no quotient, no update)
template <int L>
__global__ void __launch_bounds__(64)
k_lu_div_col_w(Bases bs, MatRef a, int64_t c)
{
    const int64_t i = c + 1 + blockIdx.x;
    const WMP<L> d = wld<L>(bs, a, c, c);
    if (wis_zero<L>(d)) return;
    wst<L>(bs, a, i, c, div_rn<L>(wld<L>(bs, a, i, c), d));
}

// a_ij := a_ij - l_i a_cj for the rows i in (c, n) and the panel columns j in
// (c, je), one wave per element; l_i is a_ic, which k_lu_div_col_w has just
// made the multiplier (nothing to do after a zero pivot)
template <int L>
__global__ void __launch_bounds__(WT)
k_lu_rank1_w(Bases bs, MatRef a, int64_t n, int64_t c, int64_t je)
{
    const int64_t wj = je - c - 1;
    const int64_t e = (int64_t)blockIdx.x * WW + wave_id();
    if (e >= (n - c - 1) * wj) return;
    const int64_t i = c + 1 + e / wj, j = c + 1 + e % wj;
    if (wis_zero<L>(wld<L>(bs, a, c, c))) return;
    wst<L>(bs, a, i, j, sub_rn<L>(wld<L>(bs, a, i, j), mul_rn<L>(wld<L>(bs, a, i, c), wld<L>(bs, a, c, j))));
}

// U12 := L11^-1 A12, one workgroup of WU / 64 waves per column j >= je: step t
// updates the rows r > t of the panel with row t (rows split over the waves, a
// barrier between steps), the same order as the one-value-per-lane kernel
constexpr int WU = 512;

template <int L>
__global__ void __launch_bounds__(WU)
k_lu_u12_w(Bases bs, MatRef a, int64_t j0, int64_t kb, int64_t je)
{
    const int64_t j = je + blockIdx.x;
    const int w = wave_id();
    for (int64_t t = 0; t < kb - 1; t++) {
        const WMP<L> u = wld<L>(bs, a, j0 + t, j);
        for (int64_t r = t + 1 + w; r < kb; r += WU / 64)
            wst<L>(bs, a, j0 + r, j, sub_rn<L>(wld<L>(bs, a, j0 + r, j), mul_rn<L>(wld<L>(bs, a, j0 + r, j0 + t), u)));
        __syncthreads();
    }
}

// x := U^-1 L^-1 P b in one workgroup of 16 waves (the vector in global
// memory, a barrier between steps)
// The solve, one launch per step so that every row has its own wave on any CU
// (one workgroup would give each of its 16 waves n / 16 rows per step):
// k_lu_solve_perm_w applies the row exchanges to b in order (one wave);
// k_lu_fwd_w (step t of L y = P b, unit diagonal) updates the rows r > t with
// the finished y_t; k_lu_div_w finishes x_(n-1) = y_(n-1) / u_(n-1,n-1);
// k_lu_bwd_w (step t of U x = y) updates the rows r < t with the finished
// x_t, and the wave of row t - 1, whose update was its last, divides it by
// u_(t-1,t-1) so that the next step finds it finished.  Every element sees
// the operations of the one-workgroup solve in the same order.
template <int L>
__global__ void __launch_bounds__(64)
k_lu_solve_perm_w(Bases bs, MatRef x, const int32_t* piv, int64_t n)
{
    for (int64_t k = 0; k < n; k++) {
        const int64_t r = piv[k];
        if (r == k) continue;
        const WMP<L> u = wld<L>(bs, x, k, 0), v = wld<L>(bs, x, r, 0);
        wst<L>(bs, x, k, 0, v);
        wst<L>(bs, x, r, 0, u);
    }
}

template <int L>
__global__ void __launch_bounds__(WT)
k_lu_fwd_w(Bases bs, MatRef lu, MatRef x, int64_t n, int64_t t)
{
    const int64_t r = t + 1 + (int64_t)blockIdx.x * WW + wave_id();
    if (r >= n) return;
    const WMP<L> yt = wld<L>(bs, x, t, 0);
    wst<L>(bs, x, r, 0, sub_rn<L>(wld<L>(bs, x, r, 0), mul_rn<L>(wld<L>(bs, lu, r, t), yt)));
}

template <int L>
__global__ void __launch_bounds__(64)
k_lu_div_w(Bases bs, MatRef lu, MatRef x, int64_t t)
{
    wst<L>(bs, x, t, 0, div_rn<L>(wld<L>(bs, x, t, 0), wld<L>(bs, lu, t, t)));
}

template <int L>
__global__ void __launch_bounds__(WT)
k_lu_bwd_w(Bases bs, MatRef lu, MatRef x, int64_t t)
{
    const int64_t r = (int64_t)blockIdx.x * WW + wave_id();
    if (r >= t) return;
    const WMP<L> xt = wld<L>(bs, x, t, 0);
    WMP<L> v = sub_rn<L>(wld<L>(bs, x, r, 0), mul_rn<L>(wld<L>(bs, lu, r, t), xt));
    if (r == t - 1) v = div_rn<L>(v, wld<L>(bs, lu, r, r));
    wst<L>(bs, x, r, 0, v);
}

}  // namespace

#define MPG_DISPATCH_WIDE(L_, CALL)                    \
    switch (L_) {                                      \
    case 64: { constexpr int LL = 64; CALL; break; }   \
    case 128: { constexpr int LL = 128; CALL; break; } \
    case 256: { constexpr int LL = 256; CALL; break; } \
    case 320: { constexpr int LL = 320; CALL; break; } \
    default: return hipErrorInvalidValue;              \
    }

hipError_t launch_gemm_wide(int L, const GemmTask* tasks, const int32_t* tile_task, int64_t ntiles, const Bases& bs,
                            int64_t grid, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(grid * SPLIT, int64_t(1) << 30);
    MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_gemm_w<LL>), dim3((unsigned)g), dim3(WT), 0, s, tasks, tile_task,
                                            ntiles, bs));
    return hipGetLastError();
}

template <int L>
static hipError_t node_wide_L(int op, const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles,
                              const Bases& bs, int64_t grid, hipStream_t s)
{
    const dim3 g((unsigned)grid), b(WT);
    switch (op) {
    case OP_ADD: hipLaunchKernelGGL((k_node_w<L, OP_ADD>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_SUB: hipLaunchKernelGGL((k_node_w<L, OP_SUB>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_MUL: hipLaunchKernelGGL((k_node_w<L, OP_MUL>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_DIV: hipLaunchKernelGGL((k_node_w<L, OP_DIV>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_COPY: hipLaunchKernelGGL((k_node_w<L, OP_COPY>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_PADCOPY: hipLaunchKernelGGL((k_node_w<L, OP_PADCOPY>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_WINO_A: hipLaunchKernelGGL((k_node_w<L, OP_WINO_A>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_WINO_B: hipLaunchKernelGGL((k_node_w<L, OP_WINO_B>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_WINO_C: hipLaunchKernelGGL((k_node_w<L, OP_WINO_C>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_STR_A: hipLaunchKernelGGL((k_node_w<L, OP_STR_A>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_STR_B: hipLaunchKernelGGL((k_node_w<L, OP_STR_B>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    case OP_STR_C: hipLaunchKernelGGL((k_node_w<L, OP_STR_C>), g, b, 0, s, tasks, tile_task, ntiles, bs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_node_wide(int L, int op, const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles,
                            const Bases& bs, int64_t grid, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(grid * SPLIT, int64_t(1) << 30);
    switch (L) {
    case 64: return node_wide_L<64>(op, tasks, tile_task, ntiles, bs, g, s);
    case 128: return node_wide_L<128>(op, tasks, tile_task, ntiles, bs, g, s);
    case 256: return node_wide_L<256>(op, tasks, tile_task, ntiles, bs, g, s);
    case 320: return node_wide_L<320>(op, tasks, tile_task, ntiles, bs, g, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lu_pivot_swap_wide(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                     int32_t* piv, int32_t* info, int search, hipStream_t s)
{
    MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_pivot_swap_w<LL>), dim3(1), dim3(WT), 0, s, bs, a, n, c, j0, je,
                                            piv, info, search));
    return hipGetLastError();
}

hipError_t launch_lu_eliminate_wide(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t je,
                                    hipStream_t s)
{
    if (n - c - 1 <= 0) return hipSuccess;
    // the multipliers (one wave per row), then the rank-one update of the
    // panel (one wave per element)
    MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_div_col_w<LL>), dim3((unsigned)(n - c - 1)), dim3(64), 0, s, bs,
                                            a, c));
    const int64_t cnt = (n - c - 1) * (je - c - 1);
    if (cnt > 0) {
        const unsigned g = (unsigned)((cnt + WW - 1) / WW);
        MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_rank1_w<LL>), dim3(g), dim3(WT), 0, s, bs, a, n, c, je));
    }
    return hipGetLastError();
}

hipError_t launch_lu_u12_wide(int L, const Bases& bs, MatRef a, int64_t j0, int64_t kb, int64_t je, int64_t n,
                              hipStream_t s)
{
    if (n - je <= 0 || kb <= 1) return hipSuccess;
    MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_u12_w<LL>), dim3((unsigned)(n - je)), dim3(WU), 0, s, bs, a, j0,
                                            kb, je));
    return hipGetLastError();
}

hipError_t launch_lu_solve_wide(int L, const Bases& bs, MatRef lu, MatRef x, const int32_t* piv, int64_t n,
                                hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_solve_perm_w<LL>), dim3(1), dim3(64), 0, s, bs, x, piv, n));
    for (int64_t t = 0; t + 1 < n; t++) {
        const unsigned g = (unsigned)((n - t - 1 + WW - 1) / WW);
        MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_fwd_w<LL>), dim3(g), dim3(WT), 0, s, bs, lu, x, n, t));
    }
    MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_div_w<LL>), dim3(1), dim3(64), 0, s, bs, lu, x, n - 1));
    for (int64_t t = n - 1; t >= 1; t--) {
        const unsigned g = (unsigned)((t + WW - 1) / WW);
        MPG_DISPATCH_WIDE(L, hipLaunchKernelGGL((k_lu_bwd_w<LL>), dim3(g), dim3(WT), 0, s, bs, lu, x, t));
    }
    return hipGetLastError();
}

}  // namespace mpg
