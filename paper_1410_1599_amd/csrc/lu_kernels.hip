// lu_kernels.hip -- the steps of blocked LU with partial pivoting (Section 4)
// and of the triangular solves.  The matrix is one MatRef; every element
// update is c := sub_rn(c, mul_rn(l, u)), so each element sees the same
// sequence of correctly rounded operations as the CPU oracle.
#include "launch.hpp"
#include "mp_arith.hpp"

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

constexpr int PIV_THREADS = 1024;

// one workgroup: the pivot of column c is the first row index r >= c of the
// largest |a_rc| (exact comparison; a tree reduction in LDS, ties to the
// smaller index); piv[c] = r, info = c + 1 for the first exactly zero pivot;
// then the same workgroup swaps rows c and r over the panel columns [j0, je)
template <int L>
__global__ void __launch_bounds__(PIV_THREADS)
k_lu_pivot_swap(Bases bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je, int32_t* piv, int32_t* info)
{
    __shared__ int32_t sidx[PIV_THREADS];
    const int tid = threadIdx.x;
    int32_t best = -1;
    MP<L> bv = mp_zero<L>();
    for (int64_t i = c + tid; i < n; i += PIV_THREADS) {
        const MP<L> v = ldm<L>(bs, a, i, c);
        if (best < 0 || cmp_abs<L>(v, bv) > 0) {
            best = (int32_t)i;
            bv = v;
        }
    }
    sidx[tid] = best;
    __syncthreads();
    for (int s = PIV_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const int32_t i1 = sidx[tid], i2 = sidx[tid + s];
            if (i2 >= 0) {
                if (i1 < 0) {
                    sidx[tid] = i2;
                } else {
                    const int cm = cmp_abs<L>(ldm<L>(bs, a, i2, c), ldm<L>(bs, a, i1, c));
                    if (cm > 0 || (cm == 0 && i2 < i1)) sidx[tid] = i2;
                }
            }
        }
        __syncthreads();
    }
    const int64_t r = sidx[0];
    if (tid == 0) {
        piv[c] = (int32_t)r;
        if (is_zero<L>(ldm<L>(bs, a, r, c)) && info[0] == 0) info[0] = (int32_t)(c + 1);
    }
    if (r != c) {
        uint32_t* p = base_ptr(bs, a.base) + a.off;
        const int64_t w = je - j0;
        for (int64_t e = tid; e < w * (L + 2); e += PIV_THREADS) {
            const int64_t j = j0 + e % w, q = e / w;
            uint32_t* x = p + q * a.ps + c * a.ld + j;
            uint32_t* y = p + q * a.ps + r * a.ld + j;
            const uint32_t t = *x;
            *x = *y;
            *y = t;
        }
    }
}

// one workgroup per row i in (c, n): l = a_ic / a_cc by one lane, shared in
// LDS, then a_ij := a_ij - l a_cj for the panel columns j in (c, je)
constexpr int ELIM_THREADS = 64;

template <int L>
__global__ void __launch_bounds__(ELIM_THREADS)
k_lu_eliminate(Bases bs, MatRef a, int64_t c, int64_t je)
{
    __shared__ uint32_t sl[L + 2];
    const int64_t i = c + 1 + blockIdx.x;
    if (threadIdx.x == 0) {
        const MP<L> l = div_rn<L>(ldm<L>(bs, a, i, c), ldm<L>(bs, a, c, c));
        stm<L>(bs, a, i, c, l);
#pragma unroll
        for (int q = 0; q < L; q++) sl[q] = l.m[q];
        sl[L] = (uint32_t)l.e;
        sl[L + 1] = l.s;
    }
    __syncthreads();
    MP<L> l;
#pragma unroll
    for (int q = 0; q < L; q++) l.m[q] = sl[q];
    l.e = (int32_t)sl[L];
    l.s = sl[L + 1];
    for (int64_t j = c + 1 + threadIdx.x; j < je; j += ELIM_THREADS)
        stm<L>(bs, a, i, j, sub_rn<L>(ldm<L>(bs, a, i, j), mul_rn<L>(l, ldm<L>(bs, a, c, j))));
}

// U12 := L11^-1 A12: one workgroup per column j >= je, one lane per panel row;
// step t updates rows r > t with row t, which step t-1 finished
template <int L>
__global__ void __launch_bounds__(64)
k_lu_u12(Bases bs, MatRef a, int64_t j0, int64_t kb, int64_t je)
{
    const int64_t j = je + blockIdx.x;
    for (int64_t t = 0; t < kb - 1; t++) {
        const MP<L> u = ldm<L>(bs, a, j0 + t, j);
        for (int64_t r = t + 1 + threadIdx.x; r < kb; r += 64)
            stm<L>(bs, a, j0 + r, j, sub_rn<L>(ldm<L>(bs, a, j0 + r, j), mul_rn<L>(ldm<L>(bs, a, j0 + r, j0 + t), u)));
        __syncthreads();
    }
}

// apply the swaps piv[k0 .. k1) in order to columns [col0, col1)
template <int L>
__global__ void __launch_bounds__(256)
k_lu_laswp(Bases bs, MatRef a, const int32_t* piv, int64_t k0, int64_t k1, int64_t col0, int64_t col1)
{
    const int64_t j = col0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= col1) return;
    uint32_t* p = base_ptr(bs, a.base) + a.off;
    for (int64_t k = k0; k < k1; k++) {
        const int64_t r = piv[k];
        if (r == k) continue;
#pragma unroll
        for (int q = 0; q < L + 2; q++) {
            uint32_t* x = p + q * a.ps + k * a.ld + j;
            uint32_t* y = p + q * a.ps + r * a.ld + j;
            const uint32_t t = *x;
            *x = *y;
            *y = t;
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

#define MPG_DISPATCH_L(L_, CALL)           \
    switch (L_) {                          \
    case 4: { constexpr int LL = 4; CALL; break; }   \
    case 8: { constexpr int LL = 8; CALL; break; }   \
    case 16: { constexpr int LL = 16; CALL; break; } \
    default: return hipErrorInvalidValue;  \
    }

hipError_t launch_lu_pivot_swap(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                int32_t* piv, int32_t* info, hipStream_t s)
{
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_pivot_swap<LL>), dim3(1), dim3(PIV_THREADS), 0, s, bs, a, n, c, j0, je,
                                         piv, info));
    return hipGetLastError();
}

hipError_t launch_lu_eliminate(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t je, hipStream_t s)
{
    if (n - c - 1 <= 0) return hipSuccess;
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_eliminate<LL>), dim3((unsigned)(n - c - 1)), dim3(ELIM_THREADS), 0, s,
                                         bs, a, c, je));
    return hipGetLastError();
}

hipError_t launch_lu_u12(int L, const Bases& bs, MatRef a, int64_t j0, int64_t kb, int64_t je, int64_t n,
                         hipStream_t s)
{
    if (n - je <= 0 || kb <= 1) return hipSuccess;
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_u12<LL>), dim3((unsigned)(n - je)), dim3(64), 0, s, bs, a, j0, kb, je));
    return hipGetLastError();
}

hipError_t launch_lu_laswp(int L, const Bases& bs, MatRef a, const int32_t* piv, int64_t k0, int64_t k1,
                           int64_t col0, int64_t col1, int64_t /*ncols_total*/, hipStream_t s)
{
    if (col1 <= col0 || k1 <= k0) return hipSuccess;
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_laswp<LL>), dim3(blocks_for(col1 - col0, 256)), dim3(256), 0, s, bs,
                                         a, piv, k0, k1, col0, col1));
    return hipGetLastError();
}

hipError_t launch_lu_solve(int L, const Bases& bs, MatRef lu, MatRef x, const int32_t* piv, int64_t n,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    MPG_DISPATCH_L(L, hipLaunchKernelGGL((k_lu_solve<LL>), dim3(1), dim3(SOLVE_THREADS), 0, s, bs, lu, x, piv, n));
    return hipGetLastError();
}

}  // namespace mpg
