// lu.cpp -- host driver of the blocked LU with partial pivoting (Section 4),
// of the paper's unpivoted LU and of the solve; the C-ABI functions mp_lu,
// mp_lu_ex, mp_lu_async, mp_lu_nopivot and mp_lu_solve.
//
// For each panel of K columns starting at j0 (the last one may be narrower):
//   per column c: pivot search, row swap inside the panel, multipliers
//   a_ic / a_cc, rank-one update of the panel's remaining columns;
//   then the panel's swaps on the columns left and right of it;
//   U12 := L11^-1 A12 by one rank-one update of the panel rows per column t;
//   P := L21 U12 with the chosen product algorithm, then A22 := A22 - P.
// Every element therefore sees the operation sequence of the CPU oracle.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"
#include "mpgemm_internal.hpp"
#include "plan.hpp"

using namespace mpg;

namespace {

#define MPG_TRY(expr)                                                    \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) {                                          \
            g_err = std::string("launch failed: ") + hipGetErrorString(e_); \
            return MP_E_DEVICE;                                          \
        }                                                                \
    } while (0)

// info_dev: device int32 that receives info (the first zero pivot + 1, or 0);
// with info_host non-NULL the stream is synchronised and info copied there
// pivot == 0: the paper's LU as published (no row exchanges; piv = identity)
int lu_run(int64_t n, int L, uint32_t* A, int64_t lda, int64_t psa, int32_t* piv, int32_t* info_host,
           int32_t* info_dev, int panel, int algo, int cutoff, int policy, hipStream_t s, int pivot)
{
    int rc = MP_OK;
    const int64_t m2max = n > panel ? n - panel : 0;
    const size_t pwords = (size_t)(L + 2) * (size_t)(m2max * m2max);
    // below 2048 bits the step of column c leaves the keys and a copy of the
    // panel rows for column c + 1 (or, unpivoted, checks its diagonal), and
    // the pivot search of a later column of the panel runs inside its step
    const bool keyed = L < 64;
    const int64_t cld = keyed && pivot ? (panel < n ? panel : n) : 0;
    const size_t cwords = (size_t)(L + 2) * (size_t)n * (size_t)cld;
    const int64_t nch = (n + 3) / 4;
    // aux buffer: the trailing product P, one int32 status word, two sets of
    // n 64-bit keys and nch two-word group records, and two panel copies
    // ((L + 2) is even, so the keys are 8-byte aligned)
    uint32_t* aux = workspace(pwords + 64 + 4 * (size_t)n + 8 * (size_t)nch + 2 * cwords, s, WS_LU, &rc);
    if (rc) return rc;
    int32_t* status = info_dev ? info_dev : (int32_t*)(aux + pwords);
    unsigned long long* k64 = (unsigned long long*)(aux + pwords + 64);
    unsigned long long* keys[2] = {k64, k64 + n};
    unsigned long long* cmax[2] = {k64 + 2 * n, k64 + 2 * n + 2 * nch};
    uint32_t* cand[2] = {(uint32_t*)(k64 + 2 * n + 4 * nch), (uint32_t*)(k64 + 2 * n + 4 * nch) + cwords};
    MPG_TRY(launch_fill_i32(status, 1, 0, s));
    Bases bs{};
    bs.p[BASE_A] = A;
    const MatRef a{BASE_A, 0, 0, lda, psa};
    for (int64_t j0 = 0; j0 < n; j0 += panel) {
        const int64_t kb = (panel < n - j0) ? panel : n - j0;
        const int64_t je = j0 + kb;
        for (int64_t c = j0; c < je; c++) {
            // pivot search and the swap inside the panel; then multipliers and
            // the panel's rank-one update (a zero pivot leaves a zero column, whose
            // quotients and updates are exact no-ops).  Keyed and pivoted, a
            // later step of the panel takes its pivot from the copy the step
            // before left, inside its own launch up to 512 bits (at 1024 the
            // column step has no registers to spare: a launch of its own).
            const bool later = keyed && pivot && c > j0, fused = later && L <= 16;
            const int next = (keyed && c + 1 < je) ? (pivot ? 1 : 2) : 0;
            const int in = (int)((c - j0) & 1), out = in ^ 1;
            const PanelCopy pc{keys[in],  cand[in],  cmax[in],         keys[out], cand[out],
                               cmax[out], (int64_t)n * cld, cld, nch};
            if (c == j0 || !keyed) MPG_TRY(launch_lu_pivot_swap(L, bs, a, n, c, j0, je, piv, status, pivot, s));
            else if (later && !fused) MPG_TRY(launch_lu_pivot_copy(L, bs, a, n, c, j0, je, piv, status, pc, s));
            MPG_TRY(launch_lu_eliminate(L, bs, a, n, c, j0, je, piv, status, pc, next, fused ? 1 : 0, s));
        }
        if (pivot) MPG_TRY(launch_lu_laswp(L, bs, a, piv, j0, je, 0, j0, je, n, s));
        if (je >= n) break;
        MPG_TRY(launch_lu_u12(L, bs, a, j0, kb, je, n, s));
        const int64_t m2 = n - je;
        uint32_t* P = aux;
        const uint32_t* L21 = A + je * lda + j0;
        const uint32_t* U12 = A + j0 * lda + je;
        uint32_t* A22 = A + je * lda + je;
        if ((rc = gemm_internal(m2, kb, m2, L, algo, cutoff, policy, g_leaf, L21, lda, psa, U12, lda, psa, P, m2,
                                m2 * m2, s)))
            return rc;
        if ((rc = ew_internal(OP_SUB, m2, m2, L, A22, lda, psa, P, m2, m2 * m2, A22, lda, psa, s))) return rc;
    }
    if (info_host) {
        MPG_TRY(hipMemcpyAsync(info_host, status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MPG_TRY(hipStreamSynchronize(s));
    }
    return MP_OK;
}

int lu_check(int64_t n, int prec, uint32_t* A, int64_t lda, int64_t psa, int32_t* piv, int panel, int algo,
             int cutoff, int policy, int* L)
{
    int rc;
    if ((rc = check_prec(prec, L))) return rc;
    if ((rc = check_mat("A", A, n, n, lda, psa))) return rc;
    if (panel < 1) return set_err(MP_E_ARG, "panel must be >= 1");
    if (algo < ALGO_SIMPLE || algo > ALGO_WINOGRAD) return set_err(MP_E_ARG, "unknown algorithm");
    if ((algo == ALGO_STRASSEN || algo == ALGO_WINOGRAD) && cutoff < 1) return set_err(MP_E_ARG, "cutoff must be >= 1");
    if (policy < POLICY_PEEL || policy > POLICY_MIXED) return set_err(MP_E_ARG, "unknown odd-size policy");
    if (n > 0 && !piv) return set_err(MP_E_ARG, "piv is NULL");
    return MP_OK;
}

}  // namespace

extern "C" {

int mp_lu_ex(int64_t n, int prec, uint32_t* A, int64_t lda, int64_t psa, int32_t* piv, int32_t* info, int panel,
             int algo, int cutoff, int policy)
{
    int L, rc;
    if (!info) return set_err(MP_E_ARG, "info is NULL");
    *info = 0;
    if ((rc = lu_check(n, prec, A, lda, psa, piv, panel, algo, cutoff, policy, &L))) return rc;
    if (n == 0) return MP_OK;
    if ((rc = device_check())) return rc;
    if ((rc = lu_run(n, L, A, lda, psa, piv, info, nullptr, panel, algo, cutoff, policy, g_stream, 1))) return rc;
    return device_check();
}

int mp_lu_async(int64_t n, int prec, uint32_t* A, int64_t lda, int64_t psa, int32_t* piv, int32_t* info_dev,
                int panel, int algo, int cutoff, int policy)
{
    int L, rc;
    if (!info_dev) return set_err(MP_E_ARG, "info_dev is NULL");
    if ((rc = lu_check(n, prec, A, lda, psa, piv, panel, algo, cutoff, policy, &L))) return rc;
    if (n == 0) return launch_fill_i32(info_dev, 1, 0, g_stream) == hipSuccess ? MP_OK : MP_E_DEVICE;
    if ((rc = device_check())) return rc;
    if ((rc = lu_run(n, L, A, lda, psa, piv, nullptr, info_dev, panel, algo, cutoff, policy, g_stream, 1))) return rc;
    return device_check();
}

int mp_lu_nopivot(int64_t n, int prec, uint32_t* A, int64_t lda, int64_t psa, int32_t* piv, int32_t* info, int panel,
                  int algo, int cutoff, int policy)
{
    int L, rc;
    if (!info) return set_err(MP_E_ARG, "info is NULL");
    *info = 0;
    if ((rc = lu_check(n, prec, A, lda, psa, piv, panel, algo, cutoff, policy, &L))) return rc;
    if (n == 0) return MP_OK;
    if ((rc = device_check())) return rc;
    if ((rc = lu_run(n, L, A, lda, psa, piv, info, nullptr, panel, algo, cutoff, policy, g_stream, 0))) return rc;
    return device_check();
}

int mp_lu(int64_t n, int prec, uint32_t* A, int64_t lda, int64_t psa, int32_t* piv, int32_t* info)
{
    return mp_lu_ex(n, prec, A, lda, psa, piv, info, 64, ALGO_WINOGRAD, 32, g_policy);
}

int mp_lu_solve(int64_t n, int prec, const uint32_t* LU, int64_t lda, int64_t psa, const int32_t* piv, uint32_t* b,
                int64_t psb)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if ((rc = check_mat("LU", LU, n, n, lda, psa)) || (rc = check_mat("b", b, n, 1, 1, psb))) return rc;
    if (n == 0) return MP_OK;
    if (!piv) return set_err(MP_E_ARG, "piv is NULL");
    if (overlaps(b, psb, LU, psa, L)) return set_err(MP_E_ALIAS, "b overlaps LU");
    if ((rc = device_check())) return rc;
    Bases bs{};
    bs.p[BASE_A] = const_cast<uint32_t*>(LU);
    bs.p[BASE_B] = b;
    const MatRef lu{BASE_A, 0, 0, lda, psa};
    const MatRef x{BASE_B, 0, 0, 1, psb};
    // the transposed factors for the one-workgroup solve (below 2048 bits)
    uint32_t* luT = nullptr;
    if (L < 64 && n <= 4096) {
        luT = workspace((size_t)n * (size_t)n * (size_t)(L + 2), g_stream, WS_SOLVE, &rc);
        if (rc) return rc;
    }
    MPG_TRY(launch_lu_solve(L, bs, lu, x, piv, n, luT, g_stream));
    return device_check();
}

}  // extern "C"
