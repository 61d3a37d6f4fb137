/*
 * mpgemm.h -- C ABI of libmpgemm: multiple-precision (MP) binary floating-point
 * matrix multiplication and LU decomposition on one AMD Instinct MI355X
 * (gfx950) GPU.
 *
 * Method: Kouya, "Accelerated Multiple Precision Matrix Multiplication using
 * Strassen's Algorithm and Winograd's Variant" (arXiv 1410.1599): C := AB for
 * any m, l, n at a fixed binary precision with round-to-nearest after every
 * scalar operation (Sections 1 and 3), by Simple (eq. (1)), Block (eq. (2)),
 * Strassen (Section 2, P1..P7) or Winograd's variant (eqs. (winograd_mod1) to
 * (winograd_mod3)), recursing to a cutoff n_min with odd sizes peeled or
 * padded (Section 2, last paragraph); and the blocked LU of Section 4, whose
 * trailing update A22 := A22 - L21 U12 forms the product with one of these
 * algorithms (here with partial pivoting).
 *
 * ------------------------------------------------------------------ numbers
 * prec p is 128, 256, 512, 1024, 2048, 4096, 8192 or 10240 bits (Section 3
 * uses 128 to 8192, Section 4 also 8650; 10240 is the next width here above
 * it); L = p / 32.  Up to 1024 bits a GPU lane holds one value; from
 * 2048 bits a whole wavefront does (its 64 lanes each hold L / 64 limbs), with
 * the same results.  A value is
 *     (-1)^s * M * 2^(e - p),   2^(p-1) <= M < 2^p   (M normalised),
 * or zero (M = 0, e = 0, s = 0; there is one zero, +0).  Every operation
 * rounds its exact result to the nearest p-bit value, ties to the even
 * mantissa.  Precondition: |e| < 2^29 for every input (not checked).
 *
 * ------------------------------------------------------------------ matrices
 * An r x c matrix is one device buffer of uint32 words in "plane" layout:
 * element (i, j) has
 *     limb k (k = 0 least significant) at  X[k * ps + i * ld + j],  k < L,
 *     exponent e (int32 bits)          at  X[L * ps + i * ld + j],
 *     sign s (0 or 1)                  at  X[(L + 1) * ps + i * ld + j],
 * with leading dimension ld >= c and plane stride ps >= (r - 1) ld + c.  The
 * buffer spans (L + 2) * ps words.  A sub-matrix is a pointer offset with the
 * same ld and ps.  Limb-major planes make the reads of consecutive elements
 * coalesce.
 *
 * ------------------------------------------------------------------ conventions
 * Pointers are device pointers unless a parameter says "host".  The caller
 * owns every matrix and pivot array.  The library owns only its workspace (one
 * per stream, grown on demand, freed by mp_release_workspace) and cached
 * launch plans.
 *
 * Work is enqueued on the stream last set by mp_set_stream on the calling
 * thread (the null stream by default) and the call returns without waiting,
 * except where stated.  Calls that share a stream are ordered; calls on
 * different streams use different workspaces.
 *
 * Return codes: MP_OK (0) or a negative MP_E_* code.  A negative return means
 * nothing was enqueued and nothing was written; mp_last_error() then gives a
 * message (thread-local).  An asynchronous device fault of earlier work is
 * reported as MP_E_DEVICE by the next call.
 */
#ifndef MPGEMM_H
#define MPGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPGEMM_VERSION 1

enum mp_algo {
    MP_SIMPLE = 0,    /* eq. (1): c_ij = sum_k a_ik b_kj, k ascending from exact 0 */
    MP_BLOCK = 1,     /* eq. (2): LDS-staged tiles, same per-element order as Simple (bit-identical) */
    MP_STRASSEN = 2,  /* Section 2: P1..P7 and the C quadrants, recursing above the cutoff */
    MP_WINOGRAD = 3,  /* Section 2: Winograd's variant S1..S8, M1..M7, T1, T2 */
    MP_AUTO = 4       /* the autotuner's choice for the shape and precision (mp_tune), else
                         MP_WINOGRAD with cutoff 64 when min(m, l, n) > 64 and MP_SIMPLE below;
                         mp_auto_choice reports which, so the result can be reproduced */
};

enum mp_policy {      /* odd dimensions above the cutoff (Section 2, last paragraph) */
    MP_PEEL = 0,      /* peel the last row / column / inner index (default) */
    MP_PAD = 1,       /* pad with an exact zero row / column */
    MP_MIXED = 2      /* pad d = 3 mod 4, peel d = 1 mod 4 (reproduces Table 1) */
};

enum mp_leaf {        /* kernel for the products below the cutoff */
    MP_LEAF_SIMPLE = 0,
    MP_LEAF_BLOCK = 1
};

enum mp_status {
    MP_OK = 0,
    MP_E_ARG = -1,    /* bad size, stride, pointer or enum */
    MP_E_PREC = -2,   /* prec not 128 .. 8192 as above (or above 1024 where an entry says so) */
    MP_E_ALIAS = -3,  /* output buffer overlaps an input buffer */
    MP_E_NOMEM = -4,  /* device allocation failed */
    MP_E_DEVICE = -5, /* HIP error (launch failure or earlier asynchronous fault) */
    MP_E_RANGE = -6   /* a dimension above 2^31 - 1 */
};

/* Stream for later calls from this thread (a hipStream_t; NULL = null stream). */
int mp_set_stream(void *hip_stream);

/* Message of the last failed call on this thread (static storage, thread-local). */
const char *mp_last_error(void);

/* MPGEMM_VERSION of the built library. */
int mp_version(void);

/*
 * Defaults used by mp_gemm: odd-size policy (enum mp_policy) and leaf kernel
 * (enum mp_leaf).  Process-wide.  MP_E_ARG for an unknown value.
 */
int mp_set_policy(int odd_policy, int leaf);

/*
 * C := A B at precision prec (Section 2).  A is m x l, B is l x n, C is m x n,
 * each in plane layout with its own ld and plane stride.  algo: enum mp_algo.
 * cutoff: the recursion threshold n_min for MP_STRASSEN / MP_WINOGRAD (>= 1):
 * a product recurses while min(m, l, n) > cutoff, and below it is Simple;
 * ignored by MP_SIMPLE and MP_BLOCK.  Odd sizes follow mp_set_policy (PEEL by
 * default).  Zero m or n is a no-op; zero l writes C = 0.  C must not overlap
 * A or B (MP_E_ALIAS); A may alias B.  The result is bit-identical to the
 * CPU oracle performing the same sequence of correctly rounded operations.
 */
int mp_gemm(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff,
            const uint32_t *A, int64_t lda, int64_t psa,
            const uint32_t *B, int64_t ldb, int64_t psb,
            uint32_t *C, int64_t ldc, int64_t psc);

/*
 * mp_gemm without any device allocation, for callers that cannot allocate
 * (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks, policy and leaf settings, kernels and
 * result bits as mp_gemm; the caller passes A, B and C as there.  The plan's
 * task arrays and every temporary of the recursion live in one device array
 * of the library, 256 MiB per GPU, held from the library's load until the
 * process ends; a product needing more (mp_plan_info's ws_bytes plus its task
 * arrays: e.g. Winograd at cutoff 64 to n = 512 at 128 bits, n = 256 at 512
 * bits; Simple and Block at any size) returns MP_E_RANGE before anything is
 * launched.  Calls on one GPU share that array: calls that overlap in time on
 * one GPU (different streams or threads) race and must be ordered by the
 * caller; calls in one stream are ordered by it.  Nothing in the array needs
 * to start at zero.  Asynchronous on the stream of mp_set_stream.
 */
int mp_gemm_noalloc(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff,
                    const uint32_t *A, int64_t lda, int64_t psa,
                    const uint32_t *B, int64_t ldb, int64_t psb,
                    uint32_t *C, int64_t ldc, int64_t psc);

/* mp_gemm with an explicit odd-size policy (enum mp_policy) and leaf kernel (enum mp_leaf). */
int mp_gemm_ex(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff, int policy, int leaf,
               const uint32_t *A, int64_t lda, int64_t psa,
               const uint32_t *B, int64_t ldb, int64_t psb,
               uint32_t *C, int64_t ldc, int64_t psc);

/*
 * A batch of `count` products C_r := A_r B_r of one precision with one
 * algorithm and cutoff, shapes free (host arrays of count entries; the
 * matrices are device buffers in plane layout).  All products are planned
 * together: every recursion level's passes of all items share one grouped
 * launch, and every leaf product of every item shares one launch (the
 * paper's seven sub-products per level and many uneven products issued
 * together).  Each C_r is bit-identical to mp_gemm of that item alone.
 * Results must not overlap one another or any operand of any item
 * (MP_E_ALIAS, checked over all items before anything is launched); operands
 * may share memory.  Items with m or n zero are skipped.  Odd sizes and leaf
 * kernel follow mp_set_policy.
 */
int mp_gemm_batched(int count, const int64_t *m, const int64_t *l, const int64_t *n, int prec, int algo, int cutoff,
                    const uint32_t *const *A, const int64_t *lda, const int64_t *psa,
                    const uint32_t *const *B, const int64_t *ldb, const int64_t *psb,
                    uint32_t *const *C, const int64_t *ldc, const int64_t *psc);

/*
 * Elementwise C := A op B on m x n matrices, one rounding per element: the
 * matrix additions and subtractions of Strassen's and Winograd's levels
 * (Section 2), and products and true quotients for completeness.  C may alias
 * A or B exactly (same pointer and strides: in-place update).
 */
int mp_add(int64_t m, int64_t n, int prec, const uint32_t *A, int64_t lda, int64_t psa,
           const uint32_t *B, int64_t ldb, int64_t psb, uint32_t *C, int64_t ldc, int64_t psc);
int mp_sub(int64_t m, int64_t n, int prec, const uint32_t *A, int64_t lda, int64_t psa,
           const uint32_t *B, int64_t ldb, int64_t psb, uint32_t *C, int64_t ldc, int64_t psc);
int mp_mul_ew(int64_t m, int64_t n, int prec, const uint32_t *A, int64_t lda, int64_t psa,
              const uint32_t *B, int64_t ldb, int64_t psb, uint32_t *C, int64_t ldc, int64_t psc);
/* B must have no zero entry (a zero divisor gives an unspecified value). */
int mp_div_ew(int64_t m, int64_t n, int prec, const uint32_t *A, int64_t lda, int64_t psa,
              const uint32_t *B, int64_t ldb, int64_t psb, uint32_t *C, int64_t ldc, int64_t psc);

/*
 * Host-only description of the plan mp_gemm would run for (m, l, n) with
 * contiguous operands (ld = column count, ps = rows x cols): recursion depth,
 * scalar MP multiplications and additions/subtractions (the Mul and Addsub
 * counts of Section 2 / Table 1), workspace bytes and number of grouped
 * launches.  Any output pointer may be NULL.  Needs no GPU.
 */
int mp_plan_info(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff, int policy,
                 int *depth, double *n_mul, double *n_addsub, int64_t *ws_bytes, int64_t *n_launches);

/*
 * INT8-slice product C ~ A B on the matrix cores (an extension beside the
 * paper's per-operation rounding).  Each row of A is scaled by its largest
 * exponent e_i and each column of B by its own f_j; every entry becomes an
 * integer in a window of W = prec + min(spread, extra) bits (spread = the
 * largest exponent spread among the nonzero entries of a row of A, resp. a
 * column of B), truncated toward zero; those integers are cut into balanced
 * signed 8-bit digits, all digit-plane products are exact INT8 MFMA GEMMs with
 * INT32 accumulation, the exact integer sum is recombined and rounded once to
 * nearest even:  c_ij = RN(2^(e_i+f_j-W_A-W_B) sum_k trunc(a_ik) trunc(b_kj)).
 * When every spread is at most `extra` (0..64) nothing is truncated and c_ij is
 * the correctly rounded exact product (error <= 1/2 ulp).  Otherwise an entry
 * more than `extra` binades below its row's (column's) largest keeps only the
 * bits at or above 2^(e_i - W_A) (2^(f_j - W_B)): its truncation error is below
 * that power of two.  window_out (host, 2 int32, may be NULL) gets
 * W_A, W_B.  Synchronises the stream (the window depends on the data).
 * prec 128 .. 1024 only (MP_E_PREC above); inner size l <= 131008 (MP_E_RANGE
 * above: the INT32 digit sums and the 64-bit recombination are exact only
 * up to there).
 */
int mp_gemm_slice(int64_t m, int64_t l, int64_t n, int prec, int extra,
                  const uint32_t *A, int64_t lda, int64_t psa,
                  const uint32_t *B, int64_t ldb, int64_t psb,
                  uint32_t *C, int64_t ldc, int64_t psc, int32_t *window_out);

/*
 * Early stop of mp_gemm_slice (the same result, less matrix-core work).  The
 * exact sum is sum_u 256^u G_u over digit-pair diagonals u.  A first pass
 * computes the diagonals u >= u0 only and rounds every entry whose rounding the
 * omitted part, below a proven bound 2^D, cannot change (its bits between 2^D
 * and its round bit are neither all zero nor all one); a second pass computes
 * the diagonals u < u0 and rounds from all of them for the 256 x 256 output
 * tiles that hold any other entry.  u0 leaves `guard_bits` bits between 2^D
 * and the last kept bit of an entry of magnitude 2^(W_A+W_B) (the largest
 * product of two window-scaled entries): more guard bits, fewer recomputed
 * tiles on sums that cancel.  guard_bits < 0 computes every diagonal in one
 * pass.  Default 32.  Process-wide setting; MP_E_ARG above 2^20.
 */
int mp_set_slice_guard(int guard_bits);
/*
 * What the last mp_gemm_slice on this process did, in info5 (host, 5 int32):
 * u0 (0: one pass), the number of diagonals, the output tiles recomputed by the
 * second pass, the number of output tiles, and D.
 */
int mp_slice_last(int32_t *info5);

/*
 * LU decomposition with partial pivoting of the n x n matrix A in place
 * (Section 4, blocked with panel width K, trailing update A22 := A22 - L21 U12
 * with the product formed by `algo`; the paper's LU does not pivot, this one
 * pivots by rows).  On return A holds U on and above the diagonal and the
 * multipliers of the unit lower L below it.  piv (device, n int32) receives
 * LAPACK getrf-style 0-based pivots: at step k rows k and piv[k] were swapped.
 * *info (host) is 0, or k + 1 for the first column k whose pivot was exactly
 * zero (the factorisation still completes).  Pivot = the first row index of
 * the largest |a_ik|; multipliers are true quotients.  Synchronises the
 * stream to read info.
 * mp_lu uses panel 64, MP_WINOGRAD, cutoff 32 and the policy of mp_set_policy.
 */
int mp_lu(int64_t n, int prec, uint32_t *A, int64_t lda, int64_t psa, int32_t *piv, int32_t *info);
int mp_lu_ex(int64_t n, int prec, uint32_t *A, int64_t lda, int64_t psa, int32_t *piv, int32_t *info,
             int panel, int algo, int cutoff, int policy);

/*
 * mp_lu_ex without waiting: info is written to the device int32 *info_dev and
 * nothing synchronises (for request loops that overlap several factorisations
 * on different streams).
 */
int mp_lu_async(int64_t n, int prec, uint32_t *A, int64_t lda, int64_t psa, int32_t *piv, int32_t *info_dev,
                int panel, int algo, int cutoff, int policy);

/*
 * The LU of the paper as published (Section 4): the same blocked algorithm
 * without row exchanges, every pivot the diagonal entry a_cc.  piv (device, n
 * int32) receives the identity, so mp_lu_solve applies to the factors
 * unchanged.  *info (host) is 0, or c + 1 for the first column whose diagonal
 * entry became exactly zero; that column is skipped (no quotients, no update)
 * and the factorisation completes.  Arguments and errors as mp_lu_ex.
 * Synchronises the stream to read info.
 */
int mp_lu_nopivot(int64_t n, int prec, uint32_t *A, int64_t lda, int64_t psa, int32_t *piv, int32_t *info,
                  int panel, int algo, int cutoff, int policy);

/*
 * Solve A x = b from the factors of mp_lu: the row swaps of piv in order,
 * forward substitution with the unit lower factor, back substitution with the
 * upper factor (true quotients by the diagonal).  b (n x 1, plane stride psb)
 * is overwritten by x.  Asynchronous.
 */
int mp_lu_solve(int64_t n, int prec, const uint32_t *LU, int64_t lda, int64_t psa, const int32_t *piv,
                uint32_t *b, int64_t psb);

/*
 * Step profiler.  mp_profile(1) makes every later grouped launch of the
 * library record a HIP event pair on its own stream; mp_profile(0) stops.
 * mp_profile_read waits for the recorded launches, writes up to `max` records
 * (host arrays): kind (0 = leaf products, 1 = elementwise / per-node pass),
 * op (leaf kernel enum mp_leaf for kind 0, internal pass code for kind 1), L
 * (limbs), units (scalar multiply-adds for kind 0, elements for kind 1),
 * ntiles (workgroup tiles) and ms (elapsed milliseconds), clears the record
 * list and returns the number of records it held.
 */
int mp_profile(int enable);
int mp_profile_read(int max, int *kind, int *op, int *L, double *units, int64_t *ntiles, float *ms);

/*
 * Fill the rows x cols matrix X with seeded p-bit values uniform on (-1, 1):
 * x = +-W 2^-p, W a p-bit integer hashed from (seed, element index, limb),
 * normalised (so device-resident test and request operands need no host
 * copy).  Asynchronous.  prec 128 .. 1024 only (MP_E_PREC above).
 */
int mp_fill_uniform(int64_t rows, int64_t cols, int prec, uint32_t *X, int64_t ld, int64_t ps, uint64_t seed);

/*
 * Graph mode (process-wide, default off): each mp_gemm / mp_add-style call
 * captures its grouped launches into a hipGraph the first time a given plan
 * runs with given operand pointers on a given non-null stream, and replays the
 * graph afterwards (no per-launch host cost).  Calls on the null stream launch
 * directly.  Graphs are freed by mp_release_workspace.
 */
int mp_set_graph_mode(int enable);

/*
 * Launch shape of the products (process-wide; the paper leaves tuning to
 * future work, Section 5).  tile_cols_log2: a leaf tile of the Simple kernel
 * covers 2^t columns x 256 / 2^t rows (t = 4, 5 or 6; 0 is the default, 64
 * columns; Block always uses 64).  persistent = 1: every grouped launch runs
 * a grid of as many workgroups as the device keeps resident, which stride over
 * the tiles; 0: one workgroup per tile.  Neither changes any result bit (each
 * element's operation order is fixed).  MP_E_ARG for other values.
 */
int mp_set_launch(int tile_cols_log2, int persistent);

/*
 * Autotuner.  mp_tune times Simple, Block, and Strassen / Winograd with cutoffs
 * 32, 64, 128, 256 (below min(m, l, n)) and both leaf kernels on library-owned
 * scratch operands of the given shape (uniform (-1, 1) values), `reps` runs
 * each on the calling thread's stream, then the fastest with leaf tiles of 16,
 * 32 and 64 columns, each with and without persistent grids, and records the
 * fastest for (prec, ceil(log2 m), ceil(log2 l), ceil(log2 n)).  Outputs
 * (host, may be NULL): the choice and its milliseconds.  Synchronises the
 * stream.  mp_auto_choice reports what MP_AUTO would use, mp_auto_launch also
 * its launch shape (as mp_set_launch takes it).  mp_tune_save writes the
 * table as JSON; mp_tune_load reads such a file and returns the entries read
 * (negative on error).  Different algorithm choices give different (each
 * correctly rounded per operation) results; the launch shape gives none.
 */
int mp_tune(int64_t m, int64_t l, int64_t n, int prec, int reps, int *algo, int *cutoff, int *leaf, float *ms);
int mp_auto_choice(int64_t m, int64_t l, int64_t n, int prec, int *algo, int *cutoff, int *leaf);
int mp_auto_launch(int64_t m, int64_t l, int64_t n, int prec, int *algo, int *cutoff, int *leaf,
                   int *tile_cols_log2, int *persistent);
int mp_tune_save(const char *path);
int mp_tune_load(const char *path);

/* Free the workspaces, captured graphs and cached plans of the current device (synchronises the device). */
int mp_release_workspace(void);

#ifdef __cplusplus
}
#endif

#endif /* MPGEMM_H */
