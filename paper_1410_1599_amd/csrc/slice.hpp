// slice.hpp -- host/kernel interface of the INT8-slice product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// bits kept below p at most (the window W = p + extra, extra <= this)
constexpr int SLICE_MAX_EXTRA = 64;
// digit words per element: S = ceil((W + 2) / 8) digits at W = p + 64
constexpr int SLICE_NW4 = 7, SLICE_NW8 = 11, SLICE_NW16 = 19, SLICE_NW32 = 35;
// 32-bit positions of the recombined sum: 8 (S_A + S_B - 2) + 40 bits plus one
constexpr int SLICE_NWZ4 = 15, SLICE_NWZ8 = 23, SLICE_NWZ16 = 39, SLICE_NWZ32 = 71;
// |digit| <= 128, so a product is at most 2^14 and an INT32 sum of K of them
// is exact while K * 2^14 < 2^31
constexpr int64_t SLICE_KMAX = 131008;
constexpr int SLICE_TILE_M = 256, SLICE_TILE_N = 256, SLICE_KSTEP = 64;

struct SliceTask {
    int32_t u;       // diagonal: pairs (s, u - s)
    int32_t s0, s1;  // pairs s0 <= s < s1
    int32_t slot;    // output plane of G
    int32_t ti, tj;  // SLICE_TILE_M x SLICE_TILE_N output tile
};

// tmp: 2 * ceil(inner / 64) * outer int32 of scratch (column scan only)
hipError_t launch_slice_scan(int L, const uint32_t* X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
                             int by_cols, int32_t* emax, int32_t* emin, int32_t* tmp, hipStream_t s);
hipError_t launch_slice_digits(int L, const uint32_t* X, int64_t ld, int64_t ps, int64_t outer, int64_t inner,
                               int by_cols, const int32_t* emax, int32_t W, int32_t S, int8_t* D, int64_t dps,
                               int64_t outer_pad, int64_t kpad, hipStream_t s);
hipError_t launch_slice_gemm(const SliceTask* tasks, int64_t ntasks, const int8_t* A8, const int8_t* B8, int32_t* G,
                             int64_t a_plane, int64_t b_plane, int64_t g_plane, int32_t kpad, int32_t npad,
                             const int32_t* flags, int32_t tj_n, hipStream_t s);
hipError_t launch_slice_fill(int32_t* p, int64_t count, int32_t v, hipStream_t s);
hipError_t launch_slice_combine(int L, const int32_t* G, int64_t g_plane, int32_t npad, const int32_t* slot_begin,
                                int32_t ndiag, const int32_t* ea, const int32_t* fb, int32_t WA, int32_t WB,
                                uint32_t* C, int64_t ldc, int64_t psc, int64_t m, int64_t n, int32_t mode,
                                int32_t ulo, int32_t D, int32_t* flags, int32_t tj_n, hipStream_t s);

}  // namespace mpg
