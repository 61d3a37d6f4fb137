// launch.hpp -- host-side entry points of the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tasks.hpp"

namespace mpg {

constexpr int GEMM_TM = 4;          // rows (waves) per workgroup of a leaf product
// k-depth of one LDS stage of the Block kernel: two stages of B's 4 x 64 and
// A's 4 x 4 elements are 22 KB at 256 bits (seven workgroups fit a CU's LDS),
// 39 KB at 512, 74 KB at 1024
constexpr int block_tk(int L) { return (void)L, 4; }

// waves per SIMD the leaf kernels are compiled for (the register budget is
// 512 / waves per lane; the compiler spills the rest to scratch): one wave's
// memory and dependency waits need others to cover them.  Measured on the
// MI355X: at 1024 bits 2 instead of 1 (280 registers) took the 1024^3
// Simple product from 88.6 to 49.9 ms and Winograd from 53.3 to 31.7 ms; at
// 512 bits 4 instead of 3, 4 % less; at 256 bits 6 instead of 5, 2 % less
// (7 no better).  Same code, same bits.
constexpr int leaf_waves(int L) { return L >= 32 ? 2 : (L == 16 ? 4 : (L == 8 ? 6 : 1)); }

enum LeafKind { LEAF_SIMPLE = 0, LEAF_BLOCK = 1 };

// grouped leaf products; tile_task[t] is the index (into tasks) of tile t's task
hipError_t launch_gemm(int L, int kind, const GemmTask* tasks, const int32_t* tile_task, int64_t ntiles,
                       const Bases& bs, int64_t grid, hipStream_t s);

// grouped elementwise / per-node passes
hipError_t launch_node(int L, int op, const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles,
                       const Bases& bs, int64_t grid, hipStream_t s);

// rows x cols seeded p-bit values uniform on (-1, 1) (a hash of seed, element
// index and limb)
hipError_t launch_fill_uniform(int L, uint32_t* X, int64_t ld, int64_t ps, int64_t rows, int64_t cols, uint64_t seed,
                               hipStream_t s);

// X[0 .. count) = value (int32); used instead of a memset so captured
// sequences hold kernels only
hipError_t launch_fill_i32(int32_t* X, int64_t count, int32_t value, hipStream_t s);

// LU building blocks (lu_kernels.hip); the matrix is one MatRef on base A
// search == 0: no row exchange, the pivot is a_cc
hipError_t launch_lu_pivot_swap(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                int32_t* piv, int32_t* info, int search, hipStream_t s);
// Copies of the panel that the column steps leave for the next one (row
// exchanges, below 2048 bits): after the step of column c - 1, keys_in[pos] is
// the 64-bit key (exponent, top limb; 0 for zero) of a_pos,c and the panel
// columns [c, je) of row pos are also in cand_in (plane q at cand + q cps +
// pos cld + (j - j0), cld >= the panel width), for pos in [c, n); for the
// rows [c + 4 g, c + 4 g + 4) (a column step's workgroup) cmax_in[2 g] is
// their largest key and cmax_in[2 g + 1] the first of them holding it, plus
// 2^63 when another does.  The step of column c reads the _in set and writes
// the _out set; the caller alternates two sets (n keys, nch = ceil(n / 4)
// two-word records and (L + 2) cld n words each).
struct PanelCopy {
    const unsigned long long* keys_in;
    const uint32_t* cand_in;
    const unsigned long long* cmax_in;
    unsigned long long* keys_out;
    uint32_t* cand_out;
    unsigned long long* cmax_out;
    int64_t cps, cld, nch;
};
// The step of column c of the panel [j0, je): multipliers of the rows below c
// and the panel's rank-one update.  next: 0 plain; 1 also write the _out copy
// for column c + 1 < je; 2 also check a_c+1,c+1 for the unpivoted LU.
// fused (c > j0, next != 2): the pivot search of column c and the exchange of
// rows c and r inside the panel happen in the same launch, from the _in copy
// (otherwise launch_lu_pivot_swap has done them).  Precisions of 2048 bits
// and more take next = 0 and fused = 0 only.
hipError_t launch_lu_eliminate(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                               int32_t* piv, int32_t* info, const PanelCopy& pc, int next, int fused, hipStream_t s);
// the pivot step of a column c > j0 from the _in copy, and the exchange of
// rows c and r inside the panel, as a launch of its own (then
// launch_lu_eliminate with fused = 0)
hipError_t launch_lu_pivot_copy(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                int32_t* piv, int32_t* info, const PanelCopy& pc, hipStream_t s);
hipError_t launch_lu_u12(int L, const Bases& bs, MatRef a, int64_t j0, int64_t kb, int64_t je, int64_t n,
                         hipStream_t s);
// piv[k0 .. k1) applied in order to the columns [c0, c1) and [c2, c3)
hipError_t launch_lu_laswp(int L, const Bases& bs, MatRef a, const int32_t* piv, int64_t k0, int64_t k1,
                           int64_t c0, int64_t c1, int64_t c2, int64_t c3, hipStream_t s);
// luT: workspace of n * n * (L + 2) words for the transposed factors (the
// one-workgroup solves below 2048 bits, n <= 4096); unused otherwise
hipError_t launch_lu_solve(int L, const Bases& bs, MatRef lu, MatRef x, const int32_t* piv, int64_t n, uint32_t* luT,
                           hipStream_t s);

// the same operations for p = 2048, 4096, 8192, 10240 bits (L = 64, 128, 256,
// 320), one value per wavefront (wide_kernels.hip); the launchers above
// forward to them
hipError_t launch_gemm_wide(int L, const GemmTask* tasks, const int32_t* tile_task, int64_t ntiles, const Bases& bs,
                            int64_t grid, hipStream_t s);
hipError_t launch_node_wide(int L, int op, const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles,
                            const Bases& bs, int64_t grid, hipStream_t s);
hipError_t launch_lu_pivot_swap_wide(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t j0, int64_t je,
                                     int32_t* piv, int32_t* info, int search, hipStream_t s);
hipError_t launch_lu_eliminate_wide(int L, const Bases& bs, MatRef a, int64_t n, int64_t c, int64_t je,
                                    hipStream_t s);
hipError_t launch_lu_u12_wide(int L, const Bases& bs, MatRef a, int64_t j0, int64_t kb, int64_t je, int64_t n,
                              hipStream_t s);
hipError_t launch_lu_solve_wide(int L, const Bases& bs, MatRef lu, MatRef x, const int32_t* piv, int64_t n,
                                hipStream_t s);

}  // namespace mpg
