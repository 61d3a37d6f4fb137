// tasks.hpp -- work descriptors shared by the host planner and the kernels.
//
// A matrix operand is named relative to one of a launch's base pointers
// (the caller's A, B and C, and the library workspace), so a plan built once
// for a shape can be replayed with any operands: the task arrays never hold a
// caller pointer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

enum BaseId : int32_t { BASE_A = 0, BASE_B = 1, BASE_C = 2, BASE_WS = 3, NBASES = 4 };

// base pointers of a launch: ids 0..3 inline, ids >= 4 in a device table
// (the operands of a batched launch)
struct Bases {
    uint32_t* p[NBASES];
    uint32_t* const* ext;
};

// In a kernel the id is the same for the whole wave: the inline pointers are
// chosen by selects (an indexed kernel-argument array would be read with a
// vector load), and the table, which no kernel writes, is read through the
// constant address space, so the pointer lands in scalar registers.
__host__ __device__ inline uint32_t* base_ptr(const Bases& b, int32_t id)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if (id < NBASES) {
        uint32_t* r = b.p[0];
#pragma unroll
        for (int q = 1; q < NBASES; q++) r = id == q ? b.p[q] : r;
        return r;
    }
    typedef uint32_t* const __attribute__((address_space(4))) kptr;
    return ((const kptr*)b.ext)[id - NBASES];
#else
    return id < NBASES ? b.p[id] : b.ext[id - NBASES];
#endif
}

// element (i, j), limb k of a matrix view: p[base][off + k * ps + i * ld + j];
// the exponent is "limb" L and the sign "limb" L + 1
struct MatRef {
    int32_t base;
    int32_t pad_;
    int64_t off;
    int64_t ld;
    int64_t ps;
};

// C (m x n) := A (m x l) B (l x n) in Simple order; with accum != 0 the sum
// starts from the value already in C instead of from zero
struct GemmTask {
    MatRef A, B, C;
    int32_t m, l, n, accum;
    int32_t tcl;              // tile width 2^tcl columns (the Block kernel needs 6)
    int32_t at;               // A stored transposed: element (i, k) of A is element (k, i) of the view
                              // (Simple kernels only)
    int64_t tile0;            // first tile of this task in the launch
};

// elementwise and fused per-node operations over a rows x cols index space
enum NodeOp : int32_t {
    OP_ADD = 0,               // out0 = in0 + in1
    OP_SUB = 1,               // out0 = in0 - in1
    OP_MUL = 2,               // out0 = in0 * in1
    OP_DIV = 3,               // out0 = in0 / in1
    OP_COPY = 4,              // out0 = in0
    OP_PADCOPY = 5,           // out0 = in0 inside aux0 x aux1, exact zero outside
    OP_WINO_A = 6,            // S1..S4 from A11, A12, A21, A22
    OP_WINO_B = 7,            // S5..S8 from B11, B12, B21, B22
    OP_WINO_C = 8,            // C11..C22 from M1..M7
    OP_STR_A = 9,             // the five A-side sums of Strassen
    OP_STR_B = 10,            // the five B-side sums of Strassen
    OP_STR_C = 11,            // C11..C22 from P1..P7
    OP_TRANSPOSE = 12,        // out0 (cols x rows) = in0 (rows x cols) transposed, every plane copied
    NUM_NODE_OPS = 13
};

struct NodeTask {
    MatRef in[7];
    MatRef out[5];
    int32_t rows, cols;
    int32_t aux0, aux1;
    int64_t tile0;
};

constexpr int NODE_TILE = 256;    // elements per workgroup of a node kernel

}  // namespace mpg
