// node_ops.hpp -- the elementwise and per-node operations of a recursion
// level (Section 2): Strassen's operand sums and combination, Winograd's S,
// T and C formulas, padding copies, and the plain elementwise operations.
// One body serves both number layouts: MP<L> (one value per lane) and WMP<L>
// (one value per wavefront).
#pragma once

#include "mp_arith.hpp"
#include "tasks.hpp"
#include "wide.hpp"

namespace mpg {

template <class Num>
struct NumIO;

template <int L>
struct NumIO<MP<L>> {
    static __device__ __forceinline__ MP<L> ld(const Bases& bs, const MatRef& r, int64_t i, int64_t j)
    {
        return load<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j);
    }
    static __device__ __forceinline__ void st(const Bases& bs, const MatRef& r, int64_t i, int64_t j, const MP<L>& v)
    {
        store<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j, v);
    }
    static __device__ __forceinline__ MP<L> zero() { return mp_zero<L>(); }
};

template <int L>
struct NumIO<WMP<L>> {
    static __device__ __forceinline__ WMP<L> ld(const Bases& bs, const MatRef& r, int64_t i, int64_t j)
    {
        return wload<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j);
    }
    static __device__ __forceinline__ void st(const Bases& bs, const MatRef& r, int64_t i, int64_t j, const WMP<L>& v)
    {
        wstore<L>(base_ptr(bs, r.base) + r.off, r.ps, i * r.ld + j, v);
    }
    static __device__ __forceinline__ WMP<L> zero() { return wzero<L>(); }
};

// element (i, j) of node task T
template <class Num, int L, int OP>
__device__ __forceinline__ void node_apply(const Bases& bs, const NodeTask& T, int64_t i, int64_t j)
{
    using IO = NumIO<Num>;
    if constexpr (OP == OP_ADD) {
        IO::st(bs, T.out[0], i, j, add_rn<L>(IO::ld(bs, T.in[0], i, j), IO::ld(bs, T.in[1], i, j)));
    } else if constexpr (OP == OP_SUB) {
        IO::st(bs, T.out[0], i, j, sub_rn<L>(IO::ld(bs, T.in[0], i, j), IO::ld(bs, T.in[1], i, j)));
    } else if constexpr (OP == OP_MUL) {
        IO::st(bs, T.out[0], i, j, mul_rn<L>(IO::ld(bs, T.in[0], i, j), IO::ld(bs, T.in[1], i, j)));
    } else if constexpr (OP == OP_DIV) {
        IO::st(bs, T.out[0], i, j, div_rn<L>(IO::ld(bs, T.in[0], i, j), IO::ld(bs, T.in[1], i, j)));
    } else if constexpr (OP == OP_COPY) {
        IO::st(bs, T.out[0], i, j, IO::ld(bs, T.in[0], i, j));
    } else if constexpr (OP == OP_PADCOPY) {
        const bool in = i < T.aux0 && j < T.aux1;
        IO::st(bs, T.out[0], i, j, in ? IO::ld(bs, T.in[0], i, j) : IO::zero());
    } else if constexpr (OP == OP_WINO_A) {
        // S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2
        const Num a11 = IO::ld(bs, T.in[0], i, j), a12 = IO::ld(bs, T.in[1], i, j);
        const Num a21 = IO::ld(bs, T.in[2], i, j), a22 = IO::ld(bs, T.in[3], i, j);
        const Num s1 = add_rn<L>(a21, a22);
        const Num s2 = sub_rn<L>(s1, a11);
        IO::st(bs, T.out[0], i, j, s1);
        IO::st(bs, T.out[1], i, j, s2);
        IO::st(bs, T.out[2], i, j, sub_rn<L>(a11, a21));
        IO::st(bs, T.out[3], i, j, sub_rn<L>(a12, s2));
    } else if constexpr (OP == OP_WINO_B) {
        // S5 = B12 - B11, S6 = B22 - S5, S7 = B22 - B12, S8 = S6 - B21
        const Num b11 = IO::ld(bs, T.in[0], i, j), b12 = IO::ld(bs, T.in[1], i, j);
        const Num b21 = IO::ld(bs, T.in[2], i, j), b22 = IO::ld(bs, T.in[3], i, j);
        const Num s5 = sub_rn<L>(b12, b11);
        const Num s6 = sub_rn<L>(b22, s5);
        IO::st(bs, T.out[0], i, j, s5);
        IO::st(bs, T.out[1], i, j, s6);
        IO::st(bs, T.out[2], i, j, sub_rn<L>(b22, b12));
        IO::st(bs, T.out[3], i, j, sub_rn<L>(s6, b21));
    } else if constexpr (OP == OP_WINO_C) {
        // T1 = M1 + M2, T2 = T1 + M4; C11 = M2 + M3, C12 = (T1 + M5) + M6,
        // C21 = T2 - M7, C22 = T2 + M5
        const Num m1 = IO::ld(bs, T.in[0], i, j), m2 = IO::ld(bs, T.in[1], i, j);
        const Num m3 = IO::ld(bs, T.in[2], i, j), m4 = IO::ld(bs, T.in[3], i, j);
        const Num m5 = IO::ld(bs, T.in[4], i, j), m6 = IO::ld(bs, T.in[5], i, j);
        const Num m7 = IO::ld(bs, T.in[6], i, j);
        const Num t1 = add_rn<L>(m1, m2);
        const Num t2 = add_rn<L>(t1, m4);
        IO::st(bs, T.out[0], i, j, add_rn<L>(m2, m3));
        IO::st(bs, T.out[1], i, j, add_rn<L>(add_rn<L>(t1, m5), m6));
        IO::st(bs, T.out[2], i, j, sub_rn<L>(t2, m7));
        IO::st(bs, T.out[3], i, j, add_rn<L>(t2, m5));
    } else if constexpr (OP == OP_STR_A) {
        // A11 + A22, A21 + A22, A11 + A12, A21 - A11, A12 - A22
        const Num a11 = IO::ld(bs, T.in[0], i, j), a12 = IO::ld(bs, T.in[1], i, j);
        const Num a21 = IO::ld(bs, T.in[2], i, j), a22 = IO::ld(bs, T.in[3], i, j);
        IO::st(bs, T.out[0], i, j, add_rn<L>(a11, a22));
        IO::st(bs, T.out[1], i, j, add_rn<L>(a21, a22));
        IO::st(bs, T.out[2], i, j, add_rn<L>(a11, a12));
        IO::st(bs, T.out[3], i, j, sub_rn<L>(a21, a11));
        IO::st(bs, T.out[4], i, j, sub_rn<L>(a12, a22));
    } else if constexpr (OP == OP_STR_B) {
        // B11 + B22, B12 - B22, B21 - B11, B11 + B12, B21 + B22
        const Num b11 = IO::ld(bs, T.in[0], i, j), b12 = IO::ld(bs, T.in[1], i, j);
        const Num b21 = IO::ld(bs, T.in[2], i, j), b22 = IO::ld(bs, T.in[3], i, j);
        IO::st(bs, T.out[0], i, j, add_rn<L>(b11, b22));
        IO::st(bs, T.out[1], i, j, sub_rn<L>(b12, b22));
        IO::st(bs, T.out[2], i, j, sub_rn<L>(b21, b11));
        IO::st(bs, T.out[3], i, j, add_rn<L>(b11, b12));
        IO::st(bs, T.out[4], i, j, add_rn<L>(b21, b22));
    } else if constexpr (OP == OP_STR_C) {
        // C11 = ((P1 + P4) - P5) + P7, C12 = P3 + P5, C21 = P2 + P4,
        // C22 = ((P1 + P3) - P2) + P6
        const Num p1 = IO::ld(bs, T.in[0], i, j), p2 = IO::ld(bs, T.in[1], i, j);
        const Num p3 = IO::ld(bs, T.in[2], i, j), p4 = IO::ld(bs, T.in[3], i, j);
        const Num p5 = IO::ld(bs, T.in[4], i, j), p6 = IO::ld(bs, T.in[5], i, j);
        const Num p7 = IO::ld(bs, T.in[6], i, j);
        IO::st(bs, T.out[0], i, j, add_rn<L>(sub_rn<L>(add_rn<L>(p1, p4), p5), p7));
        IO::st(bs, T.out[1], i, j, add_rn<L>(p3, p5));
        IO::st(bs, T.out[2], i, j, add_rn<L>(p2, p4));
        IO::st(bs, T.out[3], i, j, add_rn<L>(sub_rn<L>(add_rn<L>(p1, p3), p2), p6));
    }
}

}  // namespace mpg
