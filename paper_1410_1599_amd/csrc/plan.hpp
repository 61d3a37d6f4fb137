// plan.hpp -- host planner for one MP matrix product.
//
// A plan turns (m, l, n, precision, algorithm, cutoff, odd-size policy) into
// a fixed sequence of grouped launches:
//
//   for each recursion level, top down: zero-padded operand copies, then the
//       fused operand passes (Winograd S1..S4 / S5..S8, Strassen's five A-
//       and five B-side sums) of every node of the level;
//   one grouped launch of every leaf product (Simple below the cutoff, and
//       the peeled border rows and columns, Simple over the full inner size);
//   for each level, bottom up: the fused combination pass of every node
//       (M1..M7 or P1..P7 into the four C quadrants), crops of padded results,
//       and the rank-one fix-up of a peeled inner index.
//
// The recursion itself follows Section 2: recurse while min(m, l, n) exceeds
// the cutoff; odd dimensions are peeled or padded ("a mixture of dynamic
// padding and peeling"; PEEL, PAD, or MIXED = pad d = 3 mod 4, peel d = 1
// mod 4).  Every temporary lives in one workspace; the tasks name the
// caller's matrices only by base id, so a plan is reusable for any operands
// with the same shapes and strides.
#pragma once

#include <stdint.h>

#include <vector>

#include "tasks.hpp"

namespace mpg {

enum Algo { ALGO_SIMPLE = 0, ALGO_BLOCK = 1, ALGO_STRASSEN = 2, ALGO_WINOGRAD = 3, ALGO_AUTO = 4 };
enum Policy { POLICY_PEEL = 0, POLICY_PAD = 1, POLICY_MIXED = 2 };

struct Step {
    int kind;                  // 0 = leaf products, 1 = node pass
    int op;                    // NodeOp for kind 1, LeafKind for kind 0
    int64_t task0, ntasks;     // range in the plan's gemm or node task array
    int64_t tile0, ntiles;     // range in the plan's tile map
    double units = 0;          // scalar MP multiply-adds (kind 0) or elements (kind 1)
};

struct PlanKey {
    int64_t m, l, n;
    int L, algo, cutoff, policy, leaf;
    int64_t lda, psa, ldb, psb, ldc, psc;
    int tcl = 0;          // leaf tile width 2^tcl columns (4..6; 0: 64 columns), Simple leaves only
    int persist = 0;      // 1: grids of resident workgroups that stride over the tiles
    bool operator==(const PlanKey& o) const;
};

struct PlanKeyHash {
    size_t operator()(const PlanKey& k) const;
};

struct Plan {
    PlanKey key;
    std::vector<GemmTask> gemm;
    std::vector<NodeTask> node;
    std::vector<int32_t> tiles;     // tile -> task index (into gemm or node, per step)
    std::vector<Step> steps;
    int64_t ws_words = 0;           // workspace size in uint32 words
    std::vector<int64_t> base_words;  // extent in words of every base id (for validation)
    int depth = 0;
    // operation counts of the plan (scalar MP multiplies and adds/subs)
    double n_mul = 0, n_addsub = 0;
    // device copies (made on the first launch through mp_gemm)
    bool on_device = false;
    GemmTask* d_gemm = nullptr;
    NodeTask* d_node = nullptr;
    int32_t* d_tiles = nullptr;
};

// Build the host side of a plan (no device allocation).
void build_plan(Plan& P, const PlanKey& k);

// One product of a batch: shapes and strides; its operands are base ids
// 4 + 3r (A), 5 + 3r (B), 6 + 3r (C) for item r.
struct BatchItem {
    int64_t m, l, n, lda, psa, ldb, psb, ldc, psc;
};

// All products of a batch in one plan: the passes of a recursion level of
// every item share a launch, and all leaves of all items share one.  k gives
// L, algo, cutoff, policy and leaf; its shape fields are unused.
void build_plan_batched(Plan& P, const PlanKey& k, const std::vector<BatchItem>& items);

// Check that every element any task of the plan touches lies inside its
// buffer: the caller's A, B, C spanning (L + 2) * ps words from their base
// pointers and the workspace of ws_words.  Returns false (and the first bad
// task in *why) on a violation; run on every plan before its first launch.
bool validate_plan(const Plan& P, const char** why);

}  // namespace mpg
