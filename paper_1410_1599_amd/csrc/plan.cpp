// plan.cpp -- builds the launch sequence of one MP product (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <functional>

namespace mpg {

bool PlanKey::operator==(const PlanKey& o) const
{
    return m == o.m && l == o.l && n == o.n && L == o.L && algo == o.algo && cutoff == o.cutoff &&
           policy == o.policy && leaf == o.leaf && lda == o.lda && psa == o.psa && ldb == o.ldb &&
           psb == o.psb && ldc == o.ldc && psc == o.psc && tcl == o.tcl && persist == o.persist;
}

size_t PlanKeyHash::operator()(const PlanKey& k) const
{
    size_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) { h = (h ^ (size_t)v) * 1099511628211ull; };
    mix(k.m); mix(k.l); mix(k.n); mix(k.L); mix(k.algo); mix(k.cutoff); mix(k.policy); mix(k.leaf);
    mix(k.lda); mix(k.psa); mix(k.ldb); mix(k.psb); mix(k.ldc); mix(k.psc); mix(k.tcl); mix(k.persist);
    return h;
}

namespace {

MatRef sub(const MatRef& r, int64_t i0, int64_t j0)
{
    MatRef o = r;
    o.off += i0 * r.ld + j0;
    return o;
}

int ceil_log2(int64_t v)
{
    int c = 0;
    while ((int64_t(1) << c) < v) c++;
    return c;
}

enum Act { EVEN = 0, PEEL = 1, PAD = 2 };

Act odd_action(int64_t d, int policy)
{
    if (d % 2 == 0) return EVEN;
    if (policy == POLICY_PEEL) return PEEL;
    if (policy == POLICY_PAD) return PAD;
    return (d % 4 == 3) ? PAD : PEEL;
}

int64_t core(int64_t d, Act a) { return a == PAD ? d + 1 : (a == PEEL ? d - 1 : d); }

struct Builder {
    const PlanKey& k;
    int L;
    int64_t ws = 0;
    std::vector<std::vector<NodeTask>> pads, opsA, opsB, trans, combs, crops;
    std::vector<std::vector<GemmTask>> fixes;
    std::vector<GemmTask> leaves;
    double n_mul = 0, n_addsub = 0;
    int depth = 0;

    explicit Builder(const PlanKey& key) : k(key), L(key.L) {}

    MatRef alloc(int64_t rows, int64_t cols)
    {
        MatRef r{BASE_WS, 0, ws, cols, rows * cols};
        ws += ((int64_t)(L + 2) * rows * cols + 63) & ~int64_t(63);
        return r;
    }

    void level_lists(int d)
    {
        const size_t need = (size_t)d + 1;
        if (pads.size() < need) {
            pads.resize(need); opsA.resize(need); opsB.resize(need); trans.resize(need);
            combs.resize(need); crops.resize(need); fixes.resize(need);
        }
        depth = std::max(depth, d + 1);
    }

    static NodeTask node(int64_t rows, int64_t cols)
    {
        NodeTask t{};
        t.rows = (int32_t)rows;
        t.cols = (int32_t)cols;
        return t;
    }

    void gemm_task(std::vector<GemmTask>& v, const MatRef& A, const MatRef& B, const MatRef& C,
                   int64_t m, int64_t l, int64_t n, int accum, int at = 0)
    {
        if (m <= 0 || n <= 0) return;
        GemmTask t{};
        t.A = A; t.B = B; t.C = C;
        t.m = (int32_t)m; t.l = (int32_t)l; t.n = (int32_t)n; t.accum = accum; t.at = at;
        t.tcl = (k.leaf == 1) ? 6 : std::min(k.tcl > 0 ? k.tcl : 6, ceil_log2(n));
        v.push_back(t);
        n_mul += (double)m * l * n;
        n_addsub += (double)m * l * n;
    }

    // R(A, B) into C: recurse iff min(m, l, n) > cutoff
    void rec(const MatRef& A, const MatRef& B, const MatRef& C, int64_t m, int64_t l, int64_t n, int d)
    {
        if (m == 0 || n == 0) return;
        const bool fast = k.algo == ALGO_STRASSEN || k.algo == ALGO_WINOGRAD;
        if (!fast || std::min(m, std::min(l, n)) <= k.cutoff) {
            gemm_task(leaves, A, B, C, m, l, n, 0);
            return;
        }
        level_lists(d);
        const Act am = odd_action(m, k.policy), al = odd_action(l, k.policy), an = odd_action(n, k.policy);
        const int64_t me = core(m, am), le = core(l, al), ne = core(n, an);
        const int64_t mi = std::min(m, me), ni = std::min(n, ne);
        MatRef Ae = A, Be = B, Ce = C;
        if (am == PAD || al == PAD) {
            Ae = alloc(me, le);
            NodeTask t = node(me, le);
            t.in[0] = A; t.out[0] = Ae; t.aux0 = (int32_t)std::min(m, me); t.aux1 = (int32_t)std::min(l, le);
            pads[d].push_back(t);
        }
        if (al == PAD || an == PAD) {
            Be = alloc(le, ne);
            NodeTask t = node(le, ne);
            t.in[0] = B; t.out[0] = Be; t.aux0 = (int32_t)std::min(l, le); t.aux1 = (int32_t)std::min(n, ne);
            pads[d].push_back(t);
        }
        if (am == PAD || an == PAD) {
            Ce = alloc(me, ne);
            NodeTask t = node(mi, ni);
            t.in[0] = Ce; t.out[0] = C;
            crops[d].push_back(t);
        }
        const int64_t h = me / 2, g = le / 2, w = ne / 2;
        const MatRef A11 = Ae, A12 = sub(Ae, 0, g), A21 = sub(Ae, h, 0), A22 = sub(Ae, h, g);
        const MatRef B11 = Be, B12 = sub(Be, 0, w), B21 = sub(Be, g, 0), B22 = sub(Be, g, w);
        const MatRef C11 = Ce, C12 = sub(Ce, 0, w), C21 = sub(Ce, h, 0), C22 = sub(Ce, h, w);
        MatRef M[7];
        if (k.algo == ALGO_WINOGRAD) {
            MatRef S[8];
            for (int i = 0; i < 4; i++) S[i] = alloc(h, g);
            for (int i = 4; i < 8; i++) S[i] = alloc(g, w);
            for (int i = 0; i < 7; i++) M[i] = alloc(h, w);
            NodeTask ta = node(h, g);
            ta.in[0] = A11; ta.in[1] = A12; ta.in[2] = A21; ta.in[3] = A22;
            for (int i = 0; i < 4; i++) ta.out[i] = S[i];
            opsA[d].push_back(ta);
            NodeTask tb = node(g, w);
            tb.in[0] = B11; tb.in[1] = B12; tb.in[2] = B21; tb.in[3] = B22;
            for (int i = 0; i < 4; i++) tb.out[i] = S[4 + i];
            opsB[d].push_back(tb);
            n_addsub += 4.0 * h * g + 4.0 * g * w + 7.0 * h * w;
            // M1 = S2 S6, M2 = A11 B11, M3 = A12 B21, M4 = S3 S7, M5 = S1 S5, M6 = S4 B22, M7 = A22 S8
            rec(S[1], S[5], M[0], h, g, w, d + 1);
            rec(A11, B11, M[1], h, g, w, d + 1);
            rec(A12, B21, M[2], h, g, w, d + 1);
            rec(S[2], S[6], M[3], h, g, w, d + 1);
            rec(S[0], S[4], M[4], h, g, w, d + 1);
            rec(S[3], B22, M[5], h, g, w, d + 1);
            rec(A22, S[7], M[6], h, g, w, d + 1);
            NodeTask tc = node(h, w);
            for (int i = 0; i < 7; i++) tc.in[i] = M[i];
            tc.out[0] = C11; tc.out[1] = C12; tc.out[2] = C21; tc.out[3] = C22;
            combs[d].push_back(tc);
        } else {
            MatRef SA[5], SB[5];
            for (int i = 0; i < 5; i++) SA[i] = alloc(h, g);
            for (int i = 0; i < 5; i++) SB[i] = alloc(g, w);
            for (int i = 0; i < 7; i++) M[i] = alloc(h, w);
            NodeTask ta = node(h, g);
            ta.in[0] = A11; ta.in[1] = A12; ta.in[2] = A21; ta.in[3] = A22;
            for (int i = 0; i < 5; i++) ta.out[i] = SA[i];
            opsA[d].push_back(ta);
            NodeTask tb = node(g, w);
            tb.in[0] = B11; tb.in[1] = B12; tb.in[2] = B21; tb.in[3] = B22;
            for (int i = 0; i < 5; i++) tb.out[i] = SB[i];
            opsB[d].push_back(tb);
            n_addsub += 5.0 * h * g + 5.0 * g * w + 8.0 * h * w;
            // P1 = (A11+A22)(B11+B22), P2 = (A21+A22)B11, P3 = A11(B12-B22),
            // P4 = A22(B21-B11), P5 = (A11+A12)B22, P6 = (A21-A11)(B11+B12),
            // P7 = (A12-A22)(B21+B22)
            rec(SA[0], SB[0], M[0], h, g, w, d + 1);
            rec(SA[1], B11, M[1], h, g, w, d + 1);
            rec(A11, SB[1], M[2], h, g, w, d + 1);
            rec(A22, SB[2], M[3], h, g, w, d + 1);
            rec(SA[2], B22, M[4], h, g, w, d + 1);
            rec(SA[3], SB[3], M[5], h, g, w, d + 1);
            rec(SA[4], SB[4], M[6], h, g, w, d + 1);
            NodeTask tc = node(h, w);
            for (int i = 0; i < 7; i++) tc.in[i] = M[i];
            tc.out[0] = C11; tc.out[1] = C12; tc.out[2] = C21; tc.out[3] = C22;
            combs[d].push_back(tc);
        }
        // peeled borders: Simple over the full inner size, written into C directly.
        // The column border gives each lane a row of A to walk along k; with the
        // Simple leaf it reads a transposed copy of A[0:mi, 0:l] instead, so
        // that a wave's loads of one k are consecutive words (the same values,
        // the same order: the results do not change)
        if (an == PEEL) {
            if (k.leaf == 0 && mi > 1) {
                const MatRef At = alloc(l, mi);
                NodeTask tt = node(mi, l);
                tt.in[0] = A;
                tt.out[0] = At;
                trans[d].push_back(tt);
                gemm_task(leaves, At, sub(B, 0, n - 1), sub(C, 0, n - 1), mi, l, 1, 0, 1);
            } else {
                gemm_task(leaves, A, sub(B, 0, n - 1), sub(C, 0, n - 1), mi, l, 1, 0);
            }
        }
        if (am == PEEL) gemm_task(leaves, sub(A, m - 1, 0), B, sub(C, m - 1, 0), 1, l, n, 0);
        // peeled inner index: C[0:mi, 0:ni] += a_{i,l-1} b_{l-1,j}, after the combination
        if (al == PEEL) gemm_task(fixes[d], sub(A, 0, l - 1), sub(B, l - 1, 0), C, mi, 1, ni, 1);
    }
};

int64_t node_tiles(const NodeTask& t, int op)
{
    if (op == OP_TRANSPOSE)      // 16 x 16 blocks of the source
        return ((int64_t)(t.rows + 15) / 16) * ((t.cols + 15) / 16);
    return ((int64_t)t.rows * t.cols + NODE_TILE - 1) / NODE_TILE;
}

int64_t gemm_tiles(const GemmTask& t)
{
    const int64_t tc = int64_t(1) << t.tcl;
    const int64_t tr = (64 * 4) >> t.tcl;
    return ((t.m + tr - 1) / tr) * ((t.n + tc - 1) / tc);
}

}  // namespace

namespace {

void assemble(Plan& P, Builder& b)
{
    const PlanKey& k = P.key;
    auto add_node_step = [&](std::vector<NodeTask>& v, int op) {
        if (v.empty()) return;
        Step s{1, op, (int64_t)P.node.size(), (int64_t)v.size(), (int64_t)P.tiles.size(), 0};
        int64_t tile = 0;
        for (auto& t : v) {
            t.tile0 = tile;
            s.units += (double)t.rows * t.cols;
            const int64_t nt = node_tiles(t, op);
            const int32_t idx = (int32_t)P.node.size();
            P.node.push_back(t);
            for (int64_t q = 0; q < nt; q++) P.tiles.push_back(idx);
            tile += nt;
        }
        s.ntiles = tile;
        if (tile) P.steps.push_back(s);
    };
    auto add_gemm_step = [&](std::vector<GemmTask>& v, int kind) {
        if (v.empty()) return;
        Step s{0, kind, (int64_t)P.gemm.size(), (int64_t)v.size(), (int64_t)P.tiles.size(), 0};
        int64_t tile = 0;
        for (auto& t : v) {
            t.tile0 = tile;
            s.units += (double)t.m * t.l * t.n;
            const int64_t nt = gemm_tiles(t);
            const int32_t idx = (int32_t)P.gemm.size();
            P.gemm.push_back(t);
            for (int64_t q = 0; q < nt; q++) P.tiles.push_back(idx);
            tile += nt;
        }
        s.ntiles = tile;
        if (tile) P.steps.push_back(s);
    };
    const bool wino = k.algo == ALGO_WINOGRAD;
    for (int d = 0; d < b.depth; d++) {
        add_node_step(b.pads[d], OP_PADCOPY);
        add_node_step(b.opsA[d], wino ? OP_WINO_A : OP_STR_A);
        add_node_step(b.opsB[d], wino ? OP_WINO_B : OP_STR_B);
        add_node_step(b.trans[d], OP_TRANSPOSE);
    }
    // the leaf launch's tasks are independent; a lane's work is its task's
    // inner length, so the long ones (peeled borders, Simple over the full
    // inner size) go first and overlap with the many short leaves instead of
    // trailing them.  The leaf kernels give each of the 8 XCDs one contiguous
    // eighth of the tile list, so the tasks, longest first, are dealt round
    // robin into 8 runs laid end to end: every XCD starts on its share of the
    // long tasks (all of them at the head of one list would leave them to one
    // XCD), and a task's tiles stay together.
    std::stable_sort(b.leaves.begin(), b.leaves.end(),
                     [](const GemmTask& x, const GemmTask& y) { return x.l > y.l; });
    {
        constexpr size_t NX = 8;
        std::vector<GemmTask> dealt;
        dealt.reserve(b.leaves.size());
        for (size_t x = 0; x < NX; x++)
            for (size_t i = x; i < b.leaves.size(); i += NX) dealt.push_back(b.leaves[i]);
        b.leaves.swap(dealt);
    }
    add_gemm_step(b.leaves, k.leaf == 1 ? 1 : 0);
    for (int d = b.depth - 1; d >= 0; d--) {
        add_node_step(b.combs[d], wino ? OP_WINO_C : OP_STR_C);
        add_node_step(b.crops[d], OP_COPY);
        add_gemm_step(b.fixes[d], 0);
    }
    P.ws_words = b.ws;
    P.depth = b.depth;
    P.n_mul = b.n_mul;
    P.n_addsub = b.n_addsub;
}

}  // namespace

void build_plan(Plan& P, const PlanKey& k)
{
    P.key = k;
    Builder b(k);
    MatRef A{BASE_A, 0, 0, k.lda, k.psa};
    MatRef B{BASE_B, 0, 0, k.ldb, k.psb};
    MatRef C{BASE_C, 0, 0, k.ldc, k.psc};
    b.rec(A, B, C, k.m, k.l, k.n, 0);
    assemble(P, b);
    P.base_words = {(int64_t)(k.L + 2) * k.psa, (int64_t)(k.L + 2) * k.psb, (int64_t)(k.L + 2) * k.psc, P.ws_words};
}

void build_plan_batched(Plan& P, const PlanKey& k, const std::vector<BatchItem>& items)
{
    P.key = k;
    Builder b(k);
    P.base_words.assign(NBASES, 0);
    for (size_t r = 0; r < items.size(); r++) {
        const BatchItem& it = items[r];
        const int32_t a = NBASES + 3 * (int32_t)r;
        MatRef A{a, 0, 0, it.lda, it.psa};
        MatRef B{a + 1, 0, 0, it.ldb, it.psb};
        MatRef C{a + 2, 0, 0, it.ldc, it.psc};
        b.rec(A, B, C, it.m, it.l, it.n, 0);
        P.base_words.push_back((int64_t)(k.L + 2) * it.psa);
        P.base_words.push_back((int64_t)(k.L + 2) * it.psb);
        P.base_words.push_back((int64_t)(k.L + 2) * it.psc);
    }
    assemble(P, b);
    P.base_words[BASE_WS] = P.ws_words;
}

namespace {

// largest word index touched by a rows x cols view (all L + 2 planes), or -1
int64_t extent(const MatRef& r, int64_t rows, int64_t cols, int L)
{
    if (rows <= 0 || cols <= 0) return -1;
    return r.off + (int64_t)(L + 1) * r.ps + (rows - 1) * r.ld + (cols - 1);
}

bool view_ok(const MatRef& r, int64_t rows, int64_t cols, int L, const int64_t* size, int32_t nb)
{
    if (rows <= 0 || cols <= 0) return true;
    if (r.base < 0 || r.base >= nb || r.off < 0 || r.ld < cols || r.ps < (rows - 1) * r.ld + cols) return false;
    return extent(r, rows, cols, L) < size[r.base];
}

}  // namespace

bool validate_plan(const Plan& P, const char** why)
{
    const int L = P.key.L;
    const int64_t* size = P.base_words.data();
    const int32_t nb = (int32_t)P.base_words.size();
    for (const GemmTask& t : P.gemm) {
        const bool aok = t.at ? view_ok(t.A, t.l, t.m, L, size, nb) : view_ok(t.A, t.m, t.l, L, size, nb);
        if (!aok || !view_ok(t.B, t.l, t.n, L, size, nb) || !view_ok(t.C, t.m, t.n, L, size, nb)) {
            *why = "gemm task out of bounds";
            return false;
        }
    }
    for (const Step& s : P.steps) {
        for (int64_t q = s.task0; q < s.task0 + s.ntasks; q++) {
            if (s.kind == 0) continue;
            const NodeTask& t = P.node[(size_t)q];
            int nin = 0, nout = 0;
            int64_t irows = t.rows, icols = t.cols, orows = t.rows, ocols = t.cols;
            switch (s.op) {
            case OP_ADD: case OP_SUB: case OP_MUL: case OP_DIV: nin = 2; nout = 1; break;
            case OP_COPY: nin = 1; nout = 1; break;
            case OP_TRANSPOSE: nin = 1; nout = 1; orows = t.cols; ocols = t.rows; break;
            case OP_PADCOPY: nin = 1; nout = 1; irows = t.aux0; icols = t.aux1; break;
            case OP_WINO_A: case OP_WINO_B: nin = 4; nout = 4; break;
            case OP_STR_A: case OP_STR_B: nin = 4; nout = 5; break;
            case OP_WINO_C: case OP_STR_C: nin = 7; nout = 4; break;
            default: *why = "unknown node op"; return false;
            }
            for (int i = 0; i < nin; i++)
                if (!view_ok(t.in[i], irows, icols, L, size, nb)) { *why = "node input out of bounds"; return false; }
            for (int i = 0; i < nout; i++)
                if (!view_ok(t.out[i], orows, ocols, L, size, nb)) { *why = "node output out of bounds"; return false; }
        }
    }
    for (const Step& s : P.steps) {
        if (s.tile0 < 0 || s.tile0 + s.ntiles > (int64_t)P.tiles.size()) { *why = "tile range"; return false; }
        for (int64_t q = s.tile0; q < s.tile0 + s.ntiles; q++) {
            const int64_t ti = P.tiles[(size_t)q];
            if (ti < s.task0 || ti >= s.task0 + s.ntasks) { *why = "tile maps outside its step"; return false; }
        }
    }
    return true;
}

}  // namespace mpg
