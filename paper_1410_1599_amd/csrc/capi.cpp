// capi.cpp -- the C ABI of libmpgemm (declared in include/mpgemm.h).
//
// Argument checking happens before anything is enqueued: a negative return
// means nothing was launched and nothing was written.  Work is enqueued on the
// calling thread's stream (mp_set_stream) and the calls return without
// waiting, except mp_lu / mp_lu_ex, which return the LAPACK-style info.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "launch.hpp"
#include "mpgemm_internal.hpp"
#include "plan.hpp"

namespace mpg {

thread_local hipStream_t g_stream = nullptr;
thread_local std::string g_err;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct GraphKey {
    const Plan* plan;
    uint32_t* p[NBASES];
    hipStream_t s;
    bool operator<(const GraphKey& o) const
    {
        if (plan != o.plan) return plan < o.plan;
        for (int i = 0; i < NBASES; i++)
            if (p[i] != o.p[i]) return p[i] < o.p[i];
        return s < o.s;
    }
};

struct TuneEntry {
    int algo, cutoff, leaf;
    float ms;
    int tcl = 0, persist = 0;       // leaf tile width (log2 columns, 0: 64) and persistent grids
};

struct DeviceState {
    std::mutex mu;
    std::unordered_map<PlanKey, std::unique_ptr<Plan>, PlanKeyHash> plans;
    std::map<std::pair<hipStream_t, int>, DevBuf> ws;     // per stream and slot
    std::map<GraphKey, hipGraphExec_t> graphs;            // captured plans (graph mode)
};

std::mutex g_tune_mu;
std::map<std::array<int64_t, 4>, TuneEntry> g_tune;      // (prec, m, l, n bucket) -> choice
int g_graph_mode = 0;

std::mutex g_dev_mu;
std::map<int, std::unique_ptr<DeviceState>> g_dev;

DeviceState& dev_state()
{
    int d = 0;
    (void)hipGetDevice(&d);
    std::lock_guard<std::mutex> g(g_dev_mu);
    auto& p = g_dev[d];
    if (!p) p.reset(new DeviceState());
    return *p;
}

void free_plan_device(Plan& P)
{
    if (P.d_gemm) (void)hipFree(P.d_gemm);
    if (P.d_node) (void)hipFree(P.d_node);
    if (P.d_tiles) (void)hipFree(P.d_tiles);
    P.d_gemm = nullptr;
    P.d_node = nullptr;
    P.d_tiles = nullptr;
    P.on_device = false;
}

template <class T>
int upload(T** dst, const std::vector<T>& v)
{
    if (v.empty()) return MP_OK;
    if (hipMalloc((void**)dst, sizeof(T) * v.size()) != hipSuccess) return set_err(MP_E_NOMEM, "hipMalloc of a plan failed");
    if (hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return set_err(MP_E_DEVICE, "upload of a plan failed");
    return MP_OK;
}

}  // namespace

int set_err(int code, const char* msg)
{
    g_err = msg;
    return code;
}

int check_prec(int prec, int* L)
{
    if (prec != 128 && prec != 256 && prec != 512 && prec != 1024 && prec != 2048 && prec != 4096 && prec != 8192 &&
        prec != 10240)
        return set_err(MP_E_PREC, "prec must be 128, 256, 512, 1024, 2048, 4096, 8192 or 10240");
    *L = prec / 32;
    return MP_OK;
}

int check_mat(const char* name, const uint32_t* p, int64_t rows, int64_t cols, int64_t ld, int64_t ps)
{
    if (rows < 0 || cols < 0) return set_err(MP_E_ARG, "negative dimension");
    if (rows > INT32_MAX || cols > INT32_MAX) return set_err(MP_E_RANGE, "dimension above 2^31 - 1");
    if (rows == 0 || cols == 0) return MP_OK;
    if (!p) {
        g_err = std::string(name) + " is NULL";
        return MP_E_ARG;
    }
    if (ld < cols) {
        g_err = std::string(name) + ": leading dimension smaller than the column count";
        return MP_E_ARG;
    }
    if (ps < (rows - 1) * ld + cols) {
        g_err = std::string(name) + ": plane stride smaller than the matrix";
        return MP_E_ARG;
    }
    return MP_OK;
}

bool overlaps(const uint32_t* a, int64_t psa, const uint32_t* b, int64_t psb, int L)
{
    const uintptr_t a0 = (uintptr_t)a, a1 = a0 + 4ull * (uint64_t)(L + 2) * (uint64_t)psa;
    const uintptr_t b0 = (uintptr_t)b, b1 = b0 + 4ull * (uint64_t)(L + 2) * (uint64_t)psb;
    return a0 < b1 && b0 < a1;
}

int device_check()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_err = std::string("device error: ") + hipGetErrorString(e);
        return MP_E_DEVICE;
    }
    return MP_OK;
}

Plan* get_plan(const PlanKey& key, int* rc, bool device)
{
    DeviceState& S = dev_state();
    std::lock_guard<std::mutex> g(S.mu);
    Plan* raw;
    auto it = S.plans.find(key);
    if (it != S.plans.end()) {
        raw = it->second.get();
    } else {
        std::unique_ptr<Plan> P(new Plan());
        build_plan(*P, key);
        const char* why = nullptr;
        if (!validate_plan(*P, &why)) {
            *rc = set_err(MP_E_ARG, why);      // a planner defect: refuse rather than launch
            return nullptr;
        }
        raw = P.get();
        S.plans[key] = std::move(P);
    }
    // device copies of the task arrays, made on the plan's first launch
    // through the library's own buffers (mp_gemm_noalloc copies them into its
    // scratch array on every call instead)
    if (device && !raw->on_device) {
        if ((*rc = upload(&raw->d_gemm, raw->gemm)) || (*rc = upload(&raw->d_node, raw->node)) ||
            (*rc = upload(&raw->d_tiles, raw->tiles))) {
            free_plan_device(*raw);
            return nullptr;
        }
        raw->on_device = true;
    }
    return raw;
}

uint32_t* workspace(size_t words, hipStream_t s, int slot, int* rc)
{
    *rc = MP_OK;
    if (words == 0) return nullptr;
    DeviceState& S = dev_state();
    std::lock_guard<std::mutex> g(S.mu);
    DevBuf& b = S.ws[std::make_pair(s, slot)];
    const size_t bytes = words * 4;
    if (b.bytes < bytes) {
        if (b.p) {
            (void)hipStreamSynchronize(s);    // earlier work on this stream may still use it
            (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
        }
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *rc = set_err(MP_E_NOMEM, "workspace allocation failed");
            return nullptr;
        }
        b.bytes = bytes;
    }
    return (uint32_t*)b.p;
}

int64_t grid_for(int64_t ntiles)
{
    return ntiles < (int64_t(1) << 30) ? ntiles : (int64_t(1) << 30);
}

// ---- step profiler: HIP events around every grouped launch, on its stream
struct ProfRec {
    int kind, op, L;
    double units;
    int64_t ntiles;
    hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
thread_local bool g_capturing = false;
std::vector<ProfRec> g_prof;

ProfScope::ProfScope(hipStream_t s, int kind, int op, int L, double units, int64_t ntiles)
    : s_(s), kind_(kind), op_(op), L_(L), units_(units), ntiles_(ntiles), on_(g_prof_on && !g_capturing)
{
    if (on_) {
        (void)hipEventCreate(&e0_);
        (void)hipEventCreate(&e1_);
        (void)hipEventRecord(e0_, s_);
    }
}

ProfScope::~ProfScope()
{
    if (!on_) return;
    (void)hipEventRecord(e1_, s_);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back(ProfRec{kind_, op_, L_, units_, ntiles_, e0_, e1_});
}

int launch_steps(const Plan& P, const Bases& bs, hipStream_t s);

// Graph mode: the first call of a plan with given operand pointers and stream
// captures its launches into a hipGraph; later calls replay it.  The null
// stream cannot be captured: calls on it launch directly.
int run_plan(const Plan& P, Bases bs, hipStream_t s)
{
    int rc = MP_OK;
    bs.p[BASE_WS] = workspace((size_t)P.ws_words, s, WS_PLAN, &rc);
    if (rc) return rc;
    if (!g_graph_mode || s == nullptr) return launch_steps(P, bs, s);
    DeviceState& S = dev_state();
    GraphKey key{&P, {bs.p[0], bs.p[1], bs.p[2], bs.p[3]}, s};
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> g(S.mu);
        auto it = S.graphs.find(key);
        if (it != S.graphs.end()) exec = it->second;
    }
    if (!exec) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return set_err(MP_E_DEVICE, "stream capture failed to start");
        g_capturing = true;                    // no event records inside a capture
        rc = launch_steps(P, bs, s);
        g_capturing = false;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        if (rc) return rc;
        if (e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return set_err(MP_E_DEVICE, "graph capture failed");
        }
        (void)hipGraphDestroy(graph);
        std::lock_guard<std::mutex> g(S.mu);
        S.graphs[key] = exec;
    }
    ProfScope ps(s, 4, 0, P.key.L, P.n_mul, 0);
    if (hipGraphLaunch(exec, s) != hipSuccess) return set_err(MP_E_DEVICE, "graph launch failed");
    return MP_OK;
}

int launch_steps(const Plan& P, const Bases& bs, hipStream_t s)
{
    return launch_plan_steps(P, P.d_gemm, P.d_node, P.d_tiles, bs, s);
}

int launch_plan_steps(const Plan& P, const GemmTask* d_gemm, const NodeTask* d_node, const int32_t* d_tiles,
                      const Bases& bs, hipStream_t s)
{
    // the tile map holds indices into the plan's whole task arrays
    for (const Step& st : P.steps) {
        hipError_t e;
        ProfRec pr{};
        const bool prof = g_prof_on && !g_capturing;
        if (prof) {
            pr = ProfRec{st.kind, st.op, P.key.L, st.units, st.ntiles, nullptr, nullptr};
            (void)hipEventCreate(&pr.e0);
            (void)hipEventCreate(&pr.e1);
            (void)hipEventRecord(pr.e0, s);
        }
        // persistent plans launch grids of resident workgroups (grid 0: sized by the launcher)
        const int64_t grid = P.key.persist ? 0 : grid_for(st.ntiles);
        if (st.kind == 0)
            e = launch_gemm(P.key.L, st.op, d_gemm, d_tiles + st.tile0, st.ntiles, bs, grid, s);
        else
            e = launch_node(P.key.L, st.op, d_node, d_tiles + st.tile0, st.ntiles, bs, grid, s);
        if (prof) {
            (void)hipEventRecord(pr.e1, s);
            std::lock_guard<std::mutex> g(g_prof_mu);
            g_prof.push_back(pr);
        }
        if (e != hipSuccess) {
            g_err = std::string("launch failed: ") + hipGetErrorString(e);
            return MP_E_DEVICE;
        }
    }
    return MP_OK;
}

int gemm_internal(int64_t m, int64_t l, int64_t n, int L, int algo, int cutoff, int policy, int leaf,
                  const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb,
                  uint32_t* C, int64_t ldc, int64_t psc, hipStream_t s, int tcl, int persist)
{
    if (m == 0 || n == 0) return MP_OK;
    PlanKey key{m, l, n, L, algo, cutoff, policy, algo == ALGO_BLOCK ? 1 : leaf, lda, psa, ldb, psb, ldc, psc};
    key.tcl = tcl >= 0 ? tcl : g_tcl;
    key.persist = persist >= 0 ? persist : g_persist;
    if (algo == ALGO_BLOCK) key.tcl = 0;
    if (algo == ALGO_SIMPLE || algo == ALGO_BLOCK) key.cutoff = 0, key.policy = 0;
    int rc = MP_OK;
    Plan* P = get_plan(key, &rc, true);
    if (!P) return rc ? rc : MP_E_NOMEM;
    Bases bs{};
    bs.p[BASE_A] = const_cast<uint32_t*>(A);
    bs.p[BASE_B] = const_cast<uint32_t*>(B);
    bs.p[BASE_C] = C;
    return run_plan(*P, bs, s);
}

int ew_internal(int op, int64_t m, int64_t n, int L, const uint32_t* A, int64_t lda, int64_t psa,
                const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc, hipStream_t s)
{
    if (m == 0 || n == 0) return MP_OK;
    int rc;
    // a one-task plan, cached like a product plan (algo field = 100 + op)
    PlanKey key{m, 0, n, L, 100 + op, 0, 0, 0, lda, psa, ldb, psb, ldc, psc};
    DeviceState& S = dev_state();
    Plan* P = nullptr;
    {
        std::lock_guard<std::mutex> g(S.mu);
        auto it = S.plans.find(key);
        if (it != S.plans.end()) P = it->second.get();
    }
    if (!P) {
        std::unique_ptr<Plan> np(new Plan());
        np->key = key;
        NodeTask t{};
        t.in[0] = MatRef{BASE_A, 0, 0, lda, psa};
        t.in[1] = MatRef{BASE_B, 0, 0, ldb, psb};
        t.out[0] = MatRef{BASE_C, 0, 0, ldc, psc};
        t.rows = (int32_t)m;
        t.cols = (int32_t)n;
        t.tile0 = 0;
        np->node.push_back(t);
        const int64_t nt = (m * n + NODE_TILE - 1) / NODE_TILE;
        np->tiles.assign((size_t)nt, 0);
        np->steps.push_back(Step{1, op, 0, 1, 0, nt});
        if ((rc = upload(&np->d_node, np->node)) || (rc = upload(&np->d_tiles, np->tiles))) {
            free_plan_device(*np);
            return rc;
        }
        std::lock_guard<std::mutex> g(S.mu);
        P = np.get();
        S.plans[key] = std::move(np);
    }
    Bases bs{};
    bs.p[BASE_A] = const_cast<uint32_t*>(A);
    bs.p[BASE_B] = const_cast<uint32_t*>(B);
    bs.p[BASE_C] = C;
    return run_plan(*P, bs, s);
}

// ---- autotuner: times candidate (algorithm, cutoff, leaf kernel) choices
// for a shape and precision on library-owned scratch operands and remembers
// the fastest per (prec, power-of-two bucket of m, l, n)
std::array<int64_t, 4> tune_key(int64_t m, int64_t l, int64_t n, int prec)
{
    auto b = [](int64_t v) { int64_t c = 0; while ((int64_t(1) << c) < v) c++; return c; };
    return {prec, b(m), b(l), b(n)};
}

bool tune_lookup(int64_t m, int64_t l, int64_t n, int prec, TuneEntry* out)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key(m, l, n, prec));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

extern int g_tcl, g_persist;

// default when nothing was tuned: Winograd down to 64 (Simple below)
TuneEntry tune_default(int64_t m, int64_t l, int64_t n)
{
    if (std::min(m, std::min(l, n)) > 64) return TuneEntry{ALGO_WINOGRAD, 64, LEAF_SIMPLE, 0.f, g_tcl, g_persist};
    return TuneEntry{ALGO_SIMPLE, 0, LEAF_SIMPLE, 0.f, g_tcl, g_persist};
}

int g_leaf = LEAF_SIMPLE;
int g_policy = POLICY_PEEL;
int g_tcl = 0;
int g_persist = 0;

}  // namespace mpg

using namespace mpg;

extern "C" {

int mp_set_stream(void* stream)
{
    g_stream = (hipStream_t)stream;
    return MP_OK;
}

const char* mp_last_error(void)
{
    return g_err.c_str();
}

int mp_version(void)
{
    return MPGEMM_VERSION;
}

int mp_set_policy(int odd_policy, int leaf)
{
    if (odd_policy < POLICY_PEEL || odd_policy > POLICY_MIXED) return set_err(MP_E_ARG, "unknown odd-size policy");
    if (leaf != LEAF_SIMPLE && leaf != LEAF_BLOCK) return set_err(MP_E_ARG, "unknown leaf kernel");
    g_policy = odd_policy;
    g_leaf = leaf;
    return MP_OK;
}

}  // extern "C"

namespace mpg {

int gemm_validate(int64_t m, int64_t l, int64_t n, int prec, int* algo_io, int* cutoff_io, int policy, int* leaf_io,
                  const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb,
                  const uint32_t* C, int64_t ldc, int64_t psc, int* L_out, int* tcl_out, int* persist_out)
{
    int L, rc;
    int algo = *algo_io, cutoff = *cutoff_io, leaf = *leaf_io;
    int tcl = g_tcl, persist = g_persist;
    if ((rc = check_prec(prec, &L))) return rc;
    if (algo < ALGO_SIMPLE || algo > ALGO_AUTO) return set_err(MP_E_ARG, "unknown algorithm");
    if ((algo == ALGO_STRASSEN || algo == ALGO_WINOGRAD) && cutoff < 1) return set_err(MP_E_ARG, "cutoff must be >= 1");
    if (policy < POLICY_PEEL || policy > POLICY_MIXED) return set_err(MP_E_ARG, "unknown odd-size policy");
    if (leaf != LEAF_SIMPLE && leaf != LEAF_BLOCK) return set_err(MP_E_ARG, "unknown leaf kernel");
    if (m < 0 || l < 0 || n < 0) return set_err(MP_E_ARG, "negative dimension");
    if (algo == ALGO_AUTO) {
        TuneEntry t;
        if (!tune_lookup(m, l, n, prec, &t)) t = tune_default(m, l, n);
        algo = t.algo;
        cutoff = t.cutoff;
        leaf = t.leaf;
        tcl = t.tcl;
        persist = t.persist;
    }
    if ((rc = check_mat("A", A, m, l, lda, psa)) || (rc = check_mat("B", B, l, n, ldb, psb)) ||
        (rc = check_mat("C", C, m, n, ldc, psc)))
        return rc;
    if (m > 0 && n > 0 && l > 0 && (overlaps(C, psc, A, psa, L) || overlaps(C, psc, B, psb, L)))
        return set_err(MP_E_ALIAS, "C overlaps A or B");
    *algo_io = algo;
    *cutoff_io = cutoff;
    *leaf_io = leaf;
    *L_out = L;
    if (tcl_out) *tcl_out = tcl;
    if (persist_out) *persist_out = persist;
    return MP_OK;
}

}  // namespace mpg

extern "C" {

int mp_gemm_ex(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff, int policy, int leaf,
               const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb,
               uint32_t* C, int64_t ldc, int64_t psc)
{
    int L, rc, tcl, persist;
    if ((rc = gemm_validate(m, l, n, prec, &algo, &cutoff, policy, &leaf, A, lda, psa, B, ldb, psb, C, ldc, psc, &L,
                            &tcl, &persist)))
        return rc;
    if (m == 0 || n == 0) return MP_OK;
    if ((rc = device_check())) return rc;
    rc = gemm_internal(m, l, n, L, algo, cutoff, policy, leaf, A, lda, psa, B, ldb, psb, C, ldc, psc, g_stream, tcl,
                       persist);
    if (rc) return rc;
    return device_check();
}

int mp_gemm(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff, const uint32_t* A, int64_t lda,
            int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc)
{
    return mp_gemm_ex(m, l, n, prec, algo, cutoff, g_policy, g_leaf, A, lda, psa, B, ldb, psb, C, ldc, psc);
}

static int elementwise(int op, int64_t m, int64_t n, int prec, const uint32_t* A, int64_t lda, int64_t psa,
                       const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if ((rc = check_mat("A", A, m, n, lda, psa)) || (rc = check_mat("B", B, m, n, ldb, psb)) ||
        (rc = check_mat("C", C, m, n, ldc, psc)))
        return rc;
    if (m == 0 || n == 0) return MP_OK;
    if ((rc = device_check())) return rc;
    if ((rc = ew_internal(op, m, n, L, A, lda, psa, B, ldb, psb, C, ldc, psc, g_stream))) return rc;
    return device_check();
}

int mp_add(int64_t m, int64_t n, int prec, const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B,
           int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc)
{
    return elementwise(OP_ADD, m, n, prec, A, lda, psa, B, ldb, psb, C, ldc, psc);
}

int mp_sub(int64_t m, int64_t n, int prec, const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B,
           int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc)
{
    return elementwise(OP_SUB, m, n, prec, A, lda, psa, B, ldb, psb, C, ldc, psc);
}

int mp_mul_ew(int64_t m, int64_t n, int prec, const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B,
              int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc)
{
    return elementwise(OP_MUL, m, n, prec, A, lda, psa, B, ldb, psb, C, ldc, psc);
}

int mp_div_ew(int64_t m, int64_t n, int prec, const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B,
              int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc)
{
    return elementwise(OP_DIV, m, n, prec, A, lda, psa, B, ldb, psb, C, ldc, psc);
}

int mp_plan_info(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff, int policy, int* depth,
                 double* n_mul, double* n_addsub, int64_t* ws_bytes, int64_t* n_launches)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if (algo < ALGO_SIMPLE || algo > ALGO_WINOGRAD) return set_err(MP_E_ARG, "unknown algorithm");
    if ((algo == ALGO_STRASSEN || algo == ALGO_WINOGRAD) && cutoff < 1) return set_err(MP_E_ARG, "cutoff must be >= 1");
    if (policy < POLICY_PEEL || policy > POLICY_MIXED) return set_err(MP_E_ARG, "unknown odd-size policy");
    if (m < 0 || l < 0 || n < 0) return set_err(MP_E_ARG, "negative dimension");
    Plan P;
    PlanKey key{m, l, n, L, algo, cutoff, policy, 0, l, m * l, n, l * n, n, m * n};
    build_plan(P, key);
    const char* why = nullptr;
    if (!validate_plan(P, &why)) return set_err(MP_E_ARG, why);
    if (depth) *depth = P.depth;
    if (n_mul) *n_mul = P.n_mul;
    if (n_addsub) *n_addsub = P.n_addsub;
    if (ws_bytes) *ws_bytes = P.ws_words * 4;
    if (n_launches) *n_launches = (int64_t)P.steps.size();
    return MP_OK;
}

int mp_profile(int enable)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = enable != 0;
    return MP_OK;
}

int mp_profile_read(int max, int* kind, int* op, int* L, double* units, int64_t* ntiles, float* ms)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    int n = 0;
    for (ProfRec& r : g_prof) {
        if (n < max) {
            (void)hipEventSynchronize(r.e1);
            float t = 0;
            (void)hipEventElapsedTime(&t, r.e0, r.e1);
            kind[n] = r.kind; op[n] = r.op; L[n] = r.L; units[n] = r.units; ntiles[n] = r.ntiles; ms[n] = t;
        }
        n++;
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_prof.clear();
    return n;
}

int mp_gemm_batched(int count, const int64_t* m, const int64_t* l, const int64_t* n, int prec, int algo, int cutoff,
                    const uint32_t* const* A, const int64_t* lda, const int64_t* psa, const uint32_t* const* B,
                    const int64_t* ldb, const int64_t* psb, uint32_t* const* C, const int64_t* ldc, const int64_t* psc)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if (count < 0) return set_err(MP_E_ARG, "negative count");
    if (count == 0) return MP_OK;
    if (!m || !l || !n || !A || !lda || !psa || !B || !ldb || !psb || !C || !ldc || !psc)
        return set_err(MP_E_ARG, "a batch array is NULL");
    if (algo < ALGO_SIMPLE || algo > ALGO_WINOGRAD) return set_err(MP_E_ARG, "unknown algorithm");
    if ((algo == ALGO_STRASSEN || algo == ALGO_WINOGRAD) && cutoff < 1) return set_err(MP_E_ARG, "cutoff must be >= 1");
    std::vector<BatchItem> items;
    std::vector<uint32_t*> table;
    for (int r = 0; r < count; r++) {
        if (m[r] < 0 || l[r] < 0 || n[r] < 0) return set_err(MP_E_ARG, "negative dimension");
        if ((rc = check_mat("A", A[r], m[r], l[r], lda[r], psa[r])) || (rc = check_mat("B", B[r], l[r], n[r], ldb[r], psb[r])) ||
            (rc = check_mat("C", C[r], m[r], n[r], ldc[r], psc[r])))
            return rc;
        if (m[r] == 0 || n[r] == 0) continue;
        items.push_back(BatchItem{m[r], l[r], n[r], lda[r], psa[r], ldb[r], psb[r], ldc[r], psc[r]});
        table.push_back(const_cast<uint32_t*>(A[r]));
        table.push_back(const_cast<uint32_t*>(B[r]));
        table.push_back(C[r]);
    }
    if (items.empty()) return MP_OK;
    // every leaf of every item runs in one grouped launch, so no result may
    // overlap any operand or result of any item (inputs may share memory)
    {
        struct Extent { uintptr_t lo, hi; bool out; };
        std::vector<Extent> ext;
        for (size_t q = 0; q < items.size(); q++) {
            auto add = [&](const uint32_t* p, int64_t ps, bool out) {
                const uintptr_t lo = (uintptr_t)p, hi = lo + 4ull * (uint64_t)(L + 2) * (uint64_t)ps;
                if (hi > lo) ext.push_back(Extent{lo, hi, out});
            };
            if (items[q].l > 0) {
                add(table[3 * q], items[q].psa, false);
                add(table[3 * q + 1], items[q].psb, false);
            }
            add(table[3 * q + 2], items[q].psc, true);
        }
        std::sort(ext.begin(), ext.end(), [](const Extent& a, const Extent& b) { return a.lo < b.lo; });
        uintptr_t end_in = 0, end_out = 0;           // largest end so far of inputs / of results
        for (const Extent& e : ext) {
            if (e.lo < end_out || (e.out && e.lo < end_in))
                return set_err(MP_E_ALIAS, "a result of the batch overlaps an operand or another result");
            (e.out ? end_out : end_in) = std::max(e.out ? end_out : end_in, e.hi);
        }
    }
    if ((rc = device_check())) return rc;
    hipStream_t s = g_stream;
    Plan P;
    PlanKey key{0, 0, 0, L, algo, (algo == ALGO_STRASSEN || algo == ALGO_WINOGRAD) ? cutoff : 0, g_policy,
                algo == ALGO_BLOCK ? 1 : g_leaf, 0, 0, 0, 0, 0, 0};
    key.tcl = algo == ALGO_BLOCK ? 0 : g_tcl;
    key.persist = g_persist;
    build_plan_batched(P, key, items);
    const char* why = nullptr;
    if (!validate_plan(P, &why)) return set_err(MP_E_ARG, why);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t bg = al(P.gemm.size() * sizeof(GemmTask)), bn = al(P.node.size() * sizeof(NodeTask));
    const size_t bt = al(P.tiles.size() * 4), bb = al(table.size() * sizeof(uint32_t*));
    uint8_t* buf = (uint8_t*)workspace((bg + bn + bt + bb) / 4 + 64, s, WS_BATCH, &rc);
    if (rc) return rc;
    P.d_gemm = (GemmTask*)buf;
    P.d_node = (NodeTask*)(buf + bg);
    P.d_tiles = (int32_t*)(buf + bg + bn);
    uint32_t** d_table = (uint32_t**)(buf + bg + bn + bt);
    // pageable sources: each copy has read its source when the call returns
    if ((!P.gemm.empty() && hipMemcpyAsync(P.d_gemm, P.gemm.data(), P.gemm.size() * sizeof(GemmTask), hipMemcpyHostToDevice, s)) ||
        (!P.node.empty() && hipMemcpyAsync(P.d_node, P.node.data(), P.node.size() * sizeof(NodeTask), hipMemcpyHostToDevice, s)) ||
        (!P.tiles.empty() && hipMemcpyAsync(P.d_tiles, P.tiles.data(), P.tiles.size() * 4, hipMemcpyHostToDevice, s)) ||
        hipMemcpyAsync(d_table, table.data(), table.size() * sizeof(uint32_t*), hipMemcpyHostToDevice, s))
        return set_err(MP_E_DEVICE, "batch upload failed");
    Bases bs{};
    bs.ext = d_table;
    bs.p[BASE_WS] = workspace((size_t)P.ws_words, s, WS_PLAN, &rc);
    if (rc) return rc;
    rc = launch_steps(P, bs, s);
    P.d_gemm = nullptr;                        // the buffer belongs to the workspace
    P.d_node = nullptr;
    P.d_tiles = nullptr;
    if (rc) return rc;
    return device_check();
}

int mp_fill_uniform(int64_t rows, int64_t cols, int prec, uint32_t* X, int64_t ld, int64_t ps, uint64_t seed)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if (L > 32) return set_err(MP_E_PREC, "mp_fill_uniform takes prec 128 .. 1024");
    if ((rc = check_mat("X", X, rows, cols, ld, ps))) return rc;
    if (rows == 0 || cols == 0) return MP_OK;
    if ((rc = device_check())) return rc;
    if (launch_fill_uniform(L, X, ld, ps, rows, cols, seed, g_stream) != hipSuccess)
        return set_err(MP_E_DEVICE, "fill launch failed");
    return device_check();
}

int mp_set_graph_mode(int enable)
{
    g_graph_mode = enable ? 1 : 0;
    return MP_OK;
}

int mp_auto_choice(int64_t m, int64_t l, int64_t n, int prec, int* algo, int* cutoff, int* leaf)
{
    return mp_auto_launch(m, l, n, prec, algo, cutoff, leaf, nullptr, nullptr);
}

int mp_auto_launch(int64_t m, int64_t l, int64_t n, int prec, int* algo, int* cutoff, int* leaf, int* tile_cols_log2,
                   int* persistent)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    TuneEntry t;
    if (!tune_lookup(m, l, n, prec, &t)) t = tune_default(m, l, n);
    if (algo) *algo = t.algo;
    if (cutoff) *cutoff = t.cutoff;
    if (leaf) *leaf = t.leaf;
    if (tile_cols_log2) *tile_cols_log2 = t.tcl;
    if (persistent) *persistent = t.persist;
    return MP_OK;
}

int mp_set_launch(int tile_cols_log2, int persistent)
{
    if (tile_cols_log2 != 0 && (tile_cols_log2 < 4 || tile_cols_log2 > 6))
        return set_err(MP_E_ARG, "tile_cols_log2 must be 0 (64 columns) or 4 .. 6");
    if (persistent != 0 && persistent != 1) return set_err(MP_E_ARG, "persistent must be 0 or 1");
    g_tcl = tile_cols_log2 == 6 ? 0 : tile_cols_log2;
    g_persist = persistent;
    return MP_OK;
}

int mp_tune(int64_t m, int64_t l, int64_t n, int prec, int reps, int* algo, int* cutoff, int* leaf, float* ms)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if (m < 1 || l < 1 || n < 1 || m > INT32_MAX || l > INT32_MAX || n > INT32_MAX)
        return set_err(MP_E_ARG, "dimensions must be in 1 .. 2^31 - 1");
    if ((rc = device_check())) return rc;
    reps = reps < 1 ? 1 : reps;
    hipStream_t s = g_stream;
    const size_t wa = (size_t)(L + 2) * m * l, wb = (size_t)(L + 2) * l * n, wc = (size_t)(L + 2) * m * n;
    uint32_t* buf = nullptr;
    if (hipMalloc(&buf, 4 * (wa + wb + wc)) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(MP_E_NOMEM, "tuner scratch allocation failed");
    }
    uint32_t *A = buf, *B = buf + wa, *C = buf + wa + wb;
    if (launch_fill_uniform(L, A, l, m * l, m, l, 12345u, s) != hipSuccess ||
        launch_fill_uniform(L, B, n, l * n, l, n, 67890u, s) != hipSuccess) {
        (void)hipFree(buf);
        return set_err(MP_E_DEVICE, "tuner fill failed");
    }
    // stage 1: algorithm, cutoff and leaf kernel with the default launch
    // (64-column tiles, a workgroup per tile); stage 2: the tile width and
    // the persistent grid for the winner
    std::vector<TuneEntry> cand = {{ALGO_SIMPLE, 0, LEAF_SIMPLE, 0.f}, {ALGO_BLOCK, 0, LEAF_BLOCK, 0.f}};
    const int64_t mn = std::min(m, std::min(l, n));
    for (int a : {ALGO_WINOGRAD, ALGO_STRASSEN})
        for (int c : {32, 64, 128, 256})
            if (mn > c)
                for (int lf : {LEAF_SIMPLE, LEAF_BLOCK}) cand.push_back(TuneEntry{a, c, lf, 0.f});
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto time_one = [&](TuneEntry& t) {
        rc = gemm_internal(m, l, n, L, t.algo, t.cutoff, POLICY_PEEL, t.leaf, A, l, m * l, B, n, l * n, C, n, m * n, s,
                           t.tcl, t.persist);
        if (rc) return;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && !rc; r++)
            rc = gemm_internal(m, l, n, L, t.algo, t.cutoff, POLICY_PEEL, t.leaf, A, l, m * l, B, n, l * n, C, n,
                               m * n, s, t.tcl, t.persist);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float t_ms = 0;
        (void)hipEventElapsedTime(&t_ms, e0, e1);
        t.ms = t_ms / reps;
    };
    TuneEntry best{ALGO_SIMPLE, 0, LEAF_SIMPLE, 1e30f};
    for (TuneEntry& t : cand) {
        time_one(t);
        if (rc) break;
        if (t.ms < best.ms) best = t;
    }
    if (!rc) {
        std::vector<TuneEntry> launch;
        for (int tc : {0, 5, 4})
            for (int pe : {0, 1}) {
                if ((tc == 0 && pe == 0) || (tc != 0 && best.leaf == LEAF_BLOCK)) continue;
                TuneEntry t = best;
                t.tcl = tc;
                t.persist = pe;
                launch.push_back(t);
            }
        for (TuneEntry& t : launch) {
            time_one(t);
            if (rc) break;
            if (t.ms < best.ms) best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[tune_key(m, l, n, prec)] = best;
    }
    if (algo) *algo = best.algo;
    if (cutoff) *cutoff = best.cutoff;
    if (leaf) *leaf = best.leaf;
    if (ms) *ms = best.ms;
    return device_check();
}

int mp_tune_save(const char* path)
{
    if (!path) return set_err(MP_E_ARG, "path is NULL");
    FILE* f = fopen(path, "w");
    if (!f) return set_err(MP_E_ARG, "cannot open the tuning file");
    std::lock_guard<std::mutex> g(g_tune_mu);
    fprintf(f, "[");
    bool first = true;
    for (auto& kv : g_tune) {
        fprintf(f, "%s\n {\"prec\": %lld, \"m_log2\": %lld, \"l_log2\": %lld, \"n_log2\": %lld, \"algo\": %d, "
                   "\"cutoff\": %d, \"leaf\": %d, \"ms\": %.4f, \"tile_cols_log2\": %d, \"persistent\": %d}",
                first ? "" : ",", (long long)kv.first[0], (long long)kv.first[1], (long long)kv.first[2],
                (long long)kv.first[3], kv.second.algo, kv.second.cutoff, kv.second.leaf, kv.second.ms,
                kv.second.tcl, kv.second.persist);
        first = false;
    }
    fprintf(f, "\n]\n");
    fclose(f);
    return MP_OK;
}

int mp_tune_load(const char* path)
{
    if (!path) return set_err(MP_E_ARG, "path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return set_err(MP_E_ARG, "cannot open the tuning file");
    long long pr, a, b, c;
    int al, cu, lf, tc = 0, pe = 0;
    float t;
    int got = 0;
    std::lock_guard<std::mutex> g(g_tune_mu);
    char line[512];
    while (fgets(line, sizeof line, f)) {
        if (sscanf(line, " {\"prec\": %lld, \"m_log2\": %lld, \"l_log2\": %lld, \"n_log2\": %lld, \"algo\": %d, "
                         "\"cutoff\": %d, \"leaf\": %d, \"ms\": %f}",
                   &pr, &a, &b, &c, &al, &cu, &lf, &t) == 8) {
            // the launch fields are optional (files written before they existed)
            const char* q = strstr(line, "\"tile_cols_log2\":");
            if (!q || sscanf(q, "\"tile_cols_log2\": %d, \"persistent\": %d", &tc, &pe) != 2) tc = 0, pe = 0;
            if (al < ALGO_SIMPLE || al > ALGO_WINOGRAD || lf < 0 || lf > 1 || cu < 0) continue;
            if ((tc != 0 && (tc < 4 || tc > 6)) || (pe != 0 && pe != 1)) continue;
            g_tune[{pr, a, b, c}] = TuneEntry{al, cu, lf, t, tc == 6 ? 0 : tc, pe};
            got++;
        }
    }
    fclose(f);
    return got;
}

int mp_release_workspace(void)
{
    DeviceState& S = dev_state();
    std::lock_guard<std::mutex> g(S.mu);
    (void)hipDeviceSynchronize();
    for (auto& kv : S.ws)
        if (kv.second.p) (void)hipFree(kv.second.p);
    S.ws.clear();
    for (auto& kv : S.graphs) (void)hipGraphExecDestroy(kv.second);
    S.graphs.clear();
    for (auto& kv : S.plans) free_plan_device(*kv.second);
    S.plans.clear();
    return MP_OK;
}

}  // extern "C"
