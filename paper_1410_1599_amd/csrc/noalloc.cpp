// noalloc.cpp -- mp_gemm_noalloc: the product of mp_gemm without any device
// allocation, for callers that cannot allocate (code under stream capture,
// serving loops or harnesses that forbid hipMalloc).
//
// mp_gemm keeps a plan's task arrays in device buffers made on its first
// launch and its temporaries (the Strassen / Winograd operand sums and
// sub-products of every level) in a workspace pool that grows on demand.
// Here both live in one file-scope device array, `scratch`, of a fixed size:
// on every call the plan's task arrays are copied to its start and the
// temporaries follow.  The launches, kernels and order of operations are
// mp_gemm's, so the result is the same bit for bit.
//
// Host code never passes `scratch` itself to a kernel or a copy: its name is
// a host-side stand-in, not the device address.  The address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// kept per device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "mpgemm_internal.hpp"
#include "plan.hpp"
#include "tasks.hpp"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;

static __device__ __align__(256) uint32_t scratch[NOALLOC_SCRATCH_BYTES / 4];

std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch_addr;     // device id -> device address of that device's `scratch`

int scratch_address(uint8_t** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return mpg::set_err(MP_E_DEVICE, "no current device");
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return MP_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return mpg::set_err(MP_E_DEVICE, (std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                          hipGetErrorString(e)).c_str());
    }
    g_scratch_addr[dev] = (uint8_t*)ptr;
    *out = (uint8_t*)ptr;
    return MP_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

using namespace mpg;

extern "C" int mp_gemm_noalloc(int64_t m, int64_t l, int64_t n, int prec, int algo, int cutoff, const uint32_t* A,
                               int64_t lda, int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C,
                               int64_t ldc, int64_t psc)
{
    int L, rc, tcl, persist;
    int leaf = g_leaf, policy = g_policy;
    if ((rc = gemm_validate(m, l, n, prec, &algo, &cutoff, policy, &leaf, A, lda, psa, B, ldb, psb, C, ldc, psc, &L,
                            &tcl, &persist)))
        return rc;
    if (m == 0 || n == 0) return MP_OK;
    PlanKey key{m, l, n, L, algo, cutoff, policy, algo == ALGO_BLOCK ? 1 : leaf, lda, psa, ldb, psb, ldc, psc};
    key.tcl = algo == ALGO_BLOCK ? 0 : tcl;
    key.persist = persist;
    if (algo == ALGO_SIMPLE || algo == ALGO_BLOCK) key.cutoff = 0, key.policy = 0;
    // the plan is host memory only (built and validated once, cached)
    Plan* P = get_plan(key, &rc, false);
    if (!P) return rc ? rc : MP_E_ARG;
    const size_t bg = align256(P->gemm.size() * sizeof(GemmTask));
    const size_t bn = align256(P->node.size() * sizeof(NodeTask));
    const size_t bt = align256(P->tiles.size() * sizeof(int32_t));
    const size_t need = bg + bn + bt + (size_t)P->ws_words * 4;
    if (need > NOALLOC_SCRATCH_BYTES) {
        char msg[160];
        snprintf(msg, sizeof msg, "mp_gemm_noalloc: this product needs %zu bytes of scratch, above the %zu-byte maximum",
                 need, NOALLOC_SCRATCH_BYTES);
        return set_err(MP_E_RANGE, msg);
    }
    if ((rc = device_check())) return rc;
    uint8_t* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    hipStream_t s = g_stream;
    GemmTask* dg = (GemmTask*)base;
    NodeTask* dn = (NodeTask*)(base + bg);
    int32_t* dt = (int32_t*)(base + bg + bn);
    // pageable sources: each copy has read its source when the call returns
    if ((!P->gemm.empty() && hipMemcpyAsync(dg, P->gemm.data(), P->gemm.size() * sizeof(GemmTask),
                                            hipMemcpyHostToDevice, s) != hipSuccess) ||
        (!P->node.empty() && hipMemcpyAsync(dn, P->node.data(), P->node.size() * sizeof(NodeTask),
                                            hipMemcpyHostToDevice, s) != hipSuccess) ||
        (!P->tiles.empty() && hipMemcpyAsync(dt, P->tiles.data(), P->tiles.size() * sizeof(int32_t),
                                             hipMemcpyHostToDevice, s) != hipSuccess)) {
        (void)hipGetLastError();
        return set_err(MP_E_DEVICE, "copy of the plan into the scratch array failed");
    }
    Bases bs{};
    bs.p[BASE_A] = const_cast<uint32_t*>(A);
    bs.p[BASE_B] = const_cast<uint32_t*>(B);
    bs.p[BASE_C] = C;
    bs.p[BASE_WS] = P->ws_words ? (uint32_t*)(base + bg + bn + bt) : nullptr;
    if ((rc = launch_plan_steps(*P, dg, dn, dt, bs, s))) return rc;
    return device_check();
}
