// mpgemm_internal.hpp -- helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mpgemm.h"

namespace mpg {

extern thread_local hipStream_t g_stream;
extern thread_local std::string g_err;
extern int g_leaf;
extern int g_policy;
extern int g_tcl;         // leaf tile width, log2 columns (0: 64 columns)
extern int g_persist;     // persistent grids

int set_err(int code, const char* msg);
int check_prec(int prec, int* L);
int check_mat(const char* name, const uint32_t* p, int64_t rows, int64_t cols, int64_t ld, int64_t ps);
bool overlaps(const uint32_t* a, int64_t psa, const uint32_t* b, int64_t psb, int L);
int device_check();
enum WsSlot { WS_PLAN = 0, WS_LU = 1, WS_SLICE = 2, WS_SLICE_EXP = 3, WS_BATCH = 4, WS_SOLVE = 5 };
// per-stream, per-slot device buffer of at least `words` uint32 (grown on demand)
uint32_t* workspace(size_t words, hipStream_t s, int slot, int* rc);

// C := A B through a cached plan (no argument checks); tcl / persist < 0
// take the process settings of mp_set_launch
int gemm_internal(int64_t m, int64_t l, int64_t n, int L, int algo, int cutoff, int policy, int leaf,
                  const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb,
                  uint32_t* C, int64_t ldc, int64_t psc, hipStream_t s, int tcl = -1, int persist = -1);

struct Plan;
struct PlanKey;
struct GemmTask;
struct NodeTask;
struct Bases;

// The cached plan for key, built and validated on first use; with device
// true its task arrays are also copied to device buffers of the library.
Plan* get_plan(const PlanKey& key, int* rc, bool device);

// Enqueue the plan's launches on s, reading its task arrays and tile map
// from the given device copies.
int launch_plan_steps(const Plan& P, const GemmTask* d_gemm, const NodeTask* d_node, const int32_t* d_tiles,
                      const Bases& bs, hipStream_t s);

// The argument checks of mp_gemm_ex; resolves MP_AUTO (algo, cutoff, leaf)
// and returns the limb count in *L_out.
int gemm_validate(int64_t m, int64_t l, int64_t n, int prec, int* algo_io, int* cutoff_io, int policy, int* leaf_io,
                  const uint32_t* A, int64_t lda, int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb,
                  const uint32_t* C, int64_t ldc, int64_t psc, int* L_out, int* tcl_out = nullptr,
                  int* persist_out = nullptr);

// C := A op B elementwise through a cached one-task plan (no argument checks)
int ew_internal(int op, int64_t m, int64_t n, int L, const uint32_t* A, int64_t lda, int64_t psa,
                const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc, hipStream_t s);

// Records a HIP event pair around the launches of its lifetime on stream s
// when the step profiler is on (mp_profile); kind 0 = leaf products,
// 1 = node passes, 2 = INT8 MFMA products, 3 = other slice kernels.
class ProfScope {
public:
    ProfScope(hipStream_t s, int kind, int op, int L, double units, int64_t ntiles);
    ~ProfScope();

private:
    hipStream_t s_;
    int kind_, op_, L_;
    double units_;
    int64_t ntiles_;
    bool on_;
    hipEvent_t e0_ = nullptr, e1_ = nullptr;
};

// INT8-slice product (slice.cpp); synchronises the stream
int slice_internal(int64_t m, int64_t l, int64_t n, int L, int extra, const uint32_t* A, int64_t lda, int64_t psa,
                   const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc,
                   int32_t* window_out, hipStream_t s);

}  // namespace mpg
