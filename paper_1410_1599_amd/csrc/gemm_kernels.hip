// gemm_kernels.hip -- leaf products and per-node elementwise passes.
//
// Leaf product (Section 2, eq. (1)): every output element is owned by one
// lane, which runs c := add_rn(c, mul_rn(a_ik, b_kj)) for k ascending from an
// exact zero.  A workgroup owns TM rows x 64 columns of one product: each
// wave one row, each lane one column, so a wave reads one A element per k
// (the same address in every lane) and 64 consecutive B elements.
//
// Block (eq. (2)) stages TK x 64 tiles of B and TM x TK tiles of A in LDS and
// runs the same per-element k order, so it is bit-identical to Simple.
//
// Every launch is grouped: a list of GemmTasks (up to the 7^d leaves of a
// Strassen/Winograd plan plus its peel products) is cut into tiles, and
// tile_task maps a tile to its task.  The grid may be smaller than the tile
// count (persistent mode): workgroups stride over the tiles.
#include <algorithm>
#include <map>
#include <mutex>

#include "launch.hpp"
#include "mp_arith.hpp"
#include "node_ops.hpp"

namespace mpg {

// Base pointers come from a table in memory; read through vector loads they
// would count as per-lane values.  They are the same in every lane (one task
// per workgroup), so move them to scalar registers.
__device__ __forceinline__ uint32_t* wave_uniform(uint32_t* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (uint32_t*)(((uint64_t)hi << 32) | lo);
}

template <int L>
__device__ __forceinline__ const uint32_t* ref_ptr(const Bases& b, const MatRef& r)
{
    return wave_uniform(base_ptr(b, r.base)) + r.off;
}

// Word idx of a plane whose base is the same in every lane, for planes of
// fewer than 2^30 words: a global load with the base in scalar registers and
// a 32-bit lane offset, so the address costs no vector arithmetic per limb.
__device__ __forceinline__ uint32_t ld_plane(const uint32_t* base, uint32_t idx)
{
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) uint32_t gu32;
    return *(gu32*)((gchar*)base + idx * 4u);
}

template <int L>
__device__ __forceinline__ MP<L> load_planes(const uint32_t* base, int64_t ps, uint32_t idx)
{
    MP<L> x;
#pragma unroll
    for (int q = 0; q < L; q++) x.m[q] = ld_plane(base + q * ps, idx);
    x.e = (int32_t)ld_plane(base + L * ps, idx);
    x.s = ld_plane(base + (L + 1) * ps, idx);
    return x;
}

// Workgroups are handed to the eight XCDs round robin (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  Renumber them so that XCD x walks a
// contiguous run of tiles: the tiles of one leaf product, which share its B
// block (and A rows), then meet in one L2 instead of eight.  A bijection of
// [0, G) for any grid size G.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G)
{
    const int64_t q = G >> 3, r = G & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// ------------------------------------------------------------------ Simple

template <int L, int TM>
__global__ void __launch_bounds__(64 * TM) __attribute__((amdgpu_waves_per_eu(leaf_waves(L))))
k_gemm_simple(const GemmTask* __restrict__ tasks, const int32_t* __restrict__ tile_task, int64_t ntiles, Bases bs)
{
    for (int64_t t = xcd_tile(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x) {
        const GemmTask T = tasks[tile_task[t]];
        const int64_t lt = t - T.tile0;
        // a tile is (64 TM / 2^tcl) rows x 2^tcl columns, lanes along a row
        const int tc = 1 << T.tcl;
        const int tr = (64 * TM) >> T.tcl;
        const int tn = (T.n + tc - 1) >> T.tcl;
        const int64_t i = (lt / tn) * tr + (threadIdx.x >> T.tcl);
        const int64_t j = (lt % tn) * tc + (threadIdx.x & (tc - 1));
        if (i >= T.m || j >= T.n) continue;
        // C's address is formed where it is used (before and after the loop),
        // so that no register holds it across the loop
        MP<L> c = T.accum ? load<L>(wave_uniform(base_ptr(bs, T.C.base)) + T.C.off + i * T.C.ld + j, T.C.ps, 0)
                          : mp_zero<L>();
        // a_ik at A + i * ia + k * ka: row-major, or a transposed copy (T.at)
        const int64_t ia = T.at ? 1 : T.A.ld, ka = T.at ? T.A.ld : 1;
        if (T.A.ps < (1 << 30) && T.B.ps < (1 << 30)) {
            // every offset inside a plane fits 32 bits
            const uint32_t* A = ref_ptr<L>(bs, T.A);
            const uint32_t* B = ref_ptr<L>(bs, T.B);
            uint32_t oa = (uint32_t)i * (uint32_t)ia;
            const uint32_t aks = (uint32_t)ka;
            const uint32_t bld = (uint32_t)T.B.ld;
            uint32_t ob = (uint32_t)j;
            for (int k = 0; k < T.l; k++) {
                const MP<L> a = load_planes<L>(A, T.A.ps, oa);
                const MP<L> b = load_planes<L>(B, T.B.ps, ob);
                oa += aks;
                ob += bld;
                c = add_rn<L>(c, mul_rn<L>(a, b));
            }
        } else {
            const uint32_t* A = ref_ptr<L>(bs, T.A) + i * ia;
            const uint32_t* B = ref_ptr<L>(bs, T.B) + j;
            for (int k = 0; k < T.l; k++) {
                const MP<L> a = load<L>(A, T.A.ps, (int64_t)k * ka);
                const MP<L> b = load<L>(B, T.B.ps, (int64_t)k * T.B.ld);
                c = add_rn<L>(c, mul_rn<L>(a, b));
            }
        }
        store<L>(wave_uniform(base_ptr(bs, T.C.base)) + T.C.off + i * T.C.ld + j, T.C.ps, 0, c);
    }
}

// ------------------------------------------------------------------ Block (LDS tiles)

// global_load_lds_dword: each lane's word at src goes to LDS at lds + 4 * lane,
// without passing through registers.  Issued through asm so that the compiler,
// which cannot see the LDS write, leaves the waiting to the kernel's explicit
// vmcnt wait before its barrier (the instruction has no register result).
__device__ __forceinline__ void lds_dma4(const uint32_t* src, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %1\n\t"
                 "s_nop 0\n\t"
                 "global_load_lds_dword %0, off"
                 :
                 : "v"(src), "s"(lds)
                 : "m0", "memory");
}

// a value the whole wave holds, moved to scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t lds_addr32(const uint32_t* p)
{
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t*)p;
}

// Block (eq. (2)): a workgroup of TM waves owns TM rows x 64 columns and
// walks k in blocks of TK.  Both operands' k-blocks are staged in LDS, double
// buffered: B's TK x 64 elements (every plane), read there by all TM waves
// instead of every wave fetching its own copy, and A's TM x TK elements.  The
// staging is the asynchronous global-to-LDS copy, one instruction per 64
// words: B's row-planes (64 consecutive words each) and A's block in chunks
// of 64 (lane t fetches one word of one element) are dealt out over the
// waves, and one barrier per block both publishes block kb and retires the
// buffer that block kb + 1 then overwrites.  The inner loop touches LDS only,
// so the next block's copies stay in flight during the products (a global
// load there would make the compiler's wait for it also wait for them).
// Every element keeps Simple's order (k ascending from exact zero), so Block
// is bit-identical to Simple.
template <int L, int TM, int TK>
__global__ void __launch_bounds__(64 * TM) __attribute__((amdgpu_waves_per_eu(leaf_waves(L))))
k_gemm_block(const GemmTask* __restrict__ tasks, const int32_t* __restrict__ tile_task, int64_t ntiles, Bases bs)
{
    constexpr int W = L + 2;                  // words (planes) per element
    constexpr int ROWS = TK * W;              // B: row-planes of one k-block
    constexpr int AW = TM * TK * W;           // A: words of one k-block
    constexpr int NA = (AW + 63) / 64;        // A: 64-word chunks
    __shared__ uint32_t sB[2][TK][W][64];     // limb-major: a wave reads 64 consecutive words per plane
    __shared__ uint32_t sA[2][NA * 64];       // word (r * TK + kk) * W + q: row i0 + r, k kb * TK + kk, plane q
    const int lane = threadIdx.x & 63;
    // the wave's index, as a scalar for the copy loop, and as a lane value
    // for everything the products touch: A's element read through a scalar
    // index is known to be uniform, and the compiler then moves parts of the
    // product to scalar code (measured: 11% more vector and four times the
    // scalar instructions per multiply-add)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wv = threadIdx.x >> 6;
    for (int64_t t = xcd_tile(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x) {
        const GemmTask T = tasks[tile_task[t]];
        const int64_t lt = t - T.tile0;
        const int tn = (T.n + 63) >> 6;
        const int64_t i0 = (lt / tn) * TM;
        const int64_t j0 = (lt % tn) * 64;
        const int64_t i = i0 + wv, j = j0 + lane;
        const bool row_live = i < T.m;        // uniform in the wave
        const bool live = row_live && (j < T.n);
        const uint32_t* A = ref_ptr<L>(bs, T.A);
        // lanes past the last column copy the last column (their results are dropped)
        const uint32_t* Bc = ref_ptr<L>(bs, T.B) + (j < T.n ? j : T.n - 1);
        uint32_t* C = base_ptr(bs, T.C.base) + T.C.off;
        MP<L> c = (T.accum && live) ? load<L>(C + i * T.C.ld + j, T.C.ps, 0) : mp_zero<L>();
        const int nkb = (T.l + TK - 1) / TK;
        // A's copy addresses for this tile: wave w copies chunks w, w + TM,
        // ...; lane t of chunk ch fetches word u = 64 ch + t of the block,
        // row i0 + u / (TK W), k-offset kk = (u / W) mod TK, plane u mod W.
        // Rows past m fetch row m - 1 (the products never read them).
        constexpr int CPW = (NA + TM - 1) / TM;
        const uint32_t* ap[CPW];
        int akk[CPW];
#pragma unroll
        for (int s = 0; s < CPW; s++) {
            const int u = (w + s * TM) * 64 + lane;
            const int rr = u / (TK * W), v = u - rr * (TK * W);
            const int kk = v / W, q = v - kk * W;
            int64_t row = i0 + (rr < TM ? rr : TM - 1);
            row = row < T.m ? row : T.m - 1;
            ap[s] = A + q * T.A.ps + row * T.A.ld;
            akk[s] = kk;
        }
        // the copies of block kb: B's k-rows w, w + TM, ... (all W planes,
        // one scalar stride apart), then A's chunks; k past l fetches k = l - 1
        auto issue = [&](int kb) {
            const int buf = kb & 1;
            const int64_t k0 = (int64_t)kb * TK;
            for (int kk = w; kk < TK; kk += TM) {
                if (k0 + kk < T.l) {
                    const uint32_t* src = Bc + uniform64((k0 + kk) * T.B.ld);
                    const uint32_t dst = __builtin_amdgcn_readfirstlane(lds_addr32(&sB[buf][kk][0][0]));
#pragma unroll
                    for (int q = 0; q < W; q++) lds_dma4(src + q * T.B.ps, dst + q * 256);
                }
            }
#pragma unroll
            for (int s = 0; s < CPW; s++) {
                const int ch = w + s * TM;
                if (ch < NA) {
                    int64_t k = k0 + akk[s];
                    k = k < T.l ? k : T.l - 1;
                    lds_dma4(ap[s] + k, __builtin_amdgcn_readfirstlane(lds_addr32(&sA[buf][ch * 64])));
                }
            }
        };
        __syncthreads();                      // the previous tile's reads of both buffers are done
        if (nkb > 0) issue(0);
        for (int kb = 0; kb < nkb; kb++) {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies have landed
            __syncthreads();                  // every wave's copies of block kb; block kb - 1 retired
            if (kb + 1 < nkb) issue(kb + 1);
            if (row_live) {
                const int buf = kb & 1;
                const int kn = (T.l - kb * TK) < TK ? (T.l - kb * TK) : TK;
                for (int kk = 0; kk < kn; kk++) {
                    const uint32_t* sa = &sA[buf][(wv * TK + kk) * W];
                    MP<L> a, b;
#pragma unroll
                    for (int q = 0; q < L; q++) {
                        a.m[q] = sa[q];
                        b.m[q] = sB[buf][kk][q][lane];
                    }
                    a.e = (int32_t)sa[L];
                    a.s = sa[L + 1];
                    b.e = (int32_t)sB[buf][kk][L][lane];
                    b.s = sB[buf][kk][L + 1][lane];
                    c = add_rn<L>(c, mul_rn<L>(a, b));
                }
            }
        }
        if (live) store<L>(C + i * T.C.ld + j, T.C.ps, 0, c);
    }
}

// ------------------------------------------------------------------ node passes

template <int L, int OP>
__global__ void __launch_bounds__(NODE_TILE)
k_node(const NodeTask* __restrict__ tasks, const int32_t* __restrict__ tile_task, int64_t ntiles, Bases bs)
{
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const NodeTask& T = tasks[tile_task[t]];
        const int64_t e = (t - T.tile0) * NODE_TILE + threadIdx.x;
        const int64_t total = (int64_t)T.rows * T.cols;
        if (e >= total) continue;
        if (total <= (int64_t)0xffffffff) {       // 32-bit row and column (a 64-bit division costs ~170 VALU)
            const uint32_t e32 = (uint32_t)e, c32 = (uint32_t)T.cols;
            const uint32_t i32 = e32 / c32;
            node_apply<MP<L>, L, OP>(bs, T, i32, e32 - i32 * c32);
        } else {
            node_apply<MP<L>, L, OP>(bs, T, e / T.cols, e % T.cols);
        }
    }
}

// ------------------------------------------------------------------ scratch fill

__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Seeded values uniform on (-1, 1): W = L hashed words read as a p-bit
// integer, x = +-W 2^-p (sign from the hash), normalised; W = 0 is zero.
template <int L>
__global__ void __launch_bounds__(256)
k_fill_uniform(uint32_t* X, int64_t ld, int64_t ps, int64_t rows, int64_t cols, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t i = e / cols, j = e % cols;
    const uint32_t h = mix32((uint32_t)seed ^ mix32((uint32_t)(seed >> 32) ^ mix32((uint32_t)e ^ mix32((uint32_t)(e >> 32)))));
    uint32_t w[L];
#pragma unroll
    for (int k = 0; k < L; k++) w[k] = mix32(h + 0x9e3779b9u * (uint32_t)(k + 1));
    int32_t top = -1;
#pragma unroll
    for (int k = 0; k < L; k++) top = w[k] ? k : top;
    MP<L> r = mp_zero<L>();
    if (top >= 0) {
        uint32_t tw = 0;
#pragma unroll
        for (int k = 0; k < L; k++) tw = (k == top) ? w[k] : tw;
        const int32_t z = 32 * (L - 1 - top) + (int32_t)__builtin_clz(tw);   // leading zeros of W
        const int32_t q = z >> 5;
        const uint32_t b = (uint32_t)z & 31u;
#pragma unroll
        for (int k = 0; k < L; k++) {
            uint32_t hi = 0, lo = 0;
#pragma unroll
            for (int t = 0; t < L; t++) {
                hi = (t == k - q) ? w[t] : hi;
                lo = (t == k - q - 1) ? w[t] : lo;
            }
            r.m[k] = b ? funnel(hi, lo, 32u - b) : hi;
        }
        r.e = -z;
        r.s = (h >> 7) & 1u;
    }
    store<L>(X, ps, i * ld + j, r);
}

// ------------------------------------------------------------------ transpose

// out0 (cols x rows) := in0 (rows x cols) transposed, every one of the nplanes
// planes (limbs, exponent, sign) copied word for word.  A tile is a 16 x 16
// block of the source; it passes through LDS so that both the reads (along
// the source rows) and the writes (along the destination rows) are runs of
// 16 consecutive words.
__global__ void __launch_bounds__(256)
k_transpose(const NodeTask* __restrict__ tasks, const int32_t* __restrict__ tile_task, int64_t ntiles, Bases bs,
            int nplanes)
{
    __shared__ uint32_t tile[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const NodeTask& T = tasks[tile_task[t]];
        const int64_t lt = t - T.tile0;
        const int64_t nbj = (T.cols + 15) / 16;
        const int64_t i0 = (lt / nbj) * 16, j0 = (lt % nbj) * 16;
        const uint32_t* src = base_ptr(bs, T.in[0].base) + T.in[0].off;
        uint32_t* dst = base_ptr(bs, T.out[0].base) + T.out[0].off;
        for (int q = 0; q < nplanes; q++) {
            const int64_t si = i0 + ty, sj = j0 + tx;
            if (si < T.rows && sj < T.cols) tile[ty][tx] = src[q * T.in[0].ps + si * T.in[0].ld + sj];
            __syncthreads();
            const int64_t di = j0 + ty, dj = i0 + tx;           // destination row = source column
            if (di < T.cols && dj < T.rows) dst[q * T.out[0].ps + di * T.out[0].ld + dj] = tile[tx][ty];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ launchers

// Grid of a launch: `grid` workgroups, or with grid <= 0 a persistent grid of
// as many workgroups as the device keeps resident at once (compute units x
// the kernel's occupancy per unit, from its register and LDS use), capped by
// the tile count; the kernels stride over the tiles either way.
static int device_cus()
{
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
    return n;
}

template <class K>
static int64_t launch_grid(K kernel, int block, int64_t ntiles, int64_t grid)
{
    if (grid > 0) return grid;
    static std::mutex mu;
    static std::map<const void*, int> occ;            // kernel -> resident workgroups per compute unit
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = occ.find((const void*)kernel);
        if (it != occ.end()) {
            per_cu = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            occ[(const void*)kernel] = per_cu;
        }
    }
    return std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)device_cus() * per_cu));
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* X, int64_t count, int32_t value)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) X[i] = value;
}

hipError_t launch_fill_i32(int32_t* X, int64_t count, int32_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, X, count, value);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(int L, uint32_t* X, int64_t ld, int64_t ps, int64_t rows, int64_t cols, uint64_t seed,
                               hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 g((unsigned)((rows * cols + 255) / 256));
    switch (L) {
    case 4: hipLaunchKernelGGL((k_fill_uniform<4>), g, dim3(256), 0, s, X, ld, ps, rows, cols, seed); break;
    case 8: hipLaunchKernelGGL((k_fill_uniform<8>), g, dim3(256), 0, s, X, ld, ps, rows, cols, seed); break;
    case 16: hipLaunchKernelGGL((k_fill_uniform<16>), g, dim3(256), 0, s, X, ld, ps, rows, cols, seed); break;
    case 32: hipLaunchKernelGGL((k_fill_uniform<32>), g, dim3(256), 0, s, X, ld, ps, rows, cols, seed); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
static hipError_t gemm_launch_L(int kind, const GemmTask* tasks, const int32_t* tile_task, int64_t ntiles,
                                const Bases& bs, int64_t grid, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (kind == LEAF_BLOCK) {
        constexpr int TK = block_tk(L);
        const dim3 g((unsigned)launch_grid(k_gemm_block<L, GEMM_TM, TK>, 64 * GEMM_TM, ntiles, grid));
        hipLaunchKernelGGL((k_gemm_block<L, GEMM_TM, TK>), g, dim3(64 * GEMM_TM), 0, s, tasks, tile_task, ntiles, bs);
    } else {
        const dim3 g((unsigned)launch_grid(k_gemm_simple<L, GEMM_TM>, 64 * GEMM_TM, ntiles, grid));
        hipLaunchKernelGGL((k_gemm_simple<L, GEMM_TM>), g, dim3(64 * GEMM_TM), 0, s, tasks, tile_task, ntiles, bs);
    }
    return hipGetLastError();
}

hipError_t launch_gemm(int L, int kind, const GemmTask* tasks, const int32_t* tile_task, int64_t ntiles,
                       const Bases& bs, int64_t grid, hipStream_t s)
{
    if (L >= 64)                        // Block = Simple's order; a wave per element, grids per tile
        return launch_gemm_wide(L, tasks, tile_task, ntiles, bs, grid > 0 ? grid : ntiles, s);
    switch (L) {
    case 4: return gemm_launch_L<4>(kind, tasks, tile_task, ntiles, bs, grid, s);
    case 8: return gemm_launch_L<8>(kind, tasks, tile_task, ntiles, bs, grid, s);
    case 16: return gemm_launch_L<16>(kind, tasks, tile_task, ntiles, bs, grid, s);
    case 32: return gemm_launch_L<32>(kind, tasks, tile_task, ntiles, bs, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int L, int OP>
static void node_launch_one(const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles, const Bases& bs,
                            int64_t grid, hipStream_t s)
{
    const dim3 g((unsigned)launch_grid(k_node<L, OP>, NODE_TILE, ntiles, grid));
    hipLaunchKernelGGL((k_node<L, OP>), g, dim3(NODE_TILE), 0, s, tasks, tile_task, ntiles, bs);
}

template <int L>
static hipError_t node_launch_L(int op, const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles,
                                const Bases& bs, int64_t grid, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    switch (op) {
    case OP_ADD: node_launch_one<L, OP_ADD>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_SUB: node_launch_one<L, OP_SUB>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_MUL: node_launch_one<L, OP_MUL>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_DIV: node_launch_one<L, OP_DIV>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_COPY: node_launch_one<L, OP_COPY>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_PADCOPY: node_launch_one<L, OP_PADCOPY>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_WINO_A: node_launch_one<L, OP_WINO_A>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_WINO_B: node_launch_one<L, OP_WINO_B>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_WINO_C: node_launch_one<L, OP_WINO_C>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_STR_A: node_launch_one<L, OP_STR_A>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_STR_B: node_launch_one<L, OP_STR_B>(tasks, tile_task, ntiles, bs, grid, s); break;
    case OP_STR_C: node_launch_one<L, OP_STR_C>(tasks, tile_task, ntiles, bs, grid, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_node(int L, int op, const NodeTask* tasks, const int32_t* tile_task, int64_t ntiles,
                       const Bases& bs, int64_t grid, hipStream_t s)
{
    if (op == OP_TRANSPOSE) {           // word copies: one kernel for every precision
        if (ntiles <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_transpose, dim3((unsigned)launch_grid(k_transpose, 256, ntiles, grid)), dim3(256), 0, s,
                           tasks, tile_task, ntiles, bs, L + 2);
        return hipGetLastError();
    }
    if (L >= 64) return launch_node_wide(L, op, tasks, tile_task, ntiles, bs, grid > 0 ? grid : ntiles, s);
    switch (L) {
    case 4: return node_launch_L<4>(op, tasks, tile_task, ntiles, bs, grid, s);
    case 8: return node_launch_L<8>(op, tasks, tile_task, ntiles, bs, grid, s);
    case 16: return node_launch_L<16>(op, tasks, tile_task, ntiles, bs, grid, s);
    case 32: return node_launch_L<32>(op, tasks, tile_task, ntiles, bs, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mpg
