// slice.cpp -- host driver of the INT8-slice product and its C-ABI entry.
//
// 1. exponent scan: per row of A and column of B, the largest and smallest
//    exponent of the nonzero entries (read back: the window depends on them);
// 2. window W = p + min(spread, extra) per operand, S = ceil((W + 2) / 8) digits;
// 3. digit planes A8[s][i][k], B8[t][j][k] (k contiguous, zero padded);
// 4. one grouped launch of INT8 MFMA tiles: every diagonal u = s + t, split into
//    slots whose inner length stays exact in INT32;
// 5. recombination and one rounding per entry.
//
// Certified early stop: the diagonals below u0 are computed only where they
// can matter.  The first pass computes the diagonals u >= u0 and rounds every
// entry whose rounding the omitted part (bounded below) cannot change; the
// second pass computes the low diagonals, and rounds again from all of them,
// only in the 256 x 256 tiles that hold an undecided entry.  The result is
// the same as computing every diagonal.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "mpgemm_internal.hpp"
#include "slice.hpp"

using namespace mpg;

namespace {

int64_t round_up(int64_t v, int64_t q) { return (v + q - 1) / q * q; }

#define SL_TRY(expr)                                                     \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) {                                          \
            g_err = std::string("slice path: ") + hipGetErrorString(e_); \
            return MP_E_DEVICE;                                          \
        }                                                                \
    } while (0)

int ceil_log2(int64_t v)
{
    int r = 0;
    while (((int64_t)1 << r) < v) r++;
    return r;
}

// guard bits of the early stop (< 0: every diagonal in one pass) and what
// the last call did: u0, diagonals, tiles recomputed, tiles, D
int g_slice_guard = 32;
int32_t g_slice_last[5] = {0, 0, 0, 0, 0};

int max_spread(const std::vector<int32_t>& hi, const std::vector<int32_t>& lo)
{
    int64_t s = 0;
    for (size_t i = 0; i < hi.size(); i++)
        if (hi[i] != INT32_MIN) s = std::max<int64_t>(s, (int64_t)hi[i] - lo[i]);
    return (int)std::min<int64_t>(s, 1 << 20);
}

}  // namespace

namespace mpg {

int slice_internal(int64_t m, int64_t l, int64_t n, int L, int extra, const uint32_t* A, int64_t lda, int64_t psa,
                   const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc, int64_t psc,
                   int32_t* window_out, hipStream_t s)
{
    const int p = 32 * L;
    const int64_t mpad = round_up(m, SLICE_TILE_M), npad = round_up(n, SLICE_TILE_N);
    const int64_t kpad = round_up(std::max<int64_t>(l, 1), SLICE_KSTEP);
    // scratch: exponent tables (4 arrays), then the digit planes, then G
    int rc = MP_OK;
    const int64_t nchunks = (std::max<int64_t>(l, 1) + 63) / 64;
    const size_t exp_words = (size_t)(2 * m + 2 * n + 2 * nchunks * n + 64);
    uint32_t* base = workspace(exp_words, s, WS_SLICE_EXP, &rc);
    if (rc) return rc;
    int32_t *ea = (int32_t*)base, *ea_lo = ea + m, *fb = ea_lo + m, *fb_lo = fb + n, *tmp = fb_lo + n;
    {
        ProfScope ps(s, 3, 2, L, (double)(m + n) * l, 0);
        SL_TRY(launch_slice_scan(L, A, lda, psa, m, l, 0, ea, ea_lo, tmp, s));
        SL_TRY(launch_slice_scan(L, B, ldb, psb, n, l, 1, fb, fb_lo, tmp, s));
    }
    std::vector<int32_t> h(2 * (size_t)m + 2 * (size_t)n);
    SL_TRY(hipMemcpyAsync(h.data(), base, h.size() * 4, hipMemcpyDeviceToHost, s));
    SL_TRY(hipStreamSynchronize(s));
    const std::vector<int32_t> ahi(h.begin(), h.begin() + m), alo(h.begin() + m, h.begin() + 2 * m);
    const std::vector<int32_t> bhi(h.begin() + 2 * m, h.begin() + 2 * m + n), blo(h.begin() + 2 * m + n, h.end());
    const int WA = p + std::min(max_spread(ahi, alo), extra);
    const int WB = p + std::min(max_spread(bhi, blo), extra);
    if (window_out) {
        window_out[0] = WA;
        window_out[1] = WB;
    }
    const int SA = (WA + 2 + 7) / 8, SB = (WB + 2 + 7) / 8;
    const int ndiag = SA + SB - 1;
    // tasks: diagonal u, pairs split into slots of at most SLICE_KMAX inner length
    const int64_t pairs_per_slot = std::max<int64_t>(1, SLICE_KMAX / kpad);
    std::vector<int32_t> slot_begin(1, 0);
    struct Slot { int u, s0, s1; };
    std::vector<Slot> slots;
    for (int u = 0; u < ndiag; u++) {
        const int lo = std::max(0, u - SB + 1), hi = std::min(u, SA - 1) + 1;
        for (int s0 = lo; s0 < hi; s0 += (int)pairs_per_slot)
            slots.push_back(Slot{u, s0, (int)std::min<int64_t>(hi, s0 + pairs_per_slot)});
        slot_begin.push_back((int32_t)slots.size());
    }
    // early stop: the omitted diagonals u < u0 add at most
    //   sum_{u<u0} pairs(u) 256^u l 2^14 < 2^D,  D = 8 u0 + 7 + ceil(log2 l) + ceil(log2 min(u0, S_A, S_B))
    // (|digit| <= 128, pairs(u) <= min(u0, S_A, S_B), sum_{u<u0} 256^u < 2 * 256^(u0-1)).  |Z| is near
    // 2^(W_A + W_B) unless the sum cancels, and its last kept bit is p bits below its top, so u0 is the
    // largest value leaving `guard` bits between 2^D and that bit.
    int u0 = 0, D = 0;
    if (g_slice_guard >= 0 && l > 0) {
        const int lg_l = ceil_log2(l), lg_np = ceil_log2(std::min(SA, SB));
        const int64_t room = (int64_t)WA + WB - p - g_slice_guard - 7 - lg_l - lg_np;
        u0 = room > 0 ? (int)std::min<int64_t>(room / 8, ndiag - 1) : 0;
        if (u0 > 0) D = 8 * u0 + 7 + lg_l + ceil_log2(std::min(u0, std::min(SA, SB)));
    }
    const int ti_n = (int)(mpad / SLICE_TILE_M), tj_n = (int)(npad / SLICE_TILE_N);
    const int64_t ntiles = (int64_t)ti_n * tj_n;
    // two task lists (diagonals u >= u0, then u < u0), each in dispatch order
    auto build = [&](bool high) {
        std::vector<SliceTask> order;
        for (size_t q = 0; q < slots.size(); q++) {
            if ((slots[q].u >= u0) != high) continue;
            for (int ti = 0; ti < ti_n; ti++)
                for (int tj = 0; tj < tj_n; tj++)
                    order.push_back(SliceTask{slots[q].u, slots[q].s0, slots[q].s1, (int32_t)q, ti, tj});
        }
        // longest first, so the grid drains evenly; neighbours in this order
        // share digit tiles of A or B
        std::stable_sort(order.begin(), order.end(),
                         [](const SliceTask& a, const SliceTask& b) { return (a.s1 - a.s0) > (b.s1 - b.s0); });
        // workgroups are dealt to the 8 XCDs round robin (block b on XCD b mod
        // 8): give each XCD runs of RUN consecutive tasks, runs dealt round
        // robin, so an XCD's L2 sees neighbouring tiles and the XCDs stay
        // balanced.  Round r of the dispatch takes the next task of every XCD
        // that still has one; the tail (unequal counts) is filled in order.
        const size_t NX = 8, RUN = 16, nt = order.size();
        std::vector<SliceTask> out(nt);
        std::vector<std::vector<size_t>> lists(NX);
        for (size_t r = 0; r * RUN < nt; r++)
            for (size_t q = r * RUN; q < std::min(nt, (r + 1) * RUN); q++) lists[r % NX].push_back(q);
        size_t b = 0;
        for (size_t round = 0; b < nt; round++)
            for (size_t x = 0; x < NX; x++)
                if (round < lists[x].size()) out[b++] = order[lists[x][round]];
        return out;
    };
    std::vector<SliceTask> tasks = build(true);
    const std::vector<SliceTask> tasks_low = build(false);
    const size_t n_high = tasks.size();
    tasks.insert(tasks.end(), tasks_low.begin(), tasks_low.end());
    // executed digit pairs of the first pass
    int64_t pairs_high = 0;
    for (int u = u0; u < ndiag; u++) pairs_high += std::min(u, SA - 1) - std::max(0, u - SB + 1) + 1;
    const int64_t a_plane = mpad * kpad, b_plane = npad * kpad, g_plane = mpad * npad;
    const size_t bytes_a = (size_t)SA * a_plane, bytes_b = (size_t)SB * b_plane;
    const size_t bytes_g = (size_t)slots.size() * g_plane * 4;
    const size_t bytes_t = tasks.size() * sizeof(SliceTask) + slot_begin.size() * 4 + (size_t)ntiles * 4;
    const size_t words = (bytes_a + bytes_b + bytes_g + bytes_t) / 4 + 256;
    uint8_t* ws = (uint8_t*)workspace(words, s, WS_SLICE, &rc);
    if (rc) return rc;
    int8_t* A8 = (int8_t*)ws;
    int8_t* B8 = A8 + ((bytes_a + 255) & ~size_t(255));
    int32_t* G = (int32_t*)(B8 + ((bytes_b + 255) & ~size_t(255)));
    SliceTask* d_tasks = (SliceTask*)((uint8_t*)G + bytes_g);
    int32_t* d_slot_begin = (int32_t*)(d_tasks + tasks.size());
    int32_t* d_flags = d_slot_begin + slot_begin.size();
    SL_TRY(hipMemcpyAsync(d_tasks, tasks.data(), tasks.size() * sizeof(SliceTask), hipMemcpyHostToDevice, s));
    SL_TRY(hipMemcpyAsync(d_slot_begin, slot_begin.data(), slot_begin.size() * 4, hipMemcpyHostToDevice, s));
    {
        ProfScope ps(s, 3, 0, L, (double)(m + n) * l, 0);
        SL_TRY(launch_slice_digits(L, A, lda, psa, m, l, 0, ea, WA, SA, A8, a_plane, mpad, kpad, s));
        SL_TRY(launch_slice_digits(L, B, ldb, psb, n, l, 1, fb, WB, SB, B8, b_plane, npad, kpad, s));
    }
    SL_TRY(launch_slice_fill(d_flags, ntiles, 0, s));
    {
        // algorithmic INT8 operations: the digit pairs this launch computes, over the unpadded product
        ProfScope ps(s, 2, 0, L, 2.0 * (double)pairs_high * (double)m * (double)l * (double)n, (int64_t)n_high);
        SL_TRY(launch_slice_gemm(d_tasks, (int64_t)n_high, A8, B8, G, a_plane, b_plane, g_plane, (int32_t)kpad,
                                 (int32_t)npad, nullptr, tj_n, s));
    }
    {
        ProfScope ps(s, 3, 1, L, (double)m * n, 0);
        SL_TRY(launch_slice_combine(L, G, g_plane, (int32_t)npad, d_slot_begin, ndiag, ea, fb, WA, WB, C, ldc, psc,
                                    m, n, u0 > 0 ? 1 : 0, u0, D, d_flags, tj_n, s));
    }
    if (u0 > 0) {
        // second pass: the low diagonals and the full rounding, flagged tiles only
        {
            // units unknown at launch (only flagged tiles compute): recorded as 0
            ProfScope ps(s, 2, 1, L, 0.0, (int64_t)tasks_low.size());
            SL_TRY(launch_slice_gemm(d_tasks + n_high, (int64_t)tasks_low.size(), A8, B8, G, a_plane, b_plane,
                                     g_plane, (int32_t)kpad, (int32_t)npad, d_flags, tj_n, s));
        }
        ProfScope ps(s, 3, 4, L, (double)m * n, 0);
        SL_TRY(launch_slice_combine(L, G, g_plane, (int32_t)npad, d_slot_begin, ndiag, ea, fb, WA, WB, C, ldc, psc,
                                    m, n, 2, 0, D, d_flags, tj_n, s));
    }
    std::vector<int32_t> hflags((size_t)ntiles);
    SL_TRY(hipMemcpyAsync(hflags.data(), d_flags, (size_t)ntiles * 4, hipMemcpyDeviceToHost, s));
    // the host vectors above are copied before this call returns only if the
    // stream has consumed them: wait for the uploads (and the flags)
    SL_TRY(hipStreamSynchronize(s));
    int32_t flagged = 0;
    for (int32_t f : hflags) flagged += f != 0;
    g_slice_last[0] = u0;
    g_slice_last[1] = ndiag;
    g_slice_last[2] = u0 > 0 ? flagged : 0;
    g_slice_last[3] = (int32_t)ntiles;
    g_slice_last[4] = D;
    return MP_OK;
}

}  // namespace mpg

extern "C" int mp_gemm_slice(int64_t m, int64_t l, int64_t n, int prec, int extra, const uint32_t* A, int64_t lda,
                             int64_t psa, const uint32_t* B, int64_t ldb, int64_t psb, uint32_t* C, int64_t ldc,
                             int64_t psc, int32_t* window_out)
{
    int L, rc;
    if ((rc = check_prec(prec, &L))) return rc;
    if (L > 32) return set_err(MP_E_PREC, "the slice path takes prec 128 .. 1024");
    if (extra < 0 || extra > SLICE_MAX_EXTRA) return set_err(MP_E_ARG, "extra must be in 0..64");
    if (m < 0 || l < 0 || n < 0) return set_err(MP_E_ARG, "negative dimension");
    // one digit-pair GEMM sums up to l products of at most 2^14 in INT32, and
    // the recombination's 64-bit partial sums stay exact while
    // min(S_A, S_B) * l < 2^25 (S <= 137 digits at 1024 bits)
    if (l > SLICE_KMAX) return set_err(MP_E_RANGE, "the slice path takes inner sizes l <= 131008");
    if ((rc = check_mat("A", A, m, l, lda, psa)) || (rc = check_mat("B", B, l, n, ldb, psb)) ||
        (rc = check_mat("C", C, m, n, ldc, psc)))
        return rc;
    if (m == 0 || n == 0) return MP_OK;
    if (l > 0 && (overlaps(C, psc, A, psa, L) || overlaps(C, psc, B, psb, L)))
        return set_err(MP_E_ALIAS, "C overlaps A or B");
    if ((rc = device_check())) return rc;
    if ((rc = slice_internal(m, l, n, L, extra, A, lda, psa, B, ldb, psb, C, ldc, psc, window_out, g_stream)))
        return rc;
    return device_check();
}

extern "C" int mp_set_slice_guard(int guard_bits)
{
    if (guard_bits > 1 << 20) return set_err(MP_E_ARG, "guard_bits too large");
    g_slice_guard = guard_bits < 0 ? -1 : guard_bits;
    return MP_OK;
}

extern "C" int mp_slice_last(int32_t* info5)
{
    if (info5 == nullptr) return set_err(MP_E_ARG, "info5 is null");
    for (int k = 0; k < 5; k++) info5[k] = g_slice_last[k];
    return MP_OK;
}
