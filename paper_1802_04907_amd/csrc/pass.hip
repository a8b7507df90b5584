// The full pass g = Q1^T r of the QIHT iteration: the one launch that reads
// every packed code of Q1, and the bandwidth-bound kernel of the path.
#include <hip/hip_ext.h>

#include "solve_common.h"

namespace qiht {
namespace {

__device__ __forceinline__ float ub0(uint32_t x) { return static_cast<float>(x & 0xFFu); }
__device__ __forceinline__ float ub1(uint32_t x) { return static_cast<float>((x >> 8) & 0xFFu); }
__device__ __forceinline__ float ub2(uint32_t x) { return static_cast<float>((x >> 16) & 0xFFu); }
__device__ __forceinline__ float ub3(uint32_t x) { return static_cast<float>(x >> 24); }

// sum_q code_q * r[q] over the 32/BITS codes of one word (FP32 FMA),
// split over two accumulators.
template <int BITS>
__device__ __forceinline__ void dot_word(uint32_t w, const float* r, float& a0,
                                         float& a1) {
    if constexpr (BITS == 8) {
        a0 = fmaf(ub0(w), r[0], a0);
        a1 = fmaf(ub1(w), r[1], a1);
        a0 = fmaf(ub2(w), r[2], a0);
        a1 = fmaf(ub3(w), r[3], a1);
    } else if constexpr (BITS == 4) {
        const uint32_t lo = w & 0x0F0F0F0Fu;          // codes 0, 2, 4, 6
        const uint32_t hi = (w >> 4) & 0x0F0F0F0Fu;   // codes 1, 3, 5, 7
        a0 = fmaf(ub0(lo), r[0], a0);
        a1 = fmaf(ub0(hi), r[1], a1);
        a0 = fmaf(ub1(lo), r[2], a0);
        a1 = fmaf(ub1(hi), r[3], a1);
        a0 = fmaf(ub2(lo), r[4], a0);
        a1 = fmaf(ub2(hi), r[5], a1);
        a0 = fmaf(ub3(lo), r[6], a0);
        a1 = fmaf(ub3(hi), r[7], a1);
    } else if constexpr (BITS == 2) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t b = (w >> (2 * t)) & 0x03030303u;  // codes t, 4+t, 8+t, 12+t
            a0 = fmaf(ub0(b), r[t], a0);
            a1 = fmaf(ub1(b), r[4 + t], a1);
            a0 = fmaf(ub2(b), r[8 + t], a0);
            a1 = fmaf(ub3(b), r[12 + t], a1);
        }
    } else if constexpr (BITS == 1) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t b = (w >> t) & 0x01010101u;  // codes t, 8+t, 16+t, 24+t
            a0 = fmaf(ub0(b), r[t], a0);
            a1 = fmaf(ub1(b), r[8 + t], a1);
            a0 = fmaf(ub2(b), r[16 + t], a0);
            a1 = fmaf(ub3(b), r[24 + t], a1);
        }
    } else {  // 32: the word is the float itself
        a0 = fmaf(__uint_as_float(w), r[0], a0);
    }
}

// ---------------------------------------------------------------------------
// Packed-code full pass on the integer dot instructions.  The residual comes
// in as fixed-point digits, one scale per 16-byte row chunk (written by the
// residual gather).  A lane holds the digit words of its chunks in registers
// and, per column, accumulates one dot instruction per digit per code word;
// a chunk's integer sums are exact, and the chunk's scale is applied in FP64:
//   g_j = sum_chunks 2^e (alpha sum_i k_ij N_i + beta sum_i N_i),
// with the column-independent part (the code offset and beta terms) summed
// once per workgroup.  The only approximation is r -> N 2^e (a relative
// 2^-22 of the chunk's largest |r_i|); g is rounded once, from FP64, to FP32.
// ---------------------------------------------------------------------------

// DPP moves of the two halves of a double (lanes the pattern does not feed
// read 0).
template <int CTRL, int RM, int BM>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, RM, BM, false),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, BM, false));
}

// Sum over the wave in a fixed order (row shifts, then row broadcasts), read
// from lane 63.
__device__ __forceinline__ double wave_total_f64(double v) {
    const double t = v;
    v = t + dpp_f64<0x111, 0xf, 0xf>(t);  // row_shr:1
    v = v + dpp_f64<0x112, 0xf, 0xf>(t);  // row_shr:2
    v = v + dpp_f64<0x113, 0xf, 0xf>(t);  // row_shr:3
    v = v + dpp_f64<0x114, 0xf, 0xe>(v);  // row_shr:4
    v = v + dpp_f64<0x118, 0xf, 0xc>(v);  // row_shr:8
    v = v + dpp_f64<0x142, 0xa, 0xf>(v);  // row_bcast:15
    v = v + dpp_f64<0x143, 0xc, 0xf>(v);  // row_bcast:31
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Codes of columns j, j + 4, ..., j + 4 (NCI - 1) at this lane's chunk
// offsets.  Every load is issued unconditionally (so that the next step's
// loads stay in flight while the current step is reduced): a column at or past
// c1 reads column c1 - 1 and is never stored, and the chunk offsets are
// clamped into the column, where a chunk past the column has zero weight.
template <int NCI, int CPL>
__device__ __forceinline__ void load_step(const uint8_t* q, int64_t col_bytes, int j, int c1,
                                          const uint32_t (&off)[CPL], uint4 (&v)[NCI][CPL]) {
#pragma unroll
    for (int k = 0; k < NCI; ++k) {
        const int jk = min(j + 4 * k, c1 - 1);
        const uint8_t* pc = q + static_cast<size_t>(jk) * col_bytes;
#pragma unroll
        for (int c = 0; c < CPL; ++c) v[k][c] = ldg_u4(pc + off[c]);
    }
}

// Per-workgroup constants of the step epilogue.
struct StepOut {
    double bsum;  // column-independent part of g for this slab
    int c0, c1, wbase;
    bool hist;
};

// Per-lane partial sums of one step: NCI columns j, j + 4, ... against the
// digit registers, with the chunk scales applied (this lane's share of g).
template <int BITS, int CPL, int NCI>
__device__ __forceinline__ void step_partials(const uint4 (&v)[NCI][CPL],
                                              const uint32_t (&dg)[CPL][4 * QDig<BITS>::H][QDig<BITS>::ND],
                                              const double (&ac)[CPL], double* col) {
    using D = QDig<BITS>;
    constexpr int ND = D::ND, H = D::H;
#pragma unroll
    for (int k = 0; k < NCI; ++k) col[k] = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        int acc[NCI][ND];
#pragma unroll
        for (int k = 0; k < NCI; ++k)
#pragma unroll
            for (int d = 0; d < ND; ++d) acc[k][d] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int k = 0; k < NCI; ++k) {
                    const uint32_t w = q == 0 ? v[k][c].x : q == 1 ? v[k][c].y : q == 2 ? v[k][c].z : v[k][c].w;
                    const uint32_t x = D::split(w, h);
#pragma unroll
                    for (int d = 0; d < ND; ++d) acc[k][d] = D::dot(x, dg[c][q * H + h][d], acc[k][d]);
                }
#pragma unroll
        for (int k = 0; k < NCI; ++k) {
            double t;
            if constexpr (BITS == 8)
                t = static_cast<double>(acc[k][0] + 256 * acc[k][1]) + 65536.0 * acc[k][2];
            else
                t = static_cast<double>(acc[k][0] + 16 * acc[k][1] + 256 * acc[k][2]) +
                    4096.0 * static_cast<double>(acc[k][3] + 16 * acc[k][4] + 256 * acc[k][5]);
            col[k] = fma(ac[c], t, col[k]);
        }
    }
}

// a + b after exchanging the upper 32 lanes of a with the lower 32 of b
// (lanes 0-31: a's pair sums over lanes l, l + 32; lanes 32-63: b's).
__device__ __forceinline__ double fold32(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// a + b after exchanging the odd 16-lane rows of a with the even rows of b
// (rows 0, 2: a's sums over lanes l, l + 16; rows 1, 3: b's).
__device__ __forceinline__ double fold16(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Wave sums of G = 2, 4 or 8 columns at once, by a butterfly that halves the
// live registers at each exchange: partners l ^ 32, l ^ 16, l ^ 8, then
// l ^ 1, l ^ 2, l ^ 4 within each group of 8 lanes.  Every column is summed
// in this same pairwise tree whatever G and its slot (FP addition is
// commutative), so g does not depend on the instance that computed it.
// On return every lane holds the total of slot gslot(lane).
template <int G>
__device__ __forceinline__ double wave_sums(const double (&p)[G]) {
    double v;
    if constexpr (G == 8) {
        const double r0 = fold16(fold32(p[0], p[1]), fold32(p[2], p[3]));  // rows: 0, 2, 1, 3
        const double r1 = fold16(fold32(p[4], p[5]), fold32(p[6], p[7]));  // rows: 4, 6, 5, 7
        const bool up = threadIdx.x & 8;  // lanes 8-15 of a row keep r1, 0-7 keep r0
        v = (up ? r1 : r0) + dpp_f64<0x128, 0xf, 0xf>(up ? r0 : r1);  // row_ror:8
    } else if constexpr (G == 4) {
        const double r = fold16(fold32(p[0], p[1]), fold32(p[2], p[3]));  // rows: 0, 2, 1, 3
        v = r + dpp_f64<0x128, 0xf, 0xf>(r);                              // row_ror:8
    } else {
        const double q = fold32(p[0], p[1]);
        const double r = fold16(q, q);  // rows: 0, 0, 1, 1
        v = r + dpp_f64<0x128, 0xf, 0xf>(r);
    }
    v = v + dpp_f64<0xB1, 0xf, 0xf>(v);   // quad_perm [1,0,3,2]
    v = v + dpp_f64<0x4E, 0xf, 0xf>(v);   // quad_perm [2,3,0,1]
    v = v + dpp_f64<0x141, 0xf, 0xf>(v);  // row_half_mirror
    return v;
}

// The slot whose total lane l holds after wave_sums<G>.
template <int G>
__device__ __forceinline__ int gslot(int l) {
    if constexpr (G == 8) {
        const int g = l >> 3;  // 8-lane group, slot = its 3 bits reversed
        return ((g & 1) << 2) | (g & 2) | (g >> 2);
    } else if constexpr (G == 4) {
        const int r = l >> 4;  // row, slot = its 2 bits reversed
        return ((r & 1) << 1) | (r >> 1);
    } else {
        return l >> 5;
    }
}

// The columns of one loop turn (slots 0..NCI-1: j, j + 4, ...; slots
// NCI..2 NCI - 1: j + step, j + step + 4, ...) summed over the wave, g into
// LDS after the 2048 histogram bins and, off the support, the histogram;
// one lane per column.
template <int NCI>
__device__ __forceinline__ void store_turn(const double (&p)[2 * NCI], int j, int step, const StepOut& so,
                                           uint32_t* lx, const uint32_t* lbm) {
    constexpr int G = 2 * NCI;
    const double t = wave_sums<G>(p);
    const int lane = threadIdx.x & 63;
    if ((lane & (64 / G - 1)) == 0) {
        const int sl = gslot<G>(lane);
        const int jk = j + (sl < NCI ? 4 * sl : step + 4 * (sl - NCI));
        if (jk < so.c1) {
            const float gv = static_cast<float>(t + so.bsum);
            lx[2048 + jk - so.c0] = __float_as_uint(gv);
            if (so.hist && !((lbm[(jk >> 5) - so.wbase] >> (jk & 31)) & 1u))
                atomicAdd(&lx[(__float_as_uint(gv) & 0x7FFFFFFFu) >> 20], 1u);
        }
    }
}

// LDS of a pass workgroup: lx[0, 2048) histogram bins, lx[2048, 2048 + c1 -
// c0) g of the task; lbm the support bitmap of the task's columns.
struct PassLds {
    uint32_t lx[2048 + kPassMaxCols];
    uint32_t lbm[kPassMaxCols / 32 + 2];
};

template <int BITS, int CPL, bool LONG>
__device__ __forceinline__ void pass_q_body(const ProbDev& pd, const Task& tk, PassLds& L, int done_now) {
    using D = QDig<BITS>;
    constexpr int RPC = 128 / BITS;  // rows per 16-byte chunk
    constexpr int ND = D::ND, H = D::H;
    // columns per step and wave: two when the codes stream from the Infinity
    // Cache (more bytes in flight per wave, two waves per SIMD); for long
    // streams from HBM (three waves per SIMD) four, two or one, so that every
    // wave keeps about 4 KB of a step in flight whatever the column height
    constexpr int NCI = LONG ? (CPL == 1 ? 4 : (CPL == 2 ? 2 : 1))
                             : ((CPL * 4 * H * ND >= 96 && BITS == 8) ? 1 : 2);
    constexpr int STEP = 4 * NCI;
    uint32_t* lx = L.lx;
    uint32_t* lbm = L.lbm;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int col_chunks = static_cast<int>(pd.col_bytes / 16);
    const int slab_chunk0 = tk.slab * 64 * CPL;
    (void)RPC;

    // ---- this lane's chunks: digit words, scales; then the first two steps
    int chk[CPL];
    uint32_t off[CPL];  // byte offsets of this lane's chunks in a column
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        chk[c] = slab_chunk0 + lane + 64 * c;
        off[c] = static_cast<uint32_t>(min(chk[c], col_chunks - 1)) * 16u;
    }
    const size_t dwords = static_cast<size_t>(col_chunks) * 4 * H;  // digit words per digit
    uint32_t dg[CPL][4 * H][ND];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const size_t w0 = static_cast<size_t>(min(chk[c], col_chunks - 1)) * 4 * H;
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int v4 = 0; v4 < H; ++v4) {
                const uint4 t = ldg_u4(pd.rdig + d * dwords + w0 + 4 * v4);
                dg[c][4 * v4 + 0][d] = t.x;
                dg[c][4 * v4 + 1][d] = t.y;
                dg[c][4 * v4 + 2][d] = t.z;
                dg[c][4 * v4 + 3][d] = t.w;
            }
    }
    int ex[CPL], sn[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int cc = min(chk[c], col_chunks - 1);
        ex[c] = static_cast<int>(ldg_u32(pd.rexp + cc));
        sn[c] = static_cast<int>(ldg_u32(pd.rsum + cc));
    }
    uint4 cur[NCI][CPL], nxt[NCI][CPL];
    load_step<NCI, CPL>(pd.q1, pd.col_bytes, tk.c0 + wv, tk.c1, off, cur);
    load_step<NCI, CPL>(pd.q1, pd.col_bytes, tk.c0 + wv + STEP, tk.c1, off, nxt);
    // the stop flag was read alongside these loads (every address stays valid
    // after the solve has stopped); uniform over the workgroup
    if (done_now) return;

    const bool hist = pd.nslab == 1;
    const int wbase = tk.c0 >> 5;
    if (hist) {
        for (int b = tid; b < 2048; b += kPassThreads) lx[b] = 0u;
        const int nwords = ((tk.c1 - 1) >> 5) - wbase + 1;
        for (int w = tid; w < nwords; w += kPassThreads) lbm[w] = ldg_u32(pd.bmsup + wbase + w);
    }
    // chunk weights: alpha 2^e on the code sums, and the slab's
    // column-independent part 2^e (alpha off + beta) sum_i N_i
    double ac[CPL];
    double bl = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const bool in = chk[c] < col_chunks;
        ac[c] = in ? ldexp(pd.alpha, ex[c]) : 0.0;
        bl += in ? ldexp((pd.alpha * D::CODE_OFF + pd.beta) * static_cast<double>(sn[c]), ex[c]) : 0.0;
    }
    const double bsum = wave_total_f64(bl);  // every wave holds all chunks of the slab
    __syncthreads();

    // Steady state, two buffers in turn: while one step is reduced the other
    // is in flight (a register copy between them would wait for both).
    const StepOut so{bsum, tk.c0, tk.c1, wbase, hist};
    // The wave sums of both steps are taken together (their registers are
    // free again before the second buffer is reloaded).
    for (int j = tk.c0 + wv; j < tk.c1; j += 2 * STEP) {
        double p[2 * NCI];
        step_partials<BITS, CPL, NCI>(cur, dg, ac, p);
        load_step<NCI, CPL>(pd.q1, pd.col_bytes, j + 2 * STEP, tk.c1, off, cur);
        step_partials<BITS, CPL, NCI>(nxt, dg, ac, p + NCI);
        store_turn<NCI>(p, j, STEP, so, lx, lbm);
        load_step<NCI, CPL>(pd.q1, pd.col_bytes, j + 3 * STEP, tk.c1, off, nxt);
    }
    // no global store inside the loop: a store under a branch would make the
    // compiler wait for the prefetched loads as well
    __syncthreads();
    float* out = (pd.nslab == 1) ? pd.g : pd.gpart + static_cast<size_t>(tk.slab) * pd.n;
    for (int i = tid; i < tk.c1 - tk.c0; i += kPassThreads) stg(out + tk.c0 + i, __uint_as_float(lx[2048 + i]));
    if (hist)
        for (int b = tid; b < 2048; b += kPassThreads)
            if (lx[b]) atomicAdd(&pd.hist[b], lx[b]);
}

// Span queue of a full-pass launch: workgroup w runs span w, then takes the
// next unclaimed span, spans [gridDim.x, ntasks) in order, with one atomic
// on qctr[0]; the last workgroup to finish sets both counters back to zero
// for the next launch.  (A one-round static split into equal bytes left a
// sixth of the batch pass's workgroup time idle at its end: workgroups of
// equal bytes ran 530-920 us, those on odd XCDs about 9% slower.)  Each
// column is still summed by one workgroup in one order, so g does not
// depend on which workgroup takes a span.
__device__ __forceinline__ int next_span(uint32_t* qctr, int* s_next) {
    __syncthreads();  // the span's LDS reads are done, and s_next is free
    if (threadIdx.x == 0) *s_next = static_cast<int>(gridDim.x + atomicAdd(qctr, 1u));
    __syncthreads();
    return *s_next;
}

__device__ __forceinline__ void finish_queue(uint32_t* qctr) {
    if (threadIdx.x == 0 && atomicAdd(qctr + 1, 1u) == gridDim.x - 1) {
        atomicExch(qctr, 0u);
        atomicExch(qctr + 1, 0u);
    }
}

// One launch over the spans of a batch: workgroup w runs span w, then the
// spans its `next` links name; each span carries the chunks per lane of its
// problem (small columns would leave most lanes idle at the batch's largest
// CPL), the body is picked per span.
// LONG: three workgroups per CU (except where the registers of 8-bit codes
// at 8 chunks per lane would spill), for code streams larger than the
// Infinity Cache.
template <int BITS, int CMAX, bool LONG>
__global__ __launch_bounds__(kPassThreads, (LONG && !(BITS == 8 && CMAX == 8)) ? 3 : 2) void k_fullpass_q(
    const ProbDev* __restrict__ P, const Task* __restrict__ tasks, int ntasks, uint32_t* qctr) {
    __shared__ PassLds L;
    __shared__ int s_next;
    const bool queue = ntasks > static_cast<int>(gridDim.x);
    for (int t = blockIdx.x; t < ntasks;) {
        const Task tk = tasks[t];
        const ProbDev& pd = P[tk.p];
        const int dn = ldg_i32(&pd.st->done);  // checked inside, once the first loads are issued
        switch (tk.cpl) {
            case 1: pass_q_body<BITS, 1, LONG>(pd, tk, L, dn); break;
            case 2: if constexpr (CMAX >= 2) pass_q_body<BITS, 2, LONG>(pd, tk, L, dn); break;
            case 3: if constexpr (CMAX >= 4) pass_q_body<BITS, 3, LONG>(pd, tk, L, dn); break;
            case 4: if constexpr (CMAX >= 4) pass_q_body<BITS, 4, LONG>(pd, tk, L, dn); break;
            default: if constexpr (CMAX >= 8) pass_q_body<BITS, 8, LONG>(pd, tk, L, dn); break;
        }
        if (!queue) break;
        t = next_span(qctr, &s_next);
    }
    if (queue) finish_queue(qctr);
}

// ---------------------------------------------------------------------------
// FP32 full pass g = Q1^T r (32-bit "codes" are the floats themselves).  One
// wave per column: lane l owns the 16-byte chunks l, l + 64, ..., l + 64
// (CPL - 1) of its row slab and keeps the matching residual rows in registers
// for every column it visits; each column is reduced across the wave.
// ---------------------------------------------------------------------------
template <int BITS, int CPL>
__device__ __forceinline__ void pass_f_body(const ProbDev& pd, const Task& tk, PassLds& L) {
    constexpr int RPC = (BITS == 32) ? 4 : 128 / BITS;  // rows per chunk
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col_chunks = static_cast<int>(pd.col_bytes / 16);
    const int chunk0 = tk.slab * 64 * CPL + lane;

    float rr[CPL][RPC];
    bool ok[CPL];
    double sr = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int ch = chunk0 + 64 * c;
        ok[c] = ch < col_chunks;
        const float* src = pd.r32 + static_cast<size_t>(ch) * RPC;
#pragma unroll
        for (int q4 = 0; q4 < RPC / 4; ++q4) {
            const uint4 u = ok[c] ? ldg_u4(src + 4 * q4) : make_uint4(0u, 0u, 0u, 0u);
            const float4 v = make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z),
                                         __uint_as_float(u.w));
            rr[c][4 * q4 + 0] = v.x;
            rr[c][4 * q4 + 1] = v.y;
            rr[c][4 * q4 + 2] = v.z;
            rr[c][4 * q4 + 3] = v.w;
            sr += static_cast<double>(v.x) + static_cast<double>(v.y) +
                  static_cast<double>(v.z) + static_cast<double>(v.w);
        }
    }
    const float bsum = static_cast<float>(pd.beta * wave_sum(sr));
    float* out = (pd.nslab == 1) ? pd.g : pd.gpart + static_cast<size_t>(tk.slab) * pd.n;
    // Histogram of the top 11 bits of |g_j| (exponent and 3 mantissa bits)
    // over the entries off the current support, for the threshold search of
    // the H_s proposals; built where g is final.
    const bool hist = pd.nslab == 1;
    uint32_t* lh = L.lx;    // histogram bins
    uint32_t* lbm = L.lbm;  // support bitmap of this task's columns
    const int wbase = tk.c0 >> 5;
    if (hist) {
        for (int b = threadIdx.x; b < 2048; b += kPassThreads) lh[b] = 0u;
        const int nwords = ((tk.c1 - 1) >> 5) - wbase + 1;
        for (int w = threadIdx.x; w < nwords; w += kPassThreads) lbm[w] = ldg_u32(pd.bmsup + wbase + w);
        __syncthreads();
    }
    const uint8_t* base = pd.q1 + static_cast<size_t>(chunk0) * 16;

    for (int j = tk.c0 + wv; j < tk.c1; j += 8) {
        const int j2 = j + 4;
        const bool has2 = j2 < tk.c1;
        float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
        const uint8_t* pa = base + static_cast<size_t>(j) * pd.col_bytes;
        const uint8_t* pb = base + static_cast<size_t>(has2 ? j2 : j) * pd.col_bytes;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            constexpr int RW = RPC / 4;  // rows per 32-bit word
            const size_t oc = static_cast<size_t>(64 * c) * 16;
            const uint4 va = ok[c] ? ldg_u4(pa + oc) : make_uint4(0u, 0u, 0u, 0u);
            const uint4 vb = (ok[c] && has2) ? ldg_u4(pb + oc) : make_uint4(0u, 0u, 0u, 0u);
            dot_word<BITS>(va.x, &rr[c][0 * RW], a0, a1);
            dot_word<BITS>(va.y, &rr[c][1 * RW], a0, a1);
            dot_word<BITS>(va.z, &rr[c][2 * RW], a0, a1);
            dot_word<BITS>(va.w, &rr[c][3 * RW], a0, a1);
            dot_word<BITS>(vb.x, &rr[c][0 * RW], b0, b1);
            dot_word<BITS>(vb.y, &rr[c][1 * RW], b0, b1);
            dot_word<BITS>(vb.z, &rr[c][2 * RW], b0, b1);
            dot_word<BITS>(vb.w, &rr[c][3 * RW], b0, b1);
        }
        const float sa = wave_sum(a0 + a1);
        const float sb = wave_sum(b0 + b1);
        if (lane == 0) {
            const float ga = (BITS == 32) ? sa : fmaf(pd.alpha_f, sa, bsum);
            stg(out + j, ga);
            if (hist && !((lbm[(j >> 5) - wbase] >> (j & 31)) & 1u))
                atomicAdd(&lh[(__float_as_uint(ga) & 0x7FFFFFFFu) >> 20], 1u);
            if (has2) {
                const float gb = (BITS == 32) ? sb : fmaf(pd.alpha_f, sb, bsum);
                stg(out + j2, gb);
                if (hist && !((lbm[(j2 >> 5) - wbase] >> (j2 & 31)) & 1u))
                    atomicAdd(&lh[(__float_as_uint(gb) & 0x7FFFFFFFu) >> 20], 1u);
            }
        }
    }
    if (hist) {
        __syncthreads();
        for (int b = threadIdx.x; b < 2048; b += kPassThreads)
            if (lh[b]) atomicAdd(&pd.hist[b], lh[b]);
    }
}

template <int BITS, int CMAX>
__global__ __launch_bounds__(kPassThreads) void k_fullpass(
    const ProbDev* __restrict__ P, const Task* __restrict__ tasks, int ntasks, uint32_t* qctr) {
    __shared__ PassLds L;
    __shared__ int s_next;
    const bool queue = ntasks > static_cast<int>(gridDim.x);
    for (int t = blockIdx.x; t < ntasks;) {
        const Task tk = tasks[t];
        const ProbDev& pd = P[tk.p];
        if (!ldg_i32(&pd.st->done)) {  // uniform over the workgroup
            switch (tk.cpl) {
                case 1: pass_f_body<BITS, 1>(pd, tk, L); break;
                case 2: if constexpr (CMAX >= 2) pass_f_body<BITS, 2>(pd, tk, L); break;
                case 4: if constexpr (CMAX >= 4) pass_f_body<BITS, 4>(pd, tk, L); break;
                case 8: if constexpr (CMAX >= 8) pass_f_body<BITS, 8>(pd, tk, L); break;
                default: if constexpr (CMAX >= 16) pass_f_body<BITS, 16>(pd, tk, L); break;
            }
        }
        if (!queue) break;
        t = next_span(qctr, &s_next);
    }
    if (queue) finish_queue(qctr);
}

// g of columns split into row slabs: the slab partials summed in slab order
// (FP32), and the |g| histogram off the support.  Workgroup x takes
// columns [x kSlabCols, (x + 1) kSlabCols) of its problem; the histogram is
// counted in LDS and merged with one global atomic per non-empty bin (a
// global atomic per column made this kernel take a third of an FP32 pass).
constexpr int kSlabCols = 1024;

__global__ __launch_bounds__(256) void k_slab_reduce(const ProbDev* __restrict__ P) {
    const ProbDev& pd = P[blockIdx.y];
    __shared__ uint32_t lh[2048];
    const int j0 = blockIdx.x * kSlabCols;
    if (pd.st->done || pd.nslab <= 1 || j0 >= pd.n) return;  // uniform over the workgroup
    for (int b = threadIdx.x; b < 2048; b += 256) lh[b] = 0u;
    __syncthreads();
    const int j1 = min(pd.n, j0 + kSlabCols);
    for (int j = j0 + threadIdx.x; j < j1; j += 256) {
        float s = 0.f;
        for (int sl = 0; sl < pd.nslab; ++sl) s += pd.gpart[static_cast<size_t>(sl) * pd.n + j];
        pd.g[j] = s;
        if (!((pd.bmsup[j >> 5] >> (j & 31)) & 1u))
            atomicAdd(&lh[(__float_as_uint(s) & 0x7FFFFFFFu) >> 20], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2048; b += 256)
        if (lh[b]) atomicAdd(&pd.hist[b], lh[b]);
}

template <typename K>
void launch_k(K kern, int nwg, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, const ProbDev* P,
              const Task* T, int ntasks) {
    // the queue counters follow the task list
    uint32_t* qctr = reinterpret_cast<uint32_t*>(const_cast<Task*>(T) + ntasks);
    if (ev0)
        hipExtLaunchKernelGGL(kern, dim3(nwg), dim3(kPassThreads), 0, st, ev0, ev1, 0, P, T, ntasks, qctr);
    else
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(kPassThreads), 0, st, P, T, ntasks, qctr);
}

template <int BITS, bool LONG>
void launch_pass_b(int cpl, const ProbDev* P, const Task* T, int nwg, int ntasks, hipStream_t st,
                   hipEvent_t ev0, hipEvent_t ev1) {
    switch (cpl) {
#define QIHT_PASS_CASE(C)                                                                   \
    case C:                                                                                 \
        if constexpr (C <= (BITS == 32 ? 16 : BITS)) {                                      \
            if constexpr (BITS == 32)                                                       \
                launch_k(k_fullpass<BITS, C>, nwg, st, ev0, ev1, P, T, ntasks);                     \
            else                                                                            \
                launch_k(k_fullpass_q<BITS, C, LONG>, nwg, st, ev0, ev1, P, T, ntasks);                \
        }                                                                                   \
        break;
        QIHT_PASS_CASE(1)
        QIHT_PASS_CASE(2)
        QIHT_PASS_CASE(4)
        QIHT_PASS_CASE(8)
        QIHT_PASS_CASE(16)
#undef QIHT_PASS_CASE
        default: break;
    }
}

template <int BITS, bool LONG>
int pass_blocks_b(int cpl) {
    int nb = 0;
    hipError_t err = hipSuccess;
    switch (cpl) {
#define QIHT_OCC_CASE(C)                                                                        \
    case C:                                                                                     \
        if constexpr (C <= (BITS == 32 ? 16 : BITS)) {                                          \
            if constexpr (BITS == 32)                                                           \
                err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fullpass<BITS, C>,    \
                                                                   kPassThreads, 0);            \
            else                                                                                \
                err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fullpass_q<BITS, C, LONG>, \
                                                                   kPassThreads, 0);            \
        }                                                                                       \
        break;
        QIHT_OCC_CASE(1)
        QIHT_OCC_CASE(2)
        QIHT_OCC_CASE(4)
        QIHT_OCC_CASE(8)
        QIHT_OCC_CASE(16)
#undef QIHT_OCC_CASE
        default: break;
    }
    return err == hipSuccess ? nb : 0;
}

}  // namespace

int pass_slots(int bits, int cpl, bool long_stream) {
    int dev = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    switch (bits) {
        case 1: nb = long_stream ? pass_blocks_b<1, true>(cpl) : pass_blocks_b<1, false>(cpl); break;
        case 2: nb = long_stream ? pass_blocks_b<2, true>(cpl) : pass_blocks_b<2, false>(cpl); break;
        case 4: nb = long_stream ? pass_blocks_b<4, true>(cpl) : pass_blocks_b<4, false>(cpl); break;
        case 8: nb = long_stream ? pass_blocks_b<8, true>(cpl) : pass_blocks_b<8, false>(cpl); break;
        default: nb = pass_blocks_b<32, false>(cpl); break;
    }
    return nb * cus;
}

void launch_pass(int bits, int cpl, bool long_stream, const ProbDev* P, const Task* T, int nwg,
                 int ntasks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
#define QIHT_LP(B)                                                                   \
    (long_stream ? launch_pass_b<B, true>(cpl, P, T, nwg, ntasks, st, ev0, ev1)      \
                 : launch_pass_b<B, false>(cpl, P, T, nwg, ntasks, st, ev0, ev1))
    switch (bits) {
        case 1: QIHT_LP(1); break;
        case 2: QIHT_LP(2); break;
        case 4: QIHT_LP(4); break;
        case 8: QIHT_LP(8); break;
        default: launch_pass_b<32, false>(cpl, P, T, nwg, ntasks, st, ev0, ev1); break;
    }
#undef QIHT_LP
}

void launch_slab_reduce(const ProbDev* P, int count, int max_n, hipStream_t st) {
    hipLaunchKernelGGL(k_slab_reduce, dim3((max_n + kSlabCols - 1) / kSlabCols, count), dim3(256), 0, st, P);
}

}  // namespace qiht
