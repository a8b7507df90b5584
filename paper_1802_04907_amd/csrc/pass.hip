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
// Full pass g = Q1^T r.  One wave per column: lane l owns the 16-byte chunks
// l, l + 64, ..., l + 64 (CPL - 1) of its row slab and keeps the matching
// residual rows in registers for every column it visits; each column is
// reduced across the wave.  Affine dequantization is folded out of the loop:
// g_j = alpha * sum_i code_ij r_i + beta * sum_i r_i.
// ---------------------------------------------------------------------------
template <int BITS, int CPL>
__global__ __launch_bounds__(kPassThreads) void k_fullpass(
    const ProbDev* __restrict__ P, const Task* __restrict__ tasks) {
    constexpr int RPC = (BITS == 32) ? 4 : 128 / BITS;  // rows per chunk
    const Task tk = tasks[blockIdx.x];
    const ProbDev& pd = P[tk.p];
    if (pd.st->done) return;
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
        const float4* src = reinterpret_cast<const float4*>(pd.r32 + static_cast<size_t>(ch) * RPC);
#pragma unroll
        for (int q4 = 0; q4 < RPC / 4; ++q4) {
            const float4 v = ok[c] ? src[q4] : make_float4(0.f, 0.f, 0.f, 0.f);
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
    __shared__ uint32_t lh[2048];
    __shared__ uint32_t lbm[kPassMaxCols / 32 + 2];  // support bitmap of this task's columns
    const int wbase = tk.c0 >> 5;
    if (hist) {
        for (int b = threadIdx.x; b < 2048; b += kPassThreads) lh[b] = 0u;
        const int nwords = ((tk.c1 - 1) >> 5) - wbase + 1;
        for (int w = threadIdx.x; w < nwords; w += kPassThreads) lbm[w] = pd.bmsup[wbase + w];
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
            const uint4 va = ok[c] ? *reinterpret_cast<const uint4*>(pa + oc) : make_uint4(0u, 0u, 0u, 0u);
            const uint4 vb = (ok[c] && has2) ? *reinterpret_cast<const uint4*>(pb + oc)
                                             : make_uint4(0u, 0u, 0u, 0u);
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
            out[j] = ga;
            if (hist && !((lbm[(j >> 5) - wbase] >> (j & 31)) & 1u))
                atomicAdd(&lh[(__float_as_uint(ga) & 0x7FFFFFFFu) >> 20], 1u);
            if (has2) {
                const float gb = (BITS == 32) ? sb : fmaf(pd.alpha_f, sb, bsum);
                out[j2] = gb;
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

__global__ __launch_bounds__(256) void k_slab_reduce(const ProbDev* __restrict__ P) {
    const ProbDev& pd = P[blockIdx.y];
    if (pd.st->done || pd.nslab <= 1) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < pd.n; j += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int sl = 0; sl < pd.nslab; ++sl) s += pd.gpart[static_cast<size_t>(sl) * pd.n + j];
        pd.g[j] = s;
        if (!((pd.bmsup[j >> 5] >> (j & 31)) & 1u))
            atomicAdd(&pd.hist[(__float_as_uint(s) & 0x7FFFFFFFu) >> 20], 1u);
    }
}

template <int BITS>
void launch_pass_b(int cpl, const ProbDev* P, const Task* T, int ntasks, hipStream_t st,
                   hipEvent_t ev0, hipEvent_t ev1) {
    switch (cpl) {
#define QIHT_PASS_CASE(C)                                                                   \
    case C:                                                                                 \
        if constexpr (C <= (BITS == 32 ? 16 : BITS)) {                                      \
            if (ev0)                                                                        \
                hipExtLaunchKernelGGL((k_fullpass<BITS, C>), dim3(ntasks), dim3(kPassThreads), \
                                      0, st, ev0, ev1, 0, P, T);                            \
            else                                                                            \
                hipLaunchKernelGGL((k_fullpass<BITS, C>), dim3(ntasks), dim3(kPassThreads), \
                                   0, st, P, T);                                            \
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

}  // namespace

void launch_pass(int bits, int cpl, const ProbDev* P, const Task* T, int ntasks, hipStream_t st,
                 hipEvent_t ev0, hipEvent_t ev1) {
    switch (bits) {
        case 1: launch_pass_b<1>(cpl, P, T, ntasks, st, ev0, ev1); break;
        case 2: launch_pass_b<2>(cpl, P, T, ntasks, st, ev0, ev1); break;
        case 4: launch_pass_b<4>(cpl, P, T, ntasks, st, ev0, ev1); break;
        case 8: launch_pass_b<8>(cpl, P, T, ntasks, st, ev0, ev1); break;
        default: launch_pass_b<32>(cpl, P, T, ntasks, st, ev0, ev1); break;
    }
}

void launch_slab_reduce(const ProbDev* P, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_slab_reduce, dim3(64, count), dim3(256), 0, st, P);
}

}  // namespace qiht
