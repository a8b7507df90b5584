// QIHT iteration on the GPU (Algorithm 2 of the paper, on fixed
// realizations Q1 for Phi^T and Q2 for Phi).
//
// One iteration is a short, fixed sequence of launches on one stream; all
// control state (current support, step size, backtracking phase, stop flag)
// lives in device memory, so the host never waits inside the loop:
//
//   k_gather<R>      r = y_hat - Q2_G x_G        FP64 accumulation, FP32 out
//   k_fullpass       g = Q1^T r                  the bandwidth-bound pass
//   k_gather<MU>     u = Q1_G g_G, v = Q2_G g_G  -> mu (Eq. step_size)
//   k_select         x' = H_s(x + mu g), support compare, |dx|, |x'|
//   k_gather<OMEGA>  w = Q1 dx                   -> omega, step test
//   k_backtrack      rare path: shrink mu, reselect, retest (one workgroup)
//
// Every kernel first reads the per-problem state and returns at once when
// the problem is finished or the phase does not concern it, so a batch of
// problems of different sizes runs through the same launches.
// Reductions use fixed orders only (no floating-point atomics): two runs
// give bitwise identical results.
#include <algorithm>
#include <cstring>
#include <vector>

#include "qiht_internal.h"

namespace qiht {
namespace {

constexpr int kSelectThreads = 1024;
constexpr int kGatherThreads = 1024;
constexpr int kPassThreads = 256;

struct SolveState {
    int32_t cur;       // which of the two x / support buffers is current
    int32_t done;
    int32_t iter;      // completed iterations
    int32_t reason;
    int32_t phase;     // 0 idle, 1 omega pending, 2 backtracking pending
    int32_t nb;        // shrinks in this iteration
    int32_t total_bt;
    int32_t capped;
    int32_t dcount;    // length of the dx list
    int32_t err;       // 1 = NaN met in a selection
    int32_t pad0, pad1;
    double mu;
    double mu_last;
    double dx2;        // |x' - x|^2 of the current proposal
    double xn2;        // |x'|^2
};

struct ProbDev {
    const uint8_t* q1;
    const uint8_t* q2;
    int64_t col_bytes;
    int32_t rows;
    int32_t n;
    int32_t s;
    int32_t nrb;       // gather row blocks = col_bytes / 256
    int32_t nslab;     // full-pass row slabs
    int32_t pad;
    double alpha;      // dequantized value = alpha * code + beta
    double beta;
    float alpha_f;
    float pad_f;
    const double* yhat;
    float* r32;        // rows_pad
    float* g;          // n
    float* gpart;      // nslab * n (only if nslab > 1)
    float* xb[2];      // dense x, n each
    int32_t* sb[2];    // supports, s each
    int32_t* dlist;    // indices where the proposal differs from x
    double* dw;        // and the differences
    double* part;      // 2 * nrb gather partial sums
    unsigned* counter; // last-block counters, one per gather mode
    SolveState* st;
};

struct Task {
    int32_t p, slab, c0, c1;
};

enum { G_R = 0, G_MU = 1, G_OMEGA = 2 };
enum { SEL_RAW = 0, SEL_INIT = 1, SEL_STEP = 2 };

// ---------------------------------------------------------------------------
// Small block-level helpers (fixed reduction orders).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a block of `NT` threads; every thread gets the result.
template <int NT>
__device__ double block_sum(double v, double* sh) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Exclusive prefix sum over a block of `NT` threads (thread order).
template <int NT>
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t t = sh[w];
        if (w < wv) before += t;
        all += t;
    }
    __syncthreads();
    if (total) *total = all;
    return before + x - v;
}

__device__ void commit(SolveState* st, const SolveArgs& a) {
    st->cur ^= 1;
    st->iter += 1;
    st->mu_last = st->mu;
    st->total_bt += st->nb;
    st->phase = 0;
    if (a.tol >= 0.0 && st->dx2 <= a.tol * a.tol * st->xn2) {
        st->done = 1;
        st->reason = QIHT_REASON_CONVERGED;
    } else if (st->iter >= a.max_iters) {
        st->done = 1;
        st->reason = QIHT_REASON_MAX_ITERS;
    }
}

// ---------------------------------------------------------------------------
// Code unpacking.  A 32-bit word holds 32/BITS codes, code q at bit q*BITS.
// ---------------------------------------------------------------------------
template <int BITS>
__device__ __forceinline__ uint32_t code_at(uint32_t w, int q) {
    return (w >> (q * BITS)) & ((1u << BITS) - 1u);
}

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
// Column gathers: out_i = sum_t w_t * Qhat(i, col_t) for the rows of one
// 256-byte row block, FP64 accumulation.  Lanes own one 32-bit word of the
// block (coalesced across the wave); the 16 waves split the column list and
// are combined in LDS in wave order.
// ---------------------------------------------------------------------------
template <int BITS, int MODE>
__global__ __launch_bounds__(kGatherThreads) void k_gather(
    const ProbDev* __restrict__ P, SolveArgs a, int zero_x) {
    constexpr int RPW = (BITS == 32) ? 1 : 32 / BITS;
    constexpr int NM = (MODE == G_MU) ? 2 : 1;
    constexpr int CHM = (NM == 2) ? 2 : 4;
    constexpr int CH = RPW < CHM ? RPW : CHM;
    const ProbDev& pd = P[blockIdx.y];
    SolveState* st = pd.st;
    if (st->done) return;
    if (MODE == G_OMEGA && st->phase != 1) return;
    const int rb = blockIdx.x;
    if (rb >= pd.nrb) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cur = st->cur;
    const bool two = (MODE == G_MU) && (a.mu_mode == 0);

    const int32_t* cols;
    int ncols;
    if (MODE == G_OMEGA) {
        cols = pd.dlist;
        ncols = st->dcount;
    } else {
        cols = pd.sb[cur];
        ncols = (MODE == G_R && zero_x) ? 0 : pd.s;
    }
    const uint8_t* A = (MODE == G_R) ? pd.q2 : pd.q1;
    const uint8_t* B = pd.q2;
    const float* wsrc = (MODE == G_R) ? pd.xb[cur] : pd.g;
    const size_t woff = (static_cast<size_t>(rb) * 64 + lane) * 4;

    double acc[NM][RPW];
#pragma unroll
    for (int mi = 0; mi < NM; ++mi)
#pragma unroll
        for (int q = 0; q < RPW; ++q) acc[mi][q] = 0.0;
    double wsum = 0.0;

    constexpr int U = 8;
    for (int t0 = wv; t0 < ncols; t0 += 16 * U) {
        int cidx[U];
        double wt[U];
        uint32_t wa[U], wb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + 16 * u;
            cidx[u] = t < ncols ? cols[t] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + 16 * u;
            if (cidx[u] >= 0) {
                wt[u] = (MODE == G_OMEGA) ? pd.dw[t] : static_cast<double>(wsrc[cidx[u]]);
                const size_t off = static_cast<size_t>(cidx[u]) * pd.col_bytes + woff;
                wa[u] = *reinterpret_cast<const uint32_t*>(A + off);
                wb[u] = two ? *reinterpret_cast<const uint32_t*>(B + off) : 0u;
            } else {
                wt[u] = 0.0;
                wa[u] = 0u;
                wb[u] = 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (cidx[u] < 0) continue;
            wsum += wt[u];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const double va = (BITS == 32) ? static_cast<double>(__uint_as_float(wa[u]))
                                               : static_cast<double>(code_at<BITS>(wa[u], q));
                acc[0][q] = fma(wt[u], va, acc[0][q]);
                if (NM == 2) {
                    const double vb = (BITS == 32) ? static_cast<double>(__uint_as_float(wb[u]))
                                                   : static_cast<double>(code_at<BITS>(wb[u], q));
                    acc[NM - 1][q] = fma(wt[u], vb, acc[NM - 1][q]);
                }
            }
        }
    }

    __shared__ double sh[NM][16][CH][64];
    __shared__ double shw[16];
    __shared__ double shr[16];
    __shared__ int sh_last;
    if (lane == 0) shw[wv] = wsum;
    __syncthreads();
    double wtot = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) wtot += shw[w];

    double l1 = 0.0, l2 = 0.0;  // per-thread partial dot products
    for (int q0 = 0; q0 < RPW; q0 += CH) {
#pragma unroll
        for (int mi = 0; mi < NM; ++mi)
#pragma unroll
            for (int qq = 0; qq < CH; ++qq) sh[mi][wv][qq][lane] = acc[mi][q0 + qq];
        __syncthreads();
        if (threadIdx.x < 64 * CH) {
            const int qq = threadIdx.x >> 6, ln = threadIdx.x & 63;
            double tot[NM];
#pragma unroll
            for (int mi = 0; mi < NM; ++mi) {
                tot[mi] = 0.0;
#pragma unroll
                for (int w = 0; w < 16; ++w) tot[mi] += sh[mi][w][qq][ln];
            }
            const int64_t row = (static_cast<int64_t>(rb) * 64 + ln) * RPW + q0 + qq;
            double val[NM];
#pragma unroll
            for (int mi = 0; mi < NM; ++mi)
                val[mi] = (BITS == 32) ? tot[mi] : pd.alpha * tot[mi] + pd.beta * wtot;
            const bool live = row < pd.rows;
            if (MODE == G_R) {
                pd.r32[row] = live ? static_cast<float>(pd.yhat[row] - val[0]) : 0.0f;
            } else if (MODE == G_MU) {
                if (live) {
                    l2 += val[0] * val[0];
                    l1 += two ? val[0] * val[NM - 1] : val[0] * val[0];
                }
            } else {
                if (live) l1 += val[0] * val[0];
            }
        }
        __syncthreads();
    }
    if (MODE == G_R) return;

    const double s1 = block_sum<kGatherThreads>(l1, shr);
    const double s2 = (MODE == G_MU) ? block_sum<kGatherThreads>(l2, shr) : 0.0;
    if (threadIdx.x == 0) {
        pd.part[rb] = s1;
        pd.part[pd.nrb + rb] = s2;
        __threadfence();
        const unsigned prev = atomicAdd(&pd.counter[MODE], 1u);
        sh_last = (prev == static_cast<unsigned>(pd.nrb - 1));
    }
    __syncthreads();
    if (!sh_last) return;
    __threadfence();

    // Last block of this problem: finish the reduction in row-block order.
    if (MODE == G_MU) {
        double gg = 0.0;
        for (int t = threadIdx.x; t < pd.s; t += kGatherThreads) {
            const double v = static_cast<double>(pd.g[pd.sb[cur][t]]);
            gg += v * v;
        }
        const double num = block_sum<kGatherThreads>(gg, shr);
        if (threadIdx.x == 0) {
            double uv = 0.0, uu = 0.0;
            for (int b = 0; b < pd.nrb; ++b) {
                uv += pd.part[b];
                uu += pd.part[pd.nrb + b];
            }
            double den = uv;
            if (!(den > 0.0) || !isfinite(den)) den = uu;
            pd.counter[MODE] = 0u;
            if (!(num > 0.0) || !(den > 0.0) || !isfinite(num / den)) {
                st->done = 1;
                st->reason = QIHT_REASON_STATIONARY;
            } else {
                st->mu = num / den;
                st->nb = 0;
                st->phase = 0;
            }
        }
    } else {
        if (threadIdx.x == 0) {
            double ww = 0.0;
            for (int b = 0; b < pd.nrb; ++b) ww += pd.part[b];
            pd.counter[MODE] = 0u;
            const double omega = ww > 0.0 ? st->dx2 / ww : INFINITY;
            if (st->mu <= (1.0 - a.c) * omega) {
                commit(st, a);
            } else {
                st->phase = 2;
            }
        }
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
            out[j] = (BITS == 32) ? sa : fmaf(pd.alpha_f, sa, bsum);
            if (has2) out[j2] = (BITS == 32) ? sb : fmaf(pd.alpha_f, sb, bsum);
        }
    }
}

__global__ void k_slab_reduce(const ProbDev* __restrict__ P) {
    const ProbDev& pd = P[blockIdx.y];
    if (pd.st->done || pd.nslab <= 1) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < pd.n; j += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int sl = 0; sl < pd.nslab; ++sl) s += pd.gpart[static_cast<size_t>(sl) * pd.n + j];
        pd.g[j] = s;
    }
}

// ---------------------------------------------------------------------------
// Top-s selection (H_s) in one workgroup: exact radix select of the s-th
// largest |a| (31-bit keys, digits 11/10/10 bits, histograms in LDS), then an
// order-preserving compaction, so the support comes out ascending and ties
// at the threshold go to the lowest indices.  Thread t owns the contiguous
// index range [t*CPT, t*CPT + CPT).
// ---------------------------------------------------------------------------
struct SelShared {
    uint32_t hist[2048];
    uint32_t scan[16];
    uint32_t bin, krem;
    int changed;
    double red[16];
};

struct SelOut {
    bool changed;
    double dx2, xn2;
    int dcount;
};

template <int CPT>
__device__ __forceinline__ uint32_t key_of(float v) {
    return __float_as_uint(v) & 0x7FFFFFFFu;
}

template <int CPT>
__device__ SelOut select_core(int mode, int n, int s, const float* a_in,
                              const float* g, const float* x, float muf,
                              const int32_t* old_sup, int32_t* out_sup,
                              float* x_out, int32_t* dlist, double* dw,
                              SelShared& S, int* err) {
    static_assert(CPT <= 64, "selection bitmask holds 64 entries");
    const int t = threadIdx.x;
    const int j0 = t * CPT;
    float av[CPT];
    int bad = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = j0 + e;
        float v = 0.f;
        if (j < n) {
            if (mode == SEL_RAW) v = a_in[j];
            else if (mode == SEL_INIT) v = g[j];
            else v = fmaf(muf, g[j], x[j]);
            if (key_of<CPT>(v) > 0x7F800000u) bad = 1;
        }
        av[e] = v;
    }
    if (bad) atomicOr(err, 1);

    // ---- radix select: threshold key T and the number of ties to take ----
    uint32_t prefix = 0, krem = static_cast<uint32_t>(s);
#pragma unroll
    for (int pass = 0; pass < 3; ++pass) {
        // digits: bits 30..20 (2048 bins), 19..10 and 9..0 (1024 bins each)
        const int width = pass == 0 ? 11 : 10;
        const int sh = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
        const int nb = 1 << width;
        for (int b = t; b < 2048; b += kSelectThreads) S.hist[b] = 0u;
        __syncthreads();
        const int hsh = sh + width;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const uint32_t k = key_of<CPT>(av[e]);
            if (j0 + e < n && (pass == 0 || (k >> hsh) == prefix))
                atomicAdd(&S.hist[(k >> sh) & (nb - 1)], 1u);
        }
        __syncthreads();
        // Bins in descending order; thread t handles PB consecutive bins.
        const int PB = nb / kSelectThreads;  // 2 or 1
        uint32_t cnt[2] = {0u, 0u};
        uint32_t mine = 0;
        for (int i = 0; i < PB; ++i) {
            cnt[i] = S.hist[nb - 1 - (t * PB + i)];
            mine += cnt[i];
        }
        const uint32_t above = block_excl_scan<kSelectThreads>(mine, S.scan, nullptr);
        uint32_t run = above;
        for (int i = 0; i < PB; ++i) {
            if (krem > 0 && run < krem && krem <= run + cnt[i]) {
                S.bin = static_cast<uint32_t>(nb - 1 - (t * PB + i));
                S.krem = krem - run;
            }
            run += cnt[i];
        }
        __syncthreads();
        if (krem > 0) {
            prefix = (prefix << width) | S.bin;
            krem = S.krem;
        }
        __syncthreads();
    }
    const uint32_t T = prefix;      // exact s-th largest key (if s > 0)
    const uint32_t need = krem;     // how many keys equal to T are taken

    // ---- ordered compaction ----
    uint32_t gt = 0, eq = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const uint32_t k = key_of<CPT>(av[e]);
        if (j0 + e < n && s > 0) {
            gt += k > T;
            eq += k == T;
        }
    }
    const uint32_t eq_before = block_excl_scan<kSelectThreads>(eq, S.scan, nullptr);
    uint32_t my_ties = 0;
    if (need > eq_before) my_ties = min(eq, need - eq_before);
    uint32_t pos = block_excl_scan<kSelectThreads>(gt + my_ties, S.scan, nullptr);

    if (t == 0) S.changed = 0;
    __syncthreads();
    uint64_t selmask = 0;
    uint32_t ties_taken = 0;
    int changed = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = j0 + e;
        const uint32_t k = key_of<CPT>(av[e]);
        bool take = false;
        if (j < n && s > 0) {
            if (k > T) take = true;
            else if (k == T && ties_taken < my_ties) {
                take = true;
                ++ties_taken;
            }
        }
        if (take) {
            selmask |= (1ull << e);
            if (pos < static_cast<uint32_t>(s)) {
                out_sup[pos] = j;
                if (old_sup && old_sup[pos] != j) changed = 1;
            }
            ++pos;
        }
    }
    if (changed) S.changed = 1;

    SelOut res{false, 0.0, 0.0, 0};
    if (mode != SEL_STEP) {
        __syncthreads();
        return res;
    }
    // ---- proposal x', |x' - x|^2, |x'|^2, list of changed entries ----
    double dx2 = 0.0, xn2 = 0.0;
    uint32_t ndiff = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = j0 + e;
        if (j < n) {
            const float xo = x[j];
            const float xn = ((selmask >> e) & 1ull) ? av[e] : 0.f;
            x_out[j] = xn;
            const double d = static_cast<double>(xn) - static_cast<double>(xo);
            dx2 += d * d;
            xn2 += static_cast<double>(xn) * static_cast<double>(xn);
            ndiff += (xn != xo);
        }
    }
    __syncthreads();
    res.changed = S.changed != 0;
    res.dx2 = block_sum<kSelectThreads>(dx2, S.red);
    res.xn2 = block_sum<kSelectThreads>(xn2, S.red);
    if (res.changed) {
        uint32_t total = 0;
        uint32_t dp = block_excl_scan<kSelectThreads>(ndiff, S.scan, &total);
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int j = j0 + e;
            if (j < n) {
                const float xo = x[j];
                const float xn = ((selmask >> e) & 1ull) ? av[e] : 0.f;
                if (xn != xo) {
                    dlist[dp] = j;
                    dw[dp] = static_cast<double>(xn) - static_cast<double>(xo);
                    ++dp;
                }
            }
        }
        res.dcount = static_cast<int>(total);
    }
    __syncthreads();
    return res;
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_select(const ProbDev* __restrict__ P,
                                                           SolveArgs a, int mode) {
    const ProbDev& pd = P[blockIdx.x];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    if (st->done) return;
    const int cur = st->cur;
    if (mode == SEL_INIT) {
        select_core<CPT>(SEL_INIT, pd.n, pd.s, nullptr, pd.g, nullptr, 1.0f, nullptr,
                         pd.sb[cur], nullptr, nullptr, nullptr, S, &st->err);
        return;
    }
    const float muf = static_cast<float>(st->mu);
    SelOut r = select_core<CPT>(SEL_STEP, pd.n, pd.s, nullptr, pd.g, pd.xb[cur], muf,
                                pd.sb[cur], pd.sb[cur ^ 1], pd.xb[cur ^ 1], pd.dlist, pd.dw,
                                S, &st->err);
    if (threadIdx.x == 0) {
        st->dx2 = r.dx2;
        st->xn2 = r.xn2;
        if (!r.changed) {
            commit(st, a);
        } else {
            st->dcount = r.dcount;
            st->phase = 1;
        }
    }
}

// |Q1 dx|^2 by one workgroup (backtracking path).
template <int BITS>
__device__ double omega_den_block(const ProbDev& pd, int dcount, double* red) {
    constexpr int RPW = (BITS == 32) ? 1 : 32 / BITS;
    const int words = static_cast<int>(pd.col_bytes / 4);
    double tot = 0.0;
    double wsum = 0.0;
    for (int t = 0; t < dcount; ++t) wsum += pd.dw[t];
    for (int w = threadIdx.x; w < words; w += kSelectThreads) {
        double acc[RPW];
#pragma unroll
        for (int q = 0; q < RPW; ++q) acc[q] = 0.0;
        for (int t = 0; t < dcount; ++t) {
            const uint32_t word = *reinterpret_cast<const uint32_t*>(
                pd.q1 + static_cast<size_t>(pd.dlist[t]) * pd.col_bytes + static_cast<size_t>(w) * 4);
            const double wt = pd.dw[t];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const double v = (BITS == 32) ? static_cast<double>(__uint_as_float(word))
                                              : static_cast<double>(code_at<BITS>(word, q));
                acc[q] = fma(wt, v, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int64_t row = static_cast<int64_t>(w) * RPW + q;
            if (row < pd.rows) {
                const double v = (BITS == 32) ? acc[q] : pd.alpha * acc[q] + pd.beta * wsum;
                tot += v * v;
            }
        }
    }
    return block_sum<kSelectThreads>(tot, red);
}

template <int BITS, int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_backtrack(const ProbDev* __restrict__ P,
                                                              SolveArgs a) {
    const ProbDev& pd = P[blockIdx.x];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    __shared__ int s_exit;
    __shared__ double s_mu;
    if (st->done || st->phase != 2) return;
    const int cur = st->cur;
    const double shrink = a.k * (1.0 - a.c);
    for (;;) {
        if (threadIdx.x == 0) {
            s_exit = 0;
            if (st->nb >= a.max_backtracks) {
                st->capped += 1;
                commit(st, a);
                s_exit = 1;
            } else {
                st->mu = st->mu / shrink;
                st->nb += 1;
                s_mu = st->mu;
            }
        }
        __syncthreads();
        if (s_exit) return;
        const double mu = s_mu;
        const float muf = static_cast<float>(mu);
        SelOut r = select_core<CPT>(SEL_STEP, pd.n, pd.s, nullptr, pd.g, pd.xb[cur], muf,
                                    pd.sb[cur], pd.sb[cur ^ 1], pd.xb[cur ^ 1], pd.dlist,
                                    pd.dw, S, &st->err);
        if (threadIdx.x == 0) {
            st->dx2 = r.dx2;
            st->xn2 = r.xn2;
            st->dcount = r.dcount;
        }
        if (!r.changed) {
            if (threadIdx.x == 0) commit(st, a);
            return;
        }
        __syncthreads();
        const double den = omega_den_block<BITS>(pd, r.dcount, S.red);
        const double omega = den > 0.0 ? r.dx2 / den : INFINITY;
        if (mu <= (1.0 - a.c) * omega) {
            if (threadIdx.x == 0) commit(st, a);
            return;
        }
        __syncthreads();
    }
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_hard_threshold(const float* a, int n, int s,
                                                                   int32_t* out, int* err) {
    __shared__ SelShared S;
    select_core<CPT>(SEL_RAW, n, s, a, nullptr, nullptr, 0.f, nullptr, out, nullptr, nullptr,
                     nullptr, S, err);
}

struct InfoDev {
    int32_t iterations, reason, backtracks, capped, err, pad;
    double mu_last;
};

__global__ void k_finalize(const ProbDev* __restrict__ P, float* const* xouts,
                           int32_t* const* souts, InfoDev* infos) {
    const ProbDev& pd = P[blockIdx.y];
    const SolveState* st = pd.st;
    const int cur = st->cur;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < pd.n; j += gridDim.x * blockDim.x)
        xouts[blockIdx.y][j] = pd.xb[cur][j];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < pd.s; t += gridDim.x * blockDim.x)
        souts[blockIdx.y][t] = pd.sb[cur][t];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        InfoDev inf;
        inf.iterations = st->iter;
        inf.reason = st->done ? st->reason : QIHT_REASON_MAX_ITERS;
        inf.backtracks = st->total_bt;
        inf.capped = st->capped;
        inf.err = st->err;
        inf.pad = 0;
        inf.mu_last = st->mu_last;
        infos[blockIdx.y] = inf;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
int select_cpt(int64_t n) {
    int cpt = 1;
    while (static_cast<int64_t>(cpt) * kSelectThreads < n) cpt *= 2;
    return cpt;
}

// Chunks per lane of a full-pass slab: enough to cover the column, at most
// BITS (so a lane holds at most 128 residual rows in registers).
int pass_cpl(int bits, int64_t col_bytes) {
    const int64_t chunks = col_bytes / 16;
    const int maxc = bits == 32 ? 16 : bits;  // at most 128 residual rows per lane
    int c = 1;
    while (c < maxc && static_cast<int64_t>(c) * 64 < chunks) c *= 2;
    return c;
}

template <int BITS, int MODE>
void launch_gather_b(const ProbDev* P, int count, int maxrb, const SolveArgs& a, int zero_x,
                     hipStream_t st) {
    hipLaunchKernelGGL((k_gather<BITS, MODE>), dim3(maxrb, count), dim3(kGatherThreads), 0, st,
                       P, a, zero_x);
}

template <int MODE>
void launch_gather(int bits, const ProbDev* P, int count, int maxrb, const SolveArgs& a,
                   int zero_x, hipStream_t st) {
    switch (bits) {
        case 1: launch_gather_b<1, MODE>(P, count, maxrb, a, zero_x, st); break;
        case 2: launch_gather_b<2, MODE>(P, count, maxrb, a, zero_x, st); break;
        case 4: launch_gather_b<4, MODE>(P, count, maxrb, a, zero_x, st); break;
        case 8: launch_gather_b<8, MODE>(P, count, maxrb, a, zero_x, st); break;
        default: launch_gather_b<32, MODE>(P, count, maxrb, a, zero_x, st); break;
    }
}

template <int BITS>
void launch_pass_b(int cpl, const ProbDev* P, const Task* T, int ntasks, hipStream_t st) {
    switch (cpl) {
#define QIHT_PASS_CASE(C)                                                                  \
    case C:                                                                                \
        if constexpr (C <= BITS)                                                           \
            hipLaunchKernelGGL((k_fullpass<BITS, C>), dim3(ntasks), dim3(kPassThreads), 0, \
                               st, P, T);                                                  \
        break;
        QIHT_PASS_CASE(1)
        QIHT_PASS_CASE(2)
        QIHT_PASS_CASE(4)
        QIHT_PASS_CASE(8)
        QIHT_PASS_CASE(16)
        QIHT_PASS_CASE(32)
#undef QIHT_PASS_CASE
        default: break;
    }
}

void launch_pass(int bits, int cpl, const ProbDev* P, const Task* T, int ntasks, hipStream_t st) {
    switch (bits) {
        case 1: launch_pass_b<1>(cpl, P, T, ntasks, st); break;
        case 2: launch_pass_b<2>(cpl, P, T, ntasks, st); break;
        case 4: launch_pass_b<4>(cpl, P, T, ntasks, st); break;
        case 8: launch_pass_b<8>(cpl, P, T, ntasks, st); break;
        default: launch_pass_b<32>(cpl, P, T, ntasks, st); break;
    }
}

template <int CPT>
void launch_select_c(const ProbDev* P, int count, const SolveArgs& a, int mode, hipStream_t st) {
    hipLaunchKernelGGL((k_select<CPT>), dim3(count), dim3(kSelectThreads), 0, st, P, a, mode);
}

void launch_select(int cpt, const ProbDev* P, int count, const SolveArgs& a, int mode,
                   hipStream_t st) {
    switch (cpt) {
        case 1: launch_select_c<1>(P, count, a, mode, st); break;
        case 2: launch_select_c<2>(P, count, a, mode, st); break;
        case 4: launch_select_c<4>(P, count, a, mode, st); break;
        case 8: launch_select_c<8>(P, count, a, mode, st); break;
        case 16: launch_select_c<16>(P, count, a, mode, st); break;
        case 32: launch_select_c<32>(P, count, a, mode, st); break;
        default: launch_select_c<64>(P, count, a, mode, st); break;
    }
}

template <int BITS>
void launch_backtrack_b(int cpt, const ProbDev* P, int count, const SolveArgs& a,
                        hipStream_t st) {
    switch (cpt) {
#define QIHT_BT_CASE(C)                                                                     \
    case C:                                                                                 \
        hipLaunchKernelGGL((k_backtrack<BITS, C>), dim3(count), dim3(kSelectThreads), 0, st, \
                           P, a);                                                           \
        break;
        QIHT_BT_CASE(1)
        QIHT_BT_CASE(2)
        QIHT_BT_CASE(4)
        QIHT_BT_CASE(8)
        QIHT_BT_CASE(16)
        QIHT_BT_CASE(32)
        QIHT_BT_CASE(64)
#undef QIHT_BT_CASE
        default: break;
    }
}

void launch_backtrack(int bits, int cpt, const ProbDev* P, int count, const SolveArgs& a,
                      hipStream_t st) {
    switch (bits) {
        case 1: launch_backtrack_b<1>(cpt, P, count, a, st); break;
        case 2: launch_backtrack_b<2>(cpt, P, count, a, st); break;
        case 4: launch_backtrack_b<4>(cpt, P, count, a, st); break;
        case 8: launch_backtrack_b<8>(cpt, P, count, a, st); break;
        default: launch_backtrack_b<32>(cpt, P, count, a, st); break;
    }
}

// Workspace carve-out from one device allocation.
struct Carver {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count) {
        off = (off + 255) / 256 * 256;
        const size_t o = off;
        off += count * sizeof(T);
        return o;
    }
};

struct Layout {
    size_t r32, g, gpart, xb0, xb1, sb0, sb1, dlist, dw, part, counter, st;
};

constexpr int kMaxSelectN = kSelectThreads * 64;

struct Plan {
    std::vector<ProbDev> host;
    std::vector<Task> tasks;
    int bits = 0;
    int cpl = 1;
    int cpt = 1;
    int maxrb = 1;
    bool any_slab = false;
    size_t bytes = 0;
    size_t probs_off = 0, tasks_off = 0, xptr_off = 0, sptr_off = 0, info_off = 0;
    std::vector<Layout> lay;
};

qiht_status make_plan(const ProblemIn* in, int count, Plan& pl) {
    pl.bits = in[0].q->bits;
    int64_t max_cb = 0, max_n = 0;
    for (int i = 0; i < count; ++i) {
        max_cb = std::max(max_cb, in[i].q->col_bytes);
        max_n = std::max(max_n, in[i].q->n);
    }
    if (max_n > kMaxSelectN)
        return fail(QIHT_ERR_UNSUPPORTED, "n above the selection limit (65536)");
    pl.cpl = pass_cpl(pl.bits, max_cb);
    pl.cpt = select_cpt(max_n);
    const int rpc = pl.bits == 32 ? 4 : 128 / pl.bits;
    const int64_t slab_chunks = 64LL * pl.cpl;
    Carver cv;
    pl.lay.resize(count);
    pl.host.resize(count);
    for (int i = 0; i < count; ++i) {
        const qiht_qmatrix* q = in[i].q;
        const int64_t chunks = q->col_bytes / 16;
        const int nslab = static_cast<int>((chunks + slab_chunks - 1) / slab_chunks);
        const int nrb = static_cast<int>(q->col_bytes / 256);
        pl.maxrb = std::max(pl.maxrb, nrb);
        pl.any_slab = pl.any_slab || nslab > 1;
        Layout& L = pl.lay[i];
        L.r32 = cv.take<float>(q->rows_pad);
        L.g = cv.take<float>(q->n);
        L.gpart = cv.take<float>(nslab > 1 ? static_cast<size_t>(nslab) * q->n : 1);
        L.xb0 = cv.take<float>(q->n);
        L.xb1 = cv.take<float>(q->n);
        L.sb0 = cv.take<int32_t>(in[i].s);
        L.sb1 = cv.take<int32_t>(in[i].s);
        // at most n entries differ between two iterates
        L.dlist = cv.take<int32_t>(q->n);
        L.dw = cv.take<double>(q->n);
        L.part = cv.take<double>(2 * nrb);
        L.counter = cv.take<unsigned>(4);
        L.st = cv.take<SolveState>(1);
        ProbDev& p = pl.host[i];
        std::memset(&p, 0, sizeof(p));
        p.q1 = q->codes[0];
        p.q2 = q->codes[1];
        p.col_bytes = q->col_bytes;
        p.rows = static_cast<int32_t>(q->rows);
        p.n = static_cast<int32_t>(q->n);
        p.s = static_cast<int32_t>(in[i].s);
        p.nrb = nrb;
        p.nslab = nslab;
        p.alpha = q->alpha;
        p.beta = q->beta;
        p.alpha_f = static_cast<float>(q->alpha);
        p.yhat = in[i].yhat;
        // task split: about 256 KB of codes per workgroup
        const int64_t slab_bytes = std::min<int64_t>(q->col_bytes, slab_chunks * 16);
        const int64_t tc_bw = std::max<int64_t>(8, (256 * 1024) / std::max<int64_t>(slab_bytes, 1));
        const int64_t tc = std::max<int64_t>(8, std::min<int64_t>(tc_bw, (q->n + 255) / 256));
        for (int sl = 0; sl < nslab; ++sl)
            for (int64_t c0 = 0; c0 < q->n; c0 += tc)
                pl.tasks.push_back(Task{i, sl, static_cast<int32_t>(c0),
                                        static_cast<int32_t>(std::min<int64_t>(q->n, c0 + tc))});
        (void)rpc;
    }
    pl.probs_off = cv.take<ProbDev>(count);
    pl.tasks_off = cv.take<Task>(pl.tasks.size());
    pl.xptr_off = cv.take<float*>(count);
    pl.sptr_off = cv.take<int32_t*>(count);
    pl.info_off = cv.take<InfoDev>(count);
    pl.bytes = cv.off;
    return QIHT_OK;
}

void bind(Plan& pl, uint8_t* base) {
    for (size_t i = 0; i < pl.host.size(); ++i) {
        ProbDev& p = pl.host[i];
        const Layout& L = pl.lay[i];
        p.r32 = reinterpret_cast<float*>(base + L.r32);
        p.g = reinterpret_cast<float*>(base + L.g);
        p.gpart = reinterpret_cast<float*>(base + L.gpart);
        p.xb[0] = reinterpret_cast<float*>(base + L.xb0);
        p.xb[1] = reinterpret_cast<float*>(base + L.xb1);
        p.sb[0] = reinterpret_cast<int32_t*>(base + L.sb0);
        p.sb[1] = reinterpret_cast<int32_t*>(base + L.sb1);
        p.dlist = reinterpret_cast<int32_t*>(base + L.dlist);
        p.dw = reinterpret_cast<double*>(base + L.dw);
        p.part = reinterpret_cast<double*>(base + L.part);
        p.counter = reinterpret_cast<unsigned*>(base + L.counter);
        p.st = reinterpret_cast<SolveState*>(base + L.st);
    }
}

// One iteration's launches.
void launch_iteration(const Plan& pl, const ProbDev* dP, const Task* dT, int count,
                      const SolveArgs& a, bool skip_gradient, hipStream_t st) {
    if (!skip_gradient) {
        launch_gather<G_R>(pl.bits, dP, count, pl.maxrb, a, 0, st);
        launch_pass(pl.bits, pl.cpl, dP, dT, static_cast<int>(pl.tasks.size()), st);
        if (pl.any_slab) hipLaunchKernelGGL(k_slab_reduce, dim3(64, count), dim3(256), 0, st, dP);
    }
    launch_gather<G_MU>(pl.bits, dP, count, pl.maxrb, a, 0, st);
    launch_select(pl.cpt, dP, count, a, SEL_STEP, st);
    launch_gather<G_OMEGA>(pl.bits, dP, count, pl.maxrb, a, 0, st);
    launch_backtrack(pl.bits, pl.cpt, dP, count, a, st);
}

}  // namespace

qiht_status run_solve(const ProblemIn* in, int count, const SolveArgs& a, qiht_info* infos,
                      hipStream_t st) {
    Plan pl;
    qiht_status s0 = make_plan(in, count, pl);
    if (s0 != QIHT_OK) return s0;
    uint8_t* base = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&base), pl.bytes, st);
    if (e != hipSuccess || base == nullptr)
        return fail(QIHT_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    struct Guard {
        uint8_t* p;
        hipStream_t s;
        ~Guard() {
            if (p) (void)hipFreeAsync(p, s);
        }
    } guard{base, st};
    bind(pl, base);
    QIHT_HIP(hipMemsetAsync(base, 0, pl.bytes, st));
    std::vector<float*> xo(count);
    std::vector<int32_t*> so(count);
    bool warm = false;
    for (int i = 0; i < count; ++i) {
        xo[i] = in[i].x_out;
        so[i] = in[i].support_out;
        if (in[i].x0) {
            warm = true;
            QIHT_HIP(hipMemcpyAsync(pl.host[i].xb[0], in[i].x0, sizeof(float) * pl.host[i].n,
                                    hipMemcpyDeviceToDevice, st));
            QIHT_HIP(hipMemcpyAsync(pl.host[i].sb[0], in[i].support0,
                                    sizeof(int32_t) * pl.host[i].s, hipMemcpyDeviceToDevice,
                                    st));
        }
    }
    ProbDev* dP = reinterpret_cast<ProbDev*>(base + pl.probs_off);
    Task* dT = reinterpret_cast<Task*>(base + pl.tasks_off);
    QIHT_HIP(hipMemcpyAsync(dP, pl.host.data(), sizeof(ProbDev) * count, hipMemcpyHostToDevice,
                            st));
    QIHT_HIP(hipMemcpyAsync(dT, pl.tasks.data(), sizeof(Task) * pl.tasks.size(),
                            hipMemcpyHostToDevice, st));
    float** dxo = reinterpret_cast<float**>(base + pl.xptr_off);
    int32_t** dso = reinterpret_cast<int32_t**>(base + pl.sptr_off);
    QIHT_HIP(hipMemcpyAsync(dxo, xo.data(), sizeof(float*) * count, hipMemcpyHostToDevice, st));
    QIHT_HIP(hipMemcpyAsync(dso, so.data(), sizeof(int32_t*) * count, hipMemcpyHostToDevice,
                            st));

    if (!warm) {
        // x0 = 0; G0 = supp H_s(Q1^T y_hat).  g0 is reused by iteration 1.
        launch_gather<G_R>(pl.bits, dP, count, pl.maxrb, a, 1, st);
        launch_pass(pl.bits, pl.cpl, dP, dT, static_cast<int>(pl.tasks.size()), st);
        if (pl.any_slab) hipLaunchKernelGGL(k_slab_reduce, dim3(64, count), dim3(256), 0, st, dP);
        launch_select(pl.cpt, dP, count, a, SEL_INIT, st);
    }
    QIHT_HIP(hipGetLastError());

    // Iterations in chunks; between chunks the host checks the stop flags.
    const int chunk = 16;
    std::vector<SolveState> hs(count);
    for (int it = 1; it <= a.max_iters;) {
        const int end = std::min(a.max_iters, it + chunk - 1);
        for (; it <= end; ++it)
            launch_iteration(pl, dP, dT, count, a, it == 1 && !warm, st);
        QIHT_HIP(hipGetLastError());
        if (it > a.max_iters) break;
        bool all_done = true;
        for (int i = 0; i < count; ++i)
            QIHT_HIP(hipMemcpyAsync(&hs[i], pl.host[i].st, sizeof(SolveState),
                                    hipMemcpyDeviceToHost, st));
        QIHT_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < count; ++i) all_done = all_done && hs[i].done;
        if (all_done) break;
    }

    InfoDev* dinf = reinterpret_cast<InfoDev*>(base + pl.info_off);
    hipLaunchKernelGGL(k_finalize, dim3(32, count), dim3(256), 0, st, dP, dxo, dso, dinf);
    QIHT_HIP(hipGetLastError());
    std::vector<InfoDev> hinf(count);
    QIHT_HIP(hipMemcpyAsync(hinf.data(), dinf, sizeof(InfoDev) * count, hipMemcpyDeviceToHost,
                            st));
    QIHT_HIP(hipStreamSynchronize(st));
    bool nan = false;
    for (int i = 0; i < count; ++i) {
        nan = nan || hinf[i].err;
        if (infos) {
            infos[i].iterations = hinf[i].iterations;
            infos[i].reason = hinf[i].reason;
            infos[i].backtracks = hinf[i].backtracks;
            infos[i].capped_iterations = hinf[i].capped;
            infos[i].mu_last = hinf[i].mu_last;
            infos[i].status_flags = 0.0;
        }
    }
    if (nan) return fail(QIHT_ERR_NUMERIC, "NaN met in the iterate");
    return QIHT_OK;
}

qiht_status run_gradient(const qiht_qmatrix* q, const double* yhat, const float* x,
                         const int32_t* support, int64_t s, float* g_out, float* r_out,
                         hipStream_t st) {
    ProblemIn in{q, yhat, s, nullptr, nullptr, x, support};
    Plan pl;
    qiht_status s0 = make_plan(&in, 1, pl);
    if (s0 != QIHT_OK) return s0;
    uint8_t* base = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&base), pl.bytes, st);
    if (e != hipSuccess || base == nullptr)
        return fail(QIHT_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    bind(pl, base);
    QIHT_HIP(hipMemsetAsync(base, 0, pl.bytes, st));
    const ProbDev& h = pl.host[0];
    if (s > 0) {
        QIHT_HIP(hipMemcpyAsync(h.xb[0], x, sizeof(float) * h.n, hipMemcpyDeviceToDevice, st));
        QIHT_HIP(hipMemcpyAsync(h.sb[0], support, sizeof(int32_t) * s, hipMemcpyDeviceToDevice,
                                st));
    }
    ProbDev* dP = reinterpret_cast<ProbDev*>(base + pl.probs_off);
    Task* dT = reinterpret_cast<Task*>(base + pl.tasks_off);
    QIHT_HIP(hipMemcpyAsync(dP, pl.host.data(), sizeof(ProbDev), hipMemcpyHostToDevice, st));
    QIHT_HIP(hipMemcpyAsync(dT, pl.tasks.data(), sizeof(Task) * pl.tasks.size(),
                            hipMemcpyHostToDevice, st));
    SolveArgs a{1, -1.0, 2.0, 0.01, 0, 0};
    launch_gather<G_R>(pl.bits, dP, 1, pl.maxrb, a, s == 0 ? 1 : 0, st);
    launch_pass(pl.bits, pl.cpl, dP, dT, static_cast<int>(pl.tasks.size()), st);
    hipLaunchKernelGGL(k_slab_reduce, dim3(64, 1), dim3(256), 0, st, dP);
    QIHT_HIP(hipGetLastError());
    QIHT_HIP(hipMemcpyAsync(g_out, h.g, sizeof(float) * h.n, hipMemcpyDeviceToDevice, st));
    if (r_out)
        QIHT_HIP(hipMemcpyAsync(r_out, h.r32, sizeof(float) * h.rows, hipMemcpyDeviceToDevice,
                                st));
    QIHT_HIP(hipFreeAsync(base, st));
    QIHT_HIP(hipStreamSynchronize(st));
    return QIHT_OK;
}

qiht_status run_hard_threshold(const float* a, int64_t n, int64_t s, int32_t* support_out,
                               hipStream_t st) {
    if (n > kMaxSelectN) return fail(QIHT_ERR_UNSUPPORTED, "n above the selection limit (65536)");
    int* err = nullptr;
    QIHT_HIP(hipMallocAsync(reinterpret_cast<void**>(&err), sizeof(int), st));
    QIHT_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
    const int cpt = select_cpt(n);
    const int nn = static_cast<int>(n), ss = static_cast<int>(s);
    switch (cpt) {
#define QIHT_HT_CASE(C)                                                                   \
    case C:                                                                               \
        hipLaunchKernelGGL((k_hard_threshold<C>), dim3(1), dim3(kSelectThreads), 0, st, a, \
                           nn, ss, support_out, err);                                     \
        break;
        QIHT_HT_CASE(1)
        QIHT_HT_CASE(2)
        QIHT_HT_CASE(4)
        QIHT_HT_CASE(8)
        QIHT_HT_CASE(16)
        QIHT_HT_CASE(32)
        QIHT_HT_CASE(64)
#undef QIHT_HT_CASE
        default: break;
    }
    QIHT_HIP(hipGetLastError());
    int herr = 0;
    QIHT_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    QIHT_HIP(hipFreeAsync(err, st));
    QIHT_HIP(hipStreamSynchronize(st));
    if (herr) return fail(QIHT_ERR_NUMERIC, "NaN in the input of H_s");
    return QIHT_OK;
}

}  // namespace qiht
