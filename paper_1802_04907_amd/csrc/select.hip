// H_s proposals of the QIHT iteration (Sec. I-A hard threshold, Sec. II-A
// step-size rule).
//
// One workgroup builds one proposal x' = H_s(x + mu_k g) with
// mu_k = mu / (k(1-c))^k: an exact radix select of the s-th largest |a|
// (31-bit keys; digits of 11, 10 and 10 bits counted in LDS histograms),
// ties at the threshold resolved to the lowest indices, and an
// order-preserving compaction built from wave ballots, so the support comes
// out ascending.  Thread t owns indices t, t + 1024, ..., so every global
// load is coalesced; wave w of round e covers indices [1024e + 64w, +64),
// which makes (round, wave, lane) index order.
//
// k_propose runs kSpec proposals (k = 0 .. kSpec-1) side by side, one
// workgroup each; the omega gather then applies the step test to all of
// them at once (speculative backtracking: the accepted proposal is the one
// the sequential rule would reach).  k_fallback continues sequentially, in
// one workgroup, in the rare case that every speculative proposal is
// rejected.
#include "solve_common.h"

namespace qiht {
namespace {

struct SelShared {
    uint32_t hist[2048];
    uint32_t cnt[kSelectThreads];   // per (round, wave) counts, then bases
    uint32_t bm_old[kMaxSelectN / 32];
    uint32_t bm_new[kMaxSelectN / 32];
    uint32_t scan[16];
    uint32_t bin, krem;
    int changed;
    double red[16];
};

__device__ __forceinline__ uint32_t abs_key(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// Exclusive scan of S.cnt[0 .. CPT*16) in place (index order).
template <int CPT>
__device__ void scan_round_wave_counts(SelShared& S) {
    constexpr int NC = CPT * 16;
    uint32_t v = threadIdx.x < NC ? S.cnt[threadIdx.x] : 0u;
    const uint32_t before = block_excl_scan<kSelectThreads>(v, S.scan, nullptr);
    if (threadIdx.x < NC) S.cnt[threadIdx.x] = before;
    __syncthreads();
}

// The value whose magnitude is ranked: a_j = x_j + mu g_j (FP32, fused), or
// g_j (initial support), or an input vector.
template <int MODE>
__device__ __forceinline__ float value_at(const float* a_in, const float* g, const float* x,
                                          float muf, int j) {
    if (MODE == SEL_RAW) return a_in[j];
    if (MODE == SEL_INIT) return g[j];
    return fmaf(muf, g[j], x[j]);
}

// Builds one proposal.  Outputs: out_sup (ascending, s entries), and for
// SEL_STEP out_val (values on out_sup), the changed flag against old_sup,
// the difference list (union of old and new supports, ascending, with
// FP64 differences) and |x' - x|^2, |x'|^2 into *meta (written by thread 0).
template <int CPT, int MODE>
__device__ void propose_core(int n, int s, const float* a_in, const float* g, const float* x,
                             float muf, const int32_t* old_sup, int32_t* out_sup,
                             float* out_val, int32_t* dlist, double* dw, CandMeta* meta,
                             int k, double mu, SelShared& S, int* err) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    uint32_t key[CPT];
    int bad = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        key[e] = 0u;
        if (j < n) {
            key[e] = abs_key(value_at<MODE>(a_in, g, x, muf, j));
            if (key[e] > 0x7F800000u) bad = 1;
        }
    }
    if (bad) atomicOr(err, 1);

    // ---- radix select of the s-th largest key ----
    uint32_t prefix = 0, krem = static_cast<uint32_t>(s);
#pragma unroll
    for (int pass = 0; pass < 3; ++pass) {
        const int width = pass == 0 ? 11 : 10;
        const int sh = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
        const int nb = 1 << width;
        const int hsh = sh + width;
        for (int b = tid; b < 2048; b += kSelectThreads) S.hist[b] = 0u;
        __syncthreads();
        if (krem > 0) {
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                const int j = tid + kSelectThreads * e;
                if (j < n && (pass == 0 || (key[e] >> hsh) == prefix))
                    atomicAdd(&S.hist[(key[e] >> sh) & (nb - 1)], 1u);
            }
        }
        __syncthreads();
        const int PB = nb / kSelectThreads;  // bins per thread, descending
        uint32_t c0 = S.hist[nb - 1 - tid * PB];
        uint32_t c1 = PB > 1 ? S.hist[nb - 2 - tid * PB] : 0u;
        const uint32_t above = block_excl_scan<kSelectThreads>(c0 + c1, S.scan, nullptr);
        if (krem > 0) {
            if (above < krem && krem <= above + c0) {
                S.bin = static_cast<uint32_t>(nb - 1 - tid * PB);
                S.krem = krem - above;
            } else if (PB > 1 && above + c0 < krem && krem <= above + c0 + c1) {
                S.bin = static_cast<uint32_t>(nb - 2 - tid * PB);
                S.krem = krem - above - c0;
            }
        }
        __syncthreads();
        if (krem > 0) {
            prefix = (prefix << width) | S.bin;
            krem = S.krem;
        }
        __syncthreads();
    }
    const uint32_t T = prefix;   // the s-th largest key (s > 0)
    const uint32_t need = krem;  // keys equal to T that are taken

    // ---- ranks of the ties at T, in index order ----
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const uint64_t b = __ballot(s > 0 && j < n && key[e] == T);
        if (lane == 0) S.cnt[e * 16 + wv] = static_cast<uint32_t>(__popcll(b));
    }
    __syncthreads();
    scan_round_wave_counts<CPT>(S);
    uint64_t take = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const bool tie = s > 0 && j < n && key[e] == T;
        const uint64_t b = __ballot(tie);
        const uint32_t rank = S.cnt[e * 16 + wv] + static_cast<uint32_t>(__popcll(b & lanemask_lt()));
        const bool sel = s > 0 && j < n && (key[e] > T || (tie && rank < need));
        take |= static_cast<uint64_t>(sel) << e;
    }
    __syncthreads();
    // ---- output positions of the selected indices ----
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const uint64_t b = __ballot((take >> e) & 1ull);
        if (lane == 0) S.cnt[e * 16 + wv] = static_cast<uint32_t>(__popcll(b));
    }
    if (tid == 0) S.changed = 0;
    if (MODE == SEL_STEP) {
        for (int w = tid; w < (n + 31) / 32; w += kSelectThreads) {
            S.bm_old[w] = 0u;
            S.bm_new[w] = 0u;
        }
    }
    __syncthreads();
    scan_round_wave_counts<CPT>(S);
    int changed = 0;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const bool sel = (take >> e) & 1ull;
        const uint64_t b = __ballot(sel);
        if (sel) {
            const uint32_t pos = S.cnt[e * 16 + wv] + static_cast<uint32_t>(__popcll(b & lanemask_lt()));
            if (pos < static_cast<uint32_t>(s)) {
                out_sup[pos] = j;
                if (MODE == SEL_STEP) {
                    out_val[pos] = value_at<MODE>(a_in, g, x, muf, j);
                    if (old_sup[pos] != j) changed = 1;
                    atomicOr(&S.bm_new[j >> 5], 1u << (j & 31));
                }
            }
        }
    }
    if (MODE != SEL_STEP) {
        __syncthreads();
        return;
    }
    if (changed) S.changed = 1;
    for (int i = tid; i < s; i += kSelectThreads) {
        const int j = old_sup[i];
        atomicOr(&S.bm_old[j >> 5], 1u << (j & 31));
    }
    __syncthreads();

    // ---- difference list over old and new supports, |dx|^2, |x'|^2 ----
    const int words = (n + 31) / 32;
    const int wpt = (words + kSelectThreads - 1) / kSelectThreads;
    const int w0 = tid * wpt;
    uint32_t cnt = 0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) cnt += __popc(S.bm_old[w] | S.bm_new[w]);
    uint32_t total = 0;
    uint32_t pos = block_excl_scan<kSelectThreads>(cnt, S.scan, &total);
    double dx2 = 0.0, xn2 = 0.0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) {
        uint32_t u = S.bm_old[w] | S.bm_new[w];
        const uint32_t nw = S.bm_new[w];
        while (u) {
            const int b = __ffs(u) - 1;
            u &= u - 1;
            const int j = w * 32 + b;
            const float xo = x[j];
            const float xn = ((nw >> b) & 1u) ? value_at<MODE>(a_in, g, x, muf, j) : 0.0f;
            const double d = static_cast<double>(xn) - static_cast<double>(xo);
            dlist[pos] = j;
            dw[pos] = d;
            ++pos;
            dx2 += d * d;
            xn2 += static_cast<double>(xn) * static_cast<double>(xn);
        }
    }
    dx2 = block_sum<kSelectThreads>(dx2, S.red);
    xn2 = block_sum<kSelectThreads>(xn2, S.red);
    if (tid == 0) {
        CandMeta m;
        m.changed = S.changed;
        m.dcount = static_cast<int32_t>(total);
        m.k = k;
        m.pad = 0;
        m.mu = mu;
        m.dx2 = dx2;
        m.xn2 = xn2;
        m.omega = 0.0;
        *meta = m;
    }
    __syncthreads();
}

template <int CPT>
__device__ void propose_slot(const ProbDev& pd, int slot, int k, double mu, SelShared& S) {
    propose_core<CPT, SEL_STEP>(pd.n, pd.s, nullptr, pd.g, pd.x, static_cast<float>(mu), pd.sup,
                                pd.csup + static_cast<size_t>(slot) * pd.s,
                                pd.cval + static_cast<size_t>(slot) * pd.s,
                                pd.dlist + static_cast<size_t>(slot) * 2 * pd.s,
                                pd.dw + static_cast<size_t>(slot) * 2 * pd.s, &pd.meta[slot], k,
                                mu, S, &pd.st->err);
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_propose(const ProbDev* __restrict__ P,
                                                            SolveArgs a, int mode) {
    const ProbDev& pd = P[blockIdx.y];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    if (st->done) return;
    if (mode == SEL_INIT) {
        propose_core<CPT, SEL_INIT>(pd.n, pd.s, nullptr, pd.g, nullptr, 1.0f, nullptr, pd.sup,
                                    nullptr, nullptr, nullptr, nullptr, 0, 1.0, S, &st->err);
        return;
    }
    const int k = blockIdx.x;  // shrink count of this proposal
    const double mu = shrunk_mu(st->mu, a.k * (1.0 - a.c), k);
    propose_slot<CPT>(pd, k, k, mu, S);
}

// |Q1 dx|^2 of slot 0's difference list, by one workgroup.
template <int BITS>
__device__ double omega_den_block(const ProbDev& pd, int dcount, double* red) {
    constexpr int RPW = (BITS == 32) ? 1 : 32 / BITS;
    const int words = static_cast<int>(pd.col_bytes / 4);
    double wsum = 0.0;
    for (int t = 0; t < dcount; ++t) wsum += pd.dw[t];
    double tot = 0.0;
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

// Sequential continuation of the step test from shrink count base_k, one
// workgroup per problem (only when all kSpec speculative proposals failed).
template <int BITS, int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_fallback(const ProbDev* __restrict__ P,
                                                             SolveArgs a) {
    const ProbDev& pd = P[blockIdx.x];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    if (st->done || st->phase != 2) return;
    const double shrink = a.k * (1.0 - a.c);
    for (int k = st->base_k;; ++k) {
        const double mu = shrunk_mu(st->mu, shrink, k);
        propose_slot<CPT>(pd, 0, k, mu, S);
        const CandMeta m = pd.meta[0];
        bool accept = !m.changed;
        bool capped = false;
        if (!accept) {
            const double den = omega_den_block<BITS>(pd, m.dcount, S.red);
            const double omega = den > 0.0 ? m.dx2 / den : INFINITY;
            accept = mu <= (1.0 - a.c) * omega;
            if (!accept && k >= a.max_backtracks) capped = accept = true;
        }
        if (accept) {
            commit_proposal<kSelectThreads>(pd, 0, a, capped);
            return;
        }
        __syncthreads();
    }
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_hard_threshold(const float* a, int n, int s,
                                                                   int32_t* out, int* err) {
    __shared__ SelShared S;
    propose_core<CPT, SEL_RAW>(n, s, a, nullptr, nullptr, 0.f, nullptr, out, nullptr, nullptr,
                               nullptr, nullptr, 0, 0.0, S, err);
}

}  // namespace

#define QIHT_CPT_SWITCH(CPT_VAR, MACRO) \
    switch (CPT_VAR) {                  \
        MACRO(1)                        \
        MACRO(2)                        \
        MACRO(4)                        \
        MACRO(8)                        \
        MACRO(16)                       \
        MACRO(32)                       \
        MACRO(64)                       \
        default: break;                 \
    }

void launch_propose(int cpt, const ProbDev* P, int count, const SolveArgs& a, int mode,
                    hipStream_t st) {
    const dim3 grid(mode == SEL_INIT ? 1 : kSpec, count);
#define QIHT_PROPOSE(C)                                                                     \
    case C:                                                                                 \
        hipLaunchKernelGGL((k_propose<C>), grid, dim3(kSelectThreads), 0, st, P, a, mode); \
        break;
    QIHT_CPT_SWITCH(cpt, QIHT_PROPOSE)
#undef QIHT_PROPOSE
}

template <int BITS>
void launch_fallback_b(int cpt, const ProbDev* P, int count, const SolveArgs& a, hipStream_t st) {
#define QIHT_FALLBACK(C)                                                                        \
    case C:                                                                                     \
        hipLaunchKernelGGL((k_fallback<BITS, C>), dim3(count), dim3(kSelectThreads), 0, st, P, \
                           a);                                                                  \
        break;
    QIHT_CPT_SWITCH(cpt, QIHT_FALLBACK)
#undef QIHT_FALLBACK
}

void launch_fallback(int bits, int cpt, const ProbDev* P, int count, const SolveArgs& a,
                     hipStream_t st) {
    switch (bits) {
        case 1: launch_fallback_b<1>(cpt, P, count, a, st); break;
        case 2: launch_fallback_b<2>(cpt, P, count, a, st); break;
        case 4: launch_fallback_b<4>(cpt, P, count, a, st); break;
        case 8: launch_fallback_b<8>(cpt, P, count, a, st); break;
        default: launch_fallback_b<32>(cpt, P, count, a, st); break;
    }
}

void launch_hard_threshold(int cpt, const float* a, int n, int s, int32_t* out, int* err,
                           hipStream_t st) {
#define QIHT_HT(C)                                                                          \
    case C:                                                                                 \
        hipLaunchKernelGGL((k_hard_threshold<C>), dim3(1), dim3(kSelectThreads), 0, st, a, \
                           n, s, out, err);                                                 \
        break;
    QIHT_CPT_SWITCH(cpt, QIHT_HT)
#undef QIHT_HT
}

}  // namespace qiht
