// H_s proposals and the step-size test of the QIHT iteration (Sec. I-A hard
// threshold; Sec. II-A and Algorithm 2: normalized step, support-change
// test, shrinking by k(1-c)).
//
// k_propose: one workgroup per proposal x'_k = H_s(x + mu_k g) with
// mu_k = mu / (k(1-c))^k, k = 0 .. kSpec-1 side by side (speculative
// backtracking).  Each workgroup first finishes mu = |g_G|^2 / (Q1_G g_G).
// (Q2_G g_G) from the gather partials, in workgroup order.
//
// Selection, fast path: off the current support G, a_j = mu g_j, so the
// order of |a_j| there does not depend on mu.  The full pass counts |g_j| in
// a 2048-bin histogram of its top 11 bits; with G's entries removed, the bin
// B of the s-th largest |g_j| off G gives a threshold t = lo(B)(1 - 2^-20).
// An entry off G with |g_j| < t has FP32 |a_j| strictly below at least s
// entries off G, for any mu (round-to-nearest moves a product by at most
// 2^-24 relative), so the top s of G plus {j off G : |g_j| >= t} is the top
// s of all n.  That candidate set (usually a few thousand entries) is ranked
// exactly: radix select of the s-th largest |a| (31-bit keys, digits of 11,
// 10, 10 bits in LDS histograms), ties at the threshold to the lowest
// indices through an index bitmap, and the support written ascending by an
// ordered scan of the selection bitmap.  Full path (candidate set too large,
// or a plain H_s call): the same rank over all n keys held in registers.
//
// k_decide: the test mu_k <= (1-c)|x'_k - x|^2 / |Q1 (x'_k - x)|^2 applied in
// order k = 0, 1, ... (a proposal keeping the support is accepted at once);
// the first accepted proposal is committed.  If all kSpec proposals fail,
// the same workgroup continues one shrink at a time.
#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kBmWords = kMaxSelectN / 32;

struct SelShared {
    uint32_t hist[2048];
    uint32_t cnt[kSelectThreads];
    uint32_t bm_old[kBmWords];   // current support
    uint32_t bm_new[kBmWords];   // selected set
    uint32_t bm_tie[kBmWords];   // candidates equal to the threshold key
    uint32_t ckey[kCandCap];
    int32_t cidx[kCandCap];
    uint32_t scan[16];
    uint32_t bin, krem, ncand;
    int changed, overflow;
    double red[16];
};

__device__ __forceinline__ uint32_t abs_key(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

template <int MODE>
__device__ __forceinline__ float value_at(const float* a_in, const float* g, const float* x,
                                          float muf, int j) {
    if (MODE == SEL_RAW) return a_in[j];
    if (MODE == SEL_INIT) return g[j];
    return fmaf(muf, g[j], x[j]);
}

// One radix digit step: bins of `hist` (nb bins, counts already in place)
// scanned from the top; finds the bin holding the krem-th largest key.
__device__ void find_bin(SelShared& S, int nb, uint32_t& prefix, uint32_t& krem, int width) {
    const int tid = threadIdx.x;
    const int PB = nb / kSelectThreads;  // 1 or 2
    const uint32_t c0 = S.hist[nb - 1 - tid * PB];
    const uint32_t c1 = PB > 1 ? S.hist[nb - 2 - tid * PB] : 0u;
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

// Writes the support (ascending) from the selection bitmap, the values on
// it, and compares with the old support.  Returns through S.changed.
template <int MODE>
__device__ void emit_support(int n, int s, const float* a_in, const float* g, const float* x,
                             float muf, const int32_t* old_sup, int32_t* out_sup, float* out_val,
                             SelShared& S) {
    const int tid = threadIdx.x;
    const int words = (n + 31) / 32;
    const int wpt = (words + kSelectThreads - 1) / kSelectThreads;
    const int w0 = tid * wpt;
    uint32_t c = 0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) c += __popc(S.bm_new[w]);
    uint32_t pos = block_excl_scan<kSelectThreads>(c, S.scan, nullptr);
    int changed = 0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) {
        uint32_t u = S.bm_new[w];
        while (u) {
            const int b = __ffs(u) - 1;
            u &= u - 1;
            const int j = w * 32 + b;
            if (pos < static_cast<uint32_t>(s)) {
                out_sup[pos] = j;
                if (MODE == SEL_STEP) {
                    out_val[pos] = value_at<MODE>(a_in, g, x, muf, j);
                    if (old_sup[pos] != j) changed = 1;
                }
            }
            ++pos;
        }
    }
    if (changed) S.changed = 1;
    __syncthreads();
}

// Rank over keys held in registers (thread t owns t, t + 1024, ...): the
// full path.  Sets the selection bitmap S.bm_new.
template <int CPT, int MODE>
__device__ void select_full(int n, int s, const float* a_in, const float* g, const float* x,
                            float muf, SelShared& S, int* err) {
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
        find_bin(S, nb, prefix, krem, width);
    }
    const uint32_t T = prefix;
    const uint32_t need = krem;
    // ties at T ranked in index order: (round, wave, lane) is index order
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const uint64_t b = __ballot(s > 0 && j < n && key[e] == T);
        if (lane == 0) S.cnt[e * 16 + wv] = static_cast<uint32_t>(__popcll(b));
    }
    __syncthreads();
    {
        constexpr int NC = CPT * 16;
        const uint32_t v = tid < NC ? S.cnt[tid] : 0u;
        const uint32_t before = block_excl_scan<kSelectThreads>(v, S.scan, nullptr);
        if (tid < NC) S.cnt[tid] = before;
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const bool tie = s > 0 && j < n && key[e] == T;
        const uint64_t b = __ballot(tie);
        const uint32_t rank = S.cnt[e * 16 + wv] + static_cast<uint32_t>(__popcll(b & lanemask_lt()));
        if (s > 0 && j < n && (key[e] > T || (tie && rank < need)))
            atomicOr(&S.bm_new[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
}

// Fast path over the support and the histogram candidates; returns false
// (and selects nothing) when the candidate set does not fit in LDS.
// Appends (key, index) to the LDS candidate list; one LDS atomic per wave.
__device__ __forceinline__ void push_candidate(bool pred, uint32_t key, int j, SelShared& S) {
    const uint64_t b = __ballot(pred);
    if (b == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll(static_cast<long long>(b)) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&S.ncand, static_cast<uint32_t>(__popcll(b)));
    base = __shfl(base, leader, 64);
    if (pred) {
        const uint32_t c = base + static_cast<uint32_t>(__popcll(b & lanemask_lt()));
        if (c < static_cast<uint32_t>(kCandCap)) {
            S.ckey[c] = key;
            S.cidx[c] = j;
        }
    }
}

template <int CPT, int MODE>
__device__ bool select_fast(int n, int s, const float* g, const float* x, float muf,
                            const int32_t* old_sup, int nsup, const uint32_t* ghist,
                            SelShared& S, int* err) {
    const int tid = threadIdx.x;
    // every |g_j| this thread owns, loaded up front (independent loads)
    float gv[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        gv[e] = j < n ? g[j] : 0.0f;
    }
    for (int b = tid; b < 2048; b += kSelectThreads) S.hist[b] = ghist[b];
    if (tid == 0) {
        S.ncand = 0;
        S.overflow = 0;
    }
    __syncthreads();
    for (int i = tid; i < nsup; i += kSelectThreads)
        atomicSub(&S.hist[abs_key(g[old_sup[i]]) >> 20], 1u);
    __syncthreads();
    // bin of the s-th largest |g| off the support
    const int off_count = n - nsup;
    float thr = 0.0f;
    if (off_count > s) {
        uint32_t prefix = 0, krem = static_cast<uint32_t>(s);
        find_bin(S, 2048, prefix, krem, 11);
        thr = __uint_as_float(prefix << 20) * (1.0f - 0x1p-20f);
        if (!(thr >= 0x1p-100f)) return false;  // keep clear of subnormal products
    }
    // collect candidates: the support, and off-support entries above thr
    int bad = 0;
    for (int i0 = 0; i0 < nsup; i0 += kSelectThreads) {
        const int i = i0 + tid;
        const bool in = i < nsup;
        const int j = in ? old_sup[i] : 0;
        const uint32_t k = in ? abs_key(value_at<MODE>(nullptr, g, x, muf, j)) : 0u;
        if (k > 0x7F800000u) bad = 1;
        push_candidate(in, k, j, S);
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const bool in = j < n && fabsf(gv[e]) >= thr && !((S.bm_old[j >> 5] >> (j & 31)) & 1u);
        // off the support x_j = 0, so a_j = fma(mu, g_j, 0)
        const uint32_t k = in ? abs_key((MODE == SEL_STEP) ? fmaf(muf, gv[e], 0.0f) : gv[e]) : 0u;
        if (k > 0x7F800000u) bad = 1;
        push_candidate(in, k, j, S);
    }
    if (bad) atomicOr(err, 1);
    __syncthreads();
    const uint32_t nc = S.ncand;
    if (nc > static_cast<uint32_t>(kCandCap)) return false;
    // exact rank among the candidates
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
            for (uint32_t c = tid; c < nc; c += kSelectThreads) {
                const uint32_t k = S.ckey[c];
                if (pass == 0 || (k >> hsh) == prefix) atomicAdd(&S.hist[(k >> sh) & (nb - 1)], 1u);
            }
        }
        __syncthreads();
        find_bin(S, nb, prefix, krem, width);
    }
    const uint32_t T = prefix;
    const uint32_t need = krem;
    for (uint32_t c = tid; c < nc; c += kSelectThreads) {
        const uint32_t k = S.ckey[c];
        const int j = S.cidx[c];
        if (s > 0 && k > T) atomicOr(&S.bm_new[j >> 5], 1u << (j & 31));
        else if (s > 0 && k == T) atomicOr(&S.bm_tie[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    // the `need` lowest-index ties
    const int words = (n + 31) / 32;
    const int wpt = (words + kSelectThreads - 1) / kSelectThreads;
    const int w0 = tid * wpt;
    uint32_t cnt = 0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) cnt += __popc(S.bm_tie[w]);
    uint32_t rank = block_excl_scan<kSelectThreads>(cnt, S.scan, nullptr);
    for (int w = w0; w < min(words, w0 + wpt); ++w) {
        uint32_t u = S.bm_tie[w];
        while (u) {
            const int b = __ffs(u) - 1;
            u &= u - 1;
            if (rank < need) S.bm_new[w] |= 1u << b;
            ++rank;
        }
    }
    __syncthreads();
    return true;
}

// One complete proposal into `slot` (SEL_STEP) or the initial support
// (SEL_INIT, written to pd.sup).  Thread 0 writes the slot's CandMeta.
template <int CPT, int MODE>
__device__ void propose(const ProbDev& pd, int slot, int k, double mu, SelShared& S) {
    const int tid = threadIdx.x;
    const int n = pd.n, s = pd.s;
    const int words = (n + 31) / 32;
    const float muf = static_cast<float>(mu);
    const int nsup = (MODE == SEL_STEP) ? s : 0;
    for (int w = tid; w < words; w += kSelectThreads) {
        S.bm_old[w] = 0u;
        S.bm_new[w] = 0u;
        S.bm_tie[w] = 0u;
    }
    if (tid == 0) S.changed = 0;
    __syncthreads();
    for (int i = tid; i < nsup; i += kSelectThreads) {
        const int j = pd.sup[i];
        atomicOr(&S.bm_old[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    if (!select_fast<CPT, MODE>(n, s, pd.g, pd.x, muf, pd.sup, nsup, pd.hist, S, &pd.st->err)) {
        if (tid == 0) atomicAdd(&pd.st->full_selects, 1);
        for (int w = tid; w < words; w += kSelectThreads) S.bm_new[w] = 0u;
        __syncthreads();
        select_full<CPT, MODE>(n, s, nullptr, pd.g, pd.x, muf, S, &pd.st->err);
    }
    if (MODE == SEL_INIT) {
        emit_support<MODE>(n, s, nullptr, pd.g, nullptr, muf, nullptr, pd.sup, nullptr, S);
        return;
    }
    int32_t* out_sup = pd.csup + static_cast<size_t>(slot) * s;
    float* out_val = pd.cval + static_cast<size_t>(slot) * s;
    int32_t* dlist = pd.dlist + static_cast<size_t>(slot) * 2 * s;
    double* dw = pd.dw + static_cast<size_t>(slot) * 2 * s;
    emit_support<MODE>(n, s, nullptr, pd.g, pd.x, muf, pd.sup, out_sup, out_val, S);
    // difference list over the union of old and new supports, ascending
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
            const float xo = pd.x[j];
            const float xn = ((nw >> b) & 1u) ? value_at<MODE>(nullptr, pd.g, pd.x, muf, j) : 0.0f;
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
        pd.meta[slot] = m;
    }
    __syncthreads();
}

// mu = |g_G|^2 / ((Q1_G g_G).(Q2_G g_G)) from the gather partials (fixed
// order); falls back to |Q1_G g_G|^2 when the cross term is not positive.
// Returns a negative value when the iteration is stationary.
__device__ double step_from_partials(const ProbDev& pd, SelShared& S) {
    double gg = 0.0, uv = 0.0, uu = 0.0;
    for (int i = threadIdx.x; i < pd.s; i += kSelectThreads) {
        const double v = static_cast<double>(pd.g[pd.sup[i]]);
        gg += v * v;
    }
    for (int b = threadIdx.x; b < pd.nwg; b += kSelectThreads) {
        uv += pd.part_mu[2 * b + 0];
        uu += pd.part_mu[2 * b + 1];
    }
    const double num = block_sum<kSelectThreads>(gg, S.red);
    uv = block_sum<kSelectThreads>(uv, S.red);
    uu = block_sum<kSelectThreads>(uu, S.red);
    double den = uv;
    if (!(den > 0.0) || !isfinite(den)) den = uu;
    if (!(num > 0.0) || !(den > 0.0) || !isfinite(num / den)) return -1.0;
    return num / den;
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_propose(const ProbDev* __restrict__ P,
                                                            SolveArgs a, int mode) {
    const ProbDev& pd = P[blockIdx.y];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    if (st->done) return;
    if (mode == SEL_INIT) {
        propose<CPT, SEL_INIT>(pd, 0, 0, 1.0, S);
        return;
    }
    const double mu0 = step_from_partials(pd, S);
    if (mu0 < 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->reason = QIHT_REASON_STATIONARY;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->mu = mu0;
    const int k = blockIdx.x;  // shrink count of this proposal
    propose<CPT, SEL_STEP>(pd, k, k, shrunk_mu(mu0, a.k * (1.0 - a.c), k), S);
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

template <int BITS, int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_decide(const ProbDev* __restrict__ P,
                                                           SolveArgs a) {
    const ProbDev& pd = P[blockIdx.x];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    if (st->done) return;
    int pick = -1;
    bool capped = false;
    for (int t = 0; t < kSpec; ++t) {
        const CandMeta m = pd.meta[t];
        if (!m.changed) {
            pick = t;
            break;
        }
        double den = 0.0;
        for (int b = threadIdx.x; b < pd.nwg; b += kSelectThreads)
            den += pd.part_om[static_cast<size_t>(t) * pd.nwg + b];
        den = block_sum<kSelectThreads>(den, S.red);
        const double omega = den > 0.0 ? m.dx2 / den : INFINITY;
        if (m.mu <= (1.0 - a.c) * omega) {
            pick = t;
            break;
        }
        if (m.k >= a.max_backtracks) {
            pick = t;
            capped = true;
            break;
        }
    }
    if (pick < 0) {
        // every speculative proposal failed: continue one shrink at a time
        const double shrink = a.k * (1.0 - a.c);
        for (int k = kSpec;; ++k) {
            const double mu = shrunk_mu(st->mu, shrink, k);
            propose<CPT, SEL_STEP>(pd, 0, k, mu, S);
            const CandMeta m = pd.meta[0];
            bool accept = !m.changed;
            if (!accept) {
                const double den = omega_den_block<BITS>(pd, m.dcount, S.red);
                const double omega = den > 0.0 ? m.dx2 / den : INFINITY;
                accept = mu <= (1.0 - a.c) * omega;
                if (!accept && k >= a.max_backtracks) capped = accept = true;
            }
            if (accept) {
                pick = 0;
                break;
            }
            __syncthreads();
        }
    }
    commit_proposal<kSelectThreads>(pd, pick, a, capped);
    for (int b = threadIdx.x; b < 2048; b += kSelectThreads) pd.hist[b] = 0u;
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_hard_threshold(const float* a, int n, int s,
                                                                   int32_t* out, int* err) {
    __shared__ SelShared S;
    for (int w = threadIdx.x; w < (n + 31) / 32; w += kSelectThreads) S.bm_new[w] = 0u;
    if (threadIdx.x == 0) S.changed = 0;
    __syncthreads();
    select_full<CPT, SEL_RAW>(n, s, a, nullptr, nullptr, 0.f, S, err);
    emit_support<SEL_RAW>(n, s, a, nullptr, nullptr, 0.f, nullptr, out, nullptr, S);
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
void launch_decide_b(int cpt, const ProbDev* P, int count, const SolveArgs& a, hipStream_t st) {
#define QIHT_DECIDE(C)                                                                        \
    case C:                                                                                   \
        hipLaunchKernelGGL((k_decide<BITS, C>), dim3(count), dim3(kSelectThreads), 0, st, P, \
                           a);                                                                \
        break;
    QIHT_CPT_SWITCH(cpt, QIHT_DECIDE)
#undef QIHT_DECIDE
}

void launch_decide(int bits, int cpt, const ProbDev* P, int count, const SolveArgs& a,
                   hipStream_t st) {
    switch (bits) {
        case 1: launch_decide_b<1>(cpt, P, count, a, st); break;
        case 2: launch_decide_b<2>(cpt, P, count, a, st); break;
        case 4: launch_decide_b<4>(cpt, P, count, a, st); break;
        case 8: launch_decide_b<8>(cpt, P, count, a, st); break;
        default: launch_decide_b<32>(cpt, P, count, a, st); break;
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
