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
    uint32_t hist2[1024];        // second and third radix digits
    uint32_t hist3[1024];
    uint32_t bm_old[kBmWords];   // current support
    uint32_t bm_new[kBmWords];   // selected set
    uint32_t bm_tie[kBmWords];   // candidates equal to the threshold key
    uint32_t wpre[kBmWords];     // per-word prefix counts
    union {
        struct {                 // fast path: the candidate list
            uint32_t ckey[kCandCap];
            int32_t cidx[kCandCap];
            float cval[kCandCap];  // a_j = x_j + mu g_j
            float cxo[kCandCap];   // x_j (0 off the support)
        } c;
        uint32_t cnt[kSelectThreads];  // full path: per (round, wave) counts
    } u;
    uint32_t scan[16];
    uint32_t bin, krem, ncand, total;
    int changed;
    double red[16];
    double red3[3][16];
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

// Bin of the krem-th largest key of a histogram of NB bins (scanned from
// the top), found by wave 0 alone; every thread gets (S.bin, S.krem) after
// the closing barrier.
template <int NB>
__device__ void find_bin_w0(const uint32_t* hist, uint32_t krem, SelShared& S) {
    constexpr int PER = NB / 64;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int top = NB - 1 - lane * PER;  // this lane: bins top, top-1, ..., top-PER+1
        uint32_t h[PER];
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            h[i] = hist[top - i];
            c += h[i];
        }
        uint32_t x = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        uint32_t run = x - c;
        if (krem > 0 && run < krem && krem <= x) {
            bool found = false;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                if (!found && run < krem && krem <= run + h[i]) {
                    S.bin = static_cast<uint32_t>(top - i);
                    S.krem = krem - run;
                    found = true;
                }
                run += h[i];
            }
        }
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
        if (lane == 0) S.u.cnt[e * 16 + wv] = static_cast<uint32_t>(__popcll(b));
    }
    __syncthreads();
    {
        constexpr int NC = CPT * 16;
        const uint32_t v = tid < NC ? S.u.cnt[tid] : 0u;
        const uint32_t before = block_excl_scan<kSelectThreads>(v, S.scan, nullptr);
        if (tid < NC) S.u.cnt[tid] = before;
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        const bool tie = s > 0 && j < n && key[e] == T;
        const uint64_t b = __ballot(tie);
        const uint32_t rank = S.u.cnt[e * 16 + wv] + static_cast<uint32_t>(__popcll(b & lanemask_lt()));
        if (s > 0 && j < n && (key[e] > T || (tie && rank < need)))
            atomicOr(&S.bm_new[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
}

// Fast path over the support and the histogram candidates; returns false
// (and selects nothing) when the candidate set does not fit in LDS.
// Appends a candidate to the LDS list; one LDS atomic per wave.
__device__ __forceinline__ void push_candidate(bool pred, uint32_t key, int j, float a, float xo,
                                               SelShared& S) {
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
            S.u.c.ckey[c] = key;
            S.u.c.cidx[c] = j;
            S.u.c.cval[c] = a;
            S.u.c.cxo[c] = xo;
        }
    }
}

// Sum of three values over the block, fixed order; every thread gets them.
__device__ void block_sum3(double& a, double& b, double& c, SelShared& S) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if (lane == 0) {
        S.red3[0][wv] = a;
        S.red3[1][wv] = b;
        S.red3[2][wv] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll
    for (int w = 0; w < kSelectThreads / 64; ++w) {
        a += S.red3[0][w];
        b += S.red3[1][w];
        c += S.red3[2][w];
    }
    __syncthreads();
}

// Bitmap words scanned by word_prefix.
enum { BM_TIE = 0, BM_NEW = 1, BM_UNION = 2 };

template <int WHICH>
__device__ __forceinline__ uint32_t bm_word(const SelShared& S, int w) {
    if (WHICH == BM_TIE) return S.bm_tie[w];
    if (WHICH == BM_NEW) return S.bm_new[w];
    return S.bm_old[w] | S.bm_new[w];
}

// Per-word exclusive prefix of popcount(bitmap word) into S.wpre (index
// order), computed by wave 0 alone (no block-wide scan); returns the total.
template <int WHICH>
__device__ uint32_t word_prefix(int words, SelShared& S) {
    constexpr int MAXW = kBmWords / 64;  // words per lane at the largest n
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int wpl = (words + 63) / 64;
        const int w0 = lane * wpl;
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < MAXW; ++i) {
            const int w = w0 + i;
            if (i < wpl && w < words) c += static_cast<uint32_t>(__popc(bm_word<WHICH>(S, w)));
        }
        uint32_t x = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        uint32_t pos = x - c;
#pragma unroll
        for (int i = 0; i < MAXW; ++i) {
            const int w = w0 + i;
            if (i < wpl && w < words) {
                S.wpre[w] = pos;
                pos += static_cast<uint32_t>(__popc(bm_word<WHICH>(S, w)));
            }
        }
        if (lane == 63) S.total = x;
    }
    __syncthreads();
    return S.total;
}

__device__ __forceinline__ uint32_t rank_in_word(uint32_t bits, int b) {
    return static_cast<uint32_t>(__popc(bits & ((1u << b) - 1u)));
}

// Exact top-s of the candidate list (keys desc, ties to lower index) into
// S.bm_new: three radix digits (11, 10, 10 bits) over the candidate keys,
// each a histogram built by all threads and scanned by wave 0; ties at the
// threshold key resolved to the lowest indices by an ordered bitmap scan.
// S.hist, S.hist2, S.hist3 must be zero on entry.
__device__ void rank_candidates(int n, int s, SelShared& S) {
    const int tid = threadIdx.x;
    const uint32_t nc = S.ncand;
    if (s <= 0) return;
    for (uint32_t c = tid; c < nc; c += kSelectThreads) atomicAdd(&S.hist[S.u.c.ckey[c] >> 20], 1u);
    __syncthreads();
    find_bin_w0<2048>(S.hist, static_cast<uint32_t>(s), S);
    const uint32_t b1 = S.bin, k1 = S.krem;
    for (uint32_t c = tid; c < nc; c += kSelectThreads) {
        const uint32_t k = S.u.c.ckey[c];
        if ((k >> 20) == b1) atomicAdd(&S.hist2[(k >> 10) & 1023u], 1u);
    }
    __syncthreads();
    find_bin_w0<1024>(S.hist2, k1, S);
    const uint32_t p2 = (b1 << 10) | S.bin, k2 = S.krem;
    for (uint32_t c = tid; c < nc; c += kSelectThreads) {
        const uint32_t k = S.u.c.ckey[c];
        if ((k >> 10) == p2) atomicAdd(&S.hist3[k & 1023u], 1u);
    }
    __syncthreads();
    find_bin_w0<1024>(S.hist3, k2, S);
    const uint32_t T = (p2 << 10) | S.bin;  // the s-th largest key
    const uint32_t need = S.krem;           // keys equal to T that are taken
    int ties = 0;
    for (uint32_t c = tid; c < nc; c += kSelectThreads) {
        const uint32_t k = S.u.c.ckey[c];
        const int j = S.u.c.cidx[c];
        if (k > T) atomicOr(&S.bm_new[j >> 5], 1u << (j & 31));
        else if (k == T) {
            atomicOr(&S.bm_tie[j >> 5], 1u << (j & 31));
            ties = 1;
        }
    }
    (void)ties;
    __syncthreads();
    const uint32_t nties = S.hist3[T & 1023u];
    if (need >= nties) {
        // every tie is taken (the usual case): no ordering needed
        const int words = (n + 31) / 32;
        for (int w = tid; w < words; w += kSelectThreads) S.bm_new[w] |= S.bm_tie[w];
        __syncthreads();
        return;
    }
    const int words = (n + 31) / 32;
    word_prefix<BM_TIE>(words, S);
    for (int w = tid; w < words; w += kSelectThreads) {
        uint32_t u = S.bm_tie[w];
        uint32_t rank = S.wpre[w];
        while (u) {
            const int b = __ffs(u) - 1;
            u &= u - 1;
            if (rank < need) atomicOr(&S.bm_new[w], 1u << b);
            ++rank;
        }
    }
    __syncthreads();
}

// One complete proposal.  SEL_INIT writes the initial support (pd.sup, xs,
// bmsup); SEL_STEP writes proposal `slot` (support, values, difference list,
// metadata).  Every global input is loaded before the first barrier.
// With from_partials the step is mu = mu0 / (k(1-c))^k with mu0 finished
// here from the gather partials (written to *mu0_out); returns false when
// the iteration is stationary.
template <int CPT, int MODE>
__device__ bool propose(const ProbDev& pd, int slot, int k, double mu_in, bool from_partials,
                        double shrink, double* mu0_out, SelShared& S) {
    const int tid = threadIdx.x;
    const int n = pd.n, s = pd.s;
    const int words = (n + 31) / 32;
    const int nsup = (MODE == SEL_STEP) ? s : 0;
    // ---- loads (all independent)
    float gv[CPT];
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
        const int j = tid + kSelectThreads * e;
        gv[e] = j < n ? pd.g[j] : 0.0f;
    }
    const bool sreg = tid < nsup;  // first 1024 support entries in registers
    const int sj = sreg ? pd.sup[tid] : 0;
    const float sx = sreg ? pd.xs[tid] : 0.0f;
    const float sg = sreg ? pd.gs[tid] : 0.0f;
    double gg = 0.0, uv = 0.0, uu = 0.0;
    if (from_partials) {
        gg = static_cast<double>(sg) * static_cast<double>(sg);
        for (int i = tid + kSelectThreads; i < nsup; i += kSelectThreads) {
            const double v = static_cast<double>(pd.gs[i]);
            gg += v * v;
        }
        for (int b = tid; b < pd.nwg; b += kSelectThreads) {
            uv += pd.part_mu[2 * b + 0];
            uu += pd.part_mu[2 * b + 1];
        }
    }
    for (int b = tid; b < 2048; b += kSelectThreads) S.hist[b] = pd.hist[b];
    for (int b = tid; b < 1024; b += kSelectThreads) {
        S.hist2[b] = 0u;
        S.hist3[b] = 0u;
    }
    for (int w = tid; w < words; w += kSelectThreads) {
        S.bm_old[w] = (MODE == SEL_STEP) ? pd.bmsup[w] : 0u;
        S.bm_new[w] = 0u;
        S.bm_tie[w] = 0u;
    }
    if (tid == 0) {
        S.ncand = 0;
        S.changed = 0;
    }
    // ---- the step
    double mu = mu_in;
    if (from_partials) {
        block_sum3(gg, uv, uu, S);
        double den = uv;
        if (!(den > 0.0) || !isfinite(den)) den = uu;
        if (!(gg > 0.0) || !(den > 0.0) || !isfinite(gg / den)) return false;
        *mu0_out = gg / den;
        mu = shrunk_mu(gg / den, shrink, k);
    } else {
        __syncthreads();
    }
    const float muf = static_cast<float>(mu);
    // ---- threshold from the off-support histogram
    bool fast = true;
    float thr = 0.0f;
    if (n - nsup > s) {
        find_bin_w0<2048>(S.hist, static_cast<uint32_t>(s), S);
        thr = __uint_as_float(S.bin << 20) * (1.0f - 0x1p-20f);
        fast = thr >= 0x1p-100f;  // keep clear of subnormal products
    }
    for (int b = tid; b < 2048; b += kSelectThreads) S.hist[b] = 0u;
    int bad = 0;
    if (fast) {
        {
            const float a = fmaf(muf, sg, sx);
            const uint32_t key = abs_key(a);
            if (sreg && key > 0x7F800000u) bad = 1;
            push_candidate(sreg, key, sj, a, sx, S);
        }
        for (int i0 = kSelectThreads; i0 < nsup; i0 += kSelectThreads) {
            const int i = i0 + tid;
            const bool in = i < nsup;
            const int j = in ? pd.sup[i] : 0;
            const float xo = in ? pd.xs[i] : 0.0f;
            const float a = in ? fmaf(muf, pd.gs[i], xo) : 0.0f;
            const uint32_t key = abs_key(a);
            if (in && key > 0x7F800000u) bad = 1;
            push_candidate(in, key, j, a, xo, S);
        }
        // off the support: which of this thread's entries pass the
        // threshold (a bit mask), one LDS atomic per wave for the slots
        uint64_t cm = 0;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int j = tid + kSelectThreads * e;
            const bool in = j < n && fabsf(gv[e]) >= thr && !((S.bm_old[j >> 5] >> (j & 31)) & 1u);
            cm |= static_cast<uint64_t>(in) << e;
        }
        const uint32_t cnt = static_cast<uint32_t>(__popcll(cm));
        const int lane = tid & 63;
        uint32_t x = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        uint32_t base = 0;
        if (lane == 63 && x > 0) base = atomicAdd(&S.ncand, x);
        base = __shfl(base, 63, 64) + (x - cnt);
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            if ((cm >> e) & 1ull) {
                const int j = tid + kSelectThreads * e;
                // off the support x_j = 0, so a_j = fma(mu, g_j, 0)
                const float a = (MODE == SEL_STEP) ? fmaf(muf, gv[e], 0.0f) : gv[e];
                const uint32_t key = abs_key(a);
                if (key > 0x7F800000u) bad = 1;
                if (base < static_cast<uint32_t>(kCandCap)) {
                    S.u.c.ckey[base] = key;
                    S.u.c.cidx[base] = j;
                    S.u.c.cval[base] = a;
                    S.u.c.cxo[base] = 0.0f;
                }
                ++base;
            }
        }
    }
    __syncthreads();
    fast = fast && S.ncand <= static_cast<uint32_t>(kCandCap);
    if (bad) atomicOr(&pd.st->err, 1);
    if (!fast) {
        // ---- full path: every key
        if (tid == 0) atomicAdd(&pd.st->full_selects, 1);
        select_full<CPT, MODE>(n, s, nullptr, pd.g, pd.x, muf, S, &pd.st->err);
        if (MODE == SEL_INIT) {
            emit_support<MODE>(n, s, nullptr, pd.g, nullptr, muf, nullptr, pd.sup, nullptr, S);
            for (int w = tid; w < words; w += kSelectThreads) pd.bmsup[w] = S.bm_new[w];
            for (int i = tid; i < s; i += kSelectThreads) pd.xs[i] = 0.0f;
            for (int b = tid; b < 2048; b += kSelectThreads) pd.hist[b] = 0u;
            __syncthreads();
            return true;
        }
        int32_t* out_sup = pd.csup + static_cast<size_t>(slot) * s;
        float* out_val = pd.cval + static_cast<size_t>(slot) * s;
        emit_support<MODE>(n, s, nullptr, pd.g, pd.x, muf, pd.sup, out_sup, out_val, S);
        // difference list from global values (rare path)
        const uint32_t total = word_prefix<BM_UNION>(words, S);
        int32_t* dlist = pd.dlist + static_cast<size_t>(slot) * 2 * s;
        double* dw = pd.dw + static_cast<size_t>(slot) * 2 * s;
        double dx2 = 0.0, xn2 = 0.0, zero = 0.0;
        for (int w = tid; w < words; w += kSelectThreads) {
            uint32_t u = S.bm_old[w] | S.bm_new[w];
            uint32_t pos = S.wpre[w];
            while (u) {
                const int b = __ffs(u) - 1;
                u &= u - 1;
                const int j = w * 32 + b;
                const float xo = pd.x[j];
                const float xn = ((S.bm_new[w] >> b) & 1u) ? fmaf(muf, pd.g[j], xo) : 0.0f;
                const double d = static_cast<double>(xn) - static_cast<double>(xo);
                if (pos < static_cast<uint32_t>(2 * s)) {
                    dlist[pos] = j;
                    dw[pos] = d;
                }
                ++pos;
                dx2 += d * d;
                xn2 += static_cast<double>(xn) * static_cast<double>(xn);
            }
        }
        block_sum3(dx2, xn2, zero, S);
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
        return true;
    }
    // ---- fast path: rank the candidates, then emit from LDS
    rank_candidates(n, s, S);
    const uint32_t nc = S.ncand;
    if (MODE == SEL_INIT) {
        word_prefix<BM_NEW>(words, S);
        for (uint32_t c = tid; c < nc; c += kSelectThreads) {
            const int j = S.u.c.cidx[c];
            const int w = j >> 5, b = j & 31;
            if ((S.bm_new[w] >> b) & 1u) {
                const uint32_t pos = S.wpre[w] + rank_in_word(S.bm_new[w], b);
                if (pos < static_cast<uint32_t>(s)) {
                    pd.sup[pos] = j;
                    pd.xs[pos] = 0.0f;
                }
            }
        }
        for (int w = tid; w < words; w += kSelectThreads) pd.bmsup[w] = S.bm_new[w];
        // the next full pass rebuilds the histogram off the new support
        for (int b = tid; b < 2048; b += kSelectThreads) pd.hist[b] = 0u;
        __syncthreads();
        return true;
    }
    int32_t* out_sup = pd.csup + static_cast<size_t>(slot) * s;
    float* out_val = pd.cval + static_cast<size_t>(slot) * s;
    int32_t* dlist = pd.dlist + static_cast<size_t>(slot) * 2 * s;
    double* dw = pd.dw + static_cast<size_t>(slot) * 2 * s;
    // changed: the selection bitmap differs from the support bitmap
    {
        int diff = 0;
        for (int w = tid; w < words; w += kSelectThreads) diff |= (S.bm_new[w] != S.bm_old[w]);
        if (diff) S.changed = 1;
    }
    word_prefix<BM_NEW>(words, S);
    for (uint32_t c = tid; c < nc; c += kSelectThreads) {
        const int j = S.u.c.cidx[c];
        const int w = j >> 5, b = j & 31;
        if ((S.bm_new[w] >> b) & 1u) {
            const uint32_t pos = S.wpre[w] + rank_in_word(S.bm_new[w], b);
            if (pos < static_cast<uint32_t>(s)) {
                out_sup[pos] = j;
                out_val[pos] = S.u.c.cval[c];
            }
        }
    }
    __syncthreads();
    // difference list over the union of old and new supports, ascending;
    // every member of the union is exactly one candidate
    const uint32_t total = word_prefix<BM_UNION>(words, S);
    double dx2 = 0.0, xn2 = 0.0, zero = 0.0;
    for (uint32_t c = tid; c < nc; c += kSelectThreads) {
        const int j = S.u.c.cidx[c];
        const int w = j >> 5, b = j & 31;
        const uint32_t uw = S.bm_old[w] | S.bm_new[w];
        if ((uw >> b) & 1u) {
            const uint32_t pos = S.wpre[w] + rank_in_word(uw, b);
            const float xo = S.u.c.cxo[c];
            const float xn = ((S.bm_new[w] >> b) & 1u) ? S.u.c.cval[c] : 0.0f;
            const double d = static_cast<double>(xn) - static_cast<double>(xo);
            if (pos < static_cast<uint32_t>(2 * s)) {
                dlist[pos] = j;
                dw[pos] = d;
            }
            dx2 += d * d;
            xn2 += static_cast<double>(xn) * static_cast<double>(xn);
        }
    }
    block_sum3(dx2, xn2, zero, S);
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
    return true;
}

template <int CPT>
__global__ __launch_bounds__(kSelectThreads) void k_propose(const ProbDev* __restrict__ P,
                                                            SolveArgs a, int mode) {
    const ProbDev& pd = P[blockIdx.y];
    SolveState* st = pd.st;
    __shared__ SelShared S;
    if (st->done) return;
    double mu0 = 0.0;
    if (mode == SEL_INIT) {
        propose<CPT, SEL_INIT>(pd, 0, 0, 1.0, false, 1.0, &mu0, S);
        return;
    }
    const int k = blockIdx.x;  // shrink count of this proposal
    const bool ok = propose<CPT, SEL_STEP>(pd, k, k, 0.0, true, a.k * (1.0 - a.c), &mu0, S);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok) {
            st->mu = mu0;
        } else {
            st->done = 1;
            st->reason = QIHT_REASON_STATIONARY;
        }
    }
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
            double unused = 0.0;
            propose<CPT, SEL_STEP>(pd, 0, k, mu, false, shrink, &unused, S);
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
