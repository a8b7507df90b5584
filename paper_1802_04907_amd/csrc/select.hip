// H_s proposals and the step-size test of the QIHT iteration (Sec. I-A hard
// threshold; Sec. II-A and Algorithm 2: normalized step, support-change
// test, shrinking by k(1-c)).
//
// k_propose: one workgroup per proposal x'_k = H_s(x + mu_k g) with
// mu_k = mu / (k(1-c))^k, k = base_k .. base_k + kSpec-1 side by side
// (speculative backtracking).  Each workgroup first finishes mu = |g_G|^2 / (Q1_G g_G).
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
// The step-size test itself (decide_pick) and the commit run in the next
// residual gather, so no launch of its own sits between two iterations; a
// round whose proposals all fail is followed by one that proposes the next
// kSpec shrinks (base_k) from the same x.
#include "solve_common.h"

namespace qiht {
namespace {


// LDS of a proposal workgroup; NMAX bounds the entries the full path ranks
// (its bitmaps and tie counts), and with it the workgroup's LDS: the
// 65536-entry instance leaves room for two workgroups per CU.
template <int NMAX>
struct SelShared {
    static constexpr int kNMax = NMAX;
    static constexpr int kBmWords = NMAX / 32;
    uint32_t hist[2048];
    uint32_t hist2[1024];        // second and third radix digits
    uint32_t hist3[1024];
    union {
        struct {                 // fast path: the candidates in index order
            uint32_t mkey[kCandCap];  //   |a_j| as FP32 bits
            uint32_t midx[kCandCap];  //   j, bit 31 when on the support
            float mval[kCandCap];     //   a_j
            float mxo[kCandCap];      //   x_j
        } f;
        struct {                 // full path: bitmaps over all n
            uint32_t bm_old[kBmWords];   // current support
            uint32_t bm_new[kBmWords];   // selected set
            uint32_t wpre[kBmWords];     // per-word prefix counts (scratch before)
            uint32_t cnt[NMAX / 64];     // threshold ties per wave and round
        } b;
    } u;
    uint32_t scan[16];
    uint32_t flg[16];
    uint32_t bin, krem, total, nc;
    int changed, bad, full, dn;
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
    if (MODE == SEL_RAW) return ldg_f32(a_in + j);
    if (MODE == SEL_INIT) return ldg_f32(g + j);
    return fmaf(muf, ldg_f32(g + j), ldg_f32(x + j));
}

// Rank key of index j: |a_j| as FP32 bits, or with group > 0 (a complex
// unknown whose real and imaginary parts are columns j and j + group) the
// squared modulus a_j^2 + a_{j+group}^2 summed in FP64 from the FP32 parts and
// rounded once to FP32 (non-negative: the bits order as the values).
template <int MODE>
__device__ __forceinline__ uint32_t key_at(const float* a_in, const float* g, const float* x, float muf,
                                           int j, int group) {
    if (group == 0) return abs_key(value_at<MODE>(a_in, g, x, muf, j));
    const double u = value_at<MODE>(a_in, g, x, muf, j);
    const double v = value_at<MODE>(a_in, g, x, muf, j + group);
    return abs_key(static_cast<float>(u * u + v * v));
}

// One radix digit step: bins of `hist` (nb bins, counts already in place)
// scanned from the top; finds the bin holding the krem-th largest key.
template <class SS>
__device__ void find_bin(SS& S, int nb, uint32_t& prefix, uint32_t& krem, int width) {
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
template <int NB, class SS>
__device__ void find_bin_w0(const uint32_t* hist, uint32_t krem, SS& S) {
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
        const uint32_t x = wave_incl_scan(c);
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
template <int MODE, class SS>
__device__ void emit_support(int n, int s, const float* a_in, const float* g, const float* x,
                             float muf, const int32_t* old_sup, int32_t* out_sup, float* out_val,
                             SS& S) {
    const int tid = threadIdx.x;
    const int words = (n + 31) / 32;
    const int wpt = (words + kSelectThreads - 1) / kSelectThreads;
    const int w0 = tid * wpt;
    uint32_t c = 0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) c += __popc(S.u.b.bm_new[w]);
    uint32_t pos = block_excl_scan<kSelectThreads>(c, S.scan, nullptr);
    int changed = 0;
    for (int w = w0; w < min(words, w0 + wpt); ++w) {
        uint32_t u = S.u.b.bm_new[w];
        while (u) {
            const int b = __ffs(u) - 1;
            u &= u - 1;
            const int j = w * 32 + b;
            if (pos < static_cast<uint32_t>(s)) {
                stg(out_sup + pos, static_cast<int32_t>(j));
                if (MODE == SEL_STEP) {
                    stg(out_val + pos, value_at<MODE>(a_in, g, x, muf, j));
                    if (ldg_i32(old_sup + pos) != j) changed = 1;
                }
            }
            ++pos;
        }
    }
    if (changed) S.changed = 1;
    __syncthreads();
}

// Rank over all n keys: the full path (and plain H_s).  Thread t visits
// t, t + 1024, ...; the keys are recomputed from the inputs on every radix
// pass instead of being held in registers, which keeps this rarely taken path
// from inflating the register budget of the fast path it shares a kernel
// with.  Sets the selection bitmap S.u.b.bm_new.
template <int MODE, class SS>
__device__ void select_full(int n, int s, const float* a_in, const float* g, const float* x,
                            float muf, SS& S, int* err, int group = 0) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int rounds = (n + kSelectThreads - 1) / kSelectThreads;  // <= 256
    int bad = 0;
    uint32_t prefix = 0, krem = static_cast<uint32_t>(s);
    for (int pass = 0; pass < 3; ++pass) {
        const int width = pass == 0 ? 11 : 10;
        const int sh = pass == 0 ? 20 : (pass == 1 ? 10 : 0);
        const int nb = 1 << width;
        const int hsh = sh + width;
        for (int b = tid; b < 2048; b += kSelectThreads) S.hist[b] = 0u;
        __syncthreads();
        if (krem > 0) {
            for (int e = 0; e < rounds; ++e) {
                const int j = tid + kSelectThreads * e;
                if (j < n) {
                    const uint32_t key = key_at<MODE>(a_in, g, x, muf, j, group);
                    if (pass == 0 && key > 0x7F800000u) bad = 1;
                    if (pass == 0 || (key >> hsh) == prefix)
                        atomicAdd(&S.hist[(key >> sh) & (nb - 1)], 1u);
                }
            }
        }
        __syncthreads();
        find_bin(S, nb, prefix, krem, width);
    }
    if (bad) atomicOr(err, 1);
    const uint32_t T = prefix;
    const uint32_t need = krem;
    // ties at T ranked in index order: (round, wave, lane) is index order
    for (int e = 0; e < rounds; ++e) {
        const int j = tid + kSelectThreads * e;
        const bool tie = s > 0 && j < n && key_at<MODE>(a_in, g, x, muf, j, group) == T;
        const uint64_t b = __ballot(tie);
        if (lane == 0) S.u.b.cnt[e * 16 + wv] = static_cast<uint32_t>(__popcll(b));
    }
    __syncthreads();
    {
        // exclusive prefix of the nc counts, CPT consecutive ones per thread
        constexpr int CPT = SS::kNMax / 64 / kSelectThreads;
        const int nc = rounds * 16;
        uint32_t v[CPT], sum = 0;
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int c = CPT * tid + i;
            v[i] = c < nc ? S.u.b.cnt[c] : 0u;
            sum += v[i];
        }
        uint32_t before = block_excl_scan<kSelectThreads>(sum, S.scan, nullptr);
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int c = CPT * tid + i;
            if (c < nc) S.u.b.cnt[c] = before;
            before += v[i];
        }
        __syncthreads();
    }
    for (int e = 0; e < rounds; ++e) {
        const int j = tid + kSelectThreads * e;
        const uint32_t key = j < n ? key_at<MODE>(a_in, g, x, muf, j, group) : 0u;
        const bool tie = s > 0 && j < n && key == T;
        const uint64_t b = __ballot(tie);
        const uint32_t rank = S.u.b.cnt[e * 16 + wv] + static_cast<uint32_t>(__popcll(b & lanemask_lt()));
        if (s > 0 && j < n && (key > T || (tie && rank < need)))
            atomicOr(&S.u.b.bm_new[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
}

// Complex unknowns: the selection bitmap over the `group` entries (bm_new)
// becomes one over the 2 group real columns, entry p selecting columns p and
// p + group (wpre is the scratch; its prefix counts come later).
template <class SS>
__device__ void expand_group(int group, SS& S) {
    const int words = (2 * group + 31) / 32;
    for (int w = threadIdx.x; w < words; w += kSelectThreads) {
        uint32_t bits = 0u;
        for (int b = 0; b < 32; ++b) {
            const int j = 32 * w + b;
            if (j >= 2 * group) break;
            const int p = j < group ? j : j - group;
            bits |= ((S.u.b.bm_new[p >> 5] >> (p & 31)) & 1u) << b;
        }
        S.u.b.wpre[w] = bits;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < words; w += kSelectThreads) S.u.b.bm_new[w] = S.u.b.wpre[w];
    __syncthreads();
}

// Sum of three values over the block, fixed order; every thread gets them.
template <class SS>
__device__ void block_sum3(double& a, double& b, double& c, SS& S) {
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

// Three block sums (per wave, then over the waves in wave order, as
// block_sum3), the exclusive prefix of v in thread order with its total,
// and the number of threads with f set, over one barrier.  Every thread
// gets the results; S.red3, S.scan and S.flg must not be read again before
// a later barrier (their next writer follows at least one more barrier).
struct BlockAgg {
    double a, b, c;
    uint32_t before, total, nf;
};

template <class SS>
__device__ BlockAgg block_sums_scan(double a, double b, double c, uint32_t v, bool f, SS& S) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const uint32_t x = wave_incl_scan(v);
    const uint32_t nf = static_cast<uint32_t>(__popcll(__ballot(f)));
    if (lane == 63) {
        S.red3[0][wv] = a;
        S.red3[1][wv] = b;
        S.red3[2][wv] = c;
        S.scan[wv] = x;
        S.flg[wv] = nf;
    }
    __syncthreads();
    BlockAgg r{0.0, 0.0, 0.0, 0u, 0u, 0u};
#pragma unroll
    for (int w = 0; w < kSelectThreads / 64; ++w) {
        r.a += S.red3[0][w];
        r.b += S.red3[1][w];
        r.c += S.red3[2][w];
        const uint32_t t = S.scan[w];
        r.before += w < wv ? t : 0u;
        r.total += t;
        r.nf += S.flg[w];
    }
    r.before += x - v;
    return r;
}

// Bitmap words scanned by word_prefix.
enum { BM_NEW = 1, BM_UNION = 2 };

template <int WHICH, class SS>
__device__ __forceinline__ uint32_t bm_word(const SS& S, int w) {
    if (WHICH == BM_NEW) return S.u.b.bm_new[w];
    return S.u.b.bm_old[w] | S.u.b.bm_new[w];
}

// Per-word exclusive prefix of popcount(bitmap word) into S.u.b.wpre (index
// order), computed by wave 0 alone (no block-wide scan); returns the total.
template <int WHICH, class SS>
__device__ uint32_t word_prefix(int words, SS& S) {
    constexpr int MAXW = SS::kBmWords / 64;  // words per lane at the largest n
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int wpl = (words + 63) / 64;
        const int w0 = lane * wpl;
        uint32_t c = 0;
#pragma unroll 8
        for (int i = 0; i < MAXW; ++i) {
            const int w = w0 + i;
            if (i < wpl && w < words) c += static_cast<uint32_t>(__popc(bm_word<WHICH>(S, w)));
        }
        const uint32_t x = wave_incl_scan(c);
        uint32_t pos = x - c;
#pragma unroll 8
        for (int i = 0; i < MAXW; ++i) {
            const int w = w0 + i;
            if (i < wpl && w < words) {
                S.u.b.wpre[w] = pos;
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

// Rank step of the fast path: the s largest keys of the merged candidates
// (ties to the lower index).  Radix digits of 11, 10 and 10 bits in LDS
// histograms, stopping as soon as the bin holding the s-th largest key is
// taken whole; the selection rule is then (key >> sh) > P, or == P within
// the first `need` such entries in index order.  S.hist, hist2, hist3 must
// be zero on entry.
template <class SS>
__device__ void rank_merged(int nc, int s, SS& S, int& sh, uint32_t& P, uint32_t& need,
                            uint32_t& eq) {
    const int tid = threadIdx.x;
    for (int c = tid; c < nc; c += kSelectThreads) atomicAdd(&S.hist[S.u.f.mkey[c] >> 20], 1u);
    __syncthreads();
    find_bin_w0<2048>(S.hist, static_cast<uint32_t>(s), S);
    P = S.bin;
    need = S.krem;
    eq = S.hist[P];
    sh = 20;
    if (need == eq) return;
    for (int c = tid; c < nc; c += kSelectThreads) {
        const uint32_t k = S.u.f.mkey[c];
        if ((k >> 20) == P) atomicAdd(&S.hist2[(k >> 10) & 1023u], 1u);
    }
    __syncthreads();
    find_bin_w0<1024>(S.hist2, need, S);
    P = (P << 10) | S.bin;
    need = S.krem;
    eq = S.hist2[S.bin];
    sh = 10;
    if (need == eq) return;
    for (int c = tid; c < nc; c += kSelectThreads) {
        const uint32_t k = S.u.f.mkey[c];
        if ((k >> 10) == P) atomicAdd(&S.hist3[k & 1023u], 1u);
    }
    __syncthreads();
    find_bin_w0<1024>(S.hist3, need, S);
    P = (P << 10) | S.bin;
    need = S.krem;
    eq = S.hist3[S.bin];
    sh = 0;
}

// One complete proposal.  SEL_INIT writes the initial support (pd.sup, xs,
// bmsup); SEL_STEP writes proposal `slot` (support, values, difference list,
// metadata).  With from_partials the step is mu = mu0 / (k(1-c))^k with mu0
// finished here from the gather partials (written to *mu0_out); returns
// false when the iteration is stationary.
//
// Fast path: the candidates are the support (ascending, with x and g on it)
// and the off-support list of compact_candidates (ascending per index block);
// both are merged into one list in index order, ranked, and the outputs
// (support, values, difference list) are positions of a prefix sum over that
// order.  Full path (too many candidates, or a threshold the fast path cannot
// use): every key of the n in registers and bitmaps over all n.
template <int MODE, class SS>
__device__ bool propose(const ProbDev& pd, int slot, int k, double mu_in, bool from_partials,
                        double shrink, double* mu0_out, SS& S, bool* skipped = nullptr) {
    constexpr int MPT = kCandCap / kSelectThreads;  // merged positions per thread
    constexpr int PRE = 4;                          // candidates loaded ahead per thread
    const int tid = threadIdx.x;
    const int n = pd.n, s = pd.s, nw = pd.npart;
    const int words = (n + 31) / 32;
    const int nsup = (MODE == SEL_STEP) ? s : 0;
    const int per = (n + nw - 1) / nw;
    // ---- loads (one round trip): mu partials, the candidate counts of this
    // thread's index blocks [t cpw, (t + 1) cpw), and the first PRE
    // candidates of its first block
    // (with `skipped`, the solve's stop flag is read alongside these loads
    // and an already finished problem returns at the first barrier, before
    // writing any global memory)
    const int done_now = skipped ? ldg_i32(&pd.st->done) : 0;
    // Every load of this first round trip is issued before any is used, with
    // its index clamped into its array (a clamped load's value is not used):
    // a load used inside a loop or a branch is waited for before the next
    // one goes out.
    double gg = 0.0, uv = 0.0, uu = 0.0;
    float gs0 = 0.0f;
    double pm0 = 0.0, pm1 = 0.0;
    if (from_partials) {
        gs0 = ldg_f32(pd.gs + min(tid, max(nsup - 1, 0)));
        const int b0 = min(tid, nw - 1);
        pm0 = ldg_f64(pd.part_mu + 2 * b0 + 0);
        pm1 = ldg_f64(pd.part_mu + 2 * b0 + 1);
    }
    // Few index blocks: G = 2 or 4 threads share one, thread gq of the group
    // taking its entries gq, gq + G, ... (so PRE G of them arrive with the
    // first loads); many: each thread takes cpw whole blocks.
    const int G = 4 * nw <= kSelectThreads ? 4 : (2 * nw <= kSelectThreads ? 2 : 1);
    const int cpw = G > 1 ? 1 : (nw + kSelectThreads - 1) / kSelectThreads;
    const int gq = tid % G;
    const int w0 = (tid / G) * cpw, w1 = min(nw, w0 + cpw);
    uint32_t pidx[PRE];
    float2 pgx[PRE];
    const int lo0 = w0 * per, len0 = w0 < w1 ? min(n, lo0 + per) - lo0 : 0;
#pragma unroll
    for (int i = 0; i < PRE; ++i) {
        const int at = min(lo0 + min(gq + G * i, max(len0 - 1, 0)), n - 1);
        pidx[i] = ldg_u32(pd.cidx + at);
        pgx[i] = ldg_f2(pd.cgx + at);
    }
    const int cw0 = ldg_i32(pd.ccnt + min(w0, nw - 1));
    if (from_partials) {
        if (tid < nsup) gg += static_cast<double>(gs0) * static_cast<double>(gs0);
        for (int i = tid + kSelectThreads; i < nsup; i += kSelectThreads) {
            const double v = static_cast<double>(ldg_f32(pd.gs + i));
            gg += v * v;
        }
        if (tid < nw) {
            uv += pm0;
            uu += pm1;
        }
        for (int b = tid + kSelectThreads; b < nw; b += kSelectThreads) {
            uv += ldg_f64(pd.part_mu + 2 * b + 0);
            uu += ldg_f64(pd.part_mu + 2 * b + 1);
        }
    }
    uint32_t mycnt = 0;  // (counted by the group's first thread)
    int c0 = 0, bad_cnt = 0;
    if (w0 < w1) {
        c0 = cw0;
        if (cw0 < 0) bad_cnt = 1;
        else if (gq == 0) mycnt += static_cast<uint32_t>(cw0);
    }
    for (int w = w0 + 1; w < w1; ++w) {
        const int c = ldg_i32(pd.ccnt + w);
        if (c < 0) bad_cnt = 1;
        else if (gq == 0) mycnt += static_cast<uint32_t>(c);
    }
    for (int b = tid; b < 2048; b += kSelectThreads) S.hist[b] = 0u;
    for (int b = tid; b < 1024; b += kSelectThreads) {
        S.hist2[b] = 0u;
        S.hist3[b] = 0u;
    }
    if (tid == 0) {
        S.changed = 0;
        S.bad = 0;
        S.dn = done_now;  // (workgroup 0 of the same launch may stop the problem
                          // while this one runs: thread 0's reading decides)
    }
    // ---- the step, and this thread's place in the candidate list
    const BlockAgg ag = block_sums_scan(gg, uv, uu, mycnt, bad_cnt != 0, S);
    if (S.dn) {  // uniform over the workgroup
        *skipped = true;
        return false;
    }
    double mu = mu_in;
    if (from_partials) {
        double den = ag.b;
        if (!(den > 0.0) || !isfinite(den)) den = ag.c;
        if (!(ag.a > 0.0) || !(den > 0.0) || !isfinite(ag.a / den)) return false;
        *mu0_out = ag.a / den;
        mu = shrunk_mu(ag.a / den, shrink, k);
    }
    const float muf = static_cast<float>(mu);
    // the group's first thread counted the block: it starts c0 before the others
    const uint32_t obase = ag.before - (gq > 0 ? static_cast<uint32_t>(max(c0, 0)) : 0u);
    const int nc = static_cast<int>(ag.total);
    // (the list holds at least s entries unless the counts are inconsistent,
    // which the full path then handles)
    // (complex unknowns rank entry moduli: always the full path)
    const bool fast = ag.nf == 0 && nc <= kCandCap && nc >= s && pd.group == 0;
    int32_t* out_sup = (MODE == SEL_INIT) ? pd.sup : pd.csup + static_cast<size_t>(slot) * s;
    float* out_val = pd.cval + static_cast<size_t>(slot) * s;
    int32_t* dlist = pd.dlist + static_cast<size_t>(slot) * 2 * s;
    double* dw = pd.dw + static_cast<size_t>(slot) * 2 * s;
    if (!fast) {
        // ---- full path: every key
        for (int w = tid; w < words; w += kSelectThreads) {
            S.u.b.bm_old[w] = (MODE == SEL_STEP) ? ldg_u32(pd.bmsup + w) : 0u;
            S.u.b.bm_new[w] = 0u;
        }
        __syncthreads();
        if (tid == 0) atomicAdd(&pd.st->full_selects, 1);
        if (pd.group > 0) {
            // s / 2 complex entries ranked by modulus, then their 2 columns each
            select_full<MODE>(pd.group, s / 2, nullptr, pd.g, pd.x, muf, S, &pd.st->err, pd.group);
            expand_group(pd.group, S);
        } else {
            select_full<MODE>(n, s, nullptr, pd.g, pd.x, muf, S, &pd.st->err);
        }
        if (MODE == SEL_INIT) {
            emit_support<MODE>(n, s, nullptr, pd.g, nullptr, muf, nullptr, pd.sup, nullptr, S);
            for (int w = tid; w < words; w += kSelectThreads) pd.bmsup[w] = S.u.b.bm_new[w];
            for (int i = tid; i < s; i += kSelectThreads) pd.xs[i] = 0.0f;
            for (int b = tid; b < 2048; b += kSelectThreads) pd.hist[b] = 0u;
            __syncthreads();
            return true;
        }
        emit_support<MODE>(n, s, nullptr, pd.g, pd.x, muf, pd.sup, out_sup, out_val, S);
        const uint32_t total = word_prefix<BM_UNION>(words, S);
        double dx2 = 0.0, xn2 = 0.0, zero = 0.0;
        for (int w = tid; w < words; w += kSelectThreads) {
            uint32_t u = S.u.b.bm_old[w] | S.u.b.bm_new[w];
            uint32_t pos = S.u.b.wpre[w];
            while (u) {
                const int b = __ffs(u) - 1;
                u &= u - 1;
                const int j = w * 32 + b;
                const float xo = ldg_f32(pd.x + j);
                const float xn = ((S.u.b.bm_new[w] >> b) & 1u) ? fmaf(muf, ldg_f32(pd.g + j), xo) : 0.0f;
                const double d = static_cast<double>(xn) - static_cast<double>(xo);
                if (pos < static_cast<uint32_t>(2 * s)) {
                    stg(dlist + pos, static_cast<int32_t>(j));
                    stg(dw + pos, d);
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
            store_meta(pd.meta + slot, m);
        }
        __syncthreads();
        return true;
    }

    // ---- fast path: the candidates into LDS in index order, with their keys
    int bad = 0;
    {
        // a_j = x_j + mu g_j (off the support x_j = 0; SEL_INIT: a_j = g_j)
        auto put = [&](uint32_t pos, uint32_t mi, float2 gx) {
            const float a = (MODE == SEL_STEP) ? fmaf(muf, gx.x, gx.y) : gx.x;
            const uint32_t key = abs_key(a);
            if (key > 0x7F800000u) bad = 1;
            S.u.f.mkey[pos] = key;
            S.u.f.midx[pos] = mi;
            S.u.f.mval[pos] = a;
            S.u.f.mxo[pos] = gx.y;
        };
        // a block's entries i0, i0 + step, ... below c in batches whose
        // loads are issued together (clamped into the block, the extra ones
        // not stored)
        auto put_block = [&](uint32_t at, int lo, int i0, int c, int step) {
            constexpr int B = 4;
            for (int ib = i0; ib < c; ib += B * step) {
                uint32_t ti[B];
                float2 tg[B];
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    const int i = min(ib + q * step, c - 1);
                    ti[q] = ldg_u32(pd.cidx + lo + i);
                    tg[q] = ldg_f2(pd.cgx + lo + i);
                }
#pragma unroll
                for (int q = 0; q < B; ++q)
                    if (ib + q * step < c) put(at + ib + q * step, ti[q], tg[q]);
            }
        };
        uint32_t pos = obase;
        if (w0 < w1) {
#pragma unroll
            for (int i = 0; i < PRE; ++i)
                if (gq + G * i < c0) put(pos + gq + G * i, pidx[i], pgx[i]);
            put_block(pos, lo0, gq + G * PRE, c0, G);
            pos += static_cast<uint32_t>(max(c0, 0));
        }
        for (int w = w0 + 1; w < w1; ++w) {  // (G = 1 only)
            const int c = ldg_i32(pd.ccnt + w);
            put_block(pos, w * per, 0, c, 1);
            pos += static_cast<uint32_t>(max(c, 0));
        }
    }
    if (bad) atomicOr(&pd.st->err, 1);
    __syncthreads();
    // ---- rank
    int sh = 0;
    uint32_t P = 0, need = 0, eq = 0;
    if (s > 0) rank_merged(nc, s, S, sh, P, need, eq);
    // merged positions [MPT tid, MPT tid + MPT) belong to this thread
    bool sel[MPT];
    {
        uint32_t tie_rank = 0;
        if (need < eq) {  // some keys equal to the threshold are left out: index order decides
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < MPT; ++q) {
                const int m = MPT * tid + q;
                c += (m < nc && (S.u.f.mkey[m] >> sh) == P) ? 1u : 0u;
            }
            tie_rank = block_excl_scan<kSelectThreads>(c, S.scan, nullptr);
        }
#pragma unroll
        for (int q = 0; q < MPT; ++q) {
            const int m = MPT * tid + q;
            sel[q] = false;
            if (m < nc && s > 0) {
                const uint32_t kk = S.u.f.mkey[m] >> sh;
                if (kk > P) sel[q] = true;
                else if (kk == P) {
                    sel[q] = need >= eq || tie_rank < need;  // tie_rank: rank among equal keys
                    ++tie_rank;
                }
            }
        }
    }
    // ---- outputs: selection and union positions in index order (one scan,
    // selected count in the low half, union count in the high half), taken
    // together with |x' - x|^2, |x'|^2 and the support-change flag
    uint32_t v = 0;
    int changed = 0;
    double dx2 = 0.0, xn2 = 0.0;
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int m = MPT * tid + q;
        if (m < nc) {
            const bool on = (S.u.f.midx[m] >> 31) != 0u;
            v += (sel[q] ? 1u : 0u) + ((sel[q] || on) ? 0x10000u : 0u);
            if (on != sel[q]) changed = 1;
            if (MODE == SEL_STEP && (sel[q] || on)) {
                const double xo = static_cast<double>(S.u.f.mxo[m]);
                const double xn = sel[q] ? static_cast<double>(S.u.f.mval[m]) : 0.0;
                dx2 += (xn - xo) * (xn - xo);
                xn2 += xn * xn;
            }
        }
    }
    const BlockAgg out = block_sums_scan(dx2, xn2, 0.0, v, changed != 0, S);
    uint32_t pos = out.before;
#pragma unroll
    for (int q = 0; q < MPT; ++q) {
        const int m = MPT * tid + q;
        if (m < nc) {
            const uint32_t mi = S.u.f.midx[m];
            const bool on = (mi >> 31) != 0u;
            const int j = static_cast<int>(mi & 0x7FFFFFFFu);
            const uint32_t ps = pos & 0xFFFFu, pu = pos >> 16;
            if (sel[q] && ps < static_cast<uint32_t>(s)) {
                stg(out_sup + ps, static_cast<int32_t>(j));
                if (MODE == SEL_STEP) stg(out_val + ps, S.u.f.mval[m]);
            }
            if (MODE == SEL_STEP && (sel[q] || on) && pu < static_cast<uint32_t>(2 * s)) {
                const float xo = S.u.f.mxo[m];
                const float xn = sel[q] ? S.u.f.mval[m] : 0.0f;
                stg(dlist + pu, static_cast<int32_t>(j));
                stg(dw + pu, static_cast<double>(xn) - static_cast<double>(xo));
            }
            pos += (sel[q] ? 1u : 0u) + ((sel[q] || on) ? 0x10000u : 0u);
        }
    }
    if (MODE == SEL_INIT) {
        // x stays 0; the support bitmap and x on the support follow the selection
        for (int w = tid; w < words; w += kSelectThreads) pd.bmsup[w] = 0u;
        for (int i = tid; i < s; i += kSelectThreads) pd.xs[i] = 0.0f;
        __syncthreads();
        // the next full pass rebuilds the histogram off the new support
        for (int b = tid; b < 2048; b += kSelectThreads) pd.hist[b] = 0u;
#pragma unroll
        for (int q = 0; q < MPT; ++q) {
            const int m = MPT * tid + q;
            if (m < nc && sel[q]) {
                const int j = static_cast<int>(S.u.f.midx[m] & 0x7FFFFFFFu);
                atomicOr(&pd.bmsup[j >> 5], 1u << (j & 31));
            }
        }
        __syncthreads();
        return true;
    }
    if (tid == 0) {
        CandMeta mt;
        mt.changed = out.nf > 0 ? 1 : 0;
        mt.dcount = static_cast<int32_t>(out.total >> 16);
        mt.k = k;
        mt.pad = 0;
        mt.mu = mu;
        mt.dx2 = out.a;
        mt.xn2 = out.b;
        mt.omega = 0.0;
        store_meta(pd.meta + slot, mt);
    }
    __syncthreads();
    return true;
}

// Off-support candidates for the first proposal (x = 0, empty support).
__global__ __launch_bounds__(kGatherThreads) void k_candidates(const ProbDev* __restrict__ P) {
    const ProbDev& pd = P[blockIdx.y];
    if (pd.st->done || static_cast<int>(blockIdx.x) >= pd.npart) return;
    const CandPre<kGatherThreads> pre = cand_preload<kGatherThreads>(pd, blockIdx.x, pd.npart, false);
    compact_candidates<kGatherThreads>(pd, blockIdx.x, pd.npart, false, pre);
}

template <int NMAX>
__global__ __launch_bounds__(kSelectThreads) void k_propose(const ProbDev* __restrict__ P,
                                                            SolveArgs a, int mode) {
    const ProbDev& pd = P[blockIdx.y];
    SolveState* st = pd.st;
    __shared__ SelShared<NMAX> S;
    double mu0 = 0.0;
    if (mode == SEL_INIT) {
        if (st->done) return;
        propose<SEL_INIT>(pd, 0, 0, 1.0, false, 1.0, &mu0, S);
        return;
    }
    // shrink count of this proposal: after a round whose proposals all failed
    // the test, the following kSpec shrinks of the same step
    const int k = ldg_i32(&st->base_k) + static_cast<int>(blockIdx.x);
    bool skipped = false;
    const bool ok = propose<SEL_STEP>(pd, blockIdx.x, k, 0.0, true, a.k * (1.0 - a.c), &mu0, S, &skipped);
    if (skipped) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok) {
            stg(&st->phase, 1);  // the next residual gather takes the step-size test
        } else {
            stg(&st->done, 1);
            stg(&st->reason, static_cast<int32_t>(QIHT_REASON_STATIONARY));
        }
    }
}

// Batches: the step-size test and commit of the last round's proposals, one
// workgroup per problem, before the residual gather.
__global__ __launch_bounds__(kGatherThreads) void k_commit(const ProbDev* __restrict__ P, SolveArgs a) {
    const ProbDev& pd = P[blockIdx.x];
    __shared__ double s_dec[kSpec * (kGatherThreads / 64)];
    if (pd.st->done || pd.st->phase != 1) return;
    commit_round<kGatherThreads>(pd, a, s_dec);
}

template <int NMAX>
__global__ __launch_bounds__(kSelectThreads) void k_hard_threshold(const float* a, int n, int s,
                                                                   int32_t* out, int* err) {
    __shared__ SelShared<NMAX> S;
    for (int w = threadIdx.x; w < (n + 31) / 32; w += kSelectThreads) S.u.b.bm_new[w] = 0u;
    if (threadIdx.x == 0) S.changed = 0;
    __syncthreads();
    select_full<SEL_RAW>(n, s, a, nullptr, nullptr, 0.f, S, err);
    emit_support<SEL_RAW>(n, s, a, nullptr, nullptr, 0.f, nullptr, out, nullptr, S);
}

}  // namespace

void launch_candidates(const ProbDev* P, int count, int maxwg, hipStream_t st) {
    hipLaunchKernelGGL(k_candidates, dim3(maxwg, count), dim3(kGatherThreads), 0, st, P);
}

// (the 65536-entry instance up to that n: its LDS leaves room for two
// proposal workgroups per CU, which a batch of many problems uses)
constexpr int kSmallSelectN = kSelectThreads * 64;

void launch_propose(const ProbDev* P, int count, const SolveArgs& a, int mode, int max_n, hipStream_t st) {
    const dim3 grid(mode == SEL_INIT ? 1 : kSpec, count);
    if (max_n <= kSmallSelectN)
        hipLaunchKernelGGL(k_propose<kSmallSelectN>, grid, dim3(kSelectThreads), 0, st, P, a, mode);
    else
        hipLaunchKernelGGL(k_propose<kMaxSelectN>, grid, dim3(kSelectThreads), 0, st, P, a, mode);
}

void launch_commit(const ProbDev* P, int count, const SolveArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_commit, dim3(count), dim3(kGatherThreads), 0, st, P, a);
}

void launch_hard_threshold(const float* a, int n, int s, int32_t* out, int* err, hipStream_t st) {
    if (n <= kSmallSelectN)
        hipLaunchKernelGGL(k_hard_threshold<kSmallSelectN>, dim3(1), dim3(kSelectThreads), 0, st, a, n, s, out, err);
    else
        hipLaunchKernelGGL(k_hard_threshold<kMaxSelectN>, dim3(1), dim3(kSelectThreads), 0, st, a, n, s, out, err);
}

}  // namespace qiht
