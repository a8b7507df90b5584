// Device-side data structures and helpers shared by the solver kernels
// (gather.hip, pass.hip, select.hip) and their host orchestration
// (solve_host.hip).
#pragma once

#include <cstdint>

#include "qiht_internal.h"

namespace qiht {

constexpr int kSelectThreads = 1024;  // one workgroup per H_s proposal
constexpr int kGatherThreads = 256;   // column gathers
constexpr int kPassThreads = 256;     // full pass
constexpr int kPassMaxCols = 4096;    // columns of one full-pass task (at most)
constexpr int kSpec = 4;              // step sizes proposed at once
constexpr int kMaxSelectN = kSelectThreads * 256;  // 262144: a 512 x 512 image
constexpr int kCandCap = 3072;        // candidate keys a fast proposal holds in LDS

// Per-problem control state (device memory).
struct SolveState {
    int32_t done;
    int32_t iter;       // completed iterations
    int32_t reason;
    int32_t phase;      // 1 once proposals of a step await the step-size test
    int32_t total_bt;
    int32_t capped;
    int32_t err;        // NaN met in a selection
    int32_t base_k;     // shrink count of the first proposal of the next round
    int32_t full_selects;  // proposals that needed the full n-key rank
    int32_t pad;
    double mu_last;     // accepted step of the last iteration
};

// One proposal x' = H_s(x + mu_k g), k = shrink count.
struct CandMeta {
    int32_t changed;    // support differs from the current one
    int32_t dcount;     // entries where x' differs from x
    int32_t k;          // shrink count of this proposal
    int32_t pad;
    double mu;          // mu / (k(1-c))^k
    double dx2;         // |x' - x|^2
    double xn2;         // |x'|^2
    double omega;       // |x' - x|^2 / |Q1 (x' - x)|^2 (when needed)
};

struct ProbDev {
    const uint8_t* q1;
    const uint8_t* q2;
    int64_t col_bytes;
    int32_t rows;
    int32_t n;
    int32_t s;
    int32_t nwg;        // 16-byte row groups per column (gather workgroups)
    int32_t npart;      // gather row segments: nwg, or 1 KB segments for the wide
                        // gathers of a shared matrix (partials, candidate blocks)
    int32_t nslab;      // full-pass row slabs
    int32_t group;      // > 0: complex unknown, columns j and j + group are the
                        // real and imaginary parts of one entry (H_s by modulus)
    double alpha;       // dequantized value = alpha * code + beta
    double beta;
    float alpha_f;
    float pad_f;
    const double* yhat;
    float* r32;         // residual, rows_pad (zero beyond rows)
    const int32_t* rowexp; // dense formats: row exponents (value = 2^e stored)
    uint16_t* rb;       // dense formats: 2^e r as BF16 hi (rows_pad) then lo (rows_pad)
    uint32_t* rdig;     // residual digits, digit-major: ND x (nwg * 4H) words
    int32_t* rexp;      // per row chunk: fixed-point exponent e
    int32_t* rsum;      // per row chunk: sum_i N_i
    float* g;           // gradient, n
    float* gpart;       // nslab * n slab partials (nslab > 1)
    uint32_t* hist;     // 2048-bin histogram of the top 11 bits of |g|
    float* x;           // current iterate, dense n (zero off the support)
    int32_t* sup;       // current support, s ascending
    float* xs;          // x on the support, in support order
    float* gs;          // g on the support, in support order (written by G_MU)
    uint32_t* bmsup;    // support bitmap, n bits
    int32_t* csup;      // kSpec * s proposal supports
    float* cval;        // kSpec * s proposal values on their supports
    int32_t* dlist;     // kSpec * 2s indices where a proposal differs from x
    double* dw;         // kSpec * 2s the differences
    CandMeta* meta;     // kSpec
    double* part_mu;    // 2 * npart partial (Q1_G g_G).(Q2_G g_G), |Q1_G g_G|^2
    double* part_om;    // kSpec x npart (stride nwg) partial |Q1 (x'_t - x)|^2
    uint32_t* cidx;     // n slots: candidates per index block (bit 31: on the support)
    float2* cgx;        // n slots: (g_j, x_j) at those candidates
    int32_t* ccnt;      // npart: candidates of each index block (-1: use the full path)
    SolveState* st;
};

// A span of the full pass: columns [c0, c1) of row slab `slab` of problem p.
// The task list of a launch is followed in memory by two uint32 counters,
// zero between launches (the span queue of the pass kernels).
struct Task {
    int32_t p, slab, c0, c1;
    int32_t cpl;   // 16-byte chunks per lane of the problem's row slabs
};

// ---------------------------------------------------------------------------
// Fixed-point residual digits for the packed-code full pass.  The residual
// rows of one 16-byte row chunk (the rows one gather workgroup owns) share a
// scale: r~_i = N_i 2^e with |N_i| <= 2^22, e from the chunk's largest |r_i|.
// N_i is split into signed digits (six base-16 digits in [-8, 7] for codes of
// 1, 2 or 4 bits, three base-256 digits in [-128, 127] for 8-bit codes),
// transposed so that one 32-bit digit word lines up with the codes of one
// code word, and stored as rdig[d][chunk * 4H + v] (digit d, digit word v of
// the chunk).  The integer dot instructions then take the codes as stored
// (4- and 8-bit codes biased to signed by an xor):
//   sum_i k_i N_i = sum_d base^d sum_i (k_i - off) e_d(N_i) + off sum_i N_i.
// ---------------------------------------------------------------------------
template <int BITS>
struct QDig {
    static constexpr int DB = (BITS == 8) ? 8 : 4;         // digit width
    static constexpr int ND = (BITS == 8) ? 3 : 6;         // digits per row
    static constexpr int RPD = 32 / DB;                    // rows per digit word
    static constexpr int H = (BITS == 8) ? 1 : 4 / BITS;   // digit words per code word
    static constexpr int RPW = 32 / BITS;                  // rows per code word
    static constexpr uint32_t OFF = (BITS == 8) ? 0x808080u : 0x888888u;
    static constexpr int CODE_OFF = (BITS == 8) ? 128 : (BITS == 4 ? 8 : 0);
    // digit word h of code word cw holds rows cw * RPW + u * H + h, u < RPD
    // the signed operand of code word w for its h-th digit word
    static __device__ __forceinline__ uint32_t split(uint32_t w, int h) {
        if constexpr (BITS == 8) return w ^ 0x80808080u;
        else if constexpr (BITS == 4) return w ^ 0x88888888u;
        else if constexpr (BITS == 2) return (w >> (2 * h)) & 0x33333333u;
        else return (w >> h) & 0x11111111u;
    }
    static __device__ __forceinline__ int dot(uint32_t a, uint32_t b, int c) {
        if constexpr (BITS == 8) return __builtin_amdgcn_sdot4(static_cast<int>(a), static_cast<int>(b), c, false);
        else return __builtin_amdgcn_sdot8(static_cast<int>(a), static_cast<int>(b), c, false);
    }
};

// digits of RPD fixed-point values (offset form: field d of u[t] is digit d)
// transposed in place: afterwards field t of u[d] is digit d of value t.
template <int BITS>
__device__ __forceinline__ void transpose_digits(uint32_t (&u)[QDig<BITS>::RPD]) {
    if constexpr (QDig<BITS>::DB == 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t a = u[t], b = u[t + 4];
            u[t] = (a & 0x0000FFFFu) | (b << 16);
            u[t + 4] = (a >> 16) | (b & 0xFFFF0000u);
        }
#pragma unroll
        for (int t = 0; t < 8; t += 4)
#pragma unroll
            for (int v = t; v < t + 2; ++v) {
                const uint32_t a = u[v], b = u[v + 2];
                u[v] = (a & 0x00FF00FFu) | ((b << 8) & 0xFF00FF00u);
                u[v + 2] = ((a >> 8) & 0x00FF00FFu) | (b & 0xFF00FF00u);
            }
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            const uint32_t a = u[t], b = u[t + 1];
            u[t] = (a & 0x0F0F0F0Fu) | ((b << 4) & 0xF0F0F0F0u);
            u[t + 1] = ((a >> 4) & 0x0F0F0F0Fu) | (b & 0xF0F0F0F0u);
        }
    } else {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const uint32_t a = u[t], b = u[t + 2];
            u[t] = (a & 0x0000FFFFu) | (b << 16);
            u[t + 2] = (a >> 16) | (b & 0xFFFF0000u);
        }
#pragma unroll
        for (int t = 0; t < 4; t += 2) {
            const uint32_t a = u[t], b = u[t + 1];
            u[t] = (a & 0x00FF00FFu) | ((b << 8) & 0xFF00FF00u);
            u[t + 1] = ((a >> 8) & 0x00FF00FFu) | (b & 0xFF00FF00u);
        }
    }
}

// 32-bit digit words per 16-byte row chunk (0 for FP32 codes).
inline int digit_words_per_chunk(int bits) {
    switch (bits) {
        case 8: return 3 * 4;
        case 4: return 6 * 4;
        case 2: return 6 * 8;
        case 1: return 6 * 16;
        default: return 0;
    }
}

enum { G_R = 0, G_MU = 1, G_OMEGA = 2 };
enum { SEL_RAW = 0, SEL_INIT = 1, SEL_STEP = 2 };

// ---------------------------------------------------------------------------
// Block helpers (fixed reduction orders: results are bitwise reproducible).
// ---------------------------------------------------------------------------
// Load through a global-address-space pointer: pointers read out of ProbDev
// are generic, and generic (flat) loads make the compiler wait for every
// outstanding load before any use, which defeats prefetching.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ldg_u4(const void* p) {
    const u32x4_t v = *(const __attribute__((address_space(1))) u32x4_t*)(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t ldg_u32(const void* p) {
    return *(const __attribute__((address_space(1))) uint32_t*)(p);
}
__device__ __forceinline__ float ldg_f32(const void* p) {
    return *(const __attribute__((address_space(1))) float*)(p);
}
__device__ __forceinline__ double ldg_f64(const void* p) {
    return *(const __attribute__((address_space(1))) double*)(p);
}
__device__ __forceinline__ int32_t ldg_i32(const void* p) {
    return *(const __attribute__((address_space(1))) int32_t*)(p);
}
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldg_f2(const void* p) {
    const f32x2_t v = *(const __attribute__((address_space(1))) f32x2_t*)(p);
    return make_float2(v.x, v.y);
}
// Store through a global-address-space pointer (a generic store also counts
// against the LDS counter, so every later LDS wait would wait for it).
template <typename T>
__device__ __forceinline__ void stg(T* p, const T& v) {
    *(__attribute__((address_space(1))) T*)(p) = v;
}

// Cross-lane moves without LDS: DPP within rows of 16 lanes and the gfx950
// row / half-wave swaps.  dpp<CTRL>(v) reads lane CTRL(l) (0 where the
// pattern feeds nothing); swap16_sum(v) = v + v of lane l ^ 16 and
// swap32_sum(v) = v + v of lane l ^ 32, the two operands added in lane order
// (so both lanes of a pair hold the same bits).
template <int CTRL, int RM = 0xf, int BM = 0xf>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, RM, BM, false));
}
template <int CTRL, int RM = 0xf, int BM = 0xf>
__device__ __forceinline__ double dpp(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, RM, BM, false),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, RM, BM, false));
}
__device__ __forceinline__ float swap16_sum(float v) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap32_sum(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double swap16_sum(double v) {
    const uint32_t lo = static_cast<uint32_t>(__double2loint(v)), hi = static_cast<uint32_t>(__double2hiint(v));
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(static_cast<int>(b[0]), static_cast<int>(a[0])) +
           __hiloint2double(static_cast<int>(b[1]), static_cast<int>(a[1]));
}
__device__ __forceinline__ double swap32_sum(double v) {
    const uint32_t lo = static_cast<uint32_t>(__double2loint(v)), hi = static_cast<uint32_t>(__double2hiint(v));
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(static_cast<int>(b[0]), static_cast<int>(a[0])) +
           __hiloint2double(static_cast<int>(b[1]), static_cast<int>(a[1]));
}
__device__ __forceinline__ float lane0(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
}
__device__ __forceinline__ double lane0(double v) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                            __builtin_amdgcn_readlane(__double2loint(v), 0));
}

// Inclusive prefix sum over the 64 lanes of a wave, in DPP moves only:
// shifts by 1, 2, 4, 8 lanes within each row of 16 (lanes shifted in from
// outside the row add 0), then lane 15's total added to rows 1 and 3 and
// lane 31's to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x142, 0xa, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x143, 0xc, 0xf, false));
    return x;
}

// Sum over the 16 lanes of a row that share l mod 4, then over the four
// rows: lanes 0..3 end with the totals of their residues mod 4.
template <typename T>
__device__ __forceinline__ T slot_sum(T v) {
    v = v + dpp<0x124>(v);  // row_ror:4
    v = v + dpp<0x128>(v);  // row_ror:8
    v = swap16_sum(v);
    return swap32_sum(v);
}

// Value of lane l ^ (1 << BIT) for a slot bit BIT of 2..5 (lane bits 2..5
// index the 16 column slots of a wave): gfx950 half-wave and row swaps for
// bits 5 and 4, row rotations for bits 3 and 2 (bit 2: the lane 4 below or
// above within its row of 16).
template <int BIT>
__device__ __forceinline__ double slot_partner(double x, int lane) {
    if constexpr (BIT == 5 || BIT == 4) {
        const uint32_t lo = static_cast<uint32_t>(__double2loint(x)), hi = static_cast<uint32_t>(__double2hiint(x));
        const auto a = BIT == 5 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                                : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = BIT == 5 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                                : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        // [0]: the lower lane's value of the pair, [1]: the upper lane's
        const bool up = (lane >> BIT) & 1;
        return up ? __hiloint2double(static_cast<int>(b[0]), static_cast<int>(a[0]))
                  : __hiloint2double(static_cast<int>(b[1]), static_cast<int>(a[1]));
    } else if constexpr (BIT == 3) {
        return dpp<0x128>(x);  // row_ror:8
    } else {
        const double below = dpp<0x124>(x);  // row_ror:4: lane l - 4
        const double above = dpp<0x12C>(x);  // row_ror:12: lane l + 4
        return ((lane >> 2) & 1) ? below : above;
    }
}

// One exchange of the slot sums over slot bit BIT with C live values: while
// C > 1, the lanes with the bit set keep the upper half (adding the
// partner's upper half), the others the lower half, so the live values
// halve; with one left it is summed in full (both partners then hold the
// same bits: a + b = b + a).
template <int BIT, int C>
__device__ __forceinline__ void slot_exchange(double* v, int lane, int& base, int& dup) {
    if constexpr (C > 1) {
        constexpr int H = C / 2;
        const bool up = (lane >> BIT) & 1;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double give = up ? v[i] : v[H + i];
            const double keep = up ? v[H + i] : v[i];
            v[i] = keep + slot_partner<BIT>(give, lane);
        }
        if (up) base += H;
    } else {
        v[0] = v[0] + slot_partner<BIT>(v[0], lane);
        dup |= 1 << BIT;
    }
}

// Sums of V values over the column slots of a wave (lane bits LB..5; the
// bits below LB index the word), halving the live values at each of the
// slot bits 5, 4, ..., LB while more than one is live.  Afterwards lane l
// holds max(1, V >> (6 - LB)) totals in v[0..], of the value indices *base,
// *base + 1, ...; lanes that differ from l only in the bits of *dup hold the
// same totals.
template <int V, int LB = 2>
__device__ __forceinline__ void slot_sums_halving(double (&v)[V], int lane, int* base, int* dup) {
    static_assert(LB >= 2 && LB <= 5, "slot bits 2..5");
    constexpr int C5 = V, C4 = C5 > 1 ? C5 / 2 : 1, C3 = C4 > 1 ? C4 / 2 : 1, C2 = C3 > 1 ? C3 / 2 : 1;
    int b = 0, d = 0;
    slot_exchange<5, C5>(v, lane, b, d);
    if constexpr (LB <= 4) slot_exchange<4, C4>(v, lane, b, d);
    if constexpr (LB <= 3) slot_exchange<3, C3>(v, lane, b, d);
    if constexpr (LB <= 2) slot_exchange<2, C2>(v, lane, b, d);
    *base = b;
    *dup = d;
}

// Total of v over the column slots of a wave (lane bits LB..5); every lane
// of a word holds the same bits.
template <int LB>
__device__ __forceinline__ double slot_total(double v, int lane) {
    v = v + slot_partner<5>(v, lane);
    if constexpr (LB <= 4) v = v + slot_partner<4>(v, lane);
    if constexpr (LB <= 3) v = v + slot_partner<3>(v, lane);
    if constexpr (LB <= 2) v = v + slot_partner<2>(v, lane);
    return v;
}

// Sum over the wave in a fixed order, lane 0's result in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = v + dpp<0xB1>(v);  // quad_perm [1,0,3,2]
    v = v + dpp<0x4E>(v);  // quad_perm [2,3,0,1]
    return lane0(slot_sum(v));
}

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

// Exclusive prefix sum in thread order; *total (optional) gets the sum.
template <int NT>
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t x = wave_incl_scan(v);
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

// Candidates of the H_s proposals.  Off the support G the proposal value is
// a_j = mu g_j, so the order of |a_j| there does not depend on mu: the full
// pass counts |g_j| (j off G) in 2048 bins of the top 11 bits of its FP32
// pattern, the bin B of the s-th largest gives t = lo(B)(1 - 2^-20), and an
// entry off G with |g_j| < t has FP32 |a_j| strictly below at least s entries
// off G for every mu > 0 (a rounded product moves by at most 2^-24
// relative).  So the top s of all n lies in G plus {j off G : |g_j| >= t}.
// Workgroup wg of nw takes the index block [wg per, min(n, (wg + 1) per)),
// per = ceil(n / nw), and writes the candidates of that block (G's members,
// flagged by bit 31, and the entries off G that pass t) in index order to
// cidx / cgx from wg per on, and their count to ccnt[wg]; -1 when the fast
// path cannot be used (t in the subnormal range, or a non-finite g in the
// block: the full path flags those).
// Inputs of compact_candidates that do not depend on anything computed in
// the calling kernel, loaded ahead: thread t's 2048 / NT histogram bins
// (from the top: bins 2047 - (2048 / NT) t - i) and its first entry of the
// index block.
template <int NT>
struct CandPre {
    static constexpr int PER = 2048 / NT;
    static_assert(2048 % NT == 0, "the histogram is split evenly over the threads");
    uint32_t h[PER];
    float g0, x0;   // g and x at the thread's first entry of the block
    uint32_t bm0;
};

template <int NT>
__device__ __forceinline__ CandPre<NT> cand_preload(const ProbDev& pd, int wg, int nw, bool with_support) {
    CandPre<NT> c;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < CandPre<NT>::PER; ++i) c.h[i] = ldg_u32(pd.hist + (2047 - CandPre<NT>::PER * tid - i));
    const int per = (pd.n + nw - 1) / nw;
    const int lo = wg * per, hi = min(pd.n, lo + per);
    const int j = min(lo + tid, hi - 1);  // clamped: a thread past the block ignores it
    c.g0 = ldg_f32(pd.g + j);
    c.bm0 = with_support ? ldg_u32(pd.bmsup + (j >> 5)) : 0u;
    c.x0 = with_support ? ldg_f32(pd.x + j) : 0.0f;  // (x is 0 off the support)
    return c;
}

template <int NT>
__device__ void compact_candidates(const ProbDev& pd, int wg, int nw, bool with_support,
                                   const CandPre<NT>& pre) {
    constexpr int NW = NT / 64;
    constexpr int PER = CandPre<NT>::PER;
    __shared__ float s_thr;
    __shared__ int s_fast;
    __shared__ uint32_t s_wc[NW];
    __shared__ uint32_t s_scan[NW];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = pd.n, s = pd.s;
    const int nsup = with_support ? s : 0;
    // more than s entries off the support: the threshold bin of the s-th
    // largest (no bin found, i.e. counts inconsistent with n: the full path)
    const bool ranked = n - nsup > s;
    if (tid == 0) {
        s_thr = 0.f;
        s_fast = ranked ? 0 : 1;
        s_bad = 0;
    }
    if (ranked) {  // uniform
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) c += pre.h[i];
        uint32_t run = block_excl_scan<NT>(c, s_scan, nullptr);  // bins from the top
        const uint32_t want = static_cast<uint32_t>(s);
        if (run < want && want <= run + c) {
            int bin = 0;
            bool found = false;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                if (!found && run + pre.h[i] >= want) {
                    bin = 2047 - PER * tid - i;
                    found = true;
                }
                run += pre.h[i];
            }
            const float thr = __uint_as_float(static_cast<uint32_t>(bin) << 20) * (1.0f - 0x1p-20f);
            s_thr = thr;
            s_fast = thr >= 0x1p-100f;  // keep clear of subnormal products
        }
    }
    __syncthreads();
    const float thr = s_thr;
    const int per = (n + nw - 1) / nw;
    const int lo = wg * per, hi = min(n, lo + per);
    uint32_t base = 0;
    int bad = 0;
    for (int r0 = lo; r0 < hi; r0 += NT) {
        const int j = r0 + tid;
        const bool in = j < hi;
        const int jc = min(j, hi - 1);
        const float gv = r0 == lo ? pre.g0 : ldg_f32(pd.g + jc);
        const uint32_t bw = r0 == lo ? pre.bm0 : (with_support ? ldg_u32(pd.bmsup + (jc >> 5)) : 0u);
        const bool on_sup = in && ((bw >> (j & 31)) & 1u);
        if (in && (__float_as_uint(gv) & 0x7FFFFFFFu) > 0x7F800000u) bad = 1;
        const bool cand = on_sup || (in && fabsf(gv) >= thr);
        const uint64_t b = __ballot(cand);
        if (lane == 0) s_wc[wv] = static_cast<uint32_t>(__popcll(b));
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            before += w < wv ? s_wc[w] : 0u;
            all += s_wc[w];
        }
        if (cand) {
            const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            const uint32_t pos = base + before + static_cast<uint32_t>(__popcll(b & lt));
            stg(pd.cidx + lo + pos, static_cast<uint32_t>(j) | (on_sup ? 0x80000000u : 0u));
            const float xj = on_sup ? (r0 == lo ? pre.x0 : ldg_f32(pd.x + j)) : 0.0f;
            stg(reinterpret_cast<f32x2_t*>(pd.cgx + lo + pos), f32x2_t{gv, xj});
        }
        base += all;
        __syncthreads();
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0) stg(pd.ccnt + wg, (s_fast && !s_bad) ? static_cast<int32_t>(base) : -1);
}

// A proposal's metadata, stored field by field through global pointers.
__device__ __forceinline__ void store_meta(CandMeta* p, const CandMeta& m) {
    stg(&p->changed, m.changed);
    stg(&p->dcount, m.dcount);
    stg(&p->k, m.k);
    stg(&p->pad, m.pad);
    stg(&p->mu, m.mu);
    stg(&p->dx2, m.dx2);
    stg(&p->xn2, m.xn2);
    stg(&p->omega, m.omega);
}

// Step after k shrinks: k successive divisions, the same rounding sequence
// as applying mu <- mu / (k(1-c)) k times.
__device__ __forceinline__ double shrunk_mu(double mu, double shrink, int k) {
    for (int i = 0; i < k; ++i) mu = mu / shrink;
    return mu;
}

// ---------------------------------------------------------------------------
// Code unpacking: a 32-bit word holds 32/BITS codes, code q at bit q*BITS.
// ---------------------------------------------------------------------------
template <int BITS>
__device__ __forceinline__ uint32_t code_at(uint32_t w, int q) {
    return (w >> (q * BITS)) & ((1u << BITS) - 1u);
}

// Dense formats: the stored value of an FP8 E4M3 byte / a BF16 half word.
__device__ __forceinline__ float e4m3_value(uint32_t b) {
    const uint32_t e = (b >> 3) & 15u, m = b & 7u;
    const float mag = e == 0u ? static_cast<float>(m) * 0x1p-9f
                              : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return (b & 0x80u) ? -mag : mag;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// Nearest BF16 of an FP64 value (ties to even), as its 16-bit pattern: the
// significand is cut at 8 bits directly from the FP64 value (one rounding).
__device__ __forceinline__ uint32_t bf16_rne(double x) {
    if (x == 0.0 || !isfinite(x)) return __float_as_uint(static_cast<float>(x)) >> 16;
    const int qe = max(ilogb(x), -126) - 7;
    const float y = static_cast<float>(ldexp(rint(ldexp(x, -qe)), qe));
    return __float_as_uint(y) >> 16;
}

// Rows held by one 32-bit word of a column, and the value of row q of the
// word before the row scaling: the integer code (packed formats), the float
// (32), or the stored low-precision value (kFmtE4M3 = 9, kFmtBF16 = 16).
template <int BITS>
constexpr int rows_per_word() {
    return BITS == 32 ? 1 : BITS == 16 ? 2 : BITS == 9 ? 4 : 32 / BITS;
}
template <int BITS>
__device__ __forceinline__ double elem_at(uint32_t w, int q) {
    if constexpr (BITS == 32) return static_cast<double>(__uint_as_float(w));
    else if constexpr (BITS == 16) return static_cast<double>(bf16_value((w >> (16 * q)) & 0xFFFFu));
    else if constexpr (BITS == 9) {
        // hardware FP8 (OCP E4M3) conversion, two bytes per instruction; exact
        typedef float f32x2_v __attribute__((ext_vector_type(2)));
        const f32x2_v pr = q >= 2 ? __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), true)
                                  : __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), false);
        return static_cast<double>((q & 1) ? pr.y : pr.x);
    }
    else return static_cast<double>(code_at<BITS>(w, q));
}

// Launchers (defined in the kernel files).
// Workgroups of a batch's gather: groups of 64 workgroups, entry g of the
// table = (grid row, first row group) of group g, a grid row being problem
// p's set t as p * sets + t; every row gets just the groups its own row
// groups need (a plain grid would give each row as many as the widest
// problem's, most of them returning at once).  tab NULL: that plain grid.
struct GatherGrid {
    const int2* tab = nullptr;
    int ngroups = 0;
    int rg = 1;  // 16-byte row groups per workgroup (4 for batches: one
                 // 64-byte piece of each listed column per workgroup)
};
void launch_gather(int mode, int bits, const ProbDev* P, int count, int maxwg,
                   const SolveArgs& a, int zero_x, bool wide, hipStream_t st,
                   const GatherGrid& gg = GatherGrid());
// ev0/ev1 (optional): events recorded by the dispatch itself around the
// kernel (timing of the bandwidth-bound pass).

// Shared-matrix pass (gemm.hip): G = Phi~^T R' on the matrix cores for all
// problems of a batch that share one dense-format or FP32 matrix.
struct SharedGemm {
    const uint8_t* a;   // stored columns
    int64_t col_bytes;
    int n;              // columns
    int rows_pad;       // rows covered by col_bytes (a multiple of 32)
    int bits;           // kFmtBF16, kFmtE4M3 or 32
    const void* b;      // R' of problem 0; problem k at + k * ldb elements
    int64_t ldb;        //   (BF16 hi/lo: 16-bit elements, lo at + lo_off; FP32: floats)
    int64_t lo_off;
    float* g;           // g of problem 0; problem k at + k * ldg
    int64_t ldg;
    int ksplit;         // row splits of the GEMM (BF16 kernel), partial G in gp
    float* gp;          //   ksplit x count x ldg floats (unused when ksplit = 1)
};
int shared_ksplit(int bits, int n, int count, int rows_pad);
// Whether the GEMM can split rows_pad rows ks ways (ks = 1, 2, 4).
bool shared_ksplit_ok(int bits, int rows_pad, int ks);
void launch_shared_pass(const SharedGemm& sg, const ProbDev* P, int count, hipStream_t st,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Bytes of the last-level Infinity Cache (MALL) that code streams up to
// this size are assumed to stay in from one pass to the next.
constexpr double kInfinityCacheBytes = 200.0 * 1024 * 1024;
// Workgroups of the full pass that the device holds at once (0 if unknown).
int pass_slots(int bits, int cpl, bool long_stream);
// T: ntasks spans (then the queue counters); workgroup w of nwg starts with span w
void launch_pass(int bits, int cpl, bool long_stream, const ProbDev* P, const Task* T, int nwg, int ntasks,
                 hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
// max_n: the largest n of the problems
void launch_slab_reduce(const ProbDev* P, int count, int max_n, hipStream_t st);
void launch_candidates(const ProbDev* P, int count, int maxwg, hipStream_t st);
// max_n: the largest n of the problems (picks the selection's LDS size)
void launch_propose(const ProbDev* P, int count, const SolveArgs& a, int mode, int max_n, hipStream_t st);
void launch_hard_threshold(const float* a, int n, int s, int32_t* out, int* err, hipStream_t st);
void launch_commit(const ProbDev* P, int count, const SolveArgs& a, hipStream_t st);

// The step-size test of Algorithm 2 (Sec. II-A) on the kSpec proposals of
// the last round, shrink counts k = base_k, base_k + 1, ... in order: a
// proposal that keeps the support is taken at once; otherwise proposal k is
// taken when mu_k <= (1 - c) |x'_k - x|^2 / |Q1 (x'_k - x)|^2, or, failing
// that, when k reaches the backtracking cap (*capped).  -1: every proposal
// failed, and the next round proposes the following kSpec shrinks from the
// same x.  Called by every thread of a workgroup of NT threads (it holds one
// barrier; red: kSpec * NT / 64 doubles of LDS); all get the same answer.
// The denominators are summed from the omega gather's partials, per wave and
// then in wave order.
// The test's inputs: the proposals' metadata and this thread's first omega
// partials.  Every load is unconditional (the partial's index clamped into the
// array; a thread past the partials does not use it), so a kernel can issue
// them with its other first loads, before it knows whether a test is due.
struct PickIn {
    int mch[kSpec], mk[kSpec];
    double mmu[kSpec], mdx2[kSpec], om0[kSpec];
};
template <int NT>
__device__ __forceinline__ PickIn pick_load(const ProbDev& pd) {
    PickIn in;
    const int b0 = min(static_cast<int>(threadIdx.x), pd.npart - 1);
#pragma unroll
    for (int t = 0; t < kSpec; ++t) {
        const CandMeta* m = pd.meta + t;
        in.mch[t] = ldg_i32(&m->changed);
        in.mk[t] = ldg_i32(&m->k);
        in.mmu[t] = ldg_f64(&m->mu);
        in.mdx2[t] = ldg_f64(&m->dx2);
        in.om0[t] = ldg_f64(pd.part_om + static_cast<size_t>(t) * pd.nwg + b0);
    }
    return in;
}

template <int NT>
__device__ int decide_pick(const ProbDev& pd, const SolveArgs& a, bool* capped, double* red, const PickIn& in) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double den[kSpec];
#pragma unroll
    for (int t = 0; t < kSpec; ++t) den[t] = 0.0;
    if (tid < pd.npart)
#pragma unroll
        for (int t = 0; t < kSpec; ++t) den[t] += in.om0[t];
    for (int b = tid + NT; b < pd.npart; b += NT)
#pragma unroll
        for (int t = 0; t < kSpec; ++t) den[t] += ldg_f64(pd.part_om + static_cast<size_t>(t) * pd.nwg + b);
#pragma unroll
    for (int t = 0; t < kSpec; ++t) {
        den[t] = wave_sum(den[t]);
        if (lane == 0) red[t * NW + wv] = den[t];
    }
    __syncthreads();
    int pick = -1;
    *capped = false;
#pragma unroll
    for (int t = 0; t < kSpec; ++t) {
        if (pick >= 0) continue;
        if (!in.mch[t]) {
            pick = t;
            continue;
        }
        double d = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) d += red[t * NW + w];
        const double omega = d > 0.0 ? in.mdx2[t] / d : INFINITY;
        if (in.mmu[t] <= (1.0 - a.c) * omega) {
            pick = t;
        } else if (in.mk[t] >= a.max_backtracks) {
            pick = t;
            *capped = true;
        }
    }
    return pick;
}
template <int NT>
__device__ int decide_pick(const ProbDev& pd, const SolveArgs& a, bool* capped, double* red) {
    return decide_pick<NT>(pd, a, capped, red, pick_load<NT>(pd));
}

// The commit workgroup of a residual gather (one per problem, NT threads):
// the proposal the step-size test picks replaces x and the support, or, when
// every proposal failed, the next round's proposals shrink further.  Either
// way the |g| histogram is cleared for the next full pass.  The other
// workgroups of the gather read the picked proposal's support and values
// (or, after a failure, the current ones), never what this one writes.
template <int NT>
__device__ void commit_round(const ProbDev& pd, const SolveArgs& a, double* red, const PickIn& in);
template <int NT>
__device__ void commit_round(const ProbDev& pd, const SolveArgs& a, double* red) {
    commit_round<NT>(pd, a, red, pick_load<NT>(pd));
}

// Device-side commit of proposal `t` (called by one whole workgroup of
// `nt` threads): x and the support take the proposal's values, the state
// records the iteration and the stop test.
template <int NT>
__device__ void commit_proposal(const ProbDev& pd, int t, const SolveArgs& a, bool capped) {
    SolveState* st = pd.st;
    const CandMeta m = pd.meta[t];
    const int32_t* cs = pd.csup + static_cast<size_t>(t) * pd.s;
    const float* cv = pd.cval + static_cast<size_t>(t) * pd.s;
    const int words = (pd.n + 31) / 32;
    for (int i = threadIdx.x; i < pd.s; i += NT) stg(pd.x + ldg_i32(pd.sup + i), 0.0f);
    for (int w = threadIdx.x; w < words; w += NT) stg(pd.bmsup + w, 0u);
    __syncthreads();
    __threadfence_block();
    for (int i = threadIdx.x; i < pd.s; i += NT) {
        const int j = ldg_i32(cs + i);
        const float v = ldg_f32(cv + i);
        stg(pd.x + j, v);
        stg(pd.xs + i, v);
        stg(pd.sup + i, static_cast<int32_t>(j));
        atomicOr(&pd.bmsup[j >> 5], 1u << (j & 31));
    }
    if (threadIdx.x == 0) {
        st->iter += 1;
        st->mu_last = m.mu;
        st->total_bt += m.k;
        st->capped += capped ? 1 : 0;
        st->base_k = 0;
        if (a.tol >= 0.0 && m.dx2 <= a.tol * a.tol * m.xn2) {
            st->done = 1;
            st->reason = QIHT_REASON_CONVERGED;
        } else if (st->iter >= a.max_iters) {
            st->done = 1;
            st->reason = QIHT_REASON_MAX_ITERS;
        }
    }
    __syncthreads();
}

template <int NT>
__device__ void commit_round(const ProbDev& pd, const SolveArgs& a, double* red, const PickIn& in) {
    bool capped = false;
    const int pick = decide_pick<NT>(pd, a, &capped, red, in);
    if (pick >= 0) {
        commit_proposal<NT>(pd, pick, a, capped);
    } else if (threadIdx.x == 0) {
        pd.st->base_k += kSpec;
    }
    for (int b = threadIdx.x; b < 2048; b += NT) stg(pd.hist + b, 0u);
}

}  // namespace qiht
