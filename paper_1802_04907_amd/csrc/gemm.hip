// Shared-matrix pass: when every problem of a batch solves against the same
// matrix A (one dense-format or FP32 handle), the per-problem passes
// g_k = A^T r_k become one GEMM, G = Phi~^T R', on the matrix cores, with
// R' = diag(2^e) R (the row scale folded into the residuals).
//
//   A operand (M x K): the stored columns of Phi~ (M = n columns of Phi, K =
//     rows), column-major storage = K-contiguous rows of the operand.
//   B operand (K x N): R' for the N = count right-hand sides, K-contiguous.
//   BF16 and E4M3 storage: BF16 MFMA (E4M3 widened exactly to BF16 on the
//     way into LDS), R' as two BF16 terms (hi + lo, about 16 significant
//     bits), FP32 accumulation.  FP32 storage: FP32 MFMA on the FP32 r.
//
// Tiling: every right-hand side of a workgroup's tile shares its reads of A
// (each element of A is read once per tile of right-hand sides), K in steps
// of 32 rows staged through LDS.
//   k_gemm_bf16_half (BF16) and k_gemm_e4m3_half (E4M3): 256 columns x 128
//     right-hand sides, two workgroups per CU, LDS-direct loads, details
//     below.
//   k_gemm_f32 (FP32): 128 columns x 256 right-hand sides.
#include <hip/hip_ext.h>

#include <algorithm>

#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kBM = 128;  // FP32 kernel: columns of Phi per workgroup
constexpr int kBN = 256;  // FP32 kernel: right-hand sides per workgroup
constexpr int kBK = 32;   // rows per step
constexpr int kBM2 = 256; // BF16 / E4M3 kernels: columns of Phi per workgroup

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf16x8_t as_bf16x8(uint4 v) {
    return __builtin_bit_cast(bf16x8_t, v);
}

// Four E4M3 bytes -> four BF16 (two words), exactly: the hardware converts
// to FP32 (every E4M3 value is exact there and in BF16), the upper halves are
// the BF16 patterns.
__device__ __forceinline__ uint2 e4m3x4_to_bf16(uint32_t w) {
    const f32x2_t lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), false);
    const f32x2_t hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(w), true);
    return make_uint2((__float_as_uint(lo.x) >> 16) | (__float_as_uint(lo.y) & 0xFFFF0000u),
                      (__float_as_uint(hi.x) >> 16) | (__float_as_uint(hi.y) & 0xFFFF0000u));
}

struct GemmArgs {
    const uint8_t* a;    // stored columns, col_bytes apart
    int64_t col_bytes;
    int n;               // columns (M)
    int rows;            // K (a multiple of 32 ksplit)
    int nrhs;            // N
    const void* b;       // R': BF16 hi/lo (ldb 16-bit elements apart per RHS; lo at +lo_off)
    int64_t ldb;         //     or FP32 r (ldb floats apart)
    int64_t lo_off;
    float* g;            // G, g_k at g + k * ldg
    int64_t ldg;
    int ksplit;          // row splits (blockIdx.z); > 1: partial G at gp + split * count * ldg
    float* gp;
};

// C tile (mt, nt) of a wave: lane holds rows 4 (lane / 16) + t (columns of
// Phi) of right-hand side 16 nt + lane % 16; four consecutive g_j per store.
template <int MT, int NT>
__device__ __forceinline__ void store_tiles(const GemmArgs& p, float* out, const f32x4_t (&acc)[MT][NT],
                                            int jw, int kw, int lane) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int k = kw + 16 * nt + (lane & 15);
        if (k >= p.nrhs) continue;
        float* gk = out + static_cast<int64_t>(k) * p.ldg;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int j = jw + 16 * mt + 4 * (lane >> 4);
            if (j + 3 < p.n) {
                *reinterpret_cast<float4*>(gk + j) =
                    make_float4(acc[mt][nt][0], acc[mt][nt][1], acc[mt][nt][2], acc[mt][nt][3]);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (j + t < p.n) gk[j + t] = acc[mt][nt][t];
            }
        }
    }
}

// LDS rows of the BF16 operands are 64 bytes (the 32 rows of one step of one
// column or right-hand side), unpadded; the four 16-byte pieces of row r sit
// at piece ^ dma_swz(r % 16).  A fragment read (16 consecutive lanes: rows
// r..r+15 of one piece) then touches every bank once: on gfx950 a 16-byte
// LDS read serves 16 lanes per cycle over 64 banks, and this is the placement
// a probe of the bank counter found conflict-free (80-byte padded rows cost
// one extra cycle per read).
__device__ __forceinline__ int dma_swz(int r) { return (r >> 1) & 3; }
__device__ __forceinline__ int lds_slot(int r, int piece) { return r * 64 + 16 * (piece ^ dma_swz(r & 15)); }

// 16 bytes per lane from g into LDS at lds + 16 lane (lds wave-uniform).  The
// compiler does not see these loads: every wait on them is explicit (vmcnt),
// and the kernel waits for all of them before it ends.
__device__ __forceinline__ void lds_dma16(const void* g, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds) : "memory");
}

// BF16 storage, two workgroups per CU: 256 columns x 128 right-hand sides
// per workgroup (each wave 128 x 64: 8 x 4 tiles of 16 x 16, 128
// accumulators), the operands loaded straight into LDS with gfx950's
// LDS-direct loads (global_load_lds_dwordx4: 16 bytes per lane at M0 +
// 16 lane), one step ahead in a two-stage ring of 32 KiB stages (A 16 KiB,
// R' hi and lo 8 KiB each), rows placed by lds_slot.  No registers stage the
// data and no LDS writes sit between the MFMAs; with two workgroups on a CU
// one workgroup's MFMAs run while the other waits at its barrier or for its
// loads.  (One workgroup of 256 x 256 per CU with 256 accumulators a wave
// and loads two steps ahead ran 8% slower; loads staged through registers
// into padded LDS 22%.)
constexpr int kHN = 128;
constexpr int kHStage = 16384 + 2 * 8192;

__global__ __launch_bounds__(256, 2) void k_gemm_bf16_half(GemmArgs p) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[2 * kHStage];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j0 = blockIdx.x * kBM2;
    const int n0 = blockIdx.y * kHN;
    const int kper = p.rows / p.ksplit;
    const int kbeg = blockIdx.z * kper;
    const int wm = (wv & 1) * 128, wn = (wv >> 1) * 64;
    const int rsub = lane >> 2;
    const int piece = (lane & 3) ^ dma_swz(rsub);
    const uint8_t* ga[4];
    const uint8_t* gh[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int col = min(j0 + 16 * (4 * wv + i) + rsub, p.n - 1);
        ga[i] = p.a + static_cast<int64_t>(col) * p.col_bytes + 16 * piece;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int rhs = min(n0 + 16 * (2 * wv + i) + rsub, p.nrhs - 1);
        gh[i] = static_cast<const uint8_t*>(p.b) + 2 * (static_cast<int64_t>(rhs) * p.ldb) + 16 * piece;
    }
    const int64_t lo_bytes = 2 * p.lo_off;
    const uint32_t lds_base = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(
        (__attribute__((address_space(3))) uint8_t*)(lds)));
    const uint32_t wa = __builtin_amdgcn_readfirstlane(lds_base + wv * 4096);
    const uint32_t wb = __builtin_amdgcn_readfirstlane(lds_base + wv * 2048);
    const int ksteps = kper / kBK;
    auto issue = [&](int t) {
        const int64_t kb = 2 * static_cast<int64_t>(kbeg + t * kBK);
        const uint32_t st = (t & 1) * kHStage;
#pragma unroll
        for (int i = 0; i < 4; ++i) lds_dma16(ga[i] + kb, wa + st + i * 1024);
#pragma unroll
        for (int i = 0; i < 2; ++i) lds_dma16(gh[i] + kb, wb + st + 16384 + i * 1024);
#pragma unroll
        for (int i = 0; i < 2; ++i) lds_dma16(gh[i] + lo_bytes + kb, wb + st + 16384 + 8192 + i * 1024);
    };

    f32x4_t acc[8][4];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    const int foff = lds_slot(lane & 15, lane >> 4);
    auto compute = [&](int t) {
        const uint8_t* sa = lds + (t & 1) * kHStage + foff;
        bf16x8_t af[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
            af[mt] = as_bf16x8(*reinterpret_cast<const uint4*>(sa + (wm + 16 * mt) * 64));
        auto bfrag = [&](int term, int nt) {
            return as_bf16x8(*reinterpret_cast<const uint4*>(sa + 16384 + 8192 * term + (wn + 16 * nt) * 64));
        };
        bf16x8_t bhn = bfrag(0, 0), bln = bfrag(1, 0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8_t bh8 = bhn, bl8 = bln;
            if (nt + 1 < 4) {
                bhn = bfrag(0, nt + 1);
                bln = bfrag(1, nt + 1);
            }
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bh8, acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bl8, acc[mt][nt], 0, 0, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x100, 10, 0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (nt + 1 < 4) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
        }
    };

    issue(0);
    for (int t = 0; t < ksteps; ++t) {
        // step t's loads (the only ones outstanding) have landed in every
        // wave, and stage (t + 1) % 2 (step t - 1) is no longer read
        asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
        if (t + 1 < ksteps) issue(t + 1);
        compute(t);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    float* out = p.ksplit > 1 ? p.gp + static_cast<int64_t>(blockIdx.z) * p.nrhs * p.ldg : p.g;
    store_tiles<8, 4>(p, out, acc, j0 + wm, n0 + wn, lane);
}

// E4M3 storage, two workgroups per CU: the tile and MFMA order of
// k_gemm_bf16_half, the codes (one byte a row) landing in LDS as stored and
// widened to BF16 as a fragment is read (8 codes, one 8-byte LDS read, two
// hardware FP8 conversions per 4 codes).  Stages of 24 KiB (A 8 KiB: rows of
// 32 bytes, the two 16-byte halves of row r at half ^ ((r >> 3) & 1); R' hi
// and lo 8 KiB each), three of them (72 KiB): loads two steps ahead.
constexpr int kE8Stage = 8192 + 2 * 8192;

__device__ __forceinline__ int e8_swz(int r) { return (r >> 3) & 1; }

__global__ __launch_bounds__(256, 2) void k_gemm_e4m3_half(GemmArgs p) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[3 * kE8Stage];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j0 = blockIdx.x * kBM2;
    const int n0 = blockIdx.y * kHN;
    const int kper = p.rows / p.ksplit;
    const int kbeg = blockIdx.z * kper;
    const int wm = (wv & 1) * 128, wn = (wv >> 1) * 64;
    // A: wave w loads columns 64 w + 32 i + lane / 2 (i < 2), half lane % 2 of
    // the column's LDS row; R' as in k_gemm_bf16_half
    const uint8_t* ga[2];
    const uint8_t* gh[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int cl = 64 * wv + 32 * i + (lane >> 1);
        const int col = min(j0 + cl, p.n - 1);
        ga[i] = p.a + static_cast<int64_t>(col) * p.col_bytes + 16 * ((lane & 1) ^ e8_swz(cl));
    }
    const int rsub = lane >> 2;
    const int piece = (lane & 3) ^ dma_swz(rsub);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int rhs = min(n0 + 16 * (2 * wv + i) + rsub, p.nrhs - 1);
        gh[i] = static_cast<const uint8_t*>(p.b) + 2 * (static_cast<int64_t>(rhs) * p.ldb) + 16 * piece;
    }
    const int64_t lo_bytes = 2 * p.lo_off;
    const uint32_t lds_base = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(
        (__attribute__((address_space(3))) uint8_t*)(lds)));
    const uint32_t wd = __builtin_amdgcn_readfirstlane(lds_base + wv * 2048);
    const int ksteps = kper / kBK;
    auto issue = [&](int t) {
        const int64_t k0 = kbeg + static_cast<int64_t>(t) * kBK;
        const uint32_t st = (t % 3) * kE8Stage;
#pragma unroll
        for (int i = 0; i < 2; ++i) lds_dma16(ga[i] + k0, wd + st + i * 1024);
#pragma unroll
        for (int i = 0; i < 2; ++i) lds_dma16(gh[i] + 2 * k0, wd + st + 8192 + i * 1024);
#pragma unroll
        for (int i = 0; i < 2; ++i) lds_dma16(gh[i] + lo_bytes + 2 * k0, wd + st + 16384 + i * 1024);
    };

    f32x4_t acc[8][4];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // A fragment: row lane % 16 of a 16-row block, codes 8 g .. 8 g + 7 (g =
    // lane / 16): half g / 2 of the row, bytes 8 (g % 2) ..
    const int r16 = lane & 15, g = lane >> 4;
    const int aoff = r16 * 32 + 16 * ((g >> 1) ^ e8_swz(r16)) + 8 * (g & 1);
    const int foff = lds_slot(lane & 15, lane >> 4);
    auto compute = [&](int t) {
        const uint8_t* sa = lds + (t % 3) * kE8Stage;
        bf16x8_t af[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            const uint2 w = *reinterpret_cast<const uint2*>(sa + (wm + 16 * mt) * 32 + aoff);
            const uint2 c0 = e4m3x4_to_bf16(w.x), c1 = e4m3x4_to_bf16(w.y);
            af[mt] = as_bf16x8(make_uint4(c0.x, c0.y, c1.x, c1.y));
        }
        auto bfrag = [&](int term, int nt) {
            return as_bf16x8(*reinterpret_cast<const uint4*>(sa + 8192 + 8192 * term + (wn + 16 * nt) * 64 + foff));
        };
        bf16x8_t bhn = bfrag(0, 0), bln = bfrag(1, 0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8_t bh8 = bhn, bl8 = bln;
            if (nt + 1 < 4) {
                bhn = bfrag(0, nt + 1);
                bln = bfrag(1, nt + 1);
            }
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bh8, acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bl8, acc[mt][nt], 0, 0, 0);
        }
    };

    issue(0);
    if (ksteps > 1) issue(1);
    for (int t = 0; t < ksteps; ++t) {
        // step t's loads have landed in every wave (step t + 1's 6 may still
        // be in flight), and stage (t + 2) % 3 (step t - 1) is no longer read
        if (t + 1 < ksteps) asm volatile("s_waitcnt vmcnt(6)\n\ts_barrier" ::: "memory");
        else asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
        if (t + 2 < ksteps) issue(t + 2);
        compute(t);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    float* out = p.ksplit > 1 ? p.gp + static_cast<int64_t>(blockIdx.z) * p.nrhs * p.ldg : p.g;
    store_tiles<8, 4>(p, out, acc, j0 + wm, n0 + wn, lane);
}

// FP32 storage: FP32 MFMA (16 x 16 x 4), r in FP32.
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs p) {
    __shared__ float la[kBM][kBK + 4];
    __shared__ float lb[kBN][kBK + 4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j0 = blockIdx.x * kBM;
    const int wm = (wv & 1) * 64, wn = (wv >> 1) * 128;
    const int acol = min(j0 + tid / 2, p.n - 1);
    const float* ap = reinterpret_cast<const float*>(p.a + static_cast<int64_t>(acol) * p.col_bytes);
    const int ahalf = tid & 1;
    const int n0 = blockIdx.y * kBN;
    const int brhs = min(n0 + tid, p.nrhs - 1);
    const float* bp = static_cast<const float*>(p.b) + static_cast<int64_t>(brhs) * p.ldb;
    uint4 ra[4], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = ldg_u4(ap + k0 + 16 * ahalf + 4 * q);
#pragma unroll
        for (int q = 0; q < 8; ++q) rb[q] = ldg_u4(bp + k0 + 4 * q);
    };
    auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(&la[tid / 2][16 * ahalf + 4 * q]) = ra[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) *reinterpret_cast<uint4*>(&lb[tid][4 * q]) = rb[q];
    };
    f32x4_t acc[4][8];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int ksteps = p.rows / kBK;
    load(0);
    for (int ks = 0; ks < ksteps; ++ks) {
        __syncthreads();
        stash();
        __syncthreads();
        if (ks + 1 < ksteps) load((ks + 1) * kBK);
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 4) {
            const int kr = kk + (lane >> 4);
            float af[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) af[mt] = la[wm + 16 * mt + (lane & 15)][kr];
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const float bv = lb[wn + 16 * nt + (lane & 15)][kr];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mt], bv, acc[mt][nt], 0, 0, 0);
            }
        }
    }
    store_tiles<4, 8>(p, p.g, acc, j0 + wm, n0 + wn, lane);
}

// Per problem (blockIdx.y): with row splits, g = the sum of the split
// partials in split order; then the histogram of the top 11 bits of |g_j| off
// the support (what the per-problem pass builds in its epilogue).
__global__ __launch_bounds__(256) void k_hist_g(const ProbDev* __restrict__ P, int ksplit,
                                                const float* __restrict__ gp, int64_t part_stride,
                                                int64_t ldg) {
    const int prob = blockIdx.y;
    const ProbDev& pd = P[prob];
    if (pd.st->done) return;
    __shared__ uint32_t lh[2048];
    for (int b = threadIdx.x; b < 2048; b += 256) lh[b] = 0u;
    __syncthreads();
    const int per = (pd.n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per, hi = min(pd.n, lo + per);
    for (int j = lo + threadIdx.x; j < hi; j += 256) {
        float gj;
        if (ksplit > 1) {
            const float* src = gp + static_cast<int64_t>(prob) * ldg + j;
            gj = src[0];
            for (int k = 1; k < ksplit; ++k) gj += src[k * part_stride];
            pd.g[j] = gj;
        } else {
            gj = pd.g[j];
        }
        if ((pd.bmsup[j >> 5] >> (j & 31)) & 1u) continue;
        atomicAdd(&lh[(__float_as_uint(gj) & 0x7FFFFFFFu) >> 20], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2048; b += 256)
        if (lh[b]) atomicAdd(&pd.hist[b], lh[b]);
}

}  // namespace

// The pass of a shared-matrix batch: G = Phi~^T R' for every problem, then
// the per-problem histograms.
void launch_shared_pass(const SharedGemm& sg, const ProbDev* P, int count, hipStream_t st,
                        hipEvent_t ev0, hipEvent_t ev1) {
    GemmArgs a;
    a.a = sg.a;
    a.col_bytes = sg.col_bytes;
    a.n = sg.n;
    a.rows = sg.rows_pad;
    a.nrhs = count;
    a.b = sg.b;
    a.ldb = sg.ldb;
    a.lo_off = sg.lo_off;
    a.g = sg.g;
    a.ldg = sg.ldg;
    a.ksplit = 1;
    a.gp = sg.gp;
    const bool bf = sg.bits == kFmtBF16 || sg.bits == kFmtE4M3;
    dim3 grid;
    if (bf) {
        a.ksplit = sg.ksplit;
        const int nb = kHN;  // right-hand sides per workgroup
        grid = dim3((sg.n + kBM2 - 1) / kBM2, (count + nb - 1) / nb, a.ksplit);
    } else {
        grid = dim3((sg.n + kBM - 1) / kBM, (count + kBN - 1) / kBN);
    }
    auto go = [&](auto kern) {
        if (ev0) hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, st, ev0, ev1, 0, a);
        else hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, a);
    };
    if (sg.bits == kFmtBF16) go(k_gemm_bf16_half);
    else if (sg.bits == kFmtE4M3) go(k_gemm_e4m3_half);
    else go(k_gemm_f32);
    hipLaunchKernelGGL(k_hist_g, dim3(std::max(1, std::min(64, (sg.n + 2047) / 2048)), count), dim3(256), 0, st,
                       P, a.ksplit, static_cast<const float*>(sg.gp), static_cast<int64_t>(count) * sg.ldg, sg.ldg);
}

// Row splits of the BF16 / E4M3 GEMMs: enough workgroups for the device (two
// per CU) while each split keeps at least 8 steps of 32 rows.
bool shared_ksplit_ok(int bits, int rows_pad, int ks) {
    if (bits != kFmtBF16 && bits != kFmtE4M3) return ks == 1;
    return (ks == 1 || ks == 2 || ks == 4) && rows_pad % (ks * kBK) == 0 && rows_pad / ks >= 8 * kBK;
}

int shared_ksplit(int bits, int n, int count, int rows_pad) {
    if (bits != kFmtBF16 && bits != kFmtE4M3) return 1;
    const int nb = kHN;
    const int want = 512;
    const int tiles = ((n + kBM2 - 1) / kBM2) * ((count + nb - 1) / nb);
    int ks = 1;
    while (ks < 4 && tiles * ks < want && shared_ksplit_ok(bits, rows_pad, 2 * ks)) ks *= 2;
    return ks;
}

}  // namespace qiht
