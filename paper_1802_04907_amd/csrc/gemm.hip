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
// (so each element of A is read once per 256 right-hand sides), K in steps
// of 32 rows staged through LDS.
//   k_gemm_bf16_half (BF16): 256 columns x 128 right-hand sides, two
//     workgroups per CU, LDS-direct loads one step ahead, details below.
//   k_gemm_bf16<9> (E4M3): 256 columns x 256 right-hand sides, one
//     workgroup per CU (a wave holds a 128 x 128 block of G: 8 x 8 tiles of
//     16 x 16 in 256 accumulator registers), loads through registers one
//     step ahead, LDS double-buffered.
//   k_gemm_f32 (FP32): 128 columns x 256 right-hand sides.
#include <hip/hip_ext.h>

#include <algorithm>

#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kBM = 128;  // FP32 kernel: columns of Phi per workgroup
constexpr int kBN = 256;  // right-hand sides per workgroup (at most)
constexpr int kBK = 32;   // rows per step
constexpr int kBM2 = 256; // BF16 kernel: columns of Phi per workgroup

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

// BF16 and E4M3 storage.  A workgroup of 4 waves computes 256 columns of Phi
// x 256 right-hand sides over its row split, each wave a 128 x 128 block (8 x 8
// tiles of 16 x 16, two MFMAs per tile and step: hi and lo), so every LDS
// fragment read feeds 8 or 16 MFMAs.  Steps of 32 rows.  The next step's global loads
// are in flight during the MFMAs; LDS is double-buffered, so one barrier per
// step both publishes a buffer and retires the other.
// LDS rows of the BF16 kernels are 64 bytes (the 32 rows of one step of one
// column or right-hand side), unpadded; the four 16-byte pieces of row r sit
// at piece ^ dma_swz(r % 16).  A fragment read (16 consecutive lanes: rows
// r..r+15 of one piece) then touches every bank once: on gfx950 a 16-byte
// LDS read serves 16 lanes per cycle over 64 banks, and this is the placement
// a probe of the bank counter found conflict-free (80-byte padded rows cost
// one extra cycle per read).
__device__ __forceinline__ int dma_swz(int r) { return (r >> 1) & 3; }
__device__ __forceinline__ int lds_slot(int r, int piece) { return r * 64 + 16 * (piece ^ dma_swz(r & 15)); }

template <int FMT>
struct Stage {
    uint4 a[FMT == 16 ? 4 : 2];  // A: 16 bytes of each of this thread's columns
    uint4 bh[4], bl[4];          // R': 16 bytes of each of its 4 right-hand sides, both terms
};

template <int FMT>  // 16: BF16 storage, 9: E4M3 storage
__global__ __launch_bounds__(256, 1) void k_gemm_bf16(GemmArgs p) {
    __shared__ __attribute__((aligned(16))) uint8_t la[2][kBM2 * 64];
    __shared__ __attribute__((aligned(16))) uint8_t lb[2][2][kBN * 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j0 = blockIdx.x * kBM2;
    const int n0 = blockIdx.y * kBN;
    const int kper = p.rows / p.ksplit;
    const int kbeg = blockIdx.z * kper;
    const int wm = (wv & 1) * 128, wn = (wv >> 1) * 128;

    // Global -> LDS mapping: consecutive lanes share a column (so a wave's
    // load touches a few long contiguous pieces, not 64 scattered ones).
    // BF16 A and both R' terms: 4 lanes x 16 bytes = the 32 rows of one
    // column, lanes tid / 4 + 64 i, i < 4.  E4M3 A: 2 lanes x 16 bytes, columns
    // tid / 2 + 128 i, i < 2.
    constexpr int AL = FMT == 16 ? 4 : 2;       // lanes per column of A
    constexpr int AI = 256 * AL / 256;          // columns of A per thread (= AL)
    const int akc = tid % AL;                   // 16-byte piece of the column
    const uint8_t* ap[AI];
#pragma unroll
    for (int i = 0; i < AI; ++i) {
        const int col = min(j0 + tid / AL + (256 / AL) * i, p.n - 1);
        ap[i] = p.a + static_cast<int64_t>(col) * p.col_bytes + 16 * akc;
    }
    const int bkc = tid % 4;
    const uint16_t* bp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rhs = min(n0 + tid / 4 + 64 * i, p.nrhs - 1);
        bp[i] = static_cast<const uint16_t*>(p.b) + static_cast<int64_t>(rhs) * p.ldb + 8 * bkc;
    }

    // k0 in rows; a 16-bit element is 2 bytes, an E4M3 one 1
    auto load = [&](Stage<FMT>& r, int k0) {
#pragma unroll
        for (int i = 0; i < AI; ++i) r.a[i] = ldg_u4(ap[i] + (FMT == 16 ? 2 : 1) * k0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            r.bh[i] = ldg_u4(bp[i] + k0);
            r.bl[i] = ldg_u4(bp[i] + p.lo_off + k0);
        }
    };
    auto stash = [&](const Stage<FMT>& r, int buf) {
        if constexpr (FMT == 16) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                *reinterpret_cast<uint4*>(&la[buf][lds_slot(tid / 4 + 64 * i, akc)]) = r.a[i];
        } else {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const uint2 a0 = e4m3x4_to_bf16(r.a[i].x), a1 = e4m3x4_to_bf16(r.a[i].y);
                const uint2 a2 = e4m3x4_to_bf16(r.a[i].z), a3 = e4m3x4_to_bf16(r.a[i].w);
                const int col = tid / 2 + 128 * i;  // 16 codes: BF16 pieces 2 akc and 2 akc + 1
                *reinterpret_cast<uint4*>(&la[buf][lds_slot(col, 2 * akc)]) = make_uint4(a0.x, a0.y, a1.x, a1.y);
                *reinterpret_cast<uint4*>(&la[buf][lds_slot(col, 2 * akc + 1)]) = make_uint4(a2.x, a2.y, a3.x, a3.y);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *reinterpret_cast<uint4*>(&lb[buf][0][lds_slot(tid / 4 + 64 * i, bkc)]) = r.bh[i];
            *reinterpret_cast<uint4*>(&lb[buf][1][lds_slot(tid / 4 + 64 * i, bkc)]) = r.bl[i];
        }
    };

    f32x4_t acc[8][8];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // this lane's fragment piece: row lane % 16 of a 16-row block, piece
    // lane / 16 (8 rows of the step)
    const int foff = lds_slot(lane & 15, lane >> 4);
    auto compute = [&](int buf) {
        bf16x8_t af[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
            af[mt] = as_bf16x8(*reinterpret_cast<const uint4*>(&la[buf][(wm + 16 * mt) * 64 + foff]));
        // B fragments one tile column ahead of the MFMAs that use them
        auto bfrag = [&](int term, int nt) {
            return as_bf16x8(*reinterpret_cast<const uint4*>(&lb[buf][term][(wn + 16 * nt) * 64 + foff]));
        };
        bf16x8_t bhn = bfrag(0, 0), bln = bfrag(1, 0);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            const bf16x8_t bh8 = bhn, bl8 = bln;
            if (nt + 1 < 8) {
                bhn = bfrag(0, nt + 1);
                bln = bfrag(1, nt + 1);
            }
            // hi terms of the 8 tiles, then the lo terms: consecutive MFMAs
            // never wait on each other's accumulator
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bh8, acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bl8, acc[mt][nt], 0, 0, 0);
        }
        // instruction order of the step: the A fragments and the first B pair,
        // then per tile column the next B pair ahead of its 16 MFMAs (so an
        // LDS read's latency hides behind MFMAs already issued)
        __builtin_amdgcn_sched_group_barrier(0x100, 10, 0);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            if (nt + 1 < 8) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
        }
    };

    // step t's data: registers (loaded one step ahead), then LDS buffer t % 2
    const int ksteps = kper / kBK;  // >= 8, see shared_ksplit
    Stage<FMT> r;
    load(r, kbeg);
    for (int ks = 0; ks < ksteps; ++ks) {
        const int buf = ks & 1;
        stash(r, buf);
        if (ks + 1 < ksteps) load(r, kbeg + (ks + 1) * kBK);
        // the stash is visible, and buffer buf ^ 1 (step ks - 1) is no longer read
        __syncthreads();
        compute(buf);
    }
    float* out = p.ksplit > 1 ? p.gp + static_cast<int64_t>(blockIdx.z) * p.nrhs * p.ldg : p.g;
    store_tiles<8, 8>(p, out, acc, j0 + wm, n0 + wn, lane);
}

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
// and loads two steps ahead ran 8% slower; the register-staged kernel 22%.)
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
        const int nb = sg.bits == kFmtBF16 ? kHN : kBN;  // right-hand sides per workgroup
        grid = dim3((sg.n + kBM2 - 1) / kBM2, (count + nb - 1) / nb, a.ksplit);
    } else {
        grid = dim3((sg.n + kBM - 1) / kBM, (count + kBN - 1) / kBN);
    }
    auto go = [&](auto kern) {
        if (ev0) hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, st, ev0, ev1, 0, a);
        else hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, a);
    };
    if (sg.bits == kFmtBF16) go(k_gemm_bf16_half);
    else if (sg.bits == kFmtE4M3) go(k_gemm_bf16<9>);
    else go(k_gemm_f32);
    hipLaunchKernelGGL(k_hist_g, dim3(std::max(1, std::min(64, (sg.n + 2047) / 2048)), count), dim3(256), 0, st,
                       P, a.ksplit, static_cast<const float*>(sg.gp), static_cast<int64_t>(count) * sg.ldg, sg.ldg);
}

// Row splits of the BF16 / E4M3 GEMMs: enough workgroups for the device (two
// per CU for BF16, one for E4M3) while each split keeps at least 8 steps of
// 32 rows.
bool shared_ksplit_ok(int bits, int rows_pad, int ks) {
    if (bits != kFmtBF16 && bits != kFmtE4M3) return ks == 1;
    return (ks == 1 || ks == 2 || ks == 4) && rows_pad % (ks * kBK) == 0 && rows_pad / ks >= 8 * kBK;
}

int shared_ksplit(int bits, int n, int count, int rows_pad) {
    if (bits != kFmtBF16 && bits != kFmtE4M3) return 1;
    const int nb = bits == kFmtBF16 ? kHN : kBN;
    const int want = bits == kFmtBF16 ? 512 : 256;
    const int tiles = ((n + kBM2 - 1) / kBM2) * ((count + nb - 1) / nb);
    int ks = 1;
    while (ks < 4 && tiles * ks < want && shared_ksplit_ok(bits, rows_pad, 2 * ks)) ks *= 2;
    return ks;
}

}  // namespace qiht
