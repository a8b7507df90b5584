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
// Tiling: a workgroup of 4 waves computes 128 columns x 256 right-hand sides
// (so each element of A is read once), K in steps of 32 rows staged through
// LDS with the next step's global loads in flight; wave w takes columns
// 64 (w & 1) .. + 64 and right-hand sides 128 (w >> 1) .. + 128 as 4 x 8
// tiles of 16 x 16.
#include <hip/hip_ext.h>

#include <algorithm>

#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kBM = 128;  // columns of Phi per workgroup
constexpr int kBN = 256;  // right-hand sides per workgroup (at most)
constexpr int kBK = 32;   // rows per step
constexpr int kPadH = 8;  // LDS row padding in 16-bit elements

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8_t as_bf16x8(uint4 v) {
    return __builtin_bit_cast(bf16x8_t, v);
}

// Exact E4M3 -> BF16 (bit patterns): normals rebias the exponent (+120),
// subnormals k 2^-9 are normal in BF16.
__device__ __forceinline__ uint32_t e4m3_to_bf16(uint32_t b) {
    const uint32_t s = (b & 0x80u) << 8, e = (b >> 3) & 15u, m = b & 7u;
    if (e != 0u) return s | ((e + 120u) << 7) | (m << 4);
    if (m == 0u) return s;
    const uint32_t f = __float_as_uint(static_cast<float>(m) * 0x1p-9f);
    return s | (f >> 16);
}

struct GemmArgs {
    const uint8_t* a;    // stored columns, col_bytes apart
    int64_t col_bytes;
    int n;               // columns (M)
    int rows;            // K
    int nrhs;            // N
    const void* b;       // R': BF16 hi/lo (ldb 16-bit elements apart per RHS; lo at +lo_off)
    int64_t ldb;         //     or FP32 r (ldb floats apart)
    int64_t lo_off;
    float* g;            // G, g_k at g + k * ldg
    int64_t ldg;
};

// C tile (mt, nt) of a wave: lane holds rows 4 (lane / 16) + t (columns of
// Phi) of right-hand side 16 nt + lane % 16; four consecutive g_j per store.
__device__ __forceinline__ void store_tiles(const GemmArgs& p, const f32x4_t (&acc)[4][8], int jw,
                                            int kw, int lane) {
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const int k = kw + 16 * nt + (lane & 15);
        if (k >= p.nrhs) continue;
        float* gk = p.g + static_cast<int64_t>(k) * p.ldg;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
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

template <int FMT>  // 16: BF16 storage, 9: E4M3 storage
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs p) {
    __shared__ uint16_t la[kBM][kBK + kPadH];
    __shared__ uint16_t lb[2][kBN][kBK + kPadH];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j0 = blockIdx.x * kBM;
    const int wm = (wv & 1) * 64, wn = (wv >> 1) * 128;

    // global -> register assignment: A: column tid / 2, rows 16 (tid % 2) .. + 16
    const int acol = min(j0 + tid / 2, p.n - 1);
    const uint8_t* ap = p.a + static_cast<int64_t>(acol) * p.col_bytes;
    const int ahalf = tid & 1;
    // B: right-hand side tid (clamped), both terms, 32 rows
    const int n0 = blockIdx.y * kBN;  // first right-hand side of this workgroup
    const int brhs = min(n0 + tid, p.nrhs - 1);
    const uint16_t* bh = static_cast<const uint16_t*>(p.b) + static_cast<int64_t>(brhs) * p.ldb;
    const uint16_t* bl = bh + p.lo_off;

    uint4 ra[2], rbh[4], rbl[4];
    auto load = [&](int k0) {
        if constexpr (FMT == 16) {
            const uint16_t* src = reinterpret_cast<const uint16_t*>(ap) + k0 + 16 * ahalf;
            ra[0] = ldg_u4(src);
            ra[1] = ldg_u4(src + 8);
        } else {
            ra[0] = ldg_u4(ap + k0 + 16 * ahalf);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rbh[q] = ldg_u4(bh + k0 + 8 * q);
            rbl[q] = ldg_u4(bl + k0 + 8 * q);
        }
    };
    auto stash = [&]() {
        uint16_t* dst = &la[tid / 2][16 * ahalf];
        if constexpr (FMT == 16) {
            *reinterpret_cast<uint4*>(dst) = ra[0];
            *reinterpret_cast<uint4*>(dst + 8) = ra[1];
        } else {
            const uint32_t w[4] = {ra[0].x, ra[0].y, ra[0].z, ra[0].w};
            uint32_t o[8];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o[2 * q] = e4m3_to_bf16(w[q] & 0xFFu) | (e4m3_to_bf16((w[q] >> 8) & 0xFFu) << 16);
                o[2 * q + 1] = e4m3_to_bf16((w[q] >> 16) & 0xFFu) | (e4m3_to_bf16(w[q] >> 24) << 16);
            }
            *reinterpret_cast<uint4*>(dst) = make_uint4(o[0], o[1], o[2], o[3]);
            *reinterpret_cast<uint4*>(dst + 8) = make_uint4(o[4], o[5], o[6], o[7]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<uint4*>(&lb[0][tid][8 * q]) = rbh[q];
            *reinterpret_cast<uint4*>(&lb[1][tid][8 * q]) = rbl[q];
        }
    };

    f32x4_t acc[4][8];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    const int ksteps = p.rows / kBK;  // rows is a multiple of 32 (columns are padded)
    load(0);
    for (int ks = 0; ks < ksteps; ++ks) {
        __syncthreads();
        stash();
        __syncthreads();
        if (ks + 1 < ksteps) load((ks + 1) * kBK);
        const int kq = (lane >> 4) * 8;  // this lane's 8 rows of the step
        bf16x8_t af[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            af[mt] = as_bf16x8(*reinterpret_cast<const uint4*>(&la[wm + 16 * mt + (lane & 15)][kq]));
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            const int col = wn + 16 * nt + (lane & 15);
            const bf16x8_t bh8 = as_bf16x8(*reinterpret_cast<const uint4*>(&lb[0][col][kq]));
            const bf16x8_t bl8 = as_bf16x8(*reinterpret_cast<const uint4*>(&lb[1][col][kq]));
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bh8, acc[mt][nt], 0, 0, 0);
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bl8, acc[mt][nt], 0, 0, 0);
            }
        }
    }
    store_tiles(p, acc, j0 + wm, n0 + wn, lane);
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
    store_tiles(p, acc, j0 + wm, n0 + wn, lane);
}

// Histogram of the top 11 bits of |g_j| off the support, per problem (what
// the per-problem pass builds in its epilogue): blockIdx.y = problem.
__global__ __launch_bounds__(256) void k_hist_g(const ProbDev* __restrict__ P) {
    const ProbDev& pd = P[blockIdx.y];
    if (pd.st->done) return;
    __shared__ uint32_t lh[2048];
    for (int b = threadIdx.x; b < 2048; b += 256) lh[b] = 0u;
    __syncthreads();
    const int per = (pd.n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per, hi = min(pd.n, lo + per);
    for (int j = lo + threadIdx.x; j < hi; j += 256) {
        if ((pd.bmsup[j >> 5] >> (j & 31)) & 1u) continue;
        atomicAdd(&lh[(__float_as_uint(pd.g[j]) & 0x7FFFFFFFu) >> 20], 1u);
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
    const dim3 grid((sg.n + kBM - 1) / kBM, (count + kBN - 1) / kBN);
    auto go = [&](auto kern) {
        if (ev0) hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, st, ev0, ev1, 0, a);
        else hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, a);
    };
    if (sg.bits == kFmtBF16) go(k_gemm_bf16<16>);
    else if (sg.bits == kFmtE4M3) go(k_gemm_bf16<9>);
    else go(k_gemm_f32);
    hipLaunchKernelGGL(k_hist_g, dim3(std::max(1, std::min(64, (sg.n + 2047) / 2048)), count), dim3(256), 0, st, P);
}

}  // namespace qiht
