// Least-squares refit of x on a fixed support, in FP64: the normal equations
// A_G^T A_G z = A_G^T y solved by a blocked Cholesky factorization.  This is
// an addition to QIHT (the method returns its last iterate); it removes the
// step-size and quantization bias of x on the recovered support.  A is the
// caller's dense Phi, or the dequantized first realization of the codes.
//
// Batched: every kernel serves a group of problems (blockIdx.z = problem, its
// parameters and workspace in a RefitDev), so the refits of a batched solve
// are one sequence of launches.
//
// Layout per problem: A_G is lda x s, column-major (column t = column sup[t]
// of A, lda = rows rounded up to 16, padding rows 0); G = A_G^T A_G is s x s,
// row-major, lower triangle used (the Cholesky factor L overwrites it);
// b = A_G^T y.
#include <algorithm>
#include <vector>

#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kNB = 32;    // Cholesky block
constexpr int kTile = 64;  // trailing-update tile (16 x 16 threads, 4 x 4 each)
constexpr int kGT = 64;    // Gram tile of one wave (4 x 4 MFMA tiles of 16 x 16)
constexpr int kGK = 16;    // rows per Gram chunk (4 MFMA steps of 4 rows)

struct RefitDev {
    const uint8_t* codes;  // stored matrix (codes path)
    int64_t col_bytes;
    double alpha, beta;
    const int32_t* rowexp;
    const void* phi;       // dense Phi (phi path)
    int64_t m, ld;
    int64_t rows, lda, n;
    int s;
    int64_t split;         // Gram rows per split (a multiple of kGK)
    const double* y;
    const int32_t* sup;
    float* x_out;
    double* xs_out;
    double *A, *Gp, *G, *b, *diag;
    int* flag;
};

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// Column t of A_G from the stored matrix: alpha code + beta (packed codes),
// the float (32), or 2^e_i times the stored value (dense formats).
template <int BITS>
__global__ __launch_bounds__(256) void k_refit_codes(const RefitDev* __restrict__ R) {
    constexpr int RPW = rows_per_word<BITS>();
    const RefitDev& r = R[blockIdx.z];
    const int t = blockIdx.y;
    if (t >= r.s) return;
    const uint8_t* col = r.codes + static_cast<int64_t>(r.sup[t]) * r.col_bytes;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < r.lda;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        double v = 0.0;
        if (i < r.rows) {
            const uint32_t w = reinterpret_cast<const uint32_t*>(col)[i / RPW];
            const double e = elem_at<BITS>(w, static_cast<int>(i % RPW));
            if constexpr (BITS == 32) v = e;
            else if constexpr (BITS == 9 || BITS == 16) v = ldexp(e, r.rowexp[i]);
            else v = r.alpha * e + r.beta;
        }
        r.A[static_cast<int64_t>(t) * r.lda + i] = v;
    }
}

// Column t of A_G from a dense row-major Phi (real, or complex interleaved:
// the stacked real matrix [Re Phi; Im Phi] of 2m rows).
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void k_refit_phi(const RefitDev* __restrict__ R) {
    const RefitDev& r = R[blockIdx.z];
    const int t = blockIdx.y;
    if (t >= r.s) return;
    const T* phi = static_cast<const T*>(r.phi);
    const int64_t j = r.sup[t];
    const int64_t m = r.m;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < r.lda;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        double v = 0.0;
        if (i < r.rows) {
            if (CPLX) {
                const int64_t q = i < m ? i : i - m;
                v = static_cast<double>(phi[2 * (q * r.ld + j) + (i < m ? 0 : 1)]);
            } else {
                v = static_cast<double>(phi[i * r.ld + j]);
            }
        }
        r.A[static_cast<int64_t>(t) * r.lda + i] = v;
    }
}

// Tile (I, J), I >= J, of the partial Gram product of row split blockIdx.y,
// on the FP64 matrix cores: one wave, 64 x 64 entries as 4 x 4 tiles of
// v_mfma_f64_16x16x4 (A operand: lane l holds row l % 16, step row l / 16;
// B operand: step row l / 16, column l % 16; result element t of lane l:
// row l / 16 + 4 t, column l % 16).  Per chunk of 16 rows lane l reads rows 4 (l / 16) .. + 3
// of its columns (one 32-byte piece; the four lanes of a column read 128
// contiguous bytes) and feeds them to the four MFMA steps in turn.  Columns
// past s read column s - 1 and are not stored.
__global__ __launch_bounds__(64) void k_refit_gram(const RefitDev* __restrict__ R) {
    const RefitDev& r = R[blockIdx.z];
    const int s = r.s;
    const int T = (s + kGT - 1) / kGT;
    if (static_cast<int>(blockIdx.x) >= T * (T + 1) / 2) return;
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * r.split;
    if (r0 >= r.lda) return;
    const int64_t r1 = min(r.lda, r0 + r.split);
    int I = 0, rem = blockIdx.x;
    while (rem > I) {
        rem -= I + 1;
        ++I;
    }
    const int J = rem;
    const int lane = threadIdx.x, c = lane & 15, kq = lane >> 4;
    const double* pa[4];
    const double* pb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        pa[q] = r.A + static_cast<int64_t>(min(I * kGT + 16 * q + c, s - 1)) * r.lda + 4 * kq;
        pb[q] = r.A + static_cast<int64_t>(min(J * kGT + 16 * q + c, s - 1)) * r.lda + 4 * kq;
    }
    f64x4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = r0; k0 < r1; k0 += kGK) {
        double4 va[4], vb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            va[q] = *reinterpret_cast<const double4*>(pa[q] + k0);
            vb[q] = *reinterpret_cast<const double4*>(pb[q] + k0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double xa = t == 0 ? va[a].x : t == 1 ? va[a].y : t == 2 ? va[a].z : va[a].w;
                    const double xb = t == 0 ? vb[b].x : t == 1 ? vb[b].y : t == 2 ? vb[b].z : vb[b].w;
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, xb, acc[a][b], 0, 0, 0);
                }
    }
    double* G = r.Gp + static_cast<int64_t>(blockIdx.y) * s * s;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = I * kGT + 16 * a + kq + 4 * t, j = J * kGT + 16 * b + c;
                if (i < s && j <= i) G[static_cast<int64_t>(i) * s + j] = acc[a][b][t];
            }
}

// G = sum of the row-split partials, in split order (lower triangle).  The
// diagonal is also kept aside: the factorization judges its pivots against it.
__global__ __launch_bounds__(256) void k_refit_gram_sum(const RefitDev* __restrict__ R, int ks) {
    const RefitDev& r = R[blockIdx.z];
    const int s = r.s;
    const int64_t total = static_cast<int64_t>(s) * s;
    const int nsplit = static_cast<int>(min<int64_t>(ks, (r.lda + r.split - 1) / r.split));
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * 256) {
        if (e % s > e / s) continue;
        double v = 0.0;
        for (int q = 0; q < nsplit; ++q) v += r.Gp[q * total + e];
        r.G[e] = v;
        if (e % s == e / s) r.diag[e / s] = v;
    }
}

// b = A^T y, one workgroup per column, fixed summation order; the flag is
// cleared here.
__global__ __launch_bounds__(256) void k_refit_rhs(const RefitDev* __restrict__ R) {
    const RefitDev& r = R[blockIdx.z];
    const int t = blockIdx.x;
    if (t >= r.s) return;
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < r.rows; i += 256) acc = fma(r.A[static_cast<int64_t>(t) * r.lda + i], r.y[i], acc);
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) {
        r.b[t] = acc;
        if (t == 0) *r.flag = 0;
    }
}

// Cholesky of the nb x nb diagonal block at (k0, k0), in LDS.  A pivot at or
// below kPivotRel times the column's own Gram diagonal means the support
// columns are (numerically) linearly dependent.
constexpr double kPivotRel = 1e-12;

__global__ __launch_bounds__(256) void k_potrf_diag(const RefitDev* __restrict__ R, int k0) {
    const RefitDev& r = R[blockIdx.z];
    const int s = r.s;
    if (k0 >= s || *r.flag) return;
    double* G = r.G;
    __shared__ double L[kNB][kNB + 1];
    const int nb = min(kNB, s - k0);
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        const int i = e / nb, j = e % nb;
        L[i][j] = G[static_cast<int64_t>(k0 + i) * s + k0 + j];
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        const double d = L[k][k];
        if (!(d > kPivotRel * r.diag[k0 + k]) || !isfinite(d)) {
            if (threadIdx.x == 0) atomicOr(r.flag, 1);
            return;  // uniform: every thread read the same d
        }
        const double rt = sqrt(d);
        __syncthreads();
        if (threadIdx.x == 0) L[k][k] = rt;
        for (int i = k + 1 + threadIdx.x; i < nb; i += 256) L[i][k] /= rt;
        __syncthreads();
        for (int e = threadIdx.x; e < nb * nb; e += 256) {
            const int i = e / nb, j = e % nb;
            if (j > k && i >= j) L[i][j] -= L[i][k] * L[j][k];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        const int i = e / nb, j = e % nb;
        if (i >= j) G[static_cast<int64_t>(k0 + i) * s + k0 + j] = L[i][j];
    }
}

// Panel below the diagonal block: rows i >= k0 + nb solve x L11^T = a.
__global__ __launch_bounds__(256) void k_trsm_panel(const RefitDev* __restrict__ R, int k0) {
    const RefitDev& r = R[blockIdx.z];
    const int s = r.s;
    if (k0 >= s || *r.flag) return;
    double* G = r.G;
    __shared__ double L[kNB][kNB + 1];
    const int nb = min(kNB, s - k0);
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        const int i = e / nb, j = e % nb;
        L[i][j] = (i >= j) ? G[static_cast<int64_t>(k0 + i) * s + k0 + j] : 0.0;
    }
    __syncthreads();
    const int i = k0 + nb + blockIdx.x * 256 + threadIdx.x;
    if (i >= s) return;
    double* row = G + static_cast<int64_t>(i) * s + k0;
    double x[kNB];
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        if (k < nb) {
            double v = row[k];
#pragma unroll
            for (int l = 0; l < kNB; ++l)
                if (l < k) v -= x[l] * L[k][l];
            x[k] = v / L[k][k];
        } else {
            x[k] = 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < kNB; ++k)
        if (k < nb) row[k] = x[k];
}

// Trailing update: A22 -= L21 L21^T on the lower triangle, 64 x 64 tiles.
__global__ __launch_bounds__(256) void k_syrk_update(const RefitDev* __restrict__ R, int k0) {
    const RefitDev& r = R[blockIdx.z];
    const int s = r.s;
    if (k0 >= s || *r.flag) return;
    const int nb = min(kNB, s - k0);
    const int base = k0 + nb;  // first trailing row / column
    const int Tr = (s - base + kTile - 1) / kTile;
    if (static_cast<int>(blockIdx.x) >= Tr * (Tr + 1) / 2) return;
    double* G = r.G;
    int I = 0, rem = blockIdx.x;
    while (rem > I) {
        rem -= I + 1;
        ++I;
    }
    const int J = rem;
    __shared__ double pa[kNB][kTile + 1];
    __shared__ double pb[kNB][kTile + 1];
    for (int e = threadIdx.x; e < kNB * kTile; e += 256) {
        const int k = e % kNB, c = e / kNB;
        const int ri = base + I * kTile + c, rj = base + J * kTile + c;
        pa[k][c] = (k < nb && ri < s) ? G[static_cast<int64_t>(ri) * s + k0 + k] : 0.0;
        pb[k][c] = (k < nb && rj < s) ? G[static_cast<int64_t>(rj) * s + k0 + k] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 8
    for (int k = 0; k < kNB; ++k) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(pa[k][ty * 4 + a], pb[k][tx * 4 + b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = base + I * kTile + ty * 4 + a, j = base + J * kTile + tx * 4 + b;
            if (i < s && j <= i) G[static_cast<int64_t>(i) * s + j] -= acc[a][b];
        }
}

// L z = b then L^T x = z, by blocks of kNB: each diagonal block (staged in
// LDS) solved by wave 0 in order, one lane per row, the rest of the
// right-hand side updated by all threads.  b (s doubles) is overwritten with x.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

__global__ __launch_bounds__(1024) void k_refit_solve(const RefitDev* __restrict__ R) {
    const RefitDev& r = R[blockIdx.z];
    if (*r.flag) return;
    const int s = r.s;
    const double* G = r.G;
    double* b = r.b;
    __shared__ double D[kNB][kNB + 1];
    __shared__ double z[kNB];
    const int tid = threadIdx.x;
    // forward: L z = b
    for (int k0 = 0; k0 < s; k0 += kNB) {
        const int nb = min(kNB, s - k0);
        for (int e = tid; e < nb * nb; e += 1024) D[e / nb][e % nb] = G[static_cast<int64_t>(k0 + e / nb) * s + k0 + e % nb];
        __syncthreads();
        if (tid < 64) {
            double v = tid < nb ? b[k0 + tid] : 0.0;
            for (int k = 0; k < nb; ++k) {
                const double zk = readlane_f64(v / D[min(tid, nb - 1)][min(tid, nb - 1)], k);
                if (tid > k && tid < nb) v -= D[tid][k] * zk;
                if (tid == k) v = zk;
            }
            if (tid < nb) {
                z[tid] = v;
                b[k0 + tid] = v;
            }
        }
        __syncthreads();
        for (int i = k0 + nb + tid; i < s; i += 1024) {
            double v = b[i];
            for (int k = 0; k < nb; ++k) v -= G[static_cast<int64_t>(i) * s + k0 + k] * z[k];
            b[i] = v;
        }
        __syncthreads();
    }
    // backward: L^T x = z
    const int last = ((s - 1) / kNB) * kNB;
    for (int k0 = last; k0 >= 0; k0 -= kNB) {
        const int nb = min(kNB, s - k0);
        for (int e = tid; e < nb * nb; e += 1024) D[e / nb][e % nb] = G[static_cast<int64_t>(k0 + e / nb) * s + k0 + e % nb];
        __syncthreads();
        if (tid < 64) {
            double v = tid < nb ? b[k0 + tid] : 0.0;
            for (int k = nb - 1; k >= 0; --k) {
                const double xk = readlane_f64(v / D[min(tid, nb - 1)][min(tid, nb - 1)], k);
                if (tid < k) v -= D[k][tid] * xk;
                if (tid == k) v = xk;
            }
            if (tid < nb) {
                z[tid] = v;
                b[k0 + tid] = v;
            }
        }
        __syncthreads();
        for (int i = tid; i < k0; i += 1024) {
            double v = b[i];
            for (int k = 0; k < nb; ++k) v -= G[static_cast<int64_t>(k0 + k) * s + i] * z[k];
            b[i] = v;
        }
        __syncthreads();
    }
}

// x_out: zero off the support, then x_out[sup[t]] = x_t (FP32); xs_out
// (optional) = x (FP64).
__global__ __launch_bounds__(256) void k_refit_zero(const RefitDev* __restrict__ R) {
    const RefitDev& r = R[blockIdx.z];
    if (*r.flag) return;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < r.n;
         j += static_cast<int64_t>(gridDim.x) * 256)
        r.x_out[j] = 0.0f;
}

__global__ __launch_bounds__(256) void k_refit_scatter(const RefitDev* __restrict__ R) {
    const RefitDev& r = R[blockIdx.z];
    if (*r.flag) return;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < r.s; t += gridDim.x * 256) {
        r.x_out[r.sup[t]] = static_cast<float>(r.b[t]);
        if (r.xs_out) r.xs_out[t] = r.b[t];
    }
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace of one problem with `ks` Gram row splits.
size_t refit_bytes(int64_t lda, int64_t s, int ks) {
    const size_t ss = static_cast<size_t>(s) * static_cast<size_t>(s) * sizeof(double);
    return up256(static_cast<size_t>(lda) * static_cast<size_t>(s) * sizeof(double)) +
           up256(static_cast<size_t>(ks) * ss) + up256(ss) + 2 * up256(static_cast<size_t>(s) * sizeof(double)) + 256;
}

int64_t lda_of(int64_t rows) { return (rows + kGK - 1) / kGK * kGK; }

// Launch the refit of problems [0, cnt) whose RefitDev array is at dR (device).
void launch_group(const RefitIn& k, const RefitDev* dR, int cnt, int ks, int64_t max_lda, int max_s,
                  int64_t max_n, hipStream_t st) {
    const dim3 gcol(static_cast<unsigned>(std::min<int64_t>((max_lda + 255) / 256, 64)), max_s, cnt);
    if (k.phi) {
        switch (k.dtype) {
            case QIHT_F64: hipLaunchKernelGGL((k_refit_phi<double, false>), gcol, dim3(256), 0, st, dR); break;
            case QIHT_F32: hipLaunchKernelGGL((k_refit_phi<float, false>), gcol, dim3(256), 0, st, dR); break;
            case QIHT_C128: hipLaunchKernelGGL((k_refit_phi<double, true>), gcol, dim3(256), 0, st, dR); break;
            default: hipLaunchKernelGGL((k_refit_phi<float, true>), gcol, dim3(256), 0, st, dR); break;
        }
    } else {
        switch (k.bits) {
            case 1: hipLaunchKernelGGL((k_refit_codes<1>), gcol, dim3(256), 0, st, dR); break;
            case 2: hipLaunchKernelGGL((k_refit_codes<2>), gcol, dim3(256), 0, st, dR); break;
            case 4: hipLaunchKernelGGL((k_refit_codes<4>), gcol, dim3(256), 0, st, dR); break;
            case 8: hipLaunchKernelGGL((k_refit_codes<8>), gcol, dim3(256), 0, st, dR); break;
            case 9: hipLaunchKernelGGL((k_refit_codes<9>), gcol, dim3(256), 0, st, dR); break;
            case 16: hipLaunchKernelGGL((k_refit_codes<16>), gcol, dim3(256), 0, st, dR); break;
            default: hipLaunchKernelGGL((k_refit_codes<32>), gcol, dim3(256), 0, st, dR); break;
        }
    }
    const int T = (max_s + kGT - 1) / kGT;
    hipLaunchKernelGGL(k_refit_gram, dim3(T * (T + 1) / 2, ks, cnt), dim3(64), 0, st, dR);
    hipLaunchKernelGGL(k_refit_gram_sum,
                       dim3(static_cast<unsigned>(std::min<int64_t>((static_cast<int64_t>(max_s) * max_s + 255) / 256, 1024)), 1, cnt),
                       dim3(256), 0, st, dR, ks);
    hipLaunchKernelGGL(k_refit_rhs, dim3(max_s, 1, cnt), dim3(256), 0, st, dR);
    for (int k0 = 0; k0 < max_s; k0 += kNB) {
        hipLaunchKernelGGL(k_potrf_diag, dim3(1, 1, cnt), dim3(256), 0, st, dR, k0);
        const int rest = max_s - k0 - std::min(kNB, max_s - k0);
        if (rest > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 255) / 256, 1, cnt), dim3(256), 0, st, dR, k0);
            const int Tr = (rest + kTile - 1) / kTile;
            hipLaunchKernelGGL(k_syrk_update, dim3(Tr * (Tr + 1) / 2, 1, cnt), dim3(256), 0, st, dR, k0);
        }
    }
    hipLaunchKernelGGL(k_refit_solve, dim3(1, 1, cnt), dim3(1024), 0, st, dR);
    hipLaunchKernelGGL(k_refit_zero, dim3(static_cast<unsigned>(std::min<int64_t>((max_n + 255) / 256, 1024)), 1, cnt),
                       dim3(256), 0, st, dR);
    hipLaunchKernelGGL(k_refit_scatter, dim3((max_s + 255) / 256, 1, cnt), dim3(256), 0, st, dR);
}

}  // namespace

qiht_status run_refit_batch(const RefitIn* in, int count, hipStream_t st) {
    // groups whose workspaces together stay under the cap
    constexpr size_t kCap = size_t(2) << 30;
    int first = 0;
    while (first < count) {
        // row splits: enough Gram waves for the device, each split >= 64 rows
        int last = first;
        size_t bytes = 0;
        int64_t tiles = 0, min_lda = INT64_MAX;
        while (last < count) {
            const int64_t lda = lda_of(in[last].rows);
            const size_t b1 = refit_bytes(lda, in[last].s, 1);
            if (last > first && bytes + b1 > kCap / 2) break;
            bytes += b1;
            const int64_t T = (in[last].s + kGT - 1) / kGT;
            tiles += T * (T + 1) / 2;
            min_lda = std::min(min_lda, lda);
            ++last;
        }
        const int cnt = last - first;
        int ks = 1;
        while (ks < 256 && tiles * ks < 2048 && min_lda / (2 * ks) >= 64) ks *= 2;
        std::vector<RefitDev> h(cnt);
        std::vector<size_t> off(cnt);
        size_t total = up256(sizeof(RefitDev) * cnt) + up256(sizeof(int) * cnt);
        int64_t max_lda = 0, max_n = 0;
        int max_s = 0;
        for (int i = 0; i < cnt; ++i) {
            const RefitIn& q = in[first + i];
            off[i] = total;
            total += refit_bytes(lda_of(q.rows), q.s, ks);
            max_lda = std::max(max_lda, lda_of(q.rows));
            max_s = std::max(max_s, static_cast<int>(q.s));
            max_n = std::max(max_n, q.n);
        }
        uint8_t* ws = nullptr;
        if (pool_malloc(reinterpret_cast<void**>(&ws), total, st) != hipSuccess || !ws) {
            (void)hipGetLastError();
            return fail(QIHT_ERR_OUT_OF_MEMORY, "refit workspace");
        }
        int* flags = reinterpret_cast<int*>(ws + up256(sizeof(RefitDev) * cnt));
        for (int i = 0; i < cnt; ++i) {
            const RefitIn& q = in[first + i];
            RefitDev& d = h[i];
            d = RefitDev{};
            d.codes = q.codes;
            d.col_bytes = q.col_bytes;
            d.alpha = q.alpha;
            d.beta = q.beta;
            d.rowexp = q.rowexp;
            d.phi = q.phi;
            d.m = q.m;
            d.ld = q.ld;
            d.rows = q.rows;
            d.lda = lda_of(q.rows);
            d.n = q.n;
            d.s = static_cast<int>(q.s);
            d.split = ((d.lda + ks - 1) / ks + kGK - 1) / kGK * kGK;
            d.y = q.y;
            d.sup = q.sup;
            d.x_out = q.x_out;
            d.xs_out = q.xs_out;
            uint8_t* p = ws + off[i];
            const size_t ss = static_cast<size_t>(q.s) * static_cast<size_t>(q.s) * sizeof(double);
            d.A = reinterpret_cast<double*>(p);
            p += up256(static_cast<size_t>(d.lda) * static_cast<size_t>(q.s) * sizeof(double));
            d.Gp = reinterpret_cast<double*>(p);
            p += up256(static_cast<size_t>(ks) * ss);
            d.G = reinterpret_cast<double*>(p);
            p += up256(ss);
            d.b = reinterpret_cast<double*>(p);
            p += up256(static_cast<size_t>(q.s) * sizeof(double));
            d.diag = reinterpret_cast<double*>(p);
            d.flag = flags + i;
        }
        RefitDev* dR = reinterpret_cast<RefitDev*>(ws);
        hipError_t e = hipMemcpyAsync(dR, h.data(), sizeof(RefitDev) * cnt, hipMemcpyHostToDevice, st);
        std::vector<int> hf(cnt, 0);
        if (e == hipSuccess) {
            launch_group(in[first], dR, cnt, ks, max_lda, max_s, max_n, st);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(hf.data(), flags, sizeof(int) * cnt, hipMemcpyDeviceToHost, st);
        (void)hipFreeAsync(ws, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(QIHT_ERR_DEVICE, std::string("refit: ") + hipGetErrorString(e));
        for (int i = 0; i < cnt; ++i)
            if (hf[i])
                return fail(QIHT_ERR_NUMERIC, "refit of problem " + std::to_string(first + i) +
                                                  ": the support columns are not linearly independent");
        first = last;
    }
    return QIHT_OK;
}

qiht_status run_refit(const RefitIn& in, hipStream_t st) { return run_refit_batch(&in, 1, st); }

}  // namespace qiht
