// Least-squares refit of x on a fixed support, in FP64: the normal equations
// A_G^T A_G z = A_G^T y solved by a blocked Cholesky factorization.  This is
// an addition to QIHT (the method returns its last iterate); it removes the
// step-size and quantization bias of x on the recovered support.  A is the
// caller's dense Phi, or the dequantized first realization of the codes.
//
// Layout: A_G is rows x s, column-major (column t = column sup[t] of A, lda =
// rows); G = A_G^T A_G is s x s, row-major, lower triangle used (the
// Cholesky factor L overwrites it); b = A_G^T y.
#include <algorithm>

#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kNB = 32;       // Cholesky block
constexpr int kTile = 64;     // Gram / update tile (16 x 16 threads, 4 x 4 each)
constexpr int kKc = 16;       // rows per LDS step of the Gram product

// Column t of A_G from the stored matrix: alpha code + beta (packed codes),
// the float (32), or 2^e_i times the stored value (dense formats).
template <int BITS>
__global__ __launch_bounds__(256) void k_refit_codes(const uint8_t* __restrict__ codes,
                                                     int64_t col_bytes, int64_t rows,
                                                     double alpha, double beta,
                                                     const int32_t* __restrict__ rowexp,
                                                     const int32_t* __restrict__ sup,
                                                     double* __restrict__ A) {
    constexpr int RPW = rows_per_word<BITS>();
    const int t = blockIdx.y;
    const uint8_t* col = codes + static_cast<int64_t>(sup[t]) * col_bytes;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < rows;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const uint32_t w = reinterpret_cast<const uint32_t*>(col)[i / RPW];
        const double e = elem_at<BITS>(w, static_cast<int>(i % RPW));
        double v;
        if constexpr (BITS == 32) v = e;
        else if constexpr (BITS == 9 || BITS == 16) v = ldexp(e, rowexp[i]);
        else v = alpha * e + beta;
        A[static_cast<int64_t>(t) * rows + i] = v;
    }
}

// Column t of A_G from a dense row-major Phi (real, or complex interleaved:
// the stacked real matrix [Re Phi; Im Phi] of 2m rows).
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void k_refit_phi(const T* __restrict__ phi, int64_t m,
                                                   int64_t ld, const int32_t* __restrict__ sup,
                                                   double* __restrict__ A) {
    const int t = blockIdx.y;
    const int64_t j = sup[t];
    const int64_t rows = CPLX ? 2 * m : m;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < rows;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        double v;
        if (CPLX) {
            const int64_t r = i < m ? i : i - m;
            v = static_cast<double>(phi[2 * (r * ld + j) + (i < m ? 0 : 1)]);
        } else {
            v = static_cast<double>(phi[i * ld + j]);
        }
        A[static_cast<int64_t>(t) * rows + i] = v;
    }
}

// Tile (I, J), I >= J, of the partial G_ks = A[rows of split ks]^T A[...]:
// 64 x 64, each thread 4 x 4 entries; blockIdx.y = ks of KS row splits.
__global__ __launch_bounds__(256) void k_refit_gram(const double* __restrict__ A, int64_t rows,
                                                    int s, int64_t split, double* __restrict__ Gp) {
    int I = 0, rem = blockIdx.x;
    while (rem > I) {
        rem -= I + 1;
        ++I;
    }
    const int J = rem;
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * split;
    const int64_t r1 = min(rows, r0 + split);
    double* G = Gp + static_cast<int64_t>(blockIdx.y) * s * s;
    __shared__ double sa[kKc][kTile + 1];
    __shared__ double sb[kKc][kTile + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int64_t k0 = r0; k0 < r1; k0 += kKc) {
        // 16 rows x 64 columns of each operand: thread (r = tid % 16, c4 = tid / 16)
        const int r = threadIdx.x & 15, c4 = threadIdx.x >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = c4 * 4 + q;
            const int64_t kr = k0 + r;
            const int ci = I * kTile + c, cj = J * kTile + c;
            sa[r][c] = (kr < r1 && ci < s) ? A[static_cast<int64_t>(ci) * rows + kr] : 0.0;
            sb[r][c] = (kr < r1 && cj < s) ? A[static_cast<int64_t>(cj) * rows + kr] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kKc; ++k) {
            double va[4], vb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) va[a] = sa[k][ty * 4 + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) vb[b] = sb[k][tx * 4 + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(va[a], vb[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = I * kTile + ty * 4 + a, j = J * kTile + tx * 4 + b;
            if (i < s && j < s) G[static_cast<int64_t>(i) * s + j] = acc[a][b];
        }
}

// G = sum of the KS partials, in split order (lower triangle).
// (The diagonal is also kept aside: the factorization judges its pivots
// against it.)
__global__ __launch_bounds__(256) void k_refit_gram_sum(const double* __restrict__ Gp, int s, int ks,
                                                        double* __restrict__ G, double* __restrict__ diag) {
    const int64_t total = static_cast<int64_t>(s) * s;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * 256) {
        if (e % s > e / s) continue;
        double v = 0.0;
        for (int q = 0; q < ks; ++q) v += Gp[q * total + e];
        G[e] = v;
        if (e % s == e / s) diag[e / s] = v;
    }
}

__global__ void k_fill_i32(int* p, int count, int v) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = v;
}

// b = A^T y, one workgroup per column, fixed summation order.
__global__ __launch_bounds__(256) void k_refit_rhs(const double* __restrict__ A, int64_t rows,
                                                   const double* __restrict__ y,
                                                   double* __restrict__ b) {
    __shared__ double red[4];
    const int t = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) acc = fma(A[static_cast<int64_t>(t) * rows + i], y[i], acc);
    acc = block_sum<256>(acc, red);
    if (threadIdx.x == 0) b[t] = acc;
}

// Cholesky of the nb x nb diagonal block at (k0, k0), in LDS.  A pivot at or
// below kPivotRel times the column's own Gram diagonal means the support
// columns are (numerically) linearly dependent.
constexpr double kPivotRel = 1e-12;

__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ G, int s, int k0,
                                                    const double* __restrict__ diag, int* flag) {
    if (*flag) return;
    __shared__ double L[kNB][kNB + 1];
    const int nb = min(kNB, s - k0);
    for (int e = threadIdx.x; e < nb * nb; e += 256) {
        const int i = e / nb, j = e % nb;
        L[i][j] = G[static_cast<int64_t>(k0 + i) * s + k0 + j];
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        const double d = L[k][k];
        if (!(d > kPivotRel * diag[k0 + k]) || !isfinite(d)) {
            if (threadIdx.x == 0) atomicOr(flag, 1);
            return;  // uniform: every thread read the same d
        }
        const double r = sqrt(d);
        __syncthreads();
        if (threadIdx.x == 0) L[k][k] = r;
        for (int i = k + 1 + threadIdx.x; i < nb; i += 256) L[i][k] /= r;
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
__global__ __launch_bounds__(256) void k_trsm_panel(double* __restrict__ G, int s, int k0, const int* flag) {
    if (*flag) return;
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
__global__ __launch_bounds__(256) void k_syrk_update(double* __restrict__ G, int s, int k0, const int* flag) {
    if (*flag) return;
    const int nb = min(kNB, s - k0);
    const int base = k0 + nb;  // first trailing row / column
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

__global__ __launch_bounds__(1024) void k_refit_solve(const double* __restrict__ G, int s,
                                                      double* __restrict__ b, const int* flag) {
    if (*flag) return;
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

// x_out: zero off the support, x_out[sup[t]] = x_t (FP32); xs_out
// (optional) = x (FP64).  The support is ascending, so one pass over n with
// a binary search would do; two launches keep it simple.
__global__ __launch_bounds__(256) void k_refit_zero(int64_t n, float* __restrict__ x_out, const int* flag) {
    if (*flag) return;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * 256)
        x_out[j] = 0.0f;
}

__global__ __launch_bounds__(256) void k_refit_scatter(const double* __restrict__ xz,
                                                       const int32_t* __restrict__ sup, int s,
                                                       float* __restrict__ x_out,
                                                       double* __restrict__ xs_out, const int* flag) {
    if (*flag) return;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < s; t += gridDim.x * 256) {
        x_out[sup[t]] = static_cast<float>(xz[t]);
        if (xs_out) xs_out[t] = xz[t];
    }
}

}  // namespace

namespace {
constexpr int kSplitK = 8;  // row splits of the Gram product

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

struct RefitWs {
    double *A, *Gp, *G, *b, *diag;
    int* flag;
    size_t bytes;
};

RefitWs refit_layout(uint8_t* base, int64_t rows, int64_t s) {
    RefitWs w{};
    size_t off = 0;
    const size_t ss = static_cast<size_t>(s) * static_cast<size_t>(s) * sizeof(double);
    w.A = reinterpret_cast<double*>(base + off);
    off += up256(static_cast<size_t>(rows) * static_cast<size_t>(s) * sizeof(double));
    w.Gp = reinterpret_cast<double*>(base + off);
    off += up256(kSplitK * ss);
    w.G = reinterpret_cast<double*>(base + off);
    off += up256(ss);
    w.b = reinterpret_cast<double*>(base + off);
    off += up256(static_cast<size_t>(s) * sizeof(double));
    w.diag = reinterpret_cast<double*>(base + off);
    off += up256(static_cast<size_t>(s) * sizeof(double));
    w.flag = reinterpret_cast<int*>(base + off);
    off += 256;
    w.bytes = off;
    return w;
}
}  // namespace

size_t refit_workspace_bytes(int64_t rows, int64_t s) {
    return refit_layout(nullptr, rows, s).bytes;
}

int* refit_flag(uint8_t* ws, int64_t rows, int64_t s) { return refit_layout(ws, rows, s).flag; }

void launch_refit(const RefitIn& in, uint8_t* ws, hipStream_t st) {
    const int64_t rows = in.rows;
    const int s = static_cast<int>(in.s);
    const RefitWs w = refit_layout(ws, rows, s);
    const dim3 gcol(static_cast<unsigned>(std::min<int64_t>((rows + 255) / 256, 64)), s);
    if (in.phi) {
        switch (in.dtype) {
            case QIHT_F64: hipLaunchKernelGGL((k_refit_phi<double, false>), gcol, dim3(256), 0, st, static_cast<const double*>(in.phi), in.m, in.ld, in.sup, w.A); break;
            case QIHT_F32: hipLaunchKernelGGL((k_refit_phi<float, false>), gcol, dim3(256), 0, st, static_cast<const float*>(in.phi), in.m, in.ld, in.sup, w.A); break;
            case QIHT_C128: hipLaunchKernelGGL((k_refit_phi<double, true>), gcol, dim3(256), 0, st, static_cast<const double*>(in.phi), in.m, in.ld, in.sup, w.A); break;
            default: hipLaunchKernelGGL((k_refit_phi<float, true>), gcol, dim3(256), 0, st, static_cast<const float*>(in.phi), in.m, in.ld, in.sup, w.A); break;
        }
    } else {
        switch (in.bits) {
            case 1: hipLaunchKernelGGL((k_refit_codes<1>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
            case 2: hipLaunchKernelGGL((k_refit_codes<2>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
            case 4: hipLaunchKernelGGL((k_refit_codes<4>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
            case 8: hipLaunchKernelGGL((k_refit_codes<8>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
            case 9: hipLaunchKernelGGL((k_refit_codes<9>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
            case 16: hipLaunchKernelGGL((k_refit_codes<16>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
            default: hipLaunchKernelGGL((k_refit_codes<32>), gcol, dim3(256), 0, st, in.codes, in.col_bytes, rows, in.alpha, in.beta, in.rowexp, in.sup, w.A); break;
        }
    }
    const int T = (s + kTile - 1) / kTile;
    const int64_t split = ((rows + kSplitK - 1) / kSplitK + kKc - 1) / kKc * kKc;
    hipLaunchKernelGGL(k_refit_gram, dim3(T * (T + 1) / 2, kSplitK), dim3(256), 0, st, w.A, rows, s, split, w.Gp);
    hipLaunchKernelGGL(k_refit_gram_sum, dim3(static_cast<unsigned>(std::min<int64_t>((static_cast<int64_t>(s) * s + 255) / 256, 4096))), dim3(256), 0, st, w.Gp, s, kSplitK, w.G, w.diag);
    hipLaunchKernelGGL(k_refit_rhs, dim3(s), dim3(256), 0, st, w.A, rows, in.y, w.b);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.flag, 1, 0);
    for (int k0 = 0; k0 < s; k0 += kNB) {
        const int nb = std::min(kNB, s - k0);
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, w.G, s, k0, w.diag, w.flag);
        const int rest = s - k0 - nb;
        if (rest > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 255) / 256), dim3(256), 0, st, w.G, s, k0, w.flag);
            const int Tr = (rest + kTile - 1) / kTile;
            hipLaunchKernelGGL(k_syrk_update, dim3(Tr * (Tr + 1) / 2), dim3(256), 0, st, w.G, s, k0, w.flag);
        }
    }
    hipLaunchKernelGGL(k_refit_solve, dim3(1), dim3(1024), 0, st, w.G, s, w.b, w.flag);
    hipLaunchKernelGGL(k_refit_zero, dim3(static_cast<unsigned>(std::min<int64_t>((in.n + 255) / 256, 1024))), dim3(256), 0, st, in.n, in.x_out, w.flag);
    hipLaunchKernelGGL(k_refit_scatter, dim3((s + 255) / 256), dim3(256), 0, st, w.b, in.sup, s, in.x_out, in.xs_out, w.flag);
}

}  // namespace qiht
