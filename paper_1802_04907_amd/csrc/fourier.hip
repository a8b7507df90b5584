// Gradient g = [Re Phi; Im Phi]^T r of a Fourier-sampled measurement matrix
// evaluated on the fly, with no matrix in memory (Sec. IV-C, on the radio
// interferometry model of Sec. IV-B):
//   Phi_jk = exp(-2 pi i (u_j l_k + v_j m_k)),
//   l_k = (k mod side) - side/2, m_k = (k div side) - side/2,
//   g_k = sum_j cos(2 pi th_jk) r_j - sin(2 pi th_jk) r_{n_vis + j}.
// The work is arithmetic, not memory: each entry costs a handful of FP32
// operations and nothing is read per entry but the visibility block in LDS.
//
// Layout of the work: a thread owns a run of kFtRun consecutive pixels of
// one image row.  For a visibility j and the run's first pixel, the FP64
// phase is reduced to [-1/2, 1/2] turns and one accurate sincospi gives
// E = exp(-2 pi i th); the residual is folded in once, z = E (r_j - i r_{n+j}),
// so that the pixel's term is Re z.  Along the run the entries differ by the
// constant factor w = exp(-2 pi i u_j): each further pixel costs one complex
// rotation z <- z w and one add.  A workgroup takes kFtThreads runs against
// one block of kFtVis visibilities staged in LDS and writes FP32 partial
// sums; a second kernel adds the blocks' partials in FP64 in a fixed order
// (deterministic).
#include <cmath>

#include "qiht_internal.h"

namespace qiht {
namespace {

constexpr int kFtThreads = 256;
constexpr int kFtRun = 16;   // pixels per thread, consecutive along l
constexpr int kFtVis = 128;  // visibilities per workgroup

__global__ __launch_bounds__(kFtThreads) void k_fourier_partial(const double* __restrict__ uv, int64_t nvis,
                                                                 int side, const float* __restrict__ r,
                                                                 float* __restrict__ part) {
    __shared__ double2 suv[kFtVis];  // (u, v)
    __shared__ float4 srw[kFtVis];   // (r_re, r_im, cos 2 pi u, sin 2 pi u)
    const int64_t j0 = static_cast<int64_t>(blockIdx.y) * kFtVis;
    const int nj = static_cast<int>(min(static_cast<int64_t>(kFtVis), nvis - j0));
    for (int t = threadIdx.x; t < nj; t += kFtThreads) {
        const double u = uv[2 * (j0 + t)], v = uv[2 * (j0 + t) + 1];
        float s, c;
        sincospif(2.0f * static_cast<float>(u - rint(u)), &s, &c);
        suv[t] = make_double2(u, v);
        srw[t] = make_float4(r[j0 + t], r[nvis + j0 + t], c, s);
    }
    __syncthreads();
    const int runs_per_row = (side + kFtRun - 1) / kFtRun;
    const int run = static_cast<int>(blockIdx.x) * kFtThreads + static_cast<int>(threadIdx.x);
    if (run >= runs_per_row * side) return;  // no barrier follows
    const int row = run / runs_per_row;
    const int c0 = (run - row * runs_per_row) * kFtRun;  // first pixel column of the run
    const double l0 = static_cast<double>(c0 - side / 2);
    const double m = static_cast<double>(row - side / 2);
    float acc[kFtRun];
#pragma unroll
    for (int q = 0; q < kFtRun; ++q) acc[q] = 0.0f;
    for (int t = 0; t < nj; ++t) {
        const double2 w2 = suv[t];
        const float4 rw = srw[t];
        const double th = fma(w2.x, l0, w2.y * m);
        float s, c;
        sincospif(2.0f * static_cast<float>(th - rint(th)), &s, &c);
        // z = (c - i s)(r_re - i r_im)
        float zr = fmaf(c, rw.x, -(s * rw.y));
        float zi = -fmaf(c, rw.y, s * rw.x);
#pragma unroll
        for (int q = 0; q < kFtRun; ++q) {
            acc[q] += zr;
            // next pixel: z (cos 2 pi u - i sin 2 pi u)
            const float nr = fmaf(zr, rw.z, zi * rw.w);
            const float ni = fmaf(zi, rw.z, -(zr * rw.w));
            zr = nr;
            zi = ni;
        }
    }
    float* out = part + static_cast<size_t>(blockIdx.y) * static_cast<size_t>(side) * side +
                 static_cast<size_t>(row) * side + c0;
#pragma unroll
    for (int q = 0; q < kFtRun; ++q)
        if (c0 + q < side) out[q] = acc[q];
}

// g_k = sum over the visibility blocks of the partials, in FP64: the blocks
// are cut into kRedSeg contiguous segments, each summed in block order by
// one thread, and the segments are added in order (a fixed tree).
constexpr int kRedPix = 32;  // pixels per workgroup
constexpr int kRedSeg = 8;   // block segments per pixel

__global__ __launch_bounds__(kRedPix * kRedSeg) void k_fourier_reduce(const float* __restrict__ part, int nblk,
                                                                      int64_t npix, float* __restrict__ g) {
    __shared__ double sh[kRedSeg][kRedPix];
    const int p = threadIdx.x % kRedPix, seg = threadIdx.x / kRedPix;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kRedPix + p;
    const int per = (nblk + kRedSeg - 1) / kRedSeg;
    const int b0 = seg * per, b1 = min(nblk, b0 + per);
    double s = 0.0;
    if (k < npix) {
        const float* src = part + k;
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = src[static_cast<size_t>(b + i) * npix];
#pragma unroll
            for (int i = 0; i < 8; ++i) s += static_cast<double>(v[i]);
        }
        for (; b < b1; ++b) s += static_cast<double>(src[static_cast<size_t>(b) * npix]);
    }
    sh[seg][p] = s;
    __syncthreads();
    if (seg == 0 && k < npix) {
        double t = sh[0][p];
#pragma unroll
        for (int i = 1; i < kRedSeg; ++i) t += sh[i][p];
        g[k] = static_cast<float>(t);
    }
}

}  // namespace

int64_t fourier_partial_blocks(int64_t nvis) { return (nvis + kFtVis - 1) / kFtVis; }

qiht_status run_fourier_gradient(const double* uv, int64_t nvis, int side, const float* r, float* g,
                                 hipStream_t st) {
    const int64_t npix = static_cast<int64_t>(side) * side;
    const int64_t nblk = fourier_partial_blocks(nvis);
    const int64_t runs = static_cast<int64_t>((side + kFtRun - 1) / kFtRun) * side;
    float* part = nullptr;
    QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&part), sizeof(float) * static_cast<size_t>(nblk * npix), st));
    hipLaunchKernelGGL(k_fourier_partial,
                       dim3(static_cast<unsigned>((runs + kFtThreads - 1) / kFtThreads), static_cast<unsigned>(nblk)),
                       dim3(kFtThreads), 0, st, uv, nvis, side, r, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fourier_reduce, dim3(static_cast<unsigned>((npix + kRedPix - 1) / kRedPix)),
                           dim3(kRedPix * kRedSeg), 0, st, part, static_cast<int>(nblk), npix, g);
        e = hipGetLastError();
    }
    (void)hipFreeAsync(part, st);
    if (e != hipSuccess) return hip_fail(e, "fourier gradient launch");
    return QIHT_OK;
}

}  // namespace qiht
