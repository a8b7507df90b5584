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
#include "solve_common.h"

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

// ---------------------------------------------------------------------------
// Normalized IHT (Algorithm 1: the b = 32 case of QIHT) with every product by
// Phi computed on the fly.  Besides the full pass above, the iteration needs
// Phi times short column lists (the support, or the support's changes):
// one thread per visibility sums over the list in FP64, the entries evaluated
// as in the pass (FP64 phase reduced to turns, FP32 sincospi).
// ---------------------------------------------------------------------------

// Pixel k's row k div side by a float reciprocal (k < 2^24 is exact in
// FP32; the rounded quotient is off by at most one, corrected).
__device__ __forceinline__ void fourier_entry(double u, double v, int k, int side, float inv_side, float& c,
                                              float& s) {
    int row = static_cast<int>(static_cast<float>(k) * inv_side);
    int col = k - row * side;
    if (col < 0) {
        --row;
        col += side;
    } else if (col >= side) {
        ++row;
        col -= side;
    }
    const double lk = static_cast<double>(col - side / 2);
    const double mk = static_cast<double>(row - side / 2);
    const double th = fma(u, lk, v * mk);
    sincospif(2.0f * static_cast<float>(th - rint(th)), &s, &c);
}

// p = Phi_L v over the list (cols[t], vals[t]), t < count (entries with
// cols[t] < 0 are skipped), stacked [Re; Im] in FP64; with y != nullptr
// r = y - p is written in FP32 instead.  kColLanes lanes share a visibility:
// lane i takes the entries t = i mod kColLanes, and the lanes' sums meet in
// a fixed xor butterfly (every lane ends with the same bits).
constexpr int kColLanes = 8;

__global__ __launch_bounds__(256) void k_fourier_cols(const double* __restrict__ uv, int64_t nvis, int side,
                                                      const int32_t* __restrict__ cols,
                                                      const double* __restrict__ vals, int count,
                                                      const double* __restrict__ y, float* __restrict__ r,
                                                      double* __restrict__ p) {
    const int64_t j = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / kColLanes;
    const int lane = static_cast<int>(threadIdx.x) % kColLanes;
    const bool live = j < nvis;  // no early exit: the whole group takes part in the shuffles
    const double u = live ? uv[2 * j] : 0.0, v = live ? uv[2 * j + 1] : 0.0;
    const float inv_side = 1.0f / static_cast<float>(side);
    double are = 0.0, aim = 0.0;
    for (int t = lane; live && t < count; t += kColLanes) {
        const int k = cols[t];
        if (k < 0) continue;
        float c, sn;
        fourier_entry(u, v, k, side, inv_side, c, sn);
        const double x = vals[t];
        are = fma(static_cast<double>(c), x, are);
        aim = fma(-static_cast<double>(sn), x, aim);
    }
#pragma unroll
    for (int d = 1; d < kColLanes; d <<= 1) {
        are += __shfl_xor(are, d, kColLanes);
        aim += __shfl_xor(aim, d, kColLanes);
    }
    if (!live || lane != 0) return;
    if (y) {
        r[j] = static_cast<float>(y[j] - are);
        r[nvis + j] = static_cast<float>(y[nvis + j] - aim);
    } else {
        p[j] = are;
        p[nvis + j] = aim;
    }
}

// Scalars of the solver, on the device.
struct FtState {
    double num;    // |g_G|^2
    double den;    // |Phi_G g_G|^2
    double mu;     // current step
    double mu0;
    double dx2;    // |x+ - x|^2
    double x2;     // |x+|^2
    double w2;     // |Phi (x+ - x)|^2
    int changed;   // proposal support differs from the current one
    int status;    // FT_*
    int nb;        // shrinks in this iteration
    int capped;
    int stop;      // accepted and |x+ - x| <= tol |x+|
    double part[64];  // per-workgroup sums of squares (k_ft_sumsq)
    int hs_err;       // set by H_s on a NaN key
};
enum { FT_GO = 0, FT_STATIONARY = 1, FT_RETRY = 2, FT_ACCEPT = 3 };

constexpr int kCtl = 1024;

__device__ double block_sum_f64(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kCtl / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double t = sh[0];
    __syncthreads();
    return t;
}

// |p|^2 over len doubles: workgroup b of 64 sums the b-th contiguous part
// into st->part[b]; the consumer adds the 64 parts in order.
constexpr int kSqBlocks = 64;

__global__ __launch_bounds__(256) void k_ft_sumsq(const double* __restrict__ p, int64_t len, FtState* st) {
    __shared__ double sh[256];
    const int64_t per = (len + kSqBlocks - 1) / kSqBlocks;
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * per, i1 = min(len, i0 + per);
    double a = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) a = fma(p[i], p[i], a);
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) st->part[blockIdx.x] = sh[0];
}

__device__ __forceinline__ double sumsq_total(const FtState* st) {
    double t = 0.0;
    for (int b = 0; b < kSqBlocks; ++b) t += st->part[b];
    return t;
}

// g_G into the value list, |g_G|^2 into st->num (one workgroup).
__global__ __launch_bounds__(kCtl) void k_ft_gsup(const float* __restrict__ g, const int32_t* __restrict__ sup, int s,
                                                   double* __restrict__ vals, FtState* st) {
    __shared__ double sh[kCtl];
    double a = 0.0;
    for (int t = threadIdx.x; t < s; t += kCtl) {
        const float v = g[sup[t]];
        vals[t] = static_cast<double>(v);
        a = fma(static_cast<double>(v), static_cast<double>(v), a);
    }
    const double num = block_sum_f64(a, sh);
    if (threadIdx.x == 0) {
        st->num = num;
        st->nb = 0;
        st->capped = 0;
    }
}

// mu = |g_G|^2 / |Phi_G g_G|^2, or stationary when either is 0.
__global__ void k_ft_mu(FtState* st) {
    if (threadIdx.x != 0) return;
    st->den = sumsq_total(st);
    const double num = st->num, den = st->den;
    if (num == 0.0 || !(den > 0.0) || !isfinite(den)) {
        st->status = FT_STATIONARY;
        return;
    }
    st->mu = num / den;
    st->mu0 = st->mu;
    st->status = FT_GO;
}

// a = x + mu g (FP32, mu rounded once).  After a stationary step the
// proposal kernels do nothing and the decision keeps the status.
__global__ __launch_bounds__(256) void k_ft_axpy(const float* __restrict__ x, const float* __restrict__ g,
                                                  const FtState* st, int64_t n, float* __restrict__ a) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n || st->status == FT_STATIONARY) return;
    a[i] = fmaf(static_cast<float>(st->mu), g[i], x[i]);
}

// The change x+ - x as a column list: the new support with a - x, then the
// old support's indices outside the new one with -x (others skipped), each
// difference of the FP32 values taken exactly in FP64 (as the packed-code
// path's proposal lists hold them); |x+ - x|^2, |x+|^2 and whether the
// support changed (one workgroup).
__global__ __launch_bounds__(kCtl) void k_ft_delta(const float* __restrict__ x, const float* __restrict__ a,
                                                    const int32_t* __restrict__ sup, const int32_t* __restrict__ sup_new,
                                                    int s, int32_t* __restrict__ cols, double* __restrict__ vals,
                                                    FtState* st) {
    __shared__ double sh[kCtl];
    __shared__ int s_changed;
    if (st->status == FT_STATIONARY) return;  // uniform: one value for the workgroup
    if (threadIdx.x == 0) s_changed = 0;
    __syncthreads();
    double d2 = 0.0, x2 = 0.0;
    for (int t = threadIdx.x; t < s; t += kCtl) {
        const int k = sup_new[t];
        const float xn = a[k];
        const double d = static_cast<double>(xn) - static_cast<double>(x[k]);
        cols[t] = k;
        vals[t] = d;
        d2 = fma(d, d, d2);
        x2 = fma(static_cast<double>(xn), static_cast<double>(xn), x2);
        if (sup[t] != k) s_changed = 1;
        // the old index: kept if absent from the new (ascending) support
        const int ko = sup[t];
        int lo = 0, hi = s;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sup_new[mid] < ko) lo = mid + 1;
            else hi = mid;
        }
        const bool in_new = lo < s && sup_new[lo] == ko;
        cols[s + t] = in_new ? -1 : ko;
        const double dold = in_new ? 0.0 : -static_cast<double>(x[ko]);
        vals[s + t] = dold;
        d2 = fma(dold, dold, d2);
    }
    const double sd2 = block_sum_f64(d2, sh);
    const double sx2 = block_sum_f64(x2, sh);
    if (threadIdx.x == 0) {
        st->dx2 = sd2;
        st->x2 = sx2;
        st->changed = s_changed;
    }
}

// The step test of a changed support: mu <= (1 - c) omega, omega =
// |dx|^2 / |Phi dx|^2 (+inf when |Phi dx| = 0); else shrink and retry, at
// most max_bt times (then the last proposal is accepted, capped).
// On acceptance, the stop test |x+ - x| <= tol |x+|.
__global__ void k_ft_decide(FtState* st, double k, double c, int max_bt, double tol) {
    if (threadIdx.x != 0 || st->status == FT_STATIONARY) return;
    st->status = FT_ACCEPT;
    st->w2 = sumsq_total(st);
    if (st->changed) {
        const double w = st->w2 == 0.0 ? INFINITY : st->dx2 / st->w2;
        if (st->mu > (1.0 - c) * w) {
            if (st->nb >= max_bt) {
                st->capped = 1;
            } else {
                st->mu = st->mu / (k * (1.0 - c));
                st->nb += 1;
                st->status = FT_RETRY;
            }
        }
    }
    st->stop = st->status == FT_ACCEPT && sqrt(st->dx2) <= tol * sqrt(st->x2);
}

// x <- x+ (the old support zeroed, the new one written), support <- new.
__global__ __launch_bounds__(256) void k_ft_accept(float* __restrict__ x, const float* __restrict__ a,
                                                    int32_t* __restrict__ sup, const int32_t* __restrict__ sup_new,
                                                    int s) {
    for (int t = threadIdx.x; t < s; t += 256) x[sup[t]] = 0.0f;
    __syncthreads();
    for (int t = threadIdx.x; t < s; t += 256) {
        const int k = sup_new[t];
        x[k] = a[k];
        sup[t] = k;
    }
}

static_assert(QIHT_FOURIER_SOLVE_MAX_PIXELS == kMaxSelectN, "the solve's pixel limit is the selection's");

}  // namespace

qiht_status run_fourier_solve(const double* uv, int64_t nvis, int side, const double* y, int64_t s,
                              const qiht_params& prm, float* x, int32_t* sup, qiht_info* info, hipStream_t st) {
    const int64_t n = static_cast<int64_t>(side) * side;
    const int64_t rows = 2 * nvis;
    const int si = static_cast<int>(s);
    // one workspace: r, g, a (floats), p (doubles), the lists, the new
    // support, the scalars
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = (off + 255) / 256 * 256;
        off = o + bytes;
        return o;
    };
    const size_t o_r = take(sizeof(float) * rows), o_g = take(sizeof(float) * n), o_a = take(sizeof(float) * n);
    const size_t o_p = take(sizeof(double) * rows), o_cols = take(sizeof(int32_t) * 2 * s);
    const size_t o_vals = take(sizeof(double) * 2 * s), o_sn = take(sizeof(int32_t) * s);
    const size_t o_st = take(sizeof(FtState));
    uint8_t* ws = nullptr;
    QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&ws), off, st));
    float* r = reinterpret_cast<float*>(ws + o_r);
    float* g = reinterpret_cast<float*>(ws + o_g);
    float* a = reinterpret_cast<float*>(ws + o_a);
    double* p = reinterpret_cast<double*>(ws + o_p);
    int32_t* cols = reinterpret_cast<int32_t*>(ws + o_cols);
    double* vals = reinterpret_cast<double*>(ws + o_vals);
    int32_t* sn = reinterpret_cast<int32_t*>(ws + o_sn);
    FtState* dst = reinterpret_cast<FtState*>(ws + o_st);
    qiht_status ret = QIHT_OK;
    qiht_info out{};
    auto body = [&]() -> qiht_status {
        const unsigned gv = static_cast<unsigned>((nvis * kColLanes + 255) / 256), gn = static_cast<unsigned>((n + 255) / 256);
        QIHT_HIP(hipMemsetAsync(x, 0, sizeof(float) * n, st));
        QIHT_HIP(hipMemsetAsync(dst, 0, sizeof(FtState), st));
        QIHT_HIP(hipMemsetAsync(a, 0, sizeof(float) * n, st));  // H_s may read it after a stationary step
        // G0 = supp H_s(Phi^T y): r = y (an empty list), then the pass
        hipLaunchKernelGGL(k_fourier_cols, dim3(gv), dim3(256), 0, st, uv, nvis, side, cols, vals, 0, y, r,
                           static_cast<double*>(nullptr));
        QIHT_HIP(hipGetLastError());
        qiht_status s0 = run_fourier_gradient(uv, nvis, side, r, g, st);
        if (s0 != QIHT_OK) return s0;
        launch_hard_threshold(g, static_cast<int>(n), si, sup, &dst->hs_err, st);
        QIHT_HIP(hipGetLastError());
        out.reason = QIHT_REASON_MAX_ITERS;
        FtState hs{};
        for (int it = 1; it <= prm.max_iters; ++it) {
            // r = y - Phi_G x_G, g = Phi^T r
            hipLaunchKernelGGL(k_ft_gsup, dim3(1), dim3(kCtl), 0, st, x, sup, si, vals, dst);
            hipLaunchKernelGGL(k_fourier_cols, dim3(gv), dim3(256), 0, st, uv, nvis, side, sup, vals, si, y, r,
                               static_cast<double*>(nullptr));
            QIHT_HIP(hipGetLastError());
            s0 = run_fourier_gradient(uv, nvis, side, r, g, st);
            if (s0 != QIHT_OK) return s0;
            // mu = |g_G|^2 / |Phi_G g_G|^2
            hipLaunchKernelGGL(k_ft_gsup, dim3(1), dim3(kCtl), 0, st, g, sup, si, vals, dst);
            hipLaunchKernelGGL(k_fourier_cols, dim3(gv), dim3(256), 0, st, uv, nvis, side, sup, vals, si,
                               static_cast<const double*>(nullptr), static_cast<float*>(nullptr), p);
            hipLaunchKernelGGL(k_ft_sumsq, dim3(kSqBlocks), dim3(256), 0, st, p, rows, dst);
            hipLaunchKernelGGL(k_ft_mu, dim3(1), dim3(64), 0, st, dst);
            QIHT_HIP(hipGetLastError());
            for (;;) {
                hipLaunchKernelGGL(k_ft_axpy, dim3(gn), dim3(256), 0, st, x, g, dst, n, a);
                QIHT_HIP(hipGetLastError());
                launch_hard_threshold(a, static_cast<int>(n), si, sn, &dst->hs_err, st);
                hipLaunchKernelGGL(k_ft_delta, dim3(1), dim3(kCtl), 0, st, x, a, sup, sn, si, cols, vals, dst);
                hipLaunchKernelGGL(k_fourier_cols, dim3(gv), dim3(256), 0, st, uv, nvis, side, cols, vals, 2 * si,
                                   static_cast<const double*>(nullptr), static_cast<float*>(nullptr), p);
                hipLaunchKernelGGL(k_ft_sumsq, dim3(kSqBlocks), dim3(256), 0, st, p, rows, dst);
                hipLaunchKernelGGL(k_ft_decide, dim3(1), dim3(64), 0, st, dst, prm.k, prm.c, prm.max_backtracks,
                                   prm.tol);
                QIHT_HIP(hipGetLastError());
                QIHT_HIP(hipMemcpyAsync(&hs, dst, sizeof(FtState), hipMemcpyDeviceToHost, st));
                QIHT_HIP(hipStreamSynchronize(st));
                if (hs.hs_err) return fail(QIHT_ERR_NUMERIC, "NaN met in the iterate");
                if (hs.status != FT_RETRY) break;
            }
            if (hs.status == FT_STATIONARY) {
                out.reason = QIHT_REASON_STATIONARY;
                break;
            }
            hipLaunchKernelGGL(k_ft_accept, dim3(1), dim3(256), 0, st, x, a, sup, sn, si);
            QIHT_HIP(hipGetLastError());
            out.iterations = it;
            out.backtracks += hs.nb;
            out.capped_iterations += hs.capped;
            out.mu_last = hs.mu;
            if (hs.stop) {
                out.reason = QIHT_REASON_CONVERGED;
                break;
            }
        }
        QIHT_HIP(hipStreamSynchronize(st));
        return QIHT_OK;
    };
    ret = body();
    (void)hipFreeAsync(ws, st);
    if (ret == QIHT_OK && info) *info = out;
    return ret;
}

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
