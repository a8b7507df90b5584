// QIHT with a complex unknown (Sec. I-A: Phi in C^{M x N}, x in C^N).
//
// With Q = Q_re + i Q_im (the codes of the stacked real matrix [Re; Im]) and
// x = x_re + i x_im, the complex residual, gradient and norms are those of the
// real problem with matrix
//     A = [ Q_re  -Q_im ]      unknown z = [ x_re ]
//         [ Q_im   Q_re ]                  [ x_im ]
// (2M x 2N): Q x = A z in stacked form, Q^H r = A^T [Re r; Im r], and every
// inner product the step size and the step-size test take is the real part of
// the complex one.  So the solve is the real solve on A, with H_s ranking the
// N entries by modulus |x_j|^2 = z_j^2 + z_{j+N}^2 and keeping both columns of
// each selected entry (ProbDev::group).  A's codes are built once per handle
// from Q's: columns [0, N) are Q's stacked columns, column N + j holds -Q_im
// (the codes of rows [M, 2M) of column j mirrored, k -> L - 1 - k, since the
// levels are symmetric about 0) over Q_re.
#include <cmath>
#include <cstring>

#include "solve_common.h"

namespace qiht {
namespace {

template <int BITS>
__global__ __launch_bounds__(256) void k_embed(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                               int64_t col_bytes, int64_t m, int64_t n, uint32_t lmax) {
    constexpr int RPW = BITS == 32 ? 1 : 32 / BITS;  // rows per 32-bit word
    const int64_t words = col_bytes / 4;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * words) return;
    const int64_t j = t / words, w = t % words;
    const uint8_t* sc = src + j * col_bytes;
    uint32_t out = 0u;
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int64_t i = w * RPW + q;  // row of the new column
        if (i >= 2 * m) break;          // padding rows stay 0
        const bool top = i < m;         // -Im part
        const int64_t si = top ? i + m : i - m;
        if constexpr (BITS == 32) {
            const uint32_t v = reinterpret_cast<const uint32_t*>(sc)[si];
            out = top ? (v ^ 0x80000000u) : v;
        } else {
            const uint32_t code = (sc[si * BITS / 8] >> ((si * BITS) % 8)) & ((1u << BITS) - 1u);
            out |= (top ? lmax - code : code) << (q * BITS);
        }
    }
    reinterpret_cast<uint32_t*>(dst + (n + j) * col_bytes)[w] = out;
}

// The handle of A for a complex-input handle q (built on first use, kept
// with q and freed with it).
qiht_status embedding(qiht_qmatrix* q, hipStream_t st, qiht_qmatrix** out) {
    if (q->embedded) {
        *out = q->embedded;
        return QIHT_OK;
    }
    qiht_qmatrix* e = new qiht_qmatrix(*q);
    e->embedded = nullptr;
    e->pooled = false;  // (its codes come from hipMalloc below)
    e->n = 2 * q->n;
    const size_t bytes = static_cast<size_t>(e->col_bytes) * static_cast<size_t>(e->n);
    uint8_t* mem = nullptr;
    if (dev_malloc(reinterpret_cast<void**>(&mem), bytes * q->realizations) != hipSuccess) {
        (void)hipGetLastError();
        delete e;
        return fail(QIHT_ERR_OUT_OF_MEMORY, "no memory for the complex embedding");
    }
    e->codes[0] = mem;
    e->codes[1] = q->realizations == 2 ? mem + bytes : mem;
    // the level index mirrored by negation: value(k) = alpha k + beta with
    // beta = -c, so -value(k) = value(L - 1 - k), L - 1 = -2 beta / alpha
    const uint32_t lmax = q->alpha > 0.0 ? static_cast<uint32_t>(std::llround(-2.0 * q->beta / q->alpha)) : 0u;
    const int64_t words = q->col_bytes / 4;
    const int64_t threads = q->n * words;
    const dim3 grid(static_cast<unsigned>((threads + 255) / 256));
    for (int r = 0; r < q->realizations; ++r) {
        hipError_t er = hipMemcpyAsync(e->codes[r], q->codes[r], static_cast<size_t>(q->col_bytes) * q->n,
                                       hipMemcpyDeviceToDevice, st);
        if (er == hipSuccess) {
            switch (q->bits) {
                case 1: hipLaunchKernelGGL(k_embed<1>, grid, dim3(256), 0, st, q->codes[r], e->codes[r], q->col_bytes, q->m, q->n, lmax); break;
                case 2: hipLaunchKernelGGL(k_embed<2>, grid, dim3(256), 0, st, q->codes[r], e->codes[r], q->col_bytes, q->m, q->n, lmax); break;
                case 4: hipLaunchKernelGGL(k_embed<4>, grid, dim3(256), 0, st, q->codes[r], e->codes[r], q->col_bytes, q->m, q->n, lmax); break;
                case 8: hipLaunchKernelGGL(k_embed<8>, grid, dim3(256), 0, st, q->codes[r], e->codes[r], q->col_bytes, q->m, q->n, lmax); break;
                default: hipLaunchKernelGGL(k_embed<32>, grid, dim3(256), 0, st, q->codes[r], e->codes[r], q->col_bytes, q->m, q->n, lmax); break;
            }
            er = hipGetLastError();
        }
        if (er != hipSuccess) {
            (void)hipFree(mem);
            delete e;
            return hip_fail(er, "complex embedding");
        }
    }
    q->embedded = e;
    *out = e;
    return QIHT_OK;
}

}  // namespace

qiht_status run_solve_complex(qiht_qmatrix* q, const double* yhat, int64_t s, const SolveArgs& a, int refit,
                              float* x_out, int32_t* support_out, qiht_info* info, hipStream_t st) {
    qiht_qmatrix* e = nullptr;
    qiht_status s0 = embedding(q, st, &e);
    if (s0 != QIHT_OK) return s0;
    int32_t* sup2 = nullptr;
    QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&sup2), sizeof(int32_t) * 2 * s, st));
    ProblemIn in{e, yhat, 2 * s, x_out, sup2, nullptr, nullptr};
    in.group = q->n;
    qiht_info tmp;
    s0 = run_solve(&in, 1, a, &tmp, st);
    if (s0 == QIHT_OK && refit) {
        RefitIn r{};
        r.codes = e->codes[0];
        r.col_bytes = e->col_bytes;
        r.bits = e->bits;
        r.alpha = e->alpha;
        r.beta = e->beta;
        r.rowexp = e->rexp;
        r.rows = e->rows;
        r.n = e->n;
        r.s = 2 * s;
        r.y = yhat;
        r.sup = sup2;
        r.x_out = x_out;
        s0 = run_refit(r, st);
    }
    // the support of z holds each selected entry j twice (j and j + N, in
    // that order after the sort): its first s indices are the entries
    if (s0 == QIHT_OK) {
        const hipError_t er = hipMemcpyAsync(support_out, sup2, sizeof(int32_t) * s, hipMemcpyDeviceToDevice, st);
        if (er != hipSuccess) s0 = hip_fail(er, "copy the support");
    }
    (void)hipFreeAsync(sup2, st);
    if (s0 == QIHT_OK) {
        QIHT_HIP(hipStreamSynchronize(st));
        if (info) *info = tmp;
    }
    return s0;
}

}  // namespace qiht
