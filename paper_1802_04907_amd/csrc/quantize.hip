// Stochastic quantization of the measurement matrix and the observation
// vector (Sec. III-A): max-abs scaling, then unbiased randomized rounding to
// one of 2^b equispaced levels in [-1, 1], driven by Philox4x32-10 so that
// every element's coin is a pure function of (seed, stream, realization,
// element index).
//
// This file is compiled with -ffp-contract=off: the FP64 position
// p = (v + c) * K, its floor and its fractional part must be the exact
// IEEE results of those three operations, so the codes are reproducible
// bit for bit by any other IEEE implementation of the same rule.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "philox_dev.h"
#include "qiht_internal.h"

namespace qiht {
namespace {

constexpr double kTwo32 = 4294967296.0;

// One stochastic rounding decision.  top = L - 2 for L levels; c the scale;
// K = (L-1)/(2c) (0 when c == 0, which sends every value to code 0).
__device__ __forceinline__ uint32_t quantize_one(double v, double c, double K,
                                                 double top, uint32_t u) {
#pragma clang fp contract(off)
    const double t = v + c;
    const double p = t * K;
    double fi = floor(p);
    fi = fmin(fmax(fi, 0.0), top);
    const double f = p - fi;
    const uint32_t up = (static_cast<double>(u) < f * kTwo32) ? 1u : 0u;
    return static_cast<uint32_t>(fi) + up;
}

// quantize_one in two parts, for a value shared by several realizations:
// its floor position fi and threshold f 2^32 (the same operations in the same
// order), then the coin of one realization.
__device__ __forceinline__ void position_of(double v, double c, double K, double top,
                                            double& fi_out, double& th_out) {
#pragma clang fp contract(off)
    const double t = v + c;
    const double p = t * K;
    double fi = floor(p);
    fi = fmin(fmax(fi, 0.0), top);
    const double f = p - fi;
    fi_out = fi;
    th_out = f * kTwo32;
}
__device__ __forceinline__ uint32_t round_at(double fi, double th, uint32_t u) {
    return static_cast<uint32_t>(fi) + ((static_cast<double>(u) < th) ? 1u : 0u);
}

// Element (i, j) of the stacked real view of a row-major matrix.
template <typename T, int NC>
__device__ __forceinline__ double load_stacked(const T* src, int64_t m,
                                               int64_t ld, int64_t i,
                                               int64_t j) {
    if constexpr (NC == 1) {
        return static_cast<double>(src[i * ld + j]);
    } else {
        const int64_t ii = i < m ? i : i - m;
        const int part = i < m ? 0 : 1;
        return static_cast<double>(src[(ii * ld + j) * 2 + part]);
    }
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_absmax(const T* __restrict__ src,
                                                int64_t m, int64_t n,
                                                int64_t ld,
                                                unsigned long long* out,
                                                int* bad) {
    // Rows blockIdx.y, +gridDim.y, ...; within a row, four independent
    // loads per thread per step.  One atomic per workgroup.
    double mx = 0.0;
    int nonfinite = 0;
    const int64_t row_len = n * NC;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
        const T* row = src + i * ld * NC;
        for (int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
             t0 < row_len; t0 += 4 * step) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t t = t0 + u * step;
                v[u] = t < row_len ? static_cast<double>(row[t]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (!isfinite(v[u])) nonfinite = 1;
                mx = fmax(mx, fabs(v[u]));
            }
        }
    }
    __shared__ double sh[256];
    __shared__ int shbad;
    if (threadIdx.x == 0) shbad = 0;
    __syncthreads();
    if (nonfinite) shbad = 1;
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // Non-negative doubles order like their bit patterns.
        atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(sh[0])));
        if (shbad) atomicOr(bad, 1);
    }
}

// FP32 rows whose length and stride are multiples of 4: 16-byte loads, four
// in flight per thread (the max of |float| values is exact in FP32).
__global__ __launch_bounds__(256) void k_absmax_f4(const float4* __restrict__ src, int64_t m,
                                                   int64_t row4, int64_t ld4,
                                                   unsigned long long* out, int* bad) {
    float mx = 0.0f;
    int nonfinite = 0;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
        const float4* row = src + i * ld4;
        for (int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t0 < row4;
             t0 += 4 * step) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t t = t0 + u * step;
                v[u] = t < row4 ? row[t] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float a[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!isfinite(a[k])) nonfinite = 1;
                    mx = fmaxf(mx, fabsf(a[k]));
                }
            }
        }
    }
    __shared__ float sh[256];
    __shared__ int shbad;
    if (threadIdx.x == 0) shbad = 0;
    __syncthreads();
    if (nonfinite) shbad = 1;
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(static_cast<double>(sh[0]))));
        if (shbad) atomicOr(bad, 1);
    }
}

// One thread = one column j and one 16-byte chunk of that column (the codes
// of RPC consecutive rows), for every realization.  Lanes of a wave take 64
// consecutive columns, so the row-major source is read in coalesced rows.
template <int BITS, typename T, int NC, bool ALIGNED>
__global__ __launch_bounds__(256) void k_quantize(
    const T* __restrict__ src, int64_t m, int64_t n, int64_t ld, int64_t rows,
    int64_t col_bytes, int64_t nchunks, double c, double K, int L, uint32_t k0,
    uint32_t k1, int R, uint8_t* __restrict__ out0,
    uint8_t* __restrict__ out1, const int32_t* __restrict__ rbase,
    const int32_t* __restrict__ stop) {
    constexpr int RPC = (BITS == 32) ? 4 : 128 / BITS;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // blockIdx.x runs over chunk groups: neighbouring workgroups fill the
    // neighbouring 64 bytes of the same 64 columns, so a cache line of codes
    // is completed while it is still in L2
    const int64_t j = static_cast<int64_t>(blockIdx.y) * 64 + lane;
    const int64_t chunk = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    if (j >= n || chunk >= nchunks) return;
    // realizations drawn per iteration: copies 2 it and 2 it + 1 for the
    // iteration it + 1 that *rbase = it completed ones precede (else 0, 1);
    // nothing to do once *stop is set
    if (stop && *stop) return;
    const uint32_t rb = rbase ? 2u * static_cast<uint32_t>(*rbase) : 0u;
    const int64_t i0 = chunk * RPC;
    const size_t off = static_cast<size_t>(j) * col_bytes + chunk * 16;
    const double top = static_cast<double>(L - 2);  // highest floor position

    if constexpr (BITS == 32) {
        float vals[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = i0 + q;
            vals[q] = i < rows ? static_cast<float>(load_stacked<T, NC>(src, m, ld, i, j))
                               : 0.0f;
        }
        *reinterpret_cast<float4*>(out0 + off) =
            make_float4(vals[0], vals[1], vals[2], vals[3]);
    } else if (ALIGNED) {
        // rows % 4 == 0: element j rows + i0 + q is word q % 4 of block
        // (j rows + i0) / 4 + q / 4.  Every row of the chunk is loaded first
        // (clamped; padding rows get code 0), then the Philox blocks.
        T v[RPC];  // the input type: every value converts to FP64 exactly
#pragma unroll
        for (int q = 0; q < RPC; ++q)
            v[q] = static_cast<T>(load_stacked<T, NC>(src, m, ld, min(i0 + q, rows - 1), j));
        const uint64_t b0 = (static_cast<uint64_t>(j) * rows + i0) >> 2;
        const int nlive = static_cast<int>(min<int64_t>(RPC, rows - i0));
        // the floor position and the rounding threshold of a value are the
        // same for both realizations: taken once, then one coin each
        uint32_t w[2][4] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
#pragma unroll
        for (int b = 0; b < RPC / 4; ++b) {
            double fl[4], th[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) position_of(static_cast<double>(v[4 * b + t]), c, K, top, fl[t], th[t]);
            const uint64_t blk = b0 + b;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (r >= R) break;
                const uint4 u = philox10(make_uint4(static_cast<uint32_t>(blk), static_cast<uint32_t>(blk >> 32),
                                                    0u, rb + static_cast<uint32_t>(r)),
                                         k0, k1);
                const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int q = 4 * b + t;
                    const uint32_t code = q < nlive ? round_at(fl[t], th[t], uu[t]) : 0u;
                    w[r][(q * BITS) >> 5] |= code << ((q * BITS) & 31);
                }
            }
        }
        *reinterpret_cast<uint4*>(out0 + off) = make_uint4(w[0][0], w[0][1], w[0][2], w[0][3]);
        if (R > 1) *reinterpret_cast<uint4*>(out1 + off) = make_uint4(w[1][0], w[1][1], w[1][2], w[1][3]);
    } else {
        PhiloxStream s0{k0, k1, 0u, rb};
        PhiloxStream s1{k0, k1, 0u, rb + 1u};
        uint32_t w0[4] = {0u, 0u, 0u, 0u};
        uint32_t w1[4] = {0u, 0u, 0u, 0u};
        const uint64_t ebase = static_cast<uint64_t>(j) * rows;
#pragma unroll 4
        for (int q = 0; q < RPC; ++q) {
            const int64_t i = i0 + q;
            if (i >= rows) break;
            const double v = load_stacked<T, NC>(src, m, ld, i, j);
            const uint64_t e = ebase + i;
            const int bit = q * BITS;
            double fl, th;
            position_of(v, c, K, top, fl, th);
            w0[bit >> 5] |= round_at(fl, th, s0.word(e)) << (bit & 31);
            if (R > 1)
                w1[bit >> 5] |= round_at(fl, th, s1.word(e)) << (bit & 31);
        }
        *reinterpret_cast<uint4*>(out0 + off) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
        if (R > 1)
            *reinterpret_cast<uint4*>(out1 + off) = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    }
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_quantize_vec(
    const T* __restrict__ y, int64_t m, int64_t rows, int bits, int L, double c,
    double K, uint32_t k0, uint32_t k1, const double* __restrict__ levels,
    double* __restrict__ yhat, uint8_t* __restrict__ codes, const int32_t* __restrict__ rbase,
    const int32_t* __restrict__ stop) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    if (stop && *stop) return;  // (realization *rbase per iteration, as the matrix)
    const double v = load_stacked<T, NC>(y, m, 1, i, 0);
    if (bits == 32) {
        yhat[i] = static_cast<double>(static_cast<float>(v));
        return;
    }
    PhiloxStream s{k0, k1, 1u, rbase ? static_cast<uint32_t>(*rbase) : 0u};
    const uint32_t code = quantize_one(v, c, K, static_cast<double>(L - 2), s.word(static_cast<uint64_t>(i)));
    yhat[i] = levels[code];
    if (codes) codes[i] = static_cast<uint8_t>(code);
}

// ---------------------------------------------------------------------------
// Dense low-precision storage (no randomness): row i of the stacked matrix is
// stored as Phi_ij / 2^e_i rounded to BF16 or FP8 E4M3 (OCP), to nearest,
// ties to the even significand; e_i is the smallest integer with
// max_j |Phi_ij| / 2^e_i <= F (F = 1 for BF16, 448 for E4M3), so the
// division is exact and the rounding is the only error.
// ---------------------------------------------------------------------------
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_rowexp(const T* __restrict__ src, int64_t m, int64_t n,
                                                int64_t ld, double top, int32_t* __restrict__ rexp,
                                                int* __restrict__ bad) {
    __shared__ double smx[4];
    __shared__ int sbad[4];
    const int64_t i = blockIdx.x;  // stacked row
    double mx = 0.0;
    int nonfin = 0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double v = fabs(load_stacked<T, NC>(src, m, ld, i, j));
        if (!isfinite(v)) nonfin = 1;
        else mx = fmax(mx, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        nonfin |= __shfl_xor(nonfin, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        smx[threadIdx.x >> 6] = mx;
        sbad[threadIdx.x >> 6] = nonfin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmax(fmax(smx[0], smx[1]), fmax(smx[2], smx[3]));
        int e = 0;
        if (mx > 0.0) {
            e = ilogb(mx) - ilogb(top);
            while (ldexp(mx, -e) > top) ++e;
            while (ldexp(mx, -(e - 1)) <= top) --e;
        }
        rexp[i] = e;
        if (sbad[0] | sbad[1] | sbad[2] | sbad[3]) atomicOr(bad, 1);
    }
}

// Nearest value with P significand bits (the leading one included), smallest
// normal exponent EMIN, saturating at +-VMAX.  Every step is exact except the
// rint, which rounds ties to even.
template <int P, int EMIN>
__device__ __forceinline__ double round_format(double x, double vmax) {
    if (x == 0.0) return 0.0;
    const int e = max(ilogb(x), EMIN);
    const int qe = e - (P - 1);
    const double y = ldexp(rint(ldexp(x, -qe)), qe);
    return fmin(fmax(y, -vmax), vmax);
}

__device__ __forceinline__ uint32_t encode_bf16(double x) {
    return __float_as_uint(static_cast<float>(round_format<8, -126>(x, 0x1.fep127))) >> 16;
}

__device__ __forceinline__ uint32_t encode_e4m3(double x) {
    const double y = round_format<4, -6>(x, 448.0);
    const uint32_t sgn = y < 0.0 ? 0x80u : 0u;
    const double a = fabs(y);
    if (a == 0.0) return sgn;
    if (a < 0x1p-6) return sgn | static_cast<uint32_t>(a * 512.0);  // subnormal: a = k 2^-9
    const int E = ilogb(a);
    return sgn | (static_cast<uint32_t>(E + 7) << 3) | (static_cast<uint32_t>(ldexp(a, 3 - E)) - 8u);
}

// One thread = one column j and one 16-byte chunk (8 BF16 or 16 E4M3 rows).
template <int FMT, typename T, int NC>
__global__ __launch_bounds__(256) void k_store(const T* __restrict__ src, int64_t m, int64_t n,
                                               int64_t ld, int64_t rows, int64_t col_bytes,
                                               int64_t nchunks, const int32_t* __restrict__ rexp,
                                               uint8_t* __restrict__ out) {
    constexpr int RPC = (FMT == 16) ? 8 : 16;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const int64_t chunk = static_cast<int64_t>(blockIdx.y) * 4 + wave;
    if (j >= n || chunk >= nchunks) return;
    const int64_t i0 = chunk * RPC;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < RPC; ++q) {
        const int64_t i = i0 + q;
        if (i >= rows) break;
        const double x = ldexp(load_stacked<T, NC>(src, m, ld, i, j), -rexp[i]);
        const int bit = q * (FMT == 16 ? 16 : 8);
        w[bit >> 5] |= (FMT == 16 ? encode_bf16(x) : encode_e4m3(x)) << (bit & 31);
    }
    *reinterpret_cast<uint4*>(out + static_cast<size_t>(j) * col_bytes + chunk * 16) =
        make_uint4(w[0], w[1], w[2], w[3]);
}

template <typename T, int NC>
qiht_status store_t(int fmt, const void* src, int64_t m, int64_t n, int64_t ld, qiht_qmatrix* q,
                    hipStream_t st) {
    int* d_bad = nullptr;
    QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&d_bad), sizeof(int), st));
    QIHT_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), st));
    hipLaunchKernelGGL((k_rowexp<T, NC>), dim3(static_cast<unsigned>(q->rows)), dim3(256), 0, st,
                       static_cast<const T*>(src), m, n, ld, fmt == 16 ? 1.0 : 448.0, q->rexp, d_bad);
    QIHT_HIP(hipGetLastError());
    const int64_t nchunks = q->col_bytes / 16;
    dim3 grid(static_cast<unsigned>((n + 63) / 64), static_cast<unsigned>((nchunks + 3) / 4));
    if (fmt == 16)
        hipLaunchKernelGGL((k_store<16, T, NC>), grid, dim3(256), 0, st, static_cast<const T*>(src),
                           m, n, ld, q->rows, q->col_bytes, nchunks, q->rexp, q->codes[0]);
    else
        hipLaunchKernelGGL((k_store<9, T, NC>), grid, dim3(256), 0, st, static_cast<const T*>(src),
                           m, n, ld, q->rows, q->col_bytes, nchunks, q->rexp, q->codes[0]);
    QIHT_HIP(hipGetLastError());
    int bad = 0;
    QIHT_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
    QIHT_HIP(hipFreeAsync(d_bad, st));
    QIHT_HIP(hipStreamSynchronize(st));
    if (bad) return fail(QIHT_ERR_NUMERIC, "input contains NaN or Inf");
    return QIHT_OK;
}

template <typename T, int NC>
qiht_status absmax_t(const void* src, int64_t m, int64_t n, int64_t ld,
                     hipStream_t st, double* c_out) {
    unsigned long long* d_max = nullptr;
    int* d_bad = nullptr;
    QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&d_max), 16, st));
    d_bad = reinterpret_cast<int*>(d_max + 1);
    QIHT_HIP(hipMemsetAsync(d_max, 0, 16, st));
    const int64_t row_len = n * NC;
    bool vec = false;
    if constexpr (std::is_same<T, float>::value)
        vec = row_len % 4 == 0 && (ld * NC) % 4 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0;
    if (vec) {
        const int64_t row4 = row_len / 4;
        const int64_t gx = std::min<int64_t>((row4 + 1023) / 1024, 16);
        const int64_t gy = std::min<int64_t>(m, std::max<int64_t>(1, 4096 / gx));
        hipLaunchKernelGGL(k_absmax_f4, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(gy)), dim3(256), 0, st,
                           static_cast<const float4*>(src), m, row4, ld * NC / 4, d_max, d_bad);
    } else {
        const int64_t gx = std::min<int64_t>((row_len + 1023) / 1024, 16);
        const int64_t gy = std::min<int64_t>(m, std::max<int64_t>(1, 4096 / gx));
        dim3 grid(static_cast<unsigned>(gx), static_cast<unsigned>(gy));
        hipLaunchKernelGGL((k_absmax<T, NC>), grid, dim3(256), 0, st,
                           static_cast<const T*>(src), m, n, ld, d_max, d_bad);
    }
    QIHT_HIP(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    QIHT_HIP(hipMemcpyAsync(h, d_max, 16, hipMemcpyDeviceToHost, st));
    QIHT_HIP(hipFreeAsync(d_max, st));
    QIHT_HIP(hipStreamSynchronize(st));
    int bad = 0;
    std::memcpy(&bad, &h[1], sizeof(int));
    if (bad) return fail(QIHT_ERR_NUMERIC, "input contains NaN or Inf");
    double c;
    std::memcpy(&c, &h[0], sizeof(double));
    *c_out = c;
    return QIHT_OK;
}

template <int BITS, typename T, int NC>
void launch_q(const void* src, int64_t m, int64_t n, int64_t ld, int R,
              uint64_t seed, double c, double K, int L, qiht_qmatrix* q,
              hipStream_t st, const int32_t* rbase, const int32_t* stop) {
    const int64_t nchunks = q->col_bytes / 16;
    dim3 grid(static_cast<unsigned>((nchunks + 3) / 4),
              static_cast<unsigned>((n + 63) / 64));  // n <= 65535 * 64 (checked by the caller)
    if (q->rows % 4 == 0)
        hipLaunchKernelGGL((k_quantize<BITS, T, NC, true>), grid, dim3(256), 0, st,
                           static_cast<const T*>(src), m, n, ld, q->rows,
                           q->col_bytes, nchunks, c, K, L,
                           static_cast<uint32_t>(seed),
                           static_cast<uint32_t>(seed >> 32), R, q->codes[0],
                           q->codes[1], rbase, stop);
    else
        hipLaunchKernelGGL((k_quantize<BITS, T, NC, false>), grid, dim3(256), 0, st,
                           static_cast<const T*>(src), m, n, ld, q->rows,
                           q->col_bytes, nchunks, c, K, L,
                           static_cast<uint32_t>(seed),
                           static_cast<uint32_t>(seed >> 32), R, q->codes[0],
                           q->codes[1], rbase, stop);
}

template <typename T, int NC>
qiht_status dispatch_bits(int bits, const void* src, int64_t m, int64_t n,
                          int64_t ld, int R, uint64_t seed, double c, double K, int L,
                          qiht_qmatrix* q, hipStream_t st, const int32_t* rbase,
                          const int32_t* stop) {
    switch (bits) {
        case 1: launch_q<1, T, NC>(src, m, n, ld, R, seed, c, K, L, q, st, rbase, stop); break;
        case 2: launch_q<2, T, NC>(src, m, n, ld, R, seed, c, K, L, q, st, rbase, stop); break;
        case 4: launch_q<4, T, NC>(src, m, n, ld, R, seed, c, K, L, q, st, rbase, stop); break;
        case 8: launch_q<8, T, NC>(src, m, n, ld, R, seed, c, K, L, q, st, rbase, stop); break;
        case 32: launch_q<32, T, NC>(src, m, n, ld, R, seed, c, K, L, q, st, rbase, stop); break;
        default: return fail(QIHT_ERR_UNSUPPORTED, "unsupported bit width");
    }
    QIHT_HIP(hipGetLastError());
    return QIHT_OK;
}

}  // namespace

qiht_status device_absmax(const void* src, qiht_dtype dt, int64_t m,
                          int64_t n, int64_t ld, hipStream_t st,
                          double* c_out) {
    switch (dt) {
        case QIHT_F32: return absmax_t<float, 1>(src, m, n, ld, st, c_out);
        case QIHT_F64: return absmax_t<double, 1>(src, m, n, ld, st, c_out);
        case QIHT_C64: return absmax_t<float, 2>(src, m, n, ld, st, c_out);
        case QIHT_C128: return absmax_t<double, 2>(src, m, n, ld, st, c_out);
    }
    return fail(QIHT_ERR_UNSUPPORTED, "unsupported dtype");
}

qiht_status launch_quantize_matrix(const void* src, qiht_dtype dt, int64_t m,
                                   int64_t n, int64_t ld, int bits, int R,
                                   uint64_t seed, double c, double K, int levels,
                                   qiht_qmatrix* q, hipStream_t st, const int32_t* rbase,
                                   const int32_t* stop) {
    switch (dt) {
        case QIHT_F32: return dispatch_bits<float, 1>(bits, src, m, n, ld, R, seed, c, K, levels, q, st, rbase, stop);
        case QIHT_F64: return dispatch_bits<double, 1>(bits, src, m, n, ld, R, seed, c, K, levels, q, st, rbase, stop);
        case QIHT_C64: return dispatch_bits<float, 2>(bits, src, m, n, ld, R, seed, c, K, levels, q, st, rbase, stop);
        case QIHT_C128: return dispatch_bits<double, 2>(bits, src, m, n, ld, R, seed, c, K, levels, q, st, rbase, stop);
    }
    return fail(QIHT_ERR_UNSUPPORTED, "unsupported dtype");
}

qiht_status launch_store_matrix(const void* src, qiht_dtype dt, int64_t m, int64_t n,
                                int64_t ld, int fmt, qiht_qmatrix* q, hipStream_t st) {
    switch (dt) {
        case QIHT_F32: return store_t<float, 1>(fmt, src, m, n, ld, q, st);
        case QIHT_F64: return store_t<double, 1>(fmt, src, m, n, ld, q, st);
        case QIHT_C64: return store_t<float, 2>(fmt, src, m, n, ld, q, st);
        case QIHT_C128: return store_t<double, 2>(fmt, src, m, n, ld, q, st);
    }
    return fail(QIHT_ERR_UNSUPPORTED, "unsupported dtype");
}

qiht_status launch_quantize_vector(const void* y, qiht_dtype dt, int64_t m,
                                   int bits, int levels, uint64_t seed, double c,
                                   double K, const double* levels_dev,
                                   double* yhat, uint8_t* codes,
                                   hipStream_t st, const int32_t* rbase, const int32_t* stop) {
    const bool cplx = (dt == QIHT_C64 || dt == QIHT_C128);
    const int64_t rows = cplx ? 2 * m : m;
    dim3 grid(static_cast<unsigned>((rows + 255) / 256));
    const uint32_t k0 = static_cast<uint32_t>(seed);
    const uint32_t k1 = static_cast<uint32_t>(seed >> 32);
    switch (dt) {
        case QIHT_F32:
            hipLaunchKernelGGL((k_quantize_vec<float, 1>), grid, dim3(256), 0, st,
                               static_cast<const float*>(y), m, rows, bits, levels, c, K, k0, k1,
                               levels_dev, yhat, codes, rbase, stop);
            break;
        case QIHT_F64:
            hipLaunchKernelGGL((k_quantize_vec<double, 1>), grid, dim3(256), 0, st,
                               static_cast<const double*>(y), m, rows, bits, levels, c, K, k0, k1,
                               levels_dev, yhat, codes, rbase, stop);
            break;
        case QIHT_C64:
            hipLaunchKernelGGL((k_quantize_vec<float, 2>), grid, dim3(256), 0, st,
                               static_cast<const float*>(y), m, rows, bits, levels, c, K, k0, k1,
                               levels_dev, yhat, codes, rbase, stop);
            break;
        case QIHT_C128:
            hipLaunchKernelGGL((k_quantize_vec<double, 2>), grid, dim3(256), 0, st,
                               static_cast<const double*>(y), m, rows, bits, levels, c, K, k0, k1,
                               levels_dev, yhat, codes, rbase, stop);
            break;
    }
    QIHT_HIP(hipGetLastError());
    return QIHT_OK;
}

}  // namespace qiht
