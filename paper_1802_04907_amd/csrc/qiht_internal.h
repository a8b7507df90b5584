// Internal declarations shared by the translation units of libqiht.
// Not part of the public ABI (see include/qiht.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "qiht.h"

// ---------------------------------------------------------------------------
// Quantized matrix handle.
//
// Device layout: column-major, one column after another, each column padded
// to `col_bytes` (a multiple of 256 bytes).  Within a column, code of row i
// sits in byte (i * bits) / 8 at bit offset (i * bits) % 8 (little-endian
// within the byte).  Padding rows hold code 0 and are never read as data:
// every kernel masks rows >= rows.  bits == 32 stores plain floats.
// ---------------------------------------------------------------------------
struct qiht_qmatrix {
    int device = 0;
    int64_t m = 0;         // rows of the caller's Phi
    int64_t n = 0;         // columns
    int64_t rows = 0;      // m, or 2m for complex input ([Re; Im])
    int bits = 0;          // stored width: 1, 2, 4, 8 or 32 (codes / plain floats),
                           // or a dense format: kFmtBF16 (16) or kFmtE4M3 (9)
    int code_bits = 0;     // width b of the codes (1..8, held in `bits`-wide fields)
    int levels = 0;        // levels of the code set (0 for 32 and dense formats)
    int realizations = 0;  // 1 or 2
    double scale = 0.0;    // c = max |Phi_ij| (0 for bits 32)
    double alpha = 0.0;    // dequantized value = alpha * code + beta
    double beta = 0.0;
    int64_t col_bytes = 0; // stride between columns
    int64_t rows_pad = 0;  // rows covered by col_bytes
    uint8_t* codes[2] = {nullptr, nullptr};  // codes[1] == codes[0] if R == 1
    bool pooled = false;   // codes from the handle memory pool (else hipMalloc)
    int32_t* rexp = nullptr;  // dense formats: row exponents e_i (device, rows)
    // complex input: the real embedding [Q_re -Q_im; Q_im Q_re] used for a
    // complex unknown (built on first use by complex.hip, freed with this)
    qiht_qmatrix* embedded = nullptr;
};

namespace qiht {

// Error reporting (thread-local message behind qiht_last_error).
void set_error(const std::string& msg);
qiht_status fail(qiht_status st, const std::string& msg);
qiht_status hip_fail(hipError_t e, const char* what);

#define QIHT_HIP(call)                                                    \
    do {                                                                  \
        hipError_t _e = (call);                                           \
        if (_e != hipSuccess) return ::qiht::hip_fail(_e, #call);         \
    } while (0)

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Internal ids of the dense formats (the public ones are QIHT_FMT_*).
constexpr int kFmtBF16 = 16;
constexpr int kFmtE4M3 = 9;
inline bool is_dense_format(int bits) { return bits == kFmtBF16 || bits == kFmtE4M3; }
// Stored bits per element.
inline int storage_bits(int bits) { return bits == kFmtE4M3 ? 8 : bits; }

// Bytes per column for a given row count and bit width (multiple of 256).
inline int64_t column_bytes(int64_t rows, int bits) {
    int64_t raw = (rows * storage_bits(bits) + 7) / 8;
    if (raw < 1) raw = 1;
    return round_up(raw, 256);
}

inline int64_t rows_in_bytes(int64_t col_bytes, int bits) {
    return col_bytes * 8 / storage_bits(bits);
}

// ---- quantization (quantize.hip) ----
// Max-abs of a row-major (complex: interleaved) matrix, and a NaN/Inf flag.
qiht_status device_absmax(const void* src, qiht_dtype dt, int64_t m,
                          int64_t n, int64_t ld, hipStream_t st,
                          double* c_out);
qiht_status launch_quantize_matrix(const void* src, qiht_dtype dt, int64_t m,
                                   int64_t n, int64_t ld, int bits, int R,
                                   uint64_t seed, double c, double K, int levels,
                                   qiht_qmatrix* q, hipStream_t st,
                                   const int32_t* rbase = nullptr, const int32_t* stop = nullptr);
qiht_status launch_store_matrix(const void* src, qiht_dtype dt, int64_t m, int64_t n,
                                int64_t ld, int fmt, qiht_qmatrix* q, hipStream_t st);
qiht_status launch_quantize_vector(const void* y, qiht_dtype dt, int64_t m,
                                   int bits, int levels, uint64_t seed, double c,
                                   double K, const double* levels_dev,
                                   double* yhat, uint8_t* codes,
                                   hipStream_t st, const int32_t* rbase = nullptr,
                                   const int32_t* stop = nullptr);

// ---- solver (solve.hip) ----
struct SolveArgs {
    int32_t max_iters;
    double tol;
    double k;
    double c;
    int32_t max_backtracks;
    int32_t mu_mode;
    int32_t profile;
    int32_t decide_in_gather;  // the residual gather takes the step-size test (else k_commit)
};


struct ProblemIn {
    const qiht_qmatrix* q;
    const double* yhat;
    int64_t s;
    float* x_out;
    int32_t* support_out;
    const float* x0;
    const int32_t* support0;
    int64_t group = 0;  // > 0: a complex unknown of `group` entries on the
                        // embedding (columns j and j + group pair up; s even)
};

// Algorithm 2 with its realizations drawn per iteration (one problem): the
// sources and quantizer constants each round re-quantizes from.
struct FreshSource {
    const void* phi;
    qiht_dtype dtype;
    int64_t m, n, ld;
    int bits, levels;       // internal bit width, levels of the code set
    uint64_t seed;
    double c, K;            // scale and (levels - 1) / (2c) of the matrix
    qiht_qmatrix* q;        // the handle whose two code buffers are rewritten
    const void* y;
    qiht_dtype ydtype;
    int ybits, ylevels;
    double yc, yK;
    const double* ylev;     // device: the level values of y
    double* yhat;           // device: the y_hat the solve reads
};

// ext_ws (optional): ext_cap bytes of device memory that hold the workspace
// instead of the library's pool (UNSUPPORTED when the solve needs more).
qiht_status run_solve(const ProblemIn* probs, int count, const SolveArgs& a,
                      qiht_info* infos, hipStream_t st, const FreshSource* fresh = nullptr,
                      uint8_t* ext_ws = nullptr, size_t ext_cap = 0);
// The autotuner's choices so far, as JSON (solve_host.hip).
std::string tune_report();
// QIHT with a complex unknown on a complex-input handle (complex.hip):
// x_out (device, 2n floats) receives [Re x; Im x], support_out the s entries.
qiht_status run_solve_complex(qiht_qmatrix* q, const double* yhat, int64_t s, const SolveArgs& a, int refit,
                              float* x_out, int32_t* support_out, qiht_info* info, hipStream_t st);
// One solve whose workspace is the library's fixed device array (no device
// allocation); calls on one device take turns.
qiht_status run_solve_noalloc(const ProblemIn& in, const SolveArgs& a, qiht_info* info,
                              hipStream_t st);

qiht_status run_gradient(const qiht_qmatrix* q, const double* yhat,
                         const float* x, const int32_t* support, int64_t s,
                         float* g_out, float* r_out, hipStream_t st);

qiht_status run_hard_threshold(const float* a, int64_t n, int64_t s,
                               int32_t* support_out, hipStream_t st);

// Least-squares refit on a support (refit.hip).  A is the dense phi when
// given (row-major m x n, leading dimension ld, real or complex stacked), else
// the dequantized codes (bits, col_bytes, alpha, beta).
struct RefitIn {
    const uint8_t* codes;
    int64_t col_bytes;
    int bits;
    double alpha, beta;
    const int32_t* rowexp;  // dense formats: row exponents
    const void* phi;
    int64_t m, ld;
    qiht_dtype dtype;
    int64_t rows, n, s;
    const double* y;
    const int32_t* sup;
    float* x_out;
    double* xs_out;
};
qiht_status run_refit(const RefitIn& in, hipStream_t st);
// The refits of `count` problems (same source kind: packed codes of one bit
// width or format, or one dense dtype) as one sequence of launches.
qiht_status run_refit_batch(const RefitIn* in, int count, hipStream_t st);

// Stream-ordered device allocation from the library's own memory pool (one per
// device, created on first use).  The pool keeps freed memory for the next
// call instead of handing it back to the driver at every synchronization
// (re-mapping a workspace of hundreds of MB cost milliseconds per solve); it
// grows to the largest workspace in use at once and is held until the
// process ends.  Free with hipFreeAsync.
// handle: memory that a qiht_qmatrix keeps (its own pool).
hipError_t pool_malloc(void** p, size_t bytes, hipStream_t st, bool handle = false);
// hipMalloc for memory that outlives the call (handles).  Both allocators
// honour QIHT_FAIL_ALLOC_AFTER (allocation-failure injection for tests).
hipError_t dev_malloc(void** p, size_t bytes);

// g = [Re Phi; Im Phi]^T r for a Fourier-sampled Phi evaluated on the fly
// (fourier.hip); arguments validated by the caller.
qiht_status run_fourier_gradient(const double* uv, int64_t nvis, int side, const float* r, float* g,
                                 hipStream_t st);
// Normalized IHT with every product by that Phi computed on the fly
// (fourier.hip); x and support are the caller's outputs, used as the state.
qiht_status run_fourier_solve(const double* uv, int64_t nvis, int side, const double* y, int64_t s,
                              const qiht_params& prm, float* x, int32_t* sup, qiht_info* info, hipStream_t st);

}  // namespace qiht
