// C ABI of libqiht: argument validation, handle management and dispatch to
// the quantization and solver launchers.  Every entry point checks its
// arguments on the host before touching the device and reports errors as
// status codes plus a thread-local message; no exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qiht_internal.h"

namespace qiht {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

qiht_status fail(qiht_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

qiht_status hip_fail(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(QIHT_ERR_OUT_OF_MEMORY, m);
    return fail(QIHT_ERR_DEVICE, m);
}

namespace {

bool bits_ok_matrix(int b) {
    return (b >= 1 && b <= 8) || b == 32 || b == QIHT_FMT_BF16 || b == QIHT_FMT_E4M3;
}
// Stored width of a b-bit code: 1, 2, 4 or 8 (3 -> 4, 5..7 -> 8), so that a
// byte holds whole codes and the pass reads one layout per width.
int container_bits(int b) { return b <= 2 ? b : (b <= 4 ? 4 : 8); }
// public bit width / format -> internal id, and back
int internal_bits(int b) { return b == QIHT_FMT_BF16 ? kFmtBF16 : b == QIHT_FMT_E4M3 ? kFmtE4M3 : b; }
int public_bits(int b) { return b == kFmtBF16 ? QIHT_FMT_BF16 : b == kFmtE4M3 ? QIHT_FMT_E4M3 : b; }
bool bits_ok_vector(int b) { return (b >= 1 && b <= 12) || b == 32; }
// Levels of a b-bit code: 2^b, or with QIHT_ODD_LEVELS 2^(b-1) + 1.
int num_levels(int b, bool odd) { return odd ? (1 << (b - 1)) + 1 : 1 << b; }
bool dtype_ok(int d) { return d >= QIHT_F64 && d <= QIHT_C128; }
bool is_complex(qiht_dtype d) { return d == QIHT_C64 || d == QIHT_C128; }

qiht_status need_device(int* dev) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return fail(QIHT_ERR_DEVICE, "no HIP device available");
    }
    QIHT_HIP(hipGetDevice(dev));
    return QIHT_OK;
}

qiht_status check_params(const qiht_params* p) {
    if (!p) return fail(QIHT_ERR_INVALID_ARG, "params is NULL");
    if (p->max_iters < 1) return fail(QIHT_ERR_INVALID_ARG, "max_iters must be >= 1");
    if (!(p->c >= 0.0 && p->c < 1.0)) return fail(QIHT_ERR_INVALID_ARG, "need 0 <= c < 1");
    if (!(p->k > 1.0 / (1.0 - p->c)))
        return fail(QIHT_ERR_INVALID_ARG, "need k > 1/(1 - c)");
    if (p->max_backtracks < 0) return fail(QIHT_ERR_INVALID_ARG, "max_backtracks must be >= 0");
    if (p->mu_mode != 0 && p->mu_mode != 1) return fail(QIHT_ERR_INVALID_ARG, "mu_mode is 0 or 1");
    if (std::isnan(p->tol)) return fail(QIHT_ERR_INVALID_ARG, "tol is NaN");
    if ((p->x0 == nullptr) != (p->support0 == nullptr))
        return fail(QIHT_ERR_INVALID_ARG, "x0 and support0 go together");
    if (p->refit != 0 && p->refit != 1) return fail(QIHT_ERR_INVALID_ARG, "refit is 0 or 1");
    if (p->profile < 0) return fail(QIHT_ERR_INVALID_ARG, "profile must be >= 0");
    return QIHT_OK;
}

SolveArgs to_args(const qiht_params* p) {
    SolveArgs a{};
    a.max_iters = p->max_iters;
    a.tol = p->tol;
    a.k = p->k;
    a.c = p->c;
    a.max_backtracks = p->max_backtracks;
    a.mu_mode = p->mu_mode;
    a.profile = p->profile;
    return a;
}

// Refit of a solve's result on its support against the first realization.
RefitIn codes_refit(const qiht_qmatrix* q, const double* y, const int32_t* sup, int64_t s,
                    float* x_out) {
    RefitIn r{};
    r.codes = q->codes[0];
    r.col_bytes = q->col_bytes;
    r.bits = q->bits;
    r.alpha = q->alpha;
    r.beta = q->beta;
    r.rowexp = q->rexp;
    r.phi = nullptr;
    r.rows = q->rows;
    r.n = q->n;
    r.s = s;
    r.y = y;
    r.sup = sup;
    r.x_out = x_out;
    r.xs_out = nullptr;
    return r;
}

qiht_status check_problem(const qiht_qmatrix* q, const double* yhat, int64_t s, const void* x_out,
                          const void* sup_out) {
    if (!q) return fail(QIHT_ERR_INVALID_ARG, "quantized matrix is NULL");
    if (!yhat) return fail(QIHT_ERR_INVALID_ARG, "yhat is NULL");
    if (!x_out || !sup_out) return fail(QIHT_ERR_INVALID_ARG, "output pointer is NULL");
    if (s < 1 || s > q->rows || s > q->n)
        return fail(QIHT_ERR_INVALID_ARG, "need 1 <= s <= min(rows, n)");
    if (q->n > (1LL << 31) - 1 || q->rows > (1LL << 31) - 1)
        return fail(QIHT_ERR_UNSUPPORTED, "dimension above 2^31 - 1");
    return QIHT_OK;
}

// Copy a device support list to the host and check it is strictly
// increasing inside [0, n).
qiht_status check_support(const int32_t* dev_sup, int64_t s, int64_t n, hipStream_t st) {
    if (s == 0) return QIHT_OK;
    std::vector<int32_t> h(static_cast<size_t>(s));
    QIHT_HIP(hipMemcpyAsync(h.data(), dev_sup, sizeof(int32_t) * s, hipMemcpyDeviceToHost, st));
    QIHT_HIP(hipStreamSynchronize(st));
    for (int64_t t = 0; t < s; ++t) {
        if (h[t] < 0 || h[t] >= n) return fail(QIHT_ERR_INVALID_ARG, "support index out of range");
        if (t > 0 && h[t] <= h[t - 1])
            return fail(QIHT_ERR_INVALID_ARG, "support must be strictly increasing");
    }
    return QIHT_OK;
}

}  // namespace

const char* last_error_cstr() { return g_last_error.c_str(); }

// Allocation-failure injection, for tests of the error paths:
// QIHT_FAIL_ALLOC_AFTER=N lets N more device allocations of the library
// succeed and fails every later one with hipErrorOutOfMemory (no device call
// is made for those).  The count starts again whenever the variable's value
// changes; unset or empty switches the injection off.
bool alloc_fault() {
    static std::mutex mu;
    static std::string seen;
    static long long left = -1;
    const char* v = std::getenv("QIHT_FAIL_ALLOC_AFTER");
    const std::string now = v ? v : "";
    std::lock_guard<std::mutex> lk(mu);
    if (now != seen) {
        seen = now;
        left = now.empty() ? -1 : std::max(0LL, std::atoll(now.c_str()));
    }
    if (left < 0) return false;
    if (left == 0) return true;
    --left;
    return false;
}

hipError_t dev_malloc(void** p, size_t bytes) {
    if (alloc_fault()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t pool_malloc(void** p, size_t bytes, hipStream_t st, bool handle) {
    if (alloc_fault()) return hipErrorOutOfMemory;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    // Three pools per device: per-call workspaces, small temporaries (flags,
    // level tables) and the codes of handles.  Kept apart so that neither a
    // temporary nor a handle splits a freed solve workspace: the next solve
    // of the same shape gets its workspace back at the same address (which
    // its captured graphs were recorded with).
    static std::mutex mu;
    static std::vector<hipMemPool_t> pools;
    const size_t kind = handle ? 2 : (bytes <= (size_t(64) << 10) ? 1 : 0);
    const size_t at = 3 * static_cast<size_t>(dev) + kind;
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (pools.size() <= at) pools.resize(at + 1, nullptr);
        if (!pools[at]) {
            hipMemPoolProps props{};
            props.allocType = hipMemAllocationTypePinned;
            props.handleTypes = hipMemHandleTypeNone;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            hipMemPool_t np = nullptr;
            e = hipMemPoolCreate(&np, &props);
            if (e != hipSuccess) return e;
            uint64_t keep = UINT64_MAX;
            e = hipMemPoolSetAttribute(np, hipMemPoolAttrReleaseThreshold, &keep);
            if (e != hipSuccess) {
                (void)hipMemPoolDestroy(np);
                return e;
            }
            pools[at] = np;
        }
        pool = pools[at];
    }
    return hipMallocFromPoolAsync(p, bytes, pool, st);
}
}  // namespace qiht

using namespace qiht;

// Deterministic dense storage (QIHT_FMT_BF16 / QIHT_FMT_E4M3): one copy,
// row exponents alongside.
qiht_status store_dense(const void* phi, qiht_dtype dtype, int64_t m, int64_t n, int64_t ld,
                        int bits, int64_t rows, int64_t cb, int dev, hipStream_t st,
                        qiht_qmatrix** out) {
    qiht_qmatrix* q = new qiht_qmatrix();
    q->device = dev;
    q->m = m;
    q->n = n;
    q->rows = rows;
    q->bits = bits;
    q->realizations = 1;
    q->col_bytes = cb;
    q->rows_pad = rows_in_bytes(cb, bits);
    const size_t bytes = static_cast<size_t>(cb) * static_cast<size_t>(n);
    const size_t rbytes = static_cast<size_t>(round_up(rows * 4, 256));
    hipError_t e = dev_malloc(reinterpret_cast<void**>(&q->codes[0]), bytes + rbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete q;
        return fail(QIHT_ERR_OUT_OF_MEMORY, "storage allocation failed");
    }
    q->codes[1] = q->codes[0];
    q->rexp = reinterpret_cast<int32_t*>(q->codes[0] + bytes);
    e = hipMemsetAsync(q->codes[0], 0, bytes, st);  // padding rows stay 0
    qiht_status s0 = (e == hipSuccess) ? launch_store_matrix(phi, dtype, m, n, ld, bits, q, st)
                                       : hip_fail(e, "clear storage");
    if (s0 != QIHT_OK) {
        (void)hipFree(q->codes[0]);
        delete q;
        return s0;
    }
    *out = q;
    return QIHT_OK;
}

extern "C" {

void qiht_default_params(qiht_params* p) {
    if (!p) return;
    p->max_iters = 300;
    p->tol = 1e-8;
    p->k = 2.0;
    p->c = 0.01;
    p->max_backtracks = 32;
    p->mu_mode = 0;
    p->x0 = nullptr;
    p->support0 = nullptr;
    p->profile = 0;
    p->refit = 0;
}

const char* qiht_last_error(void) { return last_error_cstr(); }

const char* qiht_version(void) { return "qiht-gfx950 0.1"; }

int64_t qiht_tune_report(char* buf, int64_t cap) try {
    const std::string r = tune_report();
    if (buf && cap > 0) {
        const size_t n = std::min(static_cast<size_t>(cap - 1), r.size());
        std::memcpy(buf, r.data(), n);
        buf[n] = '\0';
    }
    return static_cast<int64_t>(r.size()) + 1;
} catch (...) {
    return 0;
}

qiht_status qiht_quantize_matrix(const void* phi, int64_t m, int64_t n, int64_t ld,
                                 qiht_dtype dtype, int bits, int realizations, uint64_t seed,
                                 void* stream, qiht_qmatrix** out) try {
    set_error("");
    if (!phi || !out) return fail(QIHT_ERR_INVALID_ARG, "phi or out is NULL");
    if (m < 1 || n < 1) return fail(QIHT_ERR_INVALID_ARG, "need m >= 1 and n >= 1");
    if (n > int64_t(65535) * 64) return fail(QIHT_ERR_UNSUPPORTED, "n above 4194240 columns");
    if (ld < n) return fail(QIHT_ERR_INVALID_ARG, "need ld >= n");
    if (!dtype_ok(dtype)) return fail(QIHT_ERR_UNSUPPORTED, "unknown dtype");
    const bool odd = (bits & QIHT_ODD_LEVELS) != 0;
    bits &= ~QIHT_ODD_LEVELS;
    if (!bits_ok_matrix(bits))
        return fail(QIHT_ERR_UNSUPPORTED, "bits must be 1..8, 32, QIHT_FMT_BF16 or QIHT_FMT_E4M3");
    if (odd && (bits < 2 || bits > 8))
        return fail(QIHT_ERR_UNSUPPORTED, "QIHT_ODD_LEVELS needs packed codes of 2..8 bits");
    if (realizations != 1 && realizations != 2)
        return fail(QIHT_ERR_INVALID_ARG, "realizations must be 1 or 2");
    const int code_bits = bits;
    const int levels = (bits == 32 || bits > 8) ? 0 : num_levels(bits, odd);
    bits = (bits <= 8) ? container_bits(bits) : internal_bits(bits);
    const int64_t rows = is_complex(dtype) ? 2 * m : m;
    if (rows > (1LL << 31) - 1 || n > (1LL << 31) - 1)
        return fail(QIHT_ERR_UNSUPPORTED, "dimension above 2^31 - 1");
    const int64_t cb = column_bytes(rows, bits);
    if (cb > (int64_t(1) << 40) / n) return fail(QIHT_ERR_INVALID_ARG, "matrix too large");
    int dev = 0;
    qiht_status s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (is_dense_format(bits)) return store_dense(phi, dtype, m, n, ld, bits, rows, cb, dev, st, out);
    double c = 0.0;
    s0 = device_absmax(phi, dtype, m, n, ld, st, &c);
    if (s0 != QIHT_OK) return s0;
    const int R = (bits == 32) ? 1 : realizations;
    qiht_qmatrix* q = new qiht_qmatrix();
    q->device = dev;
    q->m = m;
    q->n = n;
    q->rows = rows;
    q->bits = bits;
    q->code_bits = code_bits;
    q->levels = levels;
    q->realizations = R;
    q->col_bytes = cb;
    q->rows_pad = rows_in_bytes(cb, bits);
    q->scale = (bits == 32) ? 0.0 : c;
    if (bits != 32 && c > 0.0) {
        q->alpha = 2.0 * c / (levels - 1.0);
        q->beta = -c;
    }
    const size_t bytes = static_cast<size_t>(cb) * static_cast<size_t>(n);
    hipError_t e = pool_malloc(reinterpret_cast<void**>(&q->codes[0]), bytes * R, st, true);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete q;
        return fail(QIHT_ERR_OUT_OF_MEMORY, "code allocation failed");
    }
    q->pooled = true;
    q->codes[1] = (R == 2) ? q->codes[0] + bytes : q->codes[0];
    const double K = (bits == 32 || c == 0.0) ? 0.0 : (levels - 1) / (2.0 * c);
    s0 = launch_quantize_matrix(phi, dtype, m, n, ld, bits, R, seed, c, K, levels, q, st);
    if (s0 == QIHT_OK) {
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) s0 = hip_fail(e, "quantize");
    }
    if (s0 != QIHT_OK) {
        qiht_qmatrix_free(q);
        return s0;
    }
    *out = q;
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_quantize_vector(const void* y, int64_t m, qiht_dtype dtype, int bits,
                                 uint64_t seed, void* stream, double* yhat_out,
                                 uint8_t* codes_out, double* scale_out) try {
    set_error("");
    if (!y || !yhat_out) return fail(QIHT_ERR_INVALID_ARG, "y or yhat_out is NULL");
    if (m < 1) return fail(QIHT_ERR_INVALID_ARG, "need m >= 1");
    if (!dtype_ok(dtype)) return fail(QIHT_ERR_UNSUPPORTED, "unknown dtype");
    const bool odd = (bits & QIHT_ODD_LEVELS) != 0;
    bits &= ~QIHT_ODD_LEVELS;
    if (!bits_ok_vector(bits)) return fail(QIHT_ERR_UNSUPPORTED, "bits must be 1..12 or 32");
    if (odd && (bits < 2 || bits > 12))
        return fail(QIHT_ERR_UNSUPPORTED, "QIHT_ODD_LEVELS needs 2..12 bits");
    if (bits > 8 && codes_out) return fail(QIHT_ERR_INVALID_ARG, "codes_out is for bits <= 8");
    int dev = 0;
    qiht_status s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double c = 0.0;
    s0 = device_absmax(y, dtype, 1, m, m, st, &c);
    if (s0 != QIHT_OK) return s0;
    double* lev = nullptr;
    double K = 0.0;
    const int levels = (bits == 32) ? 0 : num_levels(bits, odd);
    if (bits != 32) {
        const int L = levels;
        std::vector<double> h(L);
        for (int k = 0; k < L; ++k) h[k] = c * (2.0 * k / static_cast<double>(L - 1) - 1.0);
        K = c > 0.0 ? (L - 1) / (2.0 * c) : 0.0;
        QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&lev), sizeof(double) * L, st));
        QIHT_HIP(hipMemcpyAsync(lev, h.data(), sizeof(double) * L, hipMemcpyHostToDevice, st));
    }
    s0 = launch_quantize_vector(y, dtype, m, bits, levels, seed, c, K, lev, yhat_out, codes_out, st);
    if (lev) (void)hipFreeAsync(lev, st);
    hipError_t e = hipStreamSynchronize(st);
    if (s0 != QIHT_OK) return s0;
    if (e != hipSuccess) return hip_fail(e, "quantize_vector");
    if (scale_out) *scale_out = (bits == 32) ? 0.0 : c;
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_qmatrix_info(const qiht_qmatrix* q, int64_t* rows, int64_t* n, int* bits,
                              int* realizations, double* scale, int64_t* col_bytes) {
    if (!q) return fail(QIHT_ERR_INVALID_ARG, "handle is NULL");
    if (rows) *rows = q->rows;
    if (n) *n = q->n;
    if (bits) *bits = (q->bits <= 8) ? q->code_bits : public_bits(q->bits);
    if (realizations) *realizations = q->realizations;
    if (scale) *scale = q->scale;
    if (col_bytes) *col_bytes = q->col_bytes;
    return QIHT_OK;
}

qiht_status qiht_qmatrix_export_codes(const qiht_qmatrix* q, int realization,
                                      void* host_out) try {
    set_error("");
    if (!q || !host_out) return fail(QIHT_ERR_INVALID_ARG, "handle or output is NULL");
    if (realization < 0 || realization > 1) return fail(QIHT_ERR_INVALID_ARG, "realization is 0 or 1");
    const size_t bytes = static_cast<size_t>(q->col_bytes) * static_cast<size_t>(q->n);
    std::vector<uint8_t> packed(bytes);
    QIHT_HIP(hipMemcpy(packed.data(), q->codes[realization], bytes, hipMemcpyDeviceToHost));
    const int64_t rows = q->rows;
    if (q->bits == 32) {
        float* o = static_cast<float*>(host_out);
        for (int64_t j = 0; j < q->n; ++j)
            std::memcpy(o + j * rows, packed.data() + j * q->col_bytes, sizeof(float) * rows);
        return QIHT_OK;
    }
    if (q->bits == kFmtBF16) {  // stored values as floats (exact)
        float* o = static_cast<float*>(host_out);
        for (int64_t j = 0; j < q->n; ++j)
            for (int64_t i = 0; i < rows; ++i) {
                uint16_t h;
                std::memcpy(&h, packed.data() + j * q->col_bytes + 2 * i, 2);
                const uint32_t u = static_cast<uint32_t>(h) << 16;
                std::memcpy(o + j * rows + i, &u, 4);
            }
        return QIHT_OK;
    }
    if (q->bits == kFmtE4M3) {  // the raw E4M3 bytes
        uint8_t* o = static_cast<uint8_t*>(host_out);
        for (int64_t j = 0; j < q->n; ++j)
            std::memcpy(o + j * rows, packed.data() + j * q->col_bytes, rows);
        return QIHT_OK;
    }
    uint8_t* o = static_cast<uint8_t*>(host_out);
    const int b = q->bits;
    const uint32_t mask = (1u << b) - 1u;
    for (int64_t j = 0; j < q->n; ++j) {
        const uint8_t* col = packed.data() + j * q->col_bytes;
        for (int64_t i = 0; i < rows; ++i) {
            const int64_t bit = i * b;
            o[j * rows + i] = static_cast<uint8_t>((col[bit >> 3] >> (bit & 7)) & mask);
        }
    }
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_qmatrix_row_exponents(const qiht_qmatrix* q, int32_t* host_out) try {
    set_error("");
    if (!q || !host_out) return fail(QIHT_ERR_INVALID_ARG, "handle or output is NULL");
    if (!q->rexp) return fail(QIHT_ERR_INVALID_ARG, "not a dense-format matrix");
    QIHT_HIP(hipMemcpy(host_out, q->rexp, sizeof(int32_t) * q->rows, hipMemcpyDeviceToHost));
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

void qiht_qmatrix_free(qiht_qmatrix* q) {
    if (!q) return;
    if (q->embedded) qiht_qmatrix_free(q->embedded);
    if (q->codes[0]) {
        if (q->pooled) {
            // like hipFree: wait for all work on the device, then hand the
            // codes back to the pool (kept for the next handle)
            (void)hipDeviceSynchronize();
            (void)hipFreeAsync(q->codes[0], nullptr);
            (void)hipStreamSynchronize(nullptr);
        } else {
            (void)hipFree(q->codes[0]);
        }
    }
    delete q;
}

qiht_status qiht_niht_solve(const qiht_qmatrix* q, const double* yhat, int64_t s,
                            const qiht_params* p, float* x_out, int32_t* support_out,
                            qiht_info* info, void* stream) try {
    set_error("");
    qiht_status s0 = check_params(p);
    if (s0 != QIHT_OK) return s0;
    s0 = check_problem(q, yhat, s, x_out, support_out);
    if (s0 != QIHT_OK) return s0;
    int dev = 0;
    s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    if (p->support0) {
        s0 = check_support(p->support0, s, q->n, static_cast<hipStream_t>(stream));
        if (s0 != QIHT_OK) return s0;
    }
    ProblemIn in{q, yhat, s, x_out, support_out, p->x0, p->support0};
    qiht_info tmp;
    s0 = run_solve(&in, 1, to_args(p), &tmp, static_cast<hipStream_t>(stream));
    if (s0 != QIHT_OK) return s0;
    if (p->refit) {
        s0 = run_refit(codes_refit(q, yhat, support_out, s, x_out), static_cast<hipStream_t>(stream));
        if (s0 != QIHT_OK) return s0;
    }
    if (info) *info = tmp;
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_niht_solve_complex(const qiht_qmatrix* q, const double* yhat, int64_t s,
                                    const qiht_params* p, float* x_out, int32_t* support_out,
                                    qiht_info* info, void* stream) try {
    set_error("");
    qiht_status s0 = check_params(p);
    if (s0 != QIHT_OK) return s0;
    if (!q) return fail(QIHT_ERR_INVALID_ARG, "quantized matrix is NULL");
    if (!yhat) return fail(QIHT_ERR_INVALID_ARG, "yhat is NULL");
    if (!x_out || !support_out) return fail(QIHT_ERR_INVALID_ARG, "output pointer is NULL");
    if (q->rows != 2 * q->m)
        return fail(QIHT_ERR_INVALID_ARG, "the matrix was not quantized from complex input");
    if (is_dense_format(q->bits)) return fail(QIHT_ERR_UNSUPPORTED, "complex unknowns need packed codes or FP32");
    if (p->x0 || p->support0) return fail(QIHT_ERR_UNSUPPORTED, "no warm start for a complex unknown");
    if (s < 1 || s > q->m || s > q->n) return fail(QIHT_ERR_INVALID_ARG, "need 1 <= s <= min(m, n)");
    if (q->n > QIHT_COMPLEX_MAX_N)
        return fail(QIHT_ERR_UNSUPPORTED, "n above QIHT_COMPLEX_MAX_N for a complex unknown");
    int dev = 0;
    s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    return run_solve_complex(const_cast<qiht_qmatrix*>(q), yhat, s, to_args(p), p->refit, x_out, support_out,
                             info, static_cast<hipStream_t>(stream));
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_niht_solve_noalloc(const qiht_qmatrix* q, const double* yhat, int64_t s,
                                    const qiht_params* p, float* x_out, int32_t* support_out,
                                    qiht_info* info, void* stream) try {
    set_error("");
    qiht_status s0 = check_params(p);
    if (s0 != QIHT_OK) return s0;
    if (p->profile) return fail(QIHT_ERR_UNSUPPORTED, "no profiling without allocation (events)");
    if (p->refit) return fail(QIHT_ERR_UNSUPPORTED, "no refit without allocation (its workspace)");
    s0 = check_problem(q, yhat, s, x_out, support_out);
    if (s0 != QIHT_OK) return s0;
    int dev = 0;
    s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    if (p->support0) {
        s0 = check_support(p->support0, s, q->n, static_cast<hipStream_t>(stream));
        if (s0 != QIHT_OK) return s0;
    }
    ProblemIn in{q, yhat, s, x_out, support_out, p->x0, p->support0};
    qiht_info tmp;
    s0 = run_solve_noalloc(in, to_args(p), &tmp, static_cast<hipStream_t>(stream));
    if (s0 != QIHT_OK) return s0;
    if (info) *info = tmp;
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_niht_solve_fresh(const void* phi, int64_t m, int64_t n, int64_t ld,
                                  qiht_dtype dtype, int bits, const void* y,
                                  qiht_dtype ydtype, int ybits, uint64_t seed, int64_t s,
                                  const qiht_params* p, float* x_out,
                                  int32_t* support_out, qiht_info* info, void* stream) try {
    set_error("");
    if (!phi || !y || !x_out || !support_out) return fail(QIHT_ERR_INVALID_ARG, "NULL argument");
    qiht_status s0 = check_params(p);
    if (s0 != QIHT_OK) return s0;
    if (p->x0 || p->support0) return fail(QIHT_ERR_INVALID_ARG, "no warm start with per-iteration draws");
    if (p->refit) return fail(QIHT_ERR_UNSUPPORTED, "no refit with per-iteration draws");
    if (!dtype_ok(dtype) || !dtype_ok(ydtype)) return fail(QIHT_ERR_UNSUPPORTED, "unknown dtype");
    if (is_complex(dtype) != is_complex(ydtype))
        return fail(QIHT_ERR_INVALID_ARG, "y must be complex exactly when Phi is");
    const int pbits = bits & ~QIHT_ODD_LEVELS;
    if (!((pbits >= 1 && pbits <= 8) || pbits == 32))
        return fail(QIHT_ERR_UNSUPPORTED, "bits must be 1..8 or 32 (packed codes)");
    const bool yodd = (ybits & QIHT_ODD_LEVELS) != 0;
    const int yb = ybits & ~QIHT_ODD_LEVELS;
    if (!bits_ok_vector(yb) || (yodd && (yb < 2 || yb > 12)))
        return fail(QIHT_ERR_UNSUPPORTED, "ybits must be 1..12 or 32 (odd levels: 2..12)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // iteration 1's draws (matrix realizations 0 and 1, y_hat realization 0),
    // through the ordinary entry points; they validate the rest
    qiht_qmatrix* q = nullptr;
    s0 = qiht_quantize_matrix(phi, m, n, ld, dtype, bits, 2, seed, stream, &q);
    if (s0 != QIHT_OK) return s0;
    const int64_t rows = q->rows;
    double* yhat = nullptr;
    double* ylev = nullptr;
    const int ylevels = (yb == 32) ? 0 : num_levels(yb, yodd);
    auto cleanup = [&]() {
        if (yhat) (void)hipFree(yhat);
        if (ylev) (void)hipFree(ylev);
        qiht_qmatrix_free(q);
    };
    if (dev_malloc(reinterpret_cast<void**>(&yhat), sizeof(double) * rows) != hipSuccess ||
        (ylevels && dev_malloc(reinterpret_cast<void**>(&ylev), sizeof(double) * ylevels) != hipSuccess)) {
        (void)hipGetLastError();
        cleanup();
        return fail(QIHT_ERR_OUT_OF_MEMORY, "y_hat allocation failed");
    }
    double yc = 0.0;
    s0 = qiht_quantize_vector(y, m, ydtype, ybits, seed, stream, yhat, nullptr, &yc);
    if (s0 == QIHT_OK) s0 = check_problem(q, yhat, s, x_out, support_out);
    if (s0 != QIHT_OK) {
        const std::string why = last_error_cstr();
        cleanup();
        return fail(s0, why);
    }
    if (ylevels) {
        std::vector<double> h(ylevels);
        for (int k = 0; k < ylevels; ++k) h[k] = yc * (2.0 * k / static_cast<double>(ylevels - 1) - 1.0);
        if (hipMemcpy(ylev, h.data(), sizeof(double) * ylevels, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            return fail(QIHT_ERR_DEVICE, "level table copy failed");
        }
    }
    FreshSource f{};
    f.phi = phi;
    f.dtype = dtype;
    f.m = m;
    f.n = n;
    f.ld = ld;
    f.bits = q->bits;
    f.levels = q->levels;
    f.seed = seed;
    f.c = q->scale;
    f.K = (q->bits == 32 || f.c == 0.0) ? 0.0 : (f.levels - 1) / (2.0 * f.c);
    f.q = q;
    f.y = y;
    f.ydtype = ydtype;
    f.ybits = yb;
    f.ylevels = ylevels;
    f.yc = yc;
    f.yK = (ylevels && yc > 0.0) ? (ylevels - 1) / (2.0 * yc) : 0.0;
    f.ylev = ylev;
    f.yhat = yhat;
    ProblemIn in{q, yhat, s, x_out, support_out, nullptr, nullptr};
    qiht_info tmp;
    s0 = run_solve(&in, 1, to_args(p), &tmp, st, &f);
    const hipError_t e = hipStreamSynchronize(st);
    cleanup();
    if (s0 != QIHT_OK) return s0;
    if (e != hipSuccess) return hip_fail(e, "solve_fresh");
    if (info) *info = tmp;
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_niht_solve_batched(int32_t count, const qiht_problem* probs,
                                    const qiht_params* p, qiht_info* infos,
                                    void* stream) try {
    set_error("");
    if (count < 1 || !probs) return fail(QIHT_ERR_INVALID_ARG, "empty batch");
    qiht_status s0 = check_params(p);
    if (s0 != QIHT_OK) return s0;
    if (p->x0) return fail(QIHT_ERR_INVALID_ARG, "warm start is not supported in a batch");
    std::vector<ProblemIn> in(count);
    for (int i = 0; i < count; ++i) {
        s0 = check_problem(probs[i].q, probs[i].yhat, probs[i].s, probs[i].x_out,
                           probs[i].support_out);
        if (s0 != QIHT_OK) return fail(s0, "problem " + std::to_string(i) + ": " + last_error_cstr());
        if (probs[i].q->bits != probs[0].q->bits)
            return fail(QIHT_ERR_UNSUPPORTED, "problems of a batch must share the bit width");
        in[i] = ProblemIn{probs[i].q, probs[i].yhat, probs[i].s, probs[i].x_out,
                          probs[i].support_out, nullptr, nullptr};
    }
    int dev = 0;
    s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    std::vector<qiht_info> tmp(count);
    s0 = run_solve(in.data(), count, to_args(p), tmp.data(), static_cast<hipStream_t>(stream));
    if (s0 != QIHT_OK) return s0;
    if (p->refit) {
        std::vector<RefitIn> rin(count);
        for (int i = 0; i < count; ++i)
            rin[i] = codes_refit(probs[i].q, probs[i].yhat, probs[i].support_out, probs[i].s,
                                 probs[i].x_out);
        s0 = run_refit_batch(rin.data(), count, static_cast<hipStream_t>(stream));
        if (s0 != QIHT_OK) return s0;
    }
    if (infos) std::memcpy(infos, tmp.data(), sizeof(qiht_info) * count);
    return QIHT_OK;
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_gradient(const qiht_qmatrix* q, const double* yhat, const float* x,
                          const int32_t* support, int64_t s, float* g_out, float* r_out,
                          void* stream) try {
    set_error("");
    if (!q || !yhat || !g_out) return fail(QIHT_ERR_INVALID_ARG, "NULL argument");
    if (s < 0 || s > q->n) return fail(QIHT_ERR_INVALID_ARG, "need 0 <= s <= n");
    if (s > 0 && (!x || !support)) return fail(QIHT_ERR_INVALID_ARG, "x and support needed for s > 0");
    int dev = 0;
    qiht_status s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    s0 = check_support(support, s, q->n, static_cast<hipStream_t>(stream));
    if (s0 != QIHT_OK) return s0;
    return run_gradient(q, yhat, x, support, s, g_out, r_out, static_cast<hipStream_t>(stream));
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_hard_threshold(const float* a, int64_t n, int64_t s, int32_t* support_out,
                                void* stream) try {
    set_error("");
    if (!a || (!support_out && s > 0)) return fail(QIHT_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || s < 0 || s > n) return fail(QIHT_ERR_INVALID_ARG, "need n >= 1, 0 <= s <= n");
    if (s == 0) return QIHT_OK;
    int dev = 0;
    qiht_status s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    return run_hard_threshold(a, n, s, support_out, static_cast<hipStream_t>(stream));
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_fourier_gradient(const double* uv, int64_t n_vis, int64_t side, const float* r,
                                  float* g_out, void* stream) try {
    set_error("");
    if (!uv || !r || !g_out) return fail(QIHT_ERR_INVALID_ARG, "NULL argument");
    if (n_vis < 1 || n_vis > QIHT_FOURIER_MAX_VIS)
        return fail(QIHT_ERR_INVALID_ARG, "need 1 <= n_vis <= QIHT_FOURIER_MAX_VIS");
    if (side < 1 || side > QIHT_FOURIER_MAX_SIDE)
        return fail(QIHT_ERR_INVALID_ARG, "need 1 <= side <= QIHT_FOURIER_MAX_SIDE");
    int dev = 0;
    qiht_status s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    return run_fourier_gradient(uv, n_vis, static_cast<int>(side), r, g_out, static_cast<hipStream_t>(stream));
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_fourier_niht_solve(const double* uv, int64_t n_vis, int64_t side, const double* y, int64_t s,
                                    const qiht_params* p, float* x_out, int32_t* support_out, qiht_info* info,
                                    void* stream) try {
    set_error("");
    if (!uv || !y || !x_out || !support_out) return fail(QIHT_ERR_INVALID_ARG, "NULL argument");
    if (n_vis < 1 || n_vis > QIHT_FOURIER_MAX_VIS)
        return fail(QIHT_ERR_INVALID_ARG, "need 1 <= n_vis <= QIHT_FOURIER_MAX_VIS");
    if (side < 1 || side > QIHT_FOURIER_MAX_SIDE)
        return fail(QIHT_ERR_INVALID_ARG, "need 1 <= side <= QIHT_FOURIER_MAX_SIDE");
    if (s < 1 || s > std::min<int64_t>(2 * n_vis, side * side))
        return fail(QIHT_ERR_INVALID_ARG, "need 1 <= s <= min(2 n_vis, side^2)");
    if (side * side > QIHT_FOURIER_SOLVE_MAX_PIXELS)
        return fail(QIHT_ERR_UNSUPPORTED, "the solve takes at most QIHT_FOURIER_SOLVE_MAX_PIXELS pixels");
    qiht_status s0 = check_params(p);
    if (s0 != QIHT_OK) return s0;
    if (p->x0 || p->support0) return fail(QIHT_ERR_UNSUPPORTED, "no warm start with Phi on the fly");
    if (p->refit) return fail(QIHT_ERR_UNSUPPORTED, "no refit with Phi on the fly");
    int dev = 0;
    s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    return run_fourier_solve(uv, n_vis, static_cast<int>(side), y, s, *p, x_out, support_out, info,
                             static_cast<hipStream_t>(stream));
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

qiht_status qiht_refit(const qiht_qmatrix* q, const void* phi, int64_t m, int64_t n, int64_t ld,
                       qiht_dtype dtype, const double* y, const int32_t* support, int64_t s,
                       float* x_out, double* xs_out, void* stream) try {
    set_error("");
    if (!y || !support || !x_out) return fail(QIHT_ERR_INVALID_ARG, "NULL argument");
    RefitIn r{};
    if (phi) {
        if (m < 1 || n < 1 || ld < n) return fail(QIHT_ERR_INVALID_ARG, "need m, n >= 1 and ld >= n");
        if (dtype != QIHT_F32 && dtype != QIHT_F64 && dtype != QIHT_C64 && dtype != QIHT_C128)
            return fail(QIHT_ERR_UNSUPPORTED, "dtype");
        const bool cplx = dtype == QIHT_C64 || dtype == QIHT_C128;
        r.phi = phi;
        r.m = m;
        r.ld = ld;
        r.dtype = dtype;
        r.rows = cplx ? 2 * m : m;
        r.n = n;
    } else {
        if (!q) return fail(QIHT_ERR_INVALID_ARG, "need phi or a quantized matrix");
        r = codes_refit(q, y, support, s, x_out);
    }
    if (s < 1 || s > std::min(r.rows, r.n)) return fail(QIHT_ERR_INVALID_ARG, "need 1 <= s <= min(rows, n)");
    r.s = s;
    r.y = y;
    r.sup = support;
    r.x_out = x_out;
    r.xs_out = xs_out;
    int dev = 0;
    qiht_status s0 = need_device(&dev);
    if (s0 != QIHT_OK) return s0;
    s0 = check_support(support, s, r.n, static_cast<hipStream_t>(stream));
    if (s0 != QIHT_OK) return s0;
    return run_refit(r, static_cast<hipStream_t>(stream));
} catch (...) {
    return fail(QIHT_ERR_DEVICE, "unexpected exception");
}

}  // extern "C"
