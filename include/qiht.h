/*
 * qiht.h -- C ABI of the MI355X (gfx950) hot path of low-precision
 * normalized Iterative Hard Thresholding (QIHT).
 *
 * Method: N. M. Guerel, K. Kara, A. Stojanov, T. Smith, T. Lemmin,
 * D. Alistarh, M. Pueschel, C. Zhang, "Compressive Sensing Using Iterative
 * Hard Thresholding with Low Precision Data Representation: Theory and
 * Applications", IEEE Trans. Signal Process. 68 (2020), arXiv:1802.04907.
 *
 * Problem (Sec. I-A, Eq. CS_model and Eq. cost_function): given y = Phi x + e
 * with Phi an M x N real or complex matrix, find x minimizing
 * |y - Phi x|^2 subject to |x|_0 <= s.  QIHT (Sec. III-A, Algorithm 2)
 * runs normalized IHT (Algorithm 1) on stochastically quantized copies of
 * Phi and y: x+ = H_s(x + mu Q1^T (y_hat - Q2 x)) with two independent
 * quantizations Q1, Q2 of Phi ("double sampling").
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Array arguments are DEVICE pointers (memory of the current HIP device)
 *    unless marked "host".  The caller owns every buffer it passes; a
 *    qiht_qmatrix owns the device codes it holds until qiht_qmatrix_free.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is ordered on that stream.  Entry points that return results in
 *    host memory (qiht_info, scales) synchronize that stream before
 *    returning.
 *  - Every entry point validates its arguments on the host before touching
 *    the device.  On any error it returns a non-zero qiht_status, leaves
 *    the caller's outputs untouched, and stores a message retrievable with
 *    qiht_last_error() (thread-local).  No C++ exception crosses the ABI.
 *  - Not thread-safe on one qiht_qmatrix; distinct handles may be used
 *    from distinct threads.
 *  - Per-call workspaces are allocated stream-ordered from a memory pool the
 *    library creates per device; the pool keeps freed memory for reuse (it
 *    grows to the largest workspace in use at once) until the process ends.
 *  - Environment: QIHT_PASS_STREAM=cache or =long pins which instance of the
 *    full pass g = Q1^T r runs (one tuned for codes that stay in the
 *    Infinity Cache between passes, one for longer streams from HBM); by
 *    default the codes' total size picks it.  Both are valid for every
 *    problem and give the same g bit for bit; only the speed differs.
 *    QIHT_FAIL_ALLOC_AFTER=N (tests of the error paths): N more device
 *    allocations of the library succeed, every later one fails as if the
 *    device were out of memory (the call returns QIHT_ERR_OUT_OF_MEMORY);
 *    the count starts again whenever the value changes, and unsetting it
 *    ends the injection.
 */
#ifndef QIHT_H_
#define QIHT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QIHT_OK = 0,
    QIHT_ERR_INVALID_ARG = 1,   /* bad size, null pointer, s out of range */
    QIHT_ERR_UNSUPPORTED = 2,   /* bit width or dtype not implemented      */
    QIHT_ERR_OUT_OF_MEMORY = 3, /* device allocation failed                */
    QIHT_ERR_DEVICE = 4,        /* no usable device, or a HIP call failed  */
    QIHT_ERR_NUMERIC = 5        /* NaN or Inf in the input data           */
} qiht_status;

typedef enum {
    QIHT_F64 = 0,   /* double                                   */
    QIHT_F32 = 1,   /* float                                    */
    QIHT_C64 = 2,   /* complex float, interleaved (re, im)      */
    QIHT_C128 = 3,  /* complex double, interleaved (re, im)     */
    /* range markers, not dtypes: they make every 32-bit int a value of the
     * type, so that an unknown value passed in is rejected (UNSUPPORTED)
     * rather than being undefined on the C++ side */
    QIHT_DTYPE_MIN_ = -2147483647 - 1,
    QIHT_DTYPE_MAX_ = 2147483647
} qiht_dtype;

/* Why a solve stopped (qiht_info.reason). */
enum {
    QIHT_REASON_CONVERGED = 1,  /* |x^n - x^(n-1)| <= tol |x^n|            */
    QIHT_REASON_MAX_ITERS = 2,  /* iteration cap reached                    */
    QIHT_REASON_STATIONARY = 3  /* gradient vanished on the support         */
};

/* Opaque quantized measurement matrix: packed codes of one or two
 * realizations plus the max-abs scale. */
typedef struct qiht_qmatrix qiht_qmatrix;

/*
 * Solver parameters.  Algorithm 2 inputs: iteration count n* (max_iters),
 * the step-size tuning parameters k and c (Sec. II-A: on a support change
 * the step must satisfy mu <= (1 - c)|dx|^2/|Phi dx|^2, otherwise
 * mu <- mu / (k (1 - c)), with k > 1/(1 - c)).
 */
typedef struct {
    int32_t max_iters;       /* n*; >= 1                                    */
    double tol;              /* stop when |x^n - x^(n-1)| <= tol |x^n|;
                                tol < 0 disables the test (the paper gives
                                only n*); tol = 0 stops at an exact fixed
                                point                                       */
    double k;                /* shrink parameter, k > 1/(1-c); default 2    */
    double c;                /* step test margin, 0 <= c < 1; default 0.01  */
    int32_t max_backtracks;  /* shrinks per iteration (>= 0); default 32    */
    int32_t mu_mode;         /* 0: mu = |g_G|^2/((Q1_G g_G).(Q2_G g_G))
                                   (Algorithm 2); 1: |g_G|^2/|Q1_G g_G|^2   */
    const float* x0;         /* optional warm start x (device, n floats);
                                NULL = x0 = 0 and G0 = supp H_s(Q1^T y_hat) */
    const int32_t* support0; /* warm-start support (device, s ascending
                                indices); required iff x0 != NULL           */
    int32_t profile;         /* N >= 1: time the full-pass launch of the
                                first round of every N-th chunk of 16
                                rounds with HIP events recorded by the
                                dispatch on `stream` (that round is
                                launched directly, the rest of the chunk
                                may replay as a captured HIP graph;
                                qiht_info.pass_ms and pass_launches cover
                                the timed launches; each timed dispatch
                                costs a few microseconds of extra
                                latency); 0: off                           */
    int32_t refit;           /* 1: after the last iteration, replace x on
                                its support by the FP64 least-squares fit
                                against Q1 and y_hat (qiht_refit); 0 keeps
                                the last iterate (the paper's output)      */
} qiht_params;

typedef struct {
    int32_t iterations;        /* completed iterations                       */
    int32_t reason;            /* QIHT_REASON_*                              */
    int32_t backtracks;        /* total step shrinks                         */
    int32_t capped_iterations; /* iterations that hit max_backtracks         */
    double mu_last;            /* accepted step of the last iteration        */
    double pass_ms;            /* profile = 1: summed event time of the
                                  g = Q1^T r launches (0 otherwise); in a
                                  batch every problem reports the batch's
                                  launches (one GEMM per iteration when the
                                  problems share one matrix)                 */
    int32_t pass_launches;     /* number of those launches                   */
    int32_t full_selects;      /* H_s proposals that ranked all n entries
                                  (the rest ranked the histogram candidates) */
} qiht_info;

/* Fill `p` (host) with the defaults: max_iters 300, tol 1e-8, k 2, c 0.01,
 * max_backtracks 32, mu_mode 0, no warm start, profile 0, refit 0. */
void qiht_default_params(qiht_params* p);

/* OR'd into the bit width of qiht_quantize_matrix (2, 4 or 8 bits) or
 * qiht_quantize_vector (2..12 bits): the odd level set of the Remark on
 * fixed-point hardware in the appendix (after the Lemma on the quantized
 * vector): 2^(b-1) + 1 levels q_k = -1 + k / 2^(b-2), spacing 1 / 2^(b-2),
 * codes 0 .. 2^(b-1) stored in the same b bits; same rounding rule and
 * random stream.  The solver works on such handles unchanged. */
#define QIHT_ODD_LEVELS 0x100

/* Dense storage formats accepted by qiht_quantize_matrix in place of a bit
 * width (deterministic rounding, no randomness; not in the paper). */
#define QIHT_FMT_BF16 116  /* bfloat16: 8 exponent, 7 stored significand bits */
#define QIHT_FMT_E4M3 108  /* OCP FP8 E4M3: bias 7, 3 significand bits, max 448 */

/*
 * Quantize the measurement matrix: Q(Phi, b) of Sec. III-A.
 *
 *   Phi is M x N, row-major with leading dimension ld >= N (elements), on
 *   the device, of dtype F32, F64, C64 or C128.  Complex input is treated
 *   as the real matrix [Re Phi; Im Phi] of 2M rows (real unknown x).
 *   The scale c = max |Phi_ij| over the (stacked) matrix; values are mapped
 *   to [-1, 1] by 1/c and rounded at random to one of the two neighbouring
 *   levels q_k = -1 + 2k/(2^b - 1), up with probability equal to the
 *   fractional position (unbiased: E[Q(v)] = v).
 *
 *   bits: 1..8 (packed codes; 2..8 may carry QIHT_ODD_LEVELS; a b-bit
 *   code occupies a field of 1, 2, 4 or 8 bits: 3 -> 4 and 5..7 -> 8, so
 *   that a byte holds whole codes: a 3-bit matrix takes the memory and the
 *   full-pass bandwidth of a 4-bit one, 5 to 7 bits those of 8; the solver
 *   reads every width alike), or 32 (plain FP32 copy, no
 *   randomness; realizations is then forced to 1 and Q1 = Q2), or a dense
 *   format QIHT_FMT_BF16 / QIHT_FMT_E4M3: row i is stored as
 *   Phi_ij / 2^e_i rounded to nearest (ties to even significand), e_i the
 *   smallest integer with max_j |Phi_ij| / 2^e_i <= 1 (BF16) or 448 (E4M3),
 *   so the matrix the solver uses is diag(2^e) times the stored values; one
 *   copy (Q1 = Q2), realizations and seed are ignored.  Solves on such a
 *   handle run the shared-matrix path (one MFMA GEMM per iteration for all
 *   right-hand sides of a batch; see qiht_niht_solve_batched).
 *   realizations: 1 (Q1 = Q2, single sampling) or 2 (independent Q1 for
 *   Phi^T and Q2 for Phi: double sampling, Sec. III-A).
 *   seed: 64-bit Philox4x32-10 key.  Element e (column-major index over
 *   the stacked rows) of realization r draws word e & 3 of the block with
 *   counter (e >> 2, stream 0, r); code = i + [u < f 2^32] with
 *   p = (v + c)(2^b - 1)/(2c) in FP64, i = floor(p) clamped to
 *   [0, 2^b - 2], f = p - i.
 *
 *   *out receives a new handle (free with qiht_qmatrix_free).  Errors:
 *   INVALID_ARG (null, m/n < 1, ld < n), UNSUPPORTED (bits/dtype),
 *   NUMERIC (NaN/Inf in Phi), OUT_OF_MEMORY, DEVICE.  Synchronizes stream.
 */
qiht_status qiht_quantize_matrix(const void* phi, int64_t m, int64_t n,
                                 int64_t ld, qiht_dtype dtype, int bits,
                                 int realizations, uint64_t seed,
                                 void* stream, qiht_qmatrix** out);

/*
 * Quantize the observation vector: Q(y, b) of Sec. III-A, one realization
 * on Philox stream 1 (counter (e >> 2, 1, 0)), same rounding rule as the
 * matrix.  y has m entries of dtype F32/F64 (real) or C64/C128 (complex,
 * stacked [Re y; Im y], 2m rows) on the device.
 *
 *   yhat_out (device, rows doubles): the dequantized FP64 values
 *            c (2k/(2^b - 1) - 1); for bits = 32 the FP32-rounded y.
 *   codes_out (device, rows bytes, optional, bits <= 8): the codes.
 *   scale_out (host, optional): the scale c (0 for bits = 32).
 *   bits: 1..12 or 32, optionally | QIHT_ODD_LEVELS (2..12 bits; levels
 *   c (k / 2^(b-2) - 1)).  Synchronizes stream.
 */
qiht_status qiht_quantize_vector(const void* y, int64_t m, qiht_dtype dtype,
                                 int bits, uint64_t seed, void* stream,
                                 double* yhat_out, uint8_t* codes_out,
                                 double* scale_out);

/*
 * Shape of a quantized matrix (host outputs, each optional): stacked row
 * count, column count, bit width b of the codes (as requested, without
 * QIHT_ODD_LEVELS; 32 or the dense format otherwise), realizations, scale c,
 * and the byte stride between packed columns in device memory.
 */
qiht_status qiht_qmatrix_info(const qiht_qmatrix* q, int64_t* rows,
                              int64_t* n, int* bits, int* realizations,
                              double* scale, int64_t* col_bytes);

/*
 * Copy one realization's codes to host memory, unpacked: rows x n bytes,
 * column-major (byte j*rows + i is the code of element (i, j)).  For
 * bits = 32 and QIHT_FMT_BF16 the buffer receives rows x n floats instead
 * (the stored values), for QIHT_FMT_E4M3 the rows x n E4M3 bytes.  For
 * inspection and tests; the device layout is private.
 */
qiht_status qiht_qmatrix_export_codes(const qiht_qmatrix* q, int realization,
                                      void* host_out);

/*
 * Row exponents e_i of a dense-format handle (host, rows int32): the matrix
 * is diag(2^e) times the stored values.  INVALID_ARG for packed codes.
 */
qiht_status qiht_qmatrix_row_exponents(const qiht_qmatrix* q, int32_t* host_out);

/* Release a handle (NULL is a no-op). */
void qiht_qmatrix_free(qiht_qmatrix* q);

/*
 * Solve one instance with QIHT (Algorithm 2 on the fixed realizations held
 * by q; Algorithm 1 when q has bits = 32).  Per iteration, on the GPU:
 *   r = y_hat - Q2_G x_G           (FP64 gather over the s support columns)
 *   g = Q1^T r                     (full pass over the packed codes, FP32)
 *   mu = |g_G|^2/((Q1_G g_G).(Q2_G g_G))          (Eq. step_size, FP64)
 *   x' = H_s(x + mu g)             (top-s, ties to the lower index)
 *   if supp x' != G: backtrack while mu > (1-c)|dx|^2/|Q1 dx|^2 (FP64)
 *   stop on tol or max_iters.
 *
 *   yhat: device, rows doubles (from qiht_quantize_vector).
 *   s: 1 <= s <= min(rows, n) (Theorem on QIHT requires s <= M).
 *   x_out: device, n floats, the final x (zero off the support).
 *   support_out: device, s int32, the final support in ascending order.
 *   info: host, optional.  Synchronizes stream.
 */
qiht_status qiht_niht_solve(const qiht_qmatrix* q, const double* yhat,
                            int64_t s, const qiht_params* p, float* x_out,
                            int32_t* support_out, qiht_info* info,
                            void* stream);

/* One problem of a batch. */
typedef struct {
    const qiht_qmatrix* q;
    const double* yhat;      /* device, rows doubles           */
    int64_t s;
    float* x_out;            /* device, n floats               */
    int32_t* support_out;    /* device, s int32                */
} qiht_problem;

/*
 * Solve `count` independent problems of possibly different sizes in one
 * sequence of batched launches (each phase of an iteration is one launch
 * covering every unfinished problem).  Problems must share the bit width.
 * infos: host array of `count` (optional).  Same semantics per problem as
 * qiht_niht_solve; the warm start in p is not supported here (must be
 * NULL).  Synchronizes stream.
 *
 * Shared matrix: when every problem uses the same handle and that handle
 * is a dense format (QIHT_FMT_BF16 / QIHT_FMT_E4M3), or bits = 32 with
 * count > 1, the per-iteration products g_k = A^T r_k of all problems are
 * one GEMM G = A^T R on the matrix cores (FP32 accumulation; BF16 and E4M3
 * storage multiply in BF16 with each r_k carried as two BF16 terms, about
 * 16 significant bits; FP32 storage in FP32), and the column gathers read
 * 256-byte row segments.  Problems on dense-format handles must all share
 * one handle (UNSUPPORTED otherwise).
 */
qiht_status qiht_niht_solve_batched(int32_t count, const qiht_problem* probs,
                                    const qiht_params* p, qiht_info* infos,
                                    void* stream);

/*
 * QIHT with a complex unknown x in C^N (Sec. I-A states the problem for
 * complex Phi and x; the MRI images of Sec. IV are complex).  Algorithm 2 in
 * complex arithmetic: g = Q1^H (y_hat - Q2 x) (^H the conjugate transpose),
 * mu = |g_G|^2 / Re((Q1_G g_G)^H (Q2_G g_G)) (fallback and stop as for
 * qiht_niht_solve), H_s keeping the s entries of largest modulus |x_j| (ties
 * to the lower index; the modulus is ranked as the FP32 rounding of
 * Re^2 + Im^2 taken in FP64 from the FP32 parts), and the step-size test and
 * shrinking of Sec. II-A with the norms of complex vectors.
 *
 *   q: a handle quantized from complex input (dtype C64 or C128 in
 *      qiht_quantize_matrix: Q = Q(Re Phi) + i Q(Im Phi), stacked rows
 *      [Re; Im]); packed codes (1..8 bits, odd levels too) or 32.
 *      INVALID_ARG for a handle of real input, UNSUPPORTED for a dense format.
 *   yhat: device, 2m doubles [Re y_hat; Im y_hat] (qiht_quantize_vector of
 *      the complex y).
 *   1 <= s <= min(m, n); n <= QIHT_COMPLEX_MAX_N (UNSUPPORTED above).
 *   x_out: device, 2n floats: [Re x; Im x].  support_out: device, s int32,
 *      ascending.  p: as qiht_niht_solve; no warm start (UNSUPPORTED); with
 *      refit = 1 the final x is the FP64 least-squares fit on its support
 *      against Q1 and y_hat (complex least squares).
 * The solve runs the real kernels on the embedding [Q_re -Q_im; Q_im Q_re]
 * of 2m x 2n (its codes are built on the first complex solve on q, from q's,
 * and kept with q until qiht_qmatrix_free: twice q's code memory), with H_s
 * ranking moduli over the pairs of columns (j, j + n).  Synchronizes stream.
 */
#define QIHT_COMPLEX_MAX_N 131072LL
qiht_status qiht_niht_solve_complex(const qiht_qmatrix* q, const double* yhat,
                                    int64_t s, const qiht_params* p,
                                    float* x_out, int32_t* support_out,
                                    qiht_info* info, void* stream);

/*
 * For callers that cannot allocate device memory (code that runs while a HIP
 * graph is being captured elsewhere in the process, tight serving loops,
 * harnesses that forbid hipMalloc): the solve of qiht_niht_solve, whose
 * per-call workspace (residual, gradient, iterate, proposals, candidate
 * lists, partial sums, control state) lives in a fixed device array of
 * QIHT_NOALLOC_WORKSPACE_BYTES bytes instead of memory from the library's
 * pool.  Each device the library runs on holds its own copy of the array
 * until the process ends.  The call allocates and frees no device memory.
 *
 *   Arguments, outputs, results and errors as qiht_niht_solve (the same
 *   kernels run, so results are bitwise those of qiht_niht_solve), and:
 *   p->profile and p->refit must be 0 (UNSUPPORTED: profiling needs events,
 *   the refit its own workspace).  A problem whose workspace exceeds the
 *   array returns UNSUPPORTED before any device work, with the size it needs
 *   in qiht_last_error() (about 24 n bytes, 4 n more per extra row slab of
 *   the full pass, plus 8 bytes per row: 1 MB for 8192 x 32768 at 4 bits,
 *   about 3 MB for 65280 x 16384).
 *   The array keeps the last call's contents; each call clears what must
 *   start at zero.  All calls on one device share the array: the library
 *   runs the calls of one process on one device one after another (each
 *   holds the array until it has synchronized its stream).  Synchronizes
 *   stream.
 */
#define QIHT_NOALLOC_WORKSPACE_BYTES (16LL << 20)
qiht_status qiht_niht_solve_noalloc(const qiht_qmatrix* q, const double* yhat,
                                    int64_t s, const qiht_params* p,
                                    float* x_out, int32_t* support_out,
                                    qiht_info* info, void* stream);

/*
 * Algorithm 2 with its realizations drawn per iteration, as its input lists
 * them: 2n* realizations of Q(Phi) and n* of Q(y).  Iteration n uses
 * Phi_hat_{2n-1} for Phi^T and Phi_hat_{2n} for Phi (matrix realizations
 * 2n-2 and 2n-1 on the counter of qiht_quantize_matrix) and y_hat_n (vector
 * realization n-1: counter (e >> 2, 1, n-1)); the initial support uses
 * Phi_hat_1 and y_hat_1.  Backtracking within an iteration reuses its
 * draws.  Each iteration re-quantizes Phi and y on the device (a full read
 * of Phi per iteration).
 *
 *   phi: as qiht_quantize_matrix (M x N, row-major, ld, dtype); bits 1, 2,
 *        4, 8 (optionally | QIHT_ODD_LEVELS) or 32.
 *   y:   M entries of ydtype (complex exactly when dtype is); ybits as
 *        qiht_quantize_vector.  Both arrays are read by every iteration and
 *        must stay valid until the call returns.
 *   seed, s, p, x_out, support_out, info: as qiht_niht_solve (no warm start,
 *        no refit: INVALID_ARG / UNSUPPORTED).  Synchronizes stream.
 */
qiht_status qiht_niht_solve_fresh(const void* phi, int64_t m, int64_t n, int64_t ld,
                                  qiht_dtype dtype, int bits, const void* y,
                                  qiht_dtype ydtype, int ybits, uint64_t seed, int64_t s,
                                  const qiht_params* p, float* x_out,
                                  int32_t* support_out, qiht_info* info, void* stream);

/*
 * One evaluation of the gradient pair at a given sparse x:
 *   r = y_hat - Q2_G x_G (FP64 accumulation, rounded to FP32 for the pass)
 *   g = Q1^T r (FP32)
 * x: device, n floats, zero outside `support` (device, s int32 ascending).
 * g_out: device, n floats.  r_out: device, rows floats (optional).
 * This is the dense pair of Algorithm 2's first line, exposed for parity
 * tests and profiling.
 */
qiht_status qiht_gradient(const qiht_qmatrix* q, const double* yhat,
                          const float* x, const int32_t* support, int64_t s,
                          float* g_out, float* r_out, void* stream);

/*
 * Gradient of a Fourier-sampled measurement matrix computed on the fly
 * (Sec. IV-C), with no matrix in memory.  The matrix is the radio
 * interferometry model of Sec. IV-B: visibility j at baseline (u_j, v_j)
 * samples pixel k of a side x side sky at integer coordinates
 *   l_k = (k mod side) - floor(side/2),  m_k = (k div side) - floor(side/2),
 *   Phi_jk = exp(-2 pi i (u_j l_k + v_j m_k)),
 * taken in the stacked real form [Re Phi; Im Phi] (2 n_vis rows), so
 *   g_k = sum_j cos(2 pi th_jk) r_j - sin(2 pi th_jk) r_{n_vis + j},
 *   th_jk = u_j l_k + v_j m_k.
 *   uv: device, n_vis x 2 doubles, row-major (u_j, v_j) in cycles per pixel.
 *   r: device, 2 n_vis floats, stacked [Re; Im].
 *   g_out: device, side * side floats, row-major (index k).
 * Phases are reduced in FP64 to [-1/2, 1/2] turns; the sines and cosines and
 * the products are FP32, and partial sums over blocks of 128 visibilities are
 * added in FP64 in a fixed order (deterministic).  1 <= n_vis <=
 * QIHT_FOURIER_MAX_VIS, 1 <= side <= QIHT_FOURIER_MAX_SIDE, else INVALID_ARG;
 * a stream-ordered workspace of 4 side^2 ceil(n_vis / 128) bytes comes from
 * the library's pool (OUT_OF_MEMORY if it cannot be had).  Non-finite uv or r
 * give non-finite g.  Asynchronous on `stream`.
 */
#define QIHT_FOURIER_MAX_VIS 8388480LL
#define QIHT_FOURIER_MAX_SIDE 4096LL
qiht_status qiht_fourier_gradient(const double* uv, int64_t n_vis, int64_t side,
                                  const float* r, float* g_out, void* stream);

/*
 * Normalized IHT (Algorithm 1; QIHT at b = 32) on that Fourier-sampled Phi
 * with every product by Phi computed on the fly: the full pass as in
 * qiht_fourier_gradient, and Phi times the support's columns (r = y -
 * Phi_G x_G, Phi_G g_G for the step size, Phi (x+ - x) for the step test)
 * by one thread per visibility over the column list, FP64 sums.  Same
 * iteration as qiht_niht_solve with Q1 = Q2 = Phi and y_hat = y: G0 =
 * supp H_s(Phi^T y), mu = |g_G|^2 / |Phi_G g_G|^2 (mu_mode has no effect,
 * the two forms coincide), the backtracking rule with k, c, max_backtracks,
 * the stop rule with tol, max_iters.  State and proposals in FP32 (x, g,
 * x + mu g), norms and the step in FP64.
 *   uv: device, n_vis x 2 doubles (u_j, v_j).
 *   y: device, 2 n_vis doubles, the visibilities stacked [Re; Im].
 *   1 <= s <= min(2 n_vis, side^2); n_vis as for qiht_fourier_gradient;
 *   side^2 <= QIHT_FOURIER_SOLVE_MAX_PIXELS (the H_s selection's limit;
 *   512 x 512, the size of the paper's MRI image), else UNSUPPORTED.  p: as for qiht_niht_solve, without warm start
 *   (x0, support0 must be NULL) or refit (must be 0): UNSUPPORTED.
 *   x_out: device, side^2 floats; support_out: device, s int32 ascending.
 * Reads two or three status words per iteration back to the host (the next
 * launches depend on them).  Synchronizes stream.
 */
#define QIHT_FOURIER_SOLVE_MAX_PIXELS 262144LL
qiht_status qiht_fourier_niht_solve(const double* uv, int64_t n_vis, int64_t side,
                                    const double* y, int64_t s, const qiht_params* p,
                                    float* x_out, int32_t* support_out, qiht_info* info,
                                    void* stream);

/*
 * H_s selection alone (Sec. I-A): the indices of the s entries of a
 * (device, n floats) largest in magnitude, ties to the lower index,
 * written ascending to support_out (device, s int32; may be NULL when
 * s = 0).  0 <= s <= n.
 */
qiht_status qiht_hard_threshold(const float* a, int64_t n, int64_t s,
                                int32_t* support_out, void* stream);

/*
 * Least-squares refit on a support.  Not part of the paper's method (QIHT
 * returns its last iterate, Algorithm 2); a post-processing step that takes
 * the recovered support and solves, in FP64,
 *     z = argmin |y - A_G z|_2,   A_G = the columns `support` of A,
 * through the normal equations A_G^T A_G z = A_G^T y (blocked Cholesky on the
 * device), then writes x_out = z on the support and 0 elsewhere.
 *
 *   A: the caller's dense matrix when phi != NULL (device, m x n row-major,
 *      leading dimension ld >= n, dtype F32 or F64, or C64 / C128 taken as
 *      the stacked real matrix [Re Phi; Im Phi] of 2m rows; q is ignored);
 *      else the dequantized first realization Q1 of q (q's rows and n).
 *   y: device, rows doubles (m, 2m for complex phi, or q's rows).
 *   support: device, s int32 ascending, 1 <= s <= min(rows, n).
 *   x_out: device, n floats.  xs_out: device, s doubles, optional (z).
 *   Workspace: rows s + 10 s^2 doubles, allocated on `stream` and freed.
 *   Errors: INVALID_ARG, UNSUPPORTED (dtype), NUMERIC (A_G rank-deficient:
 *   the Gram matrix is not positive definite), OUT_OF_MEMORY, DEVICE.
 *   Synchronizes stream.
 */
qiht_status qiht_refit(const qiht_qmatrix* q, const void* phi, int64_t m,
                       int64_t n, int64_t ld, qiht_dtype dtype,
                       const double* y, const int32_t* support, int64_t s,
                       float* x_out, double* xs_out, void* stream);

/*
 * The autotuner's choices so far in this process, as JSON text:
 *   {"entries": [{"key": ..., "choice": ..., "default": ...,
 *                 "candidates_us": {name: microseconds, ...}}, ...]}
 * A solve tunes, on first meeting a problem shape (device architecture,
 * bit width or format, problem count, column bytes, n, total code size), the
 * launch shape of its dominant kernel by timing each candidate on the
 * problem's own codes (median of 7 launches after a warm-up): for packed
 * codes and FP32 the full pass g = Q1^T r ("cache" = two waves per SIMD with
 * two columns in flight each, "long" = three waves with one; "/r1" or "/r2" =
 * its columns cut into one or two rounds of resident workgroups), for a
 * batch on one dense-format matrix the GEMM's row splits ("ks1", "ks2",
 * "ks4").  The built-in heuristic ("default") is kept unless a candidate is
 * more than 3% faster.  QIHT_AUTOTUNE=0 disables tuning; QIHT_TUNE_FILE=path
 * reads earlier choices from that file and appends new ones to it;
 * QIHT_TUNE_FORCE=<name> pins one candidate (for comparisons).  The
 * pass candidates compute every entry of g identically; the GEMM's row
 * splits change the order of its sums (within the format's tolerance).
 * buf (host, cap bytes) receives the text, NUL-terminated and truncated to
 * fit; returns the size the full text needs (including the NUL), 0 on
 * failure.  buf may be NULL to query the size.
 */
int64_t qiht_tune_report(char* buf, int64_t cap);

/* Thread-local message of the last failed call ("" if none). */
const char* qiht_last_error(void);

/* Library version string. */
const char* qiht_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QIHT_H_ */
