// Host orchestration of the QIHT solve: workspace layout, the per-iteration
// launch sequence, and the entry points behind qiht_niht_solve,
// qiht_niht_solve_batched, qiht_gradient and qiht_hard_threshold.
//
// All control state lives on the device; the host only enqueues launches
// and, every kChunk rounds, reads the stop flags back.
#include <algorithm>
#include <cstdio>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "solve_common.h"

namespace qiht {
namespace {

constexpr int kChunk = 16;  // rounds enqueued between stop-flag reads

struct InfoDev {
    int32_t iterations, reason, backtracks, capped, err, full_selects;
    double mu_last;
};

// Warm start: x restricted to the given support, its compact copy and the
// support bitmap.
__global__ void k_warm_start(const ProbDev* __restrict__ P, const float* const* x0s) {
    const ProbDev& pd = P[blockIdx.x];
    const float* x0 = x0s[blockIdx.x];
    for (int i = threadIdx.x; i < pd.s; i += blockDim.x) {
        const int j = pd.sup[i];
        const float v = x0[j];
        pd.x[j] = v;
        pd.xs[i] = v;
        atomicOr(&pd.bmsup[j >> 5], 1u << (j & 31));
    }
}

// Stop flags of every problem, gathered for one read-back (into device
// memory, or into mapped host memory that the host reads once the launch's
// event has completed).
__global__ void k_done_flags(const ProbDev* __restrict__ P, int count, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = P[i].st->done;
    __threadfence_system();
}

__global__ void k_finalize(const ProbDev* __restrict__ P, float* const* xouts,
                           int32_t* const* souts, InfoDev* infos) {
    const ProbDev& pd = P[blockIdx.y];
    const SolveState* st = pd.st;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < pd.n; j += gridDim.x * blockDim.x)
        xouts[blockIdx.y][j] = pd.x[j];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < pd.s; t += gridDim.x * blockDim.x)
        souts[blockIdx.y][t] = pd.sup[t];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        InfoDev inf;
        inf.iterations = st->iter;
        inf.reason = st->done ? st->reason : QIHT_REASON_MAX_ITERS;
        inf.backtracks = st->total_bt;
        inf.capped = st->capped;
        inf.err = st->err;
        inf.full_selects = st->full_selects;
        inf.mu_last = st->mu_last;
        infos[blockIdx.y] = inf;
    }
}

// Chunks per lane of a full-pass row slab: enough to cover the column, at
// most 128 residual rows per lane (BITS chunks; 16 for FP32).  A power of
// two, or 3 for packed codes whose columns hold 129 .. 192 chunks (a lane
// past the column's end idles through every column: 3 per lane leaves a
// quarter of them idle where 4 would leave up to half).
int pass_cpl(int bits, int64_t col_bytes) {
    const int64_t chunks = col_bytes / 16;
    const int maxc = bits == 32 ? 16 : bits;
    int c = 1;
    while (c < maxc && static_cast<int64_t>(c) * 64 < chunks) c *= 2;
    if (c == 4 && bits <= 8 && chunks <= 3 * 64) c = 3;
    return c;
}

// The kernel instance a batch's largest chunks per lane runs in (a power
// of two: its spans switch down to their own count).
int pass_cmax(int cpl) { return cpl == 3 ? 4 : cpl; }

struct Carver {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count) {
        off = (off + 255) / 256 * 256;
        const size_t o = off;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return o;
    }
};

struct Layout {
    size_t cidx, cgx, ccnt, r32, rdig, rexp, rsum, g, gpart, hist, x, sup, xs, gs, bmsup, csup, cval, dlist, dw, meta, part_mu,
        part_om, st;
};

// Launch-shape choices the autotuner makes (tune.* below); -1 = the
// built-in heuristic.  None of them changes what a kernel computes for a
// column or a row, except ksplit (the GEMM's row splits, summed in split
// order).
struct TuneChoice {
    int long_stream = -1;  // full pass: 1 = three waves per SIMD with one
                           // column per step, 0 = two waves with two columns
    int rounds = -1;       // full pass: spans per resident workgroup in its
                           // queue (1, 2, 4 or 8)
    int ksplit = -1;       // shared-matrix GEMM: row splits (1, 2 or 4)
};

struct Plan {
    std::vector<ProbDev> host;
    std::vector<Layout> lay;
    std::vector<Task> tasks;
    int bits = 0, cpl = 1, maxwg = 1, max_n = 1;
    int rg = 1;  // 16-byte row groups per gather workgroup
    bool any_slab = false;
    bool long_stream = false;  // codes of one pass larger than the Infinity Cache
    size_t bytes = 0, probs_off = 0, tasks_off = 0, xptr_off = 0, sptr_off = 0, info_off = 0;
    size_t x0ptr_off = 0, done_off = 0;
    int npass = 0;   // full-pass workgroups
    int ntasks = 0;  // full-pass spans (pl.tasks holds one more entry: the queue counters)
    int per_wg = 1;  // full-pass spans per workgroup the spans were cut for
    // shared-matrix path: one GEMM per iteration instead of per-problem passes
    bool shared = false;
    SharedGemm sg{};
    size_t gblk_off = 0, bblk_off = 0, gpart_off = 0;
    // batches of per-problem matrices: the gathers' group tables (G_R,
    // G_MU, G_OMEGA), host copies, their workspace offsets, and (after
    // bind) the grids handed to the launches
    std::vector<int2> gtab[3];
    size_t gtab_off[3] = {0, 0, 0};
    GatherGrid gg[3];
};

qiht_status make_plan(const ProblemIn* in, int count, Plan& pl, const TuneChoice& tc = TuneChoice()) {
    pl.bits = in[0].q->bits;
    // All problems on one matrix: the pass is a GEMM on the matrix cores.
    // Dense formats have no per-problem pass; FP32 takes the GEMM from two
    // problems on.
    bool same = true;
    for (int i = 1; i < count; ++i) same = same && in[i].q == in[0].q;
    if (is_dense_format(pl.bits) && !same)
        return fail(QIHT_ERR_UNSUPPORTED, "problems on a dense-format matrix must share one handle");
    pl.shared = same && (is_dense_format(pl.bits) || (pl.bits == 32 && count > 1));
    // Gathers take 64 bytes of each listed column per workgroup (4 row
    // groups) where workgroups are plentiful -- a batch of per-problem
    // matrices, or columns of 1024 row groups or more (FP32 at 8192 rows) --
    // and fewer, wider column reads pay; a single problem with shorter
    // columns needs every workgroup it can get to hide the gathers' latency.
    int64_t max_cb = 0;
    for (int i = 0; i < count; ++i) max_cb = std::max(max_cb, in[i].q->col_bytes);
    pl.rg = ((count > 1 || max_cb / 16 >= 1024) && !pl.shared &&
             (pl.bits == 2 || pl.bits == 4 || pl.bits == 8 || pl.bits == 32)) ? 4 : 1;
    int64_t max_n = 0;
    for (int i = 0; i < count; ++i) max_n = std::max(max_n, in[i].q->n);
    if (max_n > kMaxSelectN) return fail(QIHT_ERR_UNSUPPORTED, "n above 262144");
    pl.max_n = static_cast<int>(max_n);
    // the kernel is built for the largest column; each problem's row slabs use
    // its own chunks per lane (a task carries them)
    pl.cpl = pass_cmax(pass_cpl(pl.bits, max_cb));
    Carver cv;
    pl.lay.resize(count);
    pl.host.resize(count);
    for (int i = 0; i < count; ++i) {
        const qiht_qmatrix* q = in[i].q;
        const int64_t s = in[i].s;
        const int64_t chunks = q->col_bytes / 16;
        const int64_t slab_chunks = 64LL * pass_cpl(pl.bits, q->col_bytes);
        const int nslab = static_cast<int>((chunks + slab_chunks - 1) / slab_chunks);
        const int nwg = static_cast<int>(q->col_bytes / 16);
        pl.maxwg = std::max(pl.maxwg, nwg);
        pl.any_slab = pl.any_slab || nslab > 1;
        Layout& L = pl.lay[i];
        // (FP32 on a shared matrix: r lives in the GEMM's operand block)
        L.r32 = (pl.shared && pl.bits == 32) ? 0 : cv.take<float>(q->rows_pad);
        L.cidx = cv.take<uint32_t>(q->n);
        L.cgx = cv.take<float2>(q->n);
        L.ccnt = cv.take<int32_t>(nwg);
        L.rdig = cv.take<uint32_t>(static_cast<size_t>(nwg) * digit_words_per_chunk(q->bits));
        L.rexp = cv.take<int32_t>(nwg);
        L.rsum = cv.take<int32_t>(nwg);
        L.g = pl.shared ? 0 : cv.take<float>(q->n);
        L.gpart = cv.take<float>(nslab > 1 && !pl.shared ? static_cast<size_t>(nslab) * q->n : 1);
        L.hist = cv.take<uint32_t>(2048);
        L.x = cv.take<float>(q->n);
        L.sup = cv.take<int32_t>(s);
        L.xs = cv.take<float>(s);
        L.gs = cv.take<float>(s);
        L.bmsup = cv.take<uint32_t>((q->n + 31) / 32);
        L.csup = cv.take<int32_t>(kSpec * s);
        L.cval = cv.take<float>(kSpec * s);
        L.dlist = cv.take<int32_t>(kSpec * 2 * s);
        L.dw = cv.take<double>(kSpec * 2 * s);
        L.meta = cv.take<CandMeta>(kSpec);
        L.part_mu = cv.take<double>(2 * static_cast<size_t>(nwg));
        L.part_om = cv.take<double>(static_cast<size_t>(kSpec) * nwg);
        L.st = cv.take<SolveState>(1);
        ProbDev& p = pl.host[i];
        std::memset(&p, 0, sizeof(p));
        p.q1 = q->codes[0];
        p.q2 = q->codes[1];
        p.col_bytes = q->col_bytes;
        p.rows = static_cast<int32_t>(q->rows);
        p.n = static_cast<int32_t>(q->n);
        p.s = static_cast<int32_t>(s);
        p.nwg = nwg;
        p.npart = pl.shared ? static_cast<int>((q->col_bytes + 1023) / 1024) : (nwg + pl.rg - 1) / pl.rg;
        p.nslab = pl.shared ? 1 : nslab;
        p.rowexp = q->rexp;
        p.group = static_cast<int32_t>(in[i].group);
        p.alpha = q->alpha;
        p.beta = q->beta;
        p.alpha_f = static_cast<float>(q->alpha);
        p.yhat = in[i].yhat;
    }
    if (pl.shared) {
        // G (problem k's g at k ldg) and R' (problem k's at k ldb), contiguous
        const qiht_qmatrix* q = in[0].q;
        pl.any_slab = false;
        pl.sg.a = q->codes[0];
        pl.sg.col_bytes = q->col_bytes;
        pl.sg.n = static_cast<int>(q->n);
        pl.sg.rows_pad = static_cast<int>(q->rows_pad);
        pl.sg.bits = pl.bits;
        pl.sg.ldg = round_up(q->n, 64);
        pl.gblk_off = cv.take<float>(static_cast<size_t>(count) * pl.sg.ldg);
        pl.sg.ksplit = tc.ksplit > 0 ? tc.ksplit : shared_ksplit(pl.bits, pl.sg.n, count, pl.sg.rows_pad);
        pl.gpart_off = pl.sg.ksplit > 1
                           ? cv.take<float>(static_cast<size_t>(pl.sg.ksplit) * count * pl.sg.ldg)
                           : 0;
        if (pl.bits == 32) {
            pl.sg.ldb = q->rows_pad;
            pl.sg.lo_off = 0;
            pl.bblk_off = cv.take<float>(static_cast<size_t>(count) * q->rows_pad);
        } else {
            pl.sg.ldb = 2 * q->rows_pad;
            pl.sg.lo_off = q->rows_pad;
            pl.bblk_off = cv.take<uint16_t>(static_cast<size_t>(count) * 2 * q->rows_pad);
        }
    }
    // Full-pass work: the workgroups the device holds at once (a second,
    // partial round would leave most CUs idle at the end), fed from a queue
    // of spans.  The columns of every problem's row slabs are cut into spans
    // of equal code bytes, spans running on across problem boundaries in
    // problem order; workgroup w starts with span w and then takes the next
    // unclaimed one (see the pass kernels), so workgroups that run faster
    // take more spans.  Spans per workgroup: 1 (a static split) for streams of
    // up to 1 MiB per workgroup, up to 8 for longer ones.
    double total = 0.0;
    for (int i = 0; i < count; ++i)
        total += static_cast<double>(in[i].q->n) * static_cast<double>(in[i].q->col_bytes);
    // Codes that stay in the 256 MiB Infinity Cache between passes are read
    // at cache latency: two waves per SIMD with two columns in flight each
    // do best there.  Longer streams come from HBM, where three waves per
    // SIMD with one column each hide more of the latency.
    pl.long_stream = total > kInfinityCacheBytes;
    // QIHT_PASS_STREAM=cache or =long pins the instance (for tuning; both are
    // valid for any problem and give the same g bit for bit).
    if (const char* e = std::getenv("QIHT_PASS_STREAM")) {
        if (std::strcmp(e, "long") == 0) pl.long_stream = true;
        else if (std::strcmp(e, "cache") == 0) pl.long_stream = false;
    }
    if (tc.long_stream >= 0) pl.long_stream = tc.long_stream != 0;
    const int slots = pl.shared ? 1 : std::max(1, pass_slots(pl.bits, pl.cpl, pl.long_stream));
    const double wg_bytes = std::max(1.0, std::ceil(total / slots));
    int per_wg = 1;
    while (per_wg < 8 && wg_bytes > static_cast<double>(per_wg) * (1 << 20)) per_wg *= 2;
    if (tc.rounds > 0) per_wg = tc.rounds;
    pl.per_wg = per_wg;
    const double budget = std::max(1.0, std::ceil(wg_bytes / per_wg));
    double cur = 0.0;
    for (int i = 0; i < count && !pl.shared; ++i) {
        const qiht_qmatrix* q = in[i].q;
        const ProbDev& p = pl.host[i];
        const int cpl = pass_cpl(pl.bits, q->col_bytes);
        const int64_t slab_max = 64LL * cpl * 16;
        for (int sl = 0; sl < p.nslab; ++sl) {
            const double sb = static_cast<double>(std::min<int64_t>(q->col_bytes - sl * slab_max, slab_max));
            int64_t c0 = 0;
            while (c0 < q->n) {
                const int64_t fit = std::max<int64_t>(1, static_cast<int64_t>(std::ceil((budget - cur) / sb)));
                const int64_t take = std::min<int64_t>({q->n - c0, fit, static_cast<int64_t>(kPassMaxCols)});
                pl.tasks.push_back(Task{i, sl, static_cast<int32_t>(c0), static_cast<int32_t>(c0 + take), cpl});
                c0 += take;
                cur += static_cast<double>(take) * sb;
                if (cur >= budget) cur = 0.0;
            }
        }
    }
    pl.ntasks = static_cast<int>(pl.tasks.size());
    pl.npass = std::min(slots, pl.ntasks);
    pl.tasks.push_back(Task{0, 0, 0, 0, 0});  // the queue counters (two zero words)
    // a batch's gather groups: row p * sets + t gets ceil((row groups +
    // extra) / 64) groups of 64 workgroups (the residual gather has one
    // extra workgroup per problem, its commit; the omega gather kSpec sets)
    if (count > 1 && !pl.shared) {
        for (int mode = 0; mode < 3; ++mode) {
            const int sets = mode == G_OMEGA ? kSpec : 1, extra = mode == G_R ? 1 : 0;
            std::vector<int2>& t = pl.gtab[mode];
            for (int i = 0; i < count; ++i)
                for (int k = 0; k < sets; ++k)
                    for (int g = 0; g < (pl.host[i].npart + extra + 63) / 64; ++g)
                        t.push_back(make_int2(i * sets + k, 64 * g));
            pl.gtab_off[mode] = cv.take<int2>(t.size());
        }
    }
    pl.probs_off = cv.take<ProbDev>(count);
    pl.tasks_off = cv.take<Task>(pl.tasks.size());
    pl.xptr_off = cv.take<float*>(count);
    pl.sptr_off = cv.take<int32_t*>(count);
    pl.x0ptr_off = cv.take<const float*>(count);
    pl.info_off = cv.take<InfoDev>(count);
    pl.done_off = cv.take<int32_t>(count);
    pl.bytes = cv.off;
    return QIHT_OK;
}

void bind(Plan& pl, uint8_t* base) {
    for (int mode = 0; mode < 3; ++mode) {
        pl.gg[mode] = GatherGrid();
        pl.gg[mode].rg = pl.rg;
        if (!pl.gtab[mode].empty()) {
            pl.gg[mode].tab = reinterpret_cast<const int2*>(base + pl.gtab_off[mode]);
            pl.gg[mode].ngroups = static_cast<int>(pl.gtab[mode].size());
        }
    }
    if (pl.shared) {
        pl.sg.g = reinterpret_cast<float*>(base + pl.gblk_off);
        pl.sg.b = base + pl.bblk_off;
        pl.sg.gp = pl.sg.ksplit > 1 ? reinterpret_cast<float*>(base + pl.gpart_off) : nullptr;
    }
    for (size_t i = 0; i < pl.host.size(); ++i) {
        ProbDev& p = pl.host[i];
        const Layout& L = pl.lay[i];
        p.r32 = reinterpret_cast<float*>(base + L.r32);  // replaced below for FP32 shared
        if (pl.shared) {
            p.g = pl.sg.g + static_cast<int64_t>(i) * pl.sg.ldg;
            if (pl.bits == 32)
                p.r32 = static_cast<float*>(const_cast<void*>(pl.sg.b)) + static_cast<int64_t>(i) * pl.sg.ldb;
            else
                p.rb = static_cast<uint16_t*>(const_cast<void*>(pl.sg.b)) + static_cast<int64_t>(i) * pl.sg.ldb;
        }
        p.cidx = reinterpret_cast<uint32_t*>(base + L.cidx);
        p.cgx = reinterpret_cast<float2*>(base + L.cgx);
        p.ccnt = reinterpret_cast<int32_t*>(base + L.ccnt);
        p.rdig = reinterpret_cast<uint32_t*>(base + L.rdig);
        p.rexp = reinterpret_cast<int32_t*>(base + L.rexp);
        p.rsum = reinterpret_cast<int32_t*>(base + L.rsum);
        if (!pl.shared) p.g = reinterpret_cast<float*>(base + L.g);
        p.gpart = reinterpret_cast<float*>(base + L.gpart);
        p.hist = reinterpret_cast<uint32_t*>(base + L.hist);
        p.x = reinterpret_cast<float*>(base + L.x);
        p.sup = reinterpret_cast<int32_t*>(base + L.sup);
        p.xs = reinterpret_cast<float*>(base + L.xs);
        p.gs = reinterpret_cast<float*>(base + L.gs);
        p.bmsup = reinterpret_cast<uint32_t*>(base + L.bmsup);
        p.csup = reinterpret_cast<int32_t*>(base + L.csup);
        p.cval = reinterpret_cast<float*>(base + L.cval);
        p.dlist = reinterpret_cast<int32_t*>(base + L.dlist);
        p.dw = reinterpret_cast<double*>(base + L.dw);
        p.meta = reinterpret_cast<CandMeta*>(base + L.meta);
        p.part_mu = reinterpret_cast<double*>(base + L.part_mu);
        p.part_om = reinterpret_cast<double*>(base + L.part_om);
        p.st = reinterpret_cast<SolveState*>(base + L.st);
    }
}

// Events recorded by every full-pass dispatch (profile mode): the start and
// end of the kernel itself, on its launch stream.  Creating events costs far
// more host time than an iteration takes on the device, so they come from a
// per-device pool: created on first use, handed to one solve at a time, and
// kept until the process ends.
class EventPool {
  public:
    // Moves `count` events of device `dev` into out (creating any missing).
    bool take(int dev, size_t count, std::vector<hipEvent_t>& out) {
        std::lock_guard<std::mutex> lk(m_);
        std::vector<hipEvent_t>& f = free_[dev];
        while (f.size() < count) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return false;
            f.push_back(e);
        }
        out.assign(f.end() - static_cast<std::ptrdiff_t>(count), f.end());
        f.resize(f.size() - count);
        return true;
    }
    void give(int dev, std::vector<hipEvent_t>& evs) {
        std::lock_guard<std::mutex> lk(m_);
        std::vector<hipEvent_t>& f = free_[dev];
        f.insert(f.end(), evs.begin(), evs.end());
        evs.clear();
    }

  private:
    std::mutex m_;
    std::map<int, std::vector<hipEvent_t>> free_;
};

EventPool& event_pool() {
    static EventPool p;
    return p;
}

// Profiling (qiht_params.profile = N): the full-pass dispatch of the first
// round of every N-th chunk of rounds carries HIP events; that round is
// launched directly, the rest of the chunk may replay as a captured graph.
struct PassTimer {
    bool on = false;
    int every = 1;       // time the first pass of every `every`-th chunk
    bool active = false; // the round being launched is a timed one
    int dev = 0;
    size_t used = 0;
    std::vector<hipEvent_t> ev;
    ~PassTimer() {
        if (!ev.empty()) event_pool().give(dev, ev);
    }
    // Events for up to `launches` profiled dispatches; profiling is off when
    // they cannot be had.
    void reserve(size_t launches) {
        if (!on) return;
        if (hipGetDevice(&dev) != hipSuccess || !event_pool().take(dev, 2 * launches, ev)) {
            ev.clear();
            on = false;
        }
    }
    // Called once per pass dispatch.  Returns false (no events) when
    // profiling is off, the dispatch is not in a timed chunk, or the reserve
    // is used up.
    bool pair(hipEvent_t* a, hipEvent_t* b) {
        *a = *b = nullptr;
        if (!on || !active || used + 2 > ev.size()) return false;
        *a = ev[used];
        *b = ev[used + 1];
        used += 2;
        return true;
    }
    double total_ms() const {
        double t = 0.0;
        for (size_t i = 0; i + 1 < used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) t += ms;
        }
        return t;
    }
    int launches() const { return static_cast<int>(used / 2); }
};

// Host memory the stop-flag launches write into directly: pinned, mapped and
// coherent, two slots of `count` flags (one per chunk in flight), per thread
// and device, grown to the largest batch met and kept until the process ends.
struct FlagSlots {
    int32_t* host = nullptr;
    int32_t* dev = nullptr;
    size_t cap = 0;  // flags per slot
};

FlagSlots* flag_slots(int dev, size_t count) {
    thread_local std::map<int, FlagSlots> slots;
    FlagSlots& f = slots[dev];
    if (f.cap < count) {
        void* h = nullptr;
        const size_t cap = std::max<size_t>(count, 256);
        if (hipHostMalloc(&h, 2 * cap * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(h);
            return nullptr;
        }
        if (f.host) (void)hipHostFree(f.host);  // (no launch of this thread still writes it)
        f.host = static_cast<int32_t*>(h);
        f.dev = static_cast<int32_t*>(d);
        f.cap = cap;
    }
    return &f;
}

struct Workspace {
    uint8_t* base = nullptr;
    hipStream_t st = nullptr;
    bool owned = true;  // false: the caller's memory (the no-allocation array)
    ~Workspace() {
        if (base && owned) (void)hipFreeAsync(base, st);
    }
};

void gradient_launches(const Plan& pl, const ProbDev* dP, const Task* dT, int count,
                       const SolveArgs& a, int zero_x, hipStream_t st, PassTimer* tm) {
    launch_gather(G_R, pl.bits, dP, count, pl.maxwg, a, zero_x, pl.shared, st, pl.gg[G_R]);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) tm->pair(&e0, &e1);
    if (pl.shared) {
        launch_shared_pass(pl.sg, dP, count, st, e0, e1);
        return;
    }
    launch_pass(pl.bits, pl.cpl, pl.long_stream, dP, dT, pl.npass, pl.ntasks, st, e0, e1);
    if (pl.any_slab) launch_slab_reduce(dP, count, pl.max_n, st);
}

// One round: the step-size test of the previous round's proposals and its
// commit (in the residual gather for a single problem, in k_commit before it
// for a batch), then the gradient, mu, the kSpec proposals of this round and
// their omegas.
void iteration_launches(const Plan& pl, const ProbDev* dP, const Task* dT, int count,
                        const SolveArgs& a, hipStream_t st, PassTimer* tm,
                        const FreshSource* fresh) {
    if (!a.decide_in_gather) launch_commit(dP, count, a, st);
    if (fresh) {
        // the realizations of the iteration to come: matrix copies 2 it and
        // 2 it + 1 and y_hat realization it, it = the completed iterations
        // (read on the device; a round of further shrinks redraws the same)
        const char* stb = reinterpret_cast<const char*>(pl.host[0].st);
        const int32_t* it = reinterpret_cast<const int32_t*>(stb + offsetof(SolveState, iter));
        const int32_t* done = reinterpret_cast<const int32_t*>(stb + offsetof(SolveState, done));
        launch_quantize_matrix(fresh->phi, fresh->dtype, fresh->m, fresh->n, fresh->ld, fresh->bits, 2,
                               fresh->seed, fresh->c, fresh->K, fresh->levels, fresh->q, st, it, done);
        launch_quantize_vector(fresh->y, fresh->ydtype, fresh->m, fresh->ybits, fresh->ylevels, fresh->seed,
                               fresh->yc, fresh->yK, fresh->ylev, fresh->yhat, nullptr, st, it, done);
    }
    gradient_launches(pl, dP, dT, count, a, 0, st, tm);
    launch_gather(G_MU, pl.bits, dP, count, pl.maxwg, a, 0, pl.shared, st, pl.gg[G_MU]);
    launch_propose(dP, count, a, SEL_STEP, pl.max_n, st);
    launch_gather(G_OMEGA, pl.bits, dP, count, pl.maxwg, a, 0, pl.shared, st, pl.gg[G_OMEGA]);
}

// ---------------------------------------------------------------------------
// Captured chunks: the launches of kChunk rounds recorded once as a HIP graph
// and replayed on the caller's stream (the device then runs them back to back
// without a host launch per kernel).  The recording goes to a stream of the
// library's own (the caller's may be the null stream, which cannot capture);
// nothing runs while recording.  Executable graphs are kept per device,
// keyed by everything their kernels receive as arguments or geometry (the
// workspace addresses, the plan's launch shape, the solver arguments, the
// round count), so a later solve of the same shape on pool memory at the
// same address replays them; the control state they act on is in the
// workspace, which each solve initializes.  Profiling (events around every
// pass) and draws per iteration run uncaptured.
// ---------------------------------------------------------------------------
struct ChunkKey {
    uintptr_t dP, dT;
    uintptr_t shared_a;
    uintptr_t gtab[3];  // a batch's gather group tables and their sizes
    int64_t gtab_n[3];
    int64_t shared_cb;
    int64_t nl;
    int bits, cpl, npass, maxwg, max_n, count, ksplit, shared_n;
    int flags;  // long_stream << 1 | shared << 2 | any_slab << 3
    int32_t max_iters, max_backtracks, mu_mode, decide_in_gather;
    double tol, k, c;
    bool operator<(const ChunkKey& o) const { return std::memcmp(this, &o, sizeof(ChunkKey)) < 0; }
};

class GraphCache {
  public:
    // Solves that ran with launch key `key` (round count 0) on `dev` before
    // this one; counts this one.  Capturing and instantiating a chunk costs
    // more than the launches it saves in one solve, so shapes are captured
    // only once they recur.
    int64_t count_solve(int dev, const ChunkKey& key) {
        std::lock_guard<std::mutex> lk(m_);
        return devs_[dev].solves[key]++;
    }
    // The executable graph of `key` on device `dev`, recorded by `record`
    // (called with the capture stream) on first use; nullptr if capture or
    // instantiation fails (the caller then launches directly).
    template <typename F>
    hipGraphExec_t get(int dev, const ChunkKey& key, F&& record) {
        std::lock_guard<std::mutex> lk(m_);
        Dev& d = devs_[dev];
        for (auto& e : d.items)
            if (!(e.key < key) && !(key < e.key)) {
                e.used = ++d.clock;
                return e.exec;
            }
        if (!d.cap && hipStreamCreateWithFlags(&d.cap, hipStreamNonBlocking) != hipSuccess) {
            d.cap = nullptr;
            (void)hipGetLastError();
            return nullptr;
        }
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(d.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        record(d.cap);
        const hipError_t le = hipGetLastError();
        if (hipStreamEndCapture(d.cap, &g) != hipSuccess || le != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return nullptr;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess || !ex) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (d.items.size() >= kKeep) {
            auto old = std::min_element(d.items.begin(), d.items.end(),
                                        [](const Item& a, const Item& b) { return a.used < b.used; });
            (void)hipGraphExecDestroy(old->exec);
            d.items.erase(old);
        }
        d.items.push_back(Item{key, ex, ++d.clock});
        return ex;
    }

  private:
    static constexpr size_t kKeep = 64;
    struct Item {
        ChunkKey key;
        hipGraphExec_t exec;
        uint64_t used;
    };
    struct Dev {
        hipStream_t cap = nullptr;
        std::vector<Item> items;
        uint64_t clock = 0;
        std::map<ChunkKey, int64_t> solves;
    };
    std::mutex m_;
    std::map<int, Dev> devs_;
};

GraphCache& graph_cache() {
    static GraphCache* c = new GraphCache();  // kept until the process ends
    return *c;
}

// ext (optional): memory of ext_cap bytes to carve the workspace from
// instead of the pool.  tc: the launch shapes to plan with.
qiht_status setup(const ProblemIn* in, int count, Plan& pl, Workspace& ws, hipStream_t st,
                  ProbDev** dP, Task** dT, uint8_t* ext = nullptr, size_t ext_cap = 0,
                  const TuneChoice& tc = TuneChoice()) {
    qiht_status s0 = make_plan(in, count, pl, tc);
    if (s0 != QIHT_OK) return s0;
    ws.st = st;
    if (ext) {
        if (pl.bytes > ext_cap)
            return fail(QIHT_ERR_UNSUPPORTED, "the solve needs a workspace of " + std::to_string(pl.bytes) +
                                                  " bytes, above the no-allocation array's " +
                                                  std::to_string(ext_cap));
        ws.base = ext;
        ws.owned = false;
    } else {
        hipError_t e = pool_malloc(reinterpret_cast<void**>(&ws.base), pl.bytes, st);
        if (e != hipSuccess || ws.base == nullptr) {
            ws.base = nullptr;
            (void)hipGetLastError();
            return fail(QIHT_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        }
    }
    bind(pl, ws.base);
    QIHT_HIP(hipMemsetAsync(ws.base, 0, pl.bytes, st));
    *dP = reinterpret_cast<ProbDev*>(ws.base + pl.probs_off);
    *dT = reinterpret_cast<Task*>(ws.base + pl.tasks_off);
    QIHT_HIP(hipMemcpyAsync(*dP, pl.host.data(), sizeof(ProbDev) * count, hipMemcpyHostToDevice,
                            st));
    QIHT_HIP(hipMemcpyAsync(*dT, pl.tasks.data(), sizeof(Task) * pl.tasks.size(),
                            hipMemcpyHostToDevice, st));
    for (int mode = 0; mode < 3; ++mode)
        if (!pl.gtab[mode].empty())
            QIHT_HIP(hipMemcpyAsync(const_cast<int2*>(pl.gg[mode].tab), pl.gtab[mode].data(),
                                    sizeof(int2) * pl.gtab[mode].size(), hipMemcpyHostToDevice, st));

    return QIHT_OK;
}

// ---------------------------------------------------------------------------
// Autotuner.  The launch shape of the full pass (its instance: two waves per
// SIMD with two columns in flight each, or three with one; and how many spans
// per workgroup its queue holds: 1, 2, 4 or 8) and of the
// shared-matrix GEMM (row splits 1, 2 or 4) is chosen per device architecture
// and problem shape by timing every candidate on the problem's own codes: one
// warm-up launch, then the median of kTuneReps launches between stream
// events.  The built-in heuristic stays unless a candidate beats it by more
// than kTuneMargin.  Choices are kept for the process and, when QIHT_TUNE_FILE
// names a file, read from it first and appended to it (one line per shape:
// key, choice, every candidate's microseconds).  QIHT_AUTOTUNE=0 switches
// tuning off (the heuristic runs).  Only the GEMM's row splits change a sum's
// order (its split partials are added in split order); the pass candidates
// compute every column of g the same way.
// ---------------------------------------------------------------------------
constexpr int kTuneReps = 7;
constexpr double kTuneMargin = 0.03;

struct TuneEntry {
    std::string key, choice, deflt;
    std::vector<std::pair<std::string, double>> cand_us;
};

TuneChoice choice_from_name(const std::string& nm) {
    TuneChoice c;
    if (nm.rfind("ks", 0) == 0) {
        c.ksplit = std::atoi(nm.c_str() + 2);
    } else {
        const size_t sl = nm.find("/r");
        c.long_stream = nm.compare(0, 4, "long") == 0 ? 1 : 0;
        c.rounds = sl == std::string::npos ? 1 : std::atoi(nm.c_str() + sl + 2);
    }
    return c;
}

class Tuner {
  public:
    bool enabled() const {
        const char* e = std::getenv("QIHT_AUTOTUNE");
        return !(e && std::strcmp(e, "0") == 0);
    }
    bool find(const std::string& key, TuneChoice* c) {
        std::lock_guard<std::mutex> lk(m_);
        load_locked();
        auto it = entries_.find(key);
        if (it == entries_.end()) return false;
        *c = choice_from_name(it->second.choice);
        return true;
    }
    void put(const TuneEntry& e) {
        std::lock_guard<std::mutex> lk(m_);
        load_locked();
        entries_[e.key] = e;
        const char* f = std::getenv("QIHT_TUNE_FILE");
        if (!f || !*f) return;
        if (FILE* fp = std::fopen(f, "a")) {
            std::fprintf(fp, "%s\t%s\t%s", e.key.c_str(), e.choice.c_str(), e.deflt.c_str());
            for (const auto& cu : e.cand_us) std::fprintf(fp, "\t%s=%.3f", cu.first.c_str(), cu.second);
            std::fprintf(fp, "\n");
            std::fclose(fp);
        }
    }
    std::string report() {
        std::lock_guard<std::mutex> lk(m_);
        load_locked();
        std::string o = "{\"entries\": [";
        bool first = true;
        for (const auto& kv : entries_) {
            const TuneEntry& e = kv.second;
            o += first ? "" : ", ";
            first = false;
            o += "{\"key\": \"" + e.key + "\", \"choice\": \"" + e.choice + "\", \"default\": \"" + e.deflt +
                 "\", \"candidates_us\": {";
            for (size_t i = 0; i < e.cand_us.size(); ++i) {
                char b[64];
                std::snprintf(b, sizeof(b), "%.3f", e.cand_us[i].second);
                o += (i ? ", \"" : "\"") + e.cand_us[i].first + "\": " + b;
            }
            o += "}}";
        }
        return o + "]}";
    }

  private:
    // Entries of QIHT_TUNE_FILE (later lines of a key win).
    void load_locked() {
        if (loaded_) return;
        loaded_ = true;
        const char* f = std::getenv("QIHT_TUNE_FILE");
        if (!f || !*f) return;
        FILE* fp = std::fopen(f, "r");
        if (!fp) return;
        char buf[4096];
        while (std::fgets(buf, sizeof(buf), fp)) {
            std::string ln(buf);
            while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
            std::vector<std::string> fld;
            size_t a = 0;
            while (true) {
                const size_t b = ln.find('\t', a);
                fld.push_back(ln.substr(a, b == std::string::npos ? std::string::npos : b - a));
                if (b == std::string::npos) break;
                a = b + 1;
            }
            if (fld.size() < 3) continue;
            TuneEntry e{fld[0], fld[1], fld[2], {}};
            for (size_t i = 3; i < fld.size(); ++i) {
                const size_t eq = fld[i].find('=');
                if (eq != std::string::npos)
                    e.cand_us.emplace_back(fld[i].substr(0, eq), std::atof(fld[i].c_str() + eq + 1));
            }
            entries_[e.key] = e;
        }
        std::fclose(fp);
    }
    std::mutex m_;
    bool loaded_ = false;
    std::map<std::string, TuneEntry> entries_;
};

Tuner& tuner() {
    static Tuner* t = new Tuner();  // kept until the process ends
    return *t;
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// The shape a tuned choice is kept for.
std::string tune_key(const ProblemIn* in, int count, const Plan& pl) {
    int64_t max_cb = 0, max_n = 0;
    double total = 0.0;
    for (int i = 0; i < count; ++i) {
        max_cb = std::max(max_cb, in[i].q->col_bytes);
        max_n = std::max(max_n, in[i].q->n);
        total += static_cast<double>(in[i].q->n) * static_cast<double>(in[i].q->col_bytes);
    }
    char b[256];
    std::snprintf(b, sizeof(b), "%s|%s|bits%d|count%d|col_bytes%lld|n%lld|MiB%lld", arch_name().c_str(),
                  pl.shared ? "gemm" : "pass", pl.bits, count, static_cast<long long>(max_cb),
                  static_cast<long long>(max_n), static_cast<long long>(total / 1048576.0));
    return b;
}

std::string choice_name(const Plan& pl, const TuneChoice& c) {
    if (pl.shared) return "ks" + std::to_string(c.ksplit > 0 ? c.ksplit : pl.sg.ksplit);
    return std::string(c.long_stream > 0 ? "long" : "cache") + "/r" + std::to_string(c.rounds > 0 ? c.rounds : 1);
}

// Median microseconds of the product (full pass or GEMM) under choice c.
qiht_status time_choice(const ProblemIn* in, int count, const TuneChoice& c, hipStream_t st,
                        hipEvent_t* ev, double* us) {
    Plan pl;
    Workspace ws;
    ProbDev* dP = nullptr;
    Task* dT = nullptr;
    qiht_status s0 = setup(in, count, pl, ws, st, &dP, &dT, nullptr, 0, c);
    if (s0 != QIHT_OK) return s0;
    const SolveArgs a{1, -1.0, 2.0, 0.01, 0, 0, 0, 0};
    launch_gather(G_R, pl.bits, dP, count, pl.maxwg, a, 1, pl.shared, st, pl.gg[G_R]);  // r = y_hat
    std::vector<double> t;
    for (int r = 0; r <= kTuneReps; ++r) {
        QIHT_HIP(hipEventRecord(ev[0], st));
        if (pl.shared) {
            launch_shared_pass(pl.sg, dP, count, st);
        } else {
            launch_pass(pl.bits, pl.cpl, pl.long_stream, dP, dT, pl.npass, pl.ntasks, st, nullptr, nullptr);
            if (pl.any_slab) launch_slab_reduce(dP, count, pl.max_n, st);
        }
        QIHT_HIP(hipEventRecord(ev[1], st));
        QIHT_HIP(hipEventSynchronize(ev[1]));
        float ms = 0.f;
        QIHT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        if (r > 0) t.push_back(ms * 1e3);
    }
    std::sort(t.begin(), t.end());
    *us = t[t.size() / 2];
    return QIHT_OK;
}

// The tuned launch shapes of a solve: the kept choice of its shape, or a
// new tuning of it; the heuristic when tuning is off or not possible.
qiht_status tuned_choice(const ProblemIn* in, int count, hipStream_t st, bool may_tune, TuneChoice* out) {
    *out = TuneChoice();
    if (!tuner().enabled()) return QIHT_OK;
    Plan p0;
    qiht_status s0 = make_plan(in, count, p0);
    if (s0 != QIHT_OK) return s0;
    if (p0.shared && !is_dense_format(p0.bits)) return QIHT_OK;  // FP32 GEMM: one shape
    // QIHT_TUNE_FORCE=<choice> pins one candidate of the matching kind (for
    // tests and comparisons)
    if (const char* f = std::getenv("QIHT_TUNE_FORCE")) {
        const std::string nm(f);
        if (p0.shared == (nm.rfind("ks", 0) == 0)) {
            TuneChoice c = choice_from_name(nm);
            if (!p0.shared || shared_ksplit_ok(p0.bits, p0.sg.rows_pad, c.ksplit)) *out = c;
            return QIHT_OK;
        }
    }
    const std::string key = tune_key(in, count, p0);
    if (tuner().find(key, out) || !may_tune) return QIHT_OK;
    std::vector<TuneChoice> cands;
    TuneChoice def;
    if (p0.shared) {
        def.ksplit = p0.sg.ksplit;
        for (int ks = 1; ks <= 4; ks *= 2)
            if (shared_ksplit_ok(p0.bits, p0.sg.rows_pad, ks)) {
                TuneChoice c;
                c.ksplit = ks;
                cands.push_back(c);
            }
    } else {
        def.long_stream = p0.long_stream ? 1 : 0;
        def.rounds = p0.per_wg;
        for (int ls = 0; ls <= 1; ++ls)
            for (int rd = 1; rd <= 8; rd *= 2) {
                TuneChoice c;
                c.long_stream = ls;
                c.rounds = rd;
                cands.push_back(c);
            }
    }
    int dev = 0;
    QIHT_HIP(hipGetDevice(&dev));
    std::vector<hipEvent_t> ev;
    if (!event_pool().take(dev, 2, ev)) return QIHT_OK;
    TuneEntry e{key, "", choice_name(p0, def), {}};
    double best = 0.0, tdef = 0.0;
    TuneChoice bestc = def;
    qiht_status st0 = QIHT_OK;
    for (const TuneChoice& c : cands) {
        double us = 0.0;
        st0 = time_choice(in, count, c, st, ev.data(), &us);
        if (st0 != QIHT_OK) break;
        const std::string nm = choice_name(p0, c);
        e.cand_us.emplace_back(nm, us);
        if (nm == e.deflt) tdef = us;
        if (best == 0.0 || us < best) {
            best = us;
            bestc = c;
        }
    }
    event_pool().give(dev, ev);
    if (st0 != QIHT_OK) return st0;
    if (tdef > 0.0 && tdef <= (1.0 + kTuneMargin) * best) bestc = def;
    e.choice = choice_name(p0, bestc);
    tuner().put(e);
    *out = bestc;
    return QIHT_OK;
}

}  // namespace

qiht_status run_solve(const ProblemIn* in, int count, const SolveArgs& args, qiht_info* infos,
                      hipStream_t st, const FreshSource* fresh, uint8_t* ext_ws, size_t ext_cap) {
    SolveArgs a = args;
    // (fresh draws are made between the commit and the residual gather)
    a.decide_in_gather = (count == 1 && !fresh) ? 1 : 0;
    Plan pl;
    Workspace ws;
    ProbDev* dP = nullptr;
    Task* dT = nullptr;
    TuneChoice tc;
    qiht_status s0 = tuned_choice(in, count, st, ext_ws == nullptr, &tc);
    if (s0 != QIHT_OK) return s0;
    s0 = setup(in, count, pl, ws, st, &dP, &dT, ext_ws, ext_cap, tc);
    if (s0 != QIHT_OK) return s0;
    std::vector<float*> xo(count);
    std::vector<int32_t*> so(count);
    std::vector<const float*> x0(count);
    bool warm = false;
    for (int i = 0; i < count; ++i) {
        xo[i] = in[i].x_out;
        so[i] = in[i].support_out;
        x0[i] = in[i].x0;
        if (in[i].x0) {
            warm = true;
            QIHT_HIP(hipMemcpyAsync(pl.host[i].sup, in[i].support0, sizeof(int32_t) * pl.host[i].s,
                                    hipMemcpyDeviceToDevice, st));
        }
    }
    float** dxo = reinterpret_cast<float**>(ws.base + pl.xptr_off);
    int32_t** dso = reinterpret_cast<int32_t**>(ws.base + pl.sptr_off);
    const float** dx0 = reinterpret_cast<const float**>(ws.base + pl.x0ptr_off);
    QIHT_HIP(hipMemcpyAsync(dxo, xo.data(), sizeof(float*) * count, hipMemcpyHostToDevice, st));
    QIHT_HIP(hipMemcpyAsync(dso, so.data(), sizeof(int32_t*) * count, hipMemcpyHostToDevice, st));
    QIHT_HIP(hipMemcpyAsync(dx0, x0.data(), sizeof(float*) * count, hipMemcpyHostToDevice, st));

    PassTimer timer;
    timer.on = a.profile != 0;
    timer.every = std::max(1, a.profile);
    // (the first round's pass of every timed chunk; the initial pass, which
    // follows the quantization's stream through the caches, is not timed)
    timer.reserve(static_cast<size_t>(2 * (static_cast<int64_t>(a.max_iters) + 1) / (kChunk * timer.every) + 2));
    timer.active = false;
    if (warm) {
        // x0 restricted to its support (x is zero elsewhere)
        hipLaunchKernelGGL(k_warm_start, dim3(count), dim3(256), 0, st, dP, dx0);
    } else {
        // x0 = 0; G0 = supp H_s(Q1^T y_hat).
        gradient_launches(pl, dP, dT, count, a, 1, st, &timer);
        launch_candidates(dP, count, pl.maxwg, st);
        launch_propose(dP, count, a, SEL_INIT, pl.max_n, st);
    }
    QIHT_HIP(hipGetLastError());

    // Rounds until every problem has stopped.  Iteration i is committed by
    // the residual gather of round i + 1, so max_iters iterations take
    // max_iters + 1 rounds when no test needs more than kSpec shrinks; each
    // further kSpec shrinks of one iteration take one more round, and the
    // backtracking cap bounds them.
    std::vector<int32_t> hdone(count);
    int32_t* ddone = reinterpret_cast<int32_t*>(ws.base + pl.done_off);
    const int64_t per_iter = std::max<int64_t>(1, (static_cast<int64_t>(a.max_backtracks) + kSpec) / kSpec);
    const int64_t first = a.max_iters > 0 ? static_cast<int64_t>(a.max_iters) + 1 : 0;
    const int64_t max_rounds = a.max_iters > 0 ? static_cast<int64_t>(a.max_iters) * per_iter + 1 : 0;
    // Chunks of rounds run as captured graphs once their launch shape has
    // recurred (two earlier solves with the same workspace, plan and
    // arguments), unless timed (profiling), drawn per iteration, on
    // caller-provided memory (instantiation may allocate), or switched off
    // with QIHT_GRAPH=0.
    const char* ge = std::getenv("QIHT_GRAPH");
    const bool graphs = !fresh && !ext_ws && !(ge && std::strcmp(ge, "0") == 0);
    int dev = 0;
    QIHT_HIP(hipGetDevice(&dev));
    auto record_chunk = [&](hipStream_t s, int64_t nl, PassTimer* tm) {
        for (int64_t r = 0; r < nl; ++r) iteration_launches(pl, dP, dT, count, a, s, tm, fresh);
    };
    auto chunk_key = [&](int64_t nl) {
        ChunkKey key;
        std::memset(&key, 0, sizeof(key));
        key.dP = reinterpret_cast<uintptr_t>(dP);
        key.dT = reinterpret_cast<uintptr_t>(dT);
        key.shared_a = pl.shared ? reinterpret_cast<uintptr_t>(pl.sg.a) : 0;
        key.nl = nl;
        key.bits = pl.bits;
        key.cpl = pl.cpl;
        key.npass = pl.npass;
        key.maxwg = pl.maxwg;
        key.max_n = pl.max_n;
        for (int mode = 0; mode < 3; ++mode) {
            key.gtab[mode] = reinterpret_cast<uintptr_t>(pl.gg[mode].tab);
            key.gtab_n[mode] = pl.gg[mode].ngroups;
        }
        key.count = count;
        key.ksplit = pl.shared ? pl.sg.ksplit : 0;
        key.shared_n = pl.shared ? pl.sg.n : 0;
        key.shared_cb = pl.shared ? pl.sg.col_bytes : 0;
        key.flags = (pl.long_stream ? 2 : 0) | (pl.shared ? 4 : 0) | (pl.any_slab ? 8 : 0);
        key.max_iters = a.max_iters;
        key.max_backtracks = a.max_backtracks;
        key.mu_mode = a.mu_mode;
        key.decide_in_gather = a.decide_in_gather;
        key.tol = a.tol;
        key.k = a.k;
        key.c = a.c;
        return key;
    };
    const bool recurring = graphs && graph_cache().count_solve(dev, chunk_key(0)) >= 2;
    int64_t chunk_no = 0;
    auto launch_chunk = [&](int64_t launched) -> qiht_status {
        const int64_t goal = launched < first ? first : max_rounds;
        int64_t nl = std::min<int64_t>(kChunk, goal - launched);
        // a timed chunk launches its first round itself, that round's pass
        // carrying the events; the rest of the chunk as usual
        if (timer.on && (chunk_no++ % timer.every) == 0) {
            timer.active = true;
            record_chunk(st, 1, &timer);
            timer.active = false;
            if (--nl == 0) return QIHT_OK;
        }
        hipGraphExec_t ex = nullptr;
        if (recurring)
            ex = graph_cache().get(dev, chunk_key(nl), [&](hipStream_t cs) { record_chunk(cs, nl, nullptr); });
        if (ex) QIHT_HIP(hipGraphLaunch(ex, st));
        else record_chunk(st, nl, &timer);
        return QIHT_OK;
    };
    auto chunk_rounds = [&](int64_t launched) {
        return std::min<int64_t>(kChunk, (launched < first ? first : max_rounds) - launched);
    };
    // Stop flags: with pool memory, the chunks of the first max_iters + 1
    // rounds (which every solve runs unless it stops early) are launched one
    // ahead of the check of the previous chunk's flags, written by the device
    // into mapped host memory: the device is not left idle while the host
    // reads them.  Past those rounds, or when the flags or events cannot be
    // had (or on caller-provided memory, which allows no allocation), each
    // chunk is checked before the next is launched.  A chunk launched ahead
    // of a solve that has already stopped finds every problem done and
    // returns at once.
    FlagSlots* fs = ext_ws ? nullptr : flag_slots(dev, static_cast<size_t>(count));
    std::vector<hipEvent_t> fev;
    if (fs && !event_pool().take(dev, 2, fev)) fs = nullptr;
    if (fs) {
        std::deque<int> pend;  // slots of chunks launched and not yet checked
        int slot = 0;
        int64_t launched = 0;
        qiht_status sl = QIHT_OK;
        bool all_done = false;
        while (!all_done && sl == QIHT_OK) {
            while (launched < max_rounds && (pend.empty() || (pend.size() < 2 && launched < first))) {
                const int64_t nl = chunk_rounds(launched);
                sl = launch_chunk(launched);
                if (sl != QIHT_OK) break;
                launched += nl;
                int32_t* out = fs->dev + static_cast<size_t>(slot) * fs->cap;
                hipLaunchKernelGGL(k_done_flags, dim3((count + 255) / 256), dim3(256), 0, st, dP, count, out);
                if (hipGetLastError() != hipSuccess || hipEventRecord(fev[slot], st) != hipSuccess) {
                    sl = fail(QIHT_ERR_DEVICE, "stop-flag launch failed");
                    break;
                }
                pend.push_back(slot);
                slot ^= 1;
            }
            if (sl != QIHT_OK || pend.empty()) break;
            const int chk = pend.front();
            pend.pop_front();
            if (hipEventSynchronize(fev[chk]) != hipSuccess) {
                sl = fail(QIHT_ERR_DEVICE, "stop-flag wait failed");
                break;
            }
            const volatile int32_t* h = fs->host + static_cast<size_t>(chk) * fs->cap;
            all_done = true;
            for (int i = 0; i < count; ++i) all_done = all_done && h[i] != 0;
        }
        // (the events are recorded on st: the stream order below keeps the
        // solve's later work behind any chunk still in flight)
        if (sl != QIHT_OK) (void)hipStreamSynchronize(st);
        event_pool().give(dev, fev);
        if (sl != QIHT_OK) return sl;
    } else {
        for (int64_t launched = 0; launched < max_rounds;) {
            const int64_t nl = chunk_rounds(launched);
            qiht_status sl = launch_chunk(launched);
            if (sl != QIHT_OK) return sl;
            launched += nl;
            hipLaunchKernelGGL(k_done_flags, dim3((count + 255) / 256), dim3(256), 0, st, dP, count, ddone);
            QIHT_HIP(hipGetLastError());
            QIHT_HIP(hipMemcpyAsync(hdone.data(), ddone, sizeof(int32_t) * count, hipMemcpyDeviceToHost, st));
            QIHT_HIP(hipStreamSynchronize(st));
            bool all_done = true;
            for (int i = 0; i < count; ++i) all_done = all_done && hdone[i] != 0;
            if (all_done) break;
        }
    }
    QIHT_HIP(hipGetLastError());

    InfoDev* dinf = reinterpret_cast<InfoDev*>(ws.base + pl.info_off);
    hipLaunchKernelGGL(k_finalize, dim3(32, count), dim3(256), 0, st, dP, dxo, dso, dinf);
    QIHT_HIP(hipGetLastError());
    std::vector<InfoDev> hinf(count);
    QIHT_HIP(hipMemcpyAsync(hinf.data(), dinf, sizeof(InfoDev) * count, hipMemcpyDeviceToHost,
                            st));
    QIHT_HIP(hipStreamSynchronize(st));
    bool nan = false;
    for (int i = 0; i < count; ++i) {
        nan = nan || hinf[i].err;
        if (infos) {
            infos[i].iterations = hinf[i].iterations;
            infos[i].reason = hinf[i].reason;
            infos[i].backtracks = hinf[i].backtracks;
            infos[i].capped_iterations = hinf[i].capped;
            infos[i].mu_last = hinf[i].mu_last;
            infos[i].pass_ms = timer.total_ms();
            infos[i].pass_launches = timer.launches();
            infos[i].full_selects = hinf[i].full_selects;
        }
    }
    if (nan) return fail(QIHT_ERR_NUMERIC, "NaN met in the iterate");
    return QIHT_OK;
}

qiht_status run_gradient(const qiht_qmatrix* q, const double* yhat, const float* x,
                         const int32_t* support, int64_t s, float* g_out, float* r_out,
                         hipStream_t st) {
    ProblemIn in{q, yhat, std::max<int64_t>(s, 1), nullptr, nullptr, x, support};
    Plan pl;
    Workspace ws;
    ProbDev* dP = nullptr;
    Task* dT = nullptr;
    qiht_status s0 = setup(&in, 1, pl, ws, st, &dP, &dT);
    if (s0 != QIHT_OK) return s0;
    const ProbDev& h = pl.host[0];
    if (s > 0) {
        QIHT_HIP(hipMemcpyAsync(h.sup, support, sizeof(int32_t) * s, hipMemcpyDeviceToDevice, st));
        const float** dx0 = reinterpret_cast<const float**>(ws.base + pl.x0ptr_off);
        QIHT_HIP(hipMemcpyAsync(dx0, &x, sizeof(float*), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_warm_start, dim3(1), dim3(256), 0, st, dP, dx0);
    }
    SolveArgs a{1, -1.0, 2.0, 0.01, 0, 0, 0, 0};
    gradient_launches(pl, dP, dT, 1, a, s == 0 ? 1 : 0, st, nullptr);
    QIHT_HIP(hipGetLastError());
    QIHT_HIP(hipMemcpyAsync(g_out, h.g, sizeof(float) * h.n, hipMemcpyDeviceToDevice, st));
    if (r_out)
        QIHT_HIP(hipMemcpyAsync(r_out, h.r32, sizeof(float) * h.rows, hipMemcpyDeviceToDevice, st));
    QIHT_HIP(hipStreamSynchronize(st));
    return QIHT_OK;
}

qiht_status run_hard_threshold(const float* a, int64_t n, int64_t s, int32_t* support_out,
                               hipStream_t st) {
    if (n > kMaxSelectN) return fail(QIHT_ERR_UNSUPPORTED, "n above 262144");
    int* err = nullptr;
    QIHT_HIP(pool_malloc(reinterpret_cast<void**>(&err), sizeof(int), st));
    QIHT_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
    launch_hard_threshold(a, static_cast<int>(n), static_cast<int>(s), support_out,
                          err, st);
    QIHT_HIP(hipGetLastError());
    int herr = 0;
    QIHT_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    QIHT_HIP(hipFreeAsync(err, st));
    QIHT_HIP(hipStreamSynchronize(st));
    if (herr) return fail(QIHT_ERR_NUMERIC, "NaN in the input of H_s");
    return QIHT_OK;
}

// ---------------------------------------------------------------------------
// The solve without device allocation (qiht_niht_solve_noalloc).  Its
// workspace is a file-scope device array: every device the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, so the array's device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is ever handed to kernels or copies.  Calls of one process on one
// device take turns (a per-device lock held until the call has synchronized
// its stream), since they all use the same array.
// ---------------------------------------------------------------------------
namespace {

__device__ __align__(256) uint8_t scratch[QIHT_NOALLOC_WORKSPACE_BYTES];

struct ScratchSlot {
    std::mutex run;          // held for a whole call on this device
    uint8_t* ptr = nullptr;  // the device address of `scratch` (set once)
};

ScratchSlot& scratch_slot(int dev) {
    static std::mutex mu;
    static std::map<int, ScratchSlot> slots;
    std::lock_guard<std::mutex> lk(mu);
    return slots[dev];  // (std::map never moves its elements)
}

}  // namespace

qiht_status run_solve_noalloc(const ProblemIn& in, const SolveArgs& a, qiht_info* info, hipStream_t st) {
    int dev = 0;
    QIHT_HIP(hipGetDevice(&dev));
    ScratchSlot& slot = scratch_slot(dev);
    std::lock_guard<std::mutex> lk(slot.run);
    if (!slot.ptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return fail(QIHT_ERR_DEVICE, "no device address for the no-allocation workspace");
        }
        slot.ptr = static_cast<uint8_t*>(p);
    }
    return run_solve(&in, 1, a, info, st, nullptr, slot.ptr,
                     static_cast<size_t>(QIHT_NOALLOC_WORKSPACE_BYTES));
}

std::string tune_report() { return tuner().report(); }

}  // namespace qiht
