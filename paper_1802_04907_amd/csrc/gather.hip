// Column gathers of the QIHT iteration, all in FP64 accumulation:
//
//   G_R      r = y_hat - Q2_G x_G                       -> r32 (FP32)
//   G_MU     u = Q1_G g_G, v = Q2_G g_G                 -> partial u.v, u.u
//   G_OMEGA  w_t = Q1 (x'_t - x) for kSpec proposals    -> partial |w_t|^2
//
// Work split: a workgroup owns 16 bytes (four 32-bit words) of every listed
// column, i.e. a fixed set of rows, and all the listed columns; its 64
// column slots (16 per wave, 4 lanes per slot reading 16 contiguous bytes)
// take the columns slot, slot + 64, ...  The slots are combined by an xor
// butterfly inside each wave and then in wave order through LDS, so each
// row's sum has one fixed order and results are bitwise reproducible.  No
// workgroup waits on another: the per-workgroup partial dot products of
// G_MU and G_OMEGA are finished, in workgroup order, by the next kernel.
// For a single problem, G_R after the first round also takes the step-size
// test of the previous round's proposals: every workgroup computes the same
// pick from the omega partials and gathers the picked proposal's support and
// values, and one extra workgroup commits it (decide_pick, commit_round).
// Batches commit in k_commit before the gather instead (thousands of gather
// workgroups would each repeat the test's round trip).
#include <type_traits>

#include "solve_common.h"

namespace qiht {
namespace {

// The residual rows of row chunk wg (held by threads < 4 RPW, one row each)
// as fixed-point digits for the full pass: the chunk's exponent, the sum of
// its N_i, and its digit words, in the layout the full pass reads.
template <int BITS>
__device__ void digitize_chunk(double r, int wg, const ProbDev& pd) {
    using D = QDig<BITS>;
    constexpr int NR = 4 * D::RPW;  // rows of the chunk, <= 128
    constexpr int NWR = (NR + 63) / 64;
    constexpr int H = D::H;
    __shared__ double smx[NWR];
    __shared__ int ssn[NWR];
    __shared__ int snr[NR];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double m = tid < NR ? fabs(r) : 0.0;
    if (wv < NWR) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        if (lane == 0) smx[wv] = m;
    }
    __syncthreads();
    double mx = smx[0];
#pragma unroll
    for (int w = 1; w < NWR; ++w) mx = fmax(mx, smx[w]);
    int e = 0;
    if (mx > 0.0) {
        int ex;
        frexp(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
        e = ex - 22;     // mx 2^-e in [2^21, 2^22)
    }
    if (wv < NWR) {
        const int nv = tid < NR ? static_cast<int>(rint(ldexp(r, -e))) : 0;
        if (tid < NR) snr[tid] = nv;
        int sn = nv;  // |sum| <= 64 * 2^22
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sn += __shfl_xor(sn, o, 64);
        if (lane == 0) ssn[wv] = sn;
    }
    __syncthreads();
    const size_t words = static_cast<size_t>(pd.nwg) * 4 * H;  // digit words per digit
    if (tid < 4 * H) {  // digit word tid of the chunk: code word tid / H, rows offset tid % H
        const int cw = tid / H, h = tid % H;
        uint32_t u[D::RPD];
#pragma unroll
        for (int t = 0; t < D::RPD; ++t) u[t] = (static_cast<uint32_t>(snr[cw * D::RPW + t * H + h]) + D::OFF) ^ D::OFF;
        transpose_digits<BITS>(u);
#pragma unroll
        for (int d = 0; d < D::ND; ++d) stg(pd.rdig + d * words + static_cast<size_t>(wg) * 4 * H + tid, u[d]);
    }
    if (tid == 0) {
        int sn = ssn[0];
#pragma unroll
        for (int w = 1; w < NWR; ++w) sn += ssn[w];
        stg(pd.rexp + wg, static_cast<int32_t>(e));
        stg(pd.rsum + wg, static_cast<int32_t>(sn));
    }
}

// The residual rows of the RG row chunks of segment seg (chunk k held by
// threads [k NR, (k + 1) NR), NR = 4 RPW <= 64 rows, one row each) as
// fixed-point digits, as digitize_chunk does for one chunk; chunks past the
// last row group (live) are not written.  The chunk's maximum and sum are
// taken over its NR lanes alone (xor offsets below NR).
template <int BITS, int RG>
__device__ void digitize_seg(double r, int seg, const ProbDev& pd) {
    using D = QDig<BITS>;
    constexpr int NR = 4 * D::RPW;
    constexpr int H = D::H;
    static_assert(NR <= 64 && RG * NR <= kGatherThreads, "one chunk per wave at most");
    __shared__ int snr[RG][NR];
    const int tid = threadIdx.x;
    const int k = tid / NR;
    const bool holds = tid < RG * NR;
    double m = holds ? fabs(r) : 0.0;
#pragma unroll
    for (int o = NR / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    int e = 0;
    if (m > 0.0) {
        int ex;
        frexp(m, &ex);  // m = f 2^ex, f in [0.5, 1)
        e = ex - 22;    // m 2^-e in [2^21, 2^22)
    }
    const int nv = holds ? static_cast<int>(rint(ldexp(r, -e))) : 0;
    if (holds) snr[k][tid % NR] = nv;
    int sn = nv;  // |sum| <= 64 * 2^22
#pragma unroll
    for (int o = NR / 2; o > 0; o >>= 1) sn += __shfl_xor(sn, o, 64);
    __syncthreads();
    const int rgi0 = seg * RG;
    const size_t words = static_cast<size_t>(pd.nwg) * 4 * H;  // digit words per digit
    if (tid < RG * 4 * H) {  // digit word of chunk kk: code word j / H, rows offset j % H
        const int kk = tid / (4 * H), j = tid % (4 * H);
        if (rgi0 + kk < pd.nwg) {
            const int cw = j / H, h = j % H;
            uint32_t u[D::RPD];
#pragma unroll
            for (int t = 0; t < D::RPD; ++t) u[t] = (static_cast<uint32_t>(snr[kk][cw * D::RPW + t * H + h]) + D::OFF) ^ D::OFF;
            transpose_digits<BITS>(u);
#pragma unroll
            for (int d = 0; d < D::ND; ++d) stg(pd.rdig + d * words + static_cast<size_t>(rgi0 + kk) * 4 * H + j, u[d]);
        }
    }
    if (holds && tid % NR == 0 && rgi0 + k < pd.nwg) {
        stg(pd.rexp + rgi0 + k, static_cast<int32_t>(e));
        stg(pd.rsum + rgi0 + k, static_cast<int32_t>(sn));
    }
}

// Row group of workgroup x in grid row y.  Workgroups are handed to the
// eight XCDs in turn (linear id mod 8; the grid's width is a multiple of
// 64), and each XCD has its own L2: the eight 16-byte row groups of one
// 128-byte line are given to workgroups on the same XCD, so the line is
// fetched into one L2 only, and the lines rotate over the XCDs with the
// line index and the grid row.
__device__ __forceinline__ int xcd_row_group(int x, int y) {
    const int c = x & 7, i = (x >> 3) & 7;
    return (x & ~63) + 8 * ((c - y) & 7) + i;
}

template <int BITS, int MODE, int RG>
__global__ __launch_bounds__(kGatherThreads) void k_gather(const ProbDev* __restrict__ P,
                                                           SolveArgs a, int zero_x,
                                                           const int2* __restrict__ tab) {
    constexpr int RPW = rows_per_word<BITS>();  // rows per 32-bit word
    constexpr int NSET = (MODE == G_OMEGA) ? kSpec : 1;
    constexpr int NM = (MODE == G_MU) ? 2 : 1;
    constexpr int NW = kGatherThreads / 64;
    // a workgroup owns RG 16-byte row groups (a segment) of every listed
    // column: LPS lanes per column slot, one 32-bit word each
    static_assert(RG == 1 || RG == 2 || RG == 4, "1, 2 or 4 row groups per workgroup");
    static_assert(RG == 1 || (BITS != 9 && BITS != 16), "dense formats take one row group");
    constexpr int LPS = 4 * RG;                 // lanes per slot
    constexpr int SPW = 64 / LPS;               // slots per wave
    constexpr int LB = RG == 1 ? 2 : (RG == 2 ? 3 : 4);  // lowest slot bit of the lane
    constexpr int SLOTS = NW * SPW;
    int bx = blockIdx.x, by = blockIdx.y;
    if (tab) {  // (groups of 64 keep the XCD of a workgroup at bx mod 8)
        const int2 e = tab[blockIdx.x >> 6];
        by = e.x;
        bx = e.y + static_cast<int>(blockIdx.x & 63u);
    }
    const int p = by / NSET;
    const int set = by % NSET;
    const ProbDev& pd = P[p];
    const int wg = xcd_row_group(bx, by);  // segment (RG row groups; with RG = 1 one)
    // G_R after the first round: the last round's step-size test is taken
    // here, by every workgroup alike; one extra workgroup commits it
    __shared__ double s_dec[kSpec * (kGatherThreads / 64)];
    __shared__ int s_done;
    // the state flags and (G_R) the step-size test's inputs in one round trip,
    // before it is known whether a test is due; the stop flag is checked once
    // the column loads are issued (every address stays valid after the solve
    // has stopped)
    const int phase_now = MODE == G_R ? ldg_i32(&pd.st->phase) : 0;
    int done_now = ldg_i32(&pd.st->done);
    PickIn pin;
    if constexpr (MODE == G_R) pin = pick_load<kGatherThreads>(pd);
    const bool decide = MODE == G_R && !zero_x && a.decide_in_gather && phase_now == 1;
    if (MODE == G_R && wg == pd.npart) {
        if (decide && !done_now) commit_round<kGatherThreads>(pd, a, s_dec, pin);
        return;
    }
    if (wg >= pd.npart) return;

    const int32_t* cols;
    int ncols;
    const double* wlist = nullptr;  // per-list-position weights (G_OMEGA)
    const float* wpos = nullptr;    // per-list-position weights (G_R: x on the support)
    const float* wcol = nullptr;    // per-column weights (G_MU: g)
    if (MODE == G_OMEGA) {
        // no omega needed for this proposal, nor for any when the first
        // keeps the support (the test takes it at once); the three flags
        // and the count are loaded together
        const int ch = ldg_i32(&pd.meta[set].changed);
        const int ch0 = ldg_i32(&pd.meta[0].changed);
        const int dcount = ldg_i32(&pd.meta[set].dcount);
        if (!ch || !ch0) return;
        ncols = dcount;
        cols = pd.dlist + static_cast<size_t>(set) * 2 * pd.s;
        wlist = pd.dw + static_cast<size_t>(set) * 2 * pd.s;
    } else {
        cols = pd.sup;
        ncols = (MODE == G_R && zero_x) ? 0 : pd.s;
        if (MODE == G_R) wpos = pd.xs;
        else wcol = pd.g;
    }
    if (MODE == G_R && decide) {
        // The commit workgroup of this launch may stop the problem while the
        // others run: thread 0's reading of the flag, passed on through LDS
        // across the test's barrier, is the one every wave acts on.
        if (threadIdx.x == 0) s_done = done_now;
        // the picked proposal's support and values (after a failed test the
        // current ones: the next round proposes further shrinks from this x)
        bool capped;
        const int pick = decide_pick<kGatherThreads>(pd, a, &capped, s_dec, pin);
        done_now = s_done;
        if (done_now) return;  // uniform over the workgroup
        if (pick >= 0) {
            cols = pd.csup + static_cast<size_t>(pick) * pd.s;
            wpos = pd.cval + static_cast<size_t>(pick) * pd.s;
        }
    }
    // (one copy of the matrix: Q2_G g_G = Q1_G g_G, read once)
    const bool two = (MODE == G_MU) && (a.mu_mode == 0) && (pd.q1 != pd.q2);
    // the candidate compaction's inputs go out with the gather's loads
    CandPre<kGatherThreads> cpre;
    if constexpr (MODE == G_MU) cpre = cand_preload<kGatherThreads>(pd, wg, pd.npart, true);
    const uint8_t* A = (MODE == G_R) ? pd.q2 : pd.q1;
    const uint8_t* B = pd.q2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int w = lane % LPS;                  // word within the segment
    const int slot = wv * SPW + lane / LPS;    // column slot
    // (a word past the column's last row group reads its last word; those
    // rows are not written)
    const size_t woff = min(static_cast<size_t>(wg) * 16 * RG + static_cast<size_t>(w) * 4,
                            static_cast<size_t>(pd.col_bytes) - 4);

    double acc[NM][RPW];
#pragma unroll
    for (int mi = 0; mi < NM; ++mi)
#pragma unroll
        for (int q = 0; q < RPW; ++q) acc[mi][q] = 0.0;
    double wsum = 0.0;

    // One step over U list positions per slot.  Every load of a step is
    // issued unconditionally (a position past the end reads the last entry
    // and gets weight 0), so that its loads are in flight together.  The
    // step length is picked per wave (8, 4, 2 or 1 positions, the fewest
    // covering what is left for its lowest slot), so that no step loads and
    // sums positions no lane of the wave has; the sums run over each lane's
    // positions in the same order whatever the steps.
    bool stop = false;
    auto step = [&](int t0, auto u_c) {
        constexpr int U = decltype(u_c)::value;
        int cidx[U];
        bool valid[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + SLOTS * u;
            valid[u] = t < ncols;
            cidx[u] = static_cast<int>(ldg_u32(cols + min(t, ncols - 1)));
        }
        if (done_now) {  // uniform over the workgroup
            stop = true;
            return;
        }
        double wt[U];
        uint32_t wa[U], wb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(t0 + SLOTS * u, ncols - 1);
            double wv;
            if (MODE == G_OMEGA) wv = ldg_f64(wlist + t);
            else if (MODE == G_R) wv = static_cast<double>(ldg_f32(wpos + t));
            else wv = static_cast<double>(ldg_f32(wcol + cidx[u]));
            wt[u] = valid[u] ? wv : 0.0;
            const size_t off = static_cast<size_t>(cidx[u]) * pd.col_bytes + woff;
            wa[u] = ldg_u32(A + off);
            wb[u] = two ? ldg_u32(B + off) : 0u;
        }
        // g on the support, compact (stored once every load above has been
        // issued: a store between them would serialize the loads)
        if (MODE == G_MU && wg == 0 && w == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (valid[u]) stg(pd.gs + t0 + SLOTS * u, static_cast<float>(wt[u]));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wsum += wt[u];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const double va = elem_at<BITS>(wa[u], q);
                acc[0][q] = fma(wt[u], va, acc[0][q]);
                if (NM == 2) {
                    const double vb = elem_at<BITS>(wb[u], q);
                    acc[NM - 1][q] = fma(wt[u], vb, acc[NM - 1][q]);
                }
            }
        }
    };
    for (int t0 = slot; t0 < ncols && !stop;) {
        // positions left for the wave's lowest slot (its lane 0)
        const int left = __builtin_amdgcn_readfirstlane((ncols - (t0 - lane / LPS) + SLOTS - 1) / SLOTS);
        if (left > 4) {
            step(t0, std::integral_constant<int, 8>{});
            t0 += SLOTS * 8;
        } else if (left > 2) {
            step(t0, std::integral_constant<int, 4>{});
            t0 += SLOTS * 4;
        } else if (left > 1) {
            step(t0, std::integral_constant<int, 2>{});
            t0 += SLOTS * 2;
        } else {
            step(t0, std::integral_constant<int, 1>{});
            t0 += SLOTS;
        }
    }
    if (stop) return;
    if (done_now) return;  // (a workgroup whose lanes had no list entries)
    // ---- sum over the slots of the wave (lane bits LB..5), the NM RPW row
    // sums of each word halving at every exchange (lane 0 holds the weight
    // sum)
    if constexpr (RG == 1) wsum = slot_sum(wsum);
    else wsum = slot_total<LB>(wsum, lane);
    constexpr int V = NM * RPW;
    double v[V];
#pragma unroll
    for (int mi = 0; mi < NM; ++mi)
#pragma unroll
        for (int q = 0; q < RPW; ++q) v[mi * RPW + q] = acc[mi][q];
    int vbase = 0, vdup = 0;
    slot_sums_halving<V, LB>(v, lane, &vbase, &vdup);
    // ---- then the waves, in wave order
    __shared__ double sh[NW][LPS][NM][RPW];
    __shared__ double shw[NW];
    __shared__ double shr[NW];
    if ((lane & vdup) == 0) {
        constexpr int C = V >= SPW ? V / SPW : 1;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int idx = vbase + i;
            sh[wv][lane % LPS][idx / RPW][idx % RPW] = v[i];
        }
    }
    if (lane == 0) shw[wv] = wsum;
    __syncthreads();
    double wtot = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) wtot += shw[v];
    double l1 = 0.0, l2 = 0.0, rres = 0.0;
    static_assert(LPS * RPW <= kGatherThreads, "one thread per row of the segment");
    // (rows of a row group past the column's last: not written)
    const bool exists = threadIdx.x < LPS * RPW && wg * RG + static_cast<int>(threadIdx.x) / (4 * RPW) < pd.nwg;
    if (exists) {
        const int ww = threadIdx.x / RPW, q = threadIdx.x % RPW;
        const size_t row = (static_cast<size_t>(wg) * LPS + ww) * RPW + q;
        double val[NM];
#pragma unroll
        for (int mi = 0; mi < NM; ++mi) {
            double tot = 0.0;
#pragma unroll
            for (int v = 0; v < NW; ++v) tot += sh[v][ww][mi][q];
            if constexpr (BITS == 32) val[mi] = tot;
            else if constexpr (BITS == 9 || BITS == 16)
                val[mi] = row < static_cast<size_t>(pd.rows) ? ldexp(tot, pd.rowexp[row]) : 0.0;
            else val[mi] = pd.alpha * tot + pd.beta * wtot;
        }
        const bool live = row < static_cast<size_t>(pd.rows);
        if (MODE == G_R) {
            rres = live ? ldg_f64(pd.yhat + row) - val[0] : 0.0;
            stg(pd.r32 + row, static_cast<float>(rres));
        } else if (live) {
            if (MODE == G_MU) {
                l1 = two ? val[0] * val[NM - 1] : val[0] * val[0];
                l2 = val[0] * val[0];
            } else {
                l1 = val[0] * val[0];
            }
        }
    }
    if constexpr (MODE == G_R) {
        if constexpr (BITS <= 8 && RG > 1) {
            digitize_seg<BITS, RG>(rres, wg, pd);
        } else if constexpr (BITS <= 8) {
            digitize_chunk<BITS>(rres, wg, pd);
        } else if constexpr (BITS == 9 || BITS == 16) {
            // the GEMM's operand: 2^e r as a pair of BF16 (hi + lo), both
            // rounded to nearest even from the exact FP64 value
            if (threadIdx.x < 4 * RPW) {
                const size_t row = (static_cast<size_t>(wg) * 4 + threadIdx.x / RPW) * RPW + threadIdx.x % RPW;
                const double v = row < static_cast<size_t>(pd.rows) ? ldexp(rres, pd.rowexp[row]) : 0.0;
                const uint32_t hi = bf16_rne(v);
                const uint32_t lo = bf16_rne(v - static_cast<double>(bf16_value(hi)));
                const size_t rp = static_cast<size_t>(pd.nwg) * 4 * RPW;  // rows_pad
                pd.rb[row] = static_cast<uint16_t>(hi);
                pd.rb[rp + row] = static_cast<uint16_t>(lo);
            }
        }
        return;
    }
    // rows of this group: at most 4 * RPW <= 128 threads hold values
    const double s1 = block_sum<kGatherThreads>(l1, shr);
    if (MODE == G_MU) {
        const double s2 = block_sum<kGatherThreads>(l2, shr);
        if (threadIdx.x == 0) {
            stg(pd.part_mu + 2 * wg + 0, s1);
            stg(pd.part_mu + 2 * wg + 1, s2);
        }
    } else if (threadIdx.x == 0) {
        stg(pd.part_om + static_cast<size_t>(set) * pd.nwg + wg, s1);
    }
    // g is final here: the off-support candidates of this iteration's proposals
    if constexpr (MODE == G_MU) compact_candidates<kGatherThreads>(pd, wg, pd.npart, true, cpre);
}


// ---------------------------------------------------------------------------
// Wide gathers for a batch on one shared dense-format or FP32 matrix (one
// copy: Q1 = Q2).  Hundreds of problems each list hundreds of columns, so
// the gathers move gigabytes per iteration and must run at bandwidth rather
// than latency: a workgroup owns a 1 KB row segment of every listed column
// (each lane one 16-byte piece: one coalesced 1 KB read per wave and
// column), its four waves take the listed columns w, w + 4, ..., and the
// list itself (indices and weights) is staged through LDS first.  Rows are
// summed per lane in FP64, then over the waves in wave order (fixed order,
// bitwise reproducible).  Partials and candidate lists are per segment
// (npart of them; the last segment of a column may be partial).
// ---------------------------------------------------------------------------
constexpr int kWideBytes = 1024;
constexpr int kWideList = 1024;  // list entries staged at once

template <int BITS, int MODE>
__global__ __launch_bounds__(kGatherThreads) void k_gather_wide(const ProbDev* __restrict__ P,
                                                                SolveArgs a, int zero_x) {
    constexpr int RPW = rows_per_word<BITS>();
    constexpr int NV = 4;               // words per lane
    constexpr int NA = NV * RPW;        // rows per lane
    constexpr int NSET = (MODE == G_OMEGA) ? kSpec : 1;
    constexpr int NW = kGatherThreads / 64;
    constexpr int NR = 64 * NA;         // rows of the segment
    constexpr int U = 8;  // column loads in flight per lane
    const int p = blockIdx.y / NSET;
    const int set = blockIdx.y % NSET;
    const ProbDev& pd = P[p];
    const int wg = blockIdx.x;  // 1 KB row segment
    // G_R after the first round: the last round's step-size test (as in
    // k_gather).  Its commit workgroup may stop the problem while the others
    // run, so those act on thread 0's reading of the flag, passed on through
    // LDS across the test's barrier; without a test nothing changes the flag
    // during the launch.
    __shared__ double s_dec[kSpec * (kGatherThreads / 64)];
    __shared__ int s_done;
    const bool decide = MODE == G_R && !zero_x && a.decide_in_gather && pd.st->phase == 1;
    const int done_now = pd.st->done;
    if (MODE == G_R && wg == pd.npart) {
        if (decide && !done_now) commit_round<kGatherThreads>(pd, a, s_dec);
        return;
    }
    if (wg >= pd.npart) return;
    if (!decide && done_now) return;

    const int32_t* cols;
    const float* xw = pd.xs;  // G_R: x on the listed columns
    int ncols;
    if (MODE == G_OMEGA) {
        const int ch = ldg_i32(&pd.meta[set].changed);  // as in k_gather
        const int ch0 = ldg_i32(&pd.meta[0].changed);
        const int dcount = ldg_i32(&pd.meta[set].dcount);
        if (!ch || !ch0) return;
        ncols = dcount;
        cols = pd.dlist + static_cast<size_t>(set) * 2 * pd.s;
    } else {
        cols = pd.sup;
        ncols = (MODE == G_R && zero_x) ? 0 : pd.s;
    }
    if (MODE == G_R && decide) {
        if (threadIdx.x == 0) s_done = done_now;
        bool capped;
        const int pick = decide_pick<kGatherThreads>(pd, a, &capped, s_dec);
        if (s_done) return;  // uniform over the workgroup
        if (pick >= 0) {
            cols = pd.csup + static_cast<size_t>(pick) * pd.s;
            xw = pd.cval + static_cast<size_t>(pick) * pd.s;
        }
    }
    CandPre<kGatherThreads> cpre;
    if constexpr (MODE == G_MU) cpre = cand_preload<kGatherThreads>(pd, wg, pd.npart, true);
    const uint8_t* A = pd.q1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // a lane past the end of the column reads its last piece (those rows are not used)
    const size_t woff = min(static_cast<size_t>(wg) * kWideBytes + static_cast<size_t>(lane) * 16,
                            static_cast<size_t>(pd.col_bytes) - 16);
    const size_t rows_pad = static_cast<size_t>(pd.nwg) * 4 * RPW;

    // LDS: the staged list during the loads, then the per-wave row sums
    constexpr size_t kListBytes = kWideList * (sizeof(int32_t) + sizeof(double));
    constexpr size_t kSumBytes = sizeof(double) * NW * 64 * (NA + 1);
    __shared__ __align__(16) uint8_t lds_raw[kListBytes > kSumBytes ? kListBytes : kSumBytes];
    double* lw = reinterpret_cast<double*>(lds_raw);
    int32_t* lidx = reinterpret_cast<int32_t*>(lds_raw + kWideList * sizeof(double));
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    for (int base = 0; base < ncols; base += kWideList) {
        const int cnt = min(kWideList, ncols - base);
        for (int i = tid; i < cnt; i += kGatherThreads) {
            const int c = static_cast<int>(ldg_u32(cols + base + i));
            double w;
            if (MODE == G_OMEGA) w = ldg_f64(pd.dw + static_cast<size_t>(set) * 2 * pd.s + base + i);
            else if (MODE == G_R) w = static_cast<double>(ldg_f32(xw + base + i));
            else w = static_cast<double>(ldg_f32(pd.g + c));
            lidx[i] = c;
            lw[i] = w;
            if (MODE == G_MU && wg == 0) pd.gs[base + i] = static_cast<float>(w);  // g on the support
        }
        __syncthreads();
        for (int t0 = wv; t0 < cnt; t0 += NW * U) {
            uint4 wa[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int tc = min(t0 + NW * u, cnt - 1);
                wa[u] = ldg_u4(A + static_cast<size_t>(lidx[tc]) * pd.col_bytes + woff);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + NW * u;
                const double wt = t < cnt ? lw[min(t, cnt - 1)] : 0.0;
                const uint32_t w4[NV] = {wa[u].x, wa[u].y, wa[u].z, wa[u].w};
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int q = 0; q < RPW; ++q) acc[v * RPW + q] = fma(wt, elem_at<BITS>(w4[v], q), acc[v * RPW + q]);
            }
        }
        __syncthreads();
    }
    // ---- waves in wave order; thread t then holds rows t, t + 256, ... of the segment
    // (the last __syncthreads of the loop retired the list)
    double (*sh)[64][NA + 1] = reinterpret_cast<double (*)[64][NA + 1]>(lds_raw);
    __shared__ double shr[NW];
#pragma unroll
    for (int q = 0; q < NA; ++q) sh[wv][lane][q] = acc[q];
    __syncthreads();
    double l1 = 0.0;
    for (int rr = tid; rr < NR; rr += kGatherThreads) {
        const size_t row = static_cast<size_t>(wg) * NR + rr;
        if (row >= rows_pad) break;
        const bool live = row < static_cast<size_t>(pd.rows);
        double tot = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) tot += sh[v][rr / NA][rr % NA];
        double val;
        if constexpr (BITS == 32) val = tot;
        else val = live ? ldexp(tot, pd.rowexp[row]) : 0.0;
        if constexpr (MODE == G_R) {
            const double rres = live ? ldg_f64(pd.yhat + row) - val : 0.0;
            pd.r32[row] = static_cast<float>(rres);
            if constexpr (BITS == 9 || BITS == 16) {
                // the GEMM's operand: 2^e r as a pair of BF16 (hi + lo)
                const double v = live ? ldexp(rres, pd.rowexp[row]) : 0.0;
                const uint32_t hi = bf16_rne(v);
                const uint32_t lo = bf16_rne(v - static_cast<double>(bf16_value(hi)));
                pd.rb[row] = static_cast<uint16_t>(hi);
                pd.rb[rows_pad + row] = static_cast<uint16_t>(lo);
            }
        } else if (live) {
            l1 += val * val;
        }
    }
    if constexpr (MODE == G_R) return;
    const double s1 = block_sum<kGatherThreads>(l1, shr);
    if (MODE == G_MU) {
        if (tid == 0) {
            pd.part_mu[2 * wg + 0] = s1;  // u.v with v = u (one copy of the matrix)
            pd.part_mu[2 * wg + 1] = s1;
        }
        compact_candidates<kGatherThreads>(pd, wg, pd.npart, true, cpre);
    } else if (tid == 0) {
        pd.part_om[static_cast<size_t>(set) * pd.nwg + wg] = s1;
    }
}

template <int MODE>
void launch_mode(int bits, const ProbDev* P, int count, int maxwg, const SolveArgs& a,
                 int zero_x, bool wide, hipStream_t st, const GatherGrid& gg) {
    const int nset = (MODE == G_OMEGA) ? kSpec : 1;
    // G_R: one more workgroup per problem, the commit of the last round's step
    const int extra = MODE == G_R ? 1 : 0;
    if (wide) {
        dim3 gw((maxwg * 16 + kWideBytes - 1) / kWideBytes + extra, count * nset);
        switch (bits) {
            case 9: hipLaunchKernelGGL((k_gather_wide<9, MODE>), gw, dim3(kGatherThreads), 0, st, P, a, zero_x); break;
            case 16: hipLaunchKernelGGL((k_gather_wide<16, MODE>), gw, dim3(kGatherThreads), 0, st, P, a, zero_x); break;
            default: hipLaunchKernelGGL((k_gather_wide<32, MODE>), gw, dim3(kGatherThreads), 0, st, P, a, zero_x); break;
        }
        return;
    }
    const dim3 grid = gg.tab ? dim3(static_cast<unsigned>(gg.ngroups) * 64u, 1u)
                             : dim3((maxwg + extra + 63) / 64 * 64, count * nset);
    const int2* tab = gg.tab;
    if (gg.rg == 4) {  // (batches: 2, 4, 8 bits and FP32; make_plan picks it)
        switch (bits) {
            case 2: hipLaunchKernelGGL((k_gather<2, MODE, 4>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
            case 4: hipLaunchKernelGGL((k_gather<4, MODE, 4>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
            case 8: hipLaunchKernelGGL((k_gather<8, MODE, 4>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
            default: hipLaunchKernelGGL((k_gather<32, MODE, 4>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        }
        return;
    }
    switch (bits) {
        case 1: hipLaunchKernelGGL((k_gather<1, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        case 2: hipLaunchKernelGGL((k_gather<2, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        case 4: hipLaunchKernelGGL((k_gather<4, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        case 8: hipLaunchKernelGGL((k_gather<8, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        case 9: hipLaunchKernelGGL((k_gather<9, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        case 16: hipLaunchKernelGGL((k_gather<16, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
        default: hipLaunchKernelGGL((k_gather<32, MODE, 1>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, tab); break;
    }
}

}  // namespace

void launch_gather(int mode, int bits, const ProbDev* P, int count, int maxwg, const SolveArgs& a,
                   int zero_x, bool wide, hipStream_t st, const GatherGrid& gg) {
    switch (mode) {
        case G_R: launch_mode<G_R>(bits, P, count, maxwg, a, zero_x, wide, st, gg); break;
        case G_MU: launch_mode<G_MU>(bits, P, count, maxwg, a, 0, wide, st, gg); break;
        default: launch_mode<G_OMEGA>(bits, P, count, maxwg, a, 0, wide, st, gg); break;
    }
}

}  // namespace qiht
