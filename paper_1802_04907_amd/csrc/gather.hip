// Column gathers of the QIHT iteration, all in FP64 accumulation:
//
//   G_R      r = y_hat - Q2_G x_G                       -> r32 (FP32)
//   G_MU     u = Q1_G g_G, v = Q2_G g_G                 -> mu (Eq. step_size)
//   G_OMEGA  w_t = Q1 (x'_t - x) for kSpec proposals    -> omega_t, then the
//            step test picks the accepted proposal and commits it
//
// Work split: a workgroup owns one 256-byte row block (each lane one 32-bit
// word of every listed column, so a wave reads 256 contiguous bytes per
// column) and one group of `cpg` listed columns; its four waves split the
// group.  Partial row sums go to a [set][group][row] buffer; the last
// workgroup to finish a row block (arrival counter) adds the groups in group
// order, the last row block of a set finishes the set, and for G_OMEGA the
// last set takes the decision.  Every sum has a fixed order, so results are
// bitwise reproducible; no floating-point atomics are used.
#include "solve_common.h"

namespace qiht {
namespace {

template <int BITS, int MODE>
__global__ __launch_bounds__(kGatherThreads) void k_gather(const ProbDev* __restrict__ P,
                                                           SolveArgs a, int zero_x, int cpg) {
    constexpr int RPW = (BITS == 32) ? 1 : 32 / BITS;  // rows per 32-bit word
    constexpr int NSET = (MODE == G_OMEGA) ? kSpec : 1;
    constexpr int NM = (MODE == G_MU) ? 2 : 1;
    constexpr int CH = RPW < 4 ? RPW : 4;
    constexpr int NW = kGatherThreads / 64;
    const int p = blockIdx.z / NSET;
    const int set = blockIdx.z % NSET;
    const ProbDev& pd = P[p];
    SolveState* st = pd.st;
    if (st->done) return;
    const int rb = blockIdx.x, cg = blockIdx.y;
    if (rb >= pd.nrb) return;

    const int32_t* cols;
    int ncols;
    const double* wlist = nullptr;  // per-list-position weights (G_OMEGA)
    const float* wcol = nullptr;    // per-column weights (G_R: x, G_MU: g)
    if (MODE == G_OMEGA) {
        const CandMeta& m = pd.meta[set];
        ncols = m.changed ? m.dcount : 0;
        cols = pd.dlist + static_cast<size_t>(set) * 2 * pd.s;
        wlist = pd.dw + static_cast<size_t>(set) * 2 * pd.s;
    } else {
        cols = pd.sup;
        ncols = (MODE == G_R && zero_x) ? 0 : pd.s;
        wcol = (MODE == G_R) ? pd.x : pd.g;
    }
    const int geff = ncols > 0 ? (ncols + cpg - 1) / cpg : 1;
    if (cg >= geff) return;
    const bool two = (MODE == G_MU) && (a.mu_mode == 0);
    const uint8_t* A = (MODE == G_R) ? pd.q2 : pd.q1;
    const uint8_t* B = pd.q2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t woff = (static_cast<size_t>(rb) * 64 + lane) * 4;
    const int c0 = cg * cpg;
    const int c1 = min(ncols, c0 + cpg);

    double acc[NM][RPW];
#pragma unroll
    for (int mi = 0; mi < NM; ++mi)
#pragma unroll
        for (int q = 0; q < RPW; ++q) acc[mi][q] = 0.0;
    double wsum = 0.0;

    constexpr int U = 8;
    for (int t0 = c0 + wv; t0 < c1; t0 += NW * U) {
        int cidx[U];
        double wt[U];
        uint32_t wa[U], wb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + NW * u;
            cidx[u] = t < c1 ? cols[t] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + NW * u;
            wt[u] = 0.0;
            wa[u] = 0u;
            wb[u] = 0u;
            if (cidx[u] >= 0) {
                wt[u] = (MODE == G_OMEGA) ? wlist[t] : static_cast<double>(wcol[cidx[u]]);
                const size_t off = static_cast<size_t>(cidx[u]) * pd.col_bytes + woff;
                wa[u] = *reinterpret_cast<const uint32_t*>(A + off);
                if (two) wb[u] = *reinterpret_cast<const uint32_t*>(B + off);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wsum += wt[u];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const double va = (BITS == 32) ? static_cast<double>(__uint_as_float(wa[u]))
                                               : static_cast<double>(code_at<BITS>(wa[u], q));
                acc[0][q] = fma(wt[u], va, acc[0][q]);
                if (NM == 2) {
                    const double vb = (BITS == 32) ? static_cast<double>(__uint_as_float(wb[u]))
                                                   : static_cast<double>(code_at<BITS>(wb[u], q));
                    acc[NM - 1][q] = fma(wt[u], vb, acc[NM - 1][q]);
                }
            }
        }
    }

    // ---- combine the four waves in wave order, write this group's partials
    __shared__ double sh[NW][NM][CH][64];
    __shared__ double shw[NW];
    __shared__ double shr[NW];
    __shared__ int s_last;
    if (lane == 0) shw[wv] = wsum;
    const size_t rows_pad = static_cast<size_t>(pd.nrb) * 64 * RPW;
    const size_t gbase = static_cast<size_t>(set) * pd.gmax + cg;
    for (int q0 = 0; q0 < RPW; q0 += CH) {
#pragma unroll
        for (int mi = 0; mi < NM; ++mi)
#pragma unroll
            for (int qq = 0; qq < CH; ++qq) sh[wv][mi][qq][lane] = acc[mi][q0 + qq];
        __syncthreads();
        if (threadIdx.x < 64 * CH) {
            const int qq = threadIdx.x >> 6, ln = threadIdx.x & 63;
            const size_t row = (static_cast<size_t>(rb) * 64 + ln) * RPW + q0 + qq;
#pragma unroll
            for (int mi = 0; mi < NM; ++mi) {
                double tot = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) tot += sh[w][mi][qq][ln];
                pd.part1[(gbase * NM + mi) * rows_pad + row] = tot;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double wt = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) wt += shw[w];
        pd.wsum1[gbase] = wt;
        __threadfence();
        const unsigned prev = atomicAdd(&pd.cnt1[set * pd.nrb + rb], 1u);
        s_last = (prev == static_cast<unsigned>(geff - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    // ---- last group of this row block: rows of the block in group order
    const size_t gset = static_cast<size_t>(set) * pd.gmax;
    double wtot = 0.0;
    for (int g = 0; g < geff; ++g) wtot += pd.wsum1[gset + g];
    double l1 = 0.0, l2 = 0.0;
    for (int i = threadIdx.x; i < 64 * RPW; i += kGatherThreads) {
        const size_t row = static_cast<size_t>(rb) * 64 * RPW + i;
        double val[NM];
#pragma unroll
        for (int mi = 0; mi < NM; ++mi) {
            double tot = 0.0;
            for (int g = 0; g < geff; ++g)
                tot += pd.part1[((gset + g) * NM + mi) * rows_pad + row];
            val[mi] = (BITS == 32) ? tot : pd.alpha * tot + pd.beta * wtot;
        }
        const bool live = row < static_cast<size_t>(pd.rows);
        if (MODE == G_R) {
            pd.r32[row] = live ? static_cast<float>(pd.yhat[row] - val[0]) : 0.0f;
        } else if (live) {
            if (MODE == G_MU) {
                l1 += two ? val[0] * val[NM - 1] : val[0] * val[0];
                l2 += val[0] * val[0];
            } else {
                l1 += val[0] * val[0];
            }
        }
    }
    if (threadIdx.x == 0) pd.cnt1[set * pd.nrb + rb] = 0u;
    if (MODE == G_R) return;

    const double s1 = block_sum<kGatherThreads>(l1, shr);
    const double s2 = (MODE == G_MU) ? block_sum<kGatherThreads>(l2, shr) : 0.0;
    if (threadIdx.x == 0) {
        pd.part2[(static_cast<size_t>(set) * pd.nrb + rb) * 2 + 0] = s1;
        pd.part2[(static_cast<size_t>(set) * pd.nrb + rb) * 2 + 1] = s2;
        __threadfence();
        const unsigned prev = atomicAdd(&pd.cnt2[set], 1u);
        s_last = (prev == static_cast<unsigned>(pd.nrb - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    // ---- last row block of this set
    double d1 = 0.0, d2 = 0.0;
    for (int b = 0; b < pd.nrb; ++b) {
        d1 += pd.part2[(static_cast<size_t>(set) * pd.nrb + b) * 2 + 0];
        d2 += pd.part2[(static_cast<size_t>(set) * pd.nrb + b) * 2 + 1];
    }
    if (MODE == G_MU) {
        double gg = 0.0;
        for (int t = threadIdx.x; t < pd.s; t += kGatherThreads) {
            const double v = static_cast<double>(pd.g[pd.sup[t]]);
            gg += v * v;
        }
        const double num = block_sum<kGatherThreads>(gg, shr);
        if (threadIdx.x == 0) {
            pd.cnt2[set] = 0u;
            double den = d1;
            if (!(den > 0.0) || !isfinite(den)) den = d2;
            if (!(num > 0.0) || !(den > 0.0) || !isfinite(num / den)) {
                st->done = 1;
                st->reason = QIHT_REASON_STATIONARY;
            } else {
                st->mu = num / den;
                st->base_k = 0;
                st->phase = 0;
            }
        }
        return;
    }
    // G_OMEGA
    if (threadIdx.x == 0) {
        pd.cnt2[set] = 0u;
        CandMeta* m = &pd.meta[set];
        m->omega = d1 > 0.0 ? m->dx2 / d1 : INFINITY;
        __threadfence();
        const unsigned prev = atomicAdd(pd.cnt3, 1u);
        s_last = (prev == static_cast<unsigned>(NSET - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // ---- last set: the step-size test over the kSpec proposals
    __shared__ int s_pick, s_cap;
    if (threadIdx.x == 0) {
        *pd.cnt3 = 0u;
        bool capped = false;
        s_pick = choose_proposal(pd, a, &capped);
        s_cap = capped;
        if (s_pick < 0) {
            st->phase = 2;
            st->base_k = kSpec;
        }
    }
    __syncthreads();
    if (s_pick >= 0) commit_proposal<kGatherThreads>(pd, s_pick, a, s_cap != 0);
}

template <int MODE>
void launch_mode(int bits, const ProbDev* P, int count, int maxrb, int gmax, const SolveArgs& a,
                 int zero_x, int cpg, hipStream_t st) {
    const int nset = (MODE == G_OMEGA) ? kSpec : 1;
    dim3 grid(maxrb, gmax, count * nset);
    switch (bits) {
        case 1: hipLaunchKernelGGL((k_gather<1, MODE>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, cpg); break;
        case 2: hipLaunchKernelGGL((k_gather<2, MODE>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, cpg); break;
        case 4: hipLaunchKernelGGL((k_gather<4, MODE>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, cpg); break;
        case 8: hipLaunchKernelGGL((k_gather<8, MODE>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, cpg); break;
        default: hipLaunchKernelGGL((k_gather<32, MODE>), grid, dim3(kGatherThreads), 0, st, P, a, zero_x, cpg); break;
    }
}

}  // namespace

// Columns per workgroup: the gathered lists hold up to s (G_R, G_MU) or 2s
// (G_OMEGA) columns; `gmax` groups of `cpg` columns cover the longest list.
void launch_gather(int mode, int bits, const ProbDev* P, int count, int maxrb, int gmax,
                   const SolveArgs& a, int zero_x, hipStream_t st) {
    switch (mode) {
        case G_R: launch_mode<G_R>(bits, P, count, maxrb, gmax, a, zero_x, kGatherCpg, st); break;
        case G_MU: launch_mode<G_MU>(bits, P, count, maxrb, gmax, a, 0, kGatherCpg, st); break;
        default: launch_mode<G_OMEGA>(bits, P, count, maxrb, gmax, a, 0, kGatherCpg, st); break;
    }
}

}  // namespace qiht
