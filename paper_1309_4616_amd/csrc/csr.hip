// CSR sweeps (Sec. III-D: unstructured matrices) for gfx950.
//
// `group` lanes share a row (8 for ~27 stored entries per row); each lane
// walks the row with stride `group`, the partial dot products meet by
// cross-lane butterflies, and the group's first lane applies the epilogue
// (sweep.hip lists them).  Rows are assigned to XCDs in contiguous runs, so
// with a locality-preserving row order (e.g. Morton order of graph vertices)
// the gathered vector entries are mostly hits in that XCD's L2.
#include "nonlin.h"
#include "sweep_common.h"

namespace expi {
namespace {

template <int EPI, class TIN, class TOUT, int G>
__global__ __launch_bounds__(kMaxWaves * 64) void csr_sweep(SweepArgs a) {
    using TC = compute_t<TIN, TOUT>;
    if (a.guard && a.st->done != 0) return;
    const TIN* __restrict__ x = static_cast<const TIN*>(a.x);
    TOUT* __restrict__ out = static_cast<TOUT*>(a.out);
    TOUT* __restrict__ p = static_cast<TOUT*>(a.p);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (EPI == EPI_GERSH) {
        s0 = INFINITY;
        s1 = -INFINITY;
    }
    const int g = threadIdx.x / G, sub = threadIdx.x % G;
    const int rows_per = blockDim.x / G;
    // grid-stride over row blocks in XCD-major order: in each pass the
    // workgroups of one XCD take a contiguous run of rows (the gathered
    // entries of neighbouring rows then meet in that XCD's L2), and the grid
    // stays small enough for a short finalize
    // each pass loads the next pass's row pointers ahead of its own entries
    // (clamped to a row that exists, unconditionally), so that they are not
    // a memory round trip of their own at the head of every pass
    const int nrow = a.n[0];
    int L = xcd_tile(a.per_xcd);
    int pa = 0, pb = 0;
    if (nrow > 0) {
        const int r = min(L * rows_per + g, nrow - 1);
        pa = a.rowptr[r];
        pb = a.rowptr[r + 1];
    }
    for (; L < a.ntiles; L += gridDim.x) {
    const int row = L * rows_per + g;
    // row range clamped to [0, nnz) and column indices checked against n, so
    // a malformed matrix cannot send a load out of bounds
    const int e0 = max(pa, 0), e1 = min(pb, a.nnz);
    {
        const int rn = min(min(L + (int)gridDim.x, a.ntiles - 1) * rows_per + g, nrow - 1);
        pa = a.rowptr[rn];
        pb = a.rowptr[rn + 1];
    }
    const unsigned nrows = (unsigned)nrow;
    // Products of the wave's rows (contiguous entries [wb, we)), staged in
    // LDS: every lane of the wave takes consecutive entries, so each index,
    // value and gather instruction covers 64 consecutive entries; the G
    // lanes of a row then sum its products from LDS.  Entries past the
    // first kStage of the wave are taken directly by the row's lanes.
    TC acc = 0;
    if (EPI != EPI_GERSH) {
        constexpr int kStage = 2048 / G;   // 32 entries per row of the wave
        __shared__ TC stage[kMaxWaves][kStage];
        TC* st = stage[threadIdx.x >> 6];
        const int lane = threadIdx.x & 63;
        const int wb = __shfl(e0, 0), we = __shfl(e1, 63);
        const int lastw = max(we - 1, 0);
        const bool any = a.nnz > 0;   // an empty matrix may come without arrays
        constexpr int kQ = kStage / 64;
        int col[kQ];
        TC vv[kQ], xv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int e = min(wb + lane + 64 * q, lastw);   // clamped: no branch
            col[q] = any ? a.colind[e] : 0;
            vv[q] = any ? (TC)a.val[e] : (TC)0;
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const bool ok = (wb + lane + 64 * q < we) && ((unsigned)col[q] < nrows);
            xv[q] = (TC)x[ok ? col[q] : 0];
            st[lane + 64 * q] = ok ? vv[q] * xv[q] : (TC)0;
        }
        // the same wave reads what it wrote: LDS operations of a wave
        // complete in order; the fences keep the compiler from moving them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (row < nrow) {
            const int lo = max(e0 - wb, 0), hi = min(e1 - wb, kStage);
            for (int i = lo + sub; i < hi; i += G) acc += st[i];
            for (int e = max(e0, wb + kStage) + sub; e < e1; e += G) {
                const int c = a.colind[e];
                if ((unsigned)c < nrows) acc += (TC)a.val[e] * (TC)x[c];
            }
        }
        // no wave rewrites its stage before all its lanes have read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (row < nrow) {
        if (EPI == EPI_GERSH) {
            double dg = 0.0, off = 0.0;
            for (int e = e0 + sub; e < e1; e += G) {
                const double v = a.val[e];
                if (a.colind[e] == row) dg += v; else off += fabs(v);
            }
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                dg += __shfl_xor(dg, o, G);
                off += __shfl_xor(off, o, G);
            }
            if (sub == 0) {
                s0 = fmin(s0, dg - off);
                s1 = fmax(s1, dg + off);
            }
        } else {
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
            if (sub == 0) {
                const TC wc = (TC)x[row];
                const TC alpha = (TC)a.alpha, beta = (TC)a.beta;
                if (EPI == EPI_APPLY) {
                    out[row] = (TOUT)(alpha * acc + beta * wc);
                } else if (EPI == EPI_NEWTON) {
                    const TOUT wn = (TOUT)(alpha * acc + beta * wc);
                    const TOUT pn = (TOUT)((TC)p[row] + (TC)a.d1 * (TC)wn);
                    out[row] = wn;
                    p[row] = pn;
                    s1 += (double)wn * (double)wn;
                    s2 += (double)pn * (double)pn;
                } else if (EPI == EPI_FIRST) {
                    const TOUT wn = (TOUT)(alpha * acc + beta * wc);
                    const TOUT pn = (TOUT)((TC)a.d0 * wc + (TC)a.d1 * (TC)wn);
                    out[row] = wn;
                    p[row] = pn;
                    s0 += (double)wc * (double)wc;
                    s1 += (double)wn * (double)wn;
                    s2 += (double)pn * (double)pn;
                } else if (EPI == EPI_START) {
                    TC gv;
                    if (a.gmode == G_VEC) {
                        gv = (TC)a.g[row];
                    } else if (a.gmode == G_VEC_SCALED) {
                        gv = (TC)(a.gscale * a.g[row]);
                    } else if (a.gmode == G_CUBIC_OF) {
                        gv = g_eval<TC>(a.gkind, (TC)a.g[row]);
                    } else {
                        gv = g_eval<TC>(a.gkind, wc);
                    }
                    out[row] = (TOUT)((TC)a.sigma * acc + gv);
                }
            }
        }
    }
    }
    if (EPI == EPI_NEWTON || EPI == EPI_FIRST || EPI == EPI_GERSH) finish_sweep<EPI>(a, s0, s1, s2);
}

template <int EPI, class TIN, class TOUT>
hipError_t go(const Geom& g, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(g.grid), block(64 * g.waves);
    switch (g.vec) {  // lanes per row
        case 4: hipLaunchKernelGGL((csr_sweep<EPI, TIN, TOUT, 4>), grid, block, 0, s, a); break;
        case 16: hipLaunchKernelGGL((csr_sweep<EPI, TIN, TOUT, 16>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((csr_sweep<EPI, TIN, TOUT, 8>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_csr(const Geom& g, int epi, int tin, int tout, const SweepArgs& a, hipStream_t s) {
    switch (epi) {
        case EPI_APPLY:
            if (tin == 0 && tout == 0) return go<EPI_APPLY, double, double>(g, a, s);
            if (tin == 1 && tout == 1) return go<EPI_APPLY, float, float>(g, a, s);
            break;
        case EPI_NEWTON:
            if (tin == 0 && tout == 0) return go<EPI_NEWTON, double, double>(g, a, s);
            if (tin == 1 && tout == 1) return go<EPI_NEWTON, float, float>(g, a, s);
            break;
        case EPI_FIRST:
            if (tin == 0 && tout == 0) return go<EPI_FIRST, double, double>(g, a, s);
            if (tin == 0 && tout == 1) return go<EPI_FIRST, double, float>(g, a, s);
            if (tin == 1 && tout == 1) return go<EPI_FIRST, float, float>(g, a, s);
            break;
        case EPI_START:
            if (tin == 0 && tout == 0) return go<EPI_START, double, double>(g, a, s);
            if (tin == 0 && tout == 1) return go<EPI_START, double, float>(g, a, s);
            if (tin == 1 && tout == 1) return go<EPI_START, float, float>(g, a, s);
            break;
        case EPI_GERSH:
            return go<EPI_GERSH, double, double>(g, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace expi
