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
    // stays small enough for a short finalize.
    // Software pipeline: a pass finds its own entries (column indices and
    // values) and the next pass's row pointers already in registers; it
    // issues its gathers first and then the loads of the next pass's
    // entries and of the row pointers of the pass after that, so waiting
    // for the gathers (the memory counter retires in order) never waits for
    // those streaming loads, and they are in flight while the pass
    // computes.  Row indices are clamped into the matrix (unconditional
    // loads).
    const int nrow = a.n[0];
    const unsigned nrows = (unsigned)nrow;
    // an empty matrix may come without entry arrays: its entry loads then
    // read the first row pointers instead (valid memory, values unused), so
    // that no load sits in a branch (the compiler would then wait for every
    // load in flight where the branches meet)
    const bool any = a.nnz > 0;
    const int* __restrict__ ci = any ? a.colind : a.rowptr;
    const double* __restrict__ va = any ? a.val : reinterpret_cast<const double*>(a.rowptr);
    constexpr bool kStaged = (EPI != EPI_GERSH);
    constexpr int kStage = 2048 / G;   // 32 entries per row of the wave
    constexpr int kQ = kStage / 64;
    const int lane = threadIdx.x & 63;
    int L = xcd_tile(a.per_xcd);
    auto rp_load = [&](int Lx, int& pa_, int& pb_) {
        const int r = min(min(Lx, a.ntiles - 1) * rows_per + g, nrow - 1);
        pa_ = a.rowptr[r];
        pb_ = a.rowptr[r + 1];
    };
    // the wave's rows own the contiguous entries [wb, we): every lane takes
    // consecutive ones, so each index, value and gather instruction covers
    // 64 consecutive entries (clamped to the last one: no branch)
    auto ent_load = [&](int pa_, int pb_, int (&col_)[kQ], TC (&vv_)[kQ]) {
        const int wb_ = __shfl(max(pa_, 0), 0), we_ = __shfl(min(pb_, a.nnz), 63);
        const int lastw = max(we_ - 1, 0);
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int e = min(wb_ + lane + 64 * q, lastw);
            col_[q] = ci[e];
            vv_[q] = (TC)va[e];
        }
    };
    int pa = 0, pb = 0, pa1 = 0, pb1 = 0;
    int col[kQ];
    TC vv[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        col[q] = 0;
        vv[q] = 0;
    }
    if (nrow > 0 && L < a.ntiles) {
        rp_load(L, pa, pb);
        rp_load(L + (int)gridDim.x, pa1, pb1);
        if (kStaged) ent_load(pa, pb, col, vv);
    }
    for (; L < a.ntiles; L += gridDim.x) {
    const int row = L * rows_per + g;
    // row range clamped to [0, nnz) and column indices checked against n, so
    // a malformed matrix cannot send a load out of bounds
    const int e0 = max(pa, 0), e1 = min(pb, a.nnz);
    // the row's own entry of x (and of p) for the epilogue, loaded ahead of
    // the gathers (it does not depend on them)
    TC wc_row = 0, p_row = 0;
    if (EPI != EPI_GERSH) {
        const int rc = min(row, nrow - 1);
        wc_row = (TC)x[rc];
        if (EPI == EPI_NEWTON) p_row = (TC)p[rc];
    }
    // Products of the wave's rows, staged in LDS; the G lanes of a row then
    // sum its products from there.  Entries past the first kStage of the
    // wave are taken directly by the row's lanes.
    TC acc = 0;
    int pa2 = 0, pb2 = 0;
    if (kStaged) {
        __shared__ TC stage[kMaxWaves][kStage];
        TC* st = stage[threadIdx.x >> 6];
        const int wb = __shfl(e0, 0), we = __shfl(e1, 63);
        TC xv[kQ];
        bool ok[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            ok[q] = (wb + lane + 64 * q < we) && ((unsigned)col[q] < nrows);
            xv[q] = (TC)x[ok[q] ? col[q] : 0];
        }
        // streaming loads for the passes ahead, issued after the gathers
        int coln[kQ];
        TC vvn[kQ];
        ent_load(pa1, pb1, coln, vvn);
        rp_load(L + 2 * (int)gridDim.x, pa2, pb2);
#pragma unroll
        for (int q = 0; q < kQ; ++q) st[lane + 64 * q] = ok[q] ? vv[q] * xv[q] : (TC)0;
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
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            col[q] = coln[q];
            vv[q] = vvn[q];
        }
    } else {
        rp_load(L + 2 * (int)gridDim.x, pa2, pb2);
    }
    pa = pa1;
    pb = pb1;
    pa1 = pa2;
    pb1 = pb2;
    if (EPI == EPI_NEWTON || EPI == EPI_FIRST) {
        // The Newton epilogues without a branch around their stores (the
        // compiler would otherwise wait, at the head of the next pass, for
        // every load in flight, the streaming ones included): after the
        // butterfly every lane of the row's group holds the row's sum, and
        // all of them store the same values; rows past the matrix (last
        // pass) store into the unused fourth word of this workgroup's
        // partials.  The norms count the first lane of each row.
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        const bool own = row < nrow;
        const TC wc = wc_row;
        const TC alpha = (TC)a.alpha, beta = (TC)a.beta;
        const TOUT wn = (TOUT)(alpha * acc + beta * wc);
        const TOUT pn = (EPI == EPI_NEWTON) ? (TOUT)(p_row + (TC)a.d1 * (TC)wn)
                                            : (TOUT)((TC)a.d0 * wc + (TC)a.d1 * (TC)wn);
        TOUT* spare = reinterpret_cast<TOUT*>(a.partials + 4 * (size_t)blockIdx.x + 3);
        *(own ? out + row : spare) = wn;
        *(own ? p + row : spare) = pn;
        const bool first = own && sub == 0;
        if (EPI == EPI_FIRST) s0 += first ? (double)wc * (double)wc : 0.0;
        s1 += first ? (double)wn * (double)wn : 0.0;
        s2 += first ? (double)pn * (double)pn : 0.0;
    } else if (row < nrow) {
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
                const TC wc = wc_row;
                const TC alpha = (TC)a.alpha, beta = (TC)a.beta;
                if (EPI == EPI_APPLY) {
                    out[row] = (TOUT)(alpha * acc + beta * wc);
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
