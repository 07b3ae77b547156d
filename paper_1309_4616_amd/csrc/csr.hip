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
    const int nrow = a.n[0];
    const unsigned nrows = (unsigned)nrow;
    // Row blocks (rows_per consecutive rows, G lanes each) are taken in
    // grid-stride order over an XCD-major block index: in each pass the
    // workgroups of one XCD take a contiguous run of rows (the gathered
    // entries of neighbouring rows then meet in that XCD's L2), and the grid
    // stays small enough for a short finalize.
    if constexpr (EPI == EPI_GERSH) {
        // interval bounds: each row's lanes walk its entries (once per
        // operator; row range clamped to [0, nnz))
        for (int L = xcd_tile(a.per_xcd); L < a.ntiles; L += gridDim.x) {
            const int row = L * rows_per + g;
            if (row < nrow) {
                const int e0 = max(a.rowptr[row], 0), e1 = min(a.rowptr[row + 1], a.nnz);
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
            }
        }
    } else {
        // Products.  The rows of a wave own one contiguous run of entries
        // [wb, we); a pass takes a chunk of up to kStage of them: every lane
        // takes consecutive entries, so each index, value and gather
        // instruction covers 64 consecutive entries; the products go to a
        // per-wave LDS stage, from which the G lanes of each row sum theirs.
        // A wave whose run is longer takes further passes over the same
        // rows; the row sums are complete after its last chunk.
        //
        // Software pipeline: a pass finds its chunk's column indices and
        // values and the next block's row pointers already in registers; it
        // issues its gathers first and then the loads of the next pass's
        // entries and row pointers, so waiting for the gathers (the memory
        // counter retires in order) never waits for those streaming loads,
        // which stay in flight while the pass computes.  No vector memory
        // access sits in a branch or in a loop of its own inside the pass
        // (the compiler would then wait for every load in flight at the
        // head of the next pass): row indices are clamped into the matrix,
        // loads past a run are clamped to its last entry, and the Newton
        // epilogues store without a branch (below).
        constexpr int kStage = 2048 / G;   // 32 entries per row of the wave
        constexpr int kQ = kStage / 64;
        __shared__ TC stage[kMaxWaves][kStage];
        TC* st = stage[threadIdx.x >> 6];
        const int lane = threadIdx.x & 63;
        const int gsz = (int)gridDim.x;
        // an empty matrix may come without entry arrays: its entry loads
        // then read the first row pointers instead (valid memory, unused)
        const bool any = a.nnz > 0;
        const int* __restrict__ ci = any ? a.colind : a.rowptr;
        const double* __restrict__ va = any ? a.val : reinterpret_cast<const double*>(a.rowptr);
        auto rp_load = [&](int Lx, int& pa_, int& pb_) {
            const int r = min(min(Lx, a.ntiles - 1) * rows_per + g, nrow - 1);
            pa_ = a.rowptr[r];
            pb_ = a.rowptr[r + 1];
        };
        // the wave's run of entries from its lanes' row pointers (row range
        // clamped to [0, nnz), so a malformed matrix cannot send a load out
        // of bounds)
        auto run = [&](int pa_, int pb_, int& wb_, int& we_) {
            wb_ = __shfl(max(pa_, 0), 0);
            we_ = __shfl(min(pb_, a.nnz), 63);
        };
        auto ent_load = [&](int cb_, int we_, int (&col_)[kQ], TC (&vv_)[kQ]) {
            const int lastw = max(we_ - 1, 0);
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = min(cb_ + lane + 64 * q, lastw);
                col_[q] = ci[e];
                vv_[q] = (TC)va[e];
            }
        };
        int L = xcd_tile(a.per_xcd);
        int pa = 0, pb = 0, pa1 = 0, pb1 = 0, cb = 0;
        int col[kQ];
        TC vv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            col[q] = 0;
            vv[q] = 0;
        }
        if (nrow > 0 && L < a.ntiles) {
            int wb0, we0;
            rp_load(L, pa, pb);
            rp_load(L + gsz, pa1, pb1);
            run(pa, pb, wb0, we0);
            cb = wb0;
            ent_load(cb, we0, col, vv);
        }
        TC acc = 0;   // the lane's share of its row's sum over the chunks so far
        while (L < a.ntiles) {
            const int row = L * rows_per + g;
            const int e0 = max(pa, 0), e1 = min(pb, a.nnz);
            int wb, we;
            run(pa, pb, wb, we);
            const int ce = min(cb + kStage, we);
            const bool last = ce >= we;   // the same in the whole wave
            // the row's own entry of x (and of p) for the epilogue
            const int rc = min(row, nrow - 1);
            const TC wc_row = (TC)x[rc];
            const TC p_row = (EPI == EPI_NEWTON) ? (TC)p[rc] : (TC)0;
            // gathers of this chunk
            TC xv[kQ];
            bool ok[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                ok[q] = (cb + lane + 64 * q < ce) && ((unsigned)col[q] < nrows);
                xv[q] = (TC)x[ok[q] ? col[q] : 0];
            }
            // streaming loads for the next pass: the next chunk of this
            // block, or the first chunk of the next block (and the row
            // pointers of the block after it)
            int wbn, wen;
            run(pa1, pb1, wbn, wen);
            const int cbn = last ? wbn : ce;
            int coln[kQ];
            TC vvn[kQ];
            ent_load(cbn, last ? wen : we, coln, vvn);
            int pa2, pb2;
            rp_load(last ? L + 2 * gsz : L + gsz, pa2, pb2);
#pragma unroll
            for (int q = 0; q < kQ; ++q) st[lane + 64 * q] = ok[q] ? vv[q] * xv[q] : (TC)0;
            // the same wave reads what it wrote: LDS operations of a wave
            // complete in order; the fences keep the compiler from moving them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (row < nrow) {
                const int lo = max(e0, cb) - cb, hi = min(e1, ce) - cb;
                for (int i = lo + sub; i < hi; i += G) acc += st[i];
            }
            // no wave rewrites its stage before all its lanes have read it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            TC tot = acc;
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) tot += __shfl_xor(tot, o, G);
            const bool own = last && row < nrow;
            const TC wc = wc_row;
            const TC alpha = (TC)a.alpha, beta = (TC)a.beta;
            if (EPI == EPI_NEWTON || EPI == EPI_FIRST) {
                // every lane of the row's group holds the row's sum and
                // stores the same values; passes before a block's last chunk
                // and rows past the matrix store into the unused fourth word
                // of this workgroup's partials; the norms count the first
                // lane of each row
                const TOUT wn = (TOUT)(alpha * tot + beta * wc);
                const TOUT pn = (EPI == EPI_NEWTON) ? (TOUT)(p_row + (TC)a.d1 * (TC)wn)
                                                    : (TOUT)((TC)a.d0 * wc + (TC)a.d1 * (TC)wn);
                TOUT* spare = reinterpret_cast<TOUT*>(a.partials + 4 * (size_t)blockIdx.x + 3);
                *(own ? out + row : spare) = wn;
                *(own ? p + row : spare) = pn;
                const bool first = own && sub == 0;
                if (EPI == EPI_FIRST) s0 += first ? (double)wc * (double)wc : 0.0;
                s1 += first ? (double)wn * (double)wn : 0.0;
                s2 += first ? (double)pn * (double)pn : 0.0;
            } else if (own && sub == 0) {
                if (EPI == EPI_APPLY) {
                    out[row] = (TOUT)(alpha * tot + beta * wc);
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
                    out[row] = (TOUT)((TC)a.sigma * tot + gv);
                }
            }
            // next pass
            acc = last ? (TC)0 : acc;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                col[q] = coln[q];
                vv[q] = vvn[q];
            }
            cb = cbn;
            pa = last ? pa1 : pa;
            pb = last ? pb1 : pb;
            pa1 = pa2;
            pb1 = pb2;
            L = last ? L + gsz : L;
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
