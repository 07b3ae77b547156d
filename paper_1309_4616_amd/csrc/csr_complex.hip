// Complex CSR sweeps (K = C in Sec. II-C eq. (3); the Hermitian spin-bath
// matrix of Sec. III-D is stored in the generic CSR format) for gfx950.
//
// Values and vectors are complex128 stored as interleaved (re, im) pairs of
// float64 (16 bytes), columns int32.  For phi_k(-i tau H) the Newton
// recurrence applies (alpha H + beta_j I) with REAL alpha = 1/gamma and
// beta_j = -(c/gamma + xi_j) to complex vectors ([a, b] the real interval
// of the Hermitian H), and only the divided differences d_j are complex;
// the start vector of a phi_1 substep is r = (-i tau) H y + v.
//
// `G` lanes share a row (1, 2, 4, 8 or 16; 4 by default: the paper found
// four threads per row best for its spin system with about 40 entries per
// row; with one lane per row the lanes of a wave hold consecutive rows,
// whose k-th entries of a spin system flip the same spins, so their gathers
// land in the same lines); each lane
// walks the row with stride G, so the G lanes read G consecutive 16-byte
// values per instruction, the partial sums meet by cross-lane butterflies
// and the row's first lane applies the epilogue.  Rows are taken in
// grid-stride passes over row blocks in XCD-major order (the kernel grid
// stays within the CSR bound so the finalize sums few partials).
#include "sweep_common.h"

namespace expi {
namespace {

typedef double cplx __attribute__((ext_vector_type(2)));   // (re, im)

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    cplx r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }

template <int EPI, int G>
__global__ __launch_bounds__(kMaxWaves * 64) void csr_complex_sweep(SweepArgs a) {
    if (a.guard && a.st->done != 0) return;
    const cplx* __restrict__ x = static_cast<const cplx*>(a.x);
    cplx* __restrict__ out = static_cast<cplx*>(a.out);
    cplx* __restrict__ p = static_cast<cplx*>(a.p);
    const cplx* __restrict__ val = reinterpret_cast<const cplx*>(a.val);
    const cplx* __restrict__ gv = reinterpret_cast<const cplx*>(a.g);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (EPI == EPI_GERSH) {
        s0 = INFINITY;
        s1 = -INFINITY;
    }
    const int g = threadIdx.x / G, sub = threadIdx.x % G;
    const int rows_per = blockDim.x / G;
    const int nrow = a.n[0];
    const unsigned nrows = (unsigned)nrow;
    for (int L = xcd_tile(a.per_xcd); L < a.ntiles; L += gridDim.x) {
        const int row = L * rows_per + g;
        int e0 = 0, e1 = 0;
        if (row < nrow) {
            e0 = max(a.rowptr[row], 0);
            e1 = min(a.rowptr[row + 1], a.nnz);
        }
        if (EPI == EPI_GERSH) {
            double dg = 0.0, off = 0.0;
            for (int e = e0 + sub; e < e1; e += G) {
                const cplx v = val[e];
                if (a.colind[e] == row) dg += v.x;   // Hermitian: real diagonal
                else off += sqrt(cabs2(v));
            }
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                dg += __shfl_xor(dg, o, G);
                off += __shfl_xor(off, o, G);
            }
            if (sub == 0 && row < nrow) {
                s0 = fmin(s0, dg - off);
                s1 = fmax(s1, dg + off);
            }
            continue;
        }
        // four entries per lane and pass, their loads issued together
        // (indices clamped to the row's last entry, contributions past the
        // row's end masked), so that each lane has four gathers in flight
        cplx acc = {0.0, 0.0};
        for (int e = e0 + sub; e < e1; e += 4 * G) {
            int c[4];
            cplx v[4], xc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int eq = min(e + q * G, e1 - 1);
                c[q] = a.colind[eq];
                v[q] = val[eq];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = (e + q * G < e1) && ((unsigned)c[q] < nrows);
                xc[q] = x[ok ? c[q] : row];
                if (!ok) v[q] = cplx{0.0, 0.0};
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc.x = fma(v[q].x, xc[q].x, fma(-v[q].y, xc[q].y, acc.x));
                acc.y = fma(v[q].x, xc[q].y, fma(v[q].y, xc[q].x, acc.y));
            }
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o, G);
            acc.y += __shfl_xor(acc.y, o, G);
        }
        if (sub != 0 || row >= nrow) continue;
        const cplx wc = x[row];
        if (EPI == EPI_APPLY) {
            out[row] = a.alpha * acc + a.beta * wc;
        } else if (EPI == EPI_NEWTON) {
            const cplx wn = a.alpha * acc + a.beta * wc;
            const cplx d1 = {a.d1, a.d1i};
            const cplx pn = p[row] + cmul(d1, wn);
            out[row] = wn;
            p[row] = pn;
            s1 += cabs2(wn);
            s2 += cabs2(pn);
        } else if (EPI == EPI_FIRST) {
            const cplx wn = a.alpha * acc + a.beta * wc;
            const cplx d0 = {a.d0, a.d0i}, d1 = {a.d1, a.d1i};
            const cplx pn = cmul(d0, wc) + cmul(d1, wn);
            out[row] = wn;
            p[row] = pn;
            s0 += cabs2(wc);
            s1 += cabs2(wn);
            s2 += cabs2(pn);
        } else if (EPI == EPI_START) {
            const cplx sg = {a.sigma, a.sigmai};
            out[row] = cmul(sg, acc) + gv[row];
        }
    }
    if (EPI == EPI_NEWTON || EPI == EPI_FIRST || EPI == EPI_GERSH) finish_sweep<EPI>(a, s0, s1, s2);
}

template <int EPI>
hipError_t go(const Geom& g, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(g.grid), block(64 * g.waves);
    switch (g.vec) {  // lanes per row
        case 1: hipLaunchKernelGGL((csr_complex_sweep<EPI, 1>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((csr_complex_sweep<EPI, 2>), grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL((csr_complex_sweep<EPI, 8>), grid, block, 0, s, a); break;
        case 16: hipLaunchKernelGGL((csr_complex_sweep<EPI, 16>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((csr_complex_sweep<EPI, 4>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_csr_complex(const Geom& g, int epi, const SweepArgs& a, hipStream_t s) {
    switch (epi) {
        case EPI_APPLY: return go<EPI_APPLY>(g, a, s);
        case EPI_NEWTON: return go<EPI_NEWTON>(g, a, s);
        case EPI_FIRST: return go<EPI_FIRST>(g, a, s);
        case EPI_START: return go<EPI_START>(g, a, s);
        case EPI_GERSH: return go<EPI_GERSH>(g, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace expi
