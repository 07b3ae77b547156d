// Fused sweeps of the hot path for gfx950.
//
// Every kernel here makes one pass over an operator and a few vectors.  The
// central one is the Newton product of the Leja interpolation (Sec. III-C):
//
//   w_{j+1} = (alpha A + beta_j I) w_j        (eq. (3), alpha = 1/gamma,
//   p      += d_{j+1} w_{j+1}                  beta_j = -(c/gamma + xi_j))
//
// fused with the partial sums of ||w_{j+1}||^2 and ||p||^2 and, in the last
// workgroup to finish, the two-term stop test.  The loop therefore runs
// without any host round trip inside an iteration; later products of a
// converged loop see the status flag and return at once.
//
// Memory is the bound (about 0.4 flop/byte in FP64), so the kernels are
// written for HBM traffic, not arithmetic:
//  * stencils march each thread along the slowest axis (z in 3D, y in 2D),
//    keeping the previous, current and next value of that axis in registers,
//    so the slow-axis neighbours are never re-read; x neighbours come from
//    the same cache lines as the centre, mid-axis neighbours from the rows of
//    the same workgroup or its neighbour tile;
//  * workgroup b runs on XCD b % 8, so tile indices are remapped to give each
//    XCD one contiguous block of tiles: neighbouring tiles share that XCD's L2;
//  * boundary conditions are folded into the sweep as predicated neighbour
//    terms (Sec. III-A's second option), no ghost cells;
//  * reductions are deterministic: fixed-order wave butterflies, a fixed-order
//    block combine, and a fixed-order final sum over the per-workgroup
//    partials, so the stop decision is bitwise reproducible.
#include <type_traits>

#include "expi_internal.h"

namespace expi {
namespace {

template <class TIN, class TOUT>
using compute_t =
    typename std::conditional<std::is_same<TIN, float>::value && std::is_same<TOUT, float>::value,
                              float, double>::type;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void store_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Combine three per-thread values over the block (sum, or min/max for the
// Gershgorin bounds); result valid in thread 0.
template <int EPI>
__device__ void block_combine(double& v0, double& v1, double& v2, double (*red)[3]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (EPI == EPI_GERSH) {
        v0 = wave_min(v0);
        v1 = wave_max(v1);
    } else {
        v0 = wave_sum(v0);
        v1 = wave_sum(v1);
        v2 = wave_sum(v2);
    }
    if (lane == 0) {
        red[wv][0] = v0;
        red[wv][1] = v1;
        red[wv][2] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v0 = red[0][0];
        v1 = red[0][1];
        v2 = red[0][2];
        for (int w = 1; w < kBlock / 64; ++w) {
            if (EPI == EPI_GERSH) {
                v0 = fmin(v0, red[w][0]);
                v1 = fmax(v1, red[w][1]);
            } else {
                v0 += red[w][0];
                v1 += red[w][1];
                v2 += red[w][2];
            }
        }
    }
    __syncthreads();
}

// Publish this workgroup's partials; the last workgroup to arrive combines
// all of them in index order and writes the loop status.
template <int EPI>
__device__ void finish_sweep(const SweepArgs& a, double v0, double v1, double v2) {
    __shared__ double red[kBlock / 64][3];
    __shared__ int is_last;
    block_combine<EPI>(v0, v1, v2, red);
    if (threadIdx.x == 0) {
        double* part = a.partials + 4 * (size_t)blockIdx.x;
        store_agent(part + 0, v0);
        store_agent(part + 1, v1);
        store_agent(part + 2, v2);
        __threadfence();
        unsigned prev = __hip_atomic_fetch_add(&a.st->arrive, 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    double s0, s1, s2 = 0.0;
    if (EPI == EPI_GERSH) {
        s0 = INFINITY;
        s1 = -INFINITY;
    } else {
        s0 = 0.0;
        s1 = 0.0;
    }
    for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock) {
        const double* part = a.partials + 4 * (size_t)b;
        if (EPI == EPI_GERSH) {
            s0 = fmin(s0, load_agent(part + 0));
            s1 = fmax(s1, load_agent(part + 1));
        } else {
            s0 += load_agent(part + 0);
            s1 += load_agent(part + 1);
            s2 += load_agent(part + 2);
        }
    }
    block_combine<EPI>(s0, s1, s2, red);
    if (threadIdx.x != 0) return;
    NewtonState* st = a.st;
    if (EPI == EPI_GERSH) {
        st->gmin = s0;
        st->gmax = s1;
    } else {
        const double wn = sqrt(s1), pn = sqrt(s2);
        const double t = fabs(a.d1) * wn;
        const double tprev = (EPI == EPI_FIRST) ? fabs(a.d0) * sqrt(s0) : st->t_prev;
        const int m = a.j + 1;
        const double num = tprev + t;
        const double err = (pn > 0.0) ? num / pn : (num == 0.0 ? 0.0 : INFINITY);
        int done = 0;
        if (!isfinite(wn) || !isfinite(pn) || !isfinite(tprev)) done = 2;
        else if (m >= 2 && num <= a.tol * pn) done = 1;
        st->t_prev = t;
        st->err = err;
        st->pnorm = pn;
        st->wnorm = wn;
        st->m = m;
        st->done = done;
    }
    __hip_atomic_store(&st->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Stencil sweep
// ---------------------------------------------------------------------------

// Face weight of a face of cell c towards a neighbour with coefficient anb:
// mean of the two coefficients if the neighbour exists; for a missing
// neighbour, the cell's own coefficient under homogeneous Dirichlet (the
// neighbour's value is 0) and nothing under zero-flux Neumann.
template <class TC>
__device__ __forceinline__ TC face_weight(bool exists, bool dir, TC ac, TC anb) {
    return exists ? (TC)0.5 * (ac + anb) : (dir ? ac : (TC)0);
}

template <int DIM, int COEF, int EPI, class TIN, class TOUT>
__global__ __launch_bounds__(kBlock) void stencil_sweep(SweepArgs a) {
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
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x;
    const int L = (b % kXcd) * a.per_xcd + b / kXcd;
    if (L < a.ntiles) {
        const int t0 = L % a.tiles[0];
        const int rem = L / a.tiles[0];
        const int t1 = rem % a.tiles[1];
        const int t2 = rem / a.tiles[1];
        const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
        // slow (marched) axis: z in 3D, y in 2D; mid axis: y in 3D only
        const int ns = (DIM == 3) ? n2 : n1;
        const int ss = (DIM == 3) ? n0 * n1 : n0;
        const int i = t0 * 64 + lane;
        int j, kb, ke;
        if (DIM == 3) {
            j = t1 * (kBlock / 64) + wv;
            kb = t2 * kMarchZ;
            ke = min(kb + kMarchZ, ns);
        } else {
            j = 0;
            kb = t1 * ((kBlock / 64) * kMarchY) + wv * kMarchY;
            ke = min(kb + kMarchY, ns);
        }
        const bool active = (i < n0) && (DIM == 2 || j < n1) && (kb < ke);
        if (active) {
            const bool dir = (a.bc == EXPI_DIRICHLET0);
            const bool ionly = (a.bc == EXPI_INTERIOR_ONLY);
            const TC ihx = (TC)a.ih2[0];
            const TC ihy = (TC)a.ih2[1];
            const TC ihz = (TC)a.ih2[DIM == 3 ? 2 : 1];  // slow axis
            const TC alpha = (TC)a.alpha, beta = (TC)a.beta;
            const TC d0 = (TC)a.d0, d1 = (TC)a.d1, sigma = (TC)a.sigma;
            const TC c0 = (TC)a.c0, c1 = (TC)a.c1;
            const bool exm = i > 0, exq = i < n0 - 1;
            const bool eym = (DIM == 3) && j > 0, eyq = (DIM == 3) && j < n1 - 1;
            int idx = i + ((DIM == 3) ? n0 * (j + n1 * kb) : n0 * kb);

            // separable tables: per-column constants along x (and y in 3D),
            // a marched triple along the slow axis
            TC Xm = 0, Xc = 0, Xq = 0, Ym = 0, Yc = 0, Yq = 0, Zm = 0, Zc = 0, Zq = 0;
            const double* Ts = (DIM == 3) ? a.tz : a.ty;
            if (COEF == EXPI_COEF_SEPARABLE) {
                Xc = (TC)a.tx[i];
                Xm = exm ? (TC)a.tx[i - 1] : (TC)0;
                Xq = exq ? (TC)a.tx[i + 1] : (TC)0;
                if (DIM == 3) {
                    Yc = (TC)a.ty[j];
                    Ym = eym ? (TC)a.ty[j - 1] : (TC)0;
                    Yq = eyq ? (TC)a.ty[j + 1] : (TC)0;
                }
                Zm = (kb > 0) ? (TC)Ts[kb - 1] : (TC)0;
                Zc = (TC)Ts[kb];
            }
            // coefficient field: marched triple along the slow axis
            TC Fm = 0, Fc = 0, Fq = 0;
            if (COEF == EXPI_COEF_FIELD) {
                Fm = (kb > 0) ? (TC)a.field[idx - ss] : (TC)0;
                Fc = (TC)a.field[idx];
            }
            TC wm = 0, wc = 0;
            if (EPI != EPI_GERSH) {
                wm = (kb > 0) ? (TC)x[idx - ss] : (TC)0;
                wc = (TC)x[idx];
            }

            for (int k = kb; k < ke; ++k, idx += ss) {
                const bool ezm = k > 0, ezq = k < ns - 1;
                TC wq = 0, wxm = 0, wxq = 0, wym = 0, wyq = 0;
                if (EPI != EPI_GERSH) {
                    wq = ezq ? (TC)x[idx + ss] : (TC)0;
                    wxm = exm ? (TC)x[idx - 1] : (TC)0;
                    wxq = exq ? (TC)x[idx + 1] : (TC)0;
                    if (DIM == 3) {
                        wym = eym ? (TC)x[idx - n0] : (TC)0;
                        wyq = eyq ? (TC)x[idx + n0] : (TC)0;
                    }
                }
                // coefficients at the centre and the neighbours
                TC ac, axm, axq, aym, ayq, azm, azq;
                if (COEF == EXPI_COEF_CONST) {
                    ac = axm = axq = aym = ayq = azm = azq = c0;
                } else if (COEF == EXPI_COEF_SEPARABLE) {
                    if (ezq) Zq = (TC)Ts[k + 1];
                    if (DIM == 3) {
                        const TC zy = Zc * Yc;
                        ac = c0 + c1 * (zy * Xc);
                        axm = c0 + c1 * (zy * Xm);
                        axq = c0 + c1 * (zy * Xq);
                        aym = c0 + c1 * ((Zc * Ym) * Xc);
                        ayq = c0 + c1 * ((Zc * Yq) * Xc);
                        azm = c0 + c1 * ((Zm * Yc) * Xc);
                        azq = c0 + c1 * ((Zq * Yc) * Xc);
                    } else {
                        ac = c0 + c1 * (Zc * Xc);
                        axm = c0 + c1 * (Zc * Xm);
                        axq = c0 + c1 * (Zc * Xq);
                        aym = ayq = (TC)0;
                        azm = c0 + c1 * (Zm * Xc);
                        azq = c0 + c1 * (Zq * Xc);
                    }
                } else {
                    Fq = ezq ? (TC)a.field[idx + ss] : (TC)0;
                    ac = Fc;
                    axm = exm ? (TC)a.field[idx - 1] : (TC)0;
                    axq = exq ? (TC)a.field[idx + 1] : (TC)0;
                    aym = (DIM == 3 && eym) ? (TC)a.field[idx - n0] : (TC)0;
                    ayq = (DIM == 3 && eyq) ? (TC)a.field[idx + n0] : (TC)0;
                    azm = Fm;
                    azq = Fq;
                }
                const bool inner = exm && exq && ezm && ezq && (DIM == 2 || (eym && eyq));
                const bool zero_row = ionly && !inner;
                const bool dirx = dir;
                // face weights (times 1/h^2 per axis)
                const TC fxm = face_weight<TC>(exm, dirx, ac, axm) * ihx;
                const TC fxq = face_weight<TC>(exq, dirx, ac, axq) * ihx;
                const TC fzm = face_weight<TC>(ezm, dirx, ac, azm) * ihz;
                const TC fzq = face_weight<TC>(ezq, dirx, ac, azq) * ihz;
                TC fym = 0, fyq = 0;
                if (DIM == 3) {
                    fym = face_weight<TC>(eym, dirx, ac, aym) * ihy;
                    fyq = face_weight<TC>(eyq, dirx, ac, ayq) * ihy;
                }
                if (EPI == EPI_GERSH) {
                    // row: diagonal = -(sum of all face weights), off-diagonal
                    // magnitude = weights of the faces that have a neighbour
                    TC diag = -(fxm + fxq + fym + fyq + fzm + fzq);
                    TC off = (exm ? fxm : (TC)0) + (exq ? fxq : (TC)0) + (eym ? fym : (TC)0) +
                             (eyq ? fyq : (TC)0) + (ezm ? fzm : (TC)0) + (ezq ? fzq : (TC)0);
                    if (zero_row) diag = off = 0;
                    s0 = fmin(s0, (double)(diag - off));
                    s1 = fmax(s1, (double)(diag + off));
                } else {
                    // (A w)_c = sum over faces of weight * (w_nb - w_c); a missing
                    // neighbour was loaded as 0 (Dirichlet) or has weight 0 (Neumann)
                    TC Aw = fxm * (wxm - wc) + fxq * (wxq - wc) + fzm * (wm - wc) + fzq * (wq - wc);
                    if (DIM == 3) Aw += fym * (wym - wc) + fyq * (wyq - wc);
                    if (zero_row) Aw = 0;
                    if (EPI == EPI_APPLY) {
                        out[idx] = (TOUT)(alpha * Aw + beta * wc);
                    } else if (EPI == EPI_NEWTON) {
                        const TOUT wn = (TOUT)(alpha * Aw + beta * wc);
                        const TOUT pn = (TOUT)((TC)p[idx] + d1 * (TC)wn);
                        out[idx] = wn;
                        p[idx] = pn;
                        s1 += (double)wn * (double)wn;
                        s2 += (double)pn * (double)pn;
                    } else if (EPI == EPI_FIRST) {
                        const TOUT wn = (TOUT)(alpha * Aw + beta * wc);
                        const TOUT pn = (TOUT)(d0 * wc + d1 * (TC)wn);
                        out[idx] = wn;
                        p[idx] = pn;
                        s0 += (double)wc * (double)wc;
                        s1 += (double)wn * (double)wn;
                        s2 += (double)pn * (double)pn;
                    } else if (EPI == EPI_START) {
                        TC gv;
                        if (a.gmode == G_VEC) {
                            gv = (TC)a.g[idx];
                        } else if (a.gmode == G_CUBIC_OF) {
                            const TC u = (TC)a.g[idx];
                            gv = u - u * u * u;
                        } else {
                            gv = wc - wc * wc * wc;
                        }
                        out[idx] = (TOUT)(sigma * Aw + gv);
                    }
                }
                if (COEF == EXPI_COEF_SEPARABLE) {
                    Zm = Zc;
                    Zc = Zq;
                }
                if (COEF == EXPI_COEF_FIELD) {
                    Fm = Fc;
                    Fc = Fq;
                }
                wm = wc;
                wc = wq;
            }
        }
    }
    if (EPI == EPI_NEWTON || EPI == EPI_FIRST || EPI == EPI_GERSH) finish_sweep<EPI>(a, s0, s1, s2);
}

// ---------------------------------------------------------------------------
// CSR sweep: kCsrGroup lanes per row, shuffle reduction inside the group.
// ---------------------------------------------------------------------------
template <int EPI, class TIN, class TOUT>
__global__ __launch_bounds__(kBlock) void csr_sweep(SweepArgs a) {
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
    const int b = blockIdx.x;
    const int L = (b % kXcd) * a.per_xcd + b / kXcd;
    const int g = threadIdx.x / kCsrGroup, sub = threadIdx.x % kCsrGroup;
    const int row = L * (kBlock / kCsrGroup) + g;
    if (L < a.ntiles && row < a.n[0]) {
        // row range clamped to [0, nnz) and column indices checked against
        // n, so a malformed matrix cannot send a load out of bounds
        const int e0 = max(a.rowptr[row], 0), e1 = min(a.rowptr[row + 1], a.nnz);
        const unsigned nrows = (unsigned)a.n[0];
        if (EPI == EPI_GERSH) {
            double dg = 0.0, off = 0.0;
            for (int e = e0 + sub; e < e1; e += kCsrGroup) {
                const double v = a.val[e];
                if (a.colind[e] == row) dg += v; else off += fabs(v);
            }
#pragma unroll
            for (int o = kCsrGroup / 2; o > 0; o >>= 1) {
                dg += __shfl_xor(dg, o, kCsrGroup);
                off += __shfl_xor(off, o, kCsrGroup);
            }
            s0 = dg - off;
            s1 = dg + off;
        } else {
            TC acc = 0;
            for (int e = e0 + sub; e < e1; e += kCsrGroup) {
                const int col = a.colind[e];
                if ((unsigned)col < nrows) acc += (TC)a.val[e] * (TC)x[col];
            }
#pragma unroll
            for (int o = kCsrGroup / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kCsrGroup);
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
                    s1 = (double)wn * (double)wn;
                    s2 = (double)pn * (double)pn;
                } else if (EPI == EPI_FIRST) {
                    const TOUT wn = (TOUT)(alpha * acc + beta * wc);
                    const TOUT pn = (TOUT)((TC)a.d0 * wc + (TC)a.d1 * (TC)wn);
                    out[row] = wn;
                    p[row] = pn;
                    s0 = (double)wc * (double)wc;
                    s1 = (double)wn * (double)wn;
                    s2 = (double)pn * (double)pn;
                } else if (EPI == EPI_START) {
                    TC gv;
                    if (a.gmode == G_VEC) {
                        gv = (TC)a.g[row];
                    } else if (a.gmode == G_CUBIC_OF) {
                        const TC u = (TC)a.g[row];
                        gv = u - u * u * u;
                    } else {
                        gv = wc - wc * wc * wc;
                    }
                    out[row] = (TOUT)((TC)a.sigma * acc + gv);
                }
            }
        }
        if (EPI == EPI_GERSH && sub != 0) {
            s0 = INFINITY;
            s1 = -INFINITY;
        }
    }
    if (EPI == EPI_NEWTON || EPI == EPI_FIRST || EPI == EPI_GERSH) finish_sweep<EPI>(a, s0, s1, s2);
}

// ---------------------------------------------------------------------------
// Pointwise kernels
// ---------------------------------------------------------------------------
template <class TP>
__global__ __launch_bounds__(kBlock) void update_kernel(int64_t n, double* __restrict__ out,
                                                        const double* __restrict__ yin,
                                                        const TP* __restrict__ p, double scale,
                                                        const NewtonState* st, int guard) {
    if (guard && st->done != 1) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        out[i] = (yin ? yin[i] : 0.0) + scale * (double)p[i];
}

__global__ void reset_kernel(NewtonState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->arrive = 0;
        st->done = 0;
        st->m = 0;
        st->pad = 0;
        st->t_prev = 0.0;
        st->err = 0.0;
        st->pnorm = 0.0;
        st->wnorm = 0.0;
        st->gmin = 0.0;
        st->gmax = 0.0;
    }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int DIM, int COEF, int EPI, class TIN, class TOUT>
hipError_t go_stencil(const Plan& pl, const SweepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((stencil_sweep<DIM, COEF, EPI, TIN, TOUT>), dim3(pl.grid), dim3(kBlock), 0,
                       s, a);
    return hipGetLastError();
}

template <int DIM, int COEF>
hipError_t dispatch_types(const Plan& pl, int epi, int tin, int tout, const SweepArgs& a,
                          hipStream_t s) {
    switch (epi) {
        case EPI_APPLY:
            if (tin == 0 && tout == 0) return go_stencil<DIM, COEF, EPI_APPLY, double, double>(pl, a, s);
            if (tin == 1 && tout == 1) return go_stencil<DIM, COEF, EPI_APPLY, float, float>(pl, a, s);
            break;
        case EPI_NEWTON:
            if (tin == 0 && tout == 0) return go_stencil<DIM, COEF, EPI_NEWTON, double, double>(pl, a, s);
            if (tin == 1 && tout == 1) return go_stencil<DIM, COEF, EPI_NEWTON, float, float>(pl, a, s);
            break;
        case EPI_FIRST:
            if (tin == 0 && tout == 0) return go_stencil<DIM, COEF, EPI_FIRST, double, double>(pl, a, s);
            if (tin == 0 && tout == 1) return go_stencil<DIM, COEF, EPI_FIRST, double, float>(pl, a, s);
            if (tin == 1 && tout == 1) return go_stencil<DIM, COEF, EPI_FIRST, float, float>(pl, a, s);
            break;
        case EPI_START:
            if (tin == 0 && tout == 0) return go_stencil<DIM, COEF, EPI_START, double, double>(pl, a, s);
            if (tin == 0 && tout == 1) return go_stencil<DIM, COEF, EPI_START, double, float>(pl, a, s);
            break;
        case EPI_GERSH:
            return go_stencil<DIM, COEF, EPI_GERSH, double, double>(pl, a, s);
    }
    return hipErrorInvalidValue;
}

template <int EPI, class TIN, class TOUT>
hipError_t go_csr(const Plan& pl, const SweepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((csr_sweep<EPI, TIN, TOUT>), dim3(pl.grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t dispatch_csr(const Plan& pl, int epi, int tin, int tout, const SweepArgs& a,
                        hipStream_t s) {
    switch (epi) {
        case EPI_APPLY:
            if (tin == 0 && tout == 0) return go_csr<EPI_APPLY, double, double>(pl, a, s);
            if (tin == 1 && tout == 1) return go_csr<EPI_APPLY, float, float>(pl, a, s);
            break;
        case EPI_NEWTON:
            if (tin == 0 && tout == 0) return go_csr<EPI_NEWTON, double, double>(pl, a, s);
            if (tin == 1 && tout == 1) return go_csr<EPI_NEWTON, float, float>(pl, a, s);
            break;
        case EPI_FIRST:
            if (tin == 0 && tout == 0) return go_csr<EPI_FIRST, double, double>(pl, a, s);
            if (tin == 0 && tout == 1) return go_csr<EPI_FIRST, double, float>(pl, a, s);
            if (tin == 1 && tout == 1) return go_csr<EPI_FIRST, float, float>(pl, a, s);
            break;
        case EPI_START:
            if (tin == 0 && tout == 0) return go_csr<EPI_START, double, double>(pl, a, s);
            if (tin == 0 && tout == 1) return go_csr<EPI_START, double, float>(pl, a, s);
            break;
        case EPI_GERSH:
            return go_csr<EPI_GERSH, double, double>(pl, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

Plan make_plan(const Op& op) {
    Plan pl{};
    if (op.kind == 1) {
        const int64_t rows_per = kBlock / kCsrGroup;
        pl.tiles[0] = (int)((op.nrows + rows_per - 1) / rows_per);
        pl.tiles[1] = pl.tiles[2] = 1;
    } else if (op.dim == 3) {
        pl.tiles[0] = (op.n[0] + 63) / 64;
        pl.tiles[1] = (op.n[1] + kBlock / 64 - 1) / (kBlock / 64);
        pl.tiles[2] = (op.n[2] + kMarchZ - 1) / kMarchZ;
    } else {
        const int rows = (kBlock / 64) * kMarchY;
        pl.tiles[0] = (op.n[0] + 63) / 64;
        pl.tiles[1] = (op.n[1] + rows - 1) / rows;
        pl.tiles[2] = 1;
    }
    pl.ntiles = pl.tiles[0] * pl.tiles[1] * pl.tiles[2];
    if (pl.ntiles < 1) pl.ntiles = 1;
    pl.per_xcd = (pl.ntiles + kXcd - 1) / kXcd;
    pl.grid = kXcd * pl.per_xcd;
    return pl;
}

size_t partials_bytes(const Op& op) { return (size_t)op.plan.grid * 4 * sizeof(double); }

hipError_t launch_sweep(const Op& op, int epi, int tin, int tout, SweepArgs a, hipStream_t s) {
    const Plan& pl = op.plan;
    for (int d = 0; d < 3; ++d) a.tiles[d] = pl.tiles[d];
    a.ntiles = pl.ntiles;
    a.per_xcd = pl.per_xcd;
    if (op.kind == 1) {
        a.n[0] = (int)op.nrows;
        a.nnz = (int)op.nnz;
        a.rowptr = op.rowptr;
        a.colind = op.colind;
        a.val = op.val;
        return dispatch_csr(pl, epi, tin, tout, a, s);
    }
    for (int d = 0; d < 3; ++d) {
        a.n[d] = op.n[d];
        a.ih2[d] = 1.0 / (op.h[d] * op.h[d]);
    }
    a.bc = op.bc;
    a.c0 = op.c0;
    a.c1 = op.c1;
    a.tx = op.tx;
    a.ty = op.ty;
    a.tz = op.tz;
    a.field = op.field;
    if (op.dim == 3) {
        switch (op.coef) {
            case EXPI_COEF_CONST: return dispatch_types<3, EXPI_COEF_CONST>(pl, epi, tin, tout, a, s);
            case EXPI_COEF_SEPARABLE: return dispatch_types<3, EXPI_COEF_SEPARABLE>(pl, epi, tin, tout, a, s);
            case EXPI_COEF_FIELD: return dispatch_types<3, EXPI_COEF_FIELD>(pl, epi, tin, tout, a, s);
        }
    } else {
        switch (op.coef) {
            case EXPI_COEF_CONST: return dispatch_types<2, EXPI_COEF_CONST>(pl, epi, tin, tout, a, s);
            case EXPI_COEF_SEPARABLE: return dispatch_types<2, EXPI_COEF_SEPARABLE>(pl, epi, tin, tout, a, s);
            case EXPI_COEF_FIELD: return dispatch_types<2, EXPI_COEF_FIELD>(pl, epi, tin, tout, a, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_update(int64_t n, double* out, const double* yin, const void* p, int tp,
                         double scale, NewtonState* st, int guard, hipStream_t s) {
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (tp == 0)
        hipLaunchKernelGGL(update_kernel<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, out,
                           yin, static_cast<const double*>(p), scale, st, guard);
    else
        hipLaunchKernelGGL(update_kernel<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, out,
                           yin, static_cast<const float*>(p), scale, st, guard);
    return hipGetLastError();
}

hipError_t launch_reset(NewtonState* st, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

}  // namespace expi
