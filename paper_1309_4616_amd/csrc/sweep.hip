// Launch geometry, the finalize kernel and the pointwise kernels.
//
// Every product of the Leja interpolation (Sec. III-C) is one fused sweep:
//
//   w_{j+1} = (alpha A + beta_j I) w_j        (eq. (3), alpha = 1/gamma,
//   p      += d_{j+1} w_{j+1}                  beta_j = -(c/gamma + xi_j))
//
// with per-workgroup partial sums of ||w_{j+1}||^2 and ||p||^2, followed by
// a one-workgroup finalize kernel that combines them in index order and
// applies the two-term stop test, so the stop decision is bitwise
// reproducible and needs no host round trip.  Later products of a converged
// loop read the status flag and return at once.  (A last-workgroup-done
// reduction inside the sweep would need a device-scope release fence per
// workgroup, which on a multi-XCD part writes back L2 each time; the kernel
// boundary gives the same visibility once.)
//
// Epilogues of a sweep:
//   EPI_APPLY   y = alpha A x + beta x                (eq. (3))
//   EPI_NEWTON  the fused Newton product above
//   EPI_FIRST   w_1 = alpha A w_0 + beta_0 w_0, p = d_0 w_0 + d_1 w_1
//   EPI_START   r = sigma A x + g, g = v or u - u^3   (substep start vector)
//   EPI_GERSH   Gershgorin bounds of the rows, min/max over rows
#include <cmath>

#include "sweep_common.h"

namespace expi {
namespace {

// The whole record to the host copy (thread 0, after its own writes).
__device__ __forceinline__ void mirror_state(const FinalArgs& f) {
    if (f.mirror == nullptr || threadIdx.x != 0) return;
    const unsigned long long* from = reinterpret_cast<const unsigned long long*>(f.st);
    unsigned long long* to = reinterpret_cast<unsigned long long*>(f.mirror);
    constexpr int kWords = (int)(sizeof(NewtonState) / 8);
    unsigned long long v[kWords];   // all loads, then all stores (one round trip)
#pragma unroll
    for (int q = 0; q < kWords; ++q) v[q] = from[q];
#pragma unroll
    for (int q = 0; q < kWords; ++q) to[q] = v[q];
}

template <int EPI>
__device__ void finalize_tests(const FinalArgs& f) {
    __shared__ double red[kMaxWaves][3];
    NewtonState* st = f.st;
    // every load goes out before the status flag is looked at: the flag,
    // the partials and the previous term arrive in one memory round trip
    const int done_in = st->done;
    const double tprev_in = st->t_prev;
    double s0, s1, s2 = 0.0;
    if (EPI == EPI_GERSH) {
        s0 = INFINITY;
        s1 = -INFINITY;
    } else {
        s0 = 0.0;
        s1 = 0.0;
    }
    for (int b = threadIdx.x; b < f.nparts; b += kFinalThreads) {
        const double* part = f.partials + 4 * (size_t)b;
        if (EPI == EPI_GERSH) {
            s0 = fmin(s0, part[0]);
            s1 = fmax(s1, part[1]);
        } else {
            s0 += part[0];
            s1 += part[1];
            s2 += part[2];
        }
    }
    if (f.guard && done_in != 0) return;   // the same in every thread
    block_combine<EPI>(s0, s1, s2, red);
    if (threadIdx.x != 0) return;
    if (EPI == EPI_GERSH) {
        st->gmin = s0;
        st->gmax = s1;
        return;
    }
    const double wn = sqrt(s1), pn = sqrt(s2);
    const double t = fabs(f.d1) * wn;
    const double tprev = (EPI == EPI_FIRST) ? fabs(f.d0) * sqrt(s0) : tprev_in;
    const int m = f.j + 1;
    const double num = tprev + t;
    const double err = (pn > 0.0) ? num / pn : (num == 0.0 ? 0.0 : INFINITY);
    int done = 0;
    if (!isfinite(wn) || !isfinite(pn) || !isfinite(tprev)) done = 2;
    else if (m >= 2 && num <= f.tol * pn) done = 1;
    st->t_prev = t;
    st->err = err;
    st->pnorm = pn;
    st->wnorm = wn;
    st->m = m;
    st->done = done;
    if (EPI == EPI_FIRST) {
        st->rnorm = sqrt(s0);
        st->hist[0] = tprev;
    }
    if (m < kHist) st->hist[m] = t;
}

template <int EPI>
__global__ __launch_bounds__(kFinalThreads) void finalize_kernel(FinalArgs f) {
    finalize_tests<EPI>(f);
    mirror_state(f);
}

// out = yin + scale * p (yin may be NULL for 0).  After a pair sweep that
// met the stop test at its first product, p holds one term too many:
// p - fix * wfix removes d_{m+1} w_{m+1} (wfix NULL otherwise).
template <class TP>
__global__ __launch_bounds__(256) void update_kernel(int64_t n, double* out, const double* yin,
                                                     const TP* p, double scale,
                                                     const NewtonState* st, int guard,
                                                     const TP* __restrict__ wfix, double fix) {
    if (guard && st->done != 1) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (wfix) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
            out[i] = (yin ? yin[i] : 0.0) + scale * ((double)p[i] - fix * (double)wfix[i]);
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
            out[i] = (yin ? yin[i] : 0.0) + scale * (double)p[i];
    }
}

// update_kernel with the correction read from the state (see launch_update_st)
template <class TP>
__global__ __launch_bounds__(256) void update_st_kernel(int64_t n, double* out, const double* yin,
                                                        const TP* p, double scale,
                                                        const NewtonState* st, const TP* w0,
                                                        const TP* w1) {
    if (st->done != 1) return;
    const double fix = st->fix;
    const TP* wfix = st->fixbuf ? w1 : w0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (fix != 0.0) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
            out[i] = (yin ? yin[i] : 0.0) + scale * ((double)p[i] - fix * (double)wfix[i]);
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
            out[i] = (yin ? yin[i] : 0.0) + scale * (double)p[i];
    }
}

// Stop tests after a pair sweep (pair_tests) as a kernel of its own.
__global__ __launch_bounds__(kFinalThreads) void pair_finalize_kernel(FinalArgs f) {
    pair_tests(f);
    mirror_state(f);
}

__global__ void reset_kernel(NewtonState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->arrive = 0;
        st->done = 0;
        st->m = 0;
        st->fixbuf = 0;
        st->t_prev = 0.0;
        st->err = 0.0;
        st->pnorm = 0.0;
        st->wnorm = 0.0;
        st->gmin = 0.0;
        st->gmax = 0.0;
        for (int q = 0; q < kHist; ++q) st->hist[q] = 0.0;
        st->rnorm = 0.0;
        st->pred_m = 0;
        st->pred_s = 0;
        st->fix = 0.0;
    }
}

// Smooth deterministic fill (for timing sweeps on meaningful data).
template <class T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ out, int64_t n, double scale) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (T)(scale * sin(1e-3 * (double)(i % 1000003)));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

thread_local NewtonState* tl_mirror = nullptr;

}  // namespace

void set_state_mirror(NewtonState* mirror) { tl_mirror = mirror; }

Geom make_geom(const Op& op, const Tiles& t) {
    Geom g{};
    g.vec = t.vec;
    g.waves = t.waves;
    g.march = t.march;
    if (op.kind != 0) {
        const int64_t rows_per = (64 * t.waves) / t.vec;
        g.tiles[0] = (int)((op.nrows + rows_per - 1) / rows_per);
        g.tiles[1] = g.tiles[2] = 1;
    } else if (op.dim == 3) {
        g.tiles[0] = (op.n[0] + 64 * t.vec - 1) / (64 * t.vec);
        g.tiles[1] = (op.n[1] + t.waves - 1) / t.waves;
        g.tiles[2] = (op.n[2] + t.march - 1) / t.march;
    } else {
        const int rows = t.waves * t.march;
        g.tiles[0] = (op.n[0] + 64 * t.vec - 1) / (64 * t.vec);
        g.tiles[1] = (op.n[1] + rows - 1) / rows;
        g.tiles[2] = 1;
    }
    const int64_t nt = (int64_t)g.tiles[0] * g.tiles[1] * g.tiles[2];
    g.ntiles = nt < 1 ? 1 : (int)nt;
    g.per_xcd = (g.ntiles + kXcd - 1) / kXcd;
    // CSR sweeps loop over row blocks: at most kCsrGrid workgroups, so that
    // the finalize kernel sums few partials
    if (op.kind != 0 && g.per_xcd > kCsrGrid / kXcd) g.per_xcd = kCsrGrid / kXcd;
    g.grid = kXcd * g.per_xcd;
    return g;
}

Tiles default_tiles(const Op& op) {
    Tiles t;
    if (op.kind == 2) {
        t.vec = 4;     // lanes per row (complex entries: 16 bytes each)
        t.waves = 4;
        t.march = 1;
    } else if (op.kind == 1) {
        t.vec = 8;     // lanes per row
        t.waves = 4;
        t.march = 1;
    } else {
        // measured best at 256^3 (fused Newton product, FP64 and FP32)
        t.vec = 2;
        t.waves = 4;
        t.march = (op.dim == 3) ? 32 : 8;
    }
    return t;
}

bool tiles_valid(const Op& op, const Tiles& t) {
    if (t.waves < 1 || t.waves > kMaxWaves) return false;
    if (op.kind == 2)
        return (t.vec == 1 || t.vec == 2 || t.vec == 4 || t.vec == 8 || t.vec == 16) && t.march == 1;
    if (op.kind != 0) return (t.vec == 4 || t.vec == 8 || t.vec == 16) && t.march == 1;
    return (t.vec == 1 || t.vec == 2) && t.march >= kMinMarch && t.march <= kMaxMarch &&
           t.march % 4 == 0;
}

// Largest workgroup count any accepted tile setting can produce: it sizes
// the partials buffer of the workspace.
size_t partials_bytes(const Op& op) {
    Tiles t;
    if (op.kind != 0) {
        t.vec = 16;
        t.waves = 1;
        t.march = 1;
    } else {
        t.vec = 1;
        t.waves = 1;
        t.march = kMinMarch;
    }
    // also covers the pair sweep, whose grid never exceeds max(CU count, 8)
    // workgroups of at most 8 partials each
    const size_t grid = std::max<size_t>((size_t)make_geom(op, t).grid, 1024);
    return grid * 4 * sizeof(double);
}

hipError_t launch_sweep(const Op& op, int epi, int tin, int tout, SweepArgs a, hipStream_t s,
                        hipEvent_t after_sweep, bool finalize) {
    Tiles t = op.tiles;
    if (op.kind == 0 && t.vec == 2) {
        // 16-byte vector accesses need an even row length and aligned arrays
        const bool ok = (op.n[0] % 2 == 0) && aligned16(a.x) && aligned16(a.out) &&
                        aligned16(a.p) && aligned16(a.g) && aligned16(op.field);
        if (!ok) t.vec = 1;
    }
    const Geom g = make_geom(op, t);
    for (int d = 0; d < 3; ++d) a.tiles[d] = g.tiles[d];
    a.ntiles = g.ntiles;
    a.per_xcd = g.per_xcd;
    a.march = g.march;
    hipError_t e;
    if (op.kind != 0) {
        a.n[0] = (int)op.nrows;
        a.nnz = (int)op.nnz;
        a.rowptr = op.rowptr;
        a.colind = op.colind;
        a.val = op.val;
        e = (op.kind == 2) ? launch_csr_complex(g, epi, a, s) : launch_csr(g, epi, tin, tout, a, s);
    } else {
        for (int d = 0; d < 3; ++d) {
            a.n[d] = op.n[d];
            a.ih2[d] = 1.0 / (op.h[d] * op.h[d]);
            a.hpos[d] = op.h[d];
        }
        a.bc = op.bc;
        a.c0 = op.c0;
        a.c1 = op.c1;
        a.tx = op.tx;
        a.ty = op.ty;
        a.tz = op.tz;
        a.field = op.field;
        // boundary data: in the sweep, or afterwards in a launch of their own
        const bool separate = a.bdata && op.bdata_mode == EXPI_BDATA_SEPARATE;
        const double bscale = (epi == EPI_APPLY) ? a.alpha : a.sigma;
        if (separate) a.bdata = 0;
        e = launch_stencil(op, g, epi, tin, tout, a, s);
        if (e == hipSuccess && separate) e = launch_boundary(op, bscale, a.out, tout, s);
    }
    if (e != hipSuccess) return e;
    if (after_sweep) {
        e = hipEventRecord(after_sweep, s);
        if (e != hipSuccess) return e;
    }
    if (epi != EPI_NEWTON && epi != EPI_FIRST && epi != EPI_GERSH) return hipSuccess;
    if (!finalize) return hipSuccess;
    FinalArgs f{};
    f.mirror = tl_mirror;
    f.partials = a.partials;
    f.st = a.st;
    f.nparts = g.grid;
    // the stop test needs |d_j| (complex coefficients: the modulus)
    f.d0 = std::hypot(a.d0, a.d0i);
    f.d1 = std::hypot(a.d1, a.d1i);
    f.tol = a.tol;
    f.j = a.j;
    f.guard = a.guard;
    if (epi == EPI_NEWTON) hipLaunchKernelGGL(finalize_kernel<EPI_NEWTON>, dim3(1), dim3(kFinalThreads), 0, s, f);
    else if (epi == EPI_FIRST) hipLaunchKernelGGL(finalize_kernel<EPI_FIRST>, dim3(1), dim3(kFinalThreads), 0, s, f);
    else hipLaunchKernelGGL(finalize_kernel<EPI_GERSH>, dim3(1), dim3(kFinalThreads), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_update(int64_t n, double* out, const double* yin, const void* p, int tp,
                         double scale, const NewtonState* st, int guard, hipStream_t s,
                         const void* wfix, double fix) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (fix == 0.0) wfix = nullptr;
    if (tp == 0)
        hipLaunchKernelGGL(update_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, n, out,
                           yin, static_cast<const double*>(p), scale, st, guard,
                           static_cast<const double*>(wfix), fix);
    else
        hipLaunchKernelGGL(update_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, n, out,
                           yin, static_cast<const float*>(p), scale, st, guard,
                           static_cast<const float*>(wfix), fix);
    return hipGetLastError();
}

hipError_t launch_update_st(int64_t n, double* out, const double* yin, const void* p, int tp,
                            double scale, const NewtonState* st, const void* w0, const void* w1,
                            hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (tp == 0)
        hipLaunchKernelGGL(update_st_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, n, out,
                           yin, static_cast<const double*>(p), scale, st,
                           static_cast<const double*>(w0), static_cast<const double*>(w1));
    else
        hipLaunchKernelGGL(update_st_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, n, out,
                           yin, static_cast<const float*>(p), scale, st,
                           static_cast<const float*>(w0), static_cast<const float*>(w1));
    return hipGetLastError();
}

hipError_t launch_pair_finalize(const double* partials, NewtonState* st, int nparts, int j,
                                int guard, double d0, double d1, double d2, double tol, int mode,
                                int outbuf, hipStream_t s) {
    FinalArgs f{};
    f.mirror = tl_mirror;
    f.partials = partials;
    f.st = st;
    f.nparts = nparts;
    f.j = j;
    f.guard = guard;
    f.mode = mode;
    f.outbuf = outbuf;
    f.d0 = d0;
    f.d1 = d1;
    f.d2 = d2;
    f.tol = tol;
    hipLaunchKernelGGL(pair_finalize_kernel, dim3(1), dim3(kFinalThreads), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_reset(NewtonState* st, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_fill(void* out, int64_t n, int t, double scale, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (t == 0)
        hipLaunchKernelGGL(fill_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<double*>(out), n, scale);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<float*>(out), n, scale);
    return hipGetLastError();
}

}  // namespace expi
