// Device helpers shared by the sweep kernels (HIP, gfx950).
#pragma once

#include <type_traits>

#include "expi_internal.h"

namespace expi {

// Arithmetic type of a sweep: float only when both the input and the output
// vectors are stored in float, otherwise double.
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

// Combine three per-thread values over the block in a fixed order (sums, or
// min/max for Gershgorin bounds); the result is valid in thread 0.
template <int EPI>
__device__ void block_combine(double& v0, double& v1, double& v2, double (*red)[3]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
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
        for (int w = 1; w < nw; ++w) {
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

// Write this workgroup's partials (plain stores; the finalize kernel that
// follows on the stream reads them after the kernel boundary).
template <int EPI>
__device__ void finish_sweep(const SweepArgs& a, double v0, double v1, double v2) {
    __shared__ double red[kMaxWaves][3];
    block_combine<EPI>(v0, v1, v2, red);
    if (threadIdx.x == 0) {
        double* part = a.partials + 4 * (size_t)blockIdx.x;
        part[0] = v0;
        part[1] = v1;
        part[2] = v2;
    }
}

// N per-thread sums combined over the block in a fixed order and written as
// this workgroup's partials at partials[stride * blockIdx.x + q] (the pair
// sweep: the two products' norms).
template <int N>
__device__ __forceinline__ void finish_sweep_n(double* partials, int stride, const double (&vin)[N]) {
    __shared__ double red[kMaxPairWaves][N];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    double v[N];
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = wave_sum(vin[q]);
    if (lane == 0)
        for (int q = 0; q < N; ++q) red[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double* part = partials + (size_t)stride * blockIdx.x;
        for (int q = 0; q < N; ++q) {
            double acc = red[0][q];
            for (int w = 1; w < nw; ++w) acc += red[w][q];
            part[q] = acc;
        }
    }
}

// Stop tests after a pair sweep: the two-term test at m = j+1 with
// ||w_{j+1}||, ||p_{j+1}||, and, if that one fails, at m = j+2 with
// ||w_{j+2}||, ||p_{j+2}|| (same rule as finalize_kernel: no stop at
// m = 1).  A pair that starts the loop (PAIR_FIRST, j = 0) brings ||r||^2 as
// a fifth partial sum (stride 8): it records t_0 = |d_0| ||r|| and ||r||,
// and its first test (m = 1) can only report a non-finite value.  A
// PAIR_START sweep comes with j = -1, d1 = d_0, d2 = d_1 and ||r||^2 in the
// first slot: its two tests are those at m = 0 and m = 1 and it records
// ||r||.
//
// Called by every thread of one workgroup of kFinalThreads threads.
// With f.guard, nothing happens once the state says the loop has stopped;
// the flag, the partials and the previous term are all loaded before the
// flag is looked at, so the three reads cost one memory round trip.
__device__ inline void pair_tests(const FinalArgs& f) {
    __shared__ double red[kFinalThreads / 64][5];
    NewtonState* st = f.st;
    const bool first = f.mode == PAIR_FIRST;
    const int nq = first ? 5 : 4, stride = first ? 8 : 4;
    const int done_in = st->done;
    double tprev = st->t_prev;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < f.nparts; b += kFinalThreads) {
        // all five loads at once (the fifth repeats the first where there
        // are four partials)
        const double* part = f.partials + stride * (size_t)b;
        double v[5];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = part[q];
        v[4] = part[nq == 5 ? 4 : 0];
#pragma unroll
        for (int q = 0; q < 5; ++q) s[q] += q < nq ? v[q] : 0.0;
    }
    if (f.guard && done_in != 0) return;   // the same in every thread
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int nw = kFinalThreads / 64;
    for (int q = 0; q < 5; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0)
        for (int q = 0; q < 5; ++q) red[wv][q] = s[q];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 0; q < 5; ++q) {
        s[q] = red[0][q];
        for (int w = 1; w < nw; ++w) s[q] += red[w][q];
    }
    if (f.mode == PAIR_START) st->rnorm = sqrt(s[0]);
    if (first) {
        tprev = fabs(f.d0) * sqrt(s[0]);
        st->rnorm = sqrt(s[0]);
        st->hist[0] = tprev;
        for (int q = 0; q < 4; ++q) s[q] = s[q + 1];
    }
    const double wn1 = sqrt(s[0]), pn1 = sqrt(s[1]), wn2 = sqrt(s[2]), pn2 = sqrt(s[3]);
    const double t1 = fabs(f.d1) * wn1;
    const int m1 = f.j + 1;
    const double num1 = tprev + t1;
    if (m1 < kHist) st->hist[m1] = t1;
    int done = 0;
    if (!isfinite(wn1) || !isfinite(pn1) || !isfinite(tprev)) done = 2;
    else if (m1 >= 2 && num1 <= f.tol * pn1) done = 1;
    if (done) {
        st->t_prev = t1;
        st->err = (pn1 > 0.0) ? num1 / pn1 : (num1 == 0.0 ? 0.0 : INFINITY);
        st->pnorm = pn1;
        st->wnorm = wn1;
        st->m = m1;
        st->fix = (done == 1) ? f.d2 : 0.0;
        st->fixbuf = f.outbuf;
        st->done = done;
        return;
    }
    const double t2 = fabs(f.d2) * wn2;
    const int m2 = f.j + 2;
    const double num2 = t1 + t2;
    if (m2 < kHist) st->hist[m2] = t2;
    if (!isfinite(wn2) || !isfinite(pn2)) done = 2;
    else if (m2 >= 2 && num2 <= f.tol * pn2) done = 1;
    st->t_prev = t2;
    st->err = (pn2 > 0.0) ? num2 / pn2 : (num2 == 0.0 ? 0.0 : INFINITY);
    st->pnorm = pn2;
    st->wnorm = wn2;
    st->m = m2;
    st->fix = 0.0;
    st->done = done;
}

// Face weight of the face of cell c towards a neighbour with coefficient
// anb: the mean of the two coefficients if the neighbour exists; for a
// missing neighbour the cell's own coefficient under homogeneous Dirichlet
// (the neighbour's value is 0) and nothing under zero-flux Neumann.
template <class TC>
__device__ __forceinline__ TC face_weight(bool exists, bool dir, TC ac, TC anb) {
    return exists ? (TC)0.5 * (ac + anb) : (dir ? ac : (TC)0);
}

// Workgroup b runs on XCD b % 8; this maps it to a tile index so that each
// XCD owns one contiguous run of tiles (neighbouring tiles share its L2).
__device__ __forceinline__ int xcd_tile(int per_xcd) {
    const int b = blockIdx.x;
    return (b % kXcd) * per_xcd + b / kXcd;
}

}  // namespace expi
