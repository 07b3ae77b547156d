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
