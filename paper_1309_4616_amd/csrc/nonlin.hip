// Pointwise nonlinearity kernels (Sec. III-C).
//
// g(u) of eq. (5) evaluated over a vector: one read and one write per point,
// and a division and an exponential that make the kernel arithmetic-heavy
// (Table III times exactly this).  Each thread handles 16 bytes per access
// (two doubles or four floats) in a grid-stride loop over the vector; the
// tail that does not fill a 16-byte group is done one element per thread.
// Also the difference g(U) - g(u) that the second stage of the exponential
// Runge-Kutta step needs.
#include "expi_internal.h"
#include "nonlin.h"

namespace expi {
namespace {

template <class T>
struct Vec16;
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};

template <class T, int KIND>
__global__ __launch_bounds__(256) void nonlin_kernel(int64_t n, const T* __restrict__ u,
                                                     T* __restrict__ g) {
    using V = typename Vec16<T>::type;
    constexpr int NV = Vec16<T>::n;
    const int64_t groups = n / NV;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const V* __restrict__ uv = reinterpret_cast<const V*>(u);
    V* __restrict__ gv = reinterpret_cast<V*>(g);
    for (int64_t q = t0; q < groups; q += stride) {
        const V x = uv[q];
        V y;
#pragma unroll
        for (int e = 0; e < NV; ++e) y[e] = g_eval<T>(KIND, x[e]);
        __builtin_nontemporal_store(y, &gv[q]);
    }
    for (int64_t i = groups * NV + t0; i < n; i += stride) g[i] = g_eval<T>(KIND, u[i]);
}

template <int KIND>
__global__ __launch_bounds__(256) void gdiff_kernel(int64_t n, const double* __restrict__ U,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = g_eval<double>(KIND, U[i]) - g_eval<double>(KIND, u[i]);
}

unsigned grid_for(int64_t items) {
    int64_t blocks = (items + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

template <class T>
hipError_t go(int kind, int64_t n, const void* u, void* g, hipStream_t s) {
    const T* ut = static_cast<const T*>(u);
    T* gt = static_cast<T*>(g);
    const unsigned grid = grid_for(n / Vec16<T>::n + 1);
    switch (kind) {
        case EXPI_G_CUBIC:
            hipLaunchKernelGGL((nonlin_kernel<T, EXPI_G_CUBIC>), dim3(grid), dim3(256), 0, s, n, ut, gt);
            break;
        case EXPI_G_COMBUSTION:
            hipLaunchKernelGGL((nonlin_kernel<T, EXPI_G_COMBUSTION>), dim3(grid), dim3(256), 0, s, n, ut, gt);
            break;
        case EXPI_G_COMBUSTION_FAST:
            hipLaunchKernelGGL((nonlin_kernel<T, EXPI_G_COMBUSTION_FAST>), dim3(grid), dim3(256), 0, s, n,
                               ut, gt);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_nonlin(int kind, int64_t n, const void* u, void* g, int dtype, hipStream_t s) {
    return dtype == EXPI_F32 ? go<float>(kind, n, u, g, s) : go<double>(kind, n, u, g, s);
}

hipError_t launch_gdiff(int kind, int64_t n, const double* U, const double* u, double* out,
                        hipStream_t s) {
    const unsigned grid = grid_for(n);
    switch (kind) {
        case EXPI_G_CUBIC:
            hipLaunchKernelGGL(gdiff_kernel<EXPI_G_CUBIC>, dim3(grid), dim3(256), 0, s, n, U, u, out);
            break;
        case EXPI_G_COMBUSTION:
            hipLaunchKernelGGL(gdiff_kernel<EXPI_G_COMBUSTION>, dim3(grid), dim3(256), 0, s, n, U, u, out);
            break;
        case EXPI_G_COMBUSTION_FAST:
            hipLaunchKernelGGL(gdiff_kernel<EXPI_G_COMBUSTION_FAST>, dim3(grid), dim3(256), 0, s, n, U, u,
                               out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace expi
