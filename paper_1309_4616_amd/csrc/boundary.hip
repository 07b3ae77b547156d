// The boundary term of inhomogeneous Dirichlet data as a kernel of its own
// (Sec. III-A: with expensive boundary functions the paper moves their
// evaluation out of the stencil kernel into a separate launch).
//
// After a sweep that treated the data as zero, y += scale * b_f, where b_f
// at a boundary-adjacent point sums a_c f(boundary node) / h_d^2 over the
// point's missing neighbours.  One thread per point of the boundary layer;
// each point is owned by exactly one thread, which adds all of its faces:
//   part Z: the planes k = 0 and k = n2 - 1 (whole planes),
//   part Y: the rows j = 0 and j = n1 - 1 of the planes 1 .. n2 - 2,
//   part X: the columns i = 0 and i = n0 - 1 of the remaining rows.
// At 256^3 that is 2.3% of the points; the sweep it follows moves the rest.
#include "expi_internal.h"

namespace expi {
namespace {

struct BoundaryArgs {
    void* y;
    const double *tx, *ty, *tz, *field;
    double c0, c1, scale;
    double h[3];
    int n[3];
    int coef, kind;
    int64_t cz, cy, cx;   // points of parts Z, Y, X
};

__device__ __forceinline__ double fvalue(int kind, double x, double y, double z) {
    if (kind == EXPI_BDATA_Z1MZ_XY) return z * (1.0 - z) * x * y;
    return sin(3.14159265358979323846 * z) * exp(-x * y);
}

template <class T>
__global__ __launch_bounds__(256) void boundary_kernel(BoundaryArgs b) {
    const int64_t total = b.cz + b.cy + b.cx;
    const int n0 = b.n[0], n1 = b.n[1], n2 = b.n[2];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        int i, j, k;
        if (t < b.cz) {
            const int64_t plane = t / ((int64_t)n0 * n1), r = t % ((int64_t)n0 * n1);
            k = plane == 0 ? 0 : n2 - 1;
            i = (int)(r % n0);
            j = (int)(r / n0);
        } else if (t < b.cz + b.cy) {
            const int64_t u = t - b.cz, per = (int64_t)n0 * (n2 - 2);
            const int64_t side = u / per, r = u % per;
            j = side == 0 ? 0 : n1 - 1;
            i = (int)(r % n0);
            k = 1 + (int)(r / n0);
        } else {
            const int64_t u = t - b.cz - b.cy, per = (int64_t)(n1 - 2) * (n2 - 2);
            const int64_t side = u / per, r = u % per;
            i = side == 0 ? 0 : n0 - 1;
            j = 1 + (int)(r % (n1 - 2));
            k = 1 + (int)(r / (n1 - 2));
        }
        const int64_t idx = i + (int64_t)n0 * (j + (int64_t)n1 * k);
        double ac = b.c0;
        if (b.coef == EXPI_COEF_SEPARABLE) ac = b.c0 + b.c1 * (b.tz[k] * b.ty[j]) * b.tx[i];
        else if (b.coef == EXPI_COEF_FIELD) ac = b.field[idx];
        const double x = (i + 1) * b.h[0], y = (j + 1) * b.h[1], z = (k + 1) * b.h[2];
        const double X1 = (n0 + 1) * b.h[0], Y1 = (n1 + 1) * b.h[1], Z1 = (n2 + 1) * b.h[2];
        const double ihx = 1.0 / (b.h[0] * b.h[0]), ihy = 1.0 / (b.h[1] * b.h[1]),
                     ihz = 1.0 / (b.h[2] * b.h[2]);
        double bt = 0.0;
        if (i == 0) bt += ihx * fvalue(b.kind, 0.0, y, z);
        if (i == n0 - 1) bt += ihx * fvalue(b.kind, X1, y, z);
        if (j == 0) bt += ihy * fvalue(b.kind, x, 0.0, z);
        if (j == n1 - 1) bt += ihy * fvalue(b.kind, x, Y1, z);
        if (k == 0) bt += ihz * fvalue(b.kind, x, y, 0.0);
        if (k == n2 - 1) bt += ihz * fvalue(b.kind, x, y, Z1);
        T* yy = static_cast<T*>(b.y);
        yy[idx] = (T)((double)yy[idx] + b.scale * ac * bt);
    }
}

}  // namespace

hipError_t launch_boundary(const Op& op, double scale, void* y, int t, hipStream_t s) {
    if (op.kind != 0 || op.dim != 3 || op.bdata == EXPI_BDATA_NONE) return hipErrorInvalidValue;
    BoundaryArgs b{};
    b.y = y;
    b.tx = op.tx;
    b.ty = op.ty;
    b.tz = op.tz;
    b.field = op.field;
    b.c0 = op.c0;
    b.c1 = op.c1;
    b.scale = scale;
    b.coef = op.coef;
    b.kind = op.bdata;
    for (int d = 0; d < 3; ++d) {
        b.h[d] = op.h[d];
        b.n[d] = op.n[d];
    }
    const int64_t n0 = op.n[0], n1 = op.n[1], n2 = op.n[2];
    const int64_t sz = n2 > 1 ? 2 : 1, sy = n1 > 1 ? 2 : 1, sx = n0 > 1 ? 2 : 1;
    b.cz = sz * n0 * n1;
    b.cy = sy * n0 * std::max<int64_t>(n2 - 2, 0);
    b.cx = sx * std::max<int64_t>(n1 - 2, 0) * std::max<int64_t>(n2 - 2, 0);
    int64_t blocks = (b.cz + b.cy + b.cx + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    if (t == 0)
        hipLaunchKernelGGL(boundary_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, b);
    else
        hipLaunchKernelGGL(boundary_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace expi
