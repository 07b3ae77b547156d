// Matrix-free stencil sweeps (Sec. III-A, III-B) for gfx950.
//
// One kernel template covers the 5-point (2D) and 7-point (3D) operator
// A = div(a grad .) with the boundary handling folded in, every coefficient
// kind, and every epilogue of the hot path (sweep.hip describes them).  The
// central use is the fused Newton product of the Leja interpolation
// (Sec. III-C) on eq. (3)'s (alpha A + beta I) w.
//
// Layout and traversal, designed for HBM traffic (about 0.4 flop/byte):
//  * a wave owns 64*V consecutive x points of one row (V = 2: 16-byte
//    loads and stores); the x neighbours come from the neighbouring lanes by
//    cross-lane shuffles, only the two wave-edge lanes load one value each;
//  * each thread marches along the slowest axis (z in 3D, y in 2D) with a
//    four-slot register queue of planes: plane k finds k-1, k, k+1 in
//    registers while k+2 streams in from HBM, and p of k+1 likewise.  The
//    march is unrolled four-fold so the queue rotates by renaming, not
//    copies.  Each stage first issues the next plane's cache-served loads,
//    then its HBM loads; since the memory counter retires in order, waiting
//    for a plane's neighbours then never waits for the two newest HBM loads;
//  * 3D: the waves of a workgroup hold consecutive y rows; the y neighbours
//    are loads that the workgroup itself or the neighbouring tile brought
//    into L1/L2;
//  * tiles are mapped so that each XCD owns a contiguous run of them;
//  * boundaries are predicated face terms, no ghost cells; inhomogeneous
//    Dirichlet data (Sec. III-A) are evaluated at the boundary-adjacent
//    points by instantiations of their own (EPI_APPLY_BD, EPI_START_BD);
//  * the D-Laplacian of Sec. III-B computes D = 1/sqrt(1 + x^2 + y^2) in the
//    kernel: once per thread before the march in 3D (D does not depend on
//    z), once per point and plane in 2D.
#include "stencil_tile.h"

namespace expi {
namespace {

template <int DIM, int COEF, int EPI, class TIN, class TOUT, int V>
__global__ __launch_bounds__(kMaxWaves * 64) void stencil_sweep(SweepArgs a) {
    if (a.guard && a.st->done != 0) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (EPI == EPI_GERSH) {
        s0 = INFINITY;
        s1 = -INFINITY;
    }
    const int L = xcd_tile(a.per_xcd);
    if (L < a.ntiles) {
        const int t0 = L % a.tiles[0];
        const int rem = L / a.tiles[0];
        const int t1 = rem % a.tiles[1];
        const int t2 = rem / a.tiles[1];
        tile::stencil_tile<DIM, COEF, EPI, TIN, TOUT, V>(a, t0, t1, t2, s0, s1, s2);
    }
    if (EPI == EPI_NEWTON || EPI == EPI_FIRST || EPI == EPI_GERSH) finish_sweep<EPI>(a, s0, s1, s2);
}


template <int DIM, int COEF, int EPI, class TIN, class TOUT>
hipError_t go(const Geom& g, const SweepArgs& a, hipStream_t s) {
    if (g.vec == 2)
        hipLaunchKernelGGL((stencil_sweep<DIM, COEF, EPI, TIN, TOUT, 2>), dim3(g.grid),
                           dim3(64 * g.waves), 0, s, a);
    else
        hipLaunchKernelGGL((stencil_sweep<DIM, COEF, EPI, TIN, TOUT, 1>), dim3(g.grid),
                           dim3(64 * g.waves), 0, s, a);
    return hipGetLastError();
}

template <int DIM, int COEF>
hipError_t dispatch(const Geom& g, int epi, int tin, int tout, const SweepArgs& a, hipStream_t s) {
    // boundary data of a 3D Dirichlet stencil (not with the D-Laplacian)
    constexpr bool kBD = (DIM == 3 && COEF != EXPI_COEF_DLAP);
    if (a.bdata && (epi == EPI_APPLY || epi == EPI_START)) {
        if constexpr (kBD) {
            if (epi == EPI_APPLY) {
                if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_APPLY_BD, double, double>(g, a, s);
                if (tin == 1 && tout == 1) return go<DIM, COEF, EPI_APPLY_BD, float, float>(g, a, s);
            } else {
                if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_START_BD, double, double>(g, a, s);
                if (tin == 0 && tout == 1) return go<DIM, COEF, EPI_START_BD, double, float>(g, a, s);
            }
        }
        return hipErrorInvalidValue;
    }
    switch (epi) {
        case EPI_APPLY:
            if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_APPLY, double, double>(g, a, s);
            if (tin == 1 && tout == 1) return go<DIM, COEF, EPI_APPLY, float, float>(g, a, s);
            break;
        case EPI_NEWTON:
            if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_NEWTON, double, double>(g, a, s);
            if (tin == 1 && tout == 1) return go<DIM, COEF, EPI_NEWTON, float, float>(g, a, s);
            break;
        case EPI_FIRST:
            if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_FIRST, double, double>(g, a, s);
            if (tin == 0 && tout == 1) return go<DIM, COEF, EPI_FIRST, double, float>(g, a, s);
            if (tin == 1 && tout == 1) return go<DIM, COEF, EPI_FIRST, float, float>(g, a, s);
            break;
        case EPI_START:
            if (a.gmode == G_CUBIC_SELF) {
                if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_START_SELF, double, double>(g, a, s);
                if (tin == 0 && tout == 1) return go<DIM, COEF, EPI_START_SELF, double, float>(g, a, s);
                break;
            }
            if (tin == 0 && tout == 0) return go<DIM, COEF, EPI_START, double, double>(g, a, s);
            if (tin == 0 && tout == 1) return go<DIM, COEF, EPI_START, double, float>(g, a, s);
            if (tin == 1 && tout == 1) return go<DIM, COEF, EPI_START, float, float>(g, a, s);
            break;
        case EPI_GERSH:
            return go<DIM, COEF, EPI_GERSH, double, double>(g, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_stencil(const Op& op, const Geom& g, int epi, int tin, int tout,
                          const SweepArgs& a, hipStream_t s) {
    if (op.dim == 3) {
        switch (op.coef) {
            case EXPI_COEF_CONST: return dispatch<3, EXPI_COEF_CONST>(g, epi, tin, tout, a, s);
            case EXPI_COEF_SEPARABLE: return dispatch<3, EXPI_COEF_SEPARABLE>(g, epi, tin, tout, a, s);
            case EXPI_COEF_FIELD: return dispatch<3, EXPI_COEF_FIELD>(g, epi, tin, tout, a, s);
            case EXPI_COEF_DLAP: return dispatch<3, EXPI_COEF_DLAP>(g, epi, tin, tout, a, s);
        }
    } else {
        switch (op.coef) {
            case EXPI_COEF_CONST: return dispatch<2, EXPI_COEF_CONST>(g, epi, tin, tout, a, s);
            case EXPI_COEF_SEPARABLE: return dispatch<2, EXPI_COEF_SEPARABLE>(g, epi, tin, tout, a, s);
            case EXPI_COEF_FIELD: return dispatch<2, EXPI_COEF_FIELD>(g, epi, tin, tout, a, s);
            case EXPI_COEF_DLAP: return dispatch<2, EXPI_COEF_DLAP>(g, epi, tin, tout, a, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace expi
