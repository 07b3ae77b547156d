// Two consecutive Newton products per pass on 2D constant-coefficient
// stencils (two steps of the Newton recurrence of Sec. III-C): the operator
// path's pair sweep for 2D grids, with the launch contract of the 3D pair
// sweep (pair.hip: PairArgs, modes PAIR_NEWTON and PAIR_FIRST, its finalize
// and stop tests).
//
// A wave owns a tile: a strip of 64 V points of `march` rows.  It forms
// w_{j+1} in registers on the strip, on the point just beyond each end of it
// (lane 0 the left one, lane 63 the right one, from one more column of w_j
// and the point beyond that, which lanes 1 and 62 load in the same
// instruction and hand over by a lane shuffle) and on the row above and
// below the tile; then w_{j+2} and p on the tile.  Per point w_j and p are
// read once and w_{j+2} and p written once, for two products.  The waves of
// a workgroup take tiles in grid-stride order over an XCD-major wave index
// and combine their norm sums into the workgroup's partials.
#include "sweep_common.h"

namespace expi {
namespace {

constexpr int kP2Waves = 4;     // waves per workgroup
constexpr int kP2March = 16;    // rows per tile by default (a multiple of 4)
constexpr int kP2MaxMarch = 64; // rows per tile at most
constexpr int kP2MaxGrid = 512; // workgroups at most (partials: 8 doubles each)

template <class TW, int V>
struct Pack2 {
    TW v[V];
};

// V values of the storage type by buffer instructions: the row offset in a
// scalar register, the lane's column offset fixed for the march.
template <class TW, int V>
__device__ __forceinline__ void bld2(__amdgpu_buffer_rsrc_t r, int voff, int soff, TW (&o)[V]) {
    constexpr int N = (int)sizeof(TW) * V;
    Pack2<TW, V> p;
    if constexpr (N == 4)
        p = __builtin_bit_cast(Pack2<TW, V>, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else if constexpr (N == 8)
        p = __builtin_bit_cast(Pack2<TW, V>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        p = __builtin_bit_cast(Pack2<TW, V>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = p.v[v];
}

// Stores of at most 8 bytes: a store of more bytes needs a wait state before
// its data registers are written again, which the compiler has been seen to
// omit.
template <class TW, int V>
__device__ __forceinline__ void bst2(__amdgpu_buffer_rsrc_t r, int voff, int soff, const TW (&o)[V]) {
    typedef unsigned U2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int h = 0; h < ((int)sizeof(TW) * V + 7) / 8; ++h) {
        if constexpr (sizeof(TW) * V == 4) {
            Pack2<TW, 1> q;
            q.v[0] = o[0];
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, q), r, voff, soff, 0);
        } else if constexpr (sizeof(TW) == 4) {
            Pack2<TW, 2> q;
            q.v[0] = o[2 * h];
            q.v[1] = o[2 * h + 1];
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, q), r, voff + 8 * h, soff, 0);
        } else {
            Pack2<TW, 1> q;
            q.v[0] = o[h];
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, q), r, voff + 8 * h, soff, 0);
        }
    }
}

// One tile (t0, t1) of products j+1 and j+2 (MODE PAIR_NEWTON: from w_j and
// p_j; PAIR_FIRST: from r = w_0, with p_1 = d_0 r + d_1 w_1).  A point's
// product is written as sum over faces of (alpha f) w_nb +
// (beta - alpha sum f) w_c (face weights f = c0/h^2; 0 towards a neighbour
// that does not exist, which under homogeneous Dirichlet conditions still
// takes its share of the diagonal).  IO (only the interior rows): the
// operator's rows of the outermost layer of points are zero, so there the
// product is beta w_c.  Adds the tile's sums to s:
// PAIR_NEWTON ||w_{j+1}||^2, ||p_{j+1}||^2, ||w_{j+2}||^2, ||p_{j+2}||^2;
// PAIR_FIRST ||r||^2 first, then the same four.
template <class TW, int V, int MODE, bool IO>
__device__ void pair2d_tile(const PairArgs& a, int t0, int t1, int march, double (&s)[5]) {
    using TC = TW;
    constexpr int sz = (int)sizeof(TW);
    constexpr bool kFirst = (MODE == PAIR_FIRST);
    const int lane = threadIdx.x & 63;
    const int n0 = a.n[0], n1 = a.n[1];
    const int i0 = t0 * 64 * V;
    const int i = i0 + lane * V;
    const int kb = t1 * march, ke = min(kb + march, n1);
    const bool active = i < n0;
    const int ic = active ? i : (n0 - V);
    const int xe = (lane == 0) ? i0 - 1 : (lane == 63 ? i0 + 64 * V : ic);
    const int xg = (lane == 1) ? i0 - 2 : (lane == 62 ? i0 + 64 * V + 1 : xe);
    const int gsrc = (lane == 0) ? 1 : (lane == 63 ? 62 : lane);
    const int nbytes = n0 * n1 * sz;
    const __amdgpu_buffer_rsrc_t rw =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.x), 0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(a.out, 0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(a.p, 0, nbytes, 0x00020000);
    const int vo = ic * sz;
    const int vg = min(max(xg, 0), n0 - 1) * sz;
    auto roff = [&](int k) { return n0 * min(max(k, 0), n1 - 1) * sz; };
    auto g_load = [&](int k) -> TC {
        TC t[1];
        bld2<TW, 1>(rw, vg, roff(k), t);
        return t[0];
    };
    const bool dir = (a.bc == EXPI_DIRICHLET0);
    const TC alpha = (TC)a.alpha;
    const TC beta1 = (TC)a.beta1, beta2 = (TC)a.beta2;
    const TC d0 = (TC)a.d0, d1 = (TC)a.d1, d2 = (TC)a.d2;
    const TC fx = (TC)a.c0ih[0], fy = (TC)a.c0ih[1];
    TC axm[V + 1], axq[V + 1], adx[V + 1];
    bool xb[V + 1];   // IO: a point of the outermost columns
#pragma unroll
    for (int v = 0; v <= V; ++v) {
        const int x = (v < V) ? i + v : xe;
        const bool em = x > 0, eq = x < n0 - 1;
        xb[v] = IO && !(em && eq);
        axm[v] = em ? alpha * fx : (TC)0;
        axq[v] = eq ? alpha * fx : (TC)0;
        adx[v] = alpha * (((em || dir) ? fx : (TC)0) + ((eq || dir) ? fx : (TC)0));
    }
    auto yw = [&](int q, TC beta, TC& aym, TC& ayq, TC& cdy, bool& rb) {
        const bool em = q > 0, eq = q < n1 - 1;
        rb = IO && !(em && eq);   // IO: a point of the outermost rows
        aym = em ? alpha * fy : (TC)0;
        ayq = eq ? alpha * fy : (TC)0;
        cdy = beta - alpha * (((em || dir) ? fy : (TC)0) + ((eq || dir) ? fy : (TC)0));
    };
    auto prod = [&](int v, TC wl, TC wr, TC wm, TC wq, TC wc, TC aym, TC ayq, TC cdy, TC beta, bool rb) -> TC {
        const TC u = axm[v] * wl + axq[v] * wr + aym * wm + ayq * wq + (cdy - adx[v]) * wc;
        if constexpr (IO) return (xb[v] || rb) ? beta * wc : u;
        else return u;
    };
    auto form_u = [&](const TC (&wm)[V], const TC (&wc)[V], const TC (&wq)[V], TC gm, TC gc, TC gq, int q,
                      TC (&u)[V], TC& ue) {
        TC aym, ayq, cdy;
        bool rb;
        yw(q, beta1, aym, ayq, cdy, rb);
        TC left = __shfl_up(wc[V - 1], 1, 64);
        TC right = __shfl_down(wc[0], 1, 64);
        const TC far = __shfl(gc, gsrc, 64);
        if (lane == 0) left = gc;
        if (lane == 63) right = gc;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const TC wl = (v > 0) ? wc[v - 1] : left;
            const TC wr = (v < V - 1) ? wc[v + 1] : right;
            u[v] = (TC)(TW)prod(v, wl, wr, wm[v], wq[v], wc[v], aym, ayq, cdy, beta1, rb);
        }
        const TC el = (lane == 63) ? wc[V - 1] : far;
        const TC er = (lane == 63) ? far : wc[0];
        ue = (TC)(TW)prod(V, el, er, gm, gq, gc, aym, ayq, cdy, beta1, rb);
    };
    // register queues indexed by row modulo 4 (the march is unrolled four
    // rows per block, so the queues rotate by renaming)
    TC W[4][V], P[4][V], U[4][V], G[4], Ue[2];
    {
        bld2<TW, V>(rw, vo, roff(kb - 2), W[2]);
        bld2<TW, V>(rw, vo, roff(kb - 1), W[3]);
        bld2<TW, V>(rw, vo, roff(kb), W[0]);
        bld2<TW, V>(rw, vo, roff(kb + 1), W[1]);
        G[2] = g_load(kb - 2);
        G[3] = g_load(kb - 1);
        G[0] = g_load(kb);
        G[1] = g_load(kb + 1);
        if constexpr (!kFirst) {
            bld2<TW, V>(rp, vo, roff(kb), P[0]);
            bld2<TW, V>(rp, vo, roff(kb + 1), P[1]);
        }
        TC ue_m;
        form_u(W[2], W[3], W[0], G[2], G[3], G[0], kb - 1, U[3], ue_m);
        bld2<TW, V>(rw, vo, roff(kb + 2), W[2]);
        G[2] = g_load(kb + 2);
        form_u(W[3], W[0], W[1], G[3], G[0], G[1], kb, U[0], Ue[0]);
    }
    for (int k0 = kb; k0 < ke; k0 += 4) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int k = k0 + st;
            const bool valid = k < ke;
            TC wk[V];   // r on row k (PAIR_FIRST)
#pragma unroll
            for (int v = 0; v < V; ++v) wk[v] = W[st & 3][v];
            bld2<TW, V>(rw, vo, roff(k + 3), W[(st + 3) & 3]);
            G[(st + 3) & 3] = g_load(k + 3);
            if constexpr (!kFirst) bld2<TW, V>(rp, vo, roff(k + 2), P[(st + 2) & 3]);
            form_u(W[st & 3], W[(st + 1) & 3], W[(st + 2) & 3], G[st & 3], G[(st + 1) & 3], G[(st + 2) & 3],
                   k + 1, U[(st + 1) & 3], Ue[(st + 1) & 1]);
            const TC* um = U[(st + 3) & 3];
            const TC* uc = U[st & 3];
            const TC* uq = U[(st + 1) & 3];
            TC aym, ayq, cdy;
            bool rb;
            yw(k, beta2, aym, ayq, cdy, rb);
            TC left = __shfl_up(uc[V - 1], 1, 64);
            TC right = __shfl_down(uc[0], 1, 64);
            if (lane == 0) left = Ue[st & 1];
            if (lane == 63) right = Ue[st & 1];
            TC wo[V], po[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const TC wl = (v > 0) ? uc[v - 1] : left;
                const TC wr = (v < V - 1) ? uc[v + 1] : right;
                const TC u2 = (TC)(TW)prod(v, wl, wr, um[v], uq[v], uc[v], aym, ayq, cdy, beta2, rb);
                TC p1;
                if constexpr (kFirst) p1 = (TC)(TW)(d0 * wk[v] + d1 * uc[v]);
                else p1 = (TC)(TW)(P[st & 3][v] + d1 * uc[v]);
                const TC p2 = (TC)(TW)(p1 + d2 * u2);
                wo[v] = u2;
                po[v] = p2;
                if (active && valid) {
                    if constexpr (kFirst) s[0] += (double)wk[v] * (double)wk[v];
                    constexpr int o = kFirst ? 1 : 0;
                    s[o] += (double)uc[v] * (double)uc[v];
                    s[o + 1] += (double)p1 * (double)p1;
                    s[o + 2] += (double)u2 * (double)u2;
                    s[o + 3] += (double)p2 * (double)p2;
                }
            }
            // lanes past the row end, and steps past the tile, store past
            // the buffer (dropped)
            const int vs = (active && valid) ? vo : nbytes;
            bst2<TW, V>(ro, vs, roff(k), wo);
            bst2<TW, V>(rp, vs, roff(k), po);
        }
    }
}

template <class TW, int V, int MODE, bool IO>
__global__ __launch_bounds__(kP2Waves * 64) void pair2d_sweep(PairArgs a, int tiles0, int ntiles, int march) {
    if (a.guard && a.st->done != 0) return;
    constexpr int N = (MODE == PAIR_FIRST) ? 5 : 4;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int nw = blockDim.x >> 6;
    const int G = gridDim.x * nw;
    const int L = __builtin_amdgcn_readfirstlane(xcd_tile(gridDim.x / kXcd) * nw + (int)(threadIdx.x >> 6));
    for (int t = L; t < ntiles; t += G) pair2d_tile<TW, V, MODE, IO>(a, t % tiles0, t / tiles0, march, s);
    double v[N];
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = s[q];
    finish_sweep_n<N>(a.partials, N == 5 ? 8 : 4, v);
}

template <class TW, int V, int MODE>
void go_io(bool io, int grid, int tiles0, int ntiles, int march, const PairArgs& a, hipStream_t s) {
    if (io)
        hipLaunchKernelGGL((pair2d_sweep<TW, V, MODE, true>), dim3(grid), dim3(64 * kP2Waves), 0, s, a, tiles0,
                           ntiles, march);
    else
        hipLaunchKernelGGL((pair2d_sweep<TW, V, MODE, false>), dim3(grid), dim3(64 * kP2Waves), 0, s, a, tiles0,
                           ntiles, march);
}

template <class TW, int MODE>
hipError_t go2(int vec, int grid, int tiles0, int ntiles, int march, const PairArgs& a, hipStream_t s) {
    const bool io = (a.bc == EXPI_INTERIOR_ONLY);
    if constexpr (sizeof(TW) == 4) {
        if (vec == 4) {
            go_io<TW, 4, MODE>(io, grid, tiles0, ntiles, march, a, s);
            return hipGetLastError();
        }
    }
    if (vec == 2) go_io<TW, 2, MODE>(io, grid, tiles0, ntiles, march, a, s);
    else go_io<TW, 1, MODE>(io, grid, tiles0, ntiles, march, a, s);
    return hipGetLastError();
}

}  // namespace

// Rows per tile a caller may ask for: a multiple of 4 up to kP2MaxMarch.
bool pair2d_rows_valid(int rows) { return rows >= 4 && rows <= kP2MaxMarch && rows % 4 == 0; }

bool pair2d_supported(const Op& op, int tw) {
    (void)tw;
    // buffer offsets are 32-bit byte offsets: below 2^31 bytes in FP64
    return op.kind == 0 && op.dim == 2 && op.coef == EXPI_COEF_CONST &&
           (op.bc == EXPI_DIRICHLET0 || op.bc == EXPI_NEUMANN0 || op.bc == EXPI_INTERIOR_ONLY) &&
           op.size * 8 < ((int64_t)1 << 31) - 64;
}

// rows: rows per tile (pair2d_rows_valid), or 0 for 16, fewer where the
// grid has too few tiles of 16 rows.
hipError_t launch_pair2d(const Op& op, int tw, PairArgs a, hipStream_t s, hipEvent_t after_sweep, bool finalize,
                         int mode, int cus, int rows) {
    if (mode != PAIR_NEWTON && mode != PAIR_FIRST) return hipErrorInvalidValue;
    if (rows != 0 && !pair2d_rows_valid(rows)) return hipErrorInvalidValue;
    for (int d = 0; d < 2; ++d) {
        a.n[d] = op.n[d];
        a.ih2[d] = 1.0 / (op.h[d] * op.h[d]);
        a.c0ih[d] = op.c0 * a.ih2[d];
    }
    a.bc = op.bc;
    // four FP32 points per lane where rows start on 16-byte boundaries, else
    // two points where they start on 2-value boundaries, else one
    const size_t al = 2 * (tw == 1 ? 4 : 8);
    const bool aligned = ((uintptr_t)a.x % al == 0) && ((uintptr_t)a.out % al == 0) && ((uintptr_t)a.p % al == 0);
    const bool al16 = ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.out % 16 == 0) && ((uintptr_t)a.p % 16 == 0);
    const int vec = (tw == 1 && op.n[0] % 4 == 0 && al16) ? 4 : ((op.n[0] % 2 == 0 && aligned) ? 2 : 1);
    const int tiles0 = (op.n[0] + 64 * vec - 1) / (64 * vec);
    // rows per tile: 16, or fewer (a multiple of 4) where the grid has too
    // few tiles of 16 rows for a wave on every SIMD
    const int slots = 4 * std::max(cus, kXcd);
    int march = rows ? rows : kP2March;
    while (!rows && march > 4 && (long long)tiles0 * ((op.n[1] + march - 1) / march) < slots) march /= 2;
    const int ntiles = tiles0 * ((op.n[1] + march - 1) / march);
    // enough workgroups for every tile a wave of its own, up to four per CU,
    // a multiple of the XCD count
    const int want = std::min((ntiles + kP2Waves - 1) / kP2Waves, 4 * std::max(cus, kXcd));
    const int grid = std::min(kP2MaxGrid, std::max(kXcd, (want + kXcd - 1) / kXcd * kXcd));
    hipError_t e;
    if (mode == PAIR_FIRST)
        e = tw == 1 ? go2<float, PAIR_FIRST>(vec, grid, tiles0, ntiles, march, a, s)
                    : go2<double, PAIR_FIRST>(vec, grid, tiles0, ntiles, march, a, s);
    else
        e = tw == 1 ? go2<float, PAIR_NEWTON>(vec, grid, tiles0, ntiles, march, a, s)
                    : go2<double, PAIR_NEWTON>(vec, grid, tiles0, ntiles, march, a, s);
    if (e != hipSuccess) return e;
    if (after_sweep) {
        e = hipEventRecord(after_sweep, s);
        if (e != hipSuccess) return e;
    }
    if (!finalize) return hipSuccess;
    return launch_pair_finalize(a.partials, a.st, grid, a.j, a.guard, a.d0, a.d1, a.d2, a.tol, mode, a.outbuf, s);
}

}  // namespace expi
