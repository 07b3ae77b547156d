// Two consecutive Newton products of the Leja interpolation in one sweep
// (Sec. III-C; the products are eq. (3)) for 3D stencils on gfx950:
//
//   w_{j+1} = alpha A w_j     + beta_j     w_j,     p_{j+1} = p_j     + d_{j+1} w_{j+1}
//   w_{j+2} = alpha A w_{j+1} + beta_{j+1} w_{j+1}, p_{j+2} = p_{j+1} + d_{j+2} w_{j+2}
//
// with the partial sums of ||w_{j+1}||^2, ||p_{j+1}||^2, ||w_{j+2}||^2 and
// ||p_{j+2}||^2 per workgroup, so that the finalize kernel can apply the
// two-term stop test after each of the two products.  w_{j+1} never goes to
// HBM: the sweep reads w_j and p once and writes w_{j+2} and p once, half
// the traffic of two single products.  Every value is computed by the same
// formula as in the single product, rounded to the storage type where the
// single product stores it.
//
// Layout and traversal:
//  * a workgroup is 16 waves; a wave owns 128 consecutive x points of one row
//    (2 per lane), so a row of n0 <= 512 points takes NX = 1, 2 or 4 waves
//    and the workgroup holds 16/NX rows: R = 16/NX - 2 output rows and one
//    halo row on each side (R = 2 for rows longer than 256 points: the
//    first product is then computed on twice the output rows);
//  * every wave marches along z computing w_{j+1} of its row one plane ahead;
//    the plane goes into a three-plane LDS ring, one barrier per plane, and
//    the inner waves then compute w_{j+2} of the plane behind from their own
//    registers (z neighbours) and the ring (y and wave-edge x neighbours);
//  * w_j streams through a four-slot register queue as in the single sweep
//    (y neighbours are cache-served loads of the neighbouring rows);
//  * the grid has one workgroup per CU slot; the (row tile, plane) units are
//    split into equal contiguous chunks numbered XCD-major, so that the
//    chunks that share halo rows run on the same L2 at the same time.
#include <algorithm>
#include <type_traits>

#include "sweep_common.h"

namespace expi {
namespace {

constexpr int kPairWaves = 16;
constexpr int kPairLds = kPairWaves * 128;   // points of one plane of the w_{j+1} ring
constexpr int kZSeg = 248;                   // planes per marched segment at most
constexpr int kWRingLds = 3072;              // points of one plane of the w_j ring:
                                             // (16/NX + 2) rows of 128 NX points, NX <= 4

// Face weights.  With a(x, y, z) = c0 + c1 X(x) Y(y) Z(z) the weight of the
// face between cells c and c' (the mean of a_c and a_c') is
// c0 + c1 * (product of the other two tables) * (mean of the two values of
// the table along the face's axis); a missing neighbour under homogeneous
// Dirichlet counts with the cell's own coefficient (face value := own value)
// and value 0, under zero-flux Neumann not at all.  So on a plane of a row
// every y and z face weight is A + B X(x) with A, B the same in all lanes,
// and so is the sum of the diagonal parts of those faces.  The x faces keep
// per-lane face values.  The constant coefficient is the case c1 = 0.
template <class TC>
struct RowW {          // per (row, segment): y data of the row
    TC y, gym, gyq;    // Y(y); c1 ihy e Yf for the two y faces
    TC aym, ayq;       // c0 ihy e
    TC ady, gdy;       // diagonal: c0 ihy (d_m + d_q), c1 ihy (d_m Yf_m + d_q Yf_q)
    TC hz;             // c1 ihz Y(y)
};

template <class TC>
struct PlaneW {        // per (row, plane): weights A + B X of the y, z faces
    TC sx;             // x faces: c0 ihx + sx Xf
    TC aym, bym, ayq, byq, azm, bzm, azq, bzq, ad, bd;
};

template <class TC>
struct ZPlane {        // per plane of a segment: the z data of the weights
    TC zc, zfm, zfq;   // Z(z); e_m times the face value towards z-1, e_q times the one towards z+1
    TC zd;             // d_m (face value towards z-1) + d_q (face value towards z+1)
};

// zt: z data of planes zbase, zbase+1, ... in LDS (separable coefficient)
template <int COEF, class TC>
__device__ __forceinline__ PlaneW<TC> plane_weights(const RowW<TC>& r, const ZPlane<TC>* zt, int zbase,
                                                    int q, int n2, bool dir, TC c0ihz, TC c1ihx) {
    PlaneW<TC> w;
    const bool ezm = q > 0, ezq = q < n2 - 1;
    const TC dm = (ezm || dir) ? (TC)1 : (TC)0, dq = (ezq || dir) ? (TC)1 : (TC)0;
    w.aym = r.aym;
    w.ayq = r.ayq;
    w.azm = ezm ? c0ihz : (TC)0;
    w.azq = ezq ? c0ihz : (TC)0;
    w.ad = r.ady + c0ihz * (dm + dq);
    if (COEF == EXPI_COEF_SEPARABLE) {
        const ZPlane<TC>& z = zt[q - zbase];
        w.sx = c1ihx * (r.y * z.zc);
        w.bym = r.gym * z.zc;
        w.byq = r.gyq * z.zc;
        w.bzm = r.hz * z.zfm;
        w.bzq = r.hz * z.zfq;
        w.bd = r.gdy * z.zc + r.hz * z.zd;
    } else {
        w.sx = w.bym = w.byq = w.bzm = w.bzq = w.bd = (TC)0;
    }
    return w;
}

// (A w) at the lane's two points from the values of the points (wc), their
// x neighbours outside the pair (wl, wr, already set for a missing
// neighbour: 0 under Dirichlet, the point's own value otherwise), the y and
// z neighbour values (anything finite where the neighbour is missing: its
// weight is 0) and the weights.
// The face weights of the lane's two points on one plane of its row: the
// x faces left of point 0, between the points and right of point 1, and per
// point the y and z faces and the diagonal.  Both products of a pair sweep
// use the same plane's weights (the second one two iterations later), so
// the FP32 sweep keeps them in registers between the two.
template <class TC>
struct PointW {
    TC wxl, wxc, wxr;
    TC wym[2], wyq[2], wzm[2], wzq[2], d[2];
};

template <int COEF, class TC>
__device__ __forceinline__ PointW<TC> point_weights(const PlaneW<TC>& w, TC c0ihx, const TC (&xd)[5]) {
    // xd: X of the two points, face values left, between, right
    PointW<TC> q;
    TC X[2] = {1, 1};
    if (COEF == EXPI_COEF_SEPARABLE) {
        X[0] = xd[0];
        X[1] = xd[1];
        q.wxl = c0ihx + w.sx * xd[2];
        q.wxc = c0ihx + w.sx * xd[3];
        q.wxr = c0ihx + w.sx * xd[4];
    } else {
        q.wxl = q.wxc = q.wxr = c0ihx;
    }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        if (COEF == EXPI_COEF_SEPARABLE) {
            q.wym[v] = w.aym + w.bym * X[v];
            q.wyq[v] = w.ayq + w.byq * X[v];
            q.wzm[v] = w.azm + w.bzm * X[v];
            q.wzq[v] = w.azq + w.bzq * X[v];
            q.d[v] = w.ad + w.bd * X[v];
        } else {
            q.wym[v] = w.aym;
            q.wyq[v] = w.ayq;
            q.wzm[v] = w.azm;
            q.wzq[v] = w.azq;
            q.d[v] = w.ad;
        }
    }
    return q;
}

// The same weights in another arithmetic type.
template <class TO, class TI>
__device__ __forceinline__ PointW<TO> point_weights_as(const PointW<TI>& q) {
    PointW<TO> r;
    r.wxl = (TO)q.wxl;
    r.wxc = (TO)q.wxc;
    r.wxr = (TO)q.wxr;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        r.wym[v] = (TO)q.wym[v];
        r.wyq[v] = (TO)q.wyq[v];
        r.wzm[v] = (TO)q.wzm[v];
        r.wzq[v] = (TO)q.wzq[v];
        r.d[v] = (TO)q.d[v];
    }
    return r;
}

template <class TC>
__device__ __forceinline__ void aw_pair_w(const TC (&wc)[2], TC wl, TC wr, const TC (&ym)[2],
                                          const TC (&yq)[2], const TC (&zm)[2], const TC (&zq)[2],
                                          const PointW<TC>& q, TC (&aw)[2]) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const TC left = v == 0 ? wl : wc[0];
        const TC right = v == 1 ? wr : wc[1];
        const TC fl = v == 0 ? q.wxl : q.wxc;
        const TC fr = v == 1 ? q.wxr : q.wxc;
        aw[v] = fl * (left - wc[v]) + fr * (right - wc[v]) + q.wym[v] * ym[v] + q.wyq[v] * yq[v] +
                q.wzm[v] * zm[v] + q.wzq[v] * zq[v] - q.d[v] * wc[v];
    }
}

template <int COEF, class TC>
__device__ __forceinline__ void aw_pair(const TC (&wc)[2], TC wl, TC wr, const TC (&ym)[2],
                                        const TC (&yq)[2], const TC (&zm)[2], const TC (&zq)[2],
                                        const PlaneW<TC>& w, TC c0ihx, const TC (&xd)[5], TC (&aw)[2]) {
    aw_pair_w<TC>(wc, wl, wr, ym, yq, zm, zq, point_weights<COEF, TC>(w, c0ihx, xd), aw);
}

template <class T, class TC>
__device__ __forceinline__ void ld2(const T* __restrict__ p, int idx, TC (&o)[2]) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    const T2 t = *reinterpret_cast<const T2*>(p + idx);
    o[0] = (TC)t.x;
    o[1] = (TC)t.y;
}

template <class T, class TC>
__device__ __forceinline__ void st2(T* __restrict__ p, int idx, const TC (&v)[2]) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    T2 t;
    t.x = (T)v[0];
    t.y = (T)v[1];
    *reinterpret_cast<T2*>(p + idx) = t;
}

// Streaming store: the line is not kept in L2 for reuse, which leaves L2 to
// the w_j rows that neighbouring row tiles read again.
template <class T, class TC>
__device__ __forceinline__ void st2_stream(T* __restrict__ p, int idx, const TC (&v)[2]) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    T2 t;
    t.x = (T)v[0];
    t.y = (T)v[1];
    __builtin_nontemporal_store(t, reinterpret_cast<T2*>(p + idx));
}

// Two values to p[idx], idx < 0 dropping the store (buffer store with range
// checking: an offset past the buffer's end writes nothing).  Lets a wave
// issue the same stores on every path, so that the in-order memory counter
// keeps exact counts and waits only for the loads it needs.
template <class T, class TC>
__device__ __forceinline__ void st2_buf(__amdgpu_buffer_rsrc_t r, int idx, const TC (&v)[2], bool stream) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    T2 t;
    t.x = (T)v[0];
    t.y = (T)v[1];
    const int off = idx >= 0 ? idx * (int)sizeof(T) : 0x7ffffff0;
    if constexpr (sizeof(T) == 8) {
        typedef unsigned U4 __attribute__((ext_vector_type(4)));
        if (stream) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, t), r, off, 0, 2);
        else __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, t), r, off, 0, 0);
    } else {
        typedef unsigned U2 __attribute__((ext_vector_type(2)));
        if (stream) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, t), r, off, 0, 2);
        else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, t), r, off, 0, 0);
    }
}

// A value that is the same in every lane, in scalar registers.
__device__ __forceinline__ float uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Whole-wave shifts by one lane through DPP: lane l receives `src` of lane
// l-1 (from_left) or l+1 (from_right); the lane without a source (0, resp.
// 63) keeps `edge`.
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float edge, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, src), CTRL,
                                                                 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double edge, double src) {
    const unsigned long long e = __builtin_bit_cast(unsigned long long, edge);
    const unsigned long long v = __builtin_bit_cast(unsigned long long, src);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)e, (int)(unsigned)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(e >> 32), (int)(unsigned)(v >> 32), CTRL,
                                               0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
constexpr int kDppWaveShr1 = 0x138;   // lane l <- lane l-1
constexpr int kDppWaveShl1 = 0x130;   // lane l <- lane l+1

// MODE (PairMode).  PAIR_FIRST: the pair starts the loop.  It reads the
// start vector r (= w_0), forms p_1 = d_0 r + d_1 w_1 instead of adding to
// a stored p, and reports
// ||r||^2 where the other pairs report ||p_1||^2; the inner rows load r of
// their own row a second time where the other pairs load p (a cache hit:
// the same rows entered the w_j queue two planes earlier).  PAIR_START: x is
// u; the first half forms the start vector r = sigma A u + u - u^3 of an
// exponential Euler step instead of a product, and the second half is
// product 0, w_1 = alpha A r + beta_0 r with p_1 = d_0 r + d_1 w_1 (here
// beta2, d1, d2 carry beta_0, d_0, d_1); r never leaves the chip, and its
// norm goes where the other pairs put ||w_{j+1}||.
template <int COEF, int BC, class TW, int MODE>
__global__ __launch_bounds__(kPairWaves * 64) void pair_sweep(PairArgs a) {
    using TC = compute_t<TW, TW>;
    constexpr bool FIRST = MODE == PAIR_FIRST, START = MODE == PAIR_START;
    // TX: the arithmetic of the first half (w_j, its ring and queues, step
    // 3).  TC except for PAIR_START with FP32 storage: u is read in FP64 and
    // r = sigma A u + u - u^3 is formed in FP64 (A u cancels: formed in FP32
    // from a rounded u it would lose most of its digits), then rounded to
    // FP32 for the ring and product 0, which runs in FP32 like the other
    // FP32 pairs
    using TX = typename std::conditional<START && sizeof(TW) == 4, double, TC>::type;
    // the status flag (the loop has stopped: do nothing) is looked at only
    // at the first barrier, so its load overlaps the first plane loads
    // (a.st is always a valid state record).  A buffer load: a scalar load
    // would be waited for with the first kernel-argument load after it.
    const __amdgpu_buffer_rsrc_t st_r =
        __builtin_amdgcn_make_buffer_rsrc(a.st, 0, (int)sizeof(NewtonState), 0x00020000);
    const int done_v = (int)__builtin_amdgcn_raw_buffer_load_b32(st_r, (int)offsetof(NewtonState, done), 0, 0);
    __shared__ TC ring[3 * kPairLds];     // w_{j+1}: rows y0-1 .. y0+R of three planes
    __shared__ TX wring[3 * kWRingLds];   // w_j: rows y0-2 .. y0+R+1 of three planes
    // z data of the planes of the current segment: read where used through
    // LDS (a vector load there would make the in-order memory counter wait
    // for every prefetch issued before it)
    __shared__ ZPlane<TX> ztab[kZSeg + 8];
    const TX* __restrict__ x = static_cast<const TX*>(a.x);
    TW* __restrict__ out = static_cast<TW*>(a.out);
    TW* __restrict__ pv = static_cast<TW*>(a.p);
    // w_{j+2} and p are written through buffer resources (range-checked
    // stores; the grid holds fewer than 2^31 bytes, see pair_supported)
    const int nbytes = a.n[0] * a.n[1] * a.n[2] * (int)sizeof(TW);
    const __amdgpu_buffer_rsrc_t out_r = __builtin_amdgcn_make_buffer_rsrc(out, 0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t pv_r = __builtin_amdgcn_make_buffer_rsrc(pv, 0, nbytes, 0x00020000);
    // the wave index is the same in every lane; saying so keeps the row data
    // (and everything derived from it) in scalar registers
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NX = a.nxw, R = a.rows;
    const int ry = wv / NX, xq = wv % NX;
    const int RW = 128 * NX;                      // ring row width (>= n0)
    const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
    const int plane = n0 * n1;
    const int i = xq * 128 + lane * 2;            // first of the lane's two x points
    const bool xin = i < n0;                      // n0 is even: both points in the row
    const int ic = xin ? i : n0 - 2;
    constexpr bool dir = BC == EXPI_DIRICHLET0, ionly = BC == EXPI_INTERIOR_ONLY;
    // coefficient times 1/h^2 per axis, formed on the host (kernel
    // arguments stay in scalar registers; products formed here would hold
    // vector registers for the whole sweep)
    const TC alpha = (TC)a.alpha, beta1 = (TC)a.beta1, beta2 = (TC)a.beta2;
    const TC d0 = (TC)a.d0, d1 = (TC)a.d1, d2 = (TC)a.d2;
    const TX c0ihx = (TX)a.c0ih[0], c0ihz = (TX)a.c0ih[2];
    const TX c1ihx = COEF == EXPI_COEF_SEPARABLE ? (TX)a.c1ih[0] : (TX)0;
    const TX sigmax = (TX)a.sigma;
    // Row ends.  The x neighbour of a point at a row end is 0 under
    // Dirichlet and the point's own value otherwise (no flux), so that one
    // formula serves all points.  The first lane of a row has no left
    // source lane (DPP keeps its edge value); where the row ends inside a
    // wave, the lanes past the end offer the last point's value (or 0).
    const bool lb = ic == 0, rb = ic + 2 >= n0;
    const bool partial = (xq + 1) * 128 > n0;     // the row ends inside this wave
    // x data of the lane, in registers for the whole sweep: table values of
    // its points, face values left of point 0, between the points and right
    // of point 1 (own value where the row ends)
    TX xd[5] = {1, 1, 1, 1, 1};
    if (COEF == EXPI_COEF_SEPARABLE) {
        // four loads issued together (clamped, none behind a branch)
        const TX X0 = (TX)a.tx[ic], X1 = (TX)a.tx[ic + 1];
        const TX Xm = (TX)a.tx[max(ic - 1, 0)], Xq = (TX)a.tx[min(ic + 2, n0 - 1)];
        xd[0] = X0;
        xd[1] = X1;
        xd[2] = lb ? X0 : (TX)0.5 * (Xm + X0);
        xd[3] = (TX)0.5 * (X0 + X1);
        xd[4] = rb ? X1 : (TX)0.5 * (X1 + Xq);
    }
    // (after the loads above are on their way) every ring entry holds a
    // finite value before it is read; the barrier keeps a slow wave's fill
    // from landing on a fast wave's first writes
    for (int t = threadIdx.x; t < 3 * kPairLds; t += blockDim.x) ring[t] = 0;
    for (int t = threadIdx.x; t < 3 * kWRingLds; t += blockDim.x) wring[t] = 0;
    __syncthreads();
    // Dirichlet row ends: the edge lanes take in 0
    const bool ezero = dir && ((lane == 0 && lb) || (lane == 63 && rb));
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;

    // the neighbours of the lane's pair from the adjacent lanes; el, er are
    // the values lanes 0 and 63 take in
    // (in TC for the second product, in TX for the first)
    auto neighbours = [&](const auto (&wc)[2], auto el, auto er, auto& left, auto& right) {
        using T = decltype(el);
        T srcr = wc[0];
        if (partial && !xin) srcr = dir ? (T)0 : wc[1];   // past the row end: the last point
        left = dpp_shift<kDppWaveShr1>(el, wc[1]);
        right = dpp_shift<kDppWaveShl1>(er, srcr);
        if (partial && xin && rb) right = dir ? (T)0 : wc[1];
    };

    const long long units = (long long)a.nrt * n2;
    const long long u_lo = (long long)xcd_tile(a.per_xcd) * a.chunk;
    const long long u_hi = min(u_lo + (long long)a.chunk, units);
    for (long long u = u_lo; u < u_hi;) {
        const int rt = (int)(u / n2), kb = (int)(u % n2);
        const int ke = (int)min((long long)min(n2, kb + kZSeg), kb + (u_hi - u));
        u += ke - kb;
        // this wave's row: step 1 on rows rt*R-1 .. rt*R+R, step 2 on the inner R
        const int y = rt * R - 1 + ry;
        const bool yin = y >= 0 && y < n1;
        const bool outw = yin && ry >= 1 && ry <= R;
        const int yc = min(max(y, 0), n1 - 1);
        const bool eym = y > 0, eyq = y < n1 - 1;
        const int rowb = ic + n0 * yc;
        auto at = [&](int k) { return rowb + plane * min(max(k, 0), n2 - 1); };
        // the first and last wave rows also bring in the row beyond them
        // (y0-2, y0+R+1) into the w_j ring; they compute no w_{j+2}, so they
        // carry it in the registers that hold p in the inner rows
        const int rr = ry + 1;                            // own row in the w_j ring
        const bool hal = ry == 0 || ry == R + 1;
        const int rh = ry == 0 ? 0 : R + 3;               // the extra row
        const int hoff = ry == 0 ? (eym ? -n0 : 0) : (eyq ? n0 : 0);
        // z data of planes kb-2 .. ke+5 (the ones this segment's iterations
        // touch; planes outside the grid get finite values that no nonzero
        // weight uses)
        if (COEF == EXPI_COEF_SEPARABLE) {
            const int zlen = ke - kb + 8;
            for (int t = threadIdx.x; t < zlen; t += blockDim.x) {
                const int q = kb - 2 + t;
                const bool ezm = q > 0, ezq = q < n2 - 1;
                const TX dm = (ezm || dir) ? (TX)1 : (TX)0, dq = (ezq || dir) ? (TX)1 : (TX)0;
                // three loads issued together (clamped, none behind a branch)
                const TX zc = (TX)a.tz[min(max(q, 0), n2 - 1)];
                const TX zm = (TX)a.tz[min(max(q - 1, 0), n2 - 1)];
                const TX zq = (TX)a.tz[min(max(q + 1, 0), n2 - 1)];
                const TX zfm = ezm ? (TX)0.5 * (zm + zc) : zc;
                const TX zfq = ezq ? (TX)0.5 * (zq + zc) : zc;
                ZPlane<TX> z;
                z.zc = zc;
                z.zfm = ezm ? zfm : (TX)0;
                z.zfq = ezq ? zfq : (TX)0;
                z.zd = dm * zfm + dq * zfq;
                ztab[t] = z;
            }
        }
        // y data of the row: the same in every lane, moved to scalar
        // registers for the march
        RowW<TX> rw;
        {
            const TX c0ihy = (TX)a.c0ih[1];
            const TX c1ihy = COEF == EXPI_COEF_SEPARABLE ? (TX)a.c1ih[1] : (TX)0;
            const TX c1ihz = COEF == EXPI_COEF_SEPARABLE ? (TX)a.c1ih[2] : (TX)0;
            const TX em = eym ? (TX)1 : (TX)0, eq = eyq ? (TX)1 : (TX)0;
            const TX dm = (eym || dir) ? (TX)1 : (TX)0, dq = (eyq || dir) ? (TX)1 : (TX)0;
            TX Y = 1, yfm = 1, yfq = 1;
            if (COEF == EXPI_COEF_SEPARABLE) {
                Y = (TX)a.ty[yc];
                const TX Ym = (TX)a.ty[max(yc - 1, 0)], Yq = (TX)a.ty[min(yc + 1, n1 - 1)];
                yfm = eym ? (TX)0.5 * (Ym + Y) : Y;
                yfq = eyq ? (TX)0.5 * (Yq + Y) : Y;
            }
            rw.y = Y;
            rw.gym = em * (c1ihy * yfm);
            rw.gyq = eq * (c1ihy * yfq);
            rw.aym = em * c0ihy;
            rw.ayq = eq * c0ihy;
            rw.ady = c0ihy * (dm + dq);
            rw.gdy = c1ihy * (dm * yfm + dq * yfq);
            rw.hz = c1ihz * Y;
            rw.y = uniform(rw.y);
            rw.gym = uniform(rw.gym);
            rw.gyq = uniform(rw.gyq);
            rw.aym = uniform(rw.aym);
            rw.ayq = uniform(rw.ayq);
            rw.ady = uniform(rw.ady);
            rw.gdy = uniform(rw.gdy);
            rw.hz = uniform(rw.hz);
        }

        // Iteration k, for the planes of this segment (kst = kb - 2):
        //  (1) put w_j of plane k+2 (loaded two iterations ago) into the w_j
        //      ring and start the load of plane k+4;
        //  (2) inner rows: w_{j+2} on plane k-1 from the w_{j+1} ring; the
        //      stores; then the load of p on plane k+1 (the first and last
        //      rows load their extra row of w_j, plane k+4, instead);
        //  (3) w_{j+1} on plane k+1 from the w_j ring, into the w_{j+1} ring;
        //  (4) one barrier.
        // Both rings hold three planes; a wave's own row is read back only by
        // the wave itself, other rows only after the barrier that follows
        // their write.  Registers carry only the loads in flight: w_j of two
        // planes in L (plane q in L[q & 1]) and p (or the extra row) of two
        // planes in P.  Every wave issues the same global loads and stores
        // on every path (clamped addresses, range-checked stores), so the
        // in-order memory counter waits only for the load that is needed.
        const int kst = kb - 2;
        TX L[2][2], P[2][2];
        TX Wm[2], Wc[2], Wq[2];   // the wave's own row of w_j: planes k, k+1, k+2
        // FP32 (registers to spare): the own row of w_{j+1} too, planes
        // k, k-1, k-2 (values from the rings' zero fill before the first)
        // (not with the FP64 first half of a mixed start: registers)
        constexpr bool kOwnW1 = sizeof(TW) == 4 && std::is_same<TX, TC>::value;
        TC Q0[2] = {0, 0}, Q1[2] = {0, 0}, Q2[2] = {0, 0};
        // FP32: the point weights of plane k+1 (step 3) wait two iterations
        // for step 2 on the same plane; slot (plane - kst) mod 2
        constexpr bool kKeepW = sizeof(TW) == 4 && std::is_same<TX, TC>::value;
        PointW<TC> PWq[2];
        L[0][0] = L[0][1] = L[1][0] = L[1][1] = 0;
        P[0][0] = P[0][1] = P[1][0] = P[1][1] = 0;
        // ring slot of a plane: (plane - kst) mod 3.  The march is unrolled
        // six planes per block (a multiple of both the three-plane rings and
        // the two-slot load queues, so every rotation is a renaming): within
        // a block the plane is k0 + c for a constant c, and k0 - kst is a
        // multiple of 6, so the slot is the constant c mod 3.
        auto slot_of = [&](int c) { return c % 3; };   // c >= 0
        auto wslot_c = [&](int c) { return &wring[slot_of(c) * kWRingLds]; };
        auto vslot_c = [&](int c) { return &ring[slot_of(c) * kPairLds]; };
        // (rings of TC or TX values)
        auto put = [&](auto* base, int row, const auto (&v)[2]) {
            using T = typename std::remove_pointer<decltype(base)>::type;
            typedef T T2 __attribute__((ext_vector_type(2)));
            T2 t;
            t.x = v[0];
            t.y = v[1];
            *reinterpret_cast<T2*>(base + row * RW + i) = t;
        };
        auto get = [&](const auto* base, int row, auto (&v)[2]) {
            using T = typename std::remove_const<typename std::remove_pointer<decltype(base)>::type>::type;
            typedef T T2 __attribute__((ext_vector_type(2)));
            const T2 t = *reinterpret_cast<const T2*>(base + row * RW + i);
            v[0] = t.x;
            v[1] = t.y;
        };
        {
            // planes kst and kst+1 of w_j into the ring; kst+2 and kst+3 in flight
            // (rows outside the grid load a clamped row: finite values that
            // no nonzero weight uses; the inner rows load their own row a
            // second time where the outer rows load their extra row)
            TX h0[2], h1[2], e0[2], e1[2];
            ld2(x, at(kst), h0);
            ld2(x, at(kst + 1), h1);
            ld2(x, at(kst + 2), L[0]);
            ld2(x, at(kst + 3), L[1]);
            ld2(x, at(kst) + hoff, e0);
            ld2(x, at(kst + 1) + hoff, e1);
            ld2(x, at(kst + 2) + hoff, P[1]);   // put at iteration kst from P[1]
            ld2(x, at(kst + 3) + hoff, P[0]);
            put(wslot_c(0), rr, h0);
            put(wslot_c(1), rr, h1);
            Wm[0] = h0[0];
            Wm[1] = h0[1];
            Wc[0] = h1[0];
            Wc[1] = h1[1];
            if (hal) {
                put(wslot_c(0), rh, e0);
                put(wslot_c(1), rh, e1);
            }
        }
        if (a.guard && __builtin_amdgcn_readfirstlane(done_v) != 0)
            return;   // the same in every thread; nothing stored yet
        __syncthreads();   // x and row data, the first two ring planes
        // a point of the outer layer has a zero row under interior_only
        const bool yedge = !(eym && eyq);
        // one block of six planes from k0 (k0 - kst a multiple of 6); in
        // FP32, whole blocks while six planes remain, then the last, shorter
        // one
        auto block = [&](const int k0, auto full) {
            constexpr bool kFull = decltype(full)::value;
            // FP32: the lane's squares of a block of six planes are summed in
            // FP32 and added to the FP64 sums once per block (at most twelve
            // terms per FP32 sum); FP64 adds each square
            float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const int k = k0 + s;
                // the last output plane ke-1 is done at k = ke; the rest of
                // the last block has nothing to do (only the last block of a
                // segment tests this: a test in every block would make the
                // compiler copy the queues at each possible exit)
                if constexpr (!kFull) {
                    if (k > ke) break;
                }
                // (1) w_j of plane k+2 into the ring (and the wave's own
                // registers), then load plane k+4
                {
                    TX* wb = wslot_c(s + 2);
                    Wq[0] = L[s & 1][0];
                    Wq[1] = L[s & 1][1];
                    put(wb, rr, L[s & 1]);
                    if (hal) put(wb, rh, P[(s + 1) & 1]);   // loaded two iterations ago
                    // (planes past ke+1 feed no needed value: the last
                    // needed one is loaded again, a cache hit)
                    ld2(x, at(min(k + 4, ke + 1)), L[s & 1]);
                }
                // (2) w_{j+2} on plane k-1 (inner rows)
                const int kp = k - 1;
                const bool outp = outw && kp >= kb && kp < ke;
                TC wo[2] = {0, 0}, po[2] = {0, 0};
                {
                    if (outp) {
                        const TC* vb = vslot_c(s + 2);        // plane k-1
                        TC wc[2], ym[2], yq[2], zm[2], zq[2];
                        if constexpr (kOwnW1) {               // own row from registers
#pragma unroll
                            for (int v = 0; v < 2; ++v) {
                                wc[v] = Q1[v];
                                zm[v] = Q2[v];
                                zq[v] = Q0[v];
                            }
                        } else {
                            get(vb, ry, wc);
                            get(vslot_c(s + 1), ry, zm);      // plane k-2
                            get(vslot_c(s), ry, zq);          // plane k
                        }
                        get(vb, ry - 1, ym);
                        get(vb, ry + 1, yq);
                        const TC el = vb[ry * RW + (ic > 0 ? ic - 1 : ic)];
                        const TC er = vb[ry * RW + (ic + 2 < n0 ? ic + 2 : ic + 1)];
                        TC left, right;
                        neighbours(wc, ezero ? (TC)0 : el, ezero ? (TC)0 : er, left, right);
                        TC aw[2];
                        if constexpr (kKeepW) {
                            aw_pair_w<TC>(wc, left, right, ym, yq, zm, zq, PWq[(s + 1) & 1], aw);
                        } else {
                            // (formed in TX, the type of the row and z data)
                            const PointW<TC> pw = point_weights_as<TC>(point_weights<COEF, TX>(
                                plane_weights<COEF, TX>(rw, ztab, kb - 2, kp, n2, dir, c0ihz, c1ihx), c0ihx, xd));
                            aw_pair_w<TC>(wc, left, right, ym, yq, zm, zq, pw, aw);
                        }
                        if (ionly) {
                            const bool edge = yedge || kp == 0 || kp == n2 - 1;
                            if (edge || lb) aw[0] = 0;
                            if (edge || rb) aw[1] = 0;
                        }
                        const TX* pp = P[(s + 1) & 1];        // p (FIRST: r) of plane k-1
                        constexpr bool kPairSq = sizeof(TW) == 4;
                        TC q0 = 0, q1 = 0, q2 = 0, q3 = 0;
#pragma unroll
                        for (int v = 0; v < 2; ++v) {
                            const TC p1 = FIRST ? (TC)(TW)(d0 * pp[v] + d1 * wc[v])
                                                : (TC)(TW)(pp[v] + d1 * wc[v]);
                            const TC w2 = (TC)(TW)(alpha * aw[v] + beta2 * wc[v]);
                            const TC p2 = START ? (TC)(TW)(d1 * wc[v] + d2 * w2)
                                                : (TC)(TW)(p1 + d2 * w2);
                            wo[v] = w2;
                            po[v] = p2;
                            // FIRST: ||r||^2 in place of ||p_1||^2
                            const TC n1 = FIRST ? (TC)pp[v] : p1;
                            if constexpr (kPairSq) {
                                q0 += wc[v] * wc[v];
                                if (!START) q1 += n1 * n1;
                                q2 += w2 * w2;
                                q3 += p2 * p2;
                            } else if (xin) {
                                s0 += (double)wc[v] * (double)wc[v];
                                if (!START) s1 += (double)n1 * (double)n1;
                                s2 += (double)w2 * (double)w2;
                                s3 += (double)p2 * (double)p2;
                            }
                        }
                        if (kPairSq) {
                            b0 += (float)q0;
                            if (!START) b1 += (float)q1;
                            b2 += (float)q2;
                            b3 += (float)q3;
                        }
                    }
                    // the stores, on every path (dropped where there is no
                    // output point); streaming: measured faster in FP64,
                    // slower in FP32
                    const int sidx = (outp && xin) ? at(kp) : -1;
                    st2_buf<TW>(out_r, sidx, wo, sizeof(TW) == 8);
                    st2_buf<TW>(pv_r, sidx, po, sizeof(TW) == 8);
                    // into the slot just read: p (FIRST: r) of plane k+1,
                    // used two iterations on; the outer rows load their
                    // extra row of w_j, plane k+4
                    const TX* psrc;
                    if constexpr (START) psrc = x;
                    else psrc = (FIRST || hal) ? x : static_cast<const TW*>(pv);
                    // (p outside the output planes: a neighbouring output
                    // plane's p instead, a cache hit)
                    ld2(psrc, hal ? at(min(k + 4, ke + 1)) + hoff : at(min(max(k + 1, kb), ke - 1)),
                        P[(s + 1) & 1]);
                }
                // (3) w_{j+1} on plane k+1 (values of planes or rows outside the
                // grid are never used with a nonzero weight)
                {
                    const int q = k + 1;
                    const TX* wb = wslot_c(s + 1);
                    // own row from registers: planes k, k+1, k+2
                    const TX wc[2] = {Wc[0], Wc[1]}, zm[2] = {Wm[0], Wm[1]}, zq[2] = {Wq[0], Wq[1]};
                    TX ym[2], yq[2];
                    get(wb, rr - 1, ym);
                    get(wb, rr + 1, yq);
                    const TX el = wb[rr * RW + (ic > 0 ? ic - 1 : ic)];
                    const TX er = wb[rr * RW + (ic + 2 < n0 ? ic + 2 : ic + 1)];
                    TX left, right;
                    neighbours(wc, ezero ? (TX)0 : el, ezero ? (TX)0 : er, left, right);
                    const PlaneW<TX> pw = plane_weights<COEF, TX>(rw, ztab, kb - 2, q, n2, dir, c0ihz, c1ihx);
                    const PointW<TX> qw = point_weights<COEF, TX>(pw, c0ihx, xd);
                    // plane k+1, read at k+2 (in TC)
                    if constexpr (kKeepW) PWq[(s + 1) & 1] = point_weights_as<TC>(qw);
                    TX aw[2];
                    aw_pair_w<TX>(wc, left, right, ym, yq, zm, zq, qw, aw);
                    if (ionly) {
                        const bool edge = yedge || q == 0 || q == n2 - 1;
                        if (edge || lb) aw[0] = 0;
                        if (edge || rb) aw[1] = 0;
                    }
                    TC r[2];
#pragma unroll
                    for (int v = 0; v < 2; ++v)
                        r[v] = START ? (TC)(TW)(sigmax * aw[v] + (wc[v] - wc[v] * wc[v] * wc[v]))
                                     : (TC)(TW)(alpha * aw[v] + beta1 * wc[v]);
                    put(vslot_c(s + 1), ry, r);
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        Wm[v] = Wc[v];
                        Wc[v] = Wq[v];
                        if constexpr (kOwnW1) {
                            Q2[v] = Q1[v];
                            Q1[v] = Q0[v];
                            Q0[v] = r[v];
                        }
                    }
                }
                __syncthreads();
            }
            if (sizeof(TW) == 4 && xin) {
                s0 += (double)b0;
                if (!START) s1 += (double)b1;
                s2 += (double)b2;
                s3 += (double)b3;
            }
        };
        int k0 = kst;
        if constexpr (sizeof(TW) == 4) {
            for (; k0 + 5 <= ke; k0 += 6) block(k0, std::true_type{});
        }
        // (FP64 keeps the test in every block: whole blocks there need more
        // scalar registers than it has, and the spills cost more than the
        // copies they save)
        for (; k0 <= ke; k0 += 6) block(k0, std::false_type{});

    }
    if (a.guard && __builtin_amdgcn_readfirstlane(done_v) != 0) return;   // a workgroup without a unit
    if (FIRST) {
        // ||p_1|| is not formed: a non-finite p_1 makes p_2 non-finite,
        // which the test at m = 2 reports; the slot holds 0
        const double v[5] = {s1, s0, 0.0, s2, s3};
        finish_sweep_n<5>(a.partials, 8, v);
    } else {
        const double v[4] = {s0, s1, s2, s3};
        finish_sweep_n<4>(a.partials, 4, v);
    }
}

template <int COEF, class TW, int MODE>
void go_bc(const PairGeom& g, int bc, const PairArgs& a, hipStream_t s) {
    const dim3 grid(g.grid), block(kPairWaves * 64);
    switch (bc) {
        case EXPI_DIRICHLET0:
            hipLaunchKernelGGL((pair_sweep<COEF, EXPI_DIRICHLET0, TW, MODE>), grid, block, 0, s, a);
            break;
        case EXPI_NEUMANN0:
            hipLaunchKernelGGL((pair_sweep<COEF, EXPI_NEUMANN0, TW, MODE>), grid, block, 0, s, a);
            break;
        default:
            hipLaunchKernelGGL((pair_sweep<COEF, EXPI_INTERIOR_ONLY, TW, MODE>), grid, block, 0, s, a);
            break;
    }
}

template <class TW, int MODE>
hipError_t go(const PairGeom& g, int coef, int bc, const PairArgs& a, hipStream_t s) {
    if (coef == EXPI_COEF_SEPARABLE) go_bc<EXPI_COEF_SEPARABLE, TW, MODE>(g, bc, a, s);
    else go_bc<EXPI_COEF_CONST, TW, MODE>(g, bc, a, s);
    return hipGetLastError();
}

}  // namespace

// Pair sweeps need a 3D stencil with a constant or separable coefficient,
// rows of at most 512 points (even, for the two-point vector accesses),
// fewer than 2^28 points, and 16-byte aligned vectors.
bool pair_supported(const Op& op, int tw) {
    (void)tw;
    // the stores address a vector with 32-bit byte offsets: below 2^31
    // bytes in FP64 (2^28 points)
    return op.kind == 0 && op.dim == 3 && op.n[0] % 2 == 0 && op.n[0] <= 512 &&
           (op.coef == EXPI_COEF_CONST || op.coef == EXPI_COEF_SEPARABLE) &&
           op.size * 8 < ((int64_t)1 << 31) - 64;
}

// The start vector fused into the first pair sweep (PAIR_START): u is read
// and r formed in FP64 with either storage type.
bool pair_start_supported(const Op& op) { return pair_supported(op, 0); }

PairGeom pair_geom(const Op& op, int cus) {
    PairGeom g{};
    // waves per row: 1, 2 or 4 (a divisor of the 16 waves; with 4, waves past
    // a shorter row's end are masked)
    g.nxw = op.n[0] <= 128 ? 1 : (op.n[0] <= 256 ? 2 : 4);
    g.rows = kPairWaves / g.nxw - 2;
    g.nrt = (op.n[1] + g.rows - 1) / g.rows;
    const long long units = (long long)g.nrt * op.n[2];
    // one workgroup per CU, a multiple of the XCD count, every one busy
    long long grid = std::min<long long>(cus > 0 ? cus : 256, units);
    grid = std::max<long long>(kXcd, (grid / kXcd) * kXcd);
    g.chunk = (int)((units + grid - 1) / grid);
    g.grid = (int)grid;
    g.per_xcd = g.grid / kXcd;
    return g;
}

// Compute units of the current device (cached per host thread and device).
int device_cus() {
    static thread_local int dev_cached = -1, cus_cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != dev_cached) {
        if (hipDeviceGetAttribute(&cus_cached, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus_cached = 0;
        dev_cached = dev;
    }
    return cus_cached;
}

hipError_t launch_pair(const Op& op, int tw, PairArgs a, hipStream_t s, hipEvent_t after_sweep,
                       bool finalize, int mode) {
    if (mode == PAIR_START && !pair_start_supported(op)) return hipErrorInvalidValue;
    const PairGeom g = pair_geom(op, device_cus());
    for (int d = 0; d < 3; ++d) {
        a.n[d] = op.n[d];
        a.ih2[d] = 1.0 / (op.h[d] * op.h[d]);
    }
    a.bc = op.bc;
    for (int d = 0; d < 3; ++d) {
        a.c0ih[d] = op.c0 * a.ih2[d];
        a.c1ih[d] = op.c1 * a.ih2[d];
    }
    a.tx = op.tx;
    a.ty = op.ty;
    a.tz = op.tz;
    a.nxw = g.nxw;
    a.rows = g.rows;
    a.nrt = g.nrt;
    a.chunk = g.chunk;
    a.per_xcd = g.per_xcd;
    hipError_t e;
    if (mode == PAIR_START)
        e = tw == 1 ? go<float, PAIR_START>(g, op.coef, op.bc, a, s) : go<double, PAIR_START>(g, op.coef, op.bc, a, s);
    else if (mode == PAIR_FIRST)
        e = tw == 1 ? go<float, PAIR_FIRST>(g, op.coef, op.bc, a, s) : go<double, PAIR_FIRST>(g, op.coef, op.bc, a, s);
    else
        e = tw == 1 ? go<float, PAIR_NEWTON>(g, op.coef, op.bc, a, s)
                    : go<double, PAIR_NEWTON>(g, op.coef, op.bc, a, s);
    if (e != hipSuccess) return e;
    if (after_sweep) {
        e = hipEventRecord(after_sweep, s);
        if (e != hipSuccess) return e;
    }
    if (!finalize) return hipSuccess;
    return launch_pair_finalize(a.partials, a.st, g.grid, a.j, a.guard, a.d0, a.d1, a.d2, a.tol, mode, a.outbuf, s);
}

}  // namespace expi
