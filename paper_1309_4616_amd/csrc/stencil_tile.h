// One tile of the stencil sweep, shared by the per-operator sweep kernel
// (stencil.hip) and the persistent batched kernel (batch.hip).  The layout
// and traversal are described in stencil.hip.
#pragma once

#include "nonlin.h"
#include "sweep_common.h"

namespace expi {
// EPI_START with g = x - x^3 as a stencil kernel of its own (no g operand,
// so no load inside the march); chosen by the stencil launcher for
// G_CUBIC_SELF
constexpr int EPI_START_SELF = 5;
// EPI_APPLY / EPI_START that also add the boundary term of the operator's
// Dirichlet data, f evaluated at the boundary-adjacent points (own
// instantiations, so the plain sweeps carry none of its code)
constexpr int EPI_APPLY_BD = 6;
constexpr int EPI_START_BD = 7;

namespace tile {

// Dirichlet data f at a boundary node (Sec. III-A): kind 1 z(1-z)xy,
// kind 2 sin(pi z) exp(-xy).
template <class TC>
__device__ __forceinline__ TC boundary_value(int kind, TC x, TC y, TC z) {
    if (kind == EXPI_BDATA_Z1MZ_XY) return z * ((TC)1 - z) * x * y;
    if constexpr (std::is_same<TC, float>::value)
        return sinf(3.14159265358979323846f * z) * expf(-x * y);
    else
        return sin(3.14159265358979323846 * z) * exp(-x * y);
}

// D(x, y) = 1/sqrt(1 + x^2 + y^2) of Sec. III-B
template <class TC>
__device__ __forceinline__ TC d_coefficient(TC x, TC y) {
    return (TC)1 / sqrt((TC)1 + x * x + y * y);
}

template <int V, class T, class TC>
__device__ __forceinline__ void vld(const T* __restrict__ p, int idx, TC (&o)[V]) {
    if constexpr (V == 2) {
        typedef T T2 __attribute__((ext_vector_type(2)));
        const T2 t = *reinterpret_cast<const T2*>(p + idx);
        o[0] = (TC)t.x;
        o[1] = (TC)t.y;
    } else {
        o[0] = (TC)p[idx];
    }
}

template <int V, class T, class TC>
__device__ __forceinline__ void vst(T* __restrict__ p, int idx, const TC (&v)[V]) {
    if constexpr (V == 2) {
        typedef T T2 __attribute__((ext_vector_type(2)));
        T2 t;
        t.x = (T)v[0];
        t.y = (T)v[1];
        *reinterpret_cast<T2*>(p + idx) = t;
    } else {
        p[idx] = (T)v[0];
    }
}

// Lane `t` of a value held one per lane (t the same in all lanes).
__device__ __forceinline__ float lane_value(float v, int t) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), t));
}
__device__ __forceinline__ double lane_value(double v, int t) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), t);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int V, class TC>
__device__ __forceinline__ void vzero(TC (&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = (TC)0;
}

// Coefficients of a point and its six neighbours.
template <class TC>
struct Coefs {
    TC c, xm, xq, ym, yq, zm, zq;
};

// One marched plane of one thread: registers that the pipeline fills one
// stage ahead (cache-served neighbour values) or two stages ahead (HBM).
template <class TC, int V>
struct Side {
    TC ym[V], yq[V];   // y neighbours (3D)
    TC xl, xr;         // x neighbours beyond the wave's ends (edge lanes)
};

// The work of one tile (t0, t1, t2) of operator `a`, accumulating the
// reduction values of its points into s0..s2.  The tile has nw waves, of
// which the calling wave is wv (a workgroup's waves by default; the batched
// solver passes single-wave tiles); every lane of the wave calls it (the x
// neighbours are exchanged by cross-lane shuffles).  No workgroup barrier.
template <int DIM, int COEF, int EPI, class TIN, class TOUT, int V>
__device__ __forceinline__ void stencil_tile_w(const SweepArgs& a, int t0, int t1, int t2, int wv, int nw,
                                               double& s0, double& s1, double& s2) {
    using TC = compute_t<TIN, TOUT>;
    constexpr bool kApply = (EPI == EPI_APPLY || EPI == EPI_APPLY_BD);
    constexpr bool kStart = (EPI == EPI_START || EPI == EPI_START_BD);
    constexpr bool kBD = (EPI == EPI_APPLY_BD || EPI == EPI_START_BD) && DIM == 3;
    constexpr bool kDlap = (COEF == EXPI_COEF_DLAP);
    const TIN* __restrict__ x = static_cast<const TIN*>(a.x);
    TOUT* __restrict__ out = static_cast<TOUT*>(a.out);
    TOUT* __restrict__ p = static_cast<TOUT*>(a.p);
    const double* __restrict__ fld = a.field;
    constexpr bool kW = (EPI != EPI_GERSH);          // reads the vector
    constexpr bool kP = (EPI == EPI_NEWTON);         // reads p
    constexpr bool kF = (COEF == EXPI_COEF_FIELD);   // reads the coefficient field
    const int lane = threadIdx.x & 63;
    {
        const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
        const int ns = (DIM == 3) ? n2 : n1;          // marched axis
        const int ss = (DIM == 3) ? n0 * n1 : n0;     // its stride
        const int i = t0 * (64 * V) + lane * V;
        int j, kb;
        if (DIM == 3) {
            j = t1 * nw + wv;
            kb = t2 * a.march;
        } else {
            j = 0;
            kb = t1 * (nw * a.march) + wv * a.march;
        }
        const int ke = min(kb + a.march, ns);
        // whole waves outside the grid skip the march; lanes past the row end
        // stay in it (masked) so that the x-neighbour shuffles see every lane
        const bool wave_live = (DIM == 2 || j < n1) && kb < ke;
        const bool active = wave_live && i < n0;
        if (wave_live) {
            const bool dir = (a.bc == EXPI_DIRICHLET0);
            const bool ionly = (a.bc == EXPI_INTERIOR_ONLY);
            const TC ihx = (TC)a.ih2[0];
            const TC ihy = (TC)a.ih2[1];
            const TC ihz = (TC)a.ih2[DIM == 3 ? 2 : 1];
            const TC alpha = (TC)a.alpha, beta = (TC)a.beta;
            const TC d0 = (TC)a.d0, d1 = (TC)a.d1, sigma = (TC)a.sigma;
            const TC c0 = (TC)a.c0, c1 = (TC)a.c1;
            const bool eym = (DIM == 3) && j > 0, eyq = (DIM == 3) && j < n1 - 1;
            // Every load below is unconditional, from an index clamped into
            // the grid; values of neighbours that do not exist are masked by
            // the existence flags.  Straight-line loads let the compiler track
            // each one's completion precisely.  Lanes past the row end
            // (i >= n0) load from the last column and store nothing.
            const int ic = active ? i : (n0 - V);
            const int jc = (DIM == 3) ? min(j, n1 - 1) : 0;
            const int rowb = ic + ((DIM == 3) ? n0 * jc : 0);       // (i, j) at plane 0
            const int yoffm = (DIM == 3 && eym) ? -n0 : 0;          // y neighbour offsets
            const int yoffq = (DIM == 3 && eyq) ? n0 : 0;
            // one extra load per plane feeds the wave-edge lanes: lane 0 its
            // left neighbour, lane 63 its right one, the rest reload a point
            int eoff = 0;
            if (lane == 0 && ic > 0) eoff = -1;
            if (lane == 63 && ic + V < n0) eoff = V;
            auto at = [&](int k) { return rowb + ss * min(max(k, 0), ns - 1); };

            // separable coefficient: x values of the thread's points and of
            // their outer neighbours, y values of the row; the values of the
            // marched axis for planes kb-1 .. kb+126 sit one per lane in zr0,
            // zr1 and are read with readlane (a vector load inside the march
            // would make the in-order memory counter wait for the prefetches
            // issued before it)
            TC Xv[V], Xl = 0, Xr = 0, Ym = 0, Yc = 0, Yq = 0, zr0 = 0, zr1 = 0;
            vzero<V>(Xv);
            const double* Ts = (DIM == 3) ? a.tz : a.ty;
            if (COEF == EXPI_COEF_SEPARABLE) {
#pragma unroll
                for (int v = 0; v < V; ++v) Xv[v] = (TC)a.tx[ic + v];
                Xl = (TC)a.tx[max(ic - 1, 0)];
                Xr = (TC)a.tx[min(ic + V, n0 - 1)];
                if (DIM == 3) {
                    Yc = (TC)a.ty[jc];
                    Ym = (TC)a.ty[max(jc - 1, 0)];
                    Yq = (TC)a.ty[min(jc + 1, n1 - 1)];
                }
                zr0 = (TC)Ts[min(max(kb - 1 + lane, 0), ns - 1)];
                zr1 = (TC)Ts[min(max(kb + 63 + lane, 0), ns - 1)];
            }
            // grid positions (D-Laplacian and boundary data): index i at
            // (i + off) h, off = 1 (Dirichlet nodes), 1/2 (cells), 0
            const double poff = dir ? 1.0 : (a.bc == EXPI_NEUMANN0 ? 0.5 : 0.0);
            TC Dv[V];   // 3D: D of the thread's points, constant along the march
#pragma unroll
            for (int v = 0; v < V; ++v) Dv[v] = (TC)1;
            if (kDlap && DIM == 3) {
                const TC yq = (TC)((jc + poff) * a.hpos[1]);
#pragma unroll
                for (int v = 0; v < V; ++v)
                    Dv[v] = d_coefficient<TC>((TC)((ic + v + poff) * a.hpos[0]), yq);
            }
            auto zv = [&](int k) -> TC {   // k in [kb-1, kb+126], clamped into the grid
                const int t = min(k, ns - 1) - (kb - 1);
                return t < 64 ? lane_value(zr0, t) : lane_value(zr1, t - 64);
            };
            // register queues: stage s (plane k = k0 + s) finds w at k-1, k,
            // k+1 in W[s&3], W[(s+1)&3], W[(s+2)&3] and loads k+2 into
            // W[(s+3)&3]; p and the side values alternate between two slots
            TC W[4][V], F[4][V], P[2][V];
            Side<TC, V> S[2], SF[2];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                vzero<V>(W[q]);
                vzero<V>(F[q]);
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                vzero<V>(P[q]);
                vzero<V>(S[q].ym);
                vzero<V>(S[q].yq);
                vzero<V>(SF[q].ym);
                vzero<V>(SF[q].yq);
                S[q].xl = S[q].xr = SF[q].xl = SF[q].xr = 0;
            }
            auto load_side = [&](int k, Side<TC, V>& sd, const auto* src) {
                const int b = at(k);
                if (DIM == 3) {
                    vld<V>(src, b + yoffm, sd.ym);
                    vld<V>(src, b + yoffq, sd.yq);
                }
                const TC e = (TC)src[b + eoff];
                sd.xl = e;
                sd.xr = e;
            };
            if (kW) {
                vld<V>(x, at(kb - 1), W[0]);
                vld<V>(x, at(kb), W[1]);
                vld<V>(x, at(kb + 1), W[2]);
                load_side(kb, S[0], x);
            }
            if (kP) vld<V>(p, at(kb), P[0]);
            if (kF) {
                vld<V>(fld, at(kb - 1), F[0]);
                vld<V>(fld, at(kb), F[1]);
                vld<V>(fld, at(kb + 1), F[2]);
                load_side(kb, SF[0], fld);
            }
            int idx = at(kb);

            for (int k0 = kb; k0 < ke; k0 += 4) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = k0 + s;
                    const bool kvalid = k < ke;   // all four stages run; only kvalid ones store
                    {
                        const int cur = s & 1, nxt = cur ^ 1;
                        // (1) cache-served values of the next plane
                        if (kW) load_side(k + 1, S[nxt], x);
                        if (kF) load_side(k + 1, SF[nxt], fld);
                        // (2) HBM prefetch: w two planes ahead, p one plane ahead
                        if (kW) vld<V>(x, at(k + 2), W[(s + 3) & 3]);
                        if (kP) vld<V>(p, at(k + 1), P[nxt]);
                        if (kF) vld<V>(fld, at(k + 2), F[(s + 3) & 3]);
                        const TC* wm = W[s & 3];
                        const TC* wc = W[(s + 1) & 3];
                        const TC* wq = W[(s + 2) & 3];
                        const TC* Fm = F[s & 3];
                        const TC* Fc = F[(s + 1) & 3];
                        const TC* Fq = F[(s + 2) & 3];
                        TC Zm = 0, Zc = 0, Zq = 0;
                        if (COEF == EXPI_COEF_SEPARABLE) {
                            Zm = zv(max(k - 1, 0));
                            Zc = zv(k);
                            Zq = zv(k + 1);
                        }
                        const bool ezm = k > 0, ezq = k < ns - 1;
                        // (3) x neighbours of the outer points from adjacent lanes
                        TC left = 0, right = 0, Fleft = 0, Fright = 0;
                        if (kW) {
                            left = __shfl_up(wc[V - 1], 1, 64);
                            right = __shfl_down(wc[0], 1, 64);
                            if (lane == 0) left = S[cur].xl;
                            if (lane == 63) right = S[cur].xr;
                        }
                        if (kF) {
                            Fleft = __shfl_up(Fc[V - 1], 1, 64);
                            Fright = __shfl_down(Fc[0], 1, 64);
                            if (lane == 0) Fleft = SF[cur].xl;
                            if (lane == 63) Fright = SF[cur].xr;
                        }
                        // (4) the points of this plane
                        if (active && kvalid) {
                            TC wo[V], po[V];
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const int iv = i + v;
                                const bool exm = iv > 0, exq = iv < n0 - 1;
                                Coefs<TC> cf;
                                if (COEF == EXPI_COEF_CONST || kDlap) {
                                    cf.c = cf.xm = cf.xq = cf.ym = cf.yq = cf.zm = cf.zq = c0;
                                } else if (COEF == EXPI_COEF_SEPARABLE) {
                                    const TC X_l = (v > 0) ? Xv[v - 1] : Xl;
                                    const TC X_r = (v < V - 1) ? Xv[v + 1] : Xr;
                                    if (DIM == 3) {
                                        const TC zy = Zc * Yc;
                                        cf.c = c0 + c1 * (zy * Xv[v]);
                                        cf.xm = c0 + c1 * (zy * X_l);
                                        cf.xq = c0 + c1 * (zy * X_r);
                                        cf.ym = c0 + c1 * ((Zc * Ym) * Xv[v]);
                                        cf.yq = c0 + c1 * ((Zc * Yq) * Xv[v]);
                                        cf.zm = c0 + c1 * ((Zm * Yc) * Xv[v]);
                                        cf.zq = c0 + c1 * ((Zq * Yc) * Xv[v]);
                                    } else {
                                        cf.c = c0 + c1 * (Zc * Xv[v]);
                                        cf.xm = c0 + c1 * (Zc * X_l);
                                        cf.xq = c0 + c1 * (Zc * X_r);
                                        cf.ym = cf.yq = (TC)0;
                                        cf.zm = c0 + c1 * (Zm * Xv[v]);
                                        cf.zq = c0 + c1 * (Zq * Xv[v]);
                                    }
                                } else {
                                    cf.c = Fc[v];
                                    cf.xm = (v > 0) ? Fc[v - 1] : Fleft;
                                    cf.xq = (v < V - 1) ? Fc[v + 1] : Fright;
                                    cf.ym = SF[cur].ym[v];
                                    cf.yq = SF[cur].yq[v];
                                    cf.zm = Fm[v];
                                    cf.zq = Fq[v];
                                }
                                const bool inner = exm && exq && ezm && ezq && (DIM == 2 || (eym && eyq));
                                const bool zero_row = ionly && !inner;
                                const TC fxm = face_weight<TC>(exm, dir, cf.c, cf.xm) * ihx;
                                const TC fxq = face_weight<TC>(exq, dir, cf.c, cf.xq) * ihx;
                                const TC fzm = face_weight<TC>(ezm, dir, cf.c, cf.zm) * ihz;
                                const TC fzq = face_weight<TC>(ezq, dir, cf.c, cf.zq) * ihz;
                                TC fym = 0, fyq = 0;
                                if (DIM == 3) {
                                    fym = face_weight<TC>(eym, dir, cf.c, cf.ym) * ihy;
                                    fyq = face_weight<TC>(eyq, dir, cf.c, cf.yq) * ihy;
                                }
                                // D of the D-Laplacian at this point (2D: varies along the march)
                                TC Dp = Dv[v];
                                if (kDlap && DIM == 2)
                                    Dp = d_coefficient<TC>((TC)((iv + poff) * a.hpos[0]),
                                                           (TC)((k + poff) * a.hpos[1]));
                                if (EPI == EPI_GERSH) {
                                    // diagonal = -(sum of the face weights); off-diagonal
                                    // magnitude = weights of faces that have a neighbour
                                    TC diag = -(fxm + fxq + fym + fyq + fzm + fzq);
                                    TC off = (exm ? fxm : (TC)0) + (exq ? fxq : (TC)0) +
                                             (eym ? fym : (TC)0) + (eyq ? fyq : (TC)0) +
                                             (ezm ? fzm : (TC)0) + (ezq ? fzq : (TC)0);
                                    if (kDlap) {
                                        diag *= Dp;
                                        off *= Dp;
                                    }
                                    if (zero_row) diag = off = 0;
                                    s0 = fmin(s0, (double)(diag - off));
                                    s1 = fmax(s1, (double)(diag + off));
                                } else {
                                    // sum over faces of weight * (w_nb - w_c); a missing
                                    // neighbour reads 0 (Dirichlet) or has weight 0
                                    const TC w_c = wc[v];
                                    const TC wl = exm ? ((v > 0) ? wc[v - 1] : left) : (TC)0;
                                    const TC wr = exq ? ((v < V - 1) ? wc[v + 1] : right) : (TC)0;
                                    const TC wzm = ezm ? wm[v] : (TC)0;
                                    const TC wzq = ezq ? wq[v] : (TC)0;
                                    TC Aw = fxm * (wl - w_c) + fxq * (wr - w_c) + fzm * (wzm - w_c) +
                                            fzq * (wzq - w_c);
                                    if (DIM == 3) {
                                        const TC wy0 = eym ? S[cur].ym[v] : (TC)0;
                                        const TC wy1 = eyq ? S[cur].yq[v] : (TC)0;
                                        Aw += fym * (wy0 - w_c) + fyq * (wy1 - w_c);
                                    }
                                    if constexpr (kBD) {
                                        // a missing neighbour of a boundary-adjacent point
                                        // is the boundary node, where the data are f
                                        if (dir && !(exm && exq && eym && eyq && ezm && ezq)) {
                                            const TC xp = (TC)((iv + 1) * a.hpos[0]);
                                            const TC yp = (TC)((j + 1) * a.hpos[1]);
                                            const TC zp = (TC)((k + 1) * a.hpos[2]);
                                            const int bk = a.bdata;
                                            TC bt = 0;
                                            if (!exm) bt += fxm * boundary_value<TC>(bk, (TC)0, yp, zp);
                                            if (!exq)
                                                bt += fxq * boundary_value<TC>(
                                                                bk, (TC)((n0 + 1) * a.hpos[0]), yp, zp);
                                            if (!eym) bt += fym * boundary_value<TC>(bk, xp, (TC)0, zp);
                                            if (!eyq)
                                                bt += fyq * boundary_value<TC>(
                                                                bk, xp, (TC)((n1 + 1) * a.hpos[1]), zp);
                                            if (!ezm) bt += fzm * boundary_value<TC>(bk, xp, yp, (TC)0);
                                            if (!ezq)
                                                bt += fzq * boundary_value<TC>(
                                                                bk, xp, yp, (TC)((ns + 1) * a.hpos[2]));
                                            Aw += bt;
                                        }
                                    }
                                    if (kDlap) Aw *= Dp;
                                    if (zero_row) Aw = 0;
                                    if (kApply) {
                                        wo[v] = alpha * Aw + beta * w_c;
                                    } else if (EPI == EPI_NEWTON) {
                                        const TC wn_ = (TC)(TOUT)(alpha * Aw + beta * w_c);
                                        const TC pn_ = (TC)(TOUT)(P[cur][v] + d1 * wn_);
                                        wo[v] = wn_;
                                        po[v] = pn_;
                                        s1 += (double)wn_ * (double)wn_;
                                        s2 += (double)pn_ * (double)pn_;
                                    } else if (EPI == EPI_FIRST) {
                                        const TC wn_ = (TC)(TOUT)(alpha * Aw + beta * w_c);
                                        const TC pn_ = (TC)(TOUT)(d0 * w_c + d1 * wn_);
                                        wo[v] = wn_;
                                        po[v] = pn_;
                                        s0 += (double)w_c * (double)w_c;
                                        s1 += (double)wn_ * (double)wn_;
                                        s2 += (double)pn_ * (double)pn_;
                                    } else if (EPI == EPI_START_SELF) {
                                        wo[v] = sigma * Aw + g_eval<TC>(a.gkind, w_c);
                                    } else if (kStart) {
                                        TC gv;
                                        if (a.gmode == G_VEC) {
                                            gv = (TC)a.g[idx + v];
                                        } else if (a.gmode == G_VEC_SCALED) {
                                            gv = (TC)(a.gscale * a.g[idx + v]);
                                        } else if (a.gmode == G_CUBIC_OF) {
                                            gv = g_eval<TC>(a.gkind, (TC)a.g[idx + v]);
                                        } else {
                                            gv = g_eval<TC>(a.gkind, w_c);
                                        }
                                        wo[v] = sigma * Aw + gv;
                                    }
                                }
                            }
                            if (kW) vst<V>(out, idx, wo);
                            if (EPI == EPI_NEWTON || EPI == EPI_FIRST) vst<V>(p, idx, po);
                        }
                        idx += ss;
                    }
                }
            }
        }
    }
}

template <int DIM, int COEF, int EPI, class TIN, class TOUT, int V>
__device__ __forceinline__ void stencil_tile(const SweepArgs& a, int t0, int t1, int t2,
                                             double& s0, double& s1, double& s2) {
    stencil_tile_w<DIM, COEF, EPI, TIN, TOUT, V>(a, t0, t1, t2, (int)(threadIdx.x >> 6), (int)(blockDim.x >> 6),
                                                 s0, s1, s2);
}

}  // namespace tile
}  // namespace expi
