// Batched phi_1(tau_i A_i) v_i for many independent 2D constant-coefficient
// stencil problems of uneven sizes.
//
// Each instance runs the same Leja interpolation as phi_action (Sec. III-C;
// substeps as in api.hip): per substep an optional start vector
// r = tau A y' + v, the first product, fused Newton products until the
// two-term stop test holds, and the update y' += p / s.  The host computes
// every instance's interval (the Gershgorin bound of a constant-coefficient
// 5-point operator has a closed form), substep count and divided
// differences ahead of time; they do not depend on the data.
//
// The work runs in rounds.  In each round every unfinished instance takes
// one step of its own sequence (start vector, the first product, two more
// Newton products, or the update; one product per step when pairs are off).
// A round is three ordinary kernels:
//  * two tiles kernels, one for the hot steps (the pairs of products) and
//    one for the rest: every workgroup builds the same list of unfinished
//    instances whose step is in its kernel's set and the prefix sums of
//    their tile counts from the states in memory, then works through a
//    contiguous share of the round's tiles (load balance across uneven
//    sizes; shares are contiguous per XCD so a tile's neighbours mostly sit
//    in the same L2);
//  * the finalize kernel: one workgroup per instance combines that
//    instance's tile partials in a fixed order, applies the stop test (after
//    each product of a pair) and advances its state.
// The kernel boundaries order the rounds; nothing waits on memory, so the
// rounds can be enqueued eagerly or recorded as kernel nodes of a HIP graph
// (no copies or fills inside) and replayed.  A round in which no instance is
// left returns at once.
//
// The alternative is one persistent kernel that runs every round, with grid
// barriers between the tiles of a round and its stop tests
// (expi_batch_launch_persistent; a cooperative launch, so that every
// workgroup is resident).  Every loop in it ends: the rounds are bounded,
// the tile loop is a grid-stride loop, and each barrier wait has a time
// limit past which the launch aborts.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "leja.h"
#include "stencil_tile.h"

namespace expi {

namespace {

// PH_PAIR: two Newton products in one step (w_{j+1} kept in registers)
enum Phase : int {
    PH_START = 0, PH_FIRST = 1, PH_NEWTON = 2, PH_UPDATE = 3, PH_DONE = 4, PH_FAILED = 5, PH_PAIR = 6
};

constexpr int kMaxBatch = 4096;
constexpr int kPersistWaves = 16;   // waves per workgroup of the persistent kernel
constexpr int kMaxGrid = 2048;      // workgroups of the persistent kernel at most

struct alignas(16) BatchInfo {   // static per instance
    long long off;               // offset of the instance's vectors, in elements
    int nx, ny;
    int tiles0, ntiles, vec, s;
    int dd_off, part_off;
    double ihx, ihy;             // 1/h^2 per axis
    double alpha, cg;            // 1/gamma and c/gamma of the interval map
    double tau, inv_s;
};

struct alignas(16) BatchState {  // advanced by the finalize step
    int phase, l, j, newton;
    int degree_max, degree_last, status;
    int wb;                      // which of w0 / w1 holds the newest Newton vector
    double t_prev, err_max;
    double fix;                  // d_{m+1} when a pair stopped at its first product, else 0
};

struct alignas(64) BatchCtrl {
    unsigned bar_count, bar_gen, abort, rounds;
    unsigned aux_next;           // round kernels: some instance's next step is an auxiliary one
    unsigned pad0;
    unsigned finished;           // instances done or failed (round kernels)
    unsigned hot_rounds;         // rounds with Newton products on stored vectors
    unsigned pad[8];
};

struct BatchArgs {
    const BatchInfo* info;
    BatchState* state;
    BatchCtrl* ctrl;
    const double* dd;
    const double* xi;
    double* partials;
    unsigned* bar_flag;           // grid barrier: one arrival flag per workgroup
    const double* v;
    double* y;
    void* w0;
    void* w1;
    void* p;
    int count, m_max, march, max_rounds, bc;
    int pairs;                    // Newton products two per step where the degree bound allows
    double c0, tol;
    long long deadline_ticks;   // longest wait at a barrier, GPU wall-clock ticks
};

// s_waitcnt operand that waits for vector memory operations only:
// vmcnt 0, expcnt 7 (no wait), lgkmcnt 15 (no wait).
constexpr int kWaitVmcnt0 = 0x0F70;

// Grid barrier with a time limit; returns false once any workgroup has
// aborted.  Every workgroup publishes its arrival in a flag of its own (the
// generation it waits for); one wave of workgroup 0 polls all flags, 64 at a
// time, and opens the next generation.  Arrivals go to distinct words, so
// nothing serializes on one counter (measured on the MI355X at 256
// workgroups: 5.8 us per barrier, against 7.6 us for per-XCD counters and
// 11.2 us for one counter).  Arrival releases the workgroup's writes;
// waiting polls with relaxed loads (an acquire per poll would invalidate
// caches for every waiter on every poll) and one acquire fence follows.  A
// waiter past the deadline (GPU wall clock) sets the abort flag, which every
// other waiter sees, so no wave can wait forever.  Generations only grow
// (each launch starts two past the last), so flags left by an earlier
// launch never match.
__device__ bool grid_barrier(const BatchArgs& B, int* s_ok) {
    // every wave waits for its own stores (s_waitcnt vmcnt(0)) before the
    // workgroup barrier: the workgroup barrier alone does not wait for them,
    // and the release below (L2 write-back, then the arrival) must cover the
    // stores of every wave, not only those of thread 0's
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    BatchCtrl* c = B.ctrl;
    // wave 0 of each workgroup arrives and waits; the other waves wait at
    // the workgroup barrier below
    if (threadIdx.x < 64) {
        const unsigned gen = __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x == 0)
            __hip_atomic_store(&B.bar_flag[blockIdx.x], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const long long t_end = wall_clock64() + B.deadline_ticks;
        int ok = 1;
        if (blockIdx.x == 0) {
            // every workgroup's flag, 64 at a time
            for (int b0 = 0; b0 < (int)gridDim.x && ok; b0 += 64) {
                const int b = b0 + (int)threadIdx.x;
                while (true) {
                    const bool in = b >= (int)gridDim.x ||
                                    __hip_atomic_load(&B.bar_flag[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                                        gen + 1u;
                    if (__all(in)) break;
                    if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                        wall_clock64() > t_end) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (ok) __hip_atomic_store(&c->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                else __hip_atomic_store(&c->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *s_ok = ok;
            }
        } else if (threadIdx.x == 0) {
            while (__hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() > t_end) {
                    __hip_atomic_store(&c->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
            *s_ok = ok;
        }
    }
    __syncthreads();
    return *s_ok != 0;
}

// Which steps a tiles kernel takes: all of them (persistent kernel); with
// one product per round, the products on Newton vectors of the storage type
// (first product of a later substep, Newton products: SET_HOT) and the rest
// (start vector, update, first product of the first substep, which reads
// the float64 input: SET_AUX); with two products per round, the pairs
// (SET_PAIR) and everything else (SET_REST).  Keeping the hot products in a
// kernel of their own keeps its register count, and so its occupancy, that
// of its own sweep.
enum PhaseSet : int { SET_ALL = 0, SET_HOT = 1, SET_AUX = 2, SET_PAIR = 3, SET_REST = 4 };

__device__ __forceinline__ bool in_set(int set, int phase, int l) {
    if (phase == PH_DONE || phase == PH_FAILED) return false;
    if (set == SET_ALL) return true;
    if (set == SET_PAIR) return phase == PH_PAIR;
    if (set == SET_REST) return phase != PH_PAIR;
    const bool hot = phase == PH_NEWTON || (phase == PH_FIRST && l > 0);
    return (set == SET_HOT) == hot;
}

// Steps whose code a kernel of each set holds.
template <int SET>
struct SetCode {
    static constexpr bool aux = SET == SET_ALL || SET == SET_AUX || SET == SET_REST;
    static constexpr bool single = SET == SET_ALL || SET == SET_HOT || SET == SET_REST;
    static constexpr bool pair = SET == SET_ALL || SET == SET_PAIR;
};

// Buffer loads and stores of V values of the storage type: the row offset
// goes in a scalar register, the lane's column offset in a vector register
// that stays the same along the march (no per-load address arithmetic).
template <class TW, int V>
struct Pack {
    TW v[V];
};

template <class TW, int V>
__device__ __forceinline__ void bld(__amdgpu_buffer_rsrc_t r, int voff, int soff, TW (&o)[V]) {
    constexpr int N = (int)sizeof(TW) * V;
    Pack<TW, V> p;
    if constexpr (N == 4)
        p = __builtin_bit_cast(Pack<TW, V>, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else if constexpr (N == 8)
        p = __builtin_bit_cast(Pack<TW, V>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        p = __builtin_bit_cast(Pack<TW, V>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = p.v[v];
}

//
// Stores are at most 8 bytes wide: the compiler has been seen to write the
// data registers of a 16-byte buffer store in the very next instruction,
// without the wait state such a store needs before its data registers are
// overwritten, and the store then wrote the new value for some lanes (FP64
// pair tiles, the first double of the lane's two).
template <class TW, int V>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, int voff, int soff, const TW (&o)[V]) {
    constexpr int N = (int)sizeof(TW) * V;
    Pack<TW, V> p;
#pragma unroll
    for (int v = 0; v < V; ++v) p.v[v] = o[v];
    typedef unsigned U2 __attribute__((ext_vector_type(2)));
    if constexpr (N == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, p), r, voff, soff, 0);
    } else if constexpr (N == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, p), r, voff, soff, 0);
    } else {
        static_assert(N == 16, "two 8-byte halves");
        Pack<TW, 1> lo, hi;
        lo.v[0] = o[0];
        hi.v[0] = o[1];
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, lo), r, voff, soff, 0);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, hi), r, voff + 8, soff, 0);
    }
}

// Two consecutive Newton products on one tile (two steps of the Newton
// recurrence of Sec. III-C): w_{j+1} = alpha A w_j + beta_j w_j, then
// w_{j+2} = alpha A w_{j+1} + beta_{j+1} w_{j+1}, with
// p += d_{j+1} w_{j+1} + d_{j+2} w_{j+2}.  w_{j+1} stays in registers: the
// wave forms it on its strip of 64 V points and on the point just beyond
// each end of the strip (lane 0 the left one, lane 63 the right one), on
// the tile's rows and on the row above and below them; then w_{j+2} and p
// on the tile.  Per point w_j and p are read once and w_{j+2} and p written
// once, for two products.  Partials: ||w_{j+1}||^2, ||p_{j+1}||^2,
// ||w_{j+2}||^2, ||p_{j+2}||^2 over the tile, summed in the order of the
// single product's sweep.
//
// A point's product is written as alpha A w + beta w =
// sum over faces of (alpha f) w_nb + (beta - alpha sum f) w_c, with face
// weights f = coef/h^2 (0 for a face towards a neighbour that does not
// exist, except that under homogeneous Dirichlet conditions such a face
// still takes its share of the diagonal): one multiply and four fused
// multiply-adds per point; the x weights are fixed per lane and the y ones
// per row.
template <class TW, int V>
__device__ void pair_tile(const BatchArgs& B, const BatchInfo& I, const BatchState& S, int t0, int t1,
                          double* red_partial) {
    using TC = TW;
    constexpr int sz = (int)sizeof(TW);
    const int lane = threadIdx.x & 63;
    const int n0 = I.nx, n1 = I.ny;
    const int i0 = t0 * 64 * V;
    const int i = i0 + lane * V;
    const int kb = t1 * B.march, ke = min(kb + B.march, n1);
    const bool active = i < n0;
    const int ic = active ? i : (n0 - V);
    // the point beyond the strip at which lane 0 (63) forms w_{j+1}, and the
    // w_j point beyond that one, which lane 1 (62) loads in the same load
    // and hands over
    const int xe = (lane == 0) ? i0 - 1 : (lane == 63 ? i0 + 64 * V : ic);
    const int xg = (lane == 1) ? i0 - 2 : (lane == 62 ? i0 + 64 * V + 1 : xe);
    const int gsrc = (lane == 0) ? 1 : (lane == 63 ? 62 : lane);
    const int nbytes = n0 * n1 * sz;
    const TW* w = static_cast<const TW*>(S.wb ? B.w1 : B.w0) + I.off;
    TW* out = static_cast<TW*>(S.wb ? B.w0 : B.w1) + I.off;
    TW* pp = static_cast<TW*>(B.p) + I.off;
    const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(const_cast<TW*>(w), 0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(out, 0, nbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(pp, 0, nbytes, 0x00020000);
    const int vo = ic * sz;                                  // the lane's points
    const int vg = min(max(xg, 0), n0 - 1) * sz;             // its point beyond the strip
    // every load is from a row clamped into the grid; values of rows and
    // columns that do not exist get weight 0
    auto roff = [&](int k) { return n0 * min(max(k, 0), n1 - 1) * sz; };
    auto g_load = [&](int k) -> TC {
        TC t[1];
        bld<TW, 1>(rw, vg, roff(k), t);
        return t[0];
    };
    const bool dir = (B.bc == EXPI_DIRICHLET0);
    const TC alpha = (TC)I.alpha;
    const int j = S.j;
    const TC beta1 = (TC)(-(I.cg + B.xi[j])), beta2 = (TC)(-(I.cg + B.xi[j + 1]));
    const TC d1 = (TC)B.dd[I.dd_off + j + 1], d2 = (TC)B.dd[I.dd_off + j + 2];
    const TC fx = (TC)(B.c0 * I.ihx), fy = (TC)(B.c0 * I.ihy);
    // x weights: alpha f of the two x faces of each of the lane's points and
    // of its point beyond the strip, and alpha times the x part of the
    // diagonal
    TC axm[V + 1], axq[V + 1], adx[V + 1];
#pragma unroll
    for (int v = 0; v <= V; ++v) {
        const int x = (v < V) ? i + v : xe;
        const bool em = x > 0, eq = x < n0 - 1;
        axm[v] = em ? alpha * fx : (TC)0;
        axq[v] = eq ? alpha * fx : (TC)0;
        adx[v] = alpha * (((em || dir) ? fx : (TC)0) + ((eq || dir) ? fx : (TC)0));
    }
    // y weights of row q: alpha f of its two faces and the diagonal
    // coefficient beta - alpha sum f without the x part
    auto yw = [&](int q, TC beta, TC& aym, TC& ayq, TC& cdy) {
        const bool em = q > 0, eq = q < n1 - 1;
        aym = em ? alpha * fy : (TC)0;
        ayq = eq ? alpha * fy : (TC)0;
        cdy = beta - alpha * (((em || dir) ? fy : (TC)0) + ((eq || dir) ? fy : (TC)0));
    };
    auto prod = [&](int v, TC wl, TC wr, TC wm, TC wq, TC wc, TC aym, TC ayq, TC cdy) -> TC {
        return axm[v] * wl + axq[v] * wr + aym * wm + ayq * wq + (cdy - adx[v]) * wc;
    };
    // w_{j+1} on row q of the strip (u) and at the lane's point beyond it
    // (ue), from w_j rows q-1, q, q+1 (wm, wc, wq), the beyond-strip values
    // of those rows (gm, gc, gq) and the farther point of row q (in gc of
    // the neighbouring lane)
    auto form_u = [&](const TC (&wm)[V], const TC (&wc)[V], const TC (&wq)[V], TC gm, TC gc, TC gq, int q,
                      TC (&u)[V], TC& ue) {
        TC aym, ayq, cdy;
        yw(q, beta1, aym, ayq, cdy);
        TC left = __shfl_up(wc[V - 1], 1, 64);
        TC right = __shfl_down(wc[0], 1, 64);
        const TC far = __shfl(gc, gsrc, 64);
        if (lane == 0) left = gc;
        if (lane == 63) right = gc;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const TC wl = (v > 0) ? wc[v - 1] : left;
            const TC wr = (v < V - 1) ? wc[v + 1] : right;
            u[v] = (TC)(TW)prod(v, wl, wr, wm[v], wq[v], wc[v], aym, ayq, cdy);
        }
        const TC el = (lane == 63) ? wc[V - 1] : far;
        const TC er = (lane == 63) ? far : wc[0];
        ue = (TC)(TW)prod(V, el, er, gm, gq, gc, aym, ayq, cdy);
    };
    // Register queues, indexed by row modulo 4 (the march is unrolled four
    // rows per block, so every queue rotates by renaming and no value is
    // copied: a copy of a register that a load is still filling would make
    // the wave wait for that load).  Step k (output row k) finds w_j of rows
    // k .. k+2 and their beyond-strip values, loaded a step or more ahead,
    // and issues the loads of w_j row k+3 (used next step) and of p row k+2
    // (used two steps on); w_{j+1} rows k-1, k sit in U, row k+1 is formed
    // into the slot of row k-3.
    TC W[4][V], P[4][V], U[4][V], G[4], Ue[2];
    {
        // rows kb-2 .. kb+1 of w_j (slots 2, 3, 0, 1), p rows kb, kb+1
        bld<TW, V>(rw, vo, roff(kb - 2), W[2]);
        bld<TW, V>(rw, vo, roff(kb - 1), W[3]);
        bld<TW, V>(rw, vo, roff(kb), W[0]);
        bld<TW, V>(rw, vo, roff(kb + 1), W[1]);
        G[2] = g_load(kb - 2);
        G[3] = g_load(kb - 1);
        G[0] = g_load(kb);
        G[1] = g_load(kb + 1);
        bld<TW, V>(rp, vo, roff(kb), P[0]);
        bld<TW, V>(rp, vo, roff(kb + 1), P[1]);
        TC ue_m;   // (w_{j+2} needs w_{j+1} beyond the strip on its own row only)
        form_u(W[2], W[3], W[0], G[2], G[3], G[0], kb - 1, U[3], ue_m);
        // row kb+2 into the slot of row kb-2, which is no longer needed
        bld<TW, V>(rw, vo, roff(kb + 2), W[2]);
        G[2] = g_load(kb + 2);
        form_u(W[3], W[0], W[1], G[3], G[0], G[1], kb, U[0], Ue[0]);
    }
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = kb; k0 < ke; k0 += 4) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int k = k0 + st;
            const bool valid = k < ke;   // all four steps run; only valid ones count and store
            // loads ahead: w_j row k+3 (next step), p row k+2 (two steps on)
            bld<TW, V>(rw, vo, roff(k + 3), W[(st + 3) & 3]);
            G[(st + 3) & 3] = g_load(k + 3);
            bld<TW, V>(rp, vo, roff(k + 2), P[(st + 2) & 3]);
            // w_{j+1} on row k+1, from w_j rows k, k+1, k+2
            form_u(W[st & 3], W[(st + 1) & 3], W[(st + 2) & 3], G[st & 3], G[(st + 1) & 3], G[(st + 2) & 3],
                   k + 1, U[(st + 1) & 3], Ue[(st + 1) & 1]);
            // w_{j+2} and p on row k, from w_{j+1} rows k-1, k, k+1
            const TC* um = U[(st + 3) & 3];
            const TC* uc = U[st & 3];
            const TC* uq = U[(st + 1) & 3];
            const TC* pk = P[st & 3];
            TC aym, ayq, cdy;
            yw(k, beta2, aym, ayq, cdy);
            TC left = __shfl_up(uc[V - 1], 1, 64);
            TC right = __shfl_down(uc[0], 1, 64);
            if (lane == 0) left = Ue[st & 1];
            if (lane == 63) right = Ue[st & 1];
            TC wo[V], po[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const TC wl = (v > 0) ? uc[v - 1] : left;
                const TC wr = (v < V - 1) ? uc[v + 1] : right;
                const TC u2 = (TC)(TW)prod(v, wl, wr, um[v], uq[v], uc[v], aym, ayq, cdy);
                const TC p1 = (TC)(TW)(pk[v] + d1 * uc[v]);
                const TC p2 = (TC)(TW)(p1 + d2 * u2);
                wo[v] = u2;
                po[v] = p2;
                if (active && valid) {
                    s[0] += (double)uc[v] * (double)uc[v];
                    s[1] += (double)p1 * (double)p1;
                    s[2] += (double)u2 * (double)u2;
                    s[3] += (double)p2 * (double)p2;
                }
            }
            // lanes past the row end, and steps past the tile, store past
            // the buffer (dropped)
            const int vs = (active && valid) ? vo : nbytes;
            bst<TW, V>(ro, vs, roff(k), wo);
            bst<TW, V>(rp, vs, roff(k), po);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red_partial[q] = s[q];
    }
}

// One tile of an instance: `march` rows of 64 V points, taken by one wave
// (lt = tile index within the instance).  The wave reduces its norm sums
// across its lanes and lane 0 writes them as the tile's partials; no
// workgroup barrier, so the waves of a workgroup work independently.
template <class TW, int V, int SET>
__device__ void run_tile(const BatchArgs& B, const BatchInfo& I, const BatchState& S, int phase,
                         int lt, double* red_partial) {
    const int t0 = lt % I.tiles0, t1 = lt / I.tiles0;
    SweepArgs a{};
    a.n[0] = I.nx;
    a.n[1] = I.ny;
    a.n[2] = 1;
    a.ih2[0] = I.ihx;
    a.ih2[1] = I.ihy;
    a.ih2[2] = 0.0;
    a.bc = B.bc;
    a.c0 = B.c0;
    a.march = B.march;
    TW* w0 = static_cast<TW*>(B.w0) + I.off;
    TW* w1 = static_cast<TW*>(B.w1) + I.off;
    TW* pp = static_cast<TW*>(B.p) + I.off;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (SetCode<SET>::aux && phase == PH_START) {
        a.x = B.y + I.off;
        a.out = w1;
        a.g = B.v + I.off;
        a.gmode = G_VEC;
        a.sigma = I.tau;
        tile::stencil_tile_w<2, EXPI_COEF_CONST, EPI_START, double, TW, V>(a, t0, t1, 0, 0, 1, s0, s1, s2);
        return;
    }
    if (SetCode<SET>::aux && phase == PH_UPDATE) {
        // y' <- (l == 0 ? 0 : y') + p / s over the tile's points; after a pair
        // that stopped at its first product, p - d_{m+1} w_{m+1}
        const int lane = threadIdx.x & 63;
        double* y = B.y + I.off;
        const TW* wx = S.wb ? w1 : w0;
        for (int r = 0; r < B.march; ++r) {
            const int j = t1 * B.march + r;
            if (j >= I.ny) break;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int i = t0 * 64 * V + lane * V + v;
                if (i < I.nx) {
                    const int idx = i + I.nx * j;
                    const double pv = (S.fix != 0.0) ? (double)pp[idx] - S.fix * (double)wx[idx] : (double)pp[idx];
                    y[idx] = (S.l == 0 ? 0.0 : y[idx]) + I.inv_s * pv;
                }
            }
        }
        return;
    }
    if (phase == PH_PAIR) {
        if constexpr (SetCode<SET>::pair) pair_tile<TW, V>(B, I, S, t0, t1, red_partial);
        return;
    }
    const int j = (phase == PH_FIRST) ? 0 : S.j;
    a.alpha = I.alpha;
    a.beta = -(I.cg + B.xi[j]);
    a.d0 = B.dd[I.dd_off];
    a.d1 = B.dd[I.dd_off + j + 1];
    a.p = pp;
    if (phase == PH_FIRST) {
        a.out = w0;
        if (S.l == 0) {
            if constexpr (SetCode<SET>::aux) {
                a.x = B.v + I.off;
                tile::stencil_tile_w<2, EXPI_COEF_CONST, EPI_FIRST, double, TW, V>(a, t0, t1, 0, 0, 1, s0, s1, s2);
            }
        } else {
            if constexpr (SetCode<SET>::single) {
                a.x = w1;
                tile::stencil_tile_w<2, EXPI_COEF_CONST, EPI_FIRST, TW, TW, V>(a, t0, t1, 0, 0, 1, s0, s1, s2);
            }
        }
    } else {
        if constexpr (SetCode<SET>::single) {
            a.x = S.wb ? w1 : w0;
            a.out = S.wb ? w0 : w1;
            tile::stencil_tile_w<2, EXPI_COEF_CONST, EPI_NEWTON, TW, TW, V>(a, t0, t1, 0, 0, 1, s0, s1, s2);
        }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) {
        red_partial[0] = s0;
        red_partial[1] = s1;
        red_partial[2] = s2;
    }
}

// Four per-thread sums combined over the workgroup in a fixed order (the
// order block_combine takes for three); the result is valid in thread 0.
__device__ void block_sum4(double (&v)[4], double (*red)[4]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
        for (int q = 0; q < 4; ++q) red[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 4; ++q) {
            double acc = red[0][q];
            for (int w = 1; w < nw; ++w) acc += red[w][q];
            v[q] = acc;
        }
    }
    __syncthreads();
}

// The step after Newton products that reached degree m without a stop: the
// next product, two of them when the degree bound leaves room for both.
__device__ __forceinline__ int next_products(const BatchArgs& B, int m) {
    return (B.pairs && m + 2 <= B.m_max) ? PH_PAIR : PH_NEWTON;
}

// Combine an instance's tile partials in index order and advance its state.
// Returns the new phase in thread 0 (-1 in the other threads).
__device__ int finalize_instance(const BatchArgs& B, int inst) {
    __shared__ double red[kPersistWaves][3];   // a round kernel's or the persistent kernel's waves
    const BatchInfo& I = B.info[inst];
    BatchState* S = &B.state[inst];
    const int phase = S->phase;
    // every wave has loaded the phase before thread 0 stores the next one: a
    // wave that loaded it afterwards would take the other branch and pair
    // the workgroup's later barriers wrongly
    __syncthreads();
    int next = -1;
    if (phase == PH_FIRST || phase == PH_NEWTON) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int t = threadIdx.x; t < I.ntiles; t += blockDim.x) {
            const double* q = B.partials + 4 * (size_t)(I.part_off + t);
            s0 += q[0];
            s1 += q[1];
            s2 += q[2];
        }
        block_combine<EPI_NEWTON>(s0, s1, s2, red);
        if (threadIdx.x == 0) {
            const int j = (phase == PH_FIRST) ? 0 : S->j;
            const double wn = sqrt(s1), pn = sqrt(s2);
            const double t = fabs(B.dd[I.dd_off + j + 1]) * wn;
            const double tprev = (phase == PH_FIRST) ? fabs(B.dd[I.dd_off]) * sqrt(s0) : S->t_prev;
            const int m = j + 1;
            const double num = tprev + t;
            const double err = (pn > 0.0) ? num / pn : (num == 0.0 ? 0.0 : INFINITY);
            S->newton += 1;
            S->t_prev = t;
            if (!isfinite(wn) || !isfinite(pn) || !isfinite(tprev)) {
                next = PH_FAILED;
                S->status = 2;
            } else if (m >= 2 && num <= B.tol * pn) {
                S->degree_last = m;
                S->degree_max = max(S->degree_max, m);
                S->err_max = fmax(S->err_max, err);
                next = PH_UPDATE;
            } else if (m >= B.m_max) {
                next = PH_FAILED;
                S->status = 1;
                S->err_max = fmax(S->err_max, err);
            } else {
                next = next_products(B, m);
                S->j = m;
            }
            // w_1 went to w0, a later product to the buffer it did not read
            S->wb = (phase == PH_FIRST) ? 0 : (S->wb ^ 1);
            S->phase = next;
        }
    } else if (phase == PH_PAIR) {
        // the two-term test after each product of the pair, as two single
        // steps would apply it: at m = j+1 (a stop there leaves the second
        // product's term in p, which the update takes back out), else at
        // m = j+2
        __shared__ double red4[kPersistWaves][4];
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int t = threadIdx.x; t < I.ntiles; t += blockDim.x) {
            const double* q = B.partials + 4 * (size_t)(I.part_off + t);
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] += q[k];
        }
        block_sum4(v, red4);
        if (threadIdx.x == 0) {
            const int j = S->j;
            const double w1n = sqrt(v[0]), p1n = sqrt(v[1]), w2n = sqrt(v[2]), p2n = sqrt(v[3]);
            const double d2 = B.dd[I.dd_off + j + 2];
            const double t1 = fabs(B.dd[I.dd_off + j + 1]) * w1n, t2 = fabs(d2) * w2n;
            const double tprev = S->t_prev;
            auto rel = [](double num, double pn) { return (pn > 0.0) ? num / pn : (num == 0.0 ? 0.0 : INFINITY); };
            S->newton += 2;
            S->wb ^= 1;
            if (!isfinite(w1n) || !isfinite(p1n) || !isfinite(w2n) || !isfinite(p2n) || !isfinite(tprev)) {
                next = PH_FAILED;
                S->status = 2;
            } else if (tprev + t1 <= B.tol * p1n) {   // m = j+1 >= 2
                S->degree_last = j + 1;
                S->degree_max = max(S->degree_max, j + 1);
                S->err_max = fmax(S->err_max, rel(tprev + t1, p1n));
                S->fix = d2;
                next = PH_UPDATE;
            } else if (t1 + t2 <= B.tol * p2n) {
                S->degree_last = j + 2;
                S->degree_max = max(S->degree_max, j + 2);
                S->err_max = fmax(S->err_max, rel(t1 + t2, p2n));
                next = PH_UPDATE;
            } else if (j + 2 >= B.m_max) {
                next = PH_FAILED;
                S->status = 1;
                S->err_max = fmax(S->err_max, rel(t1 + t2, p2n));
            } else {
                S->t_prev = t2;
                S->j = j + 2;
                next = next_products(B, j + 2);
            }
            S->phase = next;
        }
    } else if (threadIdx.x == 0) {
        next = phase;
        if (phase == PH_START) {
            next = PH_FIRST;
        } else if (phase == PH_UPDATE) {
            const int l = S->l + 1;
            S->l = l;
            S->j = 0;
            S->fix = 0.0;
            next = (l < I.s) ? PH_START : PH_DONE;
        }
        S->phase = next;
    }
    __syncthreads();
    return next;
}

// Exclusive prefix sum over the workgroup (blockDim a multiple of 64);
// `total` receives the sum of all values.
__device__ int block_scan(int v, int* s_wave, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < nw; ++w) {
            const int c = s_wave[w];
            s_wave[w] = acc;
            acc += c;
        }
        s_wave[nw] = acc;
    }
    __syncthreads();
    const int r = s_wave[wv] + x - v;
    *total = s_wave[nw];
    __syncthreads();
    return r;
}

__device__ __forceinline__ bool active_phase(int ph) { return ph != PH_DONE && ph != PH_FAILED; }

// Unfinished instances whose step is in `set`, in index order (s_ids), and
// the prefix sums of their tile counts (s_pref, with s_pref[nact] = total),
// built by the whole workgroup from the states in memory; every workgroup
// builds the same list.
__device__ void active_list(const BatchArgs& B, int set, int* s_pref, int* s_ids, int* s_wave,
                            int& nact, int& total) {
    const int nt = blockDim.x;
    const int per = (B.count + nt - 1) / nt;
    const int lo = min((int)threadIdx.x * per, B.count), hi = min(lo + per, B.count);
    int cnt = 0, tiles = 0;
    for (int i = lo; i < hi; ++i) {
        if (in_set(set, B.state[i].phase, B.state[i].l)) {
            ++cnt;
            tiles += B.info[i].ntiles;
        }
    }
    int n_all, t_all;
    int k = block_scan(cnt, s_wave, &n_all);
    int tp = block_scan(tiles, s_wave, &t_all);
    for (int i = lo; i < hi; ++i) {
        if (in_set(set, B.state[i].phase, B.state[i].l)) {
            s_ids[k] = i;
            s_pref[k] = tp;
            tp += B.info[i].ntiles;
            ++k;
        }
    }
    if (threadIdx.x == 0) s_pref[n_all] = t_all;
    __syncthreads();
    nact = n_all;
    total = t_all;
}

// Position of global tile t in the list: the last k with s_pref[k] <= t.
__device__ __forceinline__ int find_instance(const int* s_pref, int nact, int t) {
    int l = 0, h = nact - 1;
    while (l < h) {
        const int mid = (l + h + 1) >> 1;
        if (s_pref[mid] <= t) l = mid; else h = mid - 1;
    }
    return l;
}

// ---- round kernels -----------------------------------------------------------

// The tiles of one round whose steps are in SET.  The grid is a multiple of
// the XCD count.  The instance list lives in dynamic LDS of
// (2 count + kMaxWaves + 2) ints.
template <class TW, int SET>
__global__ __launch_bounds__(kMaxWaves * 64) void batch_tiles_kernel(BatchArgs B) {
    extern __shared__ int s_dyn[];
    int* s_pref = s_dyn;                  // count + 1
    int* s_ids = s_dyn + B.count + 1;     // count
    int* s_wave = s_ids + B.count;        // kMaxWaves + 1
    if (B.ctrl->finished >= (unsigned)B.count) return;
    // the auxiliary kernel of a round without auxiliary steps returns at
    // once (the flag is set by the previous round's stop tests and cleared
    // by the hot kernel that follows; kernel boundaries order the three)
    constexpr bool kHot = (SET == SET_HOT || SET == SET_PAIR);
    if (!kHot && B.ctrl->aux_next == 0) return;
    // a round counts when some instance is unfinished at its start (the
    // count changes only in the finalize kernel that ends the round)
    if (kHot && blockIdx.x == 0 && threadIdx.x == 0) {
        B.ctrl->rounds += 1;
        B.ctrl->aux_next = 0;
    }
    int nact, total;
    active_list(B, SET, s_pref, s_ids, s_wave, nact, total);
    // values read from LDS are the same in every lane; saying so keeps the
    // instance data and everything derived from it in scalar registers
    nact = __builtin_amdgcn_readfirstlane(nact);
    total = __builtin_amdgcn_readfirstlane(total);
    if (nact == 0) return;
    if (kHot && blockIdx.x == 0 && threadIdx.x == 0) B.ctrl->hot_rounds += 1;
    // Grid-stride order over the XCD-major logical wave index: in each pass
    // the waves together take G consecutive tiles and every XCD a contiguous
    // block of them, so tiles that share halo rows and DRAM pages run at the
    // same time on the same L2.  Each wave goes through its tiles alone.
    const int nw = blockDim.x >> 6;
    const int G = gridDim.x * nw;
    // (the same in every lane of a wave: saying so keeps the tile indices,
    // rows and row offsets in scalar registers)
    const int L = __builtin_amdgcn_readfirstlane(xcd_tile(gridDim.x / kXcd) * nw + (int)(threadIdx.x >> 6));
    if (L >= total) return;
    int q = __builtin_amdgcn_readfirstlane(find_instance(s_pref, nact, L));
    int inst = __builtin_amdgcn_readfirstlane(s_ids[q]);
    int base = __builtin_amdgcn_readfirstlane(s_pref[q]);
    int next = __builtin_amdgcn_readfirstlane(s_pref[q + 1]);
    BatchInfo I = B.info[inst];
    BatchState S = B.state[inst];
    for (int t = L; t < total; t += G) {
        if (t >= next) {
            q = __builtin_amdgcn_readfirstlane(find_instance(s_pref, nact, t));
            inst = __builtin_amdgcn_readfirstlane(s_ids[q]);
            base = __builtin_amdgcn_readfirstlane(s_pref[q]);
            next = __builtin_amdgcn_readfirstlane(s_pref[q + 1]);
            I = B.info[inst];
            S = B.state[inst];
        }
        const int lt = t - base;
        double* part = B.partials + 4 * (size_t)(I.part_off + lt);
        if (I.vec == 2) run_tile<TW, 2, SET>(B, I, S, S.phase, lt, part);
        else run_tile<TW, 1, SET>(B, I, S, S.phase, lt, part);
    }
}

size_t tiles_lds_bytes(int count) { return sizeof(int) * (2 * (size_t)count + kMaxWaves + 2); }

// Stop test and state update of one instance per workgroup.
__global__ __launch_bounds__(256) void batch_finalize_kernel(BatchArgs B) {
    const int inst = blockIdx.x;
    if (inst >= B.count || !active_phase(B.state[inst].phase)) return;
    const int next = finalize_instance(B, inst);
    if (threadIdx.x == 0) {
        if (!active_phase(next)) atomicAdd(&B.ctrl->finished, 1u);
        // (a first product made here follows a start vector: l >= 1, hot
        // with one product per round; with two, every step but a pair is
        // auxiliary)
        if (next == PH_START || next == PH_UPDATE ||
            (B.pairs && active_phase(next) && next != PH_PAIR))
            B.ctrl->aux_next = 1;
    }
}

// ---- persistent kernel --------------------------------------------------------

template <class TW>
__global__ __launch_bounds__(kPersistWaves * 64) void batch_kernel(BatchArgs B) {
    __shared__ int s_pref[kMaxBatch + 1];
    __shared__ int s_ids[kMaxBatch];
    __shared__ int s_wave[kPersistWaves + 1];
    __shared__ int s_ok;
    for (int round = 0; round < B.max_rounds; ++round) {
        // (A) active instances and the prefix sums of their tile counts
        int nact, total;
        active_list(B, SET_ALL, s_pref, s_ids, s_wave, nact, total);
        if (nact == 0) break;
        // (B) the round's tiles in grid-stride order over the XCD-major
        // wave index, as in the round kernels: each wave computes its tile
        // indices itself and goes through its tiles alone
        const int nw = blockDim.x >> 6;
        const int G = gridDim.x * nw;
        int q = -1, inst = 0, base = 0, next = 0;
        const int t_first = __builtin_amdgcn_readfirstlane(xcd_tile(gridDim.x / kXcd) * nw + (int)(threadIdx.x >> 6));
        for (int t = t_first; t < total; t += G) {
            if (q < 0 || t >= next) {
                q = __builtin_amdgcn_readfirstlane(find_instance(s_pref, nact, t));
                inst = __builtin_amdgcn_readfirstlane(s_ids[q]);
                base = __builtin_amdgcn_readfirstlane(s_pref[q]);
                next = __builtin_amdgcn_readfirstlane(s_pref[q + 1]);
            }
            const BatchInfo& I = B.info[inst];
            const BatchState S = B.state[inst];
            const int lt = t - base;
            double* part = B.partials + 4 * (size_t)(I.part_off + lt);
            if (I.vec == 2) run_tile<TW, 2, SET_ALL>(B, I, S, S.phase, lt, part);
            else run_tile<TW, 1, SET_ALL>(B, I, S, S.phase, lt, part);
        }
        // (C) all tiles of the round are done
        if (!grid_barrier(B, &s_ok)) return;
        // (D) finalize: active instance k belongs to workgroup k mod grid
        for (int q = blockIdx.x; q < nact; q += gridDim.x) finalize_instance(B, s_ids[q]);
        if (blockIdx.x == 0 && threadIdx.x == 0) B.ctrl->rounds = round + 1;
        // (E) publish the new states
        if (!grid_barrier(B, &s_ok)) return;
    }
}

__global__ void batch_reset_kernel(BatchState* st, BatchCtrl* ctrl, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        BatchState s{};
        s.phase = PH_FIRST;
        st[i] = s;
    }
    if (i == 0) {
        ctrl->bar_count = 0;
        ctrl->bar_gen += 2;   // past every flag an earlier launch left (zeroed at prepare)
        ctrl->abort = 0;
        ctrl->rounds = 0;
        ctrl->finished = 0;
        ctrl->hot_rounds = 0;
        ctrl->aux_next = 1;   // the first products read the float64 input
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct Batch {
    int last_rounds = 0;   // rounds the last eager solve needed (0: none yet)
    int count, dtype, bc, m_max, waves, march;
    int pairs = 1;                // Newton products two per round (expi_batch_set_pairs)
    double c0, tol;
    std::vector<BatchInfo> info;
    std::vector<double> dd;       // count x (m_max + 1)
    std::vector<double> xi;       // m_max + 1
    long long total_len = 0;
    int total_tiles = 0, max_rounds = 0;
    size_t off_ctrl, off_bar, off_info, off_state, off_dd, off_xi, off_part, off_w0, off_w1, off_p, ws_total;
    void* prepared_ws = nullptr;
    int grid = 0;                 // persistent kernel
    int round_grid = 0;           // tiles kernel of a round
    long long deadline_ticks = 0;
    hipGraph_t graph = nullptr;   // captured rounds (or the persistent launch)
    hipGraphExec_t graph_exec = nullptr;
    int graph_rounds = 0;
    BatchCtrl* pinned = nullptr;  // host slots for status read-backs
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

int bfail(int code, const std::string& m) {
    set_error(m);
    return code;
}

#define BHIP(expr)                                                                   \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));            \
            return EXPI_EHIP;                                                        \
        }                                                                            \
    } while (0)

void layout_tiles(Batch& b) {
    int part = 0;
    b.total_tiles = 0;
    for (auto& I : b.info) {
        I.tiles0 = (I.nx + 64 * I.vec - 1) / (64 * I.vec);
        const int tiles1 = (I.ny + b.march - 1) / b.march;   // one wave per tile
        I.ntiles = I.tiles0 * tiles1;
        I.part_off = part;
        part += I.ntiles;
    }
    b.total_tiles = part;
    const size_t tw = b.dtype == EXPI_F32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    b.off_ctrl = take(sizeof(BatchCtrl));
    b.off_bar = take(sizeof(unsigned) * kMaxGrid);
    b.off_info = take(sizeof(BatchInfo) * b.count);
    b.off_state = take(sizeof(BatchState) * b.count);
    b.off_dd = take(sizeof(double) * b.dd.size());
    b.off_xi = take(sizeof(double) * b.xi.size());
    // partial slots sized for the smallest accepted tiles (march 4)
    size_t maxpart = 0;
    for (const auto& I : b.info) {
        const int t0 = (I.nx + 63) / 64;
        maxpart += (size_t)t0 * ((I.ny + 3) / 4);
    }
    b.off_part = take(4 * sizeof(double) * maxpart);
    b.off_w0 = take(tw * b.total_len);
    b.off_w1 = take(tw * b.total_len);
    b.off_p = take(tw * b.total_len);
    b.ws_total = off;
}

BatchArgs make_args(const Batch& b, char* ws, const double* v, double* y) {
    BatchArgs a{};
    a.info = reinterpret_cast<const BatchInfo*>(ws + b.off_info);
    a.state = reinterpret_cast<BatchState*>(ws + b.off_state);
    a.ctrl = reinterpret_cast<BatchCtrl*>(ws + b.off_ctrl);
    a.dd = reinterpret_cast<const double*>(ws + b.off_dd);
    a.xi = reinterpret_cast<const double*>(ws + b.off_xi);
    a.partials = reinterpret_cast<double*>(ws + b.off_part);
    a.bar_flag = reinterpret_cast<unsigned*>(ws + b.off_bar);
    a.v = v;
    a.y = y;
    a.w0 = ws + b.off_w0;
    a.w1 = ws + b.off_w1;
    a.p = ws + b.off_p;
    a.count = b.count;
    a.m_max = b.m_max;
    a.march = b.march;
    a.max_rounds = b.max_rounds;
    a.bc = b.bc;
    a.pairs = b.pairs;
    a.c0 = b.c0;
    a.tol = b.tol;
    a.deadline_ticks = b.deadline_ticks;
    return a;
}

// The kernel of a round's hot steps (hot = true) or of the others, for the
// batch's storage type and products per round.
template <class TW>
const void* tiles_kernel_t(bool pairs, bool hot) {
    if (pairs)
        return hot ? reinterpret_cast<const void*>(batch_tiles_kernel<TW, SET_PAIR>)
                   : reinterpret_cast<const void*>(batch_tiles_kernel<TW, SET_REST>);
    return hot ? reinterpret_cast<const void*>(batch_tiles_kernel<TW, SET_HOT>)
               : reinterpret_cast<const void*>(batch_tiles_kernel<TW, SET_AUX>);
}

const void* tiles_kernel(const Batch& b, bool hot) {
    return b.dtype == EXPI_F32 ? tiles_kernel_t<float>(b.pairs != 0, hot)
                               : tiles_kernel_t<double>(b.pairs != 0, hot);
}

// The persistent kernel needs every workgroup resident at once.  The grid
// is a multiple of the XCD count and every launch is cooperative, so the runtime refuses a grid that cannot
// be co-resident instead of letting the barrier wait.
int occupancy_grid(Batch& b) {
    int dev = 0, cus = 0, per = 0, khz = 0;
    BHIP(hipGetDevice(&dev));
    BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    BHIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (b.dtype == EXPI_F32)
        BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<float>, 64 * kPersistWaves, 0));
    else
        BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel<double>, 64 * kPersistWaves, 0));
    if (per < 1) return bfail(EXPI_EHIP, "batched kernel cannot be resident");
    // one workgroup of 16 waves per CU: the waves take tiles independently,
    // and few workgroups keep every grid barrier cheap (its cost grows with
    // the workgroups that arrive)
    b.grid = std::min(kMaxGrid, std::max(kXcd, (cus / kXcd) * kXcd));
    // tiles kernels of a round: as many workgroups as fit on the device at
    // once (occupancy of the hot kernel), a multiple of the XCD count, no
    // more than the batch has tiles
    int per_hot = 0;
    BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_hot, tiles_kernel(b, true), 64 * b.waves,
                                                      tiles_lds_bytes(b.count)));
    if (per_hot < 1) return bfail(EXPI_EHIP, "batched tiles kernel cannot be resident");
    const int wgs = (b.total_tiles + b.waves - 1) / b.waves;   // a tile per wave
    const int want = std::min(per_hot * cus, ((wgs + kXcd - 1) / kXcd) * kXcd);
    b.round_grid = std::max(kXcd, (want / kXcd) * kXcd);
    // a barrier wait longer than two seconds means something is wrong
    b.deadline_ticks = 2ll * 1000ll * (long long)(khz > 0 ? khz : 100000);
    return EXPI_OK;
}

const void* kernel_ptr(const Batch& b) {
    return b.dtype == EXPI_F32 ? reinterpret_cast<const void*>(batch_kernel<float>)
                               : reinterpret_cast<const void*>(batch_kernel<double>);
}

int enqueue(Batch& b, char* ws, const double* v, double* y, hipStream_t s) {
    BatchArgs a = make_args(b, ws, v, y);
    hipLaunchKernelGGL(batch_reset_kernel, dim3((b.count + 255) / 256), dim3(256), 0, s,
                       a.state, a.ctrl, b.count);
    BHIP(hipGetLastError());
    void* params[] = {&a};
    BHIP(hipLaunchCooperativeKernel(kernel_ptr(b), dim3(b.grid), dim3(64 * kPersistWaves), params, 0, s));
    return EXPI_OK;
}

constexpr int kRoundChunk = 8;   // rounds enqueued between status read-backs

// One round: the auxiliary steps, the hot products, then the stop tests.
hipError_t enqueue_round(const Batch& b, const BatchArgs& a, hipStream_t s) {
    const size_t lds = tiles_lds_bytes(b.count);
    void* args[] = {const_cast<BatchArgs*>(&a)};
    hipError_t e = hipLaunchKernel(tiles_kernel(b, false), dim3(b.round_grid), dim3(64 * b.waves), args, lds, s);
    if (e == hipSuccess)
        e = hipLaunchKernel(tiles_kernel(b, true), dim3(b.round_grid), dim3(64 * b.waves), args, lds, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(b.count), dim3(256), 0, s, a);
    return hipGetLastError();
}

int ensure_pinned(Batch& b) {
    if (b.pinned) return EXPI_OK;
    BHIP(hipHostMalloc(reinterpret_cast<void**>(&b.pinned), 4 * sizeof(BatchCtrl), hipHostMallocDefault));
    for (auto& e : b.ev) BHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return EXPI_OK;
}

// Reset, then rounds in chunks until every instance has finished (or the
// round bound is reached).  The control block is read back after each
// chunk while the next chunk is already enqueued, so the device does not
// idle on the host's check.
int run_rounds(Batch& b, char* ws, const double* v, double* y, hipStream_t s) {
    int rc = ensure_pinned(b);
    if (rc) return rc;
    BatchArgs a = make_args(b, ws, v, y);
    hipLaunchKernelGGL(batch_reset_kernel, dim3((b.count + 255) / 256), dim3(256), 0, s,
                       a.state, a.ctrl, b.count);
    BHIP(hipGetLastError());
    int enq = 0, next = 0;
    std::deque<int> pending;
    bool done = false;
    while (!done) {
        if (enq < b.max_rounds) {
            const int cnt = std::min(kRoundChunk, b.max_rounds - enq);
            for (int q = 0; q < cnt; ++q) BHIP(enqueue_round(b, a, s));
            enq += cnt;
            const int slot = next++ & 3;
            BHIP(hipMemcpyAsync(&b.pinned[slot], a.ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, s));
            BHIP(hipEventRecord(b.ev[slot], s));
            pending.push_back(slot);
        }
        while (!pending.empty() && (pending.size() > 1 || enq >= b.max_rounds)) {
            const int slot = pending.front();
            pending.pop_front();
            BHIP(hipEventSynchronize(b.ev[slot]));
            if (b.pinned[slot].finished >= (unsigned)b.count) {
                b.last_rounds = (int)b.pinned[slot].rounds;
                done = true;
                break;
            }
        }
        if (pending.empty() && enq >= b.max_rounds) done = true;
    }
    BHIP(hipStreamSynchronize(s));
    return EXPI_OK;
}

// Graph of the reset and `rounds` rounds, built node by node as one chain.
int build_round_graph(Batch& b, char* ws, const double* v, double* y, int rounds) {
    BatchArgs a = make_args(b, ws, v, y);
    BatchState* st = a.state;
    BatchCtrl* ctrl = a.ctrl;
    int count = b.count;
    hipGraph_t g = nullptr;
    BHIP(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    void* p0[] = {&st, &ctrl, &count};
    hipKernelNodeParams k0{};
    k0.func = reinterpret_cast<void*>(batch_reset_kernel);
    k0.gridDim = dim3((b.count + 255) / 256);
    k0.blockDim = dim3(256);
    k0.kernelParams = p0;
    hipError_t e = hipGraphAddKernelNode(&prev, g, nullptr, 0, &k0);
    void* pa[] = {&a};
    hipKernelNodeParams kx{};
    kx.func = const_cast<void*>(tiles_kernel(b, false));
    kx.gridDim = dim3(b.round_grid);
    kx.blockDim = dim3(64 * b.waves);
    kx.sharedMemBytes = (unsigned)tiles_lds_bytes(b.count);
    kx.kernelParams = pa;
    hipKernelNodeParams kt = kx;
    kt.func = const_cast<void*>(tiles_kernel(b, true));
    hipKernelNodeParams kf{};
    kf.func = reinterpret_cast<void*>(batch_finalize_kernel);
    kf.gridDim = dim3(b.count);
    kf.blockDim = dim3(256);
    kf.kernelParams = pa;
    for (int r = 0; r < rounds && e == hipSuccess; ++r) {
        hipGraphNode_t nx = nullptr, nt = nullptr, nf = nullptr;
        e = hipGraphAddKernelNode(&nx, g, &prev, 1, &kx);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&nt, g, &nx, 1, &kt);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&nf, g, &nt, 1, &kf);
        prev = nf;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b.graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bfail(EXPI_EHIP, std::string("batched round graph: ") + hipGetErrorString(e));
    }
    b.graph = g;
    b.graph_rounds = rounds;
    return EXPI_OK;
}

// The same two launches as a graph built node by node, with the persistent
// kernel's node marked cooperative.
int build_graph(Batch& b, char* ws, const double* v, double* y) {
    BatchArgs a = make_args(b, ws, v, y);
    BatchState* st = a.state;
    BatchCtrl* ctrl = a.ctrl;
    int count = b.count;
    hipGraph_t g = nullptr;
    BHIP(hipGraphCreate(&g, 0));
    hipGraphNode_t n0 = nullptr, n1 = nullptr;
    void* p0[] = {&st, &ctrl, &count};
    hipKernelNodeParams k0{};
    k0.func = reinterpret_cast<void*>(batch_reset_kernel);
    k0.gridDim = dim3((b.count + 255) / 256);
    k0.blockDim = dim3(256);
    k0.kernelParams = p0;
    void* p1[] = {&a};
    hipKernelNodeParams k1{};
    k1.func = const_cast<void*>(kernel_ptr(b));
    k1.gridDim = dim3(b.grid);
    k1.blockDim = dim3(64 * kPersistWaves);
    k1.kernelParams = p1;
    hipKernelNodeAttrValue coop{};
    coop.cooperative = 1;
    hipError_t e = hipGraphAddKernelNode(&n0, g, nullptr, 0, &k0);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&n1, g, &n0, 1, &k1);
    if (e == hipSuccess) e = hipGraphKernelNodeSetAttribute(n1, hipKernelNodeAttributeCooperative, &coop);
    if (e == hipSuccess) e = hipGraphInstantiate(&b.graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bfail(EXPI_EHIP, std::string("batched graph: ") + hipGetErrorString(e));
    }
    b.graph = g;
    return EXPI_OK;
}

}  // namespace

}  // namespace expi

using namespace expi;

extern "C" {

int expi_batch_create(expi_batch** out, int count, const int32_t* nx, const int32_t* ny,
                      const double* hx, const double* hy, const double* tau, int bc, double coef,
                      double tol, int dtype, const expi_params* params) {
    if (!out) return bfail(EXPI_EINVAL, "batch is NULL");
    *out = nullptr;
    if (count < 1 || count > kMaxBatch) return bfail(EXPI_EINVAL, "count must be in [1, 4096]");
    if (!nx || !ny || !hx || !hy || !tau) return bfail(EXPI_EINVAL, "per-instance arrays must be non-NULL");
    if (bc != EXPI_DIRICHLET0 && bc != EXPI_NEUMANN0) return bfail(EXPI_EINVAL, "bc must be DIRICHLET0 or NEUMANN0");
    if (!(coef > 0) || !std::isfinite(coef)) return bfail(EXPI_EINVAL, "coef must be finite and > 0");
    if (!(tol > 0) || !std::isfinite(tol)) return bfail(EXPI_EINVAL, "tol must be finite and > 0");
    if (dtype != EXPI_F64 && dtype != EXPI_F32) return bfail(EXPI_EINVAL, "dtype must be EXPI_F64 or EXPI_F32");
    double l_max = 100.0;
    int m_max = 100;
    if (params) {
        l_max = params->l_max;
        m_max = params->m_max;
        if (params->have_interval) return bfail(EXPI_EINVAL, "batched intervals are computed per instance");
    }
    if (!(l_max > 0) || !std::isfinite(l_max)) return bfail(EXPI_EINVAL, "l_max must be finite and > 0");
    if (m_max < 2 || m_max >= kMaxLeja) return bfail(EXPI_EINVAL, "m_max must be in [2, 255]");
    Batch* b = new Batch();
    b->count = count;
    b->dtype = dtype;
    b->bc = bc;
    b->m_max = m_max;
    b->waves = 4;
    b->march = 8;
    b->c0 = coef;
    b->tol = tol;
    const int nd = m_max + 1;
    const double* xi = leja_points(nd);
    b->xi.assign(xi, xi + nd);
    b->dd.resize((size_t)count * nd);
    b->info.resize(count);
    long long off = 0;
    int max_sub = 1;
    for (int i = 0; i < count; ++i) {
        if (nx[i] < 1 || ny[i] < 1 || (long long)nx[i] * ny[i] >= (1ll << 28) ||
            !(hx[i] > 0) || !(hy[i] > 0) || !std::isfinite(hx[i]) || !std::isfinite(hy[i]) ||
            !(tau[i] >= 0) || !std::isfinite(tau[i])) {
            delete b;
            return bfail(EXPI_EINVAL, "instance " + std::to_string(i) + ": bad size, spacing or tau");
        }
        BatchInfo& I = b->info[i];
        I.off = off;
        off += ((long long)nx[i] * ny[i] + 31) / 32 * 32;   // 256-byte aligned starts
        I.nx = nx[i];
        I.ny = ny[i];
        I.vec = (nx[i] % 2 == 0) ? 2 : 1;
        I.ihx = 1.0 / (hx[i] * hx[i]);
        I.ihy = 1.0 / (hy[i] * hy[i]);
        // Gershgorin bound of the constant-coefficient 5-point operator with the
        // boundary folded in: every row lies in [-4 coef (1/hx^2 + 1/hy^2), 0]
        const double a = -4.0 * coef * (I.ihx + I.ihy), bb = 0.0;
        const double c = 0.5 * (a + bb), gamma = 0.25 * (bb - a);
        double q = std::ceil(tau[i] * (bb - a) / l_max);
        const int s = q < 1.0 ? 1 : (int)q;
        I.s = s;
        max_sub = std::max(max_sub, s);
        I.alpha = 1.0 / gamma;
        I.cg = c / gamma;
        I.tau = tau[i];
        I.inv_s = 1.0 / s;
        I.dd_off = i * nd;
        divided_differences(1, tau[i] / s, c, gamma, nd, &b->dd[(size_t)i * nd]);
    }
    b->total_len = off;
    // each substep: start, first, at most m_max - 1 products, update
    b->max_rounds = max_sub * (m_max + 2) + 2;
    layout_tiles(*b);
    *out = reinterpret_cast<expi_batch*>(b);
    return EXPI_OK;
}

int expi_batch_destroy(expi_batch* bp) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (b) {
        if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        for (auto& e : b->ev)
            if (e) (void)hipEventDestroy(e);
        if (b->pinned) (void)hipHostFree(b->pinned);
        delete b;
    }
    return EXPI_OK;
}

int expi_batch_set_tiles(expi_batch* bp, int waves, int march) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (!b) return bfail(EXPI_EINVAL, "batch is NULL");
    if (waves < 1 || waves > kMaxWaves || march < 4 || march > 64 || march % 4)
        return bfail(EXPI_EINVAL, "waves in [1, 8], march in {4, 8, ..., 64}");
    if (b->graph_exec) return bfail(EXPI_EINVAL, "tiles cannot change after a graph was captured");
    b->waves = waves;
    b->march = march;
    const size_t keep = b->ws_total;
    layout_tiles(*b);
    b->ws_total = keep > b->ws_total ? keep : b->ws_total;
    b->prepared_ws = nullptr;
    return EXPI_OK;
}

int64_t expi_batch_total_length(const expi_batch* bp) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    return b ? b->total_len : -1;
}

int expi_batch_offsets(const expi_batch* bp, int64_t* off) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    if (!b || !off) return bfail(EXPI_EINVAL, "NULL argument");
    for (int i = 0; i < b->count; ++i) off[i] = b->info[i].off;
    return EXPI_OK;
}

size_t expi_batch_workspace_bytes(const expi_batch* bp) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    return b ? b->ws_total : 0;
}

int expi_batch_prepare(expi_batch* bp, void* ws, size_t ws_bytes, void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (!b || !ws) return bfail(EXPI_EINVAL, "batch and ws must be non-NULL");
    if (((uintptr_t)ws & 255) != 0) return bfail(EXPI_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < b->ws_total) return bfail(EXPI_EWORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    BHIP(hipMemcpyAsync(w + b->off_info, b->info.data(), sizeof(BatchInfo) * b->count,
                        hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(w + b->off_dd, b->dd.data(), sizeof(double) * b->dd.size(),
                        hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(w + b->off_xi, b->xi.data(), sizeof(double) * b->xi.size(),
                        hipMemcpyHostToDevice, s));
    // the grid barrier's generation and flags start at zero once; launches
    // then only move them forward
    BHIP(hipMemsetAsync(w + b->off_ctrl, 0, b->off_info - b->off_ctrl, s));
    BHIP(hipStreamSynchronize(s));
    int rc = occupancy_grid(*b);
    if (rc) return rc;
    b->prepared_ws = ws;
    return EXPI_OK;
}

static int check_run_args(Batch* b, const double* v, double* y, void* ws, size_t ws_bytes) {
    if (!b || !v || !y || !ws) return bfail(EXPI_EINVAL, "NULL argument");
    if (ws != b->prepared_ws) return bfail(EXPI_EINVAL, "call expi_batch_prepare with this workspace first");
    if (ws_bytes < b->ws_total) return bfail(EXPI_EWORKSPACE, "workspace too small");
    const size_t vb = (size_t)b->total_len * 8;
    const char* pv = reinterpret_cast<const char*>(v);
    const char* py = reinterpret_cast<const char*>(y);
    if (pv < py + vb && py < pv + vb) return bfail(EXPI_EALIAS, "y overlaps v");
    if (((uintptr_t)v & 15) != 0 || ((uintptr_t)y & 15) != 0)
        return bfail(EXPI_EINVAL, "v and y must be 16-byte aligned");
    return EXPI_OK;
}

static void drop_graph(Batch* b) {
    if (b->graph_exec) {
        (void)hipGraphExecDestroy(b->graph_exec);
        b->graph_exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_rounds = 0;
}

int expi_batch_launch(expi_batch* bp, const double* v, double* y, void* ws, size_t ws_bytes,
                      void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    int rc = check_run_args(b, v, y, ws, ws_bytes);
    if (rc) return rc;
    return run_rounds(*b, static_cast<char*>(ws), v, y, static_cast<hipStream_t>(stream));
}

int expi_batch_capture(expi_batch* bp, const double* v, double* y, void* ws, size_t ws_bytes,
                       int rounds, void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    int rc = check_run_args(b, v, y, ws, ws_bytes);
    if (rc) return rc;
    if (rounds < 0) return bfail(EXPI_EINVAL, "rounds must be >= 0");
    if (rounds == 0) {
        // the rounds the last eager solve needed, with a margin of 1/64 + 8
        // (the same inputs need exactly as many); else the bound
        rounds = b->last_rounds > 0 ? b->last_rounds + b->last_rounds / 64 + 8 : b->max_rounds;
    }
    if (rounds > b->max_rounds) rounds = b->max_rounds;
    (void)stream;
    drop_graph(b);
    return build_round_graph(*b, static_cast<char*>(ws), v, y, rounds);
}

int expi_batch_replay(expi_batch* bp, void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (!b || !b->graph_exec) return bfail(EXPI_EINVAL, "no captured graph");
    BHIP(hipGraphLaunch(b->graph_exec, static_cast<hipStream_t>(stream)));
    return EXPI_OK;
}

int expi_batch_graph_rounds(const expi_batch* bp) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    return b ? b->graph_rounds : -1;
}

int expi_batch_max_rounds(const expi_batch* bp) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    return b ? b->max_rounds : -1;
}

int expi_batch_autotune(expi_batch* bp, const double* v, double* y, void* ws, size_t ws_bytes,
                        int reps, void* stream, int* cand, float* ms, int max_cand, int* n_cand) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (!b || !v || !y || !ws || !n_cand) return bfail(EXPI_EINVAL, "NULL argument");
    if (reps < 1 || reps > 100) return bfail(EXPI_EINVAL, "reps must be in [1, 100]");
    if (ws_bytes < b->ws_total) return bfail(EXPI_EWORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    drop_graph(b);
    const int waves_c[] = {2, 4, 8};
    const int march_c[] = {4, 8, 16, 32};
    int best_w = b->waves, best_m = b->march, n = 0;
    double best = 1e300;
    for (int wv : waves_c) {
        for (int mc : march_c) {
            int rc = expi_batch_set_tiles(bp, wv, mc);
            if (rc == EXPI_OK) rc = expi_batch_prepare(bp, ws, ws_bytes, stream);
            if (rc == EXPI_OK) rc = check_run_args(b, v, y, ws, ws_bytes);
            if (rc == EXPI_OK) rc = run_rounds(*b, static_cast<char*>(ws), v, y, s);   // warm-up
            if (rc) return rc;
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < reps && rc == EXPI_OK; ++r) rc = run_rounds(*b, static_cast<char*>(ws), v, y, s);
            if (rc) return rc;
            const double t = std::chrono::duration<double, std::milli>(
                                 std::chrono::steady_clock::now() - t0).count() / reps;
            if (cand && ms && n < max_cand) {
                cand[2 * n] = wv;
                cand[2 * n + 1] = mc;
                ms[n] = (float)t;
            }
            ++n;
            if (t < best) {
                best = t;
                best_w = wv;
                best_m = mc;
            }
        }
    }
    *n_cand = n;
    int rc = expi_batch_set_tiles(bp, best_w, best_m);
    if (rc == EXPI_OK) rc = expi_batch_prepare(bp, ws, ws_bytes, stream);
    return rc;
}

int expi_batch_set_pairs(expi_batch* bp, int on) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (!b) return bfail(EXPI_EINVAL, "batch is NULL");
    if (on != 0 && on != 1) return bfail(EXPI_EINVAL, "on must be 0 or 1");
    if (b->graph_exec) return bfail(EXPI_EINVAL, "the product setting cannot change after a graph was captured");
    b->pairs = on;
    return EXPI_OK;
}

int expi_batch_get_pairs(const expi_batch* bp, int* on) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    if (!b || !on) return bfail(EXPI_EINVAL, "NULL argument");
    *on = b->pairs;
    return EXPI_OK;
}

int expi_batch_get_tiles(const expi_batch* bp, int* waves, int* march) {
    const Batch* b = reinterpret_cast<const Batch*>(bp);
    if (!b || !waves || !march) return bfail(EXPI_EINVAL, "NULL argument");
    *waves = b->waves;
    *march = b->march;
    return EXPI_OK;
}

int expi_batch_launch_persistent(expi_batch* bp, const double* v, double* y, void* ws,
                                 size_t ws_bytes, void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    int rc = check_run_args(b, v, y, ws, ws_bytes);
    if (rc) return rc;
    return enqueue(*b, static_cast<char*>(ws), v, y, static_cast<hipStream_t>(stream));
}

int expi_batch_capture_persistent(expi_batch* bp, const double* v, double* y, void* ws,
                                  size_t ws_bytes, void* stream) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    int rc = check_run_args(b, v, y, ws, ws_bytes);
    if (rc) return rc;
    (void)stream;
    drop_graph(b);
    return build_graph(*b, static_cast<char*>(ws), v, y);
}

int expi_batch_results(expi_batch* bp, void* ws, void* stream, expi_batch_stat* out,
                       int* rounds) {
    Batch* b = reinterpret_cast<Batch*>(bp);
    if (!b || !ws) return bfail(EXPI_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<BatchState> st(b->count);
    BatchCtrl ctrl;
    char* w = static_cast<char*>(ws);
    BHIP(hipMemcpyAsync(st.data(), w + b->off_state, sizeof(BatchState) * b->count,
                        hipMemcpyDeviceToHost, s));
    BHIP(hipMemcpyAsync(&ctrl, w + b->off_ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    if (rounds) *rounds = (int)ctrl.rounds;
    int worst = EXPI_OK;
    for (int i = 0; i < b->count; ++i) {
        if (out) {
            out[i].status = st[i].phase == PH_DONE ? 0 : (st[i].status == 2 ? EXPI_ENONFINITE : EXPI_ENOTCONV);
            out[i].substeps = b->info[i].s;
            out[i].newton_steps = st[i].newton;
            out[i].degree_max = st[i].degree_max;
            out[i].degree_last = st[i].degree_last;
            out[i].reserved = 0;
            out[i].err_est = st[i].err_max;
        }
        if (st[i].phase != PH_DONE) worst = (st[i].status == 2) ? EXPI_ENONFINITE : EXPI_ENOTCONV;
    }
    if (ctrl.abort)
        return bfail(EXPI_EHIP, "persistent batched kernel aborted: a grid barrier wait passed its time limit");
    if (worst == EXPI_ENOTCONV)
        return bfail(worst, "some instances did not converge within m_max or did not finish in the rounds run");
    if (worst == EXPI_ENONFINITE) return bfail(worst, "some instances became non-finite");
    return EXPI_OK;
}

}  // extern "C"
