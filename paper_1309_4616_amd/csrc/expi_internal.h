// Internal declarations shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/expi.h"

namespace expi {

constexpr int kHist = 5;         // Newton-term norms t_0..t_4 kept per loop
constexpr int kMaxPairWaves = 16;   // waves of a pair-sweep workgroup

// ---------------------------------------------------------------------------
// Device-side status of one Newton loop (lives at the start of the workspace).
// Written by the finalize kernel after each reducing sweep; read back by the host.
// ---------------------------------------------------------------------------
struct alignas(64) NewtonState {
    unsigned int arrive;  // reserved
    int done;             // 0 running, 1 stop test met, 2 non-finite norm
    int m;                // products taken in this loop
    int fixbuf;           // with fix: which of the two w buffers holds w_{m+1}
    double t_prev;        // |d_m| ||w_m|| of the latest product
    double err;           // (t_{m-1} + t_m) / ||p|| at the latest test
    double pnorm;         // ||p||
    double wnorm;         // ||w_m||
    double gmin, gmax;    // Gershgorin reduction result
    double hist[kHist];   // t_0 .. t_4 of this loop (features of the step selector)
    double rnorm;         // ||r|| of the loop's start vector
    int pred_m;           // step selector's predicted Newton degree
    int pred_s;           // step selector's predicted substep count
    double fix;           // pair sweep met the test at its first product: d_{m+1},
                          // whose term d_{m+1} w_{m+1} p holds one too many; else 0
};
static_assert(sizeof(NewtonState) == 128, "status record is 128 bytes");

// Epilogues of the fused sweep.
enum Epilogue : int {
    EPI_APPLY = 0,   // y = alpha A x + beta x
    EPI_NEWTON = 1,  // w' = alpha A w + beta w; p += d1 w'; norms; stop test
    EPI_FIRST = 2,   // w' = alpha A w + beta w; p = d0 w + d1 w'; norms
    EPI_START = 3,   // r = sigma A x + g
    EPI_GERSH = 4,   // per-row Gershgorin bounds, min/max over rows
};

// Source of g in EPI_START: the vector g (G_VEC), gscale times it
// (G_VEC_SCALED), or the nonlinearity of kind gkind (EXPI_G_*) of the vector
// g (G_CUBIC_OF) or of the input x itself (G_CUBIC_SELF).
enum GMode : int { G_VEC = 0, G_CUBIC_OF = 1, G_CUBIC_SELF = 2, G_VEC_SCALED = 3 };

struct SweepArgs {
    const void* x;        // input vector (stencil source)
    void* out;            // w_{j+1}, y or r
    void* p;              // running Newton sum
    const double* g;      // EPI_START: v (G_VEC) or u_n (G_CUBIC_OF)
    const double* tx;     // separable coefficient tables
    const double* ty;
    const double* tz;
    const double* field;  // coefficient field
    double* partials;     // [gridDim.x][4]
    NewtonState* st;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* val;
    double c0, c1;
    double ih2[3];        // 1/h_d^2
    double hpos[3];       // h_d (grid positions of EXPI_COEF_DLAP and boundary data)
    double alpha, beta, d0, d1, sigma, tol;
    double d0i, d1i, sigmai;   // imaginary parts (complex CSR operators)
    int n[3];             // grid sizes (x, y, z); CSR: n[0] = rows
    int nnz;              // CSR stored entries
    int bc;
    int j;                // Newton index of this product
    int guard;            // 1: the sweep does nothing once st->done != 0
    int gmode;
    int gkind;            // EPI_START: nonlinearity (EXPI_G_*) of G_CUBIC_OF/SELF
    int bdata;            // EPI_APPLY / EPI_START: add the boundary term of the
                          // operator's Dirichlet data (EXPI_BDATA_*), 0: none
    double gscale;        // EPI_START: factor of g under G_VEC_SCALED
    int tiles[3];
    int ntiles;
    int per_xcd;          // tiles per XCD slot
    int march;            // points marched per thread (stencils)
};

// Arguments of the pair sweep (two Newton products in one pass, pair.hip).
// What a pair sweep computes (see pair.hip):
//   PAIR_NEWTON  products j and j+1 from w_j and p_j;
//   PAIR_FIRST   products 0 and 1 from the start vector r = w_0 (no p in);
//   PAIR_START   the start vector r = sigma A u + u - u^3 of an Euler step
//                (on chip only) and product 0: w_1 and p_1 = d_0 r + d_1 w_1.
enum PairMode : int { PAIR_NEWTON = 0, PAIR_FIRST = 1, PAIR_START = 2 };

struct PairArgs {
    const void* x;        // w_j
    void* out;            // w_{j+2}
    void* p;              // running Newton sum, p_j in, p_{j+2} out
    const double* tx;     // separable coefficient tables
    const double* ty;
    const double* tz;
    double* partials;     // [grid][4]: ||w_{j+1}||^2, ||p_{j+1}||^2, ||w_{j+2}||^2, ||p_{j+2}||^2
    NewtonState* st;
    double ih2[3];
    double c0ih[3], c1ih[3];   // c0 / h_d^2, c1 / h_d^2 (coefficient c0 + c1 X Y Z)
    double alpha, beta1, beta2, d1, d2, tol;   // beta_j, beta_{j+1}, d_{j+1}, d_{j+2}
    double d0;            // PAIR_FIRST: d_0 (p_1 = d_0 r + d_1 w_1)
    double sigma;         // PAIR_START: r = sigma A u + u - u^3 (then beta2 = beta_0,
                          // d1 = d_0, d2 = d_1, j = -1)
    int n[3];
    int bc;
    int guard;
    int outbuf;           // index of `out` among the loop's two w buffers (stop tests record it)
    int j;
    int nxw;              // waves per grid row (1 or 2)
    int rows;             // output rows per row tile
    int nrt;              // row tiles
    int chunk;            // (row tile, plane) units per workgroup
    int per_xcd;
};

struct PairGeom {
    int nxw, rows, nrt, chunk, grid, per_xcd;
};

// Arguments of the one-workgroup finalize kernel that follows a reducing sweep.
struct FinalArgs {
    const double* partials;
    NewtonState* st;
    int nparts;
    int j;
    int guard;
    int mode;             // pair sweeps: PairMode (PAIR_FIRST: 5 partials, stride 8)
    int outbuf;           // pair sweeps: index of the w buffer the sweep writes
    double d0, d1, tol;
    double d2;            // pair sweeps: d_{j+2}
    NewtonState* mirror;  // device address of a host copy of the state, written
                          // after the tests (null: none)
};

// Host copy of the state that the finalize kernels enqueued next by this
// host thread write after their tests (null: none).  The host sets it around
// a batch of launches and reads the copy after an event that follows them,
// which takes the place of a device-to-host copy of the record.
void set_state_mirror(NewtonState* mirror);

// Step-selector network (mlp.hip): predicted (substeps, degree) from the
// interval, tau, ||r|| and t_0..t_4 in `st`; written to st->pred_s/pred_m.
// `features` (device float[8], may be null) receives the raw features.
hipError_t launch_selector(const float* sel, int hidden, NewtonState* st, double a, double b,
                           double tau, int m_max, float* features, hipStream_t s);

// Tile setting of an operator's sweeps (chosen by default or by the tuner).
//   stencil: vec = x points per thread (1 or 2), waves per workgroup,
//            march = points marched per thread along the slowest axis;
//   CSR:     vec = lanes per row (4, 8, 16), waves per workgroup, march = 1.
struct Tiles {
    int vec = 2;
    int waves = 4;
    int march = 16;
};

// Launch geometry derived from a tile setting.
struct Geom {
    int vec, waves, march;
    int tiles[3];
    int ntiles;
    int per_xcd;
    int grid;             // workgroups launched (multiple of 8)
};

struct Op {
    int kind;             // 0 stencil, 1 CSR, 2 complex CSR (val: complex128 pairs)
    int dim;
    int n[3];
    double h[3];
    int bc;
    int coef;
    double c0, c1;
    const double *tx, *ty, *tz, *field;
    int64_t nrows, nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* val;
    int64_t size;
    Tiles tiles;
    int bdata = 0;        // EXPI_BDATA_* of a 3D Dirichlet stencil
    int bdata_mode = 0;   // EXPI_BDATA_IN_KERNEL or EXPI_BDATA_SEPARATE
    int use_pairs = 1;    // pair sweeps where supported (the autotuner may turn them off)
    std::mutex mu;
    bool have_interval = false;
    double ia = 0, ib = 0;
    // divided differences keyed by (k, delta, c, gamma, count)
    std::map<std::tuple<int, double, double, double, int>, std::vector<double>> dd_cache;
    // Newton degree last seen for a key, used to size the first chunk
    std::map<std::tuple<int, double, double, double, int>, int> degree_hint;
};

constexpr int kXcd = 8;          // XCDs of gfx950; workgroup b runs on XCD b % 8
constexpr int kMaxWaves = 8;     // waves per workgroup at most (512 threads)
constexpr int kFinalThreads = 256;   // threads of a finalize workgroup
constexpr int kMinMarch = 4;     // accepted march lengths of a stencil sweep (multiples of 4)
constexpr int kMaxMarch = 120;  // the marched-axis table of a separable coefficient holds 128 planes
constexpr int kCsrGrid = 2048;   // workgroups of a CSR sweep at most (grid-stride over row blocks)

Geom make_geom(const Op& op, const Tiles& t);
Tiles default_tiles(const Op& op);
bool tiles_valid(const Op& op, const Tiles& t);
size_t partials_bytes(const Op& op);

// Launchers.  TIN/TOUT codes: 0 = double, 1 = float.  launch_sweep picks the
// geometry from op.tiles and adds the finalize kernel after reducing sweeps.
// `after_sweep`, if given, is recorded on `s` between the sweep and its
// finalize kernel (profiling of the sweep alone).
hipError_t launch_sweep(const Op& op, int epi, int tin, int tout, SweepArgs a,
                        hipStream_t s, hipEvent_t after_sweep = nullptr,
                        bool finalize = true);
hipError_t launch_stencil(const Op& op, const Geom& g, int epi, int tin, int tout,
                          const SweepArgs& a, hipStream_t s);
hipError_t launch_csr(const Geom& g, int epi, int tin, int tout, const SweepArgs& a,
                      hipStream_t s);
// Complex CSR (csr_complex.hip): complex128 vectors, real alpha/beta,
// complex d0, d1 (d0i, d1i) and sigma (sigmai).
hipError_t launch_csr_complex(const Geom& g, int epi, const SweepArgs& a, hipStream_t s);
hipError_t launch_update(int64_t n, double* out, const double* yin, const void* p, int tp,
                         double scale, const NewtonState* st, int guard, hipStream_t s,
                         const void* wfix = nullptr, double fix = 0.0);
// The same update with the correction taken from the device: runs only if
// st->done == 1, and subtracts st->fix * w (w = w1 if st->fixbuf, else w0)
// when st->fix is nonzero.  Lets the host enqueue the update before it has
// read the loop's status.
hipError_t launch_update_st(int64_t n, double* out, const double* yin, const void* p, int tp,
                            double scale, const NewtonState* st, const void* w0, const void* w1,
                            hipStream_t s);
hipError_t launch_reset(NewtonState* st, hipStream_t s);

// Pair sweeps: two Newton products in one pass (pair.hip), then a finalize
// kernel that applies the stop test after each of them.
bool pair_supported(const Op& op, int tw);
// pair sweeps are supported and the operator's setting allows them
inline bool pairs_enabled(const Op& op, int tw) { return op.use_pairs != 0 && pair_supported(op, tw); }
bool pair_start_supported(const Op& op);
PairGeom pair_geom(const Op& op, int cus);
// `mode` (PairMode): PAIR_FIRST starts the loop from r = w_0 (products 0
// and 1; the finalize records t_0, t_1 and ||r|| before its stop test at
// m = 2); PAIR_START forms r itself (in FP64 from the FP64 u) and takes product 0
// (the finalize records t_0, t_1 and ||r||, and cannot stop at m = 1).
hipError_t launch_pair(const Op& op, int tw, PairArgs a, hipStream_t s,
                       hipEvent_t after_sweep = nullptr, bool finalize = true,
                       int mode = PAIR_NEWTON);
hipError_t launch_pair_finalize(const double* partials, NewtonState* st, int nparts, int j,
                                int guard, double d0, double d1, double d2, double tol, int mode,
                                int outbuf, hipStream_t s);
hipError_t launch_fill(void* out, int64_t n, int t, double scale, hipStream_t s);
// The boundary term of a stencil's Dirichlet data over its boundary layer
// (boundary.hip): y += scale * b_f, y of storage code t.
hipError_t launch_boundary(const Op& op, double scale, void* y, int t, hipStream_t s);
// Pointwise nonlinearity g = kind(u) over n values of dtype (nonlin.hip), and
// out = kind(U) - kind(u) in float64.
hipError_t launch_nonlin(int kind, int64_t n, const void* u, void* g, int dtype, hipStream_t s);
hipError_t launch_gdiff(int kind, int64_t n, const double* U, const double* u, double* out,
                        hipStream_t s);

// Error reporting (api.hip).
void set_error(const std::string& msg);

}  // namespace expi
