// Step-selector network: forward, backward and Adam kernels (float32), and
// the on-device selector that predicts the Newton degree of a Leja loop.
//
// Network: x (8) -> relu(W1 x + b1) (H) -> relu(W2 h1 + b2) (H) -> W3 h2 + b3
// (2 outputs: log2 of the substep count and the Newton degree).  Parameters
// are packed in one float array: W1 (H x 8, row-major), b1 (H), W2 (H x H),
// b2 (H), W3 (2 x H), b3 (2); H^2 + 12 H + 2 values.
//
// Loss (asymmetric squared error, weight kappa where the output is below its
// target, since under-predicting the degree costs a fallback):
//   L = 1/(2n) sum_samples sum_outputs w (o - t)^2.
// Gradients are reduced over samples in index order (deterministic).
// Adam (Kingma & Ba) with bias-corrected moments.
//
// Sizes here are tiny (thousands of parameters, about a thousand samples),
// so each kernel uses one thread per output value or per parameter.
#include <cmath>
#include <string>

#include "expi_internal.h"

namespace expi {
namespace {

constexpr int kIn = 8;
constexpr int kOut = 2;
constexpr int kMaxHidden = 256;

struct Offs {
    int w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Offs offs(int H) {
    Offs o;
    o.w1 = 0;
    o.b1 = o.w1 + H * kIn;
    o.w2 = o.b1 + H;
    o.b2 = o.w2 + H * H;
    o.w3 = o.b2 + H;
    o.b3 = o.w3 + kOut * H;
    o.total = o.b3 + kOut;
    return o;
}

// Forward pass of one sample held in LDS; every thread t < H takes part.
__device__ void mlp_forward_one(const float* __restrict__ P, int H, const float* x, float* h1,
                                float* h2, float* o, float* z1_out, float* z2_out) {
    const Offs of = offs(H);
    const int t = threadIdx.x;
    if (t < H) {
        float z = P[of.b1 + t];
        for (int k = 0; k < kIn; ++k) z += P[of.w1 + t * kIn + k] * x[k];
        if (z1_out) z1_out[t] = z;
        h1[t] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    if (t < H) {
        float z = P[of.b2 + t];
        for (int k = 0; k < H; ++k) z += P[of.w2 + t * H + k] * h1[k];
        if (z2_out) z2_out[t] = z;
        h2[t] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    if (t < kOut) {
        float z = P[of.b3 + t];
        for (int k = 0; k < H; ++k) z += P[of.w3 + t * H + k] * h2[k];
        o[t] = z;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kMaxHidden) void mlp_forward_kernel(const float* __restrict__ P, int H,
                                                                 const float* __restrict__ X, int n,
                                                                 float* __restrict__ out,
                                                                 float* __restrict__ act) {
    __shared__ float x[kIn], h1[kMaxHidden], h2[kMaxHidden], o[kOut];
    const int s = blockIdx.x;
    if (s >= n) return;
    if (threadIdx.x < kIn) x[threadIdx.x] = X[(size_t)s * kIn + threadIdx.x];
    __syncthreads();
    float* z1 = act ? act + (size_t)s * 2 * H : nullptr;
    float* z2 = act ? act + (size_t)s * 2 * H + H : nullptr;
    mlp_forward_one(P, H, x, h1, h2, o, z1, z2);
    if (threadIdx.x < kOut) out[(size_t)s * kOut + threadIdx.x] = o[threadIdx.x];
}

// Per-sample deltas: dz1 (H), dz2 (H), do (2) and the sample's loss term.
__global__ __launch_bounds__(kMaxHidden) void mlp_delta_kernel(const float* __restrict__ P, int H,
                                                               const float* __restrict__ act,
                                                               const float* __restrict__ out,
                                                               const float* __restrict__ T, int n,
                                                               float kappa, float* __restrict__ D,
                                                               float* __restrict__ lossv) {
    __shared__ float d_o[kOut], dz2[kMaxHidden];
    const Offs of = offs(H);
    const int s = blockIdx.x, t = threadIdx.x;
    if (s >= n) return;
    const float* z1 = act + (size_t)s * 2 * H;
    const float* z2 = z1 + H;
    float* Ds = D + (size_t)s * (2 * H + kOut);
    if (t < kOut) {
        const float oo = out[(size_t)s * kOut + t], tt = T[(size_t)s * kOut + t];
        const float w = oo < tt ? kappa : 1.f;
        d_o[t] = w * (oo - tt) / (float)n;
        Ds[2 * H + t] = d_o[t];
    }
    if (t == 0) {
        float l = 0.f;
        for (int c = 0; c < kOut; ++c) {
            const float oo = out[(size_t)s * kOut + c], tt = T[(size_t)s * kOut + c];
            const float w = oo < tt ? kappa : 1.f;
            l += w * (oo - tt) * (oo - tt);
        }
        lossv[s] = 0.5f * l;
    }
    __syncthreads();
    if (t < H) {
        float g = 0.f;
        for (int c = 0; c < kOut; ++c) g += d_o[c] * P[of.w3 + c * H + t];
        dz2[t] = z2[t] > 0.f ? g : 0.f;
        Ds[H + t] = dz2[t];
    }
    __syncthreads();
    if (t < H) {
        float g = 0.f;
        for (int j = 0; j < H; ++j) g += dz2[j] * P[of.w2 + j * H + t];
        Ds[t] = z1[t] > 0.f ? g : 0.f;
    }
}

// Gradient of every parameter: a sum over samples in index order.
__global__ __launch_bounds__(256) void mlp_grad_kernel(int H, const float* __restrict__ X,
                                                       const float* __restrict__ act,
                                                       const float* __restrict__ D, int n,
                                                       const float* __restrict__ lossv,
                                                       float* __restrict__ G,
                                                       float* __restrict__ loss) {
    const Offs of = offs(H);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int DS = 2 * H + kOut;
    if (q < of.total) {
        float g = 0.f;
        if (q < of.b1) {                       // W1[h][k] = sum dz1[h] x[k]
            const int h = q / kIn, k = q % kIn;
            for (int s = 0; s < n; ++s) g += D[(size_t)s * DS + h] * X[(size_t)s * kIn + k];
        } else if (q < of.w2) {                // b1[h]
            const int h = q - of.b1;
            for (int s = 0; s < n; ++s) g += D[(size_t)s * DS + h];
        } else if (q < of.b2) {                // W2[h][k] = sum dz2[h] relu(z1[k])
            const int h = (q - of.w2) / H, k = (q - of.w2) % H;
            for (int s = 0; s < n; ++s) {
                const float z = act[(size_t)s * 2 * H + k];
                g += D[(size_t)s * DS + H + h] * (z > 0.f ? z : 0.f);
            }
        } else if (q < of.w3) {                // b2[h]
            const int h = q - of.b2;
            for (int s = 0; s < n; ++s) g += D[(size_t)s * DS + H + h];
        } else if (q < of.b3) {                // W3[c][k] = sum do[c] relu(z2[k])
            const int c = (q - of.w3) / H, k = (q - of.w3) % H;
            for (int s = 0; s < n; ++s) {
                const float z = act[(size_t)s * 2 * H + H + k];
                g += D[(size_t)s * DS + 2 * H + c] * (z > 0.f ? z : 0.f);
            }
        } else {                               // b3[c]
            const int c = q - of.b3;
            for (int s = 0; s < n; ++s) g += D[(size_t)s * DS + 2 * H + c];
        }
        G[q] = g;
    }
    if (q == 0 && loss) {
        float l = 0.f;
        for (int s = 0; s < n; ++s) l += lossv[s];
        *loss = l / (float)n;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(int count, float* __restrict__ P,
                                                   const float* __restrict__ G,
                                                   float* __restrict__ M, float* __restrict__ V,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const float g = G[q];
    const float m = b1 * M[q] + (1.f - b1) * g;
    const float v = b2 * V[q] + (1.f - b2) * g * g;
    M[q] = m;
    V[q] = v;
    P[q] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Selector buffer: x_mean[8], x_std[8], y_mean[2], y_std[2], then the
// network parameters.  Features of a Newton loop (after its first four
// products): log10 tau(b-a), tau b, log10 tau, log10 ||r||, and
// log10(t_k / t_0) for k = 1..4.
__global__ __launch_bounds__(kMaxHidden) void selector_kernel(const float* __restrict__ sel, int H,
                                                              NewtonState* st, double a, double b,
                                                              double tau, int m_max, float* feat) {
    __shared__ float x[kIn], h1[kMaxHidden], h2[kMaxHidden], o[kOut];
    if (threadIdx.x == 0) {
        double f[kIn];
        f[0] = log10(fmax(tau * (b - a), 1e-300));
        f[1] = tau * b;
        f[2] = log10(fmax(tau, 1e-300));
        f[3] = log10(st->rnorm + 1e-300);
        const double t0 = st->hist[0];
        for (int k = 1; k <= 4; ++k) f[3 + k] = t0 > 0.0 ? log10(st->hist[k] / t0 + 1e-300) : -300.0;
        for (int k = 0; k < kIn; ++k) x[k] = (float)((f[k] - sel[k]) / sel[kIn + k]);
        if (feat)
            for (int k = 0; k < kIn; ++k) feat[k] = (float)f[k];
    }
    __syncthreads();
    mlp_forward_one(sel + 2 * kIn + 2 * kOut, H, x, h1, h2, o, nullptr, nullptr);
    if (threadIdx.x == 0) {
        const float ys = o[0] * sel[2 * kIn + kOut] + sel[2 * kIn];
        const float ym = o[1] * sel[2 * kIn + kOut + 1] + sel[2 * kIn + 1];
        const float sp = exp2f(fminf(fmaxf(ys, 0.f), 20.f));
        st->pred_s = max(1, (int)lrintf(sp));
        int m = (int)ceilf(ym);
        st->pred_m = min(max(m, 2), m_max);
    }
}

}  // namespace

hipError_t launch_selector(const float* sel, int hidden, NewtonState* st, double a, double b,
                           double tau, int m_max, float* features, hipStream_t s) {
    hipLaunchKernelGGL(selector_kernel, dim3(1), dim3(kMaxHidden), 0, s, sel, hidden, st, a, b,
                       tau, m_max, features);
    return hipGetLastError();
}

}  // namespace expi

using namespace expi;

namespace {
int mfail(int code, const char* m) {
    set_error(m);
    return code;
}
}  // namespace

extern "C" {

size_t expi_mlp_param_count(int hidden) {
    if (hidden < 1 || hidden > kMaxHidden) return 0;
    return (size_t)offs(hidden).total;
}

int expi_mlp_forward(int hidden, const float* params, const float* x, int n, float* out, float* act,
                     void* stream) {
    if (hidden < 1 || hidden > kMaxHidden) return mfail(EXPI_EINVAL, "hidden must be in [1, 256]");
    if (!params || !x || !out || n < 0) return mfail(EXPI_EINVAL, "NULL argument or n < 0");
    if (n == 0) return EXPI_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(n), dim3(kMaxHidden), 0,
                       static_cast<hipStream_t>(stream), params, hidden, x, n, out, act);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(EXPI_EHIP, hipGetErrorString(e));
    return EXPI_OK;
}

int expi_mlp_backward(int hidden, const float* params, const float* x, const float* act,
                      const float* out, const float* target, int n, float kappa, float* grad,
                      float* loss, float* scratch, void* stream) {
    if (hidden < 1 || hidden > kMaxHidden) return mfail(EXPI_EINVAL, "hidden must be in [1, 256]");
    if (!params || !x || !act || !out || !target || !grad || !scratch || n < 1)
        return mfail(EXPI_EINVAL, "NULL argument or n < 1");
    if (!(kappa > 0.f)) return mfail(EXPI_EINVAL, "kappa must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* D = scratch;
    float* lossv = scratch + (size_t)n * (2 * hidden + kOut);
    hipLaunchKernelGGL(mlp_delta_kernel, dim3(n), dim3(kMaxHidden), 0, s, params, hidden, act, out,
                       target, n, kappa, D, lossv);
    const int P = offs(hidden).total;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((P + 255) / 256), dim3(256), 0, s, hidden, x, act, D, n,
                       lossv, grad, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(EXPI_EHIP, hipGetErrorString(e));
    return EXPI_OK;
}

size_t expi_mlp_scratch_floats(int hidden, int n) {
    if (hidden < 1 || hidden > kMaxHidden || n < 0) return 0;
    return (size_t)n * (2 * hidden + kOut) + (size_t)n;
}

int expi_mlp_adam(int count, float* params, const float* grad, float* m, float* v, int step,
                  float lr, float beta1, float beta2, float eps, void* stream) {
    if (count < 1 || !params || !grad || !m || !v || step < 1)
        return mfail(EXPI_EINVAL, "bad Adam arguments");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((count + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), count, params, grad, m, v, lr, beta1, beta2,
                       eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(EXPI_EHIP, hipGetErrorString(e));
    return EXPI_OK;
}

}  // extern "C"
