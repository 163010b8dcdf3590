// Cost model of the tuner: a small fully connected network in FP32 (forward,
// mean-squared-error gradient by back-propagation, Adam update), as HIP
// kernels behind the C ABI.  The network and its training are not from the
// paper; they stand beside its auto-tuner (Section "Auto-tuning") as a
// learned proposer of candidates.
//
// Network: n_in inputs -> n_layers hidden layers of n_hidden units, each
// z = W a + b followed by ReLU -> one linear output.  Parameters are one flat
// array, layer by layer: W (fan_out x fan_in, row-major), then b (fan_out).
// Every sum runs in a fixed order (ascending index), so results do not depend
// on the launch configuration.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/girih.h"

namespace {

constexpr int kBlock = 256;

__global__ void linear_fwd_kernel(const float* __restrict__ W, const float* __restrict__ b,
                                  const float* __restrict__ X, int n, int fan_in, int fan_out, int relu,
                                  float* __restrict__ Y) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * fan_out) return;
    const int i = (int)(idx / fan_out), o = (int)(idx % fan_out);
    const float* w = W + (int64_t)o * fan_in;
    const float* x = X + (int64_t)i * fan_in;
    float z = b[o];
    for (int j = 0; j < fan_in; ++j) z += w[j] * x[j];
    Y[idx] = relu ? (z > 0.f ? z : 0.f) : z;
}

// Output layer's delta and the loss: d[i] = 2 (y_i - t_i) / n; loss = sum (y_i - t_i)^2 / n.
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, int n, float* __restrict__ d,
                           float* __restrict__ loss) {
    __shared__ float part[kBlock];
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        const float e = y[i] - t[i];
        d[i] = 2.f * e / (float)n;
        acc += e * e;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int k = 0; k < kBlock; ++k) s += part[k];
        *loss = s / (float)n;
    }
}

// dW[o][j] = sum_i delta[i][o] * A[i][j];  db[o] = sum_i delta[i][o]
__global__ void linear_bwd_w_kernel(const float* __restrict__ delta, const float* __restrict__ A, int n, int fan_in,
                                    int fan_out, float* __restrict__ dW, float* __restrict__ db) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)fan_out * fan_in;
    if (idx < nw) {
        const int o = (int)(idx / fan_in), j = (int)(idx % fan_in);
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += delta[(int64_t)i * fan_out + o] * A[(int64_t)i * fan_in + j];
        dW[idx] = s;
    } else if (idx < nw + fan_out) {
        const int o = (int)(idx - nw);
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += delta[(int64_t)i * fan_out + o];
        db[o] = s;
    }
}

// delta_prev[i][j] = (sum_o W[o][j] delta[i][o]) * [A[i][j] > 0]  (A: ReLU output of the layer below)
__global__ void linear_bwd_x_kernel(const float* __restrict__ W, const float* __restrict__ delta,
                                    const float* __restrict__ A, int n, int fan_in, int fan_out,
                                    float* __restrict__ delta_prev) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * fan_in) return;
    const int i = (int)(idx / fan_in), j = (int)(idx % fan_in);
    float s = 0.f;
    for (int o = 0; o < fan_out; ++o) s += W[(int64_t)o * fan_in + j] * delta[(int64_t)i * fan_out + o];
    delta_prev[idx] = A[idx] > 0.f ? s : 0.f;
}

// Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

bool shape_ok(int32_t n_in, int32_t n_hidden, int32_t n_layers) {
    return n_in >= 1 && n_in <= 4096 && n_hidden >= 1 && n_hidden <= 4096 && n_layers >= 1 && n_layers <= 16;
}

int64_t param_count(int32_t n_in, int32_t n_hidden, int32_t n_layers) {
    int64_t c = (int64_t)n_hidden * n_in + n_hidden;
    c += (int64_t)(n_layers - 1) * ((int64_t)n_hidden * n_hidden + n_hidden);
    c += n_hidden + 1;
    return c;
}

// workspace: activations of every hidden layer (n x n_hidden each), the output
// (n), and two delta buffers (n x n_hidden) plus the output delta (n) and the loss
int64_t work_count(int32_t n_hidden, int32_t n_layers, int32_t n) {
    return (int64_t)n * n_hidden * n_layers + n + 2 * (int64_t)n * n_hidden + n + 1;
}

struct Net {
    int32_t n_in, n_hidden, n_layers;
    int fan_in(int l) const { return l == 0 ? n_in : n_hidden; }
    int fan_out(int l) const { return l == n_layers ? 1 : n_hidden; }
    int64_t w_off(int l) const {
        int64_t o = 0;
        for (int q = 0; q < l; ++q) o += (int64_t)fan_out(q) * fan_in(q) + fan_out(q);
        return o;
    }
    int64_t b_off(int l) const { return w_off(l) + (int64_t)fan_out(l) * fan_in(l); }
};

#define HIPCHK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return GIRIH_E_HIP;  \
    } while (0)

int forward(const Net& net, const float* params, const float* x, int32_t n, float* work, hipStream_t s,
            float** out) {
    const float* a = x;
    for (int l = 0; l <= net.n_layers; ++l) {
        float* y = l < net.n_layers ? work + (int64_t)l * n * net.n_hidden
                                    : work + (int64_t)net.n_layers * n * net.n_hidden;
        const int64_t cnt = (int64_t)n * net.fan_out(l);
        hipLaunchKernelGGL(linear_fwd_kernel, dim3(blocks_for(cnt)), dim3(kBlock), 0, s, params + net.w_off(l),
                           params + net.b_off(l), a, n, net.fan_in(l), net.fan_out(l), l < net.n_layers ? 1 : 0, y);
        HIPCHK(hipGetLastError());
        a = y;
    }
    *out = work + (int64_t)net.n_layers * n * net.n_hidden;
    return GIRIH_OK;
}

}  // namespace

extern "C" {

int girih_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_layers, int64_t* count) {
    if (!count || !shape_ok(n_in, n_hidden, n_layers)) return GIRIH_E_INVALID;
    *count = param_count(n_in, n_hidden, n_layers);
    return GIRIH_OK;
}

int girih_mlp_work_count(int32_t n_in, int32_t n_hidden, int32_t n_layers, int32_t n, int64_t* count) {
    if (!count || !shape_ok(n_in, n_hidden, n_layers) || n < 1) return GIRIH_E_INVALID;
    *count = work_count(n_hidden, n_layers, n);
    return GIRIH_OK;
}

int girih_mlp_forward(const float* params, int32_t n_in, int32_t n_hidden, int32_t n_layers, const float* x,
                      int32_t n, float* y, float* work, int64_t work_len, void* hip_stream) {
    if (!params || !x || !y || !work || n < 1 || !shape_ok(n_in, n_hidden, n_layers)) return GIRIH_E_INVALID;
    if (work_len < work_count(n_hidden, n_layers, n)) return GIRIH_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const Net net{n_in, n_hidden, n_layers};
    float* out = nullptr;
    int rc = forward(net, params, x, n, work, s, &out);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(y, out, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, s));
    return GIRIH_OK;
}

int girih_mlp_loss_grad(const float* params, int32_t n_in, int32_t n_hidden, int32_t n_layers, const float* x,
                        const float* target, int32_t n, float* loss, float* grad, float* work, int64_t work_len,
                        void* hip_stream) {
    if (!params || !x || !target || !loss || !grad || !work || n < 1 || !shape_ok(n_in, n_hidden, n_layers))
        return GIRIH_E_INVALID;
    if (work_len < work_count(n_hidden, n_layers, n)) return GIRIH_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const Net net{n_in, n_hidden, n_layers};
    float* out = nullptr;
    int rc = forward(net, params, x, n, work, s, &out);
    if (rc) return rc;
    float* acts = work;                                            // hidden activations, layer by layer
    float* d0 = work + (int64_t)n_layers * n * n_hidden + n;       // delta buffers
    float* d1 = d0 + (int64_t)n * n_hidden;
    float* dout = d1 + (int64_t)n * n_hidden;                      // output delta (n)
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(kBlock), 0, s, out, target, n, dout, loss);
    HIPCHK(hipGetLastError());
    const float* delta = dout;
    for (int l = n_layers; l >= 0; --l) {
        const float* a_in = l == 0 ? x : acts + (int64_t)(l - 1) * n * n_hidden;
        const int fi = net.fan_in(l), fo = net.fan_out(l);
        const int64_t cw = (int64_t)fo * fi + fo;
        hipLaunchKernelGGL(linear_bwd_w_kernel, dim3(blocks_for(cw)), dim3(kBlock), 0, s, delta, a_in, n, fi, fo,
                           grad + net.w_off(l), grad + net.b_off(l));
        HIPCHK(hipGetLastError());
        if (l > 0) {
            float* dprev = (delta == d0) ? d1 : d0;
            const int64_t cx = (int64_t)n * fi;
            hipLaunchKernelGGL(linear_bwd_x_kernel, dim3(blocks_for(cx)), dim3(kBlock), 0, s, params + net.w_off(l),
                               delta, a_in, n, fi, fo, dprev);
            HIPCHK(hipGetLastError());
            delta = dprev;
        }
    }
    return GIRIH_OK;
}

int girih_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t count, float lr, float beta1,
                   float beta2, float eps, int32_t step, void* hip_stream) {
    if (!params || !grad || !m || !v || count < 1 || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return GIRIH_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // bias corrections, formed in double and rounded once
    double p1 = 1, p2 = 1;
    for (int32_t i = 0; i < step; ++i) {
        p1 *= beta1;
        p2 *= beta2;
    }
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count)), dim3(kBlock), 0, s, params, grad, m, v, count, lr, beta1,
                       beta2, eps, (float)(1.0 - p1), (float)(1.0 - p2));
    HIPCHK(hipGetLastError());
    return GIRIH_OK;
}

}  // extern "C"
