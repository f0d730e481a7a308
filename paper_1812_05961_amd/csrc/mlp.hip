// The variant selector's network on the GPU: a three-layer perceptron
// in -> H -> H -> 1 (ReLU after the first two layers, H <= 64) trained on mean
// squared error with Adam (Kingma and Ba, ICLR 2015).  Parameters are one flat
// float vector: W1 (H x in, row-major), b1 (H), W2 (H x H), b2 (H), W3 (H), b3.
//
// One wave per sample for the forward and backward passes (lane j = hidden
// unit j); weight gradients are sums over the batch computed by one thread per
// parameter in batch order (deterministic).
#include <algorithm>
#include <random>
#include <vector>

#include "common.h"

namespace cpd {
namespace {

struct Net {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

__host__ __device__ inline Net net_view(const float *p, int in, int H) {
    Net n;
    n.W1 = p;
    n.b1 = n.W1 + (int64_t)H * in;
    n.W2 = n.b1 + H;
    n.b2 = n.W2 + (int64_t)H * H;
    n.W3 = n.b2 + H;
    n.b3 = n.W3 + H;
    return n;
}

inline int64_t nparams(int in, int H) { return (int64_t)H * in + H + (int64_t)H * H + H + H + 1; }

__device__ __forceinline__ float wave_sumf(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// f[b] (and z1, z2 when given) for samples b of X (B x in)
__global__ void __launch_bounds__(256)
k_forward(const float *__restrict__ p, int in, int H, const float *__restrict__ X, int64_t B, float *__restrict__ f,
          float *__restrict__ z1, float *__restrict__ z2) {
    __shared__ float h1s[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + wave;
    if (b >= B) return;  // waves are independent
    const Net n = net_view(p, in, H);
    const float *x = X + b * in;
    const bool on = lane < H;
    float a = 0.0f;
    if (on) {
        a = n.b1[lane];
        for (int i = 0; i < in; ++i) a = fmaf(n.W1[(int64_t)lane * in + i], x[i], a);
        if (z1) z1[b * H + lane] = a;
    }
    h1s[wave][lane] = on ? fmaxf(a, 0.0f) : 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float c = 0.0f;
    if (on) {
        c = n.b2[lane];
        for (int k = 0; k < H; ++k) c = fmaf(n.W2[(int64_t)lane * H + k], h1s[wave][k], c);
        if (z2) z2[b * H + lane] = c;
    }
    const float out = wave_sumf(on ? n.W3[lane] * fmaxf(c, 0.0f) : 0.0f) + n.b3[0];
    if (lane == 0) f[b] = out;
}

// dL/dz2, dL/dz1 and dL/df per sample, for L = mean (f - y)^2
__global__ void __launch_bounds__(256)
k_backward(const float *__restrict__ p, int in, int H, const float *__restrict__ z1, const float *__restrict__ z2,
           const float *__restrict__ f, const float *__restrict__ y, int64_t B, float *__restrict__ dz1,
           float *__restrict__ dz2, float *__restrict__ df) {
    __shared__ float d2s[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + wave;
    if (b >= B) return;
    const Net n = net_view(p, in, H);
    const bool on = lane < H;
    const float d = 2.0f * (f[b] - y[b]) / (float)B;
    if (lane == 0) df[b] = d;
    const float g2 = (on && z2[b * H + lane] > 0.0f) ? d * n.W3[lane] : 0.0f;
    if (on) dz2[b * H + lane] = g2;
    d2s[wave][lane] = g2;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (on) {
        float h = 0.0f;
        for (int j = 0; j < H; ++j) h = fmaf(n.W2[(int64_t)j * H + lane], d2s[wave][j], h);
        dz1[b * H + lane] = z1[b * H + lane] > 0.0f ? h : 0.0f;
    }
}

// gradient entry t: a sum over the batch, in batch order
__global__ void k_grad(const float *__restrict__ X, int in, int H, const float *__restrict__ z1,
                       const float *__restrict__ z2, const float *__restrict__ dz1, const float *__restrict__ dz2,
                       const float *__restrict__ df, int64_t B, float *__restrict__ g) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t oW1 = 0, ob1 = (int64_t)H * in, oW2 = ob1 + H, ob2 = oW2 + (int64_t)H * H, oW3 = ob2 + H,
                  ob3 = oW3 + H;
    if (t > ob3) return;
    float s = 0.0f;
    if (t < ob1) {
        const int64_t j = t / in, i = t % in;
        for (int64_t b = 0; b < B; ++b) s = fmaf(dz1[b * H + j], X[b * in + i], s);
    } else if (t < oW2) {
        const int64_t j = t - ob1;
        for (int64_t b = 0; b < B; ++b) s += dz1[b * H + j];
    } else if (t < ob2) {
        const int64_t j = (t - oW2) / H, k = (t - oW2) % H;
        for (int64_t b = 0; b < B; ++b) s = fmaf(dz2[b * H + j], fmaxf(z1[b * H + k], 0.0f), s);
    } else if (t < oW3) {
        const int64_t j = t - ob2;
        for (int64_t b = 0; b < B; ++b) s += dz2[b * H + j];
    } else if (t < ob3) {
        const int64_t j = t - oW3;
        for (int64_t b = 0; b < B; ++b) s = fmaf(df[b], fmaxf(z2[b * H + j], 0.0f), s);
    } else {
        for (int64_t b = 0; b < B; ++b) s += df[b];
    }
    (void)oW1;
    g[t] = s;
}

// mean squared error of f against y (one block)
__global__ void k_mse(const float *__restrict__ f, const float *__restrict__ y, int64_t B, float *__restrict__ out) {
    __shared__ float red[4];
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < B; b += blockDim.x) {
        const float e = f[b] - y[b];
        s = fmaf(e, e, s);
    }
    s = wave_sumf(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (red[0] + red[1] + red[2] + red[3]) / (float)B;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t count, float lr, float beta1, float beta2, float eps, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const float gt = g[t];
    const float mt = beta1 * m[t] + (1.0f - beta1) * gt;
    const float vt = beta2 * v[t] + (1.0f - beta2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt * c1) / (sqrtf(vt * c2) + eps);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// He initialisation: weights N(0, 2/fan_in) by Box-Muller on SplitMix64 draws, biases 0
__global__ void k_init(float *p, int in, int H, uint64_t seed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ob1 = (int64_t)H * in, oW2 = ob1 + H, ob2 = oW2 + (int64_t)H * H, oW3 = ob2 + H, ob3 = oW3 + H;
    if (t > ob3) return;
    int fan = 0;
    if (t < ob1) fan = in;
    else if (t >= oW2 && t < ob2) fan = H;
    else if (t >= oW3 && t < ob3) fan = H;
    if (fan == 0) {
        p[t] = 0.0f;
        return;
    }
    const uint64_t a = mix64(seed ^ (2 * (uint64_t)t)), b = mix64(seed ^ (2 * (uint64_t)t + 1));
    const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53, u2 = (double)(b >> 11) * 0x1.0p-53;
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    p[t] = (float)(z * sqrt(2.0 / fan));
}

__global__ void k_gather_rows(const float *__restrict__ X, const float *__restrict__ y, int in,
                              const int32_t *__restrict__ idx, int64_t B, float *__restrict__ Xb,
                              float *__restrict__ yb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * in) return;
    const int64_t b = t / in, i = t % in, s = idx[b];
    Xb[t] = X[s * in + i];
    if (i == 0) yb[b] = y[s];
}

cpd_status check_shape(int in, int H) {
    if (in < 1 || in > 4096 || H < 1 || H > 64) CPD_FAIL(CPD_EINVAL, "network shape in=%d hidden=%d (hidden <= 64)", in, H);
    return CPD_OK;
}

struct Work {
    DevBuf<float> z1, z2, dz1, dz2, df, f;
    cpd_status alloc(int64_t B, int H, hipStream_t s) {
        CPD_TRY(z1.alloc((size_t)B * H, s));
        CPD_TRY(z2.alloc((size_t)B * H, s));
        CPD_TRY(dz1.alloc((size_t)B * H, s));
        CPD_TRY(dz2.alloc((size_t)B * H, s));
        CPD_TRY(df.alloc(B, s));
        CPD_TRY(f.alloc(B, s));
        return CPD_OK;
    }
};

cpd_status loss_grad(const float *p, int in, int H, const float *X, const float *y, int64_t B, float *loss, float *g,
                     Work &w, hipStream_t s) {
    const unsigned gb = (unsigned)ceil_div(B, 4);
    hipLaunchKernelGGL(k_forward, dim3(gb), dim3(256), 0, s, p, in, H, X, B, w.f.p, w.z1.p, w.z2.p);
    CPD_LAUNCH_CHECK();
    if (loss) {
        hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, (const float *)w.f.p, y, B, loss);
        CPD_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_backward, dim3(gb), dim3(256), 0, s, p, in, H, (const float *)w.z1.p, (const float *)w.z2.p,
                       (const float *)w.f.p, y, B, w.dz1.p, w.dz2.p, w.df.p);
    CPD_LAUNCH_CHECK();
    const int64_t P = nparams(in, H);
    hipLaunchKernelGGL(k_grad, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, s, X, in, H, (const float *)w.z1.p,
                       (const float *)w.z2.p, (const float *)w.dz1.p, (const float *)w.dz2.p, (const float *)w.df.p, B,
                       g);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

}  // namespace
}  // namespace cpd

using namespace cpd;

extern "C" {

int64_t cpd_mlp_param_count(int32_t n_in, int32_t hidden) {
    if (n_in < 1 || hidden < 1) return 0;
    return nparams(n_in, hidden);
}

cpd_status cpd_mlp_init(float *params, int32_t n_in, int32_t hidden, uint64_t seed, void *stream) {
    clear_error();
    CPD_TRY(check_shape(n_in, hidden));
    if (!params) CPD_FAIL(CPD_EINVAL, "null params");
    const int64_t P = nparams(n_in, hidden);
    hipLaunchKernelGGL(k_init, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, (hipStream_t)stream, params, n_in, hidden,
                       seed);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

cpd_status cpd_mlp_forward(const float *params, int32_t n_in, int32_t hidden, const float *X, int64_t batch, float *out,
                           void *stream) {
    clear_error();
    CPD_TRY(check_shape(n_in, hidden));
    if (!params || !X || !out || batch < 0) CPD_FAIL(CPD_EINVAL, "bad forward arguments");
    if (batch == 0) return CPD_OK;
    hipLaunchKernelGGL(k_forward, dim3((unsigned)ceil_div(batch, 4)), dim3(256), 0, (hipStream_t)stream, params, n_in,
                       hidden, X, batch, out, (float *)nullptr, (float *)nullptr);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

cpd_status cpd_mlp_loss_grad(const float *params, int32_t n_in, int32_t hidden, const float *X, const float *y,
                             int64_t batch, float *loss, float *grad, void *stream) {
    clear_error();
    CPD_TRY(check_shape(n_in, hidden));
    if (!params || !X || !y || !grad || batch < 1) CPD_FAIL(CPD_EINVAL, "bad loss/gradient arguments");
    hipStream_t s = (hipStream_t)stream;
    Work w;
    CPD_TRY(w.alloc(batch, hidden, s));
    return loss_grad(params, n_in, hidden, X, y, batch, loss, grad, w, s);
}

cpd_status cpd_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count, float lr, float beta1,
                        float beta2, float eps, int32_t step, void *stream) {
    clear_error();
    if (!params || !grad || !m || !v || count < 0 || step < 1) CPD_FAIL(CPD_EINVAL, "bad Adam arguments");
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    if (count == 0) return CPD_OK;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, (hipStream_t)stream, params, grad, m, v,
                       count, lr, beta1, beta2, eps, c1, c2);
    CPD_LAUNCH_CHECK();
    return CPD_OK;
}

cpd_status cpd_mlp_train(float *params, int32_t n_in, int32_t hidden, const float *X, const float *y, int64_t n,
                         int32_t epochs, int32_t batch, float lr, uint64_t seed, float *loss_trace, void *stream) {
    clear_error();
    CPD_TRY(check_shape(n_in, hidden));
    if (!params || !X || !y || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0f))
        CPD_FAIL(CPD_EINVAL, "bad training arguments");
    hipStream_t s = (hipStream_t)stream;
    const int64_t P = nparams(n_in, hidden), B = std::min<int64_t>(batch, n);
    const int64_t nb = ceil_div(n, B);
    DevBuf<float> m, v, g, Xb, yb, losses;
    DevBuf<int32_t> idx;
    Work w;
    CPD_TRY(m.alloc(P, s));
    CPD_TRY(v.alloc(P, s));
    CPD_TRY(g.alloc(P, s));
    CPD_TRY(Xb.alloc((size_t)B * n_in, s));
    CPD_TRY(yb.alloc(B, s));
    CPD_TRY(losses.alloc(nb, s));
    CPD_TRY(idx.alloc(n, s));
    CPD_TRY(w.alloc(B, hidden, s));
    CPD_HIP(hipMemsetAsync(m.p, 0, sizeof(float) * P, s));
    CPD_HIP(hipMemsetAsync(v.p, 0, sizeof(float) * P, s));
    std::vector<int32_t> order(n);
    std::vector<float> lh(nb);
    std::mt19937_64 rng(seed);
    int32_t step = 0;
    for (int e = 0; e < epochs; ++e) {
        for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
        std::shuffle(order.begin(), order.end(), rng);
        CPD_HIP(hipMemcpyAsync(idx.p, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        for (int64_t bi = 0; bi < nb; ++bi) {
            const int64_t b0 = bi * B, bn = std::min<int64_t>(B, n - b0);
            hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)ceil_div(bn * n_in, 256)), dim3(256), 0, s, X, y, n_in,
                               (const int32_t *)idx.p + b0, bn, Xb.p, yb.p);
            CPD_LAUNCH_CHECK();
            CPD_TRY(loss_grad(params, n_in, hidden, Xb.p, yb.p, bn, losses.p + bi, g.p, w, s));
            CPD_TRY(cpd_mlp_adam(params, g.p, m.p, v.p, P, lr, 0.9f, 0.999f, 1e-8f, ++step, stream));
        }
        if (loss_trace) {
            CPD_HIP(hipMemcpyAsync(lh.data(), losses.p, sizeof(float) * nb, hipMemcpyDeviceToHost, s));
            CPD_HIP(hipStreamSynchronize(s));
            double acc = 0.0;
            for (int64_t bi = 0; bi < nb; ++bi) acc += lh[bi];
            loss_trace[e] = (float)(acc / nb);
        }
    }
    CPD_HIP(hipStreamSynchronize(s));
    return CPD_OK;
}

}  // extern "C"
