// The cost model of the dispatch: a small fully connected network (fp32)
// that maps a bucket's features to the predicted log(ns per probe) of every
// dispatch option, with its training (masked mean squared error, Adam) done
// by the kernels below.
//
// Parameter buffer (float, device), for n_in inputs, H hidden units, K outputs:
//   mean[n_in], inv_std[n_in]        input normalisation (set from the data, not trained)
//   W1[H][n_in], b1[H], W2[H][H], b2[H], W3[K][H], b3[K]
// Forward: x' = (x - mean) * inv_std, h1 = relu(W1 x' + b1),
//          h2 = relu(W2 h1 + b2), y = W3 h2 + b3.
#include <cmath>
#include <vector>

#include "aot.h"
#include "kernels.hpp"

namespace aot {

namespace {

constexpr int kMaxIn = 16;
constexpr int kMaxHidden = 64;
constexpr int kMaxOut = 16;

struct Shape {
  int in, hid, out;
  __host__ __device__ int64_t o_mean() const { return 0; }
  __host__ __device__ int64_t o_istd() const { return in; }
  __host__ __device__ int64_t o_w1() const { return 2 * in; }
  __host__ __device__ int64_t o_b1() const { return o_w1() + (int64_t)hid * in; }
  __host__ __device__ int64_t o_w2() const { return o_b1() + hid; }
  __host__ __device__ int64_t o_b2() const { return o_w2() + (int64_t)hid * hid; }
  __host__ __device__ int64_t o_w3() const { return o_b2() + hid; }
  __host__ __device__ int64_t o_b3() const { return o_w3() + (int64_t)out * hid; }
  __host__ __device__ int64_t total() const { return o_b3() + out; }
  __host__ __device__ int64_t trainable() const { return total() - 2 * in; }
};

bool shape_ok(int in, int hid, int out) {
  return in >= 1 && in <= kMaxIn && hid >= 1 && hid <= kMaxHidden && out >= 1 && out <= kMaxOut;
}

// A uniform float in [-1, 1) from a counter (MurmurHash3's 32-bit finaliser
// over seed and index).
__device__ __forceinline__ float hash_uniform(uint64_t seed, uint64_t i) {
  uint32_t h = (uint32_t)(seed ^ (seed >> 32)) ^ (uint32_t)(i * 0x9E3779B1u) ^ (uint32_t)(i >> 32);
  h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
  return (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
}

// Weights uniform in +-sqrt(6 / fan_in), biases 0, identity normalisation.
__global__ void k_mlp_init(float* p, Shape s, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.total();
       i += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    if (i < s.o_istd()) v = 0.f;
    else if (i < s.o_w1()) v = 1.f;
    else if (i < s.o_b1()) v = hash_uniform(seed, i) * sqrtf(6.f / s.in);
    else if (i >= s.o_w2() && i < s.o_b2()) v = hash_uniform(seed, i) * sqrtf(6.f / s.hid);
    else if (i >= s.o_w3() && i < s.o_b3()) v = hash_uniform(seed, i) * sqrtf(6.f / s.hid);
    p[i] = v;
  }
}

// One thread per sample.
__device__ void forward_one(const float* __restrict__ p, const Shape& s, const float* x, float* xn,
                            float* h1, float* h2, float* y) {
  for (int d = 0; d < s.in; ++d) xn[d] = (x[d] - p[s.o_mean() + d]) * p[s.o_istd() + d];
  for (int h = 0; h < s.hid; ++h) {
    float a = p[s.o_b1() + h];
    for (int d = 0; d < s.in; ++d) a += p[s.o_w1() + (int64_t)h * s.in + d] * xn[d];
    h1[h] = a > 0.f ? a : 0.f;
  }
  for (int h = 0; h < s.hid; ++h) {
    float a = p[s.o_b2() + h];
    for (int g = 0; g < s.hid; ++g) a += p[s.o_w2() + (int64_t)h * s.hid + g] * h1[g];
    h2[h] = a > 0.f ? a : 0.f;
  }
  for (int k = 0; k < s.out; ++k) {
    float a = p[s.o_b3() + k];
    for (int h = 0; h < s.hid; ++h) a += p[s.o_w3() + (int64_t)k * s.hid + h] * h2[h];
    y[k] = a;
  }
}

__global__ void k_mlp_forward(const float* __restrict__ p, Shape s, const float* __restrict__ x,
                              int32_t batch, float* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  float xn[kMaxIn], h1[kMaxHidden], h2[kMaxHidden], yy[kMaxOut];
  forward_one(p, s, x + (int64_t)i * s.in, xn, h1, h2, yy);
  for (int k = 0; k < s.out; ++k) y[(int64_t)i * s.out + k] = yy[k];
}

// Per-sample gradient of the masked mean squared error
//   L = (1 / N) sum_i sum_k mask[i][k] (y[i][k] - t[i][k])^2,  N = number of set mask entries,
// written to row i of G (trainable parameters only, in buffer order), and the
// sample's share of L.
__global__ void k_mlp_grad_sample(const float* __restrict__ p, Shape s,
                                  const float* __restrict__ x, const float* __restrict__ t,
                                  const uint8_t* __restrict__ mask, int32_t batch, float inv_n,
                                  float* __restrict__ G, float* __restrict__ loss_part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  float xn[kMaxIn], h1[kMaxHidden], h2[kMaxHidden], y[kMaxOut];
  float dy[kMaxOut], dh2[kMaxHidden], dh1[kMaxHidden];
  forward_one(p, s, x + (int64_t)i * s.in, xn, h1, h2, y);
  float l = 0.f;
  for (int k = 0; k < s.out; ++k) {
    const bool on = mask[(int64_t)i * s.out + k] != 0;
    const float r = on ? y[k] - t[(int64_t)i * s.out + k] : 0.f;
    l += r * r;
    dy[k] = 2.f * r * inv_n;
  }
  loss_part[i] = l * inv_n;
  float* g = G + (int64_t)i * s.trainable();
  const int64_t base = 2 * s.in;      // trainable parameters start after the normalisation
  for (int h = 0; h < s.hid; ++h) {
    float a = 0.f;
    for (int k = 0; k < s.out; ++k) a += p[s.o_w3() + (int64_t)k * s.hid + h] * dy[k];
    dh2[h] = h2[h] > 0.f ? a : 0.f;
  }
  for (int g1 = 0; g1 < s.hid; ++g1) {
    float a = 0.f;
    for (int h = 0; h < s.hid; ++h) a += p[s.o_w2() + (int64_t)h * s.hid + g1] * dh2[h];
    dh1[g1] = h1[g1] > 0.f ? a : 0.f;
  }
  for (int h = 0; h < s.hid; ++h) {
    for (int d = 0; d < s.in; ++d) g[s.o_w1() - base + (int64_t)h * s.in + d] = dh1[h] * xn[d];
    g[s.o_b1() - base + h] = dh1[h];
  }
  for (int h = 0; h < s.hid; ++h) {
    for (int g1 = 0; g1 < s.hid; ++g1) g[s.o_w2() - base + (int64_t)h * s.hid + g1] = dh2[h] * h1[g1];
    g[s.o_b2() - base + h] = dh2[h];
  }
  for (int k = 0; k < s.out; ++k) {
    for (int h = 0; h < s.hid; ++h) g[s.o_w3() - base + (int64_t)k * s.hid + h] = dy[k] * h2[h];
    g[s.o_b3() - base + k] = dy[k];
  }
}

// grad[j] = sum over samples of G[i][j], in sample order (deterministic);
// the last thread also sums the loss.
__global__ void k_mlp_reduce(const float* __restrict__ G, int32_t batch, int64_t np,
                             float* __restrict__ grad, const float* __restrict__ loss_part,
                             float* __restrict__ loss) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < np) {
    float a = 0.f;
    for (int i = 0; i < batch; ++i) a += G[(int64_t)i * np + j];
    grad[j] = a;
  }
  if (j == np) {
    float a = 0.f;
    for (int i = 0; i < batch; ++i) a += loss_part[i];
    *loss = a;
  }
}

__global__ void k_mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, int64_t np, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  w[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// Normalisation from the data: mean and 1/std of each input (std floored).
__global__ void k_mlp_norm(float* p, Shape s, const float* __restrict__ x, int32_t batch) {
  const int d = threadIdx.x;
  if (d >= s.in) return;
  double a = 0.0, q = 0.0;
  for (int i = 0; i < batch; ++i) {
    const double v = x[(int64_t)i * s.in + d];
    a += v;
    q += v * v;
  }
  const double mean = batch ? a / batch : 0.0;
  const double var = batch ? q / batch - mean * mean : 0.0;
  const double sd = var > 1e-12 ? sqrt(var) : 1.0;
  p[s.o_mean() + d] = (float)mean;
  p[s.o_istd() + d] = (float)(1.0 / sd);
}

}  // namespace

// Forward of net on a batch (used by the learned dispatch).
int mlp_predict(const aot_mlp* net, const float* x_dev, int32_t batch, float* y_dev,
                hipStream_t s) {
  const Shape sh{net->n_in, net->n_hidden, net->n_out};
  hipLaunchKernelGGL(k_mlp_forward, dim3((batch + 63) / 64), dim3(64), 0, s, net->params, sh,
                     x_dev, batch, y_dev);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace aot

using aot::Shape;

namespace {

bool net_ok(const aot_mlp* net) {
  return net && net->params && aot::shape_ok(net->n_in, net->n_hidden, net->n_out);
}

Shape shape_of(const aot_mlp* net) { return Shape{net->n_in, net->n_hidden, net->n_out}; }

}  // namespace

extern "C" {

int aot_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t* count) {
  if (!count || !aot::shape_ok(n_in, n_hidden, n_out)) return AOT_E_ARG;
  *count = Shape{n_in, n_hidden, n_out}.total();
  return AOT_OK;
}

int aot_mlp_workspace(const aot_mlp* net, int32_t batch, size_t* bytes) {
  if (!net_ok(net) || batch < 0 || !bytes) return AOT_E_ARG;
  const Shape s = shape_of(net);
  const int64_t np = s.trainable();
  // per-sample gradients, gradient, Adam moments, loss parts, loss
  *bytes = sizeof(float) * (size_t)((int64_t)batch * np + 3 * np + batch + 64) + 1024;
  return AOT_OK;
}

int aot_mlp_init(const aot_mlp* net, uint64_t seed, void* stream) {
  if (!net_ok(net)) return AOT_E_ARG;
  const Shape s = shape_of(net);
  hipLaunchKernelGGL(aot::k_mlp_init, dim3(8), dim3(256), 0, static_cast<hipStream_t>(stream),
                     net->params, s, seed);
  return hipGetLastError() == hipSuccess ? AOT_OK : AOT_E_HIP;
}

int aot_mlp_forward(const aot_mlp* net, const float* x, int32_t batch, float* y, void* stream) {
  if (!net_ok(net) || batch < 0 || (batch > 0 && (!x || !y))) return AOT_E_ARG;
  if (batch == 0) return AOT_OK;
  hipLaunchKernelGGL(aot::k_mlp_forward, dim3((batch + 63) / 64), dim3(64), 0,
                     static_cast<hipStream_t>(stream), net->params, shape_of(net), x, batch, y);
  return hipGetLastError() == hipSuccess ? AOT_OK : AOT_E_HIP;
}

int aot_mlp_loss_grad(const aot_mlp* net, const float* x, const float* target,
                      const uint8_t* mask, int32_t batch, float* grad, float* loss, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!net_ok(net) || batch <= 0 || !x || !target || !mask || !grad || !loss) return AOT_E_ARG;
  size_t need = 0;
  aot_mlp_workspace(net, batch, &need);
  if (!ws || ws_bytes < need) return AOT_E_WORKSPACE;
  const Shape s = shape_of(net);
  const int64_t np = s.trainable();
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<uint8_t> hm((size_t)batch * s.out);
  if (hipMemcpyAsync(hm.data(), mask, hm.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return AOT_E_HIP;
  int64_t nobs = 0;
  for (uint8_t b : hm) nobs += b != 0;
  if (nobs == 0) return AOT_E_ARG;
  float* G = static_cast<float*>(ws);
  float* part = G + (int64_t)batch * np;
  hipLaunchKernelGGL(aot::k_mlp_grad_sample, dim3((batch + 63) / 64), dim3(64), 0, st,
                     net->params, s, x, target, mask, batch, 1.0f / (float)nobs, G, part);
  hipLaunchKernelGGL(aot::k_mlp_reduce, dim3((unsigned)((np + 1 + 255) / 256)), dim3(256), 0, st,
                     G, batch, np, grad, part, loss);
  return hipGetLastError() == hipSuccess ? AOT_OK : AOT_E_HIP;
}

int aot_mlp_train(const aot_mlp* net, const float* x, const float* target, const uint8_t* mask,
                  int32_t batch, int32_t epochs, float lr, float* losses, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!net_ok(net) || batch <= 0 || epochs < 0 || !(lr > 0.f) || !losses) return AOT_E_ARG;
  size_t need = 0;
  aot_mlp_workspace(net, batch, &need);
  if (!ws || ws_bytes < need) return AOT_E_WORKSPACE;
  const Shape s = shape_of(net);
  const int64_t np = s.trainable();
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* G = static_cast<float*>(ws);
  float* part = G + (int64_t)batch * np;
  float* grad = part + batch;
  float* m = grad + np;
  float* v = m + np;
  float* dloss = v + np;
  if (aot::fill_i32(reinterpret_cast<int32_t*>(m), 2 * np, 0, st) != hipSuccess) return AOT_E_HIP;
  hipLaunchKernelGGL(aot::k_mlp_norm, dim3(1), dim3(64), 0, st, net->params, s, x, batch);
  std::vector<uint8_t> hm((size_t)batch * s.out);
  if (hipMemcpyAsync(hm.data(), mask, hm.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return AOT_E_HIP;
  int64_t nobs = 0;
  for (uint8_t b : hm) nobs += b != 0;
  if (nobs == 0) return AOT_E_ARG;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float p1 = 1.f, p2 = 1.f;
  std::vector<float> dl(epochs > 0 ? epochs : 1);
  for (int e = 0; e < epochs; ++e) {
    hipLaunchKernelGGL(aot::k_mlp_grad_sample, dim3((batch + 63) / 64), dim3(64), 0, st,
                       net->params, s, x, target, mask, batch, 1.0f / (float)nobs, G, part);
    hipLaunchKernelGGL(aot::k_mlp_reduce, dim3((unsigned)((np + 1 + 255) / 256)), dim3(256), 0,
                       st, G, batch, np, grad, part, dloss + e % 64);
    p1 *= b1;
    p2 *= b2;
    hipLaunchKernelGGL(aot::k_mlp_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st,
                       net->params + 2 * s.in, grad, m, v, np, lr, b1, b2, eps, 1.f - p1,
                       1.f - p2);
    if (e % 64 == 63 || e == epochs - 1) {
      const int n = e % 64 + 1;
      if (hipMemcpyAsync(dl.data() + (e - n + 1), dloss, sizeof(float) * n, hipMemcpyDeviceToHost,
                         st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return AOT_E_HIP;
    }
  }
  for (int e = 0; e < epochs; ++e) losses[e] = dl[e];
  return hipGetLastError() == hipSuccess ? AOT_OK : AOT_E_HIP;
}

}  // extern "C"
