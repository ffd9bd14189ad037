// Learned temperature: a 16 -> 64 -> 64 -> 1 FP32 network (ReLU, ReLU, sigmoid) that maps level
// statistics to the temperature tau of a Jet round (the quantity the paper fixes by a schedule in
// Section 4.1 and studies in Section 7).  Inference, the backward pass and Adam run in the kernels
// below; every sum has a fixed order (no floating-point atomics), so training is reproducible.
//
// Flat parameter layout: W1[64][16] (row = hidden unit), b1[64], W2[64][64] (row = output unit),
// b2[64], w3[64], b3.  Inputs are raw features, standardised in the first kernel with the stored
// per-feature mean and standard deviation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "jet_internal.h"

namespace {

constexpr int kIn = 16, kH = 64;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, ow3 = ob2 + kH, ob3 = ow3 + kH;
constexpr int kParams = ob3 + 1;  // 5313
static_assert(kParams == JET_MLP_NPARAM, "parameter count");
constexpr int kFwdBlock = 64;

// One thread per sample.  Writes the standardised input, both hidden activations and the output;
// the activations are what the backward pass needs (h > 0 iff the pre-activation is > 0).
__global__ __launch_bounds__(kFwdBlock) void k_mlp_forward(const float *__restrict__ theta,
                                                           const float *__restrict__ mean,
                                                           const float *__restrict__ stdv,
                                                           const float *__restrict__ X, int32_t B,
                                                           float *__restrict__ xs, float *__restrict__ h1,
                                                           float *__restrict__ h2, float *__restrict__ y) {
  __shared__ float w[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) w[i] = theta[i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  float x[kIn], a1[kH];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = (X[s * kIn + i] - mean[i]) / stdv[i];
  for (int j = 0; j < kH; ++j) {
    float z = w[ob1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) z += w[oW1 + j * kIn + i] * x[i];
    a1[j] = z > 0.0f ? z : 0.0f;
  }
  float z3 = w[ob3];
  for (int j = 0; j < kH; ++j) {
    float z = w[ob2 + j];
    for (int i = 0; i < kH; ++i) z += w[oW2 + j * kH + i] * a1[i];
    const float a2 = z > 0.0f ? z : 0.0f;
    if (h2) h2[s * kH + j] = a2;
    z3 += w[ow3 + j] * a2;
  }
  y[s] = 1.0f / (1.0f + expf(-z3));
  if (xs) {
#pragma unroll
    for (int i = 0; i < kIn; ++i) xs[s * kIn + i] = x[i];
  }
  if (h1) {
    for (int j = 0; j < kH; ++j) h1[s * kH + j] = a1[j];
  }
}

// One thread per sample: dL/dz of every layer for L = mean over the batch of (y - t)^2.
__global__ __launch_bounds__(kFwdBlock) void k_mlp_delta(const float *__restrict__ theta,
                                                         const float *__restrict__ h1,
                                                         const float *__restrict__ h2,
                                                         const float *__restrict__ y, const float *__restrict__ t,
                                                         int32_t B, float *__restrict__ d1,
                                                         float *__restrict__ d2, float *__restrict__ d3) {
  __shared__ float w[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) w[i] = theta[i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const float ys = y[s];
  const float dy = 2.0f * (ys - t[s]) / (float)B;
  const float g3 = dy * ys * (1.0f - ys);
  d3[s] = g3;
  float g2[kH];
  for (int i = 0; i < kH; ++i) {
    g2[i] = h2[s * kH + i] > 0.0f ? g3 * w[ow3 + i] : 0.0f;
    d2[s * kH + i] = g2[i];
  }
  for (int j = 0; j < kH; ++j) {
    float acc = 0.0f;
    for (int i = 0; i < kH; ++i) acc += g2[i] * w[oW2 + i * kH + j];
    d1[s * kH + j] = h1[s * kH + j] > 0.0f ? acc : 0.0f;
  }
}

// One thread per parameter (plus one for the loss): the batch sum in sample order.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float *__restrict__ xs, const float *__restrict__ h1,
                                                   const float *__restrict__ h2, const float *__restrict__ y,
                                                   const float *__restrict__ t, const float *__restrict__ d1,
                                                   const float *__restrict__ d2, const float *__restrict__ d3,
                                                   int32_t B, float *__restrict__ grad, float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kParams) return;
  float acc = 0.0f;
  if (p == kParams) {  // the loss itself
    for (int32_t s = 0; s < B; ++s) {
      const float r = y[s] - t[s];
      acc += r * r;
    }
    *loss = acc / (float)B;
    return;
  }
  if (p < ob1) {
    const int j = (p - oW1) / kIn, i = (p - oW1) % kIn;
    for (int32_t s = 0; s < B; ++s) acc += d1[(int64_t)s * kH + j] * xs[(int64_t)s * kIn + i];
  } else if (p < oW2) {
    const int j = p - ob1;
    for (int32_t s = 0; s < B; ++s) acc += d1[(int64_t)s * kH + j];
  } else if (p < ob2) {
    const int j = (p - oW2) / kH, i = (p - oW2) % kH;
    for (int32_t s = 0; s < B; ++s) acc += d2[(int64_t)s * kH + j] * h1[(int64_t)s * kH + i];
  } else if (p < ow3) {
    const int j = p - ob2;
    for (int32_t s = 0; s < B; ++s) acc += d2[(int64_t)s * kH + j];
  } else if (p < ob3) {
    const int i = p - ow3;
    for (int32_t s = 0; s < B; ++s) acc += d3[s] * h2[(int64_t)s * kH + i];
  } else {
    for (int32_t s = 0; s < B; ++s) acc += d3[s];
  }
  grad[p] = acc;
}

// Adam (Kingma and Ba, Algorithm 1) with the bias corrections c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
// formed on the host in double.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ theta, float *__restrict__ m,
                                                  float *__restrict__ v, const float *__restrict__ g, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float gp = g[p];
  const float mp = beta1 * m[p] + (1.0f - beta1) * gp;
  const float vp = beta2 * v[p] + (1.0f - beta2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  theta[p] = theta[p] - lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) for the seeded initialisation.
uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

thread_local std::string g_mlp_error;

}  // namespace

struct jet_mlp {
  hipStream_t stream = nullptr;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *mean = nullptr, *stdv = nullptr;
  float *loss = nullptr;
  int64_t step = 0;
  int32_t cap = 0;  // batch capacity of the activation buffers
  float *xs = nullptr, *h1 = nullptr, *h2 = nullptr, *y = nullptr, *d1 = nullptr, *d2 = nullptr, *d3 = nullptr;
  std::string last_error;
};

namespace {

int mlp_fail(jet_mlp *net, int code, const std::string &msg) {
  if (net) net->last_error = msg;
  else g_mlp_error = msg;
  return code;
}

#define MLP_HIP(net, expr)                                                                   \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return mlp_fail(net, JET_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

void free_batch(jet_mlp *net) {
  float *ptrs[] = {net->xs, net->h1, net->h2, net->y, net->d1, net->d2, net->d3};
  for (float *p : ptrs)
    if (p) (void)hipFree(p);
  net->xs = net->h1 = net->h2 = net->y = net->d1 = net->d2 = net->d3 = nullptr;
  net->cap = 0;
}

int ensure_batch(jet_mlp *net, int32_t B) {
  if (B <= net->cap) return JET_OK;
  MLP_HIP(net, hipStreamSynchronize(net->stream));
  free_batch(net);
  const size_t b = (size_t)B;
  if (hipMalloc((void **)&net->xs, sizeof(float) * b * kIn) != hipSuccess ||
      hipMalloc((void **)&net->h1, sizeof(float) * b * kH) != hipSuccess ||
      hipMalloc((void **)&net->h2, sizeof(float) * b * kH) != hipSuccess ||
      hipMalloc((void **)&net->y, sizeof(float) * b) != hipSuccess ||
      hipMalloc((void **)&net->d1, sizeof(float) * b * kH) != hipSuccess ||
      hipMalloc((void **)&net->d2, sizeof(float) * b * kH) != hipSuccess ||
      hipMalloc((void **)&net->d3, sizeof(float) * b) != hipSuccess) {
    free_batch(net);
    return mlp_fail(net, JET_ENOMEM, "activation buffers");
  }
  net->cap = B;
  return JET_OK;
}

unsigned blocks_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

int forward_into(jet_mlp *net, const float *X, int32_t B, float *y, bool keep) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(B, kFwdBlock)), dim3(kFwdBlock), 0, net->stream, net->theta,
                     net->mean, net->stdv, X, B, keep ? net->xs : nullptr, keep ? net->h1 : nullptr,
                     keep ? net->h2 : nullptr, y);
  MLP_HIP(net, hipGetLastError());
  return JET_OK;
}

int grad_impl(jet_mlp *net, const float *X, const float *t, int32_t B, float *grad, float *loss) {
  if (!net || !X || !t || !grad || B < 1) return mlp_fail(net, JET_EINVAL, "bad gradient arguments");
  int rc = ensure_batch(net, B);
  if (rc != JET_OK) return rc;
  rc = forward_into(net, X, B, net->y, true);
  if (rc != JET_OK) return rc;
  hipLaunchKernelGGL(k_mlp_delta, dim3(blocks_for(B, kFwdBlock)), dim3(kFwdBlock), 0, net->stream, net->theta,
                     net->h1, net->h2, net->y, t, B, net->d1, net->d2, net->d3);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for(kParams + 1, 256)), dim3(256), 0, net->stream, net->xs, net->h1,
                     net->h2, net->y, t, net->d1, net->d2, net->d3, B, grad, net->loss);
  MLP_HIP(net, hipGetLastError());
  if (loss) {
    MLP_HIP(net, hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, net->stream));
    MLP_HIP(net, hipStreamSynchronize(net->stream));
  }
  return JET_OK;
}

}  // namespace

namespace jet {

int mlp_infer_one(jet_mlp *net, const float *x, float *y, float *tau) {
  int rc = forward_into(net, x, 1, y, false);
  if (rc != JET_OK) return rc;
  MLP_HIP(net, hipMemcpyAsync(tau, y, sizeof(float), hipMemcpyDeviceToHost, net->stream));
  MLP_HIP(net, hipStreamSynchronize(net->stream));
  return JET_OK;
}

}  // namespace jet

extern "C" {

int jet_mlp_create(jet_mlp **out, uint64_t seed, void *stream) {
  if (!out) return mlp_fail(nullptr, JET_EINVAL, "out is NULL");
  *out = nullptr;
  jet_mlp *net = new jet_mlp();
  net->stream = (hipStream_t)stream;
  float **bufs[] = {&net->theta, &net->m, &net->v, &net->grad};
  for (float **b : bufs)
    if (hipMalloc((void **)b, sizeof(float) * kParams) != hipSuccess) {
      jet_mlp_free(net);
      return mlp_fail(nullptr, JET_ENOMEM, "parameter buffers");
    }
  if (hipMalloc((void **)&net->mean, sizeof(float) * kIn) != hipSuccess ||
      hipMalloc((void **)&net->stdv, sizeof(float) * kIn) != hipSuccess ||
      hipMalloc((void **)&net->loss, sizeof(float)) != hipSuccess) {
    jet_mlp_free(net);
    return mlp_fail(nullptr, JET_ENOMEM, "parameter buffers");
  }
  // He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)), zero biases, identity standardisation
  std::vector<float> th(kParams, 0.0f), mean(kIn, 0.0f), sd(kIn, 1.0f);
  uint64_t s = seed;
  auto fill = [&](int o, int count, int fan_in) {
    const double a = sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) {
      const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
      th[o + i] = (float)((2.0 * u - 1.0) * a);
    }
  };
  fill(oW1, kH * kIn, kIn);
  fill(oW2, kH * kH, kH);
  fill(ow3, kH, kH);
  int rc = jet_mlp_set(net, th.data(), mean.data(), sd.data());
  if (rc != JET_OK) {
    jet_mlp_free(net);
    return rc;
  }
  *out = net;
  return JET_OK;
}

int jet_mlp_set(jet_mlp *net, const float *params, const float *mean, const float *stdv) {
  if (!net) return JET_EINVAL;
  if (stdv)
    for (int i = 0; i < kIn; ++i)
      if (!(stdv[i] > 0.0f)) return mlp_fail(net, JET_EINVAL, "standard deviation must be > 0");
  MLP_HIP(net, hipStreamSynchronize(net->stream));
  if (params) {
    MLP_HIP(net, hipMemcpy(net->theta, params, sizeof(float) * kParams, hipMemcpyHostToDevice));
    MLP_HIP(net, hipMemset(net->m, 0, sizeof(float) * kParams));
    MLP_HIP(net, hipMemset(net->v, 0, sizeof(float) * kParams));
    net->step = 0;
  }
  if (mean) MLP_HIP(net, hipMemcpy(net->mean, mean, sizeof(float) * kIn, hipMemcpyHostToDevice));
  if (stdv) MLP_HIP(net, hipMemcpy(net->stdv, stdv, sizeof(float) * kIn, hipMemcpyHostToDevice));
  return JET_OK;
}

int jet_mlp_get(jet_mlp *net, float *params, float *mean, float *stdv) {
  if (!net) return JET_EINVAL;
  MLP_HIP(net, hipStreamSynchronize(net->stream));
  if (params) MLP_HIP(net, hipMemcpy(params, net->theta, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  if (mean) MLP_HIP(net, hipMemcpy(mean, net->mean, sizeof(float) * kIn, hipMemcpyDeviceToHost));
  if (stdv) MLP_HIP(net, hipMemcpy(stdv, net->stdv, sizeof(float) * kIn, hipMemcpyDeviceToHost));
  return JET_OK;
}

int jet_mlp_forward(jet_mlp *net, const float *X, int32_t B, float *tau) {
  if (!net || !X || !tau || B < 1) return mlp_fail(net, JET_EINVAL, "bad forward arguments");
  return forward_into(net, X, B, tau, false);
}

int jet_mlp_grad(jet_mlp *net, const float *X, const float *t, int32_t B, float *grad, float *loss) {
  return grad_impl(net, X, t, B, grad, loss);
}

int jet_mlp_train_step(jet_mlp *net, const float *X, const float *t, int32_t B, float lr, float *loss) {
  if (!net) return JET_EINVAL;
  if (!(lr > 0.0f)) return mlp_fail(net, JET_EINVAL, "learning rate must be > 0");
  int rc = grad_impl(net, X, t, B, net->grad, nullptr);
  if (rc != JET_OK) return rc;
  net->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - pow(b1, (double)net->step)));
  const float c2 = (float)(1.0 / (1.0 - pow(b2, (double)net->step)));
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(kParams, 256)), dim3(256), 0, net->stream, net->theta, net->m,
                     net->v, net->grad, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  MLP_HIP(net, hipGetLastError());
  if (loss) {
    MLP_HIP(net, hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, net->stream));
    MLP_HIP(net, hipStreamSynchronize(net->stream));
  }
  return JET_OK;
}

int jet_mlp_save(jet_mlp *net, const char *path) {
  if (!net || !path) return JET_EINVAL;
  std::vector<float> buf(kParams + 2 * kIn);
  int rc = jet_mlp_get(net, buf.data(), buf.data() + kParams, buf.data() + kParams + kIn);
  if (rc != JET_OK) return rc;
  FILE *f = fopen(path, "wb");
  if (!f) return mlp_fail(net, JET_EINVAL, std::string("cannot open ") + path);
  const uint32_t head[2] = {0x4d4c5054u /* "TPLM" */, (uint32_t)kParams};
  bool ok = fwrite(head, sizeof head, 1, f) == 1 && fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? JET_OK : mlp_fail(net, JET_EINVAL, std::string("cannot write ") + path);
}

int jet_mlp_load(jet_mlp *net, const char *path) {
  if (!net || !path) return JET_EINVAL;
  FILE *f = fopen(path, "rb");
  if (!f) return mlp_fail(net, JET_EINVAL, std::string("cannot open ") + path);
  uint32_t head[2] = {0, 0};
  std::vector<float> buf(kParams + 2 * kIn);
  const bool ok = fread(head, sizeof head, 1, f) == 1 && head[0] == 0x4d4c5054u && head[1] == (uint32_t)kParams &&
                  fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  fclose(f);
  if (!ok) return mlp_fail(net, JET_EINVAL, std::string("not a temperature network file: ") + path);
  return jet_mlp_set(net, buf.data(), buf.data() + kParams, buf.data() + kParams + kIn);
}

int jet_mlp_free(jet_mlp *net) {
  if (!net) return JET_OK;
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  free_batch(net);
  float *ptrs[] = {net->theta, net->m, net->v, net->grad, net->mean, net->stdv, net->loss};
  for (float *p : ptrs)
    if (p) (void)hipFree(p);
  delete net;
  return JET_OK;
}

const char *jet_mlp_last_error(const jet_mlp *net) { return net ? net->last_error.c_str() : g_mlp_error.c_str(); }

}  // extern "C"
