// Training and inference kernels of the per-level scheduler model (FP32 MLP
// 6 -> 32 -> 32 -> 4, ReLU, MSE loss, Adam).  Not in the paper: the model
// picks each level's kernel variant from frontier features.
//
// A training step is two kernels with a fixed summation order, so training is
// deterministic: one thread per sample runs the forward and backward passes
// and stores its activations and deltas; then one thread per parameter sums
// that parameter's gradient over the samples in order and applies Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace ss {

namespace {

constexpr int kH = 32;
constexpr int kOutN = kVariants;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kFeatures;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kOutN * kH;
static_assert(kOffB3 + kOutN == kModelSize, "model layout");
// per-sample record: h1[32], h2[32], dh1[32], dh2[32], dout[4]
constexpr int kRec = 4 * kH + kOutN;

__global__ void mlp_fwd_bwd(const float* __restrict__ W, const float* __restrict__ X,
                            const float* __restrict__ Y, int64_t n, float* __restrict__ rec,
                            float* __restrict__ sample_loss, float* __restrict__ scores) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kFeatures], h1[kH], h2[kH], out[kOutN];
  for (int f = 0; f < kFeatures; ++f) x[f] = X[s * kFeatures + f];
  for (int i = 0; i < kH; ++i) {
    float a = W[kOffB1 + i];
    for (int f = 0; f < kFeatures; ++f) a += W[kOffW1 + i * kFeatures + f] * x[f];
    h1[i] = a > 0.f ? a : 0.f;
  }
  for (int j = 0; j < kH; ++j) {
    float a = W[kOffB2 + j];
    for (int i = 0; i < kH; ++i) a += W[kOffW2 + j * kH + i] * h1[i];
    h2[j] = a > 0.f ? a : 0.f;
  }
  for (int o = 0; o < kOutN; ++o) {
    float a = W[kOffB3 + o];
    for (int j = 0; j < kH; ++j) a += W[kOffW3 + o * kH + j] * h2[j];
    out[o] = a;
  }
  if (scores)
    for (int o = 0; o < kOutN; ++o) scores[s * kOutN + o] = out[o];
  if (!Y) return;
  // L = (1 / 4N) sum (out - y)^2
  const float scale = 2.0f / (float)(kOutN * n);
  float dout[kOutN], loss = 0.f;
  for (int o = 0; o < kOutN; ++o) {
    const float e = out[o] - Y[s * kOutN + o];
    loss += e * e;
    dout[o] = scale * e;
  }
  sample_loss[s] = loss;
  float dh2[kH], dh1[kH];
  for (int j = 0; j < kH; ++j) {
    float a = 0.f;
    for (int o = 0; o < kOutN; ++o) a += W[kOffW3 + o * kH + j] * dout[o];
    dh2[j] = h2[j] > 0.f ? a : 0.f;
  }
  for (int i = 0; i < kH; ++i) {
    float a = 0.f;
    for (int j = 0; j < kH; ++j) a += W[kOffW2 + j * kH + i] * dh2[j];
    dh1[i] = h1[i] > 0.f ? a : 0.f;
  }
  float* r = rec + s * kRec;
  for (int i = 0; i < kH; ++i) {
    r[i] = h1[i];
    r[kH + i] = h2[i];
    r[2 * kH + i] = dh1[i];
    r[3 * kH + i] = dh2[i];
  }
  for (int o = 0; o < kOutN; ++o) r[4 * kH + o] = dout[o];
}

// Gradient of parameter p summed over samples in order; optional Adam step.
// Thread kModelSize sums the loss.
__global__ void mlp_reduce(float* __restrict__ W, const float* __restrict__ X,
                           const float* __restrict__ rec, const float* __restrict__ sample_loss,
                           int64_t n, float* __restrict__ grad, float* __restrict__ loss_out,
                           float* __restrict__ m1, float* __restrict__ m2, int32_t step, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == kModelSize) {
    float l = 0.f;
    for (int64_t s = 0; s < n; ++s) l += sample_loss[s];
    *loss_out = l / (float)(kOutN * n);
    return;
  }
  if (p > kModelSize) return;
  float gsum = 0.f;
  if (p < kOffB1) {
    const int i = p / kFeatures, f = p % kFeatures;
    for (int64_t s = 0; s < n; ++s) gsum += rec[s * kRec + 2 * kH + i] * X[s * kFeatures + f];
  } else if (p < kOffW2) {
    const int i = p - kOffB1;
    for (int64_t s = 0; s < n; ++s) gsum += rec[s * kRec + 2 * kH + i];
  } else if (p < kOffB2) {
    const int j = (p - kOffW2) / kH, i = (p - kOffW2) % kH;
    for (int64_t s = 0; s < n; ++s) gsum += rec[s * kRec + 3 * kH + j] * rec[s * kRec + i];
  } else if (p < kOffW3) {
    const int j = p - kOffB2;
    for (int64_t s = 0; s < n; ++s) gsum += rec[s * kRec + 3 * kH + j];
  } else if (p < kOffB3) {
    const int o = (p - kOffW3) / kH, j = (p - kOffW3) % kH;
    for (int64_t s = 0; s < n; ++s) gsum += rec[s * kRec + 4 * kH + o] * rec[s * kRec + kH + j];
  } else {
    const int o = p - kOffB3;
    for (int64_t s = 0; s < n; ++s) gsum += rec[s * kRec + 4 * kH + o];
  }
  if (grad) grad[p] = gsum;
  if (m1) {  // Adam
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float a = b1 * m1[p] + (1.f - b1) * gsum;
    const float b = b2 * m2[p] + (1.f - b2) * gsum * gsum;
    m1[p] = a;
    m2[p] = b;
    const float ah = a / (1.f - powf(b1, (float)step));
    const float bh = b / (1.f - powf(b2, (float)step));
    W[p] -= lr * ah / (sqrtf(bh) + eps);
  }
}

struct DeviceBufs {
  float *W = nullptr, *X = nullptr, *Y = nullptr, *rec = nullptr, *sl = nullptr, *grad = nullptr,
        *loss = nullptr, *m1 = nullptr, *m2 = nullptr, *scores = nullptr;
  ~DeviceBufs() {
    for (float* p : {W, X, Y, rec, sl, grad, loss, m1, m2, scores})
      if (p) (void)hipFree(p);
  }
};

int dmalloc(float** p, int64_t count) {
  if (count < 1) count = 1;
  if (hipMalloc(p, sizeof(float) * (size_t)count) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(SS_ENOMEM, "scheduler: device allocation failed");
  }
  return SS_OK;
}

int hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return set_error(SS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return SS_OK;
}

// Seeded He-uniform start: U(-sqrt(6/fan_in), sqrt(6/fan_in)), zero biases.
void seeded_init(uint64_t seed, float* w) {
  uint64_t state = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  auto next = [&]() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  std::memset(w, 0, sizeof(float) * kModelSize);
  auto fill = [&](int off, int count, int fan_in) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) w[off + i] = (float)((2.0 * next() - 1.0) * lim);
  };
  fill(kOffW1, kH * kFeatures, kFeatures);
  fill(kOffW2, kH * kH, kH);
  fill(kOffW3, kOutN * kH, kH);
}

}  // namespace

}  // namespace ss

using namespace ss;

extern "C" {

int slimsell_sched_forward(const float* weights, const float* x, int64_t n, float* scores,
                           void* stream) {
  if (!weights || !x || !scores || n < 0) return set_error(SS_EINVAL, "bad argument");
  if (n == 0) return SS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  DeviceBufs b;
  int rc;
  if ((rc = dmalloc(&b.W, kModelSize)) || (rc = dmalloc(&b.X, n * kFeatures)) ||
      (rc = dmalloc(&b.scores, n * kOutN)))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(b.W, weights, sizeof(float) * kModelSize,
                                     hipMemcpyHostToDevice, st), "upload")) ||
      (rc = hip_check(hipMemcpyAsync(b.X, x, sizeof(float) * n * kFeatures, hipMemcpyHostToDevice,
                                     st), "upload")))
    return rc;
  mlp_fwd_bwd<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(b.W, b.X, nullptr, n, nullptr, nullptr,
                                                            b.scores);
  if ((rc = hip_check(hipGetLastError(), "mlp_fwd_bwd"))) return rc;
  if ((rc = hip_check(hipMemcpyAsync(scores, b.scores, sizeof(float) * n * kOutN,
                                     hipMemcpyDeviceToHost, st), "download")))
    return rc;
  return hip_check(hipStreamSynchronize(st), "scheduler forward");
}

int slimsell_sched_grad(const float* weights, const float* x, const float* y, int64_t n,
                        float* grad, float* loss, void* stream) {
  if (!weights || !x || !y || !grad || !loss || n < 1) return set_error(SS_EINVAL, "bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DeviceBufs b;
  int rc;
  if ((rc = dmalloc(&b.W, kModelSize)) || (rc = dmalloc(&b.X, n * kFeatures)) ||
      (rc = dmalloc(&b.Y, n * kOutN)) || (rc = dmalloc(&b.rec, n * kRec)) ||
      (rc = dmalloc(&b.sl, n)) || (rc = dmalloc(&b.grad, kModelSize)) || (rc = dmalloc(&b.loss, 1)))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(b.W, weights, sizeof(float) * kModelSize,
                                     hipMemcpyHostToDevice, st), "upload")) ||
      (rc = hip_check(hipMemcpyAsync(b.X, x, sizeof(float) * n * kFeatures, hipMemcpyHostToDevice,
                                     st), "upload")) ||
      (rc = hip_check(hipMemcpyAsync(b.Y, y, sizeof(float) * n * kOutN, hipMemcpyHostToDevice, st),
                      "upload")))
    return rc;
  mlp_fwd_bwd<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(b.W, b.X, b.Y, n, b.rec, b.sl, nullptr);
  mlp_reduce<<<(kModelSize + 1 + 255) / 256, 256, 0, st>>>(b.W, b.X, b.rec, b.sl, n, b.grad, b.loss,
                                                          nullptr, nullptr, 0, 0.f);
  if ((rc = hip_check(hipGetLastError(), "scheduler gradient"))) return rc;
  if ((rc = hip_check(hipMemcpyAsync(grad, b.grad, sizeof(float) * kModelSize,
                                     hipMemcpyDeviceToHost, st), "download")) ||
      (rc = hip_check(hipMemcpyAsync(loss, b.loss, sizeof(float), hipMemcpyDeviceToHost, st),
                      "download")))
    return rc;
  return hip_check(hipStreamSynchronize(st), "scheduler gradient");
}

int slimsell_sched_train(const float* x, const float* y, int64_t n, int32_t steps, float lr,
                         uint64_t seed, const float* init, float* weights_out, float* loss_out,
                         void* stream) {
  if (!x || !y || !weights_out || n < 1 || steps < 0 || !(lr > 0.f))
    return set_error(SS_EINVAL, "bad argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<float> w0(kModelSize);
  if (init)
    std::memcpy(w0.data(), init, sizeof(float) * kModelSize);
  else
    seeded_init(seed, w0.data());
  DeviceBufs b;
  int rc;
  if ((rc = dmalloc(&b.W, kModelSize)) || (rc = dmalloc(&b.X, n * kFeatures)) ||
      (rc = dmalloc(&b.Y, n * kOutN)) || (rc = dmalloc(&b.rec, n * kRec)) ||
      (rc = dmalloc(&b.sl, n)) || (rc = dmalloc(&b.loss, steps > 0 ? steps : 1)) ||
      (rc = dmalloc(&b.m1, kModelSize)) || (rc = dmalloc(&b.m2, kModelSize)))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(b.W, w0.data(), sizeof(float) * kModelSize,
                                     hipMemcpyHostToDevice, st), "upload")) ||
      (rc = hip_check(hipMemcpyAsync(b.X, x, sizeof(float) * n * kFeatures, hipMemcpyHostToDevice,
                                     st), "upload")) ||
      (rc = hip_check(hipMemcpyAsync(b.Y, y, sizeof(float) * n * kOutN, hipMemcpyHostToDevice, st),
                      "upload")) ||
      (rc = hip_check(hipMemsetAsync(b.m1, 0, sizeof(float) * kModelSize, st), "clear")) ||
      (rc = hip_check(hipMemsetAsync(b.m2, 0, sizeof(float) * kModelSize, st), "clear")))
    return rc;
  for (int32_t t = 1; t <= steps; ++t) {
    mlp_fwd_bwd<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(b.W, b.X, b.Y, n, b.rec, b.sl,
                                                              nullptr);
    mlp_reduce<<<(kModelSize + 1 + 255) / 256, 256, 0, st>>>(b.W, b.X, b.rec, b.sl, n, nullptr,
                                                            b.loss + (t - 1), b.m1, b.m2, t, lr);
  }
  if ((rc = hip_check(hipGetLastError(), "scheduler training"))) return rc;
  if ((rc = hip_check(hipMemcpyAsync(weights_out, b.W, sizeof(float) * kModelSize,
                                     hipMemcpyDeviceToHost, st), "download")))
    return rc;
  if (loss_out && steps > 0 &&
      (rc = hip_check(hipMemcpyAsync(loss_out, b.loss, sizeof(float) * steps,
                                     hipMemcpyDeviceToHost, st), "download")))
    return rc;
  return hip_check(hipStreamSynchronize(st), "scheduler training");
}

}  // extern "C"
