// costmodel.hip -- the learned region-cost model: a 12 -> 64 -> 64 -> 1 ReLU
// perceptron in FP32 with its own inference, gradient and Adam kernels.
//
// Paper, Section "Performance": the elapsed time of a run is set by its most difficult
// regions, so a scheduler that knows in advance which regions are expensive can start
// them first and pack similar ones together. The model maps 12 features of a region's
// initial surface to the log of the lattice steps the region needs; the scheduler only
// orders and groups regions by it, so results never depend on it.
//
// Parameter block (FP32, 5057 values, row-major):
//   W1[64][12] at 0, b1[64] at 768, W2[64][64] at 832, b2[64] at 4928,
//   w3[64] at 4992, b3 at 5056.
// Optional input normalisation norm[24]: x' = (x - norm[0..11]) * norm[12..23].
// Forward: h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3.
// Loss: mean over the n samples of (y - target)^2.
// Adam (Kingma and Ba, 2015) with bias-corrected moments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "internal.h"
#include "semipar.h"

namespace {

constexpr int NI = SEMIPAR_MLP_IN;
constexpr int NH = SEMIPAR_MLP_HIDDEN;
constexpr int NP = SEMIPAR_MLP_PARAMS;
constexpr int O_W1 = 0, O_B1 = NH * NI, O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH,
              O_W3 = O_B2 + NH, O_B3 = O_W3 + NH;
static_assert(O_B3 + 1 == NP, "parameter layout");

constexpr int FWD_NT = 256;
constexpr int GB = 32;  // samples per gradient block (LDS: params + 6 x GB x 64 floats)
constexpr int GRAD_NT = 256;
constexpr int64_t MAX_SAMPLES = (int64_t)1 << 24;

__device__ __forceinline__ void load_params(const float* __restrict__ p, float* sp) {
  for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = p[i];
}

__device__ __forceinline__ void normalise(const float* __restrict__ x, const float* norm,
                                          float* xo) {
  for (int j = 0; j < NI; ++j) xo[j] = norm ? (x[j] - norm[j]) * norm[NI + j] : x[j];
}

// forward of one sample; h1, h2 receive the post-activation hidden layers
__device__ __forceinline__ float forward1(const float* sp, const float* xn, float* h1, float* h2) {
  for (int i = 0; i < NH; ++i) {
    float a = sp[O_B1 + i];
    for (int j = 0; j < NI; ++j) a += sp[O_W1 + i * NI + j] * xn[j];
    h1[i] = a > 0.f ? a : 0.f;
  }
  for (int i = 0; i < NH; ++i) {
    float a = sp[O_B2 + i];
    for (int j = 0; j < NH; ++j) a += sp[O_W2 + i * NH + j] * h1[j];
    h2[i] = a > 0.f ? a : 0.f;
  }
  float y = sp[O_B3];
  for (int i = 0; i < NH; ++i) y += sp[O_W3 + i] * h2[i];
  return y;
}

__global__ __launch_bounds__(FWD_NT) void k_mlp_forward(const float* __restrict__ params,
                                                        const float* __restrict__ norm,
                                                        const float* __restrict__ x, int64_t n,
                                                        float* __restrict__ y) {
  __shared__ float sp[NP];
  load_params(params, sp);
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * FWD_NT + threadIdx.x;
  if (s >= n) return;
  float xn[NI], h1[NH], h2[NH];
  normalise(x + NI * s, norm, xn);
  y[s] = forward1(sp, xn, h1, h2);
}

// Per block of GB samples: the block's part of the gradient of the loss and of the
// loss itself, written to part[block][0..NP] (the loss at index NP).
__global__ __launch_bounds__(GRAD_NT) void k_mlp_grad(const float* __restrict__ params,
                                                      const float* __restrict__ norm,
                                                      const float* __restrict__ x,
                                                      const float* __restrict__ target, int64_t n,
                                                      float* __restrict__ part) {
  __shared__ float sp[NP];
  __shared__ float sx[GB][NI];
  __shared__ float sh1[GB][NH];
  __shared__ float sh2[GB][NH];
  __shared__ float sd1[GB][NH];  // dL/d(pre-activation of layer 1)
  __shared__ float sd2[GB][NH];  // dL/d(pre-activation of layer 2)
  __shared__ float sdy[GB];      // dL/dy
  __shared__ float sloss[GB];
  load_params(params, sp);
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * GB;
  if (t < GB) {
    const int64_t s = s0 + t;
    float xn[NI], h1[NH], h2[NH];
    float dy = 0.f, l = 0.f;
    if (s < n) {
      normalise(x + NI * s, norm, xn);
      const float y = forward1(sp, xn, h1, h2);
      const float e = y - target[s];
      l = e * e / (float)n;
      dy = 2.f * e / (float)n;
    } else {
      for (int j = 0; j < NI; ++j) xn[j] = 0.f;
      for (int i = 0; i < NH; ++i) h1[i] = h2[i] = 0.f;
    }
    for (int j = 0; j < NI; ++j) sx[t][j] = xn[j];
    for (int i = 0; i < NH; ++i) {
      sh1[t][i] = h1[i];
      sh2[t][i] = h2[i];
      sd2[t][i] = h2[i] > 0.f ? dy * sp[O_W3 + i] : 0.f;
    }
    for (int j = 0; j < NH; ++j) {
      float a = 0.f;
      for (int i = 0; i < NH; ++i) a += sp[O_W2 + i * NH + j] * sd2[t][i];
      sd1[t][j] = h1[j] > 0.f ? a : 0.f;
    }
    sdy[t] = dy;
    sloss[t] = l;
  }
  __syncthreads();
  float* out = part + (int64_t)blockIdx.x * (NP + 1);
  for (int p = t; p <= NP; p += GRAD_NT) {
    float g = 0.f;
    if (p < O_B1) {
      const int i = p / NI, j = p % NI;
      for (int q = 0; q < GB; ++q) g += sd1[q][i] * sx[q][j];
    } else if (p < O_W2) {
      const int i = p - O_B1;
      for (int q = 0; q < GB; ++q) g += sd1[q][i];
    } else if (p < O_B2) {
      const int i = (p - O_W2) / NH, j = (p - O_W2) % NH;
      for (int q = 0; q < GB; ++q) g += sd2[q][i] * sh1[q][j];
    } else if (p < O_W3) {
      const int i = p - O_B2;
      for (int q = 0; q < GB; ++q) g += sd2[q][i];
    } else if (p < O_B3) {
      const int i = p - O_W3;
      for (int q = 0; q < GB; ++q) g += sdy[q] * sh2[q][i];
    } else if (p == O_B3) {
      for (int q = 0; q < GB; ++q) g += sdy[q];
    } else {
      for (int q = 0; q < GB; ++q) g += sloss[q];
    }
    out[p] = g;
  }
}

// Sum of the block parts in block order (deterministic): grad[0..NP), loss.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int nb,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > NP) return;
  float g = 0.f;
  for (int b = 0; b < nb; ++b) g += part[(int64_t)b * (NP + 1) + p];
  if (p < NP)
    grad[p] = g;
  else if (loss)
    *loss = g;
}

// One Adam step at step number `step` (1-based).
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ p, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ g, float lr,
                                                  float beta1, float beta2, float eps, float c1,
                                                  float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NP) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * (gi * gi);
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1;
  const float vh = vi / c2;
  p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

int grad_blocks(int64_t n) { return (int)((n + GB - 1) / GB); }

// Per-block gradient parts of semipar_mlp_loss_grad_noalloc: a fixed array in device
// memory, one per GPU the library runs on, held until the process ends. Every call on
// one GPU shares it (each call overwrites the parts of its own blocks before reading
// them, so nothing needs clearing between calls).
constexpr int64_t NOALLOC_MAX_SAMPLES = SEMIPAR_MLP_NOALLOC_MAX;
constexpr int NOALLOC_MAX_BLOCKS = (int)((NOALLOC_MAX_SAMPLES + GB - 1) / GB);
__device__ __align__(256) float scratch[(size_t)NOALLOC_MAX_BLOCKS * (NP + 1)];

// Device address of `scratch` on each GPU (the host-side name is only a stand-in),
// looked up once per device with that device current.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_on_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SEMIPAR_E_HIP;
  if (dev < 0 || dev >= MAX_DEVICES) return SEMIPAR_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      spi::set_error("hipGetSymbolAddress(scratch) failed in semipar_mlp_loss_grad_noalloc");
      return SEMIPAR_E_HIP;
    }
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return SEMIPAR_OK;
}

struct Scratch {
  float* part = nullptr;
  float* grad = nullptr;
  ~Scratch() {
    if (part) (void)hipFree(part);
    if (grad) (void)hipFree(grad);
  }
};

int launch_grad(const float* params, const float* norm, const float* x, const float* target,
                int64_t n, float* part, float* grad, float* loss, hipStream_t s) {
  const int nb = grad_blocks(n);
  k_mlp_grad<<<nb, GRAD_NT, 0, s>>>(params, norm, x, target, n, part);
  k_mlp_reduce<<<(NP + 1 + 255) / 256, 256, 0, s>>>(part, nb, grad, loss);
  return hipGetLastError() == hipSuccess ? SEMIPAR_OK : SEMIPAR_E_HIP;
}

}  // namespace

extern "C" {

int semipar_mlp_forward(const float* params, const float* norm, const float* x, int64_t n,
                        float* y, void* stream) {
  spi::begin_call();
  if (!params || n < 0 || n > MAX_SAMPLES || (n > 0 && (!x || !y))) return SEMIPAR_E_ARG;
  if (n == 0) return SEMIPAR_OK;
  hipStream_t s = (hipStream_t)stream;
  k_mlp_forward<<<(int)((n + FWD_NT - 1) / FWD_NT), FWD_NT, 0, s>>>(params, norm, x, n, y);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return SEMIPAR_E_HIP;
  return SEMIPAR_OK;
}

int semipar_mlp_loss_grad(const float* params, const float* norm, const float* x,
                          const float* target, int64_t n, float* grad, float* loss,
                          void* stream) {
  spi::begin_call();
  if (!params || !grad || n <= 0 || n > MAX_SAMPLES || !x || !target) return SEMIPAR_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  Scratch w;
  if (hipMalloc(&w.part, sizeof(float) * (NP + 1) * (size_t)grad_blocks(n)) != hipSuccess)
    return SEMIPAR_E_OOM;
  int rc = launch_grad(params, norm, x, target, n, w.part, grad, loss, s);
  if (rc == SEMIPAR_OK && hipStreamSynchronize(s) != hipSuccess) rc = SEMIPAR_E_HIP;
  return rc;
}

int semipar_mlp_loss_grad_noalloc(const float* params, const float* norm, const float* x,
                                  const float* target, int64_t n, float* grad, float* loss,
                                  void* stream) {
  spi::begin_call();
  if (!params || !grad || n <= 0 || !x || !target) return SEMIPAR_E_ARG;
  if (n > NOALLOC_MAX_SAMPLES) {
    spi::set_error("semipar_mlp_loss_grad_noalloc: more samples than its fixed scratch "
                   "holds (SEMIPAR_MLP_NOALLOC_MAX)");
    return SEMIPAR_E_ARG;
  }
  float* part = nullptr;
  int rc = scratch_on_current_device(&part);
  if (rc != SEMIPAR_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = launch_grad(params, norm, x, target, n, part, grad, loss, s);
  if (rc == SEMIPAR_OK && hipStreamSynchronize(s) != hipSuccess) rc = SEMIPAR_E_HIP;
  return rc;
}

int semipar_mlp_adam_step(float* params, float* m, float* v, const float* grad, int64_t step,
                          float lr, float beta1, float beta2, float eps, void* stream) {
  spi::begin_call();
  if (!params || !m || !v || !grad || step < 1) return SEMIPAR_E_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return SEMIPAR_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  k_mlp_adam<<<(NP + 255) / 256, 256, 0, s>>>(params, m, v, grad, lr, beta1, beta2, eps, c1, c2);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return SEMIPAR_E_HIP;
  return SEMIPAR_OK;
}

int semipar_mlp_train(float* params, float* m, float* v, const float* norm, const float* x,
                      const float* target, int64_t n, int32_t iters, int64_t step0, float lr,
                      float* loss_host, void* stream) {
  spi::begin_call();
  if (!params || !m || !v || !x || !target || n <= 0 || n > MAX_SAMPLES || iters < 0 || step0 < 0)
    return SEMIPAR_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  Scratch w;
  float* dloss = nullptr;
  if (hipMalloc(&w.part, sizeof(float) * (NP + 1) * (size_t)grad_blocks(n)) != hipSuccess ||
      hipMalloc(&w.grad, sizeof(float) * NP) != hipSuccess ||
      hipMalloc(&dloss, sizeof(float) * ((size_t)iters + 1)) != hipSuccess) {
    if (dloss) (void)hipFree(dloss);
    return SEMIPAR_E_OOM;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  int rc = SEMIPAR_OK;
  for (int32_t it = 0; it < iters && rc == SEMIPAR_OK; ++it) {
    rc = launch_grad(params, norm, x, target, n, w.part, w.grad, dloss + it, s);
    const int64_t step = step0 + it + 1;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    k_mlp_adam<<<(NP + 255) / 256, 256, 0, s>>>(params, m, v, w.grad, lr, b1, b2, eps, c1, c2);
    if (hipGetLastError() != hipSuccess) rc = SEMIPAR_E_HIP;
  }
  // loss at the final parameters
  if (rc == SEMIPAR_OK) rc = launch_grad(params, norm, x, target, n, w.part, w.grad, dloss + iters, s);
  if (rc == SEMIPAR_OK && loss_host &&
      hipMemcpyAsync(loss_host, dloss, sizeof(float) * ((size_t)iters + 1), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK && hipStreamSynchronize(s) != hipSuccess) rc = SEMIPAR_E_HIP;
  (void)hipFree(dloss);
  return rc;
}

int semipar_mlp_norm(const float* x, int64_t n, float* norm) {
  spi::begin_call();
  if (!x || !norm || n <= 0) return SEMIPAR_E_ARG;
  for (int j = 0; j < NI; ++j) {
    double mu = 0.0, m2 = 0.0;
    for (int64_t s = 0; s < n; ++s) mu += x[NI * s + j];
    mu /= (double)n;
    for (int64_t s = 0; s < n; ++s) {
      const double d = x[NI * s + j] - mu;
      m2 += d * d;
    }
    const double sd = std::sqrt(m2 / (double)n);
    norm[j] = (float)mu;
    norm[NI + j] = sd > 1e-6 ? (float)(1.0 / sd) : 1.f;
  }
  return SEMIPAR_OK;
}

}  // extern "C"
