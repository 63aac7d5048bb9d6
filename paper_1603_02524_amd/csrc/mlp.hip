// Overlap-weight network: forward, backward and Adam kernels (FP32, gfx950).
//
// x (IN) -> tanh(W1 x + b1) (HID) -> tanh(W2 h1 + b2) (HID) -> W3 h2 + b3 (OUT).
// Parameter layout: W1 (HID x IN, row-major), b1, W2 (HID x HID), b2, W3 (OUT x HID), b3.
// Loss L = (1/B) sum_b sum_o (y_bo - t_bo)^2.  All reductions over the batch run
// in a fixed order (one thread per parameter), so gradients are reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/dgmg.h"

void dgmg_set_global_error(const std::string& msg);

namespace {

constexpr int IN = DGMG_MLP_IN, HID = DGMG_MLP_HIDDEN, OUT = DGMG_MLP_OUT;
constexpr int OW1 = 0, OB1 = OW1 + HID * IN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + OUT * HID, NPAR = OB3 + OUT;
static_assert(NPAR == DGMG_MLP_PARAMS, "parameter count");

// One block of HID threads per sample; work holds h1 and h2 (B x 2 HID).
__global__ void __launch_bounds__(HID) k_mlp_forward(const float* __restrict__ p, const float* __restrict__ X,
                                                     int B, float* __restrict__ Y, float* __restrict__ work) {
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= B) return;
  __shared__ float xs[IN], h1[HID], h2[HID];
  if (j < IN) xs[j] = X[(size_t)b * IN + j];
  __syncthreads();
  float a = p[OB1 + j];
  for (int k = 0; k < IN; ++k) a += p[OW1 + j * IN + k] * xs[k];
  h1[j] = tanhf(a);
  __syncthreads();
  a = p[OB2 + j];
  for (int k = 0; k < HID; ++k) a += p[OW2 + j * HID + k] * h1[k];
  h2[j] = tanhf(a);
  work[(size_t)b * 2 * HID + j] = h1[j];
  work[(size_t)b * 2 * HID + HID + j] = h2[j];
  __syncthreads();
  if (j < OUT) {
    float y = p[OB3 + j];
    for (int k = 0; k < HID; ++k) y += p[OW3 + j * HID + k] * h2[k];
    Y[(size_t)b * OUT + j] = y;
  }
}

// Per-sample deltas: scratch holds da1 and da2 (B x 2 HID), dy goes to scratch2 (B x OUT).
__global__ void __launch_bounds__(HID) k_mlp_delta(const float* __restrict__ p, const float* __restrict__ T, int B,
                                                   const float* __restrict__ Y, const float* __restrict__ work,
                                                   float* __restrict__ scratch, float* __restrict__ dyout) {
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= B) return;
  __shared__ float dy[OUT], da2[HID];
  if (j < OUT) {
    dy[j] = 2.0f * (Y[(size_t)b * OUT + j] - T[(size_t)b * OUT + j]) / (float)B;
    dyout[(size_t)b * OUT + j] = dy[j];
  }
  __syncthreads();
  const float h2 = work[(size_t)b * 2 * HID + HID + j];
  float s = 0.f;
  for (int o = 0; o < OUT; ++o) s += dy[o] * p[OW3 + o * HID + j];
  da2[j] = s * (1.0f - h2 * h2);
  scratch[(size_t)b * 2 * HID + HID + j] = da2[j];
  __syncthreads();
  const float h1 = work[(size_t)b * 2 * HID + j];
  s = 0.f;
  for (int k = 0; k < HID; ++k) s += da2[k] * p[OW2 + k * HID + j];
  scratch[(size_t)b * 2 * HID + j] = s * (1.0f - h1 * h1);
}

// One thread per parameter: sum over the batch in sample order.
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ X, int B, const float* __restrict__ work,
                                                  const float* __restrict__ scratch, const float* __restrict__ dy,
                                                  float* __restrict__ g) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NPAR) return;
  float s = 0.f;
  if (q < OB1) {  // W1[j][k] = sum da1[b][j] x[b][k]
    const int j = q / IN, k = q % IN;
    for (int b = 0; b < B; ++b) s += scratch[(size_t)b * 2 * HID + j] * X[(size_t)b * IN + k];
  } else if (q < OW2) {
    const int j = q - OB1;
    for (int b = 0; b < B; ++b) s += scratch[(size_t)b * 2 * HID + j];
  } else if (q < OB2) {  // W2[j][k] = sum da2[b][j] h1[b][k]
    const int r = q - OW2, j = r / HID, k = r % HID;
    for (int b = 0; b < B; ++b) s += scratch[(size_t)b * 2 * HID + HID + j] * work[(size_t)b * 2 * HID + k];
  } else if (q < OW3) {
    const int j = q - OB2;
    for (int b = 0; b < B; ++b) s += scratch[(size_t)b * 2 * HID + HID + j];
  } else if (q < OB3) {  // W3[o][k] = sum dy[b][o] h2[b][k]
    const int r = q - OW3, o = r / HID, k = r % HID;
    for (int b = 0; b < B; ++b) s += dy[(size_t)b * OUT + o] * work[(size_t)b * 2 * HID + HID + k];
  } else {
    const int o = q - OB3;
    for (int b = 0; b < B; ++b) s += dy[(size_t)b * OUT + o];
  }
  g[q] = s;
}

__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int n, float c1,
                                                  float c2, float lr, float b1, float b2, float eps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.0f - b1) * gq;
  const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

int launch_status() { return hipGetLastError() == hipSuccess ? DGMG_OK : DGMG_EHIP; }

// Work area of dgmg_mlp_forward_noalloc: the hidden activations h1, h2 of up to
// DGMG_MLP_NOALLOC_MAX_ROWS samples (4 MiB).  Every GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name is
// only a stand-in: kernels receive the device address looked up once per device
// with hipGetSymbolAddress (mlp_fwd_scratch_ptr below).
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) float mlp_fwd_scratch[(size_t)DGMG_MLP_NOALLOC_MAX_ROWS * 2 * HID];

std::mutex g_scratch_mu;
float* g_scratch_dev[MAX_DEVICES] = {};

// Device address of this device's mlp_fwd_scratch, looked up with the device
// current on its first use and kept per device.
int mlp_fwd_scratch_ptr(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    dgmg_set_global_error(std::string("mlp_forward_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    return DGMG_EHIP;
  }
  if (dev < 0 || dev >= MAX_DEVICES) {
    dgmg_set_global_error("mlp_forward_noalloc: device index beyond the supported 64");
    return DGMG_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(mlp_fwd_scratch));
    if (e != hipSuccess || !p) {
      dgmg_set_global_error(std::string("mlp_forward_noalloc: hipGetSymbolAddress: ") +
                            (e != hipSuccess ? hipGetErrorString(e) : "null address"));
      return DGMG_EHIP;
    }
    g_scratch_dev[dev] = (float*)p;
  }
  *out = g_scratch_dev[dev];
  return DGMG_OK;
}

}  // namespace

extern "C" {

int dgmg_mlp_param_count(void) { return NPAR; }

int dgmg_mlp_forward(const float* params, const float* X, int B, float* Y, float* work, void* stream) {
  if (!params || !X || !Y || !work || B < 0) return DGMG_EINVAL;
  if (B == 0) return DGMG_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(HID), 0, (hipStream_t)stream, params, X, B, Y, work);
  return launch_status();
}

int dgmg_mlp_forward_noalloc(const float* params, const float* X, int B, float* Y, void* stream) {
  if (!params || !X || !Y || B < 0) {
    dgmg_set_global_error("mlp_forward_noalloc: null pointer or negative row count");
    return DGMG_EINVAL;
  }
  if (B > DGMG_MLP_NOALLOC_MAX_ROWS) {
    dgmg_set_global_error("mlp_forward_noalloc: " + std::to_string(B) + " rows exceed the maximum of " +
                          std::to_string(DGMG_MLP_NOALLOC_MAX_ROWS) + " (use dgmg_mlp_forward with a work buffer)");
    return DGMG_EINVAL;
  }
  if (B == 0) return DGMG_OK;
  float* work = nullptr;
  int rc = mlp_fwd_scratch_ptr(&work);
  if (rc) return rc;
  hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(HID), 0, (hipStream_t)stream, params, X, B, Y, work);
  return launch_status();
}

int dgmg_mlp_backward(const float* params, const float* X, const float* T, int B, const float* Y,
                      const float* work, float* grad, float* scratch, void* stream) {
  if (!params || !X || !T || !Y || !work || !grad || !scratch || B < 1) return DGMG_EINVAL;
  float* dy = scratch + (size_t)B * 2 * HID;
  hipLaunchKernelGGL(k_mlp_delta, dim3(B), dim3(HID), 0, (hipStream_t)stream, params, T, B, Y, work, scratch, dy);
  hipLaunchKernelGGL(k_mlp_grad, dim3((NPAR + 255) / 256), dim3(256), 0, (hipStream_t)stream, X, B, work, scratch,
                     dy, grad);
  return launch_status();
}

int dgmg_mlp_adam(float* params, const float* grad, float* m, float* v, int n, int t, float lr, float b1,
                  float b2, float eps, void* stream) {
  if (!params || !grad || !m || !v || n < 0 || t < 1) return DGMG_EINVAL;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, n,
                     c1, c2, lr, b1, b2, eps);
  return launch_status();
}

}  // extern "C"
