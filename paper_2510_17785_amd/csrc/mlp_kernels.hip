// The bound-predicting network on the GPU: an MLP n_in -> 64 -> 64 -> 64 ->
// n_out with tanh hidden layers and a linear output, trained by mean squared
// error with Adam (Kingma and Ba 2015).  Inputs are standardised with the
// training-set mean and standard deviation.  Parameters are FP32, in the
// layout W1 (n_in x 64, row-major), b1, W2, b2, W3, b3, W4 (64 x n_out), b4.
//
// The kernels are plain FP32 VALU code: one forward pass costs about 42
// kFLOP per sample, so a training epoch over 1e5 patches is a few GFLOP.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.hpp"

namespace pmgi {
namespace {

constexpr int kH = 64;

__global__ void gather_rows_kernel(const float* X, const int32_t* idx, int B, int K, float* out) {
  const int64_t total = (int64_t)B * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / K), k = (int)(i % K);
    out[i] = X[(int64_t)idx[b] * K + k];
  }
}

__global__ void standardize_kernel(const float* X, int64_t B, int K, const float* mean,
                                   const float* inv_std, float* out) {
  const int64_t total = B * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % K);
    out[i] = (X[i] - mean[k]) * inv_std[k];
  }
}

// per feature: mean and 1/std over the samples (FP64 sums, fixed order)
__global__ __launch_bounds__(256) void mean_std_kernel(const float* X, int64_t n, int K, float* mean,
                                                       float* inv_std) {
  __shared__ double s1[256], s2[256];
  const int k = blockIdx.x;
  double a = 0, b = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = X[i * K + k];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = s1[0] / n;
    const double var = fmax(s2[0] / n - m * m, 0.0);
    const double sd = sqrt(var);
    mean[k] = (float)m;
    inv_std[k] = (float)(sd > 1e-12 * (fabs(m) + 1.0) ? 1.0 / sd : 1.0);
  }
}

// Y[b][j] = act(sum_k X[b][k] W[k][j] + c[j])
__global__ void dense_fwd_kernel(const float* X, int B, int K, const float* W, const float* c,
                                 int N, int tanh_act, float* Y) {
  const int64_t total = (int64_t)B * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / N), j = (int)(i % N);
    const float* x = X + (int64_t)b * K;
    float acc = c[j];
    for (int k = 0; k < K; ++k) acc += x[k] * W[k * N + j];
    Y[i] = tanh_act ? tanhf(acc) : acc;
  }
}

// dY = 2 (Y - T) / (B N); loss partials (sum of squares) per block
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* Y, const float* T, int B, int N,
                                                       float* dY, double* partial) {
  __shared__ double red[256];
  const int64_t total = (int64_t)B * N;
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.0f * d / (float)total;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// loss += sum(partial) / count (one thread, fixed order)
__global__ void loss_accumulate_kernel(const double* partial, int nb, double count, double* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < nb; ++i) s += partial[i];
    *loss += s / count;
  }
}

// dX[b][k] = (sum_j dY[b][j] W[k][j]) (1 - H[b][k]^2)   (H: tanh output of the layer below)
__global__ void dense_bwd_input_kernel(const float* dY, int B, int N, const float* W, int K,
                                       const float* H, float* dX) {
  const int64_t total = (int64_t)B * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / K), k = (int)(i % K);
    const float* d = dY + (int64_t)b * N;
    const float* w = W + (int64_t)k * N;
    float acc = 0;
    for (int j = 0; j < N; ++j) acc += d[j] * w[j];
    const float h = H[i];
    dX[i] = acc * (1.0f - h * h);
  }
}

// gW[k][j] = sum_b X[b][k] dY[b][j], gc[j] = sum_b dY[b][j] (fixed order over b)
__global__ void dense_bwd_weights_kernel(const float* X, const float* dY, int B, int K, int N,
                                         float* gW, float* gc) {
  const int total = (K + 1) * N;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int k = i / N, j = i % N;
    float acc = 0;
    if (k < K) {
      for (int b = 0; b < B; ++b) acc += X[(int64_t)b * K + k] * dY[(int64_t)b * N + j];
      gW[k * N + j] = acc;
    } else {
      for (int b = 0; b < B; ++b) acc += dY[(int64_t)b * N + j];
      gc[j] = acc;
    }
  }
}

__global__ void adam_kernel(float* theta, const float* g, float* m, float* v, int n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// largest |standardised feature| of every sample
__global__ void max_abs_z_kernel(const float* X, int64_t n, int K, const float* mean,
                                 const float* inv_std, float* zmax) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * blockDim.x) {
    float m = 0;
    for (int k = 0; k < K; ++k) m = fmaxf(m, fabsf((X[b * K + k] - mean[k]) * inv_std[k]));
    zmax[b] = m;
  }
}

int grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

// ---------------------------------------------------------------------------

MlpNet::~MlpNet() {
  for (void* p : {(void*)theta, (void*)grad, (void*)m, (void*)v, (void*)mean, (void*)inv_std,
                  (void*)xb, (void*)tb, (void*)xs, (void*)h1, (void*)h2, (void*)h3, (void*)y,
                  (void*)d3, (void*)d2, (void*)d1, (void*)dy, (void*)partial, (void*)loss,
                  (void*)idx})
    if (p) (void)hipFree(p);
}

int64_t MlpNet::offset(int layer) const {
  const int in[4] = {n_in, kH, kH, kH}, out[4] = {kH, kH, kH, n_out};
  int64_t o = 0;
  for (int l = 0; l < layer; ++l) o += (int64_t)in[l] * out[l] + out[l];
  return o;
}

int64_t mlp_param_count(int n_in, int n_out) {
  return (int64_t)n_in * kH + kH + 2 * ((int64_t)kH * kH + kH) + (int64_t)kH * n_out + n_out;
}

hipError_t MlpNet::alloc(int64_t max_batch) {
  auto A = [](auto** p, size_t bytes) { return hipMalloc((void**)p, bytes ? bytes : 8); };
  hipError_t e;
  const size_t P = (size_t)mlp_param_count(n_in, n_out);
  cap = max_batch;
  if ((e = A(&theta, P * 4)) || (e = A(&grad, P * 4)) || (e = A(&m, P * 4)) || (e = A(&v, P * 4)) ||
      (e = A(&mean, n_in * 4)) || (e = A(&inv_std, n_in * 4)) ||
      (e = A(&xb, cap * n_in * 4)) || (e = A(&tb, cap * n_out * 4)) || (e = A(&xs, cap * n_in * 4)) ||
      (e = A(&h1, cap * kH * 4)) || (e = A(&h2, cap * kH * 4)) || (e = A(&h3, cap * kH * 4)) ||
      (e = A(&y, cap * n_out * 4)) || (e = A(&d3, cap * kH * 4)) || (e = A(&d2, cap * kH * 4)) ||
      (e = A(&d1, cap * kH * 4)) || (e = A(&dy, cap * n_out * 4)) || (e = A(&partial, 4096 * 8)) ||
      (e = A(&loss, 8)) || (e = A(&idx, cap * 4)))
    return e;
  return hipSuccess;
}

// forward on standardised inputs xs (B rows), activations in h1..h3, y
hipError_t MlpNet::forward(const float* in_std, int B) {
  const float* W1 = theta + offset(0);
  const float* W2 = theta + offset(1);
  const float* W3 = theta + offset(2);
  const float* W4 = theta + offset(3);
  (void)hipGetLastError();
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(grid_of((int64_t)B * kH)), dim3(256), 0, stream, in_std, B,
                     n_in, W1, W1 + (int64_t)n_in * kH, kH, 1, h1);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(grid_of((int64_t)B * kH)), dim3(256), 0, stream, h1, B, kH,
                     W2, W2 + kH * kH, kH, 1, h2);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(grid_of((int64_t)B * kH)), dim3(256), 0, stream, h2, B, kH,
                     W3, W3 + kH * kH, kH, 1, h3);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(grid_of((int64_t)B * n_out)), dim3(256), 0, stream, h3, B,
                     kH, W4, W4 + kH * n_out, n_out, 0, y);
  return hipGetLastError();
}

// gradient of the mean squared error of the batch (xs standardised, tb targets)
hipError_t MlpNet::backward(const float* in_std, const float* targets, int B) {
  const float* W2 = theta + offset(1);
  const float* W3 = theta + offset(2);
  const float* W4 = theta + offset(3);
  float* g1 = grad + offset(0);
  float* g2 = grad + offset(1);
  float* g3 = grad + offset(2);
  float* g4 = grad + offset(3);
  const int nb = grid_of((int64_t)B * n_out);
  (void)hipGetLastError();
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, stream, y, targets, B, n_out, dy, partial);
  hipLaunchKernelGGL(loss_accumulate_kernel, dim3(1), dim3(1), 0, stream, partial, nb,
                     (double)B * n_out, loss);
  hipLaunchKernelGGL(dense_bwd_weights_kernel, dim3(grid_of((kH + 1) * n_out)), dim3(256), 0, stream,
                     h3, dy, B, kH, n_out, g4, g4 + kH * n_out);
  hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(grid_of((int64_t)B * kH)), dim3(256), 0, stream, dy, B,
                     n_out, W4, kH, h3, d3);
  hipLaunchKernelGGL(dense_bwd_weights_kernel, dim3(grid_of((kH + 1) * kH)), dim3(256), 0, stream, h2,
                     d3, B, kH, kH, g3, g3 + kH * kH);
  hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(grid_of((int64_t)B * kH)), dim3(256), 0, stream, d3, B,
                     kH, W3, kH, h2, d2);
  hipLaunchKernelGGL(dense_bwd_weights_kernel, dim3(grid_of((kH + 1) * kH)), dim3(256), 0, stream, h1,
                     d2, B, kH, kH, g2, g2 + kH * kH);
  hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(grid_of((int64_t)B * kH)), dim3(256), 0, stream, d2, B,
                     kH, W2, kH, h1, d1);
  hipLaunchKernelGGL(dense_bwd_weights_kernel, dim3(grid_of((int64_t)(n_in + 1) * kH)), dim3(256), 0,
                     stream, in_std, d1, B, n_in, kH, g1, g1 + (int64_t)n_in * kH);
  return hipGetLastError();
}

hipError_t MlpNet::standardize(const float* X, int64_t B, float* out) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(standardize_kernel, dim3(grid_of(B * n_in)), dim3(256), 0, stream, X, B, n_in,
                     mean, inv_std, out);
  return hipGetLastError();
}

hipError_t MlpNet::fit_standardizer(const float* X, int64_t n) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(mean_std_kernel, dim3(n_in), dim3(256), 0, stream, X, n, n_in, mean, inv_std);
  return hipGetLastError();
}

hipError_t MlpNet::adam_step(float lr, float b1, float b2, float eps) {
  ++t;
  const float bc1 = 1.0f - std::pow(b1, (float)t), bc2 = 1.0f - std::pow(b2, (float)t);
  const int P = (int)mlp_param_count(n_in, n_out);
  (void)hipGetLastError();
  hipLaunchKernelGGL(adam_kernel, dim3(grid_of(P)), dim3(256), 0, stream, theta, grad, m, v, P, lr, b1,
                     b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t MlpNet::gather(const float* X, const float* T, const int32_t* order, int B) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of((int64_t)B * n_in)), dim3(256), 0, stream, X,
                     order, B, n_in, xb);
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of((int64_t)B * n_out)), dim3(256), 0, stream, T,
                     order, B, n_out, tb);
  return hipGetLastError();
}

hipError_t MlpNet::gather_rows(const float* X, const int32_t* idx, int B, int K, float* out) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of((int64_t)B * K)), dim3(256), 0, stream, X, idx, B,
                     K, out);
  return hipGetLastError();
}

hipError_t MlpNet::max_abs_z(const float* X, int64_t n, float* zmax) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(max_abs_z_kernel, dim3(grid_of(n)), dim3(256), 0, stream, X, n, n_in, mean,
                     inv_std, zmax);
  return hipGetLastError();
}

}  // namespace pmgi
