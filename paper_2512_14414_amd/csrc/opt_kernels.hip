// Device kernels of the learned line-search surrogate (a two-hidden-layer
// GELU perceptron, trained with Adam) and of the L-BFGS vector algebra.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "opt_kernels.h"

namespace optk {

static unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the i-th output of the
// generator seeded with ``seed`` is mix(seed + (i + 1) * golden gamma).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// p[i] = (2u - 1) * bound with u = (splitmix64(seed, offset + i) >> 11) * 2^-53, rounded to float.
__global__ void uniform_init_kernel(float* p, int64_t n, uint64_t seed, int64_t offset, double bound) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double u = (double)(splitmix64(seed, (uint64_t)(offset + i)) >> 11) * 0x1.0p-53;
    p[i] = (float)((2.0 * u - 1.0) * bound);
  }
}

hipError_t launch_uniform_init(float* p, int64_t n, uint64_t seed, int64_t offset, double bound, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  uniform_init_kernel<<<grid_for(n), 256, 0, s>>>(p, n, seed, offset, bound);
  return hipGetLastError();
}

// The same draw in float64: p[i] = (2u - 1) * bound (test matrices of the randomized projector SVD).
__global__ void uniform_init_f64_kernel(double* p, int64_t n, uint64_t seed, int64_t offset, double bound) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double u = (double)(splitmix64(seed, (uint64_t)(offset + i)) >> 11) * 0x1.0p-53;
    p[i] = (2.0 * u - 1.0) * bound;
  }
}

hipError_t launch_uniform_init_f64(double* p, int64_t n, uint64_t seed, int64_t offset, double bound,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  uniform_init_f64_kernel<<<grid_for(n), 256, 0, s>>>(p, n, seed, offset, bound);
  return hipGetLastError();
}

// GELU with the exact error function: gelu(z) = z/2 (1 + erf(z / sqrt 2)).
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z[b][w] += bias[w]; A[b][w] = gelu(Z[b][w])  (A may be null: identity output layer)
__global__ void bias_act_kernel(float* Z, const float* bias, float* A, int64_t rows, int64_t cols) {
  int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    float z = Z[e] + bias[e % cols];
    Z[e] = z;
    if (A) A[e] = gelu(z);
  }
}

hipError_t launch_bias_act(float* Z, const float* bias, float* A, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  bias_act_kernel<<<grid_for(rows * cols), 256, 0, s>>>(Z, bias, A, rows, cols);
  return hipGetLastError();
}

// dZ = dA * gelu'(Z)
__global__ void gelu_backward_kernel(const float* Z, const float* dA, float* dZ, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dZ[e] = dA[e] * gelu_grad(Z[e]);
}

hipError_t launch_gelu_backward(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  gelu_backward_kernel<<<grid_for(n), 256, 0, s>>>(Z, dA, dZ, n);
  return hipGetLastError();
}

// out[c] = sum_r X[r][c] (one thread per column; rows are few)
__global__ void colsum_kernel(const float* X, int64_t rows, int64_t cols, float* out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int64_t r = 0; r < rows; ++r) s += X[r * cols + c];
    out[c] = s;
  }
}

hipError_t launch_colsum(const float* X, int64_t rows, int64_t cols, float* out, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  colsum_kernel<<<grid_for(cols), 256, 0, s>>>(X, rows, cols, out);
  return hipGetLastError();
}

// Mean squared error L = (1/n) sum (y_i - t_i)^2 with standardised targets
// t_i = (target_i - mu) / sigma; dy_i = 2 (y_i - t_i) / n.  One workgroup.
__global__ __launch_bounds__(256) void mse_kernel(const float* y, const float* target, int64_t n, const float* stats,
                                                  float* dy, float* loss) {
  const float mu = stats ? stats[0] : 0.0f, inv = stats ? 1.0f / stats[1] : 1.0f;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    float r = y[i] - (target[i] - mu) * inv;
    dy[i] = 2.0f * r / (float)n;
    acc += (double)r * r;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / (double)n);
}

hipError_t launch_mse(const float* y, const float* target, int64_t n, const float* stats, float* dy, float* loss,
                      hipStream_t s) {
  mse_kernel<<<1, 256, 0, s>>>(y, target, n, stats, dy, loss);
  return hipGetLastError();
}

// stats = (mean, standard deviation) of t[0..n); the deviation is replaced by 1 if it is 0.
__global__ __launch_bounds__(256) void mean_std_kernel(const float* t, int64_t n, float* stats) {
  __shared__ double r1[256], r2[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += t[i];
  r1[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) r1[threadIdx.x] += r1[threadIdx.x + w];
    __syncthreads();
  }
  double mu = r1[0] / (double)n, q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) q += ((double)t[i] - mu) * ((double)t[i] - mu);
  r2[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) r2[threadIdx.x] += r2[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sd = sqrt(r2[0] / (double)n);
    stats[0] = (float)mu;
    stats[1] = sd > 0.0 ? (float)sd : 1.0f;
  }
}

hipError_t launch_mean_std(const float* t, int64_t n, float* stats, hipStream_t s) {
  mean_std_kernel<<<1, 256, 0, s>>>(t, n, stats);
  return hipGetLastError();
}

// y = y * sigma + mu
__global__ void destandardize_kernel(float* y, int64_t n, const float* stats) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = y[i] * stats[1] + stats[0];
}

hipError_t launch_destandardize(float* y, int64_t n, const float* stats, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  destandardize_kernel<<<grid_for(n), 256, 0, s>>>(y, n, stats);
  return hipGetLastError();
}

// Adam (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  adam_kernel<<<grid_for(n), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// Per-tensor normalised float32 copy: out[t][i] = x[t][i] / |x_t| for blocks of length len.
__global__ __launch_bounds__(256) void block_normalize_kernel(const double* x, int64_t len, float* out) {
  const double* xb = x + (int64_t)blockIdx.x * len;
  float* ob = out + (int64_t)blockIdx.x * len;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 256) s += xb[i] * xb[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 256) ob[i] = (float)(xb[i] * inv);
}

hipError_t launch_block_normalize(const double* x, int64_t blocks, int64_t len, float* out, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  block_normalize_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, len, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// L-BFGS vector algebra in float64.

// out[k] = <x_k, y_k> for k < count pairs given as pointer lists (one workgroup each)
__global__ __launch_bounds__(256) void dots_kernel(DotList L, int64_t n, double* out) {
  const double* x = L.x[blockIdx.x];
  const double* y = L.y[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i] * y[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_dots(const DotList& L, int count, int64_t n, double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  dots_kernel<<<count, 256, 0, s>>>(L, n, out);
  return hipGetLastError();
}

// y = a x + b y
__global__ void axpby_kernel(double a, const double* x, double b, double* y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  axpby_kernel<<<grid_for(n), 256, 0, s>>>(a, x, b, y, n);
  return hipGetLastError();
}

// z = x + a p
__global__ void xpay_kernel(const double* x, double a, const double* p, double* z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = x[i] + a * p[i];
}

hipError_t launch_xpay(const double* x, double a, const double* p, double* z, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  xpay_kernel<<<grid_for(n), 256, 0, s>>>(x, a, p, z, n);
  return hipGetLastError();
}

// max |x_i| (one workgroup)
__global__ __launch_bounds__(256) void absmax_kernel(const double* x, int64_t n, double* out) {
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(x[i]));
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_absmax(const double* x, int64_t n, double* out, hipStream_t s) {
  absmax_kernel<<<1, 256, 0, s>>>(x, n, out);
  return hipGetLastError();
}

}  // namespace optk
