// Launch interface of the surrogate and L-BFGS kernels (opt_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace optk {

constexpr int DOT_MAX = 32;
struct DotList {
  const double* x[DOT_MAX];
  const double* y[DOT_MAX];
};

hipError_t launch_uniform_init(float* p, int64_t n, uint64_t seed, int64_t offset, double bound, hipStream_t s);
hipError_t launch_uniform_init_f64(double* p, int64_t n, uint64_t seed, int64_t offset, double bound,
                                   hipStream_t s);
hipError_t launch_bias_act(float* Z, const float* bias, float* A, int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_gelu_backward(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t s);
hipError_t launch_colsum(const float* X, int64_t rows, int64_t cols, float* out, hipStream_t s);
hipError_t launch_mse(const float* y, const float* target, int64_t n, const float* stats, float* dy, float* loss,
                      hipStream_t s);
hipError_t launch_mean_std(const float* t, int64_t n, float* stats, hipStream_t s);
hipError_t launch_destandardize(float* y, int64_t n, const float* stats, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       int t, hipStream_t s);
hipError_t launch_block_normalize(const double* x, int64_t blocks, int64_t len, float* out, hipStream_t s);

hipError_t launch_dots(const DotList& L, int count, int64_t n, double* out, hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
hipError_t launch_xpay(const double* x, double a, const double* p, double* z, int64_t n, hipStream_t s);
hipError_t launch_absmax(const double* x, int64_t n, double* out, hipStream_t s);

}  // namespace optk
