// Batched blocked Householder QR for the projector factorisations.
//
// A_b (m x n, element (i, j) at A_b[i*rs + j*cs], b < batch, A_b = A + b*stride)
// is factorised in place as A = Q R: R in the upper triangle, the Householder
// vectors v_j (v_j[j] = 1 implicit, zeros above) below it, tau_j in tau.
// Q = H_0 H_1 ... H_{k-1}, H_j = I - tau_j v_j v_j^T, k = min(m, n), as in
// LAPACK's geqrf (beta = -sign(alpha) |x|, tau = (beta - alpha)/beta,
// v = x / (alpha - beta); tau = 0 when the column below the diagonal is 0).
// Panels of NB columns are factorised by one workgroup per matrix with the
// panel held in registers (RPT rows per thread); the block reflector
// I - V T V^T of each panel (T upper triangular, LAPACK's larft) is then
// applied to the trailing columns as two matrix products on the MFMA
// contraction kernel (from the dense V and Y of build_vy_kernel), the same
// products that apply Q or Q^T to other matrices afterwards.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qr_kernels.h"

namespace qrk {

constexpr int NT = 256;   // threads of the panel and update kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums v over the workgroup; every thread receives the total.  ``red`` holds NT/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

template <int RPT, int NB>
__global__ __launch_bounds__(NT) void panel_kernel(double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m,
                                                   int64_t n, int64_t j0, double* tau, int64_t tau_stride, double* T,
                                                   int64_t T_stride) {
  __shared__ double red[NT / 64];
  __shared__ double redv[NT / 64][NB];
  __shared__ double bc[2];
  __shared__ double Gs[NB][NB];
  __shared__ double taus_s[NB];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  double* Ab = A + (int64_t)b * stride;
  const int64_t k = m < n ? m : n;
  const int nbp = (int)((k - j0) < NB ? (k - j0) : NB);   // columns of this panel
  double a[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = j0 + tid + (int64_t)NT * q;
#pragma unroll
    for (int c = 0; c < NB; ++c) a[q][c] = (i < m && c < nbp) ? Ab[i * rs + (j0 + c) * cs] : 0.0;
  }
  if (tid < NB) taus_s[tid] = 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= nbp) continue;
    // sigma = |x below the diagonal|^2, alpha = diagonal element (local row c, thread c, q = 0)
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      if (r > c && j0 + r < m) part += a[q][c] * a[q][c];
    }
    // alternate slots: the next write to this slot comes after two more block sums
    if (tid == c) bc[c & 1] = a[0][c];
    const double sigma = block_sum(part, red);   // its barriers publish bc
    const double alpha = bc[c & 1];
    double t = 0.0, beta = alpha, scale = 0.0;
    if (sigma > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (tid == 0) taus_s[c] = t;
    // v below the diagonal; beta on the diagonal
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      if (r > c && j0 + r < m) a[q][c] *= scale;
    }
    if (tid == c) a[0][c] = beta;
    if (t == 0.0) continue;
    // w_c' = v . A[:, c'] for c' > c, then A[:, c'] -= t v w_c'
    double wpart[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) wpart[cc] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      if (r < c || j0 + r >= m) continue;
      const double v = r == c ? 1.0 : a[q][c];
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) wpart[cc] += v * a[q][cc];
    }
#pragma unroll
    for (int cc = c + 1; cc < NB; ++cc) wpart[cc] = wave_sum(wpart[cc]);
    __syncthreads();
    if ((tid & 63) == 0)
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) redv[tid >> 6][cc] = wpart[cc];
    __syncthreads();
#pragma unroll
    for (int cc = c + 1; cc < NB; ++cc) {
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < NT / 64; ++i) w += redv[i][cc];
      wpart[cc] = w * t;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      if (r < c || j0 + r >= m) continue;
      const double v = r == c ? 1.0 : a[q][c];
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) a[q][cc] -= v * wpart[cc];
    }
  }
  // store the panel
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = j0 + tid + (int64_t)NT * q;
    if (i >= m) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbp) Ab[i * rs + (j0 + c) * cs] = a[q][c];
  }
  // T of the block reflector (LAPACK's larft, forward, columnwise):
  // G = V^T V, T_cc = tau_c, T[i][c] = -tau_c sum_{l=i}^{c-1} T[i][l] G[l][c].
  // Row c of G (entries cc > c) is summed over the workgroup in one reduction.
  if (tid < NB * NB) Gs[tid / NB][tid % NB] = 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c + 1 >= nbp) break;
    double gp[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) gp[cc] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      if (r <= c || j0 + r >= m) continue;   // v_cc vanishes above row cc > c, so r > c
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) {
        if (r < cc) continue;
        gp[cc] += a[q][c] * (r == cc ? 1.0 : a[q][cc]);
      }
    }
#pragma unroll
    for (int cc = c + 1; cc < NB; ++cc) gp[cc] = wave_sum(gp[cc]);
    __syncthreads();
    if ((tid & 63) == 0)
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) redv[tid >> 6][cc] = gp[cc];
    __syncthreads();
    if (tid < NB && tid > c) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NT / 64; ++i) s += redv[i][tid];
      Gs[c][tid] = s;
    }
  }
  __syncthreads();
  // thread i < NB computes row i of T (it depends on that row only)
  if (tid < NB) {
    const int i = tid;
    double* Tb = T + (int64_t)b * T_stride;
    double Trow[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double v = 0.0;
      if (c < nbp && c == i) v = taus_s[c];
      else if (c < nbp && c > i) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NB; ++l)
          if (l >= i && l < c) s += Trow[l] * Gs[l][c];
        v = -taus_s[c] * s;
      }
      Trow[c] = v;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) Tb[i * NB + c] = Trow[c];
    if (i < nbp) tau[(int64_t)b * tau_stride + j0 + i] = taus_s[i];
  }
}

// Dense factors of a panel's block reflector for the update C <- C - V (Y^T C):
// V (L x NB, row-major, L = m - j0) holds the Householder vectors of the
// panel at (j0, j0) with the unit diagonal and zeros above it (columns past
// nbp zero), and Y = V T (trans: H^T = I - V T^T V^T) or Y = V T^T (H).
template <int NB>
__global__ __launch_bounds__(256) void build_vy_kernel(const double* A, int64_t rs, int64_t cs, int64_t stride,
                                                       int64_t m, int64_t j0, int nbp, const double* T,
                                                       int64_t T_stride, int trans, double* V, double* Y) {
  __shared__ double Ts[NB * NB];
  const int b = blockIdx.y;
  const int64_t L = m - j0;
  const double* Ab = A + (int64_t)b * stride;
  const double* Tb = T + (int64_t)b * T_stride;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    Ts[e] = trans ? Tb[j * NB + i] : Tb[i * NB + j];   // Ts[c][l]: Y[r][c] = sum_l V[r][l] Ts[c][l]
  }
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < L; r += (int64_t)gridDim.x * blockDim.x) {
    double v[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      v[c] = c >= nbp ? 0.0 : (r == c ? 1.0 : (r > c ? Ab[(j0 + r) * rs + (j0 + c) * cs] : 0.0));
    double* Vr = V + ((int64_t)b * L + r) * NB;
    double* Yr = Y + ((int64_t)b * L + r) * NB;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double y = 0.0;
#pragma unroll
      for (int l = 0; l < NB; ++l) y += v[l] * Ts[c * NB + l];
      Vr[c] = v[c];
      Yr[c] = y;
    }
  }
}

static int pick_rpt(int64_t rows) {
  if (rows <= NT) return 1;
  if (rows <= 2 * NT) return 2;
  if (rows <= 4 * NT) return 4;
  if (rows <= 8 * NT) return 8;
  return 0;
}

int panel_width(int64_t m) { return pick_rpt(m) == 8 ? 8 : 16; }

hipError_t launch_panel(double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m, int64_t n, int64_t j0, int batch,
                        double* tau, int64_t tau_stride, double* T, int64_t T_stride, hipStream_t s) {
  const int rpt = pick_rpt(m - j0 > 0 ? m - j0 : 1);
  const int nb = panel_width(m);
  if (batch <= 0) return hipSuccess;
  // rows of the panel: local row r = tid + NT*q covers m - j0 rows
  if (nb == 16) {
    switch (rpt) {
      case 1: panel_kernel<1, 16><<<batch, NT, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride); break;
      case 2: panel_kernel<2, 16><<<batch, NT, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride); break;
      case 4: panel_kernel<4, 16><<<batch, NT, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    if (rpt == 0) return hipErrorInvalidValue;
    panel_kernel<8, 8><<<batch, NT, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride);
  }
  return hipGetLastError();
}

hipError_t launch_build_vy(const double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m, int64_t j0, int nbp,
                           int nb, const double* T, int64_t T_stride, bool trans, double* V, double* Y, int batch,
                           hipStream_t s) {
  const int64_t L = m - j0;
  if (L <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((unsigned)((L + 255) / 256), (unsigned)batch);
  if (nb == 16) build_vy_kernel<16><<<grid, 256, 0, s>>>(A, rs, cs, stride, m, j0, nbp, T, T_stride, trans, V, Y);
  else build_vy_kernel<8><<<grid, 256, 0, s>>>(A, rs, cs, stride, m, j0, nbp, T, T_stride, trans, V, Y);
  return hipGetLastError();
}

// R^T of the factorised A_b (upper trapezoidal k x n) as the column-major
// n x k lower-trapezoidal L_b (L[a + i*n] = R[i][a] for a >= i, else 0).
__global__ void extract_rt_kernel(const double* A, int64_t rs, int64_t cs, int64_t stride, int64_t n, int64_t k,
                                  double* L, int64_t lstride, int batch) {
  const int64_t total = n * k * batch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / (n * k), e = t - b * n * k;
    const int64_t i = e / n, a = e - i * n;
    L[b * lstride + e] = a >= i ? A[b * stride + i * rs + a * cs] : 0.0;
  }
}

hipError_t launch_extract_rt(const double* A, int64_t rs, int64_t cs, int64_t stride, int64_t n, int64_t k, double* L,
                             int64_t lstride, int batch, hipStream_t s) {
  const int64_t total = n * k * batch;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  extract_rt_kernel<<<(unsigned)blocks, 256, 0, s>>>(A, rs, cs, stride, n, k, L, lstride, batch);
  return hipGetLastError();
}

}  // namespace qrk
