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


// The value v of lane (lane ^ MASK) of the wave, moved through registers
// rather than the LDS crossbar: DPP quad permutes for masks 1 and 2, a row
// rotation by 8 for mask 8, row shifts by 4 either way for mask 4 (each lane
// takes the one whose source is its partner), and gfx950's lane swaps between
// rows (16) and halves (32) of the wave.  Every lane receives exactly its
// partner's value, as from a shuffle.
template <int MASK>
__device__ __forceinline__ double xor_lane(double v, int lane) {
  const unsigned lo = (unsigned)__double_as_longlong(v), hi = (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
  unsigned rlo, rhi;
  if constexpr (MASK == 1 || MASK == 2 || MASK == 8) {
    // quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_ror:8
    constexpr int ctrl = MASK == 1 ? 0xB1 : MASK == 2 ? 0x4E : 0x128;
    rlo = (unsigned)__builtin_amdgcn_update_dpp((int)lo, (int)lo, ctrl, 0xF, 0xF, false);
    rhi = (unsigned)__builtin_amdgcn_update_dpp((int)hi, (int)hi, ctrl, 0xF, 0xF, false);
  } else if constexpr (MASK == 4) {
    // row_shl:4 gives lane i the value of lane i + 4, row_shr:4 that of lane i - 4
    const unsigned ulo = (unsigned)__builtin_amdgcn_update_dpp((int)lo, (int)lo, 0x104, 0xF, 0xF, false);
    const unsigned uhi = (unsigned)__builtin_amdgcn_update_dpp((int)hi, (int)hi, 0x104, 0xF, 0xF, false);
    const unsigned dlo = (unsigned)__builtin_amdgcn_update_dpp((int)lo, (int)lo, 0x114, 0xF, 0xF, false);
    const unsigned dhi = (unsigned)__builtin_amdgcn_update_dpp((int)hi, (int)hi, 0x114, 0xF, 0xF, false);
    const bool up = (lane & 4) == 0;
    rlo = up ? ulo : dlo;
    rhi = up ? uhi : dhi;
  } else if constexpr (MASK == 16) {
    // odd rows of the first operand swap with even rows of the second: with both
    // equal to v, [0] holds rows 0,0,2,2 and [1] rows 1,1,3,3
    const auto plo = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto phi = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const bool odd = lane & 16;
    rlo = odd ? plo[0] : plo[1];
    rhi = odd ? phi[0] : phi[1];
  } else {
    static_assert(MASK == 32, "lane mask");
    // upper half of the first operand swaps with the lower half of the second:
    // [0] holds halves 0,0 and [1] halves 1,1
    const auto plo = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto phi = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const bool upper = lane & 32;
    rlo = upper ? plo[0] : plo[1];
    rhi = upper ? phi[0] : phi[1];
  }
  return __longlong_as_double((long long)(((unsigned long long)rhi << 32) | rlo));
}

template <int MASK>
__device__ __forceinline__ double xor_sum_levels(double v, int lane) {
  if constexpr (MASK >= 1) {
    v += xor_lane<MASK>(v, lane);
    return xor_sum_levels<MASK / 2>(v, lane);
  } else {
    return v;
  }
}

__device__ __forceinline__ double wave_sum(double v) { return xor_sum_levels<32>(v, threadIdx.x & 63); }

// Sums v over a workgroup of NTT threads; every thread receives the total.  ``red`` holds NTT/64 doubles.
template <int NTT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NTT / 64; ++i) s += red[i];
  return s;
}

// Sums NV values (NV a power of two, at most 64) over the 64 lanes of a wave by
// recursive halving: at each level a lane keeps half of its values, sends the
// other half to the partner lane and adds what it receives, so lane l ends
// with the wave total of value l / (64 / NV).  x is overwritten.  The levels
// are template recursion so that every index is a compile-time constant.
// At the levels of masks 32 and 16, gfx950's lane swaps do the exchange of a
// pair (x[i], x[i + H]) in place: v_permlane32_swap(a, b) exchanges the upper
// half of the wave's a with the lower half of its b, so that afterwards a + b
// is, in the lower half, a's sum over the two halves and, in the upper half,
// b's (v_permlane16_swap likewise for the odd and even rows of 16 lanes).
// The sums are the ones the select-and-exchange form computes (own value plus
// partner's value, in either order).
template <int MASK>
__device__ __forceinline__ double swap_sum(double a, double b) {
  const unsigned alo = (unsigned)__double_as_longlong(a), ahi = (unsigned)((unsigned long long)__double_as_longlong(a) >> 32);
  const unsigned blo = (unsigned)__double_as_longlong(b), bhi = (unsigned)((unsigned long long)__double_as_longlong(b) >> 32);
  unsigned rlo[2], rhi[2];
  if constexpr (MASK == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    rlo[0] = l[0]; rlo[1] = l[1]; rhi[0] = h[0]; rhi[1] = h[1];
  } else {
    static_assert(MASK == 16, "lane mask");
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    rlo[0] = l[0]; rlo[1] = l[1]; rhi[0] = h[0]; rhi[1] = h[1];
  }
  const double a2 = __longlong_as_double((long long)(((unsigned long long)rhi[0] << 32) | rlo[0]));
  const double b2 = __longlong_as_double((long long)(((unsigned long long)rhi[1] << 32) | rlo[1]));
  return a2 + b2;
}

template <int H, int MASK>
__device__ __forceinline__ void halving(double* x, int lane) {
  if constexpr (H >= 1) {
    if constexpr (MASK == 32 || MASK == 16) {
#pragma unroll
      for (int i = 0; i < H; ++i) x[i] = swap_sum<MASK>(x[i], x[i + H]);
    } else {
      const bool hi = lane & MASK;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const double send = hi ? x[i] : x[i + H];
        const double keep = hi ? x[i + H] : x[i];
        x[i] = keep + xor_lane<MASK>(send, lane);
      }
    }
    halving<H / 2, MASK / 2>(x, lane);
  }
}

template <int NV>
__device__ __forceinline__ double wave_reduce(double* x) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "power of two");
  const int lane = threadIdx.x & 63;
  halving<NV / 2, 32>(x, lane);
  return xor_sum_levels<32 / NV>(x[0], lane);
}

// The column loop is a real loop: unrolled, each column would run its own
// straight-line code once, and the kernel would wait on instruction fetch.
// Column c of the register panel is read and replaced by select chains over
// the (unrolled) column index, which keeps the panel in registers.
// With V and Y given, the kernel also writes the dense factors of the
// panel's block reflector for the trailing update (what build_vy_kernel
// writes with trans set: V with its unit diagonal, Y = V T; L = m - j0 rows of
// NB per matrix, stride L * NB), from the panel still in registers.
template <int RPT, int NB, int NTT>
__global__ __launch_bounds__(NTT) void panel_kernel(double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m,
                                                    int64_t n, int64_t j0, double* tau, int64_t tau_stride, double* T,
                                                    int64_t T_stride, double* V, double* Y) {
  constexpr int NW = NTT / 64;
  static_assert(NB * NB <= NTT && 64 % NB == 0, "panel shape");
  __shared__ double red[NW];
  __shared__ double redv[NW][NB];
  __shared__ double wfin[2][NB];
  __shared__ double bc[2];
  __shared__ double Gs[NB][NB];
  __shared__ double Tr[NB][NB];
  __shared__ double taus_s[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x;
  double* Ab = A + (int64_t)b * stride;
  const int64_t k = m < n ? m : n;
  const int nbp = (int)((k - j0) < NB ? (k - j0) : NB);   // columns of this panel
  double a[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = j0 + tid + (int64_t)NTT * q;
#pragma unroll
    for (int c = 0; c < NB; ++c) a[q][c] = (i < m && c < nbp) ? Ab[i * rs + (j0 + c) * cs] : 0.0;
  }
  if (tid < NB) taus_s[tid] = 0.0;
  if (tid < NB * NB) Gs[tid / NB][tid % NB] = 0.0;
#pragma unroll 1
  for (int c = 0; c < nbp; ++c) {
    double ac[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      ac[q] = a[q][0];
#pragma unroll
      for (int i = 1; i < NB; ++i) ac[q] = c == i ? a[q][i] : ac[q];
    }
    // sigma = |x below the diagonal|^2, alpha = diagonal element (local row c, thread c, q = 0)
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NTT * q;
      if (r > c && j0 + r < m) part += ac[q] * ac[q];
    }
    // alternate slots: the next write to this slot comes after two more block sums
    if (tid == c) bc[c & 1] = ac[0];
    const double sigma = block_sum<NTT>(part, red);   // its barriers publish bc
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
      const int r = tid + NTT * q;
      if (r > c && j0 + r < m) ac[q] *= scale;
    }
    if (tid == c) ac[0] = beta;
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
      for (int i = 0; i < NB; ++i) a[q][i] = c == i ? ac[q] : a[q][i];
    if (t == 0.0) continue;
    // one reduction gives w_cc = v . A[:, cc] for the trailing columns cc > c
    // and v_l . v for the earlier vectors l < c (column c of V^T V, for T):
    // below row c both read the stored column, and v vanishes above row c
    double x[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) x[cc] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NTT * q;
      if (r < c || j0 + r >= m) continue;
      const double v = r == c ? 1.0 : ac[q];
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) x[cc] += cc != c ? v * a[q][cc] : 0.0;
    }
    const double tot = wave_reduce<NB>(x);
    if (lane % (64 / NB) == 0) redv[wave][lane / (64 / NB)] = tot;
    __syncthreads();
    if (tid < NB) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += redv[w][tid];
      wfin[c & 1][tid] = sum;
      if (tid < c) Gs[tid][c] = sum;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NTT * q;
      if (r < c || j0 + r >= m) continue;
      const double vt = (r == c ? 1.0 : ac[q]) * t;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc)
        if (cc > c) a[q][cc] -= vt * wfin[c & 1][cc];
    }
  }
  // store the panel
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t i = j0 + tid + (int64_t)NTT * q;
    if (i >= m) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbp) Ab[i * rs + (j0 + c) * cs] = a[q][c];
  }
  // T of the block reflector (LAPACK's larft, forward, columnwise) from
  // G = V^T V (upper triangle, gathered above): T_cc = tau_c,
  // T[i][c] = -tau_c sum_{l=i}^{c-1} T[i][l] G[l][c]; thread i < NB computes
  // row i (it depends on that row only).  The sums are formed term by term as
  // the row's entries become known (entry l adds its terms to the sums of all
  // later columns), each in the order l = i, ..., c - 1, so that the chain
  // from one entry to the next is one product and one sum; the row and the
  // sums stay in registers.  The entries left of the diagonal are zero and
  // add exact zeros (the sums start at +0 and never become -0), so every
  // step runs the same instructions, without branches.
  __syncthreads();
  if (tid < NB) {
    const int i = tid;
    double* Tb = T + (int64_t)b * T_stride;
    double trow[NB], sum[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) sum[c] = 0.0;
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      const double tl = taus_s[l];
      const double v = (l < nbp && l == i) ? tl : ((l < nbp && l > i) ? -tl * sum[l] : 0.0);
      trow[l] = v;
#pragma unroll
      for (int c = l + 1; c < NB; ++c) sum[c] += v * Gs[l][c];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      Tr[i][c] = trow[c];
      Tb[i * NB + c] = trow[c];
    }
    if (i < nbp) tau[(int64_t)b * tau_stride + j0 + i] = taus_s[i];
  }
  if (V == nullptr) return;
  __syncthreads();   // every row of Tr
  const int64_t L = m - j0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = tid + NTT * q;
    if (r >= L) continue;
    double v[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) v[c] = c >= nbp ? 0.0 : (r == c ? 1.0 : (r > c ? a[q][c] : 0.0));
    double* Vr = V + ((int64_t)b * L + r) * NB;
    double* Yr = Y + ((int64_t)b * L + r) * NB;
#pragma unroll
    for (int c = 0; c < NB; ++c) Vr[c] = v[c];
    // the sums of build_vy_kernel, in its order (l = 0, ..., NB - 1 for every
    // column), all columns at once: one row of T per step
    // (T is upper triangular: the terms l > c are exact zeros and left out)
    double y[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) y[c] = 0.0;
#pragma unroll
    for (int l = 0; l < NB; ++l)
#pragma unroll
      for (int c = l; c < NB; ++c) y[c] += v[l] * Tr[l][c];
#pragma unroll
    for (int c = 0; c < NB; ++c) Yr[c] = y[c];
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
    for (int c = 0; c < NB; ++c) Vr[c] = v[c];
    // one output column at a time: hoisting all NB*NB entries of T would not fit the registers
#pragma unroll 1
    for (int c = 0; c < NB; ++c) {
      double y = 0.0;
#pragma unroll
      for (int l = 0; l < NB; ++l) y += v[l] * Ts[c * NB + l];
      Yr[c] = y;
    }
  }
}

// Trailing update with a panel's block reflector in one launch,
// C_b[i][j] -= (V (Y^T C_b))[i][j] for i < L, j < ncols (element (i, j) at
// C + b*cstride + i*crs + j*ccs; V, Y row-major L x NB per matrix, stride
// L*NB), with the arithmetic of the two matrix-core products it replaces,
// element for element: Z = Y^T C as MFMA chains over
// k in groups of four from each chunk start (chunks of kchunk rows when
// ksplit > 1, summed in order from 0.0 as the split-K reduction does), then
// C <- (-(V Z)) + C with the chain over the NB columns of V.  A workgroup of
// 512 threads owns 16 columns of one matrix: its 8 waves take the chunks in
// turn, their partials meet in LDS, then the waves take 16-row tiles of the
// update.  The 16 x 16 MFMA tiles follow v_mfma_f64_16x16x4f64: operand
// lane (lr, lq) holds A[m = lr][k = lq] and B[k = lq][n = lr]; result register
// e is row lq + 4 e, column lr.
constexpr int PU_MAX_SPLIT = 32;
constexpr int PU_AHEAD = 16;
template <int NB>
__global__ __launch_bounds__(512) void panel_update_mfma_kernel(double* C, int64_t crs, int64_t ccs, int64_t cstride,
                                                                int64_t L, int64_t ncols, const double* V,
                                                                const double* Y, int64_t kchunk, int ksplit) {
  typedef double d4_t __attribute__((ext_vector_type(4)));
  constexpr int NW = 8;
  __shared__ double part[PU_MAX_SPLIT][16][16];
  __shared__ double Zs[16][17];
  const int b = blockIdx.y, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 16;
  const int64_t j = j0 + lr;
  const bool jok = j < ncols;
  double* Cb = C + (int64_t)b * cstride;
  const double* Yb = Y + (int64_t)b * L * NB;
  const double* Vb = V + (int64_t)b * L * NB;
  const int nsplit = ksplit > 1 ? ksplit : 1;
  const int64_t chunk = ksplit > 1 ? kchunk : L;
  // ---- partial Z of each chunk: rows c of Z are A's rows (Y^T), columns the workgroup's
  for (int sp = wave; sp < nsplit; sp += NW) {
    const int64_t kbeg = (int64_t)sp * chunk, kend = kbeg + chunk < L ? kbeg + chunk : L;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
    // the operands of PU_AHEAD groups of 4 rows are loaded before their MFMAs
    // run (in the same order as one group at a time): the chain then waits on
    // memory once per PU_AHEAD groups
    for (int64_t k0 = kbeg; k0 < kend; k0 += 4 * PU_AHEAD) {
      double a[PU_AHEAD], x[PU_AHEAD];
#pragma unroll
      for (int u = 0; u < PU_AHEAD; ++u) {
        const int64_t k = k0 + 4 * u + lq;
        const bool kok = k < kend;
        a[u] = (kok && lr < NB) ? Yb[k * NB + lr] : 0.0;
        x[u] = (kok && jok) ? Cb[k * crs + j * ccs] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PU_AHEAD; ++u)
        if (k0 + 4 * u < kend) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], x[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) part[sp][lq + 4 * e][lr] = acc[e];
  }
  __syncthreads();
  if (tid < 256) {
    const int c = tid >> 4, n = tid & 15;
    double z;
    if (ksplit > 1) {
      z = 0.0;
      for (int sp = 0; sp < nsplit; ++sp) z += part[sp][c][n];
    } else {
      z = part[0][c][n];
    }
    Zs[c][n] = z;
  }
  __syncthreads();
  // ---- C <- (-(V Z)) + C over 16-row tiles, two tiles per wave at a time
  // (their loads issued before either chain)
  const int64_t rtiles = (L + 15) / 16;
  for (int64_t rt0 = wave; rt0 < rtiles; rt0 += 2 * NW) {
    double av[2][NB / 4], c[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r0 = (rt0 + h * NW) * 16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = r0 + lq + 4 * e;
        c[h][e] = (jok && r < L) ? Cb[r * crs + j * ccs] : 0.0;
      }
      const int64_t r = r0 + lr;
#pragma unroll
      for (int g = 0; g < NB / 4; ++g) av[h][g] = r < L ? Vb[r * NB + 4 * g + lq] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r0 = (rt0 + h * NW) * 16;
      if (r0 >= L) break;
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g = 0; g < NB / 4; ++g)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][g], Zs[4 * g + lq][lr], acc, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = r0 + lq + 4 * e;
        if (jok && r < L) Cb[r * crs + j * ccs] = -acc[e] + c[h][e];
      }
    }
  }
}

hipError_t launch_panel_update_mfma(double* C, int64_t crs, int64_t ccs, int64_t cstride, int64_t L, int64_t ncols,
                                    int nb, const double* V, const double* Y, int batch, int64_t kchunk, int ksplit,
                                    hipStream_t s) {
  if (L <= 0 || ncols <= 0 || batch <= 0) return hipSuccess;
  // a split must cover the L rows in chunks of whole MFMA groups
  if (batch > 65535 || (nb != 16 && nb != 8) || ksplit > PU_MAX_SPLIT ||
      (ksplit > 1 && (kchunk <= 0 || kchunk % 4 != 0 || kchunk * ksplit < L)))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((ncols + 15) / 16), (unsigned)batch);
  if (nb == 16) panel_update_mfma_kernel<16><<<grid, 512, 0, s>>>(C, crs, ccs, cstride, L, ncols, V, Y, kchunk, ksplit);
  else panel_update_mfma_kernel<8><<<grid, 512, 0, s>>>(C, crs, ccs, cstride, L, ncols, V, Y, kchunk, ksplit);
  return hipGetLastError();
}

int panel_update_max_split() { return PU_MAX_SPLIT; }

// Panel shapes: RPT rows per thread in a workgroup of NTT threads, one
// register row per thread up to 1024 rows (more threads rather than more
// rows per thread: the per-thread panel must stay in registers).
static int panel_threads(int64_t rows) {
  if (rows <= 256) return 256;
  if (rows <= 512) return 512;
  if (rows <= 1024) return 1024;
  if (rows <= 2048) return 256 * 8;   // eight-column panels, 8 rows per thread, 256 threads
  return 0;
}

int panel_width(int64_t m) { return m <= 1024 ? 16 : 8; }

hipError_t launch_panel(double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m, int64_t n, int64_t j0, int batch,
                        double* tau, int64_t tau_stride, double* T, int64_t T_stride, double* V, double* Y,
                        hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int64_t rows = m - j0 > 0 ? m - j0 : 1;
  const int nb = panel_width(m);
  const int nt = panel_threads(rows);
  if (nt == 0) return hipErrorInvalidValue;
  // rows of the panel: local row r = tid + NTT*q covers m - j0 rows
  if (nb == 16) {
    switch (nt) {
      case 256: panel_kernel<1, 16, 256><<<batch, 256, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride, V, Y); break;
      case 512: panel_kernel<1, 16, 512><<<batch, 512, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride, V, Y); break;
      case 1024: panel_kernel<2, 16, 512><<<batch, 512, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride, V, Y); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    panel_kernel<8, 8, 256><<<batch, 256, 0, s>>>(A, rs, cs, stride, m, n, j0, tau, tau_stride, T, T_stride, V, Y);
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
