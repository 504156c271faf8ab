// Device kernels of the nested-CTMRG library (gfx950 / CDNA4).
//
// The central kernel is a tensor contraction written as a batched matrix
// product C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] (+ C) in which each
// of the four index groups b, m, n, k may be split into an outer and an inner
// part with independent strides in every operand.  That covers the corner,
// half-system, projection and density-matrix contractions of the CTMRG sweep
// without transposing operands in memory.  The product runs on the matrix
// cores: v_mfma_f64_16x16x4f64 (FP64 mode), v_mfma_f32_16x16x4f32 (FP32 mode)
// or v_mfma_f32_16x16x16bf16_1k (BF16 mode: FP32 data rounded to bfloat16 while
// staged in LDS, FP32 accumulation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "kernels.h"

namespace ctmk {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t split_off(int64_t i, int64_t inner, int64_t so, int64_t si) {
  int64_t o = i / inner;
  return o * so + (i - o * inner) * si;
}

constexpr int BM = 64, NT = 256;

template <int MODE> struct Cfg;
template <> struct Cfg<MODE_F64> { typedef double T; typedef double L; static constexpr int BK = 16; };
template <> struct Cfg<MODE_F32> { typedef float T; typedef float L; static constexpr int BK = 16; };
template <> struct Cfg<MODE_BF16> { typedef float T; typedef unsigned short L; static constexpr int BK = 32; };

template <int MODE> __device__ __forceinline__ typename Cfg<MODE>::L to_lds(typename Cfg<MODE>::T v);
template <> __device__ __forceinline__ double to_lds<MODE_F64>(double v) { return v; }
template <> __device__ __forceinline__ float to_lds<MODE_F32>(float v) { return v; }
template <> __device__ __forceinline__ unsigned short to_lds<MODE_BF16>(float v) {
  return __builtin_bit_cast(unsigned short, (__bf16)v);   // nearest even (v_cvt_pk_bf16_f32)
}

// One workgroup computes a 64 x BN tile of C (BN = 32 WN) for one batch
// entry; the four waves each own a 32 x 16WN quarter made of 2 x WN blocks of
// 16 x 16 MFMA tiles.  WN = 4 (BN = 128) halves the re-reads of the A operand
// when N is wide (tall-skinny absorptions with N up to 128 read A once).
template <int MODE, bool AK, bool BN_FAST, int WN>
__global__ __launch_bounds__(NT) void contract_kernel(GemmArgs g) {
  typedef typename Cfg<MODE>::T T;
  typedef typename Cfg<MODE>::L L;
  constexpr int BK = Cfg<MODE>::BK;
  constexpr int BN = 32 * WN;
  __shared__ L As[BK][BM + 4];
  __shared__ L Bs[BK][BN + 4];
  __shared__ int64_t a_row[BM], b_col[BN];

  const int tid = threadIdx.x;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t tile = blockIdx.x;
  const int64_t m0 = (tile / tiles_n) * BM, n0 = (tile % tiles_n) * BN;
  const int64_t bz = blockIdx.y;
  const int64_t kbeg = g.ksplit > 1 ? (int64_t)blockIdx.z * g.kchunk : 0;
  const int64_t kend = g.ksplit > 1 ? (kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K) : g.K;
  const T* A = (const T*)g.A + split_off(bz, g.b_in, g.a_b_o, g.a_b_i);
  const T* B = (const T*)g.B + split_off(bz, g.b_in, g.b_b_o, g.b_b_i);
  T* C = (T*)g.C + split_off(bz, g.b_in, g.c_b_o, g.c_b_i);

  // offsets may be negative (reversed views); rows/columns past the edge are marked NONE
  constexpr int64_t NONE = INT64_MIN;
  if (tid < BM) {
    int64_t m = m0 + tid;
    a_row[tid] = m < g.M ? split_off(m, g.m_in, g.a_m_o, g.a_m_i) : NONE;
  } else if (tid < BM + BN) {
    int64_t n = n0 + tid - BM;
    b_col[tid - BM] = n < g.N ? split_off(n, g.n_in, g.b_n_o, g.b_n_i) : NONE;
  }
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 16 * WN;
  const int lr = lane & 15, lq = lane >> 4;

  typedef typename std::conditional<MODE == MODE_F64, d4_t, f4_t>::type acc_t;
  acc_t acc[2][WN];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < WN; ++j)
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  constexpr int PA = BM * BK / NT;   // elements of A per thread per K step
  constexpr int PB = BN * BK / NT;   // elements of B per thread per K step
  // Each thread stages fixed (k-in-tile, row/column) positions of A and of B.
  // The K index of a position advances by BK per step; its split into
  // (outer, inner) parts is carried along incrementally instead of divided.
  int a_mm[PA], a_kq[PA], a_kr[PA], a_kk[PA];
  int b_nn[PB], b_kq[PB], b_kr[PB], b_kk[PB];
  const int kin = (int)g.k_in;
#pragma unroll
  for (int i = 0; i < PA; ++i) {
    const int e = tid + i * NT;
    if (AK) { a_kk[i] = e % BK; a_mm[i] = e / BK; } else { a_mm[i] = e % BM; a_kk[i] = e / BM; }
    const int k = (int)kbeg + a_kk[i];
    a_kq[i] = k / kin; a_kr[i] = k - a_kq[i] * kin;
  }
#pragma unroll
  for (int i = 0; i < PB; ++i) {
    const int e = tid + i * NT;
    if (BN_FAST) { b_nn[i] = e % BN; b_kk[i] = e / BN; } else { b_kk[i] = e % BK; b_nn[i] = e / BK; }
    const int k = (int)kbeg + b_kk[i];
    b_kq[i] = k / kin; b_kr[i] = k - b_kq[i] * kin;
  }
  T va[PA], vb[PB];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int64_t ro = a_row[a_mm[i]];
      const bool ok = ro != NONE && k0 + a_kk[i] < kend;
      va[i] = ok ? A[ro + (int64_t)a_kq[i] * g.a_k_o + (int64_t)a_kr[i] * g.a_k_i] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int64_t co = b_col[b_nn[i]];
      const bool okb = co != NONE && k0 + b_kk[i] < kend;
      vb[i] = okb ? B[co + (int64_t)b_kq[i] * g.b_k_o + (int64_t)b_kr[i] * g.b_k_i] : (T)0;
    }
  };
  auto advance = [&]() {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      a_kr[i] += BK;
      while (a_kr[i] >= kin) { a_kr[i] -= kin; ++a_kq[i]; }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      b_kr[i] += BK;
      while (b_kr[i] >= kin) { b_kr[i] -= kin; ++b_kq[i]; }
    }
  };
  load_tiles(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int i = 0; i < PA; ++i) As[a_kk[i]][a_mm[i]] = to_lds<MODE>(va[i]);
#pragma unroll
    for (int i = 0; i < PB; ++i) Bs[b_kk[i]][b_nn[i]] = to_lds<MODE>(vb[i]);
    __syncthreads();
    // prefetch the next K tile into registers while the matrix cores work
    if (k0 + BK < kend) {
      advance();
      load_tiles(k0 + BK);
    }
    if constexpr (MODE == MODE_F64) {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        double a0 = As[ks + lq][wm + lr], a1 = As[ks + lq][wm + 16 + lr];
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          double bj = Bs[ks + lq][wn + 16 * j + lr];
          acc[0][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bj, acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bj, acc[1][j], 0, 0, 0);
        }
      }
    } else if constexpr (MODE == MODE_F32) {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        float a0 = As[ks + lq][wm + lr], a1 = As[ks + lq][wm + 16 + lr];
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          float bj = Bs[ks + lq][wn + 16 * j + lr];
          acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bj, acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bj, acc[1][j], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 16) {
        s4_t a0, a1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int kk = ks + lq * 4 + q;
          a0[q] = (short)As[kk][wm + lr];
          a1[q] = (short)As[kk][wm + 16 + lr];
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          s4_t bj;
#pragma unroll
          for (int q = 0; q < 4; ++q) bj[q] = (short)Bs[ks + lq * 4 + q][wn + 16 * j + lr];
          acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, bj, acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, bj, acc[1][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // D layout of the 16x16 MFMA tiles (measured on gfx950): register e of lane l
  // holds column l%16 and row 4*(l/16)+e for the f32 and bf16 instructions,
  // row (l/16)+4*e for v_mfma_f64_16x16x4f64.
  if (g.ksplit > 1) {
    T* W = (T*)g.work + ((int64_t)blockIdx.z * g.batch + bz) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t n = n0 + wn + j * 16 + lr;
        if (n >= g.N) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = MODE == MODE_F64 ? lq + 4 * e : lq * 4 + e;
          const int64_t m = m0 + wm + i * 16 + row;
          if (m < g.M) W[m * g.N + n] = (T)acc[i][j][e];
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      int64_t n = n0 + wn + j * 16 + lr;
      if (n >= g.N) continue;
      int64_t cn = split_off(n, g.n_in, g.c_n_o, g.c_n_i);
      double cs = g.colscale ? g.colscale[n] : 1.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = MODE == MODE_F64 ? lq + 4 * e : lq * 4 + e;
        int64_t m = m0 + wm + i * 16 + row;
        if (m >= g.M) continue;
        int64_t off = split_off(m, g.m_in, g.c_m_o, g.c_m_i) + cn;
        T v = (T)(g.alpha * cs * (double)acc[i][j][e]);
        if (g.beta) v += C[off];
        C[off] = v;
      }
    }
}

// C = alpha * colscale * (sum of the split-K partial tiles) (+ C)
template <typename T>
__global__ void split_reduce_kernel(GemmArgs g) {
  const int64_t total = g.batch * g.M * g.N;
  const T* W = (const T*)g.work;
  T* C = (T*)g.C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e % g.N, bm = e / g.N, m = bm % g.M, b = bm / g.M;
    double acc = 0.0;
    for (int64_t s = 0; s < g.ksplit; ++s) acc += (double)W[s * total + e];
    const int64_t off = split_off(b, g.b_in, g.c_b_o, g.c_b_i) + split_off(m, g.m_in, g.c_m_o, g.c_m_i) +
                        split_off(n, g.n_in, g.c_n_o, g.c_n_i);
    T v = (T)(g.alpha * (g.colscale ? g.colscale[n] : 1.0) * acc);
    if (g.beta) v += C[off];
    C[off] = v;
  }
}

template <int MODE, int WN>
static hipError_t launch_tiles(const GemmArgs& g, hipStream_t s) {
  constexpr int BN = 32 * WN;
  // all (m, n) tiles of one batch entry along x, batch entries along y, K ranges along z
  dim3 grid((unsigned)(((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM)), (unsigned)g.batch,
            (unsigned)(g.ksplit > 1 ? g.ksplit : 1));
  // choose the fastest-varying index of each staged tile so that loads coalesce
  bool ak = g.a_k_i == 1 ? true : (g.a_m_i == 1 ? false : true);
  bool bn = g.b_n_i == 1 ? true : (g.b_k_i == 1 ? false : true);
  if (ak && bn) contract_kernel<MODE, true, true, WN><<<grid, NT, 0, s>>>(g);
  else if (ak) contract_kernel<MODE, true, false, WN><<<grid, NT, 0, s>>>(g);
  else if (bn) contract_kernel<MODE, false, true, WN><<<grid, NT, 0, s>>>(g);
  else contract_kernel<MODE, false, false, WN><<<grid, NT, 0, s>>>(g);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(const GemmArgs& g, hipStream_t s) {
  // 128-wide tiles when N is wide and there are enough rows to fill the chip
  const int64_t tiles_m = (g.M + BM - 1) / BM;
  hipError_t e = (g.N > 64 && tiles_m * g.batch >= 512) ? launch_tiles<MODE, 4>(g, s) : launch_tiles<MODE, 2>(g, s);
  if (e != hipSuccess || g.ksplit <= 1) return e;
  const int64_t total = g.batch * g.M * g.N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  split_reduce_kernel<typename Cfg<MODE>::T><<<(unsigned)blocks, 256, 0, s>>>(g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Large BF16 products of plain row-major operands: C[m][n] = alpha
// sum_k A[m][k] B[k][n] (+ C), A, B, C float32 in memory, products of bf16
// (rounded to nearest even) accumulated in float32.  A 128 x 128 tile per
// workgroup, 4 waves of 64 x 64 (4 x 4 tiles of v_mfma_f32_16x16x32_bf16),
// BK = 32.  The operands are read as float4, rounded, and kept in LDS as
// As[m][k] and Bs[n][k] (k contiguous, rows padded to 40 elements), so that a
// lane's MFMA fragment (four consecutive k) is one 8-byte read.  Tiles go to
// the XCDs in contiguous ranges (consecutive workgroups are dealt round-robin
// to the eight XCDs) and, within a range, in groups of eight row tiles, so
// that neighbouring workgroups of one XCD share operand tiles in its L2.
constexpr int GB_BM = 128, GB_BN = 128, GB_BK = 32, GB_LD = GB_BK + 8;

// four floats rounded to bf16 (nearest even, v_cvt_pk_bf16_f32) and packed
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
  typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
  const bf2_t lo = {(__bf16)a, (__bf16)b}, hi = {(__bf16)c, (__bf16)d};
  uint2 r;
  r.x = __builtin_bit_cast(uint32_t, lo);
  r.y = __builtin_bit_cast(uint32_t, hi);
  return r;
}

// A_KC: A has unit stride along k (row-major A[m][k]), else along m (A[k][m]
// column by column); B_NC: B has unit stride along n (row-major B[k][n]),
// else along k.  The tile loads follow the unit stride (float4), and blocks
// read along the other index are transposed in registers on the way to LDS.
template <bool A_KC, bool B_NC>
__global__ __launch_bounds__(256) void gemm_bf16_rowmajor_kernel(GemmArgs g) {
  __shared__ __align__(16) unsigned short As[GB_BM * GB_LD];
  __shared__ __align__(16) unsigned short Bs[GB_BN * GB_LD];
  // offsets of the tile's lines (rows of A or C, columns of B or C; an index
  // split in two levels is resolved here once), NONE past the edge
  __shared__ int64_t a_line[GB_BM], b_line[GB_BN], c_row[GB_BM], c_col[GB_BN];
  constexpr int64_t NONE = INT64_MIN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
  const int64_t tiles_m = (g.M + GB_BM - 1) / GB_BM, tiles_n = (g.N + GB_BN - 1) / GB_BN;
  const int64_t T = tiles_m * tiles_n;
  const int64_t per_xcd = (T + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= T) return;
  constexpr int64_t GROUP = 8;
  const int64_t in_group = GROUP * tiles_n;
  const int64_t first_m = (t / in_group) * GROUP;
  const int64_t gsize = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
  const int64_t tm = first_m + (t % in_group) % gsize, tn = (t % in_group) / gsize;
  const int64_t m0 = tm * GB_BM, n0 = tn * GB_BN;
  const int64_t bz = blockIdx.y;
  const float* A = (const float*)g.A + bz * g.a_b_i;
  const float* B = (const float*)g.B + bz * g.b_b_i;
  float* C = (float*)g.C + bz * g.c_b_i;
  const int64_t lda = A_KC ? 0 : g.a_k_i, ldb = B_NC ? g.b_k_i : 0;
  if (tid < GB_BM) {
    const int64_t m = m0 + tid;
    a_line[tid] = m < g.M ? split_off(m, g.m_in, g.a_m_o, g.a_m_i) : NONE;
    c_row[tid] = m < g.M ? split_off(m, g.m_in, g.c_m_o, g.c_m_i) : NONE;
  } else {
    const int j = tid - GB_BM;
    const int64_t n = n0 + j;
    b_line[j] = n < g.N ? split_off(n, g.n_in, g.b_n_o, g.b_n_i) : NONE;
    c_col[j] = n < g.N ? split_off(n, g.n_in, g.c_n_o, g.c_n_i) : NONE;
  }
  __syncthreads();

  // along the unit stride: thread -> lines tid/8 + 32 i (i < 4), elements 4 (tid % 8) .. +3 of the 32
  // across it: thread -> lines 4 (tid % 32) .. +3, elements 4 (tid / 32) + j (j < 4)
  const int s_r = tid >> 3, s_k = (tid & 7) * 4;
  const int x_n = (tid & 31) * 4, x_k = (tid >> 5) * 4;
  float4 ra[4], rb[4];
  // out-of-range elements read the operand's first element (always valid) and are zeroed after the load
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int64_t off;
      bool ok;
      if (A_KC) {   // line m of A, k contiguous
        const int64_t lo = a_line[s_r + 32 * i], k = k0 + s_k;
        ok = lo != NONE && k < g.K;
        off = lo + k;
      } else {      // m contiguous (one level): four rows m .. m + 3 at one k
        const int64_t k = k0 + x_k + i, m = m0 + x_n;
        ok = k < g.K && m < g.M;
        off = k * lda + m;
      }
      const float4 v = *(const float4*)(A + (ok ? off : 0));
      ra[i] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int64_t off;
      bool ok;
      if (B_NC) {   // n contiguous within its inner group: four columns n .. n + 3 at one k
        const int64_t lo = b_line[x_n], k = k0 + x_k + j;
        ok = lo != NONE && k < g.K;
        off = k * ldb + lo;
      } else {      // line n of B, k contiguous
        const int64_t lo = b_line[s_r + 32 * j], k = k0 + s_k;
        ok = lo != NONE && k < g.K;
        off = lo + k;
      }
      const float4 v = *(const float4*)(B + (ok ? off : 0));
      rb[j] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  // a 4 x 4 block read across the k-contiguous LDS rows goes in transposed
  auto put_transposed = [](unsigned short* S, int line, int k, const float4* r) {
    *(uint2*)&S[(line + 0) * GB_LD + k] = pack_bf16x4(r[0].x, r[1].x, r[2].x, r[3].x);
    *(uint2*)&S[(line + 1) * GB_LD + k] = pack_bf16x4(r[0].y, r[1].y, r[2].y, r[3].y);
    *(uint2*)&S[(line + 2) * GB_LD + k] = pack_bf16x4(r[0].z, r[1].z, r[2].z, r[3].z);
    *(uint2*)&S[(line + 3) * GB_LD + k] = pack_bf16x4(r[0].w, r[1].w, r[2].w, r[3].w);
  };
  auto stash = [&]() {
    if (A_KC) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        *(uint2*)&As[(s_r + 32 * i) * GB_LD + s_k] = pack_bf16x4(ra[i].x, ra[i].y, ra[i].z, ra[i].w);
    } else {
      put_transposed(As, x_n, x_k, ra);
    }
    if (B_NC) {
      put_transposed(Bs, x_n, x_k, rb);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *(uint2*)&Bs[(s_r + 32 * j) * GB_LD + s_k] = pack_bf16x4(rb[j].x, rb[j].y, rb[j].z, rb[j].w);
    }
  };

  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  load(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += GB_BK) {
    stash();
    __syncthreads();
    if (k0 + GB_BK < g.K) load(k0 + GB_BK);   // next tile in flight while the matrix cores work
    {
      // v_mfma_f32_16x16x32_bf16: lane (lr, lq) supplies row lr and k = 8 lq .. 8 lq + 7 of the
      // A fragment, column lr and the same k of the B fragment (one 16-byte LDS read each)
      typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
      bf8_t af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = *(const bf8_t*)&As[(wm + 16 * i + lr) * GB_LD + 8 * lq];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = *(const bf8_t*)&Bs[(wn + 16 * j + lr) * GB_LD + 8 * lq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout: register e of lane (lr, lq) is row 4 lq + e, column lr of the 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t co = c_col[wn + 16 * j + lr];
      if (co == NONE) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t ro = c_row[wm + 16 * i + 4 * lq + e];
        if (ro == NONE) continue;
        float v = (float)(g.alpha * (double)acc[i][j][e]);
        if (g.beta) v += C[ro + co];
        C[ro + co] = v;
      }
    }
}

// The products that take this path: one level for k (and for m when A has
// unit stride along m), a unit stride along k or m in A and along n or k in B
// (an index split in two levels keeps its lines 16-byte aligned), any layout
// of C, no column scale or K split, and large enough to fill the chip.
// Returns the variant (0..3: A_KC + 2 B_NC) or -1.
static int rowmajor_bf16_variant(const GemmArgs& g) {
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  // a two-level index keeps 16-byte alignment when both strides are multiples of 4 floats
  auto lines4 = [](int64_t n_in, int64_t n, int64_t so, int64_t si) { return si % 4 == 0 && (n_in == n || so % 4 == 0); };
  if (!(g.k_in == g.K && (g.batch == 1 || g.b_in == g.batch) && !g.colscale && g.ksplit <= 1 && g.a_b_i % 4 == 0 &&
        g.b_b_i % 4 == 0 && al16(g.A) && al16(g.B) && g.M >= 512 && g.N >= 512 && g.K >= 128 && g.K % 4 == 0))
    return -1;
  int v = 0;
  if (g.a_k_i == 1 && lines4(g.m_in, g.M, g.a_m_o, g.a_m_i)) v |= 1;
  else if (!(g.a_m_i == 1 && g.m_in == g.M && g.a_k_i % 4 == 0 && g.M % 4 == 0)) return -1;
  if (g.b_n_i == 1 && g.b_k_i % 4 == 0 && g.n_in % 4 == 0 && (g.n_in == g.N || g.b_n_o % 4 == 0) && g.N % 4 == 0) v |= 2;
  else if (!(g.b_k_i == 1 && lines4(g.n_in, g.N, g.b_n_o, g.b_n_i))) return -1;
  return v;
}

// ---------------------------------------------------------------------------
// Large FP64 or FP32 products with A contiguous along k and B along n: C[m][n]
// = alpha sum_k A[m][k] B[k][n] (+ C), e.g. the density-matrix joins and their
// adjoints in FP64 and FP32 mode.  A 128 x 128 tile per workgroup, 4 waves of
// 64 x 64 (4 x 4 tiles of v_mfma_f64_16x16x4f64 or v_mfma_f32_16x16x4f32),
// BK = 16, the next K tile in registers while the matrix cores work.  Operands
// are read as pairs and kept in LDS as As[k][m] and Bs[k][n], so that a lane's
// MFMA operand (A[m = lr][k = lq], B[k = lq][n = lr]) is a read along m or n.
// Tile order and line tables as in the BF16 kernel.
constexpr int GD_BM = 128, GD_BN = 128, GD_BK = 16, GD_LD = GD_BM + 2;

template <typename T>
__global__ __launch_bounds__(256) void gemm_mfma_rowmajor_kernel(GemmArgs g) {
  constexpr bool F64 = std::is_same<T, double>::value;
  typedef typename std::conditional<F64, double2, float2>::type pair_t;
  typedef typename std::conditional<F64, d4_t, f4_t>::type acc_t;
  __shared__ __align__(16) T As[GD_BK * GD_LD];
  __shared__ __align__(16) T Bs[GD_BK * GD_LD];
  __shared__ int64_t a_line[GD_BM], b_line[GD_BN], c_row[GD_BM], c_col[GD_BN];
  constexpr int64_t NONE = INT64_MIN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
  const int64_t tiles_m = (g.M + GD_BM - 1) / GD_BM, tiles_n = (g.N + GD_BN - 1) / GD_BN;
  const int64_t Tt = tiles_m * tiles_n;
  const int64_t per_xcd = (Tt + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= Tt) return;
  constexpr int64_t GROUP = 8;
  const int64_t in_group = GROUP * tiles_n;
  const int64_t first_m = (t / in_group) * GROUP;
  const int64_t gsize = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
  const int64_t tm = first_m + (t % in_group) % gsize, tn = (t % in_group) / gsize;
  const int64_t m0 = tm * GD_BM, n0 = tn * GD_BN;
  const int64_t bz = blockIdx.y;
  const T* A = (const T*)g.A + bz * g.a_b_i;
  const T* B = (const T*)g.B + bz * g.b_b_i;
  T* C = (T*)g.C + bz * g.c_b_i;
  const int64_t ldb = g.b_k_i;
  if (tid < GD_BM) {
    const int64_t m = m0 + tid;
    a_line[tid] = m < g.M ? split_off(m, g.m_in, g.a_m_o, g.a_m_i) : NONE;
    c_row[tid] = m < g.M ? split_off(m, g.m_in, g.c_m_o, g.c_m_i) : NONE;
  } else {
    const int j = tid - GD_BM;
    const int64_t n = n0 + j;
    b_line[j] = n < g.N ? split_off(n, g.n_in, g.b_n_o, g.b_n_i) : NONE;
    c_col[j] = n < g.N ? split_off(n, g.n_in, g.c_n_o, g.c_n_i) : NONE;
  }
  __syncthreads();
  // A: thread -> lines a_r + 32 i (i < 4), k pair 2 (tid % 8); B: thread -> columns
  // pair 2 (tid % 64), k rows b_k + 4 j (j < 4).  Pairs never straddle an index
  // group or the end (even extents and strides, checked on the host).
  const int a_r = tid >> 3, a_k = (tid & 7) * 2;
  const int b_n = (tid & 63) * 2, b_k = tid >> 6;
  pair_t ra[4], rb[4];
  // A line past the edge of the tile reads the operand's first pair instead
  // (always valid), which only reaches outputs that are not written.  FP32: K
  // is a multiple of BK, so every k read lies inside the sum.  FP64: pairs
  // past K are zeroed (written this way, the FP64 instance keeps its operands
  // in registers; without the select it spilled and ran at 25 instead of 41
  // TFLOP/s).
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t lo = a_line[a_r + 32 * i], k = k0 + a_k;
      if constexpr (F64) {
        const bool ok = lo != NONE && k < g.K;
        const double2 v = *(const double2*)(A + (ok ? lo + k : 0));
        ra[i] = ok ? v : make_double2(0.0, 0.0);
      } else {
        ra[i] = *(const pair_t*)(A + (lo != NONE ? lo + k : 0));
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t lo = b_line[b_n], k = k0 + b_k + 4 * j;
      if constexpr (F64) {
        const bool ok = lo != NONE && k < g.K;
        const double2 v = *(const double2*)(B + (ok ? k * ldb + lo : 0));
        rb[j] = ok ? v : make_double2(0.0, 0.0);
      } else {
        rb[j] = *(const pair_t*)(B + (lo != NONE ? k * ldb + lo : 0));
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      As[a_k * GD_LD + a_r + 32 * i] = ra[i].x;
      As[(a_k + 1) * GD_LD + a_r + 32 * i] = ra[i].y;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) *(pair_t*)&Bs[(b_k + 4 * j) * GD_LD + b_n] = rb[j];
  };
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{(T)0, (T)0, (T)0, (T)0};
  load(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += GD_BK) {
    stash();
    __syncthreads();
    if (k0 + GD_BK < g.K) load(k0 + GD_BK);
#pragma unroll
    for (int kk = 0; kk < GD_BK / 4; ++kk) {
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[(4 * kk + lq) * GD_LD + wm + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[(4 * kk + lq) * GD_LD + wn + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if constexpr (F64) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          else acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // D layout, register e of lane (lr, lq): column lr, row lq + 4 e (FP64) or 4 lq + e (FP32)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t co = c_col[wn + 16 * j + lr];
      if (co == NONE) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t ro = c_row[wm + 16 * i + (F64 ? lq + 4 * e : 4 * lq + e)];
        if (ro == NONE) continue;
        T v = (T)(g.alpha * (double)acc[i][j][e]);
        if (g.beta) v += C[ro + co];
        C[ro + co] = v;
      }
    }
}

// The FP64 / FP32 products that take the kernel above: one level for k (even;
// for FP32 a multiple of BK), A contiguous along k and B along n with every pair aligned
// inside one index group, any layout of C, no column scale or K split, large
// enough.
static bool rowmajor_mfma_ok(const GemmArgs& g, bool f64) {
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  return g.k_in == g.K && (g.batch == 1 || g.b_in == g.batch) && !g.colscale && g.ksplit <= 1 && g.a_b_i % 2 == 0 &&
         g.b_b_i % 2 == 0 && al16(g.A) && al16(g.B) && g.M >= 512 && g.N >= 512 && g.K >= 64 &&
         g.K % (f64 ? 2 : GD_BK) == 0 &&
         g.a_k_i == 1 && g.a_m_i % 2 == 0 && (g.m_in == g.M || g.a_m_o % 2 == 0) && g.b_n_i == 1 &&
         g.b_k_i % 2 == 0 && g.n_in % 2 == 0 && (g.n_in == g.N || g.b_n_o % 2 == 0) && g.N % 2 == 0;
}

bool g_rowmajor_path = true;
bool g_rowmajor_f64 = true;
bool g_rowmajor_f32 = true;

hipError_t launch_contract(int mode, const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  const bool mf64 = mode == MODE_F64 && g_rowmajor_f64, mf32 = mode == MODE_F32 && g_rowmajor_f32;
  if ((mf64 || mf32) && rowmajor_mfma_ok(g, mf64)) {
    const int64_t T = ((g.M + GD_BM - 1) / GD_BM) * ((g.N + GD_BN - 1) / GD_BN);
    const int64_t blocks = 8 * ((T + 7) / 8);
    if (blocks > 2147483647LL || g.batch > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks, (unsigned)g.batch);
    if (mf64) gemm_mfma_rowmajor_kernel<double><<<grid, 256, 0, s>>>(g);
    else gemm_mfma_rowmajor_kernel<float><<<grid, 256, 0, s>>>(g);
    return hipGetLastError();
  }
  const int v = mode == MODE_BF16 && g_rowmajor_path ? rowmajor_bf16_variant(g) : -1;
  if (v >= 0) {
    const int64_t T = ((g.M + GB_BM - 1) / GB_BM) * ((g.N + GB_BN - 1) / GB_BN);
    const int64_t blocks = 8 * ((T + 7) / 8);
    if (blocks > 2147483647LL || g.batch > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks, (unsigned)g.batch);
    switch (v) {
      case 0: gemm_bf16_rowmajor_kernel<false, false><<<grid, 256, 0, s>>>(g); break;
      case 1: gemm_bf16_rowmajor_kernel<true, false><<<grid, 256, 0, s>>>(g); break;
      case 2: gemm_bf16_rowmajor_kernel<false, true><<<grid, 256, 0, s>>>(g); break;
      default: gemm_bf16_rowmajor_kernel<true, true><<<grid, 256, 0, s>>>(g); break;
    }
    return hipGetLastError();
  }
  if (mode == MODE_F64) return launch_mode<MODE_F64>(g, s);
  if (mode == MODE_F32) return launch_mode<MODE_F32>(g, s);
  return launch_mode<MODE_BF16>(g, s);
}

// ---------------------------------------------------------------------------
// Strided copy with optional type conversion: out (contiguous, shape dims) is
// filled from in at offset sum_i idx_i * in_stride_i.  The flat index is split
// into per-axis indices by division, so the launcher first merges axes that
// are contiguous in both tensors (fewer divisions) and, when every index and
// offset fits in 31 bits, runs the 32-bit form: the device has no integer
// divide, and a 64-bit one costs several times the 32-bit sequence.
template <typename TI, typename TO, typename IT>
__global__ __launch_bounds__(256) void permute_kernel(PermArgs p, const TI* __restrict__ in, TO* __restrict__ out,
                                                      IT total) {
  for (IT e = (IT)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (IT)gridDim.x * blockDim.x) {
    IT r = e, off_in = 0, off_out = 0;
#pragma unroll
    for (int i = PERM_MAX_DIMS - 1; i >= 0; --i) {
      if (i >= p.ndim) continue;
      const IT d = (IT)p.dims[i];
      const IT q = r / d;
      const IT idx = r - q * d;
      r = q;
      off_in += idx * (IT)p.in_strides[i];
      off_out += idx * (IT)p.out_strides[i];
    }
    TO v = (TO)in[off_in];
    if (p.accumulate) out[off_out] += v; else out[off_out] = v;
  }
}

static unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// A permutation whose fastest output axis X is not the fastest input axis Y
// (in-stride 1) is a batch of 2-D transposes: 32 x 32 tiles go through LDS,
// read along Y and written along X, so that both sides are coalesced (the
// element loop above reads one element per cache line).  The other axes form
// the batch (blockIdx.y, decomposed over them in order).  Every element is
// converted and stored or added once, as above.
constexpr int TR_T = 32;
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void transpose_kernel(PermArgs p, int ax, const TI* __restrict__ in,
                                                        TO* __restrict__ out) {
  __shared__ TO tile[TR_T][TR_T + 1];
  const int X = p.ndim - 1;
  const int64_t dx = p.dims[X], dy = p.dims[ax];
  const int64_t tiles_x = (dx + TR_T - 1) / TR_T;
  const int64_t x0 = ((int64_t)blockIdx.x % tiles_x) * TR_T, y0 = ((int64_t)blockIdx.x / tiles_x) * TR_T;
  int64_t b = blockIdx.y, off_in = 0, off_out = 0;
  for (int i = X - 1; i >= 0; --i) {
    if (i == ax) continue;
    const int64_t q = b / p.dims[i], idx = b - q * p.dims[i];
    b = q;
    off_in += idx * p.in_strides[i];
    off_out += idx * p.out_strides[i];
  }
  const int tx = threadIdx.x % TR_T, ty = threadIdx.x / TR_T;
  // rows of the tile: x; columns: y (the input's unit stride along the lanes)
  for (int r = ty; r < TR_T; r += 256 / TR_T) {
    const int64_t x = x0 + r, y = y0 + tx;
    if (x < dx && y < dy) tile[r][tx] = (TO)in[off_in + x * p.in_strides[X] + y * p.in_strides[ax]];
  }
  __syncthreads();
  for (int r = ty; r < TR_T; r += 256 / TR_T) {
    const int64_t y = y0 + r, x = x0 + tx;
    if (x < dx && y < dy) {
      TO* o = out + off_out + y * p.out_strides[ax] + x * p.out_strides[X];
      if (p.accumulate) *o += tile[tx][r]; else *o = tile[tx][r];
    }
  }
}

template <typename TI, typename TO>
static void permute_launch(const PermArgs& p, const void* in, void* out, int64_t total, bool narrow, hipStream_t s) {
  if (p.ndim >= 2) {
    const int X = p.ndim - 1;
    int ax = -1;
    for (int i = 0; i < X; ++i)
      if (p.in_strides[i] == 1) ax = i;
    if (ax >= 0 && p.out_strides[X] == 1 && p.in_strides[X] != 1 && p.dims[X] >= 8 && p.dims[ax] >= 8) {
      const int64_t tiles = ((p.dims[X] + TR_T - 1) / TR_T) * ((p.dims[ax] + TR_T - 1) / TR_T);
      const int64_t nbatch = total / (p.dims[X] * p.dims[ax]);
      if (tiles <= 2147483647LL && nbatch <= 65535) {
        transpose_kernel<TI, TO><<<dim3((unsigned)tiles, (unsigned)nbatch), 256, 0, s>>>(p, ax, (const TI*)in, (TO*)out);
        return;
      }
    }
  }
  const unsigned gb = grid_for(total);
  if (narrow)
    permute_kernel<TI, TO, uint32_t><<<gb, 256, 0, s>>>(p, (const TI*)in, (TO*)out, (uint32_t)total);
  else
    permute_kernel<TI, TO, int64_t><<<gb, 256, 0, s>>>(p, (const TI*)in, (TO*)out, total);
}

hipError_t launch_permute(const PermArgs& p0, int in_type, const void* in, int out_type, void* out, hipStream_t s) {
  int64_t total = 1;
  for (int i = 0; i < p0.ndim; ++i) total *= p0.dims[i];
  if (total <= 0) return hipSuccess;
  // merge axis i+1 into axis i where both tensors step over the pair as one axis
  PermArgs p = p0;
  int nd = 0;
  for (int i = 0; i < p0.ndim; ++i) {
    if (nd > 0 && p.out_strides[nd - 1] == p0.out_strides[i] * p0.dims[i] &&
        p.in_strides[nd - 1] == p0.in_strides[i] * p0.dims[i]) {
      p.dims[nd - 1] *= p0.dims[i];
      p.out_strides[nd - 1] = p0.out_strides[i];
      p.in_strides[nd - 1] = p0.in_strides[i];
      continue;
    }
    p.dims[nd] = p0.dims[i];
    p.in_strides[nd] = p0.in_strides[i];
    p.out_strides[nd] = p0.out_strides[i];
    ++nd;
  }
  p.ndim = nd;
  // 32-bit form: flat index (plus one grid stride) and both largest offsets below 2^31
  const int64_t lim = (int64_t)1 << 31;
  bool narrow = total + (int64_t)grid_for(total) * 256 < lim;
  int64_t max_in = 0, max_out = 0;
  for (int i = 0; i < nd; ++i) {
    if (p.in_strides[i] < 0 || p.out_strides[i] < 0 || p.dims[i] >= lim) narrow = false;
    max_in += (p.dims[i] - 1) * p.in_strides[i];
    max_out += (p.dims[i] - 1) * p.out_strides[i];
  }
  narrow = narrow && max_in < lim && max_out < lim;
  if (in_type == 0 && out_type == 0) permute_launch<double, double>(p, in, out, total, narrow, s);
  else if (in_type == 1 && out_type == 1) permute_launch<float, float>(p, in, out, total, narrow, s);
  else if (in_type == 0 && out_type == 1) permute_launch<double, float>(p, in, out, total, narrow, s);
  else permute_launch<float, double>(p, in, out, total, narrow, s);
  return hipGetLastError();
}

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

__global__ void fill_int_kernel(int* p, int v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

hipError_t launch_fill_int(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_int_kernel<<<grid_for(n), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill(int type, void* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (type == 0) fill_kernel<double><<<grid_for(n), 256, 0, s>>>((double*)p, v, n);
  else fill_kernel<float><<<grid_for(n), 256, 0, s>>>((float*)p, (float)v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Relative width of a tie in the gauge rules.  Entries whose magnitudes are
// equal in exact arithmetic (the ket-bra exchange symmetry of a reduced tensor
// makes such pairs in every projector column of the double-layer network)
// differ by rounding only; the sign is taken from the first entry within this
// width of the largest magnitude, which does not depend on where the rounding
// falls.
constexpr double kGaugeTie = 1e-9;

// Index of the sign-deciding entry of x[0], x[stride], ..., x[(n-1) stride] in
// one workgroup of 256 threads: the largest magnitude m (a max reduction),
// then the smallest index with |x| >= (1 - kGaugeTie) m (a min reduction);
// 0 when n = 0.  All threads receive the index.
template <typename T>
__device__ int64_t sign_entry_256(const T* x, int64_t n, int64_t stride, double* sv, int64_t* si) {
  double best = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) best = fmax(best, fabs((double)x[i * stride]));
  sv[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + w]);
    __syncthreads();
  }
  const double thr = sv[0] * (1.0 - kGaugeTie);
  int64_t bi = n;
  for (int64_t i = threadIdx.x; i < n; i += 256)
    if (fabs((double)x[i * stride]) >= thr) { bi = i; break; }
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w && si[threadIdx.x + w] < si[threadIdx.x]) si[threadIdx.x] = si[threadIdx.x + w];
    __syncthreads();
  }
  const int64_t r = si[0] < n ? si[0] : 0;
  __syncthreads();
  return r;
}

// Frobenius normalisation of a list of tensors with the sign that makes the
// entry chosen by the gauge rule positive: x <- sign * x / |x|, the sums of
// squares accumulated in FP64.  Three launches, so that a tensor is read by
// NORM_CHUNKS workgroups instead of one:
//  * norm_parts_kernel: per chunk of a tensor, the sum of squares and the
//    largest magnitude (fixed-order trees);
//  * norm_sign_kernel, one workgroup per tensor: the norm (chunk sums added in
//    chunk order), the largest magnitude m, and the sign-deciding entry, the
//    first with |x| >= (1 - kGaugeTie) m: it lies in the first chunk whose
//    largest magnitude reaches that threshold (every earlier chunk stays
//    below it), which is scanned alone; the factor sign / |x| goes to
//    factor[t], and optionally the signed norm sign * |x| (its reciprocal is
//    the factor the adjoint needs) to norm_out;
//  * norm_scale_kernel: x <- factor * x.
// The chosen entry is the one a scan of the whole tensor would choose.
template <typename T>
__global__ __launch_bounds__(256) void norm_parts_kernel(NormList L, double* part) {
  const int ch = blockIdx.x, t = blockIdx.y;
  const T* x = (const T*)L.ptr[t];
  const int64_t n = L.n[t], len = (n + NORM_CHUNKS - 1) / NORM_CHUNKS;
  const int64_t i0 = (int64_t)ch * len, i1 = i0 + len < n ? i0 + len : n;
  double s = 0.0, m = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double v = (double)x[i];
    s += v * v;
    m = fmax(m, fabs(v));
  }
  __shared__ double rs[256], rm[256];
  rs[threadIdx.x] = s;
  rm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)t * NORM_CHUNKS + ch) * 2] = rs[0];
    part[((int64_t)t * NORM_CHUNKS + ch) * 2 + 1] = rm[0];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void norm_sign_kernel(NormList L, const double* part, double* factor) {
  static_assert(NORM_CHUNKS <= 256, "one thread per chunk");
  const int t = blockIdx.x;
  const T* x = (const T*)L.ptr[t];
  const int64_t n = L.n[t], len = (n + NORM_CHUNKS - 1) / NORM_CHUNKS;
  const double* pt = part + (int64_t)t * NORM_CHUNKS * 2;
  __shared__ double m_s, thr_s;
  __shared__ int64_t first[256];
  __shared__ int chunk_s;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int ch = 0; ch < NORM_CHUNKS; ++ch) m = fmax(m, pt[2 * ch + 1]);
    const double thr = m * (1.0 - kGaugeTie);
    int c0 = 0;
    while (c0 < NORM_CHUNKS - 1 && !(pt[2 * c0 + 1] >= thr)) ++c0;
    m_s = m;
    thr_s = thr;
    chunk_s = c0;
  }
  __syncthreads();
  const double thr = thr_s;
  const int64_t i0 = (int64_t)chunk_s * len, i1 = i0 + len < n ? i0 + len : n;
  int64_t bi = n;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256)
    if (fabs((double)x[i]) >= thr) { bi = i; break; }
  first[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w && first[threadIdx.x + w] < first[threadIdx.x]) first[threadIdx.x] = first[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int ch = 0; ch < NORM_CHUNKS; ++ch) s += pt[2 * ch];
    const double nrm = sqrt(s);
    const int64_t im = first[0] < n ? first[0] : 0;
    const double sg = (n > 0 && (double)x[im] < 0.0) ? -1.0 : 1.0;
    if (L.norm_out) L.norm_out[t] = sg * nrm;
    // an updated environment tensor that is zero has lost the whole environment
    if (L.zero_flag && !(nrm > 0.0)) atomicAdd(L.zero_flag, 1);
    factor[t] = nrm > 0.0 ? sg / nrm : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void norm_scale_kernel(NormList L, const double* factor) {
  const int ch = blockIdx.x, t = blockIdx.y;
  T* x = (T*)L.ptr[t];
  const int64_t n = L.n[t], len = (n + NORM_CHUNKS - 1) / NORM_CHUNKS;
  const int64_t i0 = (int64_t)ch * len, i1 = i0 + len < n ? i0 + len : n;
  const double f = factor[t];
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) x[i] = (T)((double)x[i] * f);
}

int64_t normalize_work_doubles(int count) { return (int64_t)count * (2 * NORM_CHUNKS + 1); }

hipError_t launch_normalize(int type, const NormList& L, int count, double* work, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > NORM_MAX) return hipErrorInvalidValue;
  double* part = work;
  double* factor = work + (int64_t)count * 2 * NORM_CHUNKS;
  const dim3 grid(NORM_CHUNKS, (unsigned)count);
  if (type == 0) {
    norm_parts_kernel<double><<<grid, 256, 0, s>>>(L, part);
    norm_sign_kernel<double><<<count, 256, 0, s>>>(L, part, factor);
    norm_scale_kernel<double><<<grid, 256, 0, s>>>(L, factor);
  } else {
    norm_parts_kernel<float><<<grid, 256, 0, s>>>(L, part);
    norm_sign_kernel<float><<<count, 256, 0, s>>>(L, part, factor);
    norm_scale_kernel<float><<<grid, 256, 0, s>>>(L, factor);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Projector weights: w_k = s_k^(-1/2) for k < chi when s_k > cutoff * s_0,
// zero otherwise (pseudo-inverse); batched over ``batch`` spectra of length r.
__global__ void svd_weights_kernel(const double* s, int64_t r, int64_t stride_s, double* w, int64_t chi,
                                   double cutoff, int batch) {
  int b = blockIdx.x;
  const double* sb = s + b * stride_s;
  double thr = cutoff * sb[0];
  for (int64_t k = threadIdx.x; k < chi; k += blockDim.x) {
    double v = k < r ? sb[k] : 0.0;
    w[b * chi + k] = (k < r && v > thr) ? 1.0 / sqrt(v) : 0.0;
  }
}

hipError_t launch_svd_weights(const double* s, int64_t r, int64_t stride_s, double* w, int64_t chi, double cutoff,
                              int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  svd_weights_kernel<<<batch, 128, 0, st>>>(s, r, stride_s, w, chi, cutoff, batch);
  return hipGetLastError();
}

// Gauge of the projectors: for row t and kept column k, the sign of the entry
// of P[:, k] chosen by sign_entry_256; if negative, column k of
// P, Q (kd x chi, row-major) and of the singular vectors U, V (column-major,
// r rows, column stride r) is negated (another valid SVD of M).
__global__ __launch_bounds__(256) void proj_signs_kernel(SignList L, int64_t chi, int64_t r) {
  const int k = blockIdx.x, t = blockIdx.y;
  double* P = L.P[t];
  const int64_t kd = L.kd[t];
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  // column k of P is the strided sequence P[a * chi + k], a < kd
  const int64_t im = sign_entry_256(P + k, kd, chi, sv, si);
  if (!(P[im * chi + k] < 0.0)) return;   // uniform across the workgroup
  double* Q = L.Q[t];
  for (int64_t a = threadIdx.x; a < kd; a += 256) {
    P[a * chi + k] = -P[a * chi + k];
    Q[a * chi + k] = -Q[a * chi + k];
  }
  double* U = L.U[t] + (int64_t)k * r;
  double* V = L.V[t] + (int64_t)k * r;
  for (int64_t i = threadIdx.x; i < r; i += 256) {
    U[i] = -U[i];
    V[i] = -V[i];
  }
}

hipError_t launch_proj_signs(const SignList& L, int count, int64_t chi, int64_t r, hipStream_t s) {
  if (count <= 0 || chi <= 0) return hipSuccess;
  if (count > CUT_MAX) return hipErrorInvalidValue;
  proj_signs_kernel<<<dim3((unsigned)chi, (unsigned)count), 256, 0, s>>>(L, chi, r);
  return hipGetLastError();
}

// Density matrices rho_b (dim x dim, row-major, b < count, contiguous) divided
// by their traces, one workgroup each.
__global__ void rdm_normalize_kernel(double* rho, int64_t dim) {
  double* r = rho + (int64_t)blockIdx.x * dim * dim;
  double tr = 0.0;
  for (int64_t i = 0; i < dim; ++i) tr += r[i * dim + i];
  __syncthreads();   // every thread has read the diagonal before any is rescaled
  const double inv = 1.0 / tr;
  for (int64_t e = threadIdx.x; e < dim * dim; e += blockDim.x) r[e] *= inv;
}

hipError_t launch_rdm_normalize(double* rho, int count, int64_t dim, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  rdm_normalize_kernel<<<count, 256, 0, s>>>(rho, dim);
  return hipGetLastError();
}

// Empty cuts: for row t, with R_n^T and R_s^T of its half systems (Frobenius
// norms those of N and S) and the largest singular value s_1 of M = R_n R_s^T,
// count the row in *flag when s_1 <= tau |N|_F |S|_F (the bond density matrix
// N S^T vanishes to working precision and Lambda~^(-1/2) is undefined).
// First pass: workgroup (c, t) sums the squares of its chunk c of both
// factors of row t into part[(t * CUT_CHUNKS + c) * 2 + {0, 1}].
__global__ __launch_bounds__(256) void cut_norms_kernel(CutList L, double* part) {
  const int c = blockIdx.x, t = blockIdx.y;
  const int64_t n = L.n[t], len = (n + CUT_CHUNKS - 1) / CUT_CHUNKS;
  const int64_t lo = (int64_t)c * len, hi = lo + len < n ? lo + len : n;
  const double* a = L.Ln[t];
  const double* b = L.Ls[t];
  double sa = 0.0, sb = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    sa += a[i] * a[i];
    sb += b[i] * b[i];
  }
  __shared__ double ra[256], rb[256];
  ra[threadIdx.x] = sa;
  rb[threadIdx.x] = sb;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rb[threadIdx.x] += rb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)t * CUT_CHUNKS + c) * 2] = ra[0];
    part[((int64_t)t * CUT_CHUNKS + c) * 2 + 1] = rb[0];
  }
}

// Second pass: thread t adds up row t's chunks in order and tests the cut.
__global__ void cut_check_kernel(CutList L, int count, double tau, const double* part, int* flag) {
  const int t = threadIdx.x;
  if (t >= count) return;
  double na = 0.0, nb = 0.0;
  for (int c = 0; c < CUT_CHUNKS; ++c) {
    na += part[((int64_t)t * CUT_CHUNKS + c) * 2];
    nb += part[((int64_t)t * CUT_CHUNKS + c) * 2 + 1];
  }
  if (!(*L.s1[t] > tau * sqrt(na) * sqrt(nb))) atomicAdd(flag, 1);
}

hipError_t launch_cut_check(const CutList& L, int count, double tau, double* work, int* flag, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > CUT_MAX) return hipErrorInvalidValue;
  cut_norms_kernel<<<dim3(CUT_CHUNKS, (unsigned)count), 256, 0, s>>>(L, work);
  cut_check_kernel<<<1, CUT_MAX, 0, s>>>(L, count, tau, work, flag);
  return hipGetLastError();
}

// Lower-trapezoidal factor of an LQ factorisation (column-major rows x cols,
// leading dimension lda) copied to a dense column-major rows x rcols matrix
// with the Householder data above the diagonal replaced by zeros.
__global__ void extract_lower_kernel(const double* a, int64_t rows, int64_t lda, int64_t stride_a, double* l,
                                     int64_t rcols, int64_t stride_l, int batch) {
  int64_t total = rows * rcols * batch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = t / (rows * rcols), e = t - b * rows * rcols;
    int64_t j = e / rows, i = e - j * rows;
    l[b * stride_l + e] = i >= j ? a[b * stride_a + i + j * lda] : 0.0;
  }
}

hipError_t launch_extract_lower(const double* a, int64_t rows, int64_t lda, int64_t stride_a, double* l, int64_t rcols,
                                int64_t stride_l, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  extract_lower_kernel<<<grid_for(rows * rcols * batch), 256, 0, s>>>(a, rows, lda, stride_a, l, rcols, stride_l, batch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Energy from plaquette density matrices rho[(k1 k2 k3 k4), (b1 b2 b3 b4)]
// (d^4 x d^4, row-major, FP64): E = (1/n_sites) sum_t coef_t Tr(h rho_ab)/Tr rho
// with <h> = sum h[(b_a b_b), (k_a k_b)] rho_ab[(k_a k_b), (b_a b_b)].
__global__ void energy_kernel(const double* rho, int64_t rho_stride, const double* h, const EnergyTerm* terms,
                              int n_terms, int d, double inv_sites, double* E_out, double* bond_out) {
  __shared__ double part[256];
  double acc = 0.0;
  int D4 = d * d * d * d;
  for (int t = threadIdx.x; t < n_terms; t += blockDim.x) {
    const EnergyTerm tm = terms[t];
    const double* r = rho + tm.rho_index * rho_stride;
    double tr = 0.0;
    for (int i = 0; i < D4; ++i) tr += r[(int64_t)i * D4 + i];
    double val = 0.0;
    int dd[4] = {d * d * d, d * d, d, 1};
    for (int ka = 0; ka < d; ++ka)
      for (int kb = 0; kb < d; ++kb)
        for (int ba = 0; ba < d; ++ba)
          for (int bb = 0; bb < d; ++bb) {
            double hv = h[(ba * d + bb) * d * d + ka * d + kb];
            if (hv == 0.0) continue;
            // partial trace over the two other sites q1 < q2
            int q1 = -1, q2 = -1;
            for (int q = 0; q < 4; ++q)
              if (q != tm.a && q != tm.b) { if (q1 < 0) q1 = q; else q2 = q; }
            double rab = 0.0;
            for (int o1 = 0; o1 < d; ++o1)
              for (int o2 = 0; o2 < d; ++o2) {
                int ko[4], bo[4];
                ko[tm.a] = ka; ko[tm.b] = kb; bo[tm.a] = ba; bo[tm.b] = bb;
                ko[q1] = bo[q1] = o1;
                ko[q2] = bo[q2] = o2;
                int ik = 0, ib = 0;
                for (int q = 0; q < 4; ++q) { ik += ko[q] * dd[q]; ib += bo[q] * dd[q]; }
                rab += r[(int64_t)ik * D4 + ib];
              }
            val += hv * rab;
          }
    double bond = val / tr;
    if (bond_out) bond_out[t] = bond;
    acc += tm.coef * bond;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E_out = part[0] * inv_sites;
}

hipError_t launch_energy(const double* rho, int64_t rho_stride, const double* h, const EnergyTerm* terms, int n_terms,
                         int d, double inv_sites, double* E_out, double* bond_out, hipStream_t s) {
  energy_kernel<<<1, 256, 0, s>>>(rho, rho_stride, h, terms, n_terms, d, inv_sites, E_out, bond_out);
  return hipGetLastError();
}

// Order parameters of spin-1/2 plaquettes (Eqs. Mag1, Mag2) from the density
// matrices of the energy, rho[(k1 k2 k3 k4), (b1 b2 b3 b4)] (16 x 16, FP64, site
// q at digit weight 2^(3-q); sites TL, TR, BL, BR; basis up, down).  One
// workgroup per plaquette, one thread per output: slots 0..11 the moments
// (<S^x>, <S^y>, <S^z>) of the four sites, <O> = Tr(O rho_s) / Tr rho_s over the
// one-site matrix; slots 12..17 <S_a . S_b> over the two-site matrix of the
// pairs (TL,TR) (BL,BR) (TL,BL) (TR,BR) (TL,BR) (TR,BL).  Real rho: <S^y> is the
// real part of an imaginary trace, zero.
__global__ __launch_bounds__(64) void observables_kernel(const double* __restrict__ rho, int64_t rho_stride,
                                                         double* __restrict__ out) {
  constexpr int NOBS = 18;
  const int slot = threadIdx.x;
  if (slot >= NOBS) return;
  const double* r = rho + (int64_t)blockIdx.x * rho_stride;
  double v = 0.0;
  if (slot < 12) {
    const int s = slot / 3, comp = slot % 3, w = 8 >> s;
    double rs[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int o = 0; o < 16; ++o) {
      if (o & w) continue;   // o runs over the configurations of the three other sites
      for (int k = 0; k < 2; ++k)
        for (int b = 0; b < 2; ++b) rs[k][b] += r[(int64_t)(o | (k * w)) * 16 + (o | (b * w))];
    }
    const double tr = rs[0][0] + rs[1][1];
    if (comp == 0) v = 0.5 * (rs[0][1] + rs[1][0]) / tr;
    else if (comp == 2) v = 0.5 * (rs[0][0] - rs[1][1]) / tr;
  } else {
    const int pa[6] = {0, 2, 0, 1, 0, 1}, pb[6] = {1, 3, 2, 3, 3, 2};
    const int wa = 8 >> pa[slot - 12], wb = 8 >> pb[slot - 12];
    double r2[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) r2[i][j] = 0.0;
    for (int o = 0; o < 16; ++o) {
      if (o & (wa | wb)) continue;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          const int ki = o | ((i >> 1) * wa) | ((i & 1) * wb), bj = o | ((j >> 1) * wa) | ((j & 1) * wb);
          r2[i][j] += r[(int64_t)ki * 16 + bj];
        }
    }
    // S_a . S_b = S^z S^z + (S^+ S^- + S^- S^+) / 2 in the basis (uu, ud, du, dd)
    const double tr = r2[0][0] + r2[1][1] + r2[2][2] + r2[3][3];
    v = (0.25 * (r2[0][0] + r2[3][3] - r2[1][1] - r2[2][2]) + 0.5 * (r2[1][2] + r2[2][1])) / tr;
  }
  out[(int64_t)blockIdx.x * NOBS + slot] = v;
}

hipError_t launch_observables(const double* rho, int64_t rho_stride, int n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  observables_kernel<<<n, 64, 0, s>>>(rho, rho_stride, out);
  return hipGetLastError();
}

// Non-finite detector: sets *flag = 1 if any entry of x is NaN or Inf.
template <typename T>
__global__ void nonfinite_kernel(const T* x, int64_t n, int* flag) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double v = (double)x[e];
    if (!(v == v) || v - v != 0.0) atomicOr(flag, 1);
  }
}

hipError_t launch_nonfinite(int type, const void* x, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (type == 0) nonfinite_kernel<double><<<grid_for(n), 256, 0, s>>>((const double*)x, n, flag);
  else nonfinite_kernel<float><<<grid_for(n), 256, 0, s>>>((const float*)x, n, flag);
  return hipGetLastError();
}

// Largest |a_i - b_i| (b == nullptr: largest |a_i|) over n entries, into
// *out (zero before the launch): per-workgroup maxima combined by an atomic
// maximum on the bit pattern (non-negative doubles order as their bits).
template <typename T>
__global__ __launch_bounds__(256) void max_abs_kernel(const T* a, const T* b, int64_t n, unsigned long long* out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = b ? (double)a[i] - (double)b[i] : (double)a[i];
    m = fmax(m, fabs(v));
  }
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

hipError_t launch_max_abs(int type, const void* a, const void* b, int64_t n, double* out, hipStream_t s) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(double), s);
  if (e != hipSuccess || n <= 0) return e;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  if (type == 0)
    max_abs_kernel<double><<<(unsigned)blocks, 256, 0, s>>>((const double*)a, (const double*)b, n,
                                                           (unsigned long long*)out);
  else
    max_abs_kernel<float><<<(unsigned)blocks, 256, 0, s>>>((const float*)a, (const float*)b, n,
                                                          (unsigned long long*)out);
  return hipGetLastError();
}

// Spectra test: for each of ``count`` spectra of length r (descending singular
// values), normalise to unit sum, store, and reduce max_c sum_k |s_k - prev_k|.
__global__ void spectra_delta_kernel(const double* sv, int64_t r, int64_t chi, double* cur, const double* prev,
                                     int count, double* delta_out) {
  __shared__ double best[256];
  double mx = 0.0;
  for (int c = threadIdx.x; c < count; c += blockDim.x) {
    const double* s = sv + (int64_t)c * r;
    double tot = 0.0;
    for (int64_t k = 0; k < r; ++k) tot += s[k];
    double inv = tot > 0.0 ? 1.0 / tot : 0.0;
    double d = 0.0;
    for (int64_t k = 0; k < chi; ++k) {
      double v = k < r ? s[k] * inv : 0.0;
      cur[(int64_t)c * chi + k] = v;
      if (prev) d += fabs(v - prev[(int64_t)c * chi + k]);
    }
    mx = fmax(mx, d);
  }
  best[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) best[threadIdx.x] = fmax(best[threadIdx.x], best[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *delta_out = prev ? best[0] : 1e300;
}

hipError_t launch_spectra_delta(const double* sv, int64_t r, int64_t chi, double* cur, const double* prev, int count,
                                double* delta_out, hipStream_t s) {
  spectra_delta_kernel<<<1, 256, 0, s>>>(sv, r, chi, cur, prev, count, delta_out);
  return hipGetLastError();
}

// flag |= (any src[i] != 0), for solver status codes
__global__ void flag_or_kernel(const int* src, int n, int* flag) {
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (src[i] != 0) atomicOr(flag, 1);
}

hipError_t launch_flag_or(const int* src, int n, int* flag, hipStream_t s) {
  flag_or_kernel<<<1, 64, 0, s>>>(src, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched one-sided (Hestenes) Jacobi SVD of n x n column-major matrices A_b:
// column pairs are rotated until all columns are mutually orthogonal, then
// A_b V_b = U_b diag(s_b).  One wave per column pair; the pairs of a round of
// the round-robin tournament are disjoint and run in one launch.  A pair (p,q)
// is rotated when |a_p . a_q| > tol sqrt(|a_p|^2 |a_q|^2); ``rot`` counts the
// rotations of the current sweep (one counter per matrix).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(64) void jacobi_round_kernel(double* A, double* V, int64_t n, int64_t np, int64_t stride,
                                                          int round, double tol, const double* tiny2, int* rot) {
  const int k = blockIdx.x;            // pair index within the round
  const int b = blockIdx.y;            // matrix
  const int lane = threadIdx.x;
  // tournament pairing over np (even) players; player np-1 is fixed
  int64_t p, q;
  if (k == 0) { p = round; q = np - 1; }
  else { p = (round + k) % (np - 1); q = (round - k + (np - 1)) % (np - 1); }
  if (p >= n || q >= n) return;        // padding player for odd n
  if (p > q) { int64_t t = p; p = q; q = t; }
  double* Ab = A + (int64_t)b * stride;
  double* Vb = V + (int64_t)b * stride;
  double* ap = Ab + p * n;
  double* aq = Ab + q * n;
  double al = 0, be = 0, ga = 0;
  for (int64_t i = lane; i < n; i += 64) {
    double x = ap[i], y = aq[i];
    al += x * x; be += y * y; ga += x * y;
  }
  al = wave_sum(al); be = wave_sum(be); ga = wave_sum(ga);
  // columns below eps*|A|_F are numerically zero: rotating them only moves rounding noise
  if (fmin(al, be) <= tiny2[b] || ga == 0.0 || fabs(ga) <= tol * sqrt(al * be)) return;
  double zeta = (be - al) / (2.0 * ga);
  double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
  for (int64_t i = lane; i < n; i += 64) {
    double x = ap[i], y = aq[i];
    ap[i] = c * x - sn * y;
    aq[i] = sn * x + c * y;
  }
  double* vp = Vb + p * n;
  double* vq = Vb + q * n;
  for (int64_t i = lane; i < n; i += 64) {
    double x = vp[i], y = vq[i];
    vp[i] = c * x - sn * y;
    vq[i] = sn * x + c * y;
  }
  if (lane == 0) atomicAdd(rot + b, 1);
}

hipError_t launch_jacobi_round(double* A, double* V, int64_t n, int64_t stride, int batch, int round, double tol,
                               const double* tiny2, int* rot, hipStream_t s) {
  int64_t np = n + (n & 1);
  dim3 grid((unsigned)(np / 2), (unsigned)batch);
  jacobi_round_kernel<<<grid, 64, 0, s>>>(A, V, n, np, stride, round, tol, tiny2, rot);
  return hipGetLastError();
}

// tiny2[b] = (eps * |A_b|_F)^2: FROB_CHUNKS workgroups per matrix sum the
// squares of a chunk each (float64, fixed-order tree), then one thread per
// matrix adds the chunk sums in chunk order.
constexpr int FROB_CHUNKS = 64;
__global__ __launch_bounds__(256) void frob_parts_kernel(const double* A, int64_t len, int64_t stride, double* part) {
  __shared__ double red[256];
  const int ch = blockIdx.x, b = blockIdx.y;
  const double* Ab = A + (int64_t)b * stride;
  const int64_t cl = (len + FROB_CHUNKS - 1) / FROB_CHUNKS;
  const int64_t i0 = (int64_t)ch * cl, i1 = i0 + cl < len ? i0 + cl : len;
  double s = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += Ab[i] * Ab[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)b * FROB_CHUNKS + ch] = red[0];
}

__global__ void frob_tiny_kernel(const double* part, int batch, double eps, double* tiny2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double s = 0;
  for (int ch = 0; ch < FROB_CHUNKS; ++ch) s += part[(int64_t)b * FROB_CHUNKS + ch];
  tiny2[b] = eps * eps * s;
}

int64_t frob_tiny_work_doubles(int batch) { return (int64_t)batch * FROB_CHUNKS; }

hipError_t launch_frob_tiny(const double* A, int64_t len, int64_t stride, int batch, double eps, double* tiny2,
                            double* work, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  frob_parts_kernel<<<dim3(FROB_CHUNKS, (unsigned)batch), 256, 0, s>>>(A, len, stride, work);
  frob_tiny_kernel<<<(batch + 63) / 64, 64, 0, s>>>(work, batch, eps, tiny2);
  return hipGetLastError();
}

// X_b = R_b^T for the upper-triangular factor R_b stored by a QR factorisation
// in the upper triangle of A_b (column-major n x n).
__global__ void rt_from_qr_kernel(const double* A, double* X, int64_t n, int64_t stride, int batch) {
  int64_t total = n * n * batch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = t / (n * n), e = t - b * n * n;
    int64_t j = e / n, i = e - j * n;
    X[b * stride + e] = i >= j ? A[b * stride + j + i * n] : 0.0;
  }
}

hipError_t launch_rt_from_qr(const double* A, double* X, int64_t n, int64_t stride, int batch, hipStream_t s) {
  rt_from_qr_kernel<<<grid_for(n * n * batch), 256, 0, s>>>(A, X, n, stride, batch);
  return hipGetLastError();
}

__global__ void identity_kernel(double* V, int64_t n, int64_t stride, int batch) {
  int64_t total = n * n * batch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = t % (n * n);
    V[(t / (n * n)) * stride + e] = (e % n == e / n) ? 1.0 : 0.0;
  }
}

hipError_t launch_identity(double* V, int64_t n, int64_t stride, int batch, hipStream_t s) {
  identity_kernel<<<grid_for(n * n * batch), 256, 0, s>>>(V, n, stride, batch);
  return hipGetLastError();
}

// After convergence: s_j = |a_j|; the k largest (k <= kmax) in descending
// order go to sv[b][k], their left vectors a_j / s_j to U[b] (n x kmax,
// column-major) and right vectors to Vk[b] (n x kmax); all n sorted values are
// written to sv (length n per matrix).  Three launches:
//  * col_norms_kernel: one wave per column (rows across the lanes, then a
//    butterfly over the wave), four columns per workgroup;
//  * rank_kernel, one workgroup of 1024 threads per matrix: ranks by counting
//    (ties broken by column index), the sorted values and the column of each
//    rank;
//  * gather_kernel: the selected columns, scaled, with the elements across
//    the whole grid.
// work holds n norms and then n ranks (as int) per matrix.
__global__ __launch_bounds__(256) void col_norms_kernel(const double* A, int64_t n, int64_t stride, double* nrm) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y;
  if (j >= n) return;
  const double* Ab = A + (int64_t)b * stride;
  double s = 0;
  for (int64_t i = lane; i < n; i += 64) { const double x = Ab[j * n + i]; s += x * x; }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) nrm[(int64_t)b * n + j] = sqrt(s);
}

__global__ __launch_bounds__(1024) void rank_kernel(const double* nrm_g, int64_t n, double* sv, int* by_rank_g) {
  extern __shared__ double nrm[];
  const int b = blockIdx.x;
  for (int64_t j = threadIdx.x; j < n; j += 1024) nrm[j] = nrm_g[(int64_t)b * n + j];
  __syncthreads();
  for (int64_t j = threadIdx.x; j < n; j += 1024) {
    const double v = nrm[j];
    int64_t rank = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double w = nrm[i];
      rank += (w > v) || (w == v && i < j);
    }
    sv[(int64_t)b * n + rank] = v;
    by_rank_g[(int64_t)b * n + rank] = (int)j;
  }
}

__global__ void gather_kernel(const double* __restrict__ A, const double* __restrict__ V, int64_t n, int64_t stride,
                              int64_t kk, int64_t kmax, const double* __restrict__ nrm, const int* __restrict__ by_rank,
                              int batch, double* __restrict__ U, double* __restrict__ Vk) {
  const int64_t total = kk * n * batch;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / (kk * n), e = t - b * kk * n;
    const int64_t r = e / n, i = e - r * n;
    const int64_t j = by_rank[b * n + r];
    const double v = nrm[b * n + j];
    const double inv = v > 0 ? 1.0 / v : 0.0;
    U[b * n * kmax + r * n + i] = A[b * stride + j * n + i] * inv;
    Vk[b * n * kmax + r * n + i] = V[b * stride + j * n + i];
  }
}

int64_t jacobi_finish_work_doubles(int64_t n, int batch) { return 2 * n * batch; }

hipError_t launch_jacobi_finish(const double* A, const double* V, int64_t n, int64_t stride, int batch, int64_t kmax,
                                double* sv, double* U, double* Vk, double* work, hipStream_t s) {
  if (n > 4096) return hipErrorInvalidValue;
  if (batch <= 0 || n <= 0) return hipSuccess;
  double* nrm = work;
  int* by_rank = (int*)(work + n * batch);
  col_norms_kernel<<<dim3((unsigned)((n + 3) / 4), (unsigned)batch), 256, 0, s>>>(A, n, stride, nrm);
  rank_kernel<<<batch, 1024, n * sizeof(double), s>>>(nrm, n, sv, by_rank);
  const int64_t kk = kmax < n ? kmax : n;
  if (kk > 0) gather_kernel<<<grid_for(kk * n * batch), 256, 0, s>>>(A, V, n, stride, kk, kmax, nrm, by_rank, batch, U, Vk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kernels of the reverse pass.

// Adjoint of y = x / |x| (in place on the adjoint): xbar = (ybar - y <y, ybar>) / |x|.
template <typename T>
__global__ __launch_bounds__(256) void normalize_backward_kernel(NormList Y, NormList Yb) {
  int t = blockIdx.x;
  const T* y = (const T*)Y.ptr[t];
  T* yb = (T*)Yb.ptr[t];
  int64_t n = Y.n[t];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)y[i] * (double)yb[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  // norm_out holds the signed norm sign * |x| of the forward pass
  double dot = red[0], nrm = Y.norm_out[t];
  double inv = nrm != 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) yb[i] = (T)(((double)yb[i] - (double)y[i] * dot) * inv);
}

hipError_t launch_normalize_backward(int type, const NormList& Y, const NormList& Yb, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (type == 0) normalize_backward_kernel<double><<<count, 256, 0, s>>>(Y, Yb);
  else normalize_backward_kernel<float><<<count, 256, 0, s>>>(Y, Yb);
  return hipGetLastError();
}

// Adjoint of the energy with respect to the plaquette density matrices:
// with e_t = Tr(h_t rho)/Tr rho, d e_t / d rho[x][y] = (h_t[y][x] - e_t delta_xy) / Tr rho,
// where h_t is the bond operator on sites (a, b) times the identity on the other two.
__global__ void energy_backward_kernel(const double* rho, int64_t rho_stride, const double* h, const EnergyTerm* terms,
                                       int n_terms, int d, double inv_sites, const double* bond, int n_rho,
                                       double* rho_bar) {
  const int D4 = d * d * d * d;
  const int64_t total = (int64_t)n_rho * D4 * D4;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int p = (int)(e / ((int64_t)D4 * D4));
    int ik = (int)((e / D4) % D4), ib = (int)(e % D4);
    const double* r = rho + p * rho_stride;
    double tr = 0.0;
    for (int i = 0; i < D4; ++i) tr += r[(int64_t)i * D4 + i];
    int ko[4], bo[4], dd[4] = {d * d * d, d * d, d, 1};
    for (int q = 0; q < 4; ++q) { ko[q] = (ik / dd[q]) % d; bo[q] = (ib / dd[q]) % d; }
    double g = 0.0;
    for (int t = 0; t < n_terms; ++t) {
      const EnergyTerm tm = terms[t];
      if (tm.rho_index != p) continue;
      bool spect = true;
      for (int q = 0; q < 4; ++q)
        if (q != tm.a && q != tm.b && ko[q] != bo[q]) spect = false;
      double hv = spect ? h[(bo[tm.a] * d + bo[tm.b]) * d * d + ko[tm.a] * d + ko[tm.b]] : 0.0;
      double diag = ik == ib ? bond[t] : 0.0;
      g += tm.coef * (hv - diag) / tr;
    }
    rho_bar[e] += g * inv_sites;
  }
}

hipError_t launch_energy_backward(const double* rho, int64_t rho_stride, const double* h, const EnergyTerm* terms,
                                  int n_terms, int d, double inv_sites, const double* bond, int n_rho, double* rho_bar,
                                  hipStream_t s) {
  int64_t total = (int64_t)n_rho * d * d * d * d * d * d * d * d;
  energy_backward_kernel<<<grid_for(total), 256, 0, s>>>(rho, rho_stride, h, terms, n_terms, d, inv_sites, bond, n_rho,
                                                          rho_bar);
  return hipGetLastError();
}

// out[i][k] (row-major rows x cols) = in[i*s_row + k*s_col] * w[k]; w may be null (factor 1).
__global__ void colscale_copy_kernel(const double* in, int64_t s_row, int64_t s_col, int64_t rows, int64_t cols,
                                     const double* w, double* out) {
  int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / cols, k = e - i * cols;
    double v = in[i * s_row + k * s_col];
    out[e] = w ? v * w[k] : v;
  }
}

hipError_t launch_colscale_copy(const double* in, int64_t s_row, int64_t s_col, int64_t rows, int64_t cols,
                                const double* w, double* out, hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  colscale_copy_kernel<<<grid_for(rows * cols), 256, 0, s>>>(in, s_row, s_col, rows, cols, w, out);
  return hipGetLastError();
}

// sbar[k] = -1/2 w_k^3 (sum_j Vr[j][k] Xb[j][k] + sum_i Ur[i][k] Yb[i][k]) for k < chi, 0 for chi <= k < r.
// Ur, Vr: column-major (rows x r, leading dimension rows); Xb, Yb: row-major rows x chi.
__global__ __launch_bounds__(256) void svd_sbar_kernel(const double* Ur, const double* Vr, const double* Xb,
                                                       const double* Yb, int64_t rows, int64_t r, int64_t chi,
                                                       const double* w, double* sbar) {
  int64_t k = blockIdx.x;
  double acc = 0.0;
  if (k < chi)
    for (int64_t i = threadIdx.x; i < rows; i += 256)
      acc += Vr[i + k * rows] * Xb[i * chi + k] + Ur[i + k * rows] * Yb[i * chi + k];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) sbar[k] = k < chi ? -0.5 * red[0] * w[k] * w[k] * w[k] : 0.0;
}

hipError_t launch_svd_sbar(const double* Ur, const double* Vr, const double* Xb, const double* Yb, int64_t rows,
                           int64_t r, int64_t chi, const double* w, double* sbar, hipStream_t s) {
  svd_sbar_kernel<<<(unsigned)r, 256, 0, s>>>(Ur, Vr, Xb, Yb, rows, r, chi, w, sbar);
  return hipGetLastError();
}

// Core of the SVD adjoint (row-major r x r):
//   core = (F o (G - G^T)) diag(s) + diag(sbar) + diag(s) (F o (H - H^T)),
// G = U^T Ubar and H = V^T Vbar given as r x chi (columns >= chi are zero),
// F_qp = D / (D^2 + (eta m)^2), D = s_p^2 - s_q^2, m = max(s_q^2, s_p^2), F_qq = 0.
__global__ void svd_core_kernel(const double* G, const double* H, const double* s, const double* sbar, int64_t r,
                                int64_t chi, double eta, double* core) {
  int64_t total = r * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t q = e / r, p = e - q * r;
    double v;
    if (q == p) {
      v = sbar[q];
    } else {
      double sq = s[q] * s[q], sp = s[p] * s[p];
      double Dl = sp - sq, m = fmax(sq, sp) * eta;
      double den = Dl * Dl + m * m;
      double F = den > 0.0 ? Dl / den : 0.0;
      double gqp = p < chi ? G[q * chi + p] : 0.0, gpq = q < chi ? G[p * chi + q] : 0.0;
      double hqp = p < chi ? H[q * chi + p] : 0.0, hpq = q < chi ? H[p * chi + q] : 0.0;
      v = F * (gqp - gpq) * s[p] + s[q] * F * (hqp - hpq);
    }
    core[e] = v;
  }
}

hipError_t launch_svd_core(const double* G, const double* H, const double* s, const double* sbar, int64_t r,
                           int64_t chi, double eta, double* core, hipStream_t st) {
  svd_core_kernel<<<grid_for(r * r), 256, 0, st>>>(G, H, s, sbar, r, chi, eta, core);
  return hipGetLastError();
}

// out[i][k] = (A[i][k] - B[i][k]) * sinv_k (row-major rows x chi), sinv_k = 1/s_k where w_k != 0, else 0.
__global__ void sub_sinv_kernel(const double* A, const double* B, int64_t rows, int64_t chi, const double* s,
                                const double* w, double* out) {
  int64_t total = rows * chi;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = e % chi;
    double si = w[k] != 0.0 ? 1.0 / s[k] : 0.0;
    out[e] = (A[e] - B[e]) * si;
  }
}

hipError_t launch_sub_sinv(const double* A, const double* B, int64_t rows, int64_t chi, const double* s,
                           const double* w, double* out, hipStream_t st) {
  if (rows * chi <= 0) return hipSuccess;
  sub_sinv_kernel<<<grid_for(rows * chi), 256, 0, st>>>(A, B, rows, chi, s, w, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi: one round of the round-robin tournament over blocks
// of BW columns.  One workgroup per block pair (C = 2 BW columns of the n x n
// column-major matrix A_b):
//  * the Gram matrix G = X^T X of the pair's columns X (n x C) on the FP64
//    matrix cores: X^T X is a product whose two operands are the same
//    registers (a lane holds X[k][m] for the A operand and X[k][n] for the B
//    operand, with k the row of X), each wave summing a range of rows, the
//    wave partials reduced through LDS in wave order;
//  * the first wave runs cyclic two-sided Jacobi sweeps on G (at most
//    ``inner`` sweeps, each pair rotated when |g_pq| > tol sqrt(g_pp g_qq) and
//    both columns are above the negligible size tiny2), accumulating the
//    rotations in R; meanwhile the other waves have their 16-row tiles of the
//    pair's columns of A and V in flight;
//  * if any rotation was applied, X <- X R and V_pair <- V_pair R, a 16 x C
//    tile times the C x C matrix R per MFMA chain.
// The number of rotations is added to rot[b], and the largest |x_p.x_q| /
// (|x_p||x_q|) of a rotated pair is folded into ovl_max[b] (a float64 stored
// by atomic maximum on its bit pattern).  The pair threshold is the one
// of the scalar method, evaluated on dot products of the current columns, so
// a round with no rotation anywhere certifies the same orthogonality.
constexpr int BJ_BW = 8;            // columns per block
constexpr int BJ_C = 2 * BJ_BW;     // columns per pair (the MFMA tile width)
constexpr int BJ_NT = 1024;         // threads per workgroup (one workgroup per CU: latency, not occupancy)
constexpr int BJ_NW = BJ_NT / 64;   // waves
constexpr int BJ_GK = 8;            // Gram k-steps (4 rows each) in flight per wave
constexpr int BJ_TPW = 4;           // tiles per wave held in registers across the inner Jacobi
static_assert(BJ_C == 16, "the pair is one 16-wide MFMA tile");

// LDS traffic between the lanes of one wave: order the accesses without a
// workgroup barrier (the other waves are not taking part).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int BJ_GS = BJ_C + 1;   // padded row stride of G and R (column accesses spread over banks)
constexpr int BJ_SR = 4 * BJ_GK;   // rows of a wave's Gram block (GK k-steps of 4)
struct BjacShared {
  double part[BJ_NW][BJ_C * BJ_C];   // per-wave Gram partials
  double G[BJ_C * BJ_GS];
  double R[BJ_C * BJ_GS];
  double stage[BJ_NW][BJ_SR * BJ_GS];   // per-wave Gram block, [row][column], padded rows
  int nrot;
};

// Column element loads and stores of a round.  COH: at device scope (each
// access coherent across the L2s of the device), for rounds that other
// workgroups of the same launch read after a grid barrier.
template <bool COH>
__device__ __forceinline__ double col_load(const double* p) {
  if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool COH>
__device__ __forceinline__ void col_store(double* p, double v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// Blocks P < Q of pair k in round `round` of the tournament over np players
// (the round-robin circle: player np - 1 fixed, the others turned by one).
__device__ __forceinline__ void bjac_pair(int k, int round, int64_t np, int64_t& P, int64_t& Q) {
  if (k == 0) { P = round; Q = np - 1; }
  else { P = (round + k) % (np - 1); Q = (round - k + (np - 1)) % (np - 1); }
  if (P > Q) { const int64_t t = P; P = Q; Q = t; }
}

// 1 / sqrt(x) for normal x > 0: the hardware estimate and two Newton steps
// y <- y (3 - x y^2) / 2, which converge quadratically to a few ulp.
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// One round for the block pair blockIdx.x of matrix blockIdx.y.  Every thread
// of the workgroup calls it and leaves it together or after its last barrier.
template <bool COH>
__device__ __forceinline__ void bjac_round(BjacShared& sh, double* A, double* V, int64_t n, int64_t nblk, int64_t np,
                                           int64_t stride, int round, double tol, const double* tiny2, int inner,
                                           int* rot, unsigned long long* ovl_max) {
  constexpr int GS = BJ_GS;
  auto& part = sh.part;
  double* G = sh.G;
  double* R = sh.R;
  int& nrot_s = sh.nrot;
  const int k = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  int64_t P, Q;
  bjac_pair(k, round, np, P, Q);
  // a block paired with the padding player (odd block count, or a single
  // block) is still rotated within itself: the missing columns read as absent
  if (P >= nblk && Q >= nblk) return;
  double* Ab = A + (int64_t)b * stride;
  double* Vb = V + (int64_t)b * stride;
  // global column of local column c, or -1 past the end of the matrix
  const int64_t c0P = P * BJ_BW, c0Q = Q * BJ_BW;
  auto gcol = [&](int c) -> int64_t {
    const int64_t g = c < BJ_BW ? c0P + c : c0Q + (c - BJ_BW);
    return g < n ? g : -1;
  };
  const int wave = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;

  // ---- Gram matrix: wave w takes the k-steps [w GK, (w + 1) GK) + j NW GK;
  // lane (lr, lq) holds X[4 k + lq][lr].  The block of 4 GK rows x C columns
  // is loaded with 32 lanes per column (consecutive rows, so that a load
  // instruction reads two 256-byte column segments instead of C 32-byte
  // pieces) into the wave's LDS stage, and read back in the operand layout.
  {
    d4_t gacc = {0.0, 0.0, 0.0, 0.0};
    const int64_t nks = (n + 3) / 4;
    double* stg = sh.stage[wave];
    const int sr = lane & 31, sc = lane >> 5;
    static_assert(BJ_SR == 32 && BJ_C % 2 == 0, "two columns of 32 rows per load instruction");
    for (int64_t kb = (int64_t)wave * BJ_GK; kb < nks; kb += (int64_t)BJ_GK * BJ_NW) {
      double y[BJ_C / 2];
#pragma unroll
      for (int i = 0; i < BJ_C / 2; ++i) {
        const int64_t g = gcol(2 * i + sc), row = kb * 4 + sr;
        y[i] = (g >= 0 && row < n) ? col_load<COH>(Ab + g * n + row) : 0.0;
      }
#pragma unroll
      for (int i = 0; i < BJ_C / 2; ++i) stg[sr * BJ_GS + 2 * i + sc] = y[i];
      wave_sync();
      double x[BJ_GK];
#pragma unroll
      for (int u = 0; u < BJ_GK; ++u) x[u] = stg[(4 * u + lq) * BJ_GS + lr];
      wave_sync();   // the reads are done before the next block's writes
#pragma unroll
      for (int u = 0; u < BJ_GK; ++u) gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], x[u], gacc, 0, 0, 0);
    }
    // D layout of v_mfma_f64_16x16x4f64: register e of lane l holds row l/16 + 4 e, column l % 16
#pragma unroll
    for (int e = 0; e < 4; ++e) part[wave][(lq + 4 * e) * BJ_C + lr] = gacc[e];
  }

  // ---- tiles of the rotation: task t < 2 * tiles is the 16-row tile
  // t mod tiles of A (t < tiles) or of V; lane (lr, lq) holds rows i0 + lr of
  // the columns 4 ks + lq.  The waves after the first take tasks
  // wave - 1 + (NW - 1) u and load the first TPW of them while the first wave
  // runs the inner Jacobi.
  const int64_t tiles = (n + 15) / 16, ntask = 2 * tiles;
  int64_t gA[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) gA[ks] = gcol(4 * ks + lq);
  auto load_tile = [&](int64_t t, double* x) {
    const bool isA = t < tiles;
    const double* M = isA ? Ab : Vb;
    const int64_t row = (isA ? t : t - tiles) * 16 + lr;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      x[ks] = (t < ntask && gA[ks] >= 0 && row < n) ? col_load<COH>(M + gA[ks] * n + row) : 0.0;
  };
  constexpr int AW = BJ_NW - 1;   // waves applying the rotation
  double pf[BJ_TPW][4];

  for (int el = tid; el < BJ_C * BJ_C; el += BJ_NT) R[(el / BJ_C) * GS + el % BJ_C] = (el / BJ_C == el % BJ_C) ? 1.0 : 0.0;
  __syncthreads();
  if (tid < BJ_C * BJ_C) {
    // the upper triangle's sums serve both halves, so G is exactly symmetric
    const int m = tid / BJ_C, c = tid % BJ_C;
    if (m <= c) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < BJ_NW; ++w) s += part[w][m * BJ_C + c];
      G[m * GS + c] = s;
      G[c * GS + m] = s;
    }
  }
  __syncthreads();
  if (wave > 0) {
#pragma unroll
    for (int u = 0; u < BJ_TPW; ++u) load_tile(wave - 1 + (int64_t)AW * u, pf[u]);
  }
  // inner Jacobi on G (first wave): a round of the C-player tournament rotates
  // C/2 disjoint pairs; lane (j, k) = (lane / 8, lane % 8) owns the 2 x 2
  // blocks of G and R in the rows of pair j and the columns of pair k, so the
  // round's update G <- J^T G J, R <- R J is local to the lane once it has the
  // rotations of pairs j and k, which lane (j, j) computes from its block
  if (tid < 64) {
    const double t2 = tiny2[b], tol2 = tol * tol;
    const int pj = lane >> 3, pk = lane & 7;
    unsigned present = 0;   // bit c: local column c lies inside the matrix
#pragma unroll
    for (int cc = 0; cc < BJ_C; ++cc) present |= (gcol(cc) >= 0 ? 1u : 0u) << cc;
    int nrot = 0;
    double ovl = 0.0;   // largest |cos| between two columns this lane rotated
    for (int sw = 0; sw < inner; ++sw) {
      int sweep_rot = 0;
#pragma unroll 1
      for (int rd = 0; rd < BJ_C - 1; ++rd) {
        auto players = [&](int x, int& p, int& q) {
          if (x == 0) { p = rd; q = BJ_C - 1; }
          else { p = (rd + x) % (BJ_C - 1); q = (rd - x + (BJ_C - 1)) % (BJ_C - 1); }
          if (p > q) { int t = p; p = q; q = t; }
        };
        int p, q, p2, q2;
        players(pj, p, q);
        players(pk, p2, q2);
        const double g00 = G[p * GS + p2], g01 = G[p * GS + q2], g10 = G[q * GS + p2], g11 = G[q * GS + q2];
        const double r00 = R[p * GS + p2], r01 = R[p * GS + q2], r10 = R[q * GS + p2], r11 = R[q * GS + q2];
        double c = 1.0, sn = 0.0;
        // the pair test |g01| > tol sqrt(g00 g11) in squares (g00, g11 > t2 keep the product
        // normal), all conditions evaluated without short circuit: one branch
        const bool rotate = (pj == pk) & (((present >> p) & (present >> q) & 1u) != 0u) & (fmin(g00, g11) > t2) &
                            (g01 != 0.0) & (g01 * g01 > tol2 * (g00 * g11));
        if (rotate) {
          // |cos| of the pair, for the stop test only: the hardware reciprocal square root suffices
          ovl = fmax(ovl, fabs(g01) * __builtin_amdgcn_rsq(g00 * g11));
          // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with zeta = d / (2 g01), d = g11 - g00,
          // written with den = |d| + sqrt(d^2 + 4 g01^2): t = +-2 g01 / den, and
          // c = 1 / sqrt(1 + t^2) = den / sqrt(den^2 + 4 g01^2), s = c t (two reciprocal square
          // roots; the squares stay finite for Gram entries below 1e150, far above those of the
          // normalised half systems)
          const double d = g11 - g00, e = 2.0 * g01;
          const double x1 = fma(d, d, e * e);
          const double den = fabs(d) + x1 * rsqrt_refined(x1);
          const double rn = rsqrt_refined(fma(den, den, e * e));
          c = den * rn;
          sn = (d >= 0.0 ? e : -e) * rn;
        }
        const unsigned long long live = __ballot(sn != 0.0);
        if (live) {
          sweep_rot += __popcll(live);
          const double cj = __shfl(c, pj * 9), sj = __shfl(sn, pj * 9);
          const double ck = __shfl(c, pk * 9), sk = __shfl(sn, pk * 9);
          // rows p, q by pair j, then columns p2, q2 by pair k
          const double a00 = cj * g00 - sj * g10, a01 = cj * g01 - sj * g11;
          const double a10 = sj * g00 + cj * g10, a11 = sj * g01 + cj * g11;
          G[p * GS + p2] = ck * a00 - sk * a01;
          G[p * GS + q2] = sk * a00 + ck * a01;
          G[q * GS + p2] = ck * a10 - sk * a11;
          G[q * GS + q2] = sk * a10 + ck * a11;
          R[p * GS + p2] = ck * r00 - sk * r01;
          R[p * GS + q2] = sk * r00 + ck * r01;
          R[q * GS + p2] = ck * r10 - sk * r11;
          R[q * GS + q2] = sk * r10 + ck * r11;
        }
        wave_sync();
      }
      nrot += sweep_rot;
      if (sweep_rot == 0) break;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ovl = fmax(ovl, __shfl_xor(ovl, o, 64));
    if (lane == 0) {
      nrot_s = nrot;
      if (nrot) atomicAdd(rot + b, nrot);
      // non-negative doubles order as their bit patterns
      if (ovl > 0.0) atomicMax(ovl_max + b, (unsigned long long)__double_as_longlong(ovl));
    }
  }
  __syncthreads();
  if (nrot_s == 0 || wave == 0) return;

  // ---- X <- X R, V_pair <- V_pair R, formed transposed, (X R)^T = R^T X^T,
  // so that a store instruction writes whole 16-row column segments: the A
  // operand is R^T (lane (lr, lq) holds R[4 ks + lq][lr]), the B operand X^T
  // is the tile as loaded, and register e of lane (lr, lq) is row i0 + lr of
  // column lq + 4 e
  double rb[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) rb[ks] = R[(4 * ks + lq) * GS + lr];
  int64_t gD[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) gD[e] = gcol(lq + 4 * e);
  auto store_tile = [&](int64_t t, const double* x) {
    if (t >= ntask) return;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(rb[ks], x[ks], acc, 0, 0, 0);
    const bool isA = t < tiles;
    double* M = isA ? Ab : Vb;
    const int64_t row = (isA ? t : t - tiles) * 16 + lr;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (gD[e] >= 0 && row < n) col_store<COH>(M + gD[e] * n + row, acc[e]);
  };
#pragma unroll
  for (int u = 0; u < BJ_TPW; ++u) store_tile(wave - 1 + (int64_t)AW * u, pf[u]);
  for (int64_t t = wave - 1 + (int64_t)AW * BJ_TPW; t < ntask; t += AW) {
    double x[4];
    load_tile(t, x);
    store_tile(t, x);
  }
}

__global__ __launch_bounds__(BJ_NT) void bjac_round_kernel(double* A, double* V, int64_t n, int64_t nblk, int64_t np,
                                                           int64_t stride, int round, double tol, const double* tiny2,
                                                           int inner, int* rot, unsigned long long* ovl_max) {
  __shared__ BjacShared sh;
  bjac_round<false>(sh, A, V, n, nblk, np, stride, round, tol, tiny2, inner, rot, ovl_max);
}

// Ordering of the rounds inside one launch.  Round t + 1 of a pair needs
// only its two blocks as round t left them, each rotated by one other
// workgroup of the same matrix, so the workgroups synchronise per block, not
// per round: ver[(b * np + B) * BJ_VS] counts the rounds finished on block B of matrix b
// (across sweeps: round t of sweep s is number s * rounds + t).  A workgroup
// publishes a round by waiting until every wave's stores are acknowledged and
// then raising the counters of its two blocks; it starts round number g once
// both of its blocks have count g.  The exchanged column data is
// loaded and stored at device scope (col_load / col_store<true>), so no cache
// write-back or invalidation is needed.  All workgroups must be resident
// (round 0 waits for nothing, and by induction every round's producers
// finish).  The wait is bounded: a workgroup that polls more than BAR_SPINS
// times sets *abort and every workgroup then leaves the kernel.
constexpr unsigned BAR_SPINS = 1u << 21;
// The block counters sit BJ_VS words apart (one 128-byte line each), so that
// the workgroups polling and raising them do not contend for shared lines.
constexpr int64_t BJ_VS = 32;

__device__ __forceinline__ void publish_blocks(unsigned* ver, int64_t P, int64_t Q, int64_t nblk, unsigned done) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    // the workgroup's column stores (ordered before this point by the
    // barrier) happen before the counters' new values at agent scope
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (P < nblk) __hip_atomic_store(ver + P * BJ_VS, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (Q < nblk) __hip_atomic_store(ver + Q * BJ_VS, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ bool wait_blocks(const unsigned* ver, int64_t P, int64_t Q, int64_t nblk, unsigned need,
                                            unsigned* abort, int& ok_s) {
  if (threadIdx.x == 0) {
    int ok = 1;
    unsigned spins = 0;
    for (;;) {
      const bool p_ready = P >= nblk || __hip_atomic_load(ver + P * BJ_VS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
      const bool q_ready = Q >= nblk || __hip_atomic_load(ver + Q * BJ_VS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
      if (p_ready && q_ready) break;
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) { ok = 0; break; }
      if (++spins > BAR_SPINS) {
        __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // pairs with the release of the workgroups that published the blocks
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

// Barrier over all workgroups of the grid at the end of a sweep: *count
// collects arrivals (one counter per sweep, zero at launch).  Bounded like
// wait_blocks.
__device__ __forceinline__ bool sweep_barrier(unsigned* count, unsigned target, unsigned* abort, int& ok_s) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) { ok = 0; break; }
      if (++spins > BAR_SPINS) {
        __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

// The whole Jacobi iteration in one launch: sweeps of `rounds` rounds (the
// round of bjac_round_kernel, ordered per block as above), and after each
// sweep the stop rule on the totals of the whole batch: stop once no pair was
// rotated or the largest rotated |cos| is at most `stop`, the same decision,
// from the same sums, as a host loop over per-round launches.  rot and ovl
// hold one slot per sweep ([sweep][batch]).  sync[0] is the abort flag,
// sync[BJ_VS + (b * np + B) * BJ_VS] the round counters of the blocks
// (counting across sweeps), then one arrival counter per sweep; everything
// zero at launch.
// *sweeps receives the number of sweeps run.  No convergence within
// max_sweeps, or a wait that ran out, adds one to *fail.  Every workgroup
// must be resident at once: the host launches it cooperatively (the runtime
// refuses a grid the device cannot hold) or, with cooperative launches
// switched off, only when the occupancy of the device holds the whole grid.
__global__ __launch_bounds__(BJ_NT) void bjac_svd_kernel(double* A, double* V, int64_t n, int64_t nblk, int64_t np,
                                                         int64_t stride, int rounds, int max_sweeps, double tol,
                                                         double stop, const double* tiny2, int* rot,
                                                         unsigned long long* ovl, unsigned* sync, int* fail,
                                                         int* sweeps) {
  __shared__ BjacShared sh;
  __shared__ int ok_s, go_s;
  const int batch = (int)gridDim.y;
  const unsigned wgs = gridDim.x * gridDim.y;
  unsigned* ver = sync + BJ_VS + (int64_t)blockIdx.y * np * BJ_VS;
  unsigned* arrive = sync + BJ_VS + (int64_t)batch * np * BJ_VS;
  const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int* rot_s = rot + (int64_t)sw * batch;
    unsigned long long* ovl_s = ovl + (int64_t)sw * batch;
    for (int t = 0; t < rounds; ++t) {
      int64_t P, Q;
      bjac_pair(blockIdx.x, t, np, P, Q);
      const unsigned g = (unsigned)sw * (unsigned)rounds + (unsigned)t;
      if (g > 0 && !wait_blocks(ver, P, Q, nblk, g, sync, ok_s)) {
        if (threadIdx.x == 0) atomicAdd(fail, 1);
        return;
      }
      bjac_round<true>(sh, A, V, n, nblk, np, stride, t, tol, tiny2, 1, rot_s, ovl_s);
      publish_blocks(ver, P, Q, nblk, g + 1);
    }
    if (!sweep_barrier(arrive + sw, wgs, sync, ok_s)) {
      if (threadIdx.x == 0) atomicAdd(fail, 1);
      return;
    }
    if (threadIdx.x == 0) {
      bool any = false;
      unsigned long long big = 0;   // non-negative doubles order as their bit patterns
      for (int b = 0; b < batch; ++b) {
        any |= __hip_atomic_load(rot_s + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        const unsigned long long o = __hip_atomic_load(ovl_s + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        big = o > big ? o : big;
      }
      go_s = any && __longlong_as_double((long long)big) > stop;
    }
    __syncthreads();
    if (!go_s) {
      if (lead) *sweeps = sw + 1;
      return;
    }
  }
  if (lead) {
    *sweeps = max_sweeps;
    atomicAdd(fail, 1);
  }
}

hipError_t launch_bjac_round(double* A, double* V, int64_t n, int64_t stride, int batch, int round, double tol,
                             const double* tiny2, int inner, int* rot, double* ovl_max, hipStream_t s) {
  const int64_t nblk = (n + BJ_BW - 1) / BJ_BW;
  const int64_t np = nblk + (nblk & 1);
  dim3 grid((unsigned)(np / 2), (unsigned)batch);
  bjac_round_kernel<<<grid, BJ_NT, 0, s>>>(A, V, n, nblk, np, stride, round, tol, tiny2, inner, rot,
                                           (unsigned long long*)ovl_max);
  return hipGetLastError();
}

// Workgroups of bjac_svd_kernel the device holds at once (0 if unknown).
int64_t bjac_sweep_capacity() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bjac_svd_kernel, BJ_NT, 0) != hipSuccess) return 0;
  return (int64_t)cus * per_cu;
}

int64_t bjac_grid(int64_t n, int batch) {
  const int64_t nblk = (n + BJ_BW - 1) / BJ_BW;
  return (nblk + (nblk & 1)) / 2 * batch;
}

int64_t bjac_sync_words(int64_t n, int batch, int max_sweeps) {
  const int64_t nblk = (n + BJ_BW - 1) / BJ_BW;
  return BJ_VS + (nblk + (nblk & 1)) * batch * BJ_VS + max_sweeps;
}

hipError_t launch_bjac_svd(double* A, double* V, int64_t n, int64_t stride, int batch, int max_sweeps, double tol,
                           double stop, const double* tiny2, int* rot, double* ovl, unsigned* sync, int* fail,
                           int* sweeps, bool cooperative, hipStream_t s) {
  const int64_t nblk = (n + BJ_BW - 1) / BJ_BW;
  const int64_t np = nblk + (nblk & 1);
  dim3 grid((unsigned)(np / 2), (unsigned)batch);
  int rounds = (int)(np - 1);
  unsigned long long* ovl_u = (unsigned long long*)ovl;
  if (cooperative) {
    void* args[] = {&A, &V, &n, (void*)&nblk, (void*)&np, &stride, &rounds, &max_sweeps, &tol, &stop, &tiny2,
                    &rot, &ovl_u, &sync, &fail, &sweeps};
    return hipLaunchCooperativeKernel((const void*)bjac_svd_kernel, grid, dim3(BJ_NT), args, 0, s);
  }
  bjac_svd_kernel<<<grid, BJ_NT, 0, s>>>(A, V, n, nblk, np, stride, rounds, max_sweeps, tol, stop, tiny2, rot, ovl_u,
                                         sync, fail, sweeps);
  return hipGetLastError();
}

int bjac_pair_columns() { return BJ_C; }

int64_t bjac_rounds(int64_t n) {
  const int64_t nblk = (n + BJ_BW - 1) / BJ_BW;
  return nblk + (nblk & 1) - 1;
}

}  // namespace ctmk
