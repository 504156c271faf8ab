// Launch interface of the device kernels (kernels.hip).  Host code of the
// library only; not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctmk {

enum { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2 };

// Batched contraction C[b][m][n] = alpha * sum_k A[b][m][k] * B[b][k][n] (+ C if beta).
// Every index i of a group of total size X with inner size X_in sits at
// (i / X_in) * stride_outer + (i % X_in) * stride_inner in each operand.
// Element types: double (F64 mode) or float (F32 and BF16 modes).
struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  int64_t M, N, K, batch;
  int64_t m_in, n_in, k_in, b_in;
  int64_t a_m_o, a_m_i, a_k_o, a_k_i, a_b_o, a_b_i;
  int64_t b_k_o, b_k_i, b_n_o, b_n_i, b_b_o, b_b_i;
  int64_t c_m_o, c_m_i, c_n_o, c_n_i, c_b_o, c_b_i;
  double alpha;
  int beta;                 // 0: overwrite C, 1: accumulate into C
  const double* colscale;   // optional factor per n (device, length N)
  // split K: ksplit > 1 workgroups share one output tile, each summing a K
  // range of kchunk (a multiple of 32); their partial tiles go to ``work``
  // ([ksplit][batch][M][N], element type of C) and launch_contract adds them up.
  int64_t ksplit, kchunk;
  void* work;
};

constexpr int PERM_MAX_DIMS = 10;
struct PermArgs {
  int ndim;
  int accumulate;
  int64_t dims[PERM_MAX_DIMS];
  int64_t in_strides[PERM_MAX_DIMS];
  int64_t out_strides[PERM_MAX_DIMS];
};

constexpr int NORM_MAX = 64;
struct NormList {
  void* ptr[NORM_MAX];
  int64_t n[NORM_MAX];
  double* norm_out;         // optional, one value per tensor
  int* zero_flag;           // optional: incremented for every tensor whose norm is 0
};

// Rows of a column step checked for an empty cut (launch_cut_check).
constexpr int CUT_MAX = 64;
constexpr int CUT_CHUNKS = 64;   // workgroups per row for the factors' norms
struct CutList {
  const double* Ln[CUT_MAX];   // R_n^T of the row (any layout, n entries)
  const double* Ls[CUT_MAX];   // R_s^T of the row
  const double* s1[CUT_MAX];   // largest singular value of M
  int64_t n[CUT_MAX];
};

struct EnergyTerm {
  int rho_index;            // which plaquette density matrix
  int a, b;                 // sites 0..3 of the plaquette
  double coef;
};

// Large BF16 products of plain row-major operands take a dedicated kernel
// (gemm_bf16_rowmajor_kernel) unless this process-wide switch is off.
extern bool g_rowmajor_path;
// FP64 (FP32) products with A contiguous along k and B along n, M, N >= 512,
// on a dedicated 128 x 128-tile kernel (else the general one); process-wide.
extern bool g_rowmajor_f64;
extern bool g_rowmajor_f32;
hipError_t launch_contract(int mode, const GemmArgs& g, hipStream_t s);
hipError_t launch_permute(const PermArgs& p, int in_type, const void* in, int out_type, void* out, hipStream_t s);
hipError_t launch_fill(int type, void* p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill_int(int* p, int v, int64_t n, hipStream_t s);
// Workspace of launch_normalize: normalize_work_doubles(count) doubles.
constexpr int NORM_CHUNKS = 64;   // workgroups per tensor for its sums and its scaling
int64_t normalize_work_doubles(int count);
hipError_t launch_normalize(int type, const NormList& L, int count, double* work, hipStream_t s);
hipError_t launch_svd_weights(const double* s, int64_t r, int64_t stride_s, double* w, int64_t chi, double cutoff,
                              int batch, hipStream_t st);
// Rows of a column step whose projector signs are fixed (launch_proj_signs).
struct SignList {
  double* P[CUT_MAX];   // kd x chi row-major
  double* Q[CUT_MAX];
  double* U[CUT_MAX];   // column-major, r rows, at least chi columns
  double* V[CUT_MAX];
  int64_t kd[CUT_MAX];
};
// Negates column k < chi of P, Q, U, V of a row when the first entry of
// P[:, k] within a relative 1e-9 of the column's largest magnitude is negative.
hipError_t launch_proj_signs(const SignList& L, int count, int64_t chi, int64_t r, hipStream_t s);
// Adds one to *flag for every row whose s_1 <= tau |N|_F |S|_F.
// Divides each of the count dim x dim row-major matrices at rho (contiguous) by its trace.
hipError_t launch_rdm_normalize(double* rho, int count, int64_t dim, hipStream_t s);
// work: count * CUT_CHUNKS * 2 doubles of device scratch (partial sums of squares).
hipError_t launch_cut_check(const CutList& L, int count, double tau, double* work, int* flag, hipStream_t s);
hipError_t launch_extract_lower(const double* a, int64_t rows, int64_t lda, int64_t stride_a, double* l, int64_t rcols,
                                int64_t stride_l, int batch, hipStream_t s);
hipError_t launch_observables(const double* rho, int64_t rho_stride, int n, double* out, hipStream_t s);
hipError_t launch_energy(const double* rho, int64_t rho_stride, const double* h, const EnergyTerm* terms, int n_terms,
                         int d, double inv_sites, double* E_out, double* bond_out, hipStream_t s);
hipError_t launch_nonfinite(int type, const void* x, int64_t n, int* flag, hipStream_t s);
hipError_t launch_spectra_delta(const double* sv, int64_t r, int64_t chi, double* cur, const double* prev, int count,
                                double* delta_out, hipStream_t s);

hipError_t launch_flag_or(const int* src, int n, int* flag, hipStream_t s);
// *out (device double) = max_i |a_i - b_i| (b == nullptr: max_i |a_i|), a and b of type T_F64 (0) or T_F32.
hipError_t launch_max_abs(int type, const void* a, const void* b, int64_t n, double* out, hipStream_t s);

hipError_t launch_jacobi_round(double* A, double* V, int64_t n, int64_t stride, int batch, int round, double tol,
                               const double* tiny2, int* rot, hipStream_t s);
// work: frob_tiny_work_doubles(batch) doubles
int64_t frob_tiny_work_doubles(int batch);
hipError_t launch_frob_tiny(const double* A, int64_t len, int64_t stride, int batch, double eps, double* tiny2,
                            double* work, hipStream_t s);
hipError_t launch_identity(double* V, int64_t n, int64_t stride, int batch, hipStream_t s);
hipError_t launch_rt_from_qr(const double* A, double* X, int64_t n, int64_t stride, int batch, hipStream_t s);
// work: jacobi_finish_work_doubles(n, batch) doubles
int64_t jacobi_finish_work_doubles(int64_t n, int batch);
hipError_t launch_jacobi_finish(const double* A, const double* V, int64_t n, int64_t stride, int batch, int64_t kmax,
                                double* sv, double* U, double* Vk, double* work, hipStream_t s);

hipError_t launch_bjac_round(double* A, double* V, int64_t n, int64_t stride, int batch, int round, double tol,
                             const double* tiny2, int inner, int* rot, double* ovl_max, hipStream_t s);
// The whole Jacobi iteration in one launch: sweeps of tournament rounds
// (workgroups ordered per block between rounds) and the host loop's stop rule
// (no rotation, or largest rotated |cos| <= stop, over the batch) taken on the
// device after each sweep.  rot: max_sweeps * batch ints, ovl: max_sweeps *
// batch doubles, sync: bjac_sync_words(n, batch, max_sweeps) unsigned ints, all
// zero before the launch.  *sweeps (device) receives the sweeps run; no
// convergence, or a wait that ran out, adds one to *fail (device).  With
// ``cooperative`` the launch is a cooperative one, which the runtime refuses
// (an error return, nothing queued) when the device cannot hold the grid at
// once; otherwise only for grids of at most bjac_sweep_capacity() workgroups
// (bjac_grid(n, batch)).
hipError_t launch_bjac_svd(double* A, double* V, int64_t n, int64_t stride, int batch, int max_sweeps, double tol,
                           double stop, const double* tiny2, int* rot, double* ovl, unsigned* sync, int* fail,
                           int* sweeps, bool cooperative, hipStream_t s);
int64_t bjac_sync_words(int64_t n, int batch, int max_sweeps);
int64_t bjac_sweep_capacity();
int64_t bjac_grid(int64_t n, int batch);
int64_t bjac_rounds(int64_t n);
int bjac_pair_columns();

// reverse pass
hipError_t launch_normalize_backward(int type, const NormList& Y, const NormList& Yb, int count, hipStream_t s);
hipError_t launch_energy_backward(const double* rho, int64_t rho_stride, const double* h, const EnergyTerm* terms,
                                  int n_terms, int d, double inv_sites, const double* bond, int n_rho, double* rho_bar,
                                  hipStream_t s);
hipError_t launch_colscale_copy(const double* in, int64_t s_row, int64_t s_col, int64_t rows, int64_t cols,
                                const double* w, double* out, hipStream_t s);
hipError_t launch_svd_sbar(const double* Ur, const double* Vr, const double* Xb, const double* Yb, int64_t rows,
                           int64_t r, int64_t chi, const double* w, double* sbar, hipStream_t s);
hipError_t launch_svd_core(const double* G, const double* H, const double* s, const double* sbar, int64_t r,
                           int64_t chi, double eta, double* core, hipStream_t st);
hipError_t launch_sub_sinv(const double* A, const double* B, int64_t rows, int64_t chi, const double* s,
                           const double* w, double* out, hipStream_t st);

}  // namespace ctmk
