// Launch interface of the batched Householder QR kernels (qr_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrk {

// Panel width used for matrices of m rows (16, or 8 above 1024 rows).
int panel_width(int64_t m);

// Factorise the panel of columns j0 .. j0+nb-1 (nb = panel_width(m)) of every
// matrix; writes tau[b*tau_stride + j] and the nb x nb T of the block
// reflector (row-major) at T + b*T_stride.  If V is not NULL, also writes V
// and Y = V T as launch_build_vy does with trans set (Y too must be given).
hipError_t launch_panel(double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m, int64_t n, int64_t j0, int batch,
                        double* tau, int64_t tau_stride, double* T, int64_t T_stride, double* V, double* Y,
                        hipStream_t s);

// Dense V (L x nb) and Y = V T (trans) or V T^T of the panel at (j0, j0), L = m - j0,
// both row-major per matrix (stride L*nb), for C <- C - V (Y^T C).
hipError_t launch_build_vy(const double* A, int64_t rs, int64_t cs, int64_t stride, int64_t m, int64_t j0, int nbp,
                           int nb, const double* T, int64_t T_stride, bool trans, double* V, double* Y, int batch,
                           hipStream_t s);

// C_b[i][j] -= (V (Y^T C_b))[i][j] for i < L, j < ncols in one launch (element
// (i, j) at C + b*cstride + i*crs + j*ccs; V, Y row-major L x nb per matrix,
// stride L*nb; nb 16 or 8) with, element for element, the arithmetic of the
// two matrix-core products it replaces: Z = Y^T C split over K in
// ksplit chunks of kchunk rows (ksplit <= 1: no split) as the contraction
// planner splits it, then C <- (-(V Z)) + C.  ksplit at most
// panel_update_max_split(), kchunk a multiple of 4.
hipError_t launch_panel_update_mfma(double* C, int64_t crs, int64_t ccs, int64_t cstride, int64_t L, int64_t ncols,
                                    int nb, const double* V, const double* Y, int batch, int64_t kchunk, int ksplit,
                                    hipStream_t s);
int panel_update_max_split();

// Column-major n x k L_b = R_b^T (zero above the diagonal) of the factorised A_b.
hipError_t launch_extract_rt(const double* A, int64_t rs, int64_t cs, int64_t stride, int64_t n, int64_t k, double* L,
                             int64_t lstride, int batch, hipStream_t s);

}  // namespace qrk
