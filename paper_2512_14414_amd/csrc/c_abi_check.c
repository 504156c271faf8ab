/* The C ABI of include/ctm.h used from plain C, without Python or PyTorch.
 *
 * Builds the Neel product state on the 2x2 cell (D = 1, site tensors |up>
 * and |down> in a checkerboard), sweeps, and checks the energy per site of
 * the Heisenberg model against its closed form, -1/4 per bond, two bonds per
 * site: -1/2.  Also checks that an invalid chi is refused before any device
 * work with CTM_EINVAL and a message.  Device memory for the site tensors is
 * allocated with the HIP runtime, as any C caller would.  Exit status 0 on
 * success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "ctm.h"

#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      fprintf(stderr, __VA_ARGS__);       \
      fprintf(stderr, "\n");              \
      return 1;                           \
    }                                     \
  } while (0)

int main(void) {
  enum { d = 2, D = 1, chi = 2, Lx = 2, Ly = 2, nt = 2 };
  /* A_t[s][l][u][r][d] with D = 1: A_0 = |up>, A_1 = |down> */
  const double hA[nt * d] = {1.0, 0.0, 0.0, 1.0};
  const int pattern[Lx * Ly] = {0, 1, 1, 0};
  /* S_a . S_b as H[(s_a s_b), (s_a' s_b')] in the basis (up, down) */
  const double H[16] = {0.25, 0.0, 0.0, 0.0,
                        0.0, -0.25, 0.5, 0.0,
                        0.0, 0.5, -0.25, 0.0,
                        0.0, 0.0, 0.0, 0.25};
  /* every plaquette carries its four edges with weight 1/2 (each bond lies on two plaquettes) */
  ctm_term terms[16];
  int nterm = 0;
  for (int py = 0; py < Ly; ++py)
    for (int px = 0; px < Lx; ++px) {
      const int pairs[4][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}};
      for (int k = 0; k < 4; ++k) {
        ctm_term t = {px, py, pairs[k][0], pairs[k][1], 0.5};
        terms[nterm++] = t;
      }
    }

  ctm_ctx* bad = NULL;
  int rc = ctm_init(&bad, (const double*)8, d, 3, 4, Lx, Ly, pattern, nt, CTM_FP64, NULL);
  CHECK(rc == CTM_EINVAL && bad == NULL, "chi < D*d not refused (rc %d)", rc);
  CHECK(ctm_last_error(NULL)[0] != '\0', "no message for the refused init");

  double* dA = NULL;
  CHECK(hipMalloc((void**)&dA, sizeof hA) == hipSuccess, "hipMalloc failed");
  CHECK(hipMemcpy(dA, hA, sizeof hA, hipMemcpyHostToDevice) == hipSuccess, "hipMemcpy failed");
  ctm_ctx* ctx = NULL;
  rc = ctm_init(&ctx, dA, d, D, chi, Lx, Ly, pattern, nt, CTM_FP64, NULL);
  CHECK(rc == CTM_OK, "ctm_init: %d %s", rc, ctm_last_error(NULL));
  int sweeps = 0;
  double delta = 0.0, E = 0.0;
  rc = ctm_sweep(ctx, 4, 0.0, &sweeps, &delta);
  CHECK(rc == CTM_OK && sweeps == 4, "ctm_sweep: %d %s", rc, ctm_last_error(ctx));
  rc = ctm_energy(ctx, H, nterm, terms, &E);
  CHECK(rc == CTM_OK, "ctm_energy: %d %s", rc, ctm_last_error(ctx));
  CHECK(fabs(E + 0.5) < 1e-12, "Neel energy %.15f, expected -0.5", E);
  ctm_free(ctx);
  CHECK(hipFree(dA) == hipSuccess, "hipFree failed");
  printf("c_abi_check: Neel state, E = %.15f per site after %d sweeps\n", E, sweeps);
  return 0;
}
