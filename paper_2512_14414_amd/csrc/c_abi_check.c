/* The C ABI of include/ctm.h used from plain C, without Python or PyTorch.
 *
 * Builds the Neel product state on the 2x2 cell (D = 1, site tensors |up>
 * and |down> in a checkerboard), sweeps, and checks the energy per site of
 * the Heisenberg model against its closed form, -1/4 per bond, two bonds per
 * site: -1/2.  Also checks that an invalid chi is refused before any device
 * work with CTM_EINVAL and a message.  Device memory for the site tensors is
 * allocated with the HIP runtime, as any C caller would; a second context
 * takes its own device memory from the caller's allocator (ctm_set_allocator,
 * hipMalloc/hipFree with a count of the live blocks) and must hand every
 * block back by ctm_free.  Exit status 0 on success. */
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

/* caller allocator: hipMalloc / hipFree with a count of the live blocks */
static int g_live = 0, g_made = 0;
static void* my_alloc(size_t bytes, void* stream, void* user) {
  (void)stream;
  (void)user;
  void* p = NULL;
  if (hipMalloc(&p, bytes) != hipSuccess) return NULL;
  ++g_live;
  ++g_made;
  return p;
}
static void my_free(void* p, void* stream, void* user) {
  (void)stream;
  (void)user;
  if (hipFree(p) == hipSuccess) --g_live;
}

/* the Neel state's energy per site after 4 sweeps, with or without the caller allocator */
static int neel_energy(const double* dA, const int* pattern, const double* H, const ctm_term* terms, int nterm,
                       int caller_alloc, double* E, int* sweeps) {
  enum { d = 2, D = 1, chi = 2, Lx = 2, Ly = 2, nt = 2 };
  ctm_ctx* ctx = NULL;
  int rc = ctm_init(&ctx, dA, d, D, chi, Lx, Ly, pattern, nt, CTM_FP64, NULL);
  CHECK(rc == CTM_OK, "ctm_init: %d %s", rc, ctm_last_error(NULL));
  if (caller_alloc) {
    rc = ctm_set_allocator(ctx, my_alloc, NULL, NULL);
    CHECK(rc == CTM_EINVAL, "ctm_set_allocator with one callback not refused (rc %d)", rc);
    rc = ctm_set_allocator(ctx, my_alloc, my_free, NULL);
    CHECK(rc == CTM_OK, "ctm_set_allocator: %d %s", rc, ctm_last_error(ctx));
  }
  double delta = 0.0;
  rc = ctm_sweep(ctx, 4, 0.0, sweeps, &delta);
  CHECK(rc == CTM_OK && *sweeps == 4, "ctm_sweep: %d %s", rc, ctm_last_error(ctx));
  rc = ctm_energy(ctx, H, nterm, terms, E);
  CHECK(rc == CTM_OK, "ctm_energy: %d %s", rc, ctm_last_error(ctx));
  ctm_free(ctx);
  return 0;
}

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
  int sweeps = 0;
  double E = 0.0, E2 = 0.0;
  if (neel_energy(dA, pattern, H, terms, nterm, 0, &E, &sweeps)) return 1;
  CHECK(fabs(E + 0.5) < 1e-12, "Neel energy %.15f, expected -0.5", E);
  if (neel_energy(dA, pattern, H, terms, nterm, 1, &E2, &sweeps)) return 1;
  CHECK(E2 == E, "caller allocator: energy %.17g, default allocator %.17g", E2, E);
  CHECK(g_made > 0 && g_live == 0, "caller allocator: %d blocks made, %d not handed back", g_made, g_live);
  CHECK(hipFree(dA) == hipSuccess, "hipFree failed");
  printf("c_abi_check: Neel state, E = %.15f per site after %d sweeps; caller allocator %d blocks, all back\n", E,
         sweeps, g_made);
  return 0;
}
