/* C ABI of the single-layer (nested) CTMRG library for MI355X (gfx950).
 *
 * Method: arXiv:2512.14414, "Single-layer framework of variational tensor
 * network states".  The norm <Psi|Psi> of an iPEPS is contracted as one nested
 * single-layer network (Sec. II B, Eq. XY, Fig. NTN): the ket tensor A and the
 * bra tensor A* are absorbed into the corner (C) and edge (T) tensors one
 * layer at a time, on a nested cell of 2Lx x 2Ly sites (Sec. II C).  The
 * environment is computed by multi-site CTMRG (Fig. CTMRG) with projectors
 * from a QR decomposition of the two halves of a 2x2 cluster followed by a
 * truncated SVD (Eqs. PQ, QRSVD); the energy per site is E = <H>/<Psi|Psi>
 * (Eq. ExpH) from 2x2 reduced density matrices with opened physical lines
 * (the impurity tensors of Sec. II B); the gradient is the reverse-mode
 * derivative of that chain (Eq. AD), shortened as proposed in Sec. IV.
 *
 * Conventions
 * -----------
 * Site tensors: n_tensors real tensors A_t[s][l][u][r][d] (C order, float64),
 *   physical index s of dimension d, virtual legs l, u, r, d of dimension D.
 * Unit cell: Lx columns x Ly rows of PEPS sites; pattern[y*Lx + x] is the
 *   tensor index at column x, row y (rows grow downward).
 * Terms: a ctm_term (px, py, a, b, coef) is the bond operator H_bond acting on
 *   sites a and b (0 = top-left, 1 = top-right, 2 = bottom-left, 3 =
 *   bottom-right) of the plaquette whose top-left site is (px, py); the energy
 *   per site is (1/(Lx*Ly)) * sum coef * <H_bond>_ab.
 * H_bond: d^2 x d^2 row-major matrix H[(s_a s_b)][(s_a' s_b')] on the host.
 * Environment layout ("flat env", float64): the nested positions (I, J) of the
 *   2Ly x 2Lx cell in row-major order; for each, C1, C2, C3, C4 (chi x chi)
 *   then T1, T2, T3, T4 (chi x leg x chi).  Legs are listed counter-clockwise
 *   around the site: C1[down][right], C2[left][down], C3[up][left],
 *   C4[right][up], T1[left][s][right], T2[up][s][down], T3[right][s][left],
 *   T4[down][s][up]; the s leg of T1/T2/T3/T4 is the up/right/down/left leg
 *   of the nested site at (I, J).  Nested site kinds: K (ket, legs D, D, D*d,
 *   D) at (even, even), Y (D*d, D, D, D*d) at (even, odd), X (D, D, D, D) at
 *   (odd, even), B (bra, D, D*d, D, D) at (odd, odd); a fused leg is (virtual
 *   index major, physical index minor).
 *
 * Memory: every pointer documented as "device" is a HIP device pointer on the
 * current device; "host" pointers are ordinary host memory.  The caller owns
 * all buffers it passes; the library copies what it keeps.  Work is queued on
 * the stream given to ctm_init (a hipStream_t passed as void*, NULL for the
 * default stream); calls that return host values synchronise that stream.
 *
 * Errors: every call returns CTM_OK (0), a warning (> 0) or an error (< 0).
 * ctm_last_error gives the message.  After an error the context stays valid.
 * A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CTM_H
#define CTM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_ctx ctm_ctx;

enum {
  CTM_OK = 0,
  CTM_ENOTCONV = 1,      /* warning: max_sweeps reached before delta < tol (results still written) */
  CTM_EINVAL = -1,       /* invalid argument */
  CTM_ENOMEM = -2,       /* device allocation failed */
  CTM_EHIP = -3,         /* HIP runtime or kernel launch error */
  CTM_ESOLVER = -4,      /* a projector or corner SVD did not converge (or a bounded wait of the one-launch
                            Jacobi iteration ran out), a cut carries no weight (its bond density matrix
                            N S^T vanishes to working precision: s_1 <= 1e-12 |N|_F |S|_F, so the
                            projectors of Eq. PQ do not exist), or an updated environment tensor is zero */
  CTM_ENONFINITE = -5    /* NaN or Inf found in the environment or the result */
};

enum { CTM_FP64 = 0, CTM_FP32 = 1, CTM_BF16 = 2, CTM_MIXED = 3 };

typedef struct {
  int px, py;    /* plaquette: top-left PEPS site, 0 <= px < Lx, 0 <= py < Ly */
  int a, b;      /* two distinct sites of the plaquette, 0..3 */
  double coef;   /* weight of <H_bond>_ab in the energy per site times Lx*Ly */
} ctm_term;

/* Create a context for site tensors A (device, n_tensors*d*D^4 float64, copied)
 * of the iPEPS of Eq. PEPS on an Lx x Ly unit cell, build the nested cell of
 * Sec. II B-C (Eq. XY: ket K and bra B sites with the crossing tensors X, Y on
 * 2Lx x 2Ly nested positions), and set the sites-derived starting environment
 * (the paper leaves the start open): every C and T is the neighbouring nested
 * site with its outward legs summed over all indices.  The context owns all
 * device memory it allocates; *out receives it (free with ctm_free).
 * precision: CTM_FP64 (all contractions FP64), CTM_FP32 (environment and
 * contractions FP32), CTM_BF16 (environment FP32, contraction operands
 * rounded to bfloat16, FP32 accumulation) or CTM_MIXED (environment and the
 * sweep's contractions FP64, the energy's density-matrix contractions and
 * their adjoints FP32 on the matrix cores: the sweep feeds the SVD
 * derivative, whose 1/(s_i^2 - s_j^2) terms amplify rounding, while the
 * energy holds most of the contraction flops and enters the gradient
 * linearly).  In every mode the projector QR and SVD (Eq. QRSVD), the
 * projector weights, the norms and the energy sum are FP64.  Requires d >= 1, D >= 1, chi >= D*d, Lx, Ly >= 1, pattern ids in
 * [0, n_tensors).  On error *out is NULL. */
int ctm_init(ctm_ctx** out, const double* A, int d, int D, int chi, int Lx, int Ly, const int* pattern,
             int n_tensors, int precision, void* stream);

/* The conventional double-layer method that the nested one is compared with
 * (Eq. Tred; Appendix, Fig. SM-Compare): a context over the Lx x Ly lattice
 * of reduced tensors a_t[(l l'), (u u'), (r r'), (d d')] = sum_s A_t[s,l,u,r,d]
 * A_t[s,l',u',r',d'] (legs of dimension D^2, ket index major), formed on the
 * device from A with the same arguments, ownership and errors as ctm_init.
 * The sweep, its options, the projectors (now of (chi D^2) x chi; the
 * randomized partial SVD of option "svd_method" suits these larger cuts), the
 * convergence measures and the environment layout (Lx*Ly positions, T legs
 * of dimension D^2) are those of the nested context; the sweep absorbs every
 * site layer by layer (its D^2 legs split into ket and bra halves: A, then A*),
 * and ctm_energy, ctm_last_rdms and ctm_observables contract each plaquette
 * quadrant with the ket and then the bra tensor of its site, without forming
 * the open reduced tensor.  ctm_energy_grad and ctm_energy_grad_fp
 * differentiate this network the same way (the adjoints of the per-frame
 * copies of A and of the density matrices' A are added up into dE/dA).
 * Requires chi >= D*D. */
int ctm_init_double_layer(ctm_ctx** out, const double* A, int d, int D, int chi, int Lx, int Ly, const int* pattern,
                          int n_tensors, int precision, void* stream);

/* Replace the site tensors (device, same shape as in ctm_init); the environment is kept. */
int ctm_set_tensors(ctm_ctx* ctx, const double* A);

/* Restore the sites-derived starting environment of ctm_init. */
int ctm_reset_env(ctm_ctx* ctx);

/* Number of float64 values of the flat environment layout. */
int64_t ctm_env_size(const ctm_ctx* ctx);

/* Copy the environment in from / out to a device float64 buffer of ctm_env_size values. */
int ctm_set_env(ctm_ctx* ctx, const double* env);
int ctm_get_env(ctm_ctx* ctx, double* env);

/* CTMRG iterations (Sec. II C): each sweep is a left, right, up and down move;
 * a move has 2Lx (left/right) or 2Ly (up/down) column steps, and each step
 * computes the projectors of all rows (Eqs. PQ, QRSVD) and then updates
 * C1, T4, C4 of the next column (Fig. CTMRG b) with Frobenius normalisation.
 * If tol > 0, after each sweep delta = max over corners of the L1 distance of
 * the normalised singular-value spectra to the previous sweep (for the first
 * sweep after ctm_init, ctm_reset_env or ctm_set_env: to the environment the
 * sweep started from; the spectra are those of ctm_corner_spectra), and the loop
 * stops once delta < tol; returns CTM_ENOTCONV if max_sweeps is reached
 * first.  sweeps_done and delta (host, may be NULL) receive the count and the
 * last delta (delta is -1 when tol <= 0). */
int ctm_sweep(ctm_ctx* ctx, int max_sweeps, double tol, int* sweeps_done, double* delta);

/* Corner spectra of the current environment (the quantity whose convergence
 * ends the iteration, Sec. II C): for every position (I, J) of the cell in
 * row-major order (2Ly x 2Lx nested positions; Ly x Lx on a double-layer
 * context) and each corner C1..C4, the singular values of the chi x chi corner
 * in descending order, divided by their sum and zero-padded to chi.  out (host)
 * receives 4 * (positions) * chi float64 values, capacity is its length in
 * values; with out == NULL only *n_written (host, may be NULL otherwise) is
 * set to the required length.  CTM_EINVAL if capacity is too small;
 * CTM_ESOLVER if a corner SVD fails.  The sweep's own convergence state is not
 * changed.  Synchronises the context's stream. */
int ctm_corner_spectra(ctm_ctx* ctx, double* out, int64_t capacity, int64_t* n_written);

/* Energy per site (Eq. ExpH) from the current environment: for every plaquette
 * named by a term, the 2x2 reduced density matrix rho (d^4 x d^4, ket indices
 * of the four sites as row, bra indices as column, Sec. II B impurities) is
 * contracted; <H>_ab = sum H[(b_a b_b)][(k_a k_b)] rho_ab[(k_a k_b)][(b_a b_b)] / Tr rho.
 * H_bond and terms are host arrays; E (host) receives the result. */
int ctm_energy(ctm_ctx* ctx, const double* H_bond, int n_terms, const ctm_term* terms, double* E);

/* Energy and its gradient (Eq. AD): E(A) = energy per site after n_sweeps
 * sweeps started from the context's current environment, which is held
 * constant (the shortened derivative chain of Sec. IV: from a given, ideally
 * converged, environment).  If A (device, as in ctm_init) is not NULL it
 * replaces the site tensors first.  dEdA (device, n_tensors*d*D^4 float64)
 * receives dE/dA in the layout of A.  The derivative of every step is
 * hand-written: contractions by their transposed contractions, the
 * normalisations, the plaquette density matrices and the projectors, whose
 * SVD derivative uses the Lorentzian-broadened F_ij = D/(D^2 + (eta m)^2),
 * D = s_j^2 - s_i^2, m = max(s_i^2, s_j^2) (option "lorentz_eta").
 * Checkpointing: the last sweep and the energy are recorded in the forward
 * pass; one environment snapshot is kept per earlier sweep, and each earlier
 * sweep is recomputed once during the reverse pass.  Afterwards the environment is
 * the one reached by the n_sweeps sweeps.  H_bond, terms as in ctm_energy;
 * E (host) receives the energy. */
int ctm_energy_grad(ctm_ctx* ctx, const double* A, int n_sweeps, const double* H_bond, int n_terms,
                    const ctm_term* terms, double* E, double* dEdA);

/* Gradient of the converged energy E(A) = E(env*(A), A), where env* is the
 * fixed point of one sweep, env* = f(env*, A) (the fixed-point form of the
 * derivative of Eq. AD, Sec. IV): by implicit differentiation dE/dA =
 * dE/dA|_env + lam df/dA with lam = dE/denv + lam df/denv, summed as the
 * series lam = mu_0 + mu_1 + ..., mu_{k+1} = mu_k df/denv, each term one
 * reverse pass over a single recorded sweep.  The context's current
 * environment must be converged (ctm_sweep to a small delta): the gauge rules
 * (projector column signs, tensor signs) make a converged environment a fixed
 * point of the sweep entry by entry, and *gap (host, may be NULL) receives
 * max|f(env) - env| / max|env| of the recorded sweep to check it.  The series
 * stops once max|mu_k| <= tol * max|mu_1| or after max_iter terms (then
 * CTM_ENOTCONV, results still written); *iters (host, may be NULL) receives
 * the number of terms beyond the first.  A (device, optional) replaces the
 * site tensors first; E (host) receives the energy after the recorded sweep,
 * dEdA (device, layout of A) the gradient.  The environment is left at the
 * result of the recorded sweep.  Derivatives of the projectors as in
 * ctm_energy_grad. */
int ctm_energy_grad_fp(ctm_ctx* ctx, const double* A, double tol, int max_iter, const double* H_bond, int n_terms,
                       const ctm_term* terms, double* E, double* dEdA, int* iters, double* gap);

/* Plaquette density matrices of the last ctm_energy call, copied to a host
 * buffer of n * d^8 float64 values in the order of first appearance of the
 * plaquettes in the term list; n (host) receives the count. */
int ctm_last_rdms(ctm_ctx* ctx, double* rho, int capacity, int* n);

/* Order parameters of spin-1/2 sites (d = 2) from the plaquette density
 * matrices of the last ctm_energy call (Eq. Mag1: site moments m_i, whose mean
 * length over the inequivalent sites is the magnetisation M; Eq. Mag2: bond
 * correlations, whose edge sums on two empty plaquettes give M_p).  out (host)
 * receives CTM_N_OBS float64 values per plaquette, for the first
 * min(capacity, n) plaquettes in the order of ctm_last_rdms: the moments
 * (<S^x>, <S^y>, <S^z>) of the sites TL, TR, BL, BR, each <O> = Tr(O rho_s) /
 * Tr rho_s over the one-site matrix (basis up, down; the tensors are real, so
 * <S^y> is the real part of an imaginary trace, 0), then <S_a . S_b> =
 * Tr((S_a . S_b) rho_ab) / Tr rho_ab for the pairs (TL,TR) (BL,BR) (TL,BL)
 * (TR,BR) (TL,BR) (TR,BL).  n (host) receives the plaquette count (0 before any
 * ctm_energy).  CTM_EINVAL for d != 2 or a NULL pointer.  Synchronises the
 * context's stream. */
#define CTM_N_OBS 18
int ctm_observables(ctm_ctx* ctx, double* out, int capacity, int* n);

/* Options (key, value):
 *   "svd_cutoff"  relative cutoff below which s^(-1/2) is set to zero (default 1e-10)
 *   "lorentz_eta" relative Lorentzian width of the SVD derivative (default 1e-12)
 *   "check_finite" 1 to test the environment for NaN/Inf after every sweep (default 1)
 *   "streams"     2 (default) to run the odd rows of a column step (half systems,
 *                 their QR) on a second stream created by the library, joined
 *                 back before the SVD, in sweeps that are not differentiated;
 *                 1 for one stream.  Both give identical results.
 *   "rowmajor_bf16" 1 (default) to run large BF16-mode products of plain
 *                 row-major operands on the dedicated 128 x 128-tile kernel, 0
 *                 for the general contraction kernel; a process-wide switch.
 *   "rowmajor_f64", "rowmajor_f32" 1 (default) to run large FP64 (FP32-mode)
 *                 products with A contiguous along k and B along n on the
 *                 dedicated 128 x 128-tile kernel, 0 for the general contraction
 *                 kernel; process-wide switches.
 *   "jacobi_one_launch" 1 (default) to run the whole Jacobi iteration of the
 *                 projector SVD (all sweeps, the stop test taken on the device)
 *                 in one launch, when the device holds its grid at once (else
 *                 one launch per round); 0 for one launch per round and the stop
 *                 test on the host.  Both give identical results.  No
 *                 convergence, or a wait between rounds that runs out (waits
 *                 are bounded), fails the call with CTM_ESOLVER when it returns.
 *   "proj_cache"  1 (default): in ctm_energy_grad with n > 1, the forward sweeps
 *                 that the checkpointed reverse pass recomputes keep their
 *                 projector blocks (projectors, singular vectors of N S^T,
 *                 singular values and weights of every cut: about 0.45 GB per
 *                 sweep at D=6, chi=72), and the recomputation takes them
 *                 instead of repeating the QR and SVD (same results bit for
 *                 bit); 0 recomputes them.
 *   "conv_rdm"    1 to take the delta of ctm_sweep as the largest change of any
 *                 entry of the trace-normalised plaquette density matrices of
 *                 all Lx*Ly plaquettes (the quantities the energy and the order
 *                 parameters are made of), computed in the energy's precision
 *                 after every sweep (FP32 in the mixed mode: deltas level off
 *                 near 1e-7 there); on the nested network they settle in tens
 *                 of sweeps where the corner spectra and the environment
 *                 entries take hundreds.  Takes precedence over "conv_env";
 *                 default 0.
 *   "conv_env"    1 to take the delta of ctm_sweep as max|env_new - env_old| /
 *                 max|env_old| over all environment entries (meaningful because
 *                 the gauge rules make a converged environment a fixed point
 *                 entry by entry; the corner spectra alone stop too early when the
 *                 corners are of rank one while the edges still move), 0
 *                 (default) for the corner spectra.
 *   "svd_method"  0 (default) exact projector SVD; 1 randomized partial SVD
 *                 (range finder with "svd_oversample" extra columns, default 8,
 *                 "svd_power" subspace passes, default 2, test matrix from
 *                 SplitMix64 with "svd_seed", default 0) in ctm_sweep; the
 *                 sweeps of ctm_energy_grad (also those the reverse pass
 *                 recomputes) and of ctm_energy_grad_fp take the exact SVD.
 *   "energy_precision" CTM_FP64, CTM_FP32 or CTM_BF16: the precision of the
 *                 energy's density-matrix contractions (and their adjoints) alone,
 *                 whatever the sweep's (default: that of the context's precision).
 *   "jacobi_cooperative" 1 (default) to make that one launch a cooperative
 *                 launch, whose workgroups the runtime guarantees to be resident
 *                 together (a grid the device cannot hold is refused and the
 *                 call falls back to one launch per round); 0 for a plain launch
 *                 taken only when the occupancy API says the grid fits.
 *   "jacobi_max_sweeps" the most Jacobi sweeps of one projector SVD (1..1000,
 *                 default 40); an SVD that needs more fails the call with
 *                 CTM_ESOLVER.
 *   "qr_fused_vy" 1 (default) to have the Householder panel kernel write the
 *                 dense factors of its block reflector for the trailing update
 *                 itself, 0 for a separate launch; a process-wide switch.  Both
 *                 give identical results.
 *   "qr_one_update" 1 (default) to run each panel's trailing update of the
 *                 Householder QR as one launch (16 columns per workgroup), 0
 *                 for two matrix-core products with a split sum; a
 *                 process-wide switch.  Both give identical results: the one
 *                 launch repeats the products' MFMA chains, K split and order
 *                 of partial sums. */
int ctm_set_option(ctm_ctx* ctx, const char* key, double value);

/* Device memory from the caller's allocator (the boundary's ownership rule:
 * the context owns its memory, and a framework's caching allocator, such as
 * PyTorch's, may back it).  From this call on, every new block the context
 * needs comes from alloc(bytes, stream, user), which returns a device pointer
 * aligned to 256 bytes, or NULL when it has no memory (the library then
 * returns the cached blocks of all its contexts and asks once more; if that
 * fails too, the call that needed the block fails with CTM_ENOMEM).  stream is the context's stream that will use
 * the block (a hipStream_t as void*: the stream given to ctm_init, or the
 * context's second stream).  The context keeps freed blocks for reuse and
 * hands each back with free(ptr, stream, user), to the allocator that made
 * it and with the stream it was made for, when it releases its cache: at
 * ctm_free at the latest, or earlier when an allocation fails.  Blocks made
 * before the call keep their allocator (the device's stream-ordered pool by
 * default).  Both callbacks run on the thread that calls into the context.
 * alloc = free = NULL restores the default for new blocks; CTM_EINVAL when
 * exactly one of them is NULL. */
typedef void* (*ctm_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*ctm_free_fn)(void* ptr, void* stream, void* user);
int ctm_set_allocator(ctm_ctx* ctx, ctm_alloc_fn alloc, ctm_free_fn free, void* user);

/* Live timing of the library's main kernel families.  Between
 * ctm_profile_begin and ctm_profile_end every launch of a timed family, by
 * any context of the process, is bracketed by two HIP events on its stream.
 * ctm_profile_end fills three host arrays of 5 entries each (any may be NULL),
 * indexed by family: 0, 1, 2 = the MFMA contraction kernel on the FP64, FP32
 * and BF16 paths (flops 2*M*N*K per launch), 3 = the block Jacobi rounds of
 * the projector SVD (flops of the Gram matrices and column rotations), 4 = the
 * Householder QR panels: the summed kernel time in milliseconds, the summed
 * algorithmic flops and the launch count. */
int ctm_profile_begin(ctm_ctx* ctx);
int ctm_profile_end(ctm_ctx* ctx, double* kernel_ms, double* kernel_flops, int64_t* launches);

/* Message of the last error of this context (or of the last failed ctm_init if ctx is NULL). */
const char* ctm_last_error(const ctm_ctx* ctx);

/* Release the context and its device memory (NULL is allowed). */
void ctm_free(ctm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CTM_H */
