/* C ABI of the optimisation layer: L-BFGS on the energy and the learned
 * line-search surrogate (arXiv:2512.14414, Sec. II A: the variational energy
 * E(X) of Eq. OptPro is minimised with L-BFGS on the gradient of Eq. AD).
 *
 * Surrogate.  A perceptron with two hidden GELU layers (gelu(z) = z/2 (1 +
 * erf(z/sqrt 2))), y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3, float32
 * parameters flattened as W1 [width][n_in], b1 [width], W2 [width][width],
 * b2 [width], W3 [width], b3 [1].  It is trained on (input, energy) pairs that
 * the optimisation itself produces and ranks the trial steps of a line
 * search; every accepted step is still confirmed by an exact evaluation.
 * Forward, backward and Adam run in the library's kernels.
 *
 * Conventions as in ctm.h: "device" pointers are HIP device memory, "host"
 * pointers ordinary memory; the caller owns all buffers it passes; work is
 * queued on the stream given at creation; calls returning host values
 * synchronise it.  Status codes are the CTM_* codes of ctm.h.
 */
#ifndef CTM_OPT_H
#define CTM_OPT_H

#include <stdint.h>

#include "ctm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sur_net sur_net;

/* Create a network with n_in inputs and two hidden layers of ``width``.
 * Every parameter is drawn uniform in +-1/sqrt(fan_in) (fan_in = n_in for
 * W1, b1 and width for the others) from SplitMix64: parameter i of the flat
 * vector is (2u - 1)/sqrt(fan_in), u = (splitmix64(seed, i) >> 11) * 2^-53,
 * where splitmix64(seed, i) is the (i+1)-th output of the generator seeded
 * with ``seed``; rounded to float32.  Target statistics start at mean 0,
 * deviation 1.  stream: hipStream_t as void* (NULL: default stream). */
int sur_init(sur_net** out, int n_in, int width, uint64_t seed, void* stream);

/* Number of float32 parameters. */
int64_t sur_param_count(const sur_net* net);

/* Copy the flat parameters out to / in from a device float32 buffer. */
int sur_get_params(sur_net* net, float* params);
int sur_set_params(sur_net* net, const float* params);

/* Predicted energies y[b] (device, batch floats) of the inputs X (device,
 * batch x n_in floats, row-major), in the units of the training targets
 * (the network output times the target deviation plus the target mean of the
 * last sur_train call). */
int sur_predict(sur_net* net, const float* X, int batch, float* y);

/* Allocation-free variant of sur_predict, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and the same result (the same
 * kernels on the same data): every workspace of the forward pass (hidden
 * activations, split-K partial sums) is cut from a fixed 16 MiB device array
 * of the library, one per GPU, held until the process ends; the call makes no
 * device allocation or free.  CTM_EINVAL (message with the sizes) if the
 * batch needs more than 16 MiB of workspace (about 3000 inputs of a
 * 5000 -> 256 -> 256 -> 1 network).  Every call on one GPU shares that array,
 * and a call's array contents are only valid until the next call on that
 * GPU: calls that overlap on one GPU (other streams or threads) race. */
int sur_predict_noalloc(sur_net* net, const float* X, int batch, float* y);

/* Mean squared error (1/n) sum (f(x_i) - t_i)^2 of the raw network output f
 * against targets t (device, n floats; no standardisation) and its gradient
 * (device, sur_param_count floats, flat layout); loss (host) may be NULL. */
int sur_loss_grad(sur_net* net, const float* X, const float* t, int n, float* loss, float* grad);

/* Fit: the targets t (device, n floats) are standardised by their mean and
 * deviation (kept for sur_predict); then ``steps`` full-batch Adam steps
 * (beta 0.9, 0.999, eps 1e-8, learning rate lr, moments reset at each call,
 * parameters kept) on the mean squared error.  loss (host, may be NULL)
 * receives the loss evaluated before the last step. */
int sur_train(sur_net* net, const float* X, const float* t, int n, int steps, float lr, float* loss);

const char* sur_last_error(const sur_net* net);
void sur_free(sur_net* net);

/* ------------------------------------------------------------------------- */
/* Objective: f (host) and gradient g (device, n doubles) at x (device).
 * Returns 0 on success; any other value stops the optimisation with that code. */
typedef int (*ctm_objective_fn)(void* user, const double* x, double* f, double* g);

typedef struct {
  int max_iter;        /* iterations (default 100) */
  int history;         /* stored (s, y) pairs (default 10) */
  double c1, c2;       /* strong Wolfe constants (default 1e-4, 0.9) */
  double gtol;         /* stop once max|g| < gtol (default 1e-6) */
  int max_ls;          /* evaluations of one plain line search (default 20) */
  double alpha0;       /* first trial step without history is alpha0 / max|g| (default 1) */
  int sur_start;       /* first iteration screened by the surrogate; 0 = never (default 0) */
  int n_trials;        /* trial steps alpha_init 2^(extrap-j), j < n_trials (default 8) */
  int max_screened;    /* screened candidates evaluated before the plain search (default 1) */
  int refit_every;     /* refit after iteration sur_start-1 and every refit_every iterations (default 10) */
  int refit_steps;     /* Adam steps per refit (default 200) */
  float lr;            /* Adam learning rate (default 1e-3) */
  int n_blocks;        /* surrogate input: x split into n_blocks equal blocks, each normalised (default 1) */
  int extrap;          /* largest screened step is alpha_init 2^extrap (default 2) */
  int window;          /* refit on the last ``window`` exact evaluations; 0 = all of them (default 0) */
} ctm_lbfgs_params;

typedef struct {
  int iter;            /* 1-based iteration */
  int evals;           /* exact evaluations so far */
  int screened;        /* 1 if the step was a surrogate-screened candidate */
  double f;            /* objective after the step */
  double gmax;         /* max|g| after the step */
  double step;         /* accepted step length */
} ctm_lbfgs_record;

/* Fill *p with the defaults above. */
void ctm_lbfgs_default_params(ctm_lbfgs_params* p);

/* Minimise fg from x (device, n doubles; overwritten with the last iterate)
 * with L-BFGS: two-loop recursion (Nocedal and Wright, Algorithms 7.4, 7.5)
 * with scaling s.y/y.y; plain line search by bracketing and zoom for the
 * strong Wolfe conditions (their Algorithms 3.5, 3.6) with safeguarded cubic
 * interpolation (bisection outside the middle 80 % of the bracket); when its
 * max_ls evaluations run out, the trial point of lowest f that passed the
 * Armijo test with a strict decrease is taken, and if there is none the
 * history is dropped and the iteration is retried along -g (the run ends
 * when a search along -g fails as well).  Without
 * history the first trial step alpha_init is alpha0/max|g|, else 1.  If sur
 * is not NULL, from iteration sur_start on (once trained) the n_trials steps
 * alpha_init 2^(extrap-j) are ranked by the predicted objective relative to
 * the prediction at the current point, f + y(x + alpha p) - y(x); the best
 * max_screened candidates whose predicted decrease passes the Armijo test are
 * evaluated exactly in that order and the first that satisfies the strong
 * Wolfe conditions is taken; otherwise the plain search runs.  Every exact
 * evaluation becomes a training pair (normalised x, f).  trace (host, may be
 * NULL) receives up to ``capacity`` records, n_iter (host, may be NULL) the
 * iteration count.  Returns CTM_OK when max|g| < gtol was reached,
 * CTM_ENOTCONV when max_iter ran out or a search along -g failed,
 * CTM_ENONFINITE when the gradient at an accepted iterate is not finite.  An
 * objective may return f = +inf (with any finite g) for a point it cannot
 * evaluate: the search treats it as a failed Armijo test and such values are
 * kept out of the surrogate's training set. */
int ctm_lbfgs(int64_t n, double* x, ctm_objective_fn fg, void* user, sur_net* sur, const ctm_lbfgs_params* p,
              void* stream, ctm_lbfgs_record* trace, int capacity, int* n_iter);

/* Message of the last failed ctm_lbfgs call of this thread. */
const char* ctm_lbfgs_last_error(void);

/* The energy objective: x are the site tensors (layout of ctm_init); an
 * evaluation replaces the tensors of ctx, runs up to conv_sweeps sweeps
 * (stopping at delta < conv_tol) from the environment of the previous
 * evaluation, then ctm_energy_grad with grad_sweeps differentiated sweeps. */
typedef struct {
  ctm_ctx* ctx;
  const double* H_bond;   /* host, as in ctm_energy */
  int n_terms;
  const ctm_term* terms;  /* host */
  int conv_sweeps;
  double conv_tol;
  int grad_sweeps;
} ctm_energy_objective;

int ctm_energy_objective_fn(void* user, const double* x, double* f, double* g);

#ifdef __cplusplus
}
#endif

#endif /* CTM_OPT_H */
