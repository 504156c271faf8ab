"""L-BFGS with a strong-Wolfe line search, optionally screened by a surrogate.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper minimises E(X) (Eq. OptPro) with L-BFGS on the gradient of Eq. AD
(Sec. II A).  Its details are not given; the reading used here:

* search direction from the two-loop recursion over the last ``history``
  pairs (s, y), initial scaling gamma = s.y / y.y (Nocedal and Wright,
  Algorithms 7.4 and 7.5); without history the first trial step is
  alpha0 / max|g|, else 1; a non-descent direction resets the history;
* plain line search: bracketing and zoom for the strong Wolfe conditions
  (Nocedal and Wright, Algorithms 3.5 and 3.6) with safeguarded cubic
  interpolation (their Eq. 3.59; bisection when the minimiser falls outside
  the middle 80 % of the bracket), at most ``max_ls`` evaluations; when they
  run out, the lowest trial point that passed the Armijo test with a strict
  decrease is taken, and
  if there is none the history is dropped and the iteration is retried
  along -g (the run stops when a search along -g fails as well);
* surrogate screening (from iteration ``sur_start``, once trained): the trial
  steps alpha_j = alpha_init 2^(extrap - j) (j < n_trials, so from
  2^extrap down to 2^(extrap - n_trials + 1) times the unit step) are ranked
  by the predicted energy relative to the prediction at the current point,
  f + (y(x + alpha_j p) - y(x)), which cancels a smooth bias of the model;
  the best ``max_screened`` candidates whose predicted decrease passes the
  Armijo test are evaluated exactly in that order and the first that
  satisfies the strong Wolfe conditions is taken; otherwise the plain search
  runs.  Every exact evaluation is added to the training set; the surrogate
  is refitted (on the last ``window`` pairs, or all) after iteration
  sur_start - 1 and then every ``refit_every`` iterations.

Plain numpy in float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Params:
    max_iter: int = 100
    history: int = 10
    c1: float = 1e-4
    c2: float = 0.9
    gtol: float = 1e-6
    max_ls: int = 20
    alpha0: float = 1.0
    sur_start: int = 0          # 0: no screening
    n_trials: int = 8
    max_screened: int = 1
    refit_every: int = 10
    extrap: int = 2
    window: int = 0             # refit on the last ``window`` pairs; 0: all


@dataclass
class Result:
    x: np.ndarray
    f: float
    records: list = field(default_factory=list)   # (iter, evals, screened, f, max|g|, step)
    evals: int = 0
    resets: int = 0
    data_x: list = field(default_factory=list)
    data_f: list = field(default_factory=list)


def cubic_step(lo, flo, dlo, hi, fhi, dhi):
    """Minimiser of the cubic through (lo, flo, dlo) and (hi, fhi, dhi), safeguarded."""
    a_min, a_max = min(lo, hi), max(lo, hi)
    w = a_max - a_min
    d1 = dlo + dhi - 3.0 * (flo - fhi) / (lo - hi)
    disc = d1 * d1 - dlo * dhi
    a = None
    if disc >= 0.0:
        d2 = math.copysign(math.sqrt(disc), hi - lo)
        den = dhi - dlo + 2.0 * d2
        if den != 0.0:
            a = hi - (hi - lo) * (dhi + d2 - d1) / den
    if a is None or not math.isfinite(a) or a < a_min + 0.1 * w or a > a_max - 0.1 * w:
        a = 0.5 * (lo + hi)
    return a


def minimize(fg, x0, p: Params, predictor=None, train=None, features=None):
    """L-BFGS from x0.  fg(x) -> (f, g).  predictor(list of feature vectors) ->
    predicted f; train(data_x, data_f) refits it; features(x) -> its input."""
    res = Result(x=np.array(x0, dtype=np.float64), f=0.0)
    x = res.x.copy()
    f, g = fg(x)
    res.evals = 1
    if predictor is not None:
        res.data_x.append(features(x))
        res.data_f.append(f)

    def evaluate(xt):
        ft, gt = fg(xt)
        res.evals += 1
        if predictor is not None:
            res.data_x.append(features(xt))
            res.data_f.append(ft)
        return ft, gt

    S, Y = [], []
    trained = False
    k = 0
    while k < p.max_iter:
        k += 1
        gmax = float(np.max(np.abs(g)))
        if gmax < p.gtol:
            break
        q = g.copy()
        alphas = []
        for s_i, y_i in zip(reversed(S), reversed(Y)):
            rho = 1.0 / float(y_i @ s_i)
            a = rho * float(s_i @ q)
            q = q - a * y_i
            alphas.append((rho, a))
        gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1]) if S else 1.0
        r = gamma * q
        for (s_i, y_i), (rho, a) in zip(zip(S, Y), reversed(alphas)):
            b = rho * float(y_i @ r)
            r = r + (a - b) * s_i
        pdir = -r
        d0 = float(g @ pdir)
        if d0 >= 0.0:
            S, Y = [], []
            pdir = -g
            d0 = -float(g @ g)
        a_init = p.alpha0 / gmax if not S else 1.0

        accepted, screened = None, 0
        if predictor is not None and trained and p.sur_start > 0 and k >= p.sur_start:
            cands = [a_init * 2.0 ** (p.extrap - j) for j in range(p.n_trials)]
            preds = np.asarray(predictor([features(x)] + [features(x + a * pdir) for a in cands]), dtype=np.float64)
            pc = f + (preds[1:] - preds[0])
            order = np.argsort(pc, kind="stable")
            for j in order[: p.max_screened]:
                a = cands[int(j)]
                if not pc[int(j)] <= f + p.c1 * a * d0:
                    break
                xt = x + a * pdir
                ft, gt = evaluate(xt)
                if ft <= f + p.c1 * a * d0 and abs(float(gt @ pdir)) <= -p.c2 * d0:
                    accepted, screened = (a, xt, ft, gt), 1
                    break
        if accepted is None:
            accepted = _line_search(evaluate, x, f, pdir, d0, a_init, p)
            if accepted is None:
                if not S:
                    break
                # a failed search along a quasi-Newton direction: forget the
                # curvature pairs and retry this iteration along -g
                S, Y = [], []
                res.resets += 1
                k -= 1
                continue
        a, xn, fn, gn = accepted
        s, y = xn - x, gn - g
        if float(s @ y) > 0.0:
            S.append(s)
            Y.append(y)
            if len(S) > p.history:
                S.pop(0)
                Y.pop(0)
        x, f, g = xn, fn, gn
        res.records.append((k, res.evals, screened, f, float(np.max(np.abs(g))), a))
        if predictor is not None and p.sur_start > 0 and k >= p.sur_start - 1 and \
                (k - (p.sur_start - 1)) % p.refit_every == 0:
            w = p.window if p.window > 0 else len(res.data_f)
            train(res.data_x[-w:], res.data_f[-w:])
            trained = True
    res.x, res.f = x, f
    return res


def _line_search(evaluate, x, f0, pdir, d0, a_init, p):
    """Strong Wolfe search: bracketing, then zoom.  If the budget runs out, the
    trial point of lowest f among those that passed the Armijo test with a
    strict decrease is taken
    (the curvature test can fail for good where f has kinks, e.g. where the
    set of kept singular values changes); None if there is none."""
    used = 0
    a_prev, f_prev, d_prev = 0.0, f0, d0
    a = a_init
    best = [None]

    def trial(a):
        xt = x + a * pdir
        ft, gt = evaluate(xt)
        if ft <= f0 + p.c1 * a * d0 and ft < f0 and (best[0] is None or ft < best[0][2]):
            best[0] = (a, xt, ft, gt)
        return xt, ft, gt, float(gt @ pdir)

    while used < p.max_ls:
        xt, ft, gt, dt = trial(a)
        used += 1
        if ft > f0 + p.c1 * a * d0 or (used > 1 and ft >= f_prev):
            return _zoom(trial, f0, d0, (a_prev, f_prev, d_prev), (a, ft, dt), used, p, best)
        if abs(dt) <= -p.c2 * d0:
            return a, xt, ft, gt
        if dt >= 0.0:
            return _zoom(trial, f0, d0, (a, ft, dt), (a_prev, f_prev, d_prev), used, p, best)
        a_prev, f_prev, d_prev = a, ft, dt
        a = 2.0 * a
    return best[0]


def _zoom(trial, f0, d0, lo, hi, used, p, best):
    lo_a, lo_f, lo_d = lo
    hi_a, hi_f, hi_d = hi
    while used < p.max_ls:
        a = cubic_step(lo_a, lo_f, lo_d, hi_a, hi_f, hi_d)
        xt, ft, gt, dt = trial(a)
        used += 1
        if ft > f0 + p.c1 * a * d0 or ft >= lo_f:
            hi_a, hi_f, hi_d = a, ft, dt
        else:
            if abs(dt) <= -p.c2 * d0:
                return a, xt, ft, gt
            if dt * (hi_a - lo_a) >= 0.0:
                hi_a, hi_f, hi_d = lo_a, lo_f, lo_d
            lo_a, lo_f, lo_d = a, ft, dt
    return best[0]
