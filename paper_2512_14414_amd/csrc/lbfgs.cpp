// L-BFGS with a strong-Wolfe line search, optionally screened by the learned
// surrogate (Sec. II A: the energy of Eq. OptPro is minimised with L-BFGS on
// the gradient of Eq. AD).  Vectors stay on the device (float64); the host
// runs the scalar control flow.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ctm_opt.h"
#include "engine.h"
#include "opt_kernels.h"

using namespace ctm;

namespace {

thread_local std::string g_opt_error;

struct Vec {
  Dev* dev;
  DBuf b;
  Vec(Dev* d, int64_t n) : dev(d), b(d, (size_t)n * 8) {}
  double* p() const { return (double*)b.p; }
};

struct Opt {
  Dev dev;
  int64_t n = 0;
  ctm_objective_fn fg = nullptr;
  void* user = nullptr;
  sur_net* sur = nullptr;
  ctm_lbfgs_params p{};
  DBuf scal;                       // device scalars
  // surrogate training set (normalised inputs, objective values), float32
  DBuf dX, dF;
  int64_t cap = 0, count = 0;
  int evals = 0;

  double dot(const double* a, const double* b) {
    optk::DotList L;
    L.x[0] = a;
    L.y[0] = b;
    HIP_CHECK(optk::launch_dots(L, 1, n, (double*)scal.p, dev.stream));
    double r = 0;
    HIP_CHECK(hipMemcpyAsync(&r, scal.p, 8, hipMemcpyDeviceToHost, dev.stream));
    HIP_CHECK(hipStreamSynchronize(dev.stream));
    return r;
  }
  double absmax(const double* a) {
    HIP_CHECK(optk::launch_absmax(a, n, (double*)scal.p, dev.stream));
    double r = 0;
    HIP_CHECK(hipMemcpyAsync(&r, scal.p, 8, hipMemcpyDeviceToHost, dev.stream));
    HIP_CHECK(hipStreamSynchronize(dev.stream));
    return r;
  }
  void features(const double* x, float* out) {
    const int64_t blocks = std::max(1, p.n_blocks);
    HIP_CHECK(optk::launch_block_normalize(x, blocks, n / blocks, out, dev.stream));
  }
  // exact evaluation; the pair joins the training set
  void evaluate(const double* x, double* f, double* g) {
    HIP_CHECK(hipStreamSynchronize(dev.stream));
    int rc = fg(user, x, f, g);
    if (rc != 0) throw Error(rc < 0 ? rc : CTM_EINVAL, "objective returned " + std::to_string(rc));
    ++evals;
    if (!sur || !std::isfinite(*f)) return;
    if (count == cap) {
      int64_t nc = std::max<int64_t>(64, 2 * cap);
      DBuf nX(&dev, (size_t)nc * n * 4), nF(&dev, (size_t)nc * 4);
      if (count) {
        HIP_CHECK(hipMemcpyAsync(nX.p, dX.p, (size_t)count * n * 4, hipMemcpyDeviceToDevice, dev.stream));
        HIP_CHECK(hipMemcpyAsync(nF.p, dF.p, (size_t)count * 4, hipMemcpyDeviceToDevice, dev.stream));
      }
      dX = std::move(nX);
      dF = std::move(nF);
      cap = nc;
    }
    features(x, (float*)dX.p + count * n);
    float fv = (float)*f;
    HIP_CHECK(hipMemcpyAsync((float*)dF.p + count, &fv, 4, hipMemcpyHostToDevice, dev.stream));
    HIP_CHECK(hipStreamSynchronize(dev.stream));
    ++count;
  }
};

// Safeguarded minimiser of the cubic through (lo, flo, dlo) and (hi, fhi, dhi)
// (Nocedal and Wright, Eq. 3.59); bisection outside the middle 80 % of the bracket.
double cubic_step(double lo, double flo, double dlo, double hi, double fhi, double dhi) {
  const double amin = std::min(lo, hi), amax = std::max(lo, hi), w = amax - amin;
  const double d1 = dlo + dhi - 3.0 * (flo - fhi) / (lo - hi);
  const double disc = d1 * d1 - dlo * dhi;
  double a = NAN;
  if (disc >= 0.0) {
    const double d2 = std::copysign(std::sqrt(disc), hi - lo);
    const double den = dhi - dlo + 2.0 * d2;
    if (den != 0.0) a = hi - (hi - lo) * (dhi + d2 - d1) / den;
  }
  if (!std::isfinite(a) || a < amin + 0.1 * w || a > amax - 0.1 * w) a = 0.5 * (lo + hi);
  return a;
}

// Strong Wolfe line search along pdir from x (f0, d0 = g.pdir); on success xt,
// gt hold the accepted point and its gradient.  When the evaluations run out
// the trial point of lowest f among those that passed the Armijo test with a
// strict decrease is taken (kept in xb, gb): where f has kinks the curvature
// test can fail at every trial point.
bool line_search(Opt& o, const double* x, double f0, const double* pdir, double d0, double a_init, double* xt,
                 double* gt, double* xb, double* gb, double& a_out, double& f_out) {
  const ctm_lbfgs_params& p = o.p;
  int used = 0;
  double a_prev = 0.0, f_prev = f0, d_prev = d0, a = a_init;
  double lo = 0, flo = 0, dlo = 0, hi = 0, fhi = 0, dhi = 0;
  bool zoom = false, have_best = false;
  double a_best = 0, f_best = 0;
  auto keep = [&](double at, double ft) {
    if (!(ft <= f0 + p.c1 * at * d0 && ft < f0) || (have_best && ft >= f_best)) return;
    HIP_CHECK(hipMemcpyAsync(xb, xt, (size_t)o.n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
    HIP_CHECK(hipMemcpyAsync(gb, gt, (size_t)o.n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
    have_best = true;
    a_best = at;
    f_best = ft;
  };
  auto fallback = [&]() {
    if (!have_best) return false;
    HIP_CHECK(hipMemcpyAsync(xt, xb, (size_t)o.n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
    HIP_CHECK(hipMemcpyAsync(gt, gb, (size_t)o.n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
    a_out = a_best;
    f_out = f_best;
    return true;
  };
  while (used < p.max_ls) {
    HIP_CHECK(optk::launch_xpay(x, a, pdir, xt, o.n, o.dev.stream));
    double ft;
    o.evaluate(xt, &ft, gt);
    ++used;
    keep(a, ft);
    const double dt = o.dot(gt, pdir);
    if (ft > f0 + p.c1 * a * d0 || (used > 1 && ft >= f_prev)) {
      lo = a_prev; flo = f_prev; dlo = d_prev; hi = a; fhi = ft; dhi = dt;
      zoom = true;
      break;
    }
    if (std::fabs(dt) <= -p.c2 * d0) { a_out = a; f_out = ft; return true; }
    if (dt >= 0.0) {
      lo = a; flo = ft; dlo = dt; hi = a_prev; fhi = f_prev; dhi = d_prev;
      zoom = true;
      break;
    }
    a_prev = a; f_prev = ft; d_prev = dt;
    a = 2.0 * a;
  }
  if (!zoom) return fallback();
  while (used < p.max_ls) {
    a = cubic_step(lo, flo, dlo, hi, fhi, dhi);
    HIP_CHECK(optk::launch_xpay(x, a, pdir, xt, o.n, o.dev.stream));
    double ft;
    o.evaluate(xt, &ft, gt);
    ++used;
    keep(a, ft);
    const double dt = o.dot(gt, pdir);
    if (ft > f0 + p.c1 * a * d0 || ft >= flo) {
      hi = a; fhi = ft; dhi = dt;
    } else {
      if (std::fabs(dt) <= -p.c2 * d0) { a_out = a; f_out = ft; return true; }
      if (dt * (hi - lo) >= 0.0) { hi = lo; fhi = flo; dhi = dlo; }
      lo = a; flo = ft; dlo = dt;
    }
  }
  return fallback();
}

}  // namespace

extern "C" {

void ctm_lbfgs_default_params(ctm_lbfgs_params* p) {
  if (!p) return;
  p->max_iter = 100;
  p->history = 10;
  p->c1 = 1e-4;
  p->c2 = 0.9;
  p->gtol = 1e-6;
  p->max_ls = 20;
  p->alpha0 = 1.0;
  p->sur_start = 0;
  p->n_trials = 8;
  p->max_screened = 1;
  p->refit_every = 10;
  p->refit_steps = 200;
  p->lr = 1e-3f;
  p->n_blocks = 1;
  p->extrap = 2;
  p->window = 0;
}

int ctm_lbfgs(int64_t n, double* x_io, ctm_objective_fn fg, void* user, sur_net* sur, const ctm_lbfgs_params* params,
              void* stream, ctm_lbfgs_record* trace, int capacity, int* n_iter) {
  if (n < 1 || !x_io || !fg || !params) return CTM_EINVAL;
  const ctm_lbfgs_params& p = *params;
  if (p.history < 1 || p.max_ls < 1 || p.n_trials < 1 || p.n_trials > 64 || p.max_screened < 1 || p.extrap < 0 ||
      p.extrap > 30 || p.window < 0 ||
      p.refit_every < 1 || p.n_blocks < 1 || n % p.n_blocks != 0 || p.c1 <= 0 || p.c2 <= p.c1 || p.c2 >= 1)
    return CTM_EINVAL;
  int iters = 0;
  try {
    Opt o;
    o.dev.stream = (hipStream_t)stream;
    o.n = n;
    o.fg = fg;
    o.user = user;
    o.sur = p.sur_start > 0 ? sur : nullptr;
    o.p = p;
    o.scal = DBuf(&o.dev, 64);
    Vec x(&o.dev, n), g(&o.dev, n), pd(&o.dev, n), q(&o.dev, n), xt(&o.dev, n), gt(&o.dev, n), xb(&o.dev, n),
        gb(&o.dev, n);
    HIP_CHECK(hipMemcpyAsync(x.p(), x_io, (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
    std::vector<Vec> S, Y;
    std::vector<double> rho;
    S.reserve(p.history + 1);
    Y.reserve(p.history + 1);
    double f = 0;
    o.evaluate(x.p(), &f, g.p());
    bool trained = false, converged = false;
    const int nt = p.n_trials;
    // screening candidates: row 0 is the current point, rows 1..nt the trial points
    DBuf cand_x(&o.dev, (size_t)nt * n * 8), cand_f(&o.dev, (size_t)(nt + 1) * n * 4),
        cand_y(&o.dev, (size_t)(nt + 1) * 4);
    for (int k = 1; k <= p.max_iter; ++k) {
      const double gmax = o.absmax(g.p());
      if (!std::isfinite(gmax)) throw Error(CTM_ENONFINITE, "non-finite gradient at the current iterate");
      if (gmax < p.gtol) { converged = true; break; }
      // two-loop recursion
      HIP_CHECK(hipMemcpyAsync(q.p(), g.p(), (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
      const int h = (int)S.size();
      std::vector<double> al(h);
      for (int i = h - 1; i >= 0; --i) {
        al[i] = rho[i] * o.dot(S[i].p(), q.p());
        HIP_CHECK(optk::launch_axpby(-al[i], Y[i].p(), 1.0, q.p(), n, o.dev.stream));
      }
      const double gamma = h ? o.dot(S[h - 1].p(), Y[h - 1].p()) / o.dot(Y[h - 1].p(), Y[h - 1].p()) : 1.0;
      HIP_CHECK(optk::launch_axpby(0.0, q.p(), gamma, q.p(), n, o.dev.stream));   // r = gamma q (in q)
      for (int i = 0; i < h; ++i) {
        const double b = rho[i] * o.dot(Y[i].p(), q.p());
        HIP_CHECK(optk::launch_axpby(al[i] - b, S[i].p(), 1.0, q.p(), n, o.dev.stream));
      }
      HIP_CHECK(optk::launch_axpby(-1.0, q.p(), 0.0, pd.p(), n, o.dev.stream));   // pdir = -r
      double d0 = o.dot(g.p(), pd.p());
      if (d0 >= 0.0) {
        S.clear(); Y.clear(); rho.clear();
        HIP_CHECK(optk::launch_axpby(-1.0, g.p(), 0.0, pd.p(), n, o.dev.stream));
        d0 = -o.dot(g.p(), g.p());
      }
      const double a_init = S.empty() ? p.alpha0 / gmax : 1.0;
      bool accepted = false;
      int screened = 0;
      double a_acc = 0, f_acc = 0;
      if (o.sur && trained && k >= p.sur_start) {
        std::vector<double> as(nt);
        o.features(x.p(), (float*)cand_f.p);
        for (int j = 0; j < nt; ++j) {
          as[j] = a_init * std::ldexp(1.0, p.extrap - j);
          double* cx = (double*)cand_x.p + (size_t)j * n;
          HIP_CHECK(optk::launch_xpay(x.p(), as[j], pd.p(), cx, n, o.dev.stream));
          o.features(cx, (float*)cand_f.p + (size_t)(j + 1) * n);
        }
        int rc = sur_predict(o.sur, (const float*)cand_f.p, nt + 1, (float*)cand_y.p);
        if (rc != CTM_OK) throw Error(rc, std::string("surrogate: ") + sur_last_error(o.sur));
        std::vector<float> pred(nt + 1);
        HIP_CHECK(hipMemcpyAsync(pred.data(), cand_y.p, (size_t)(nt + 1) * 4, hipMemcpyDeviceToHost, o.dev.stream));
        HIP_CHECK(hipStreamSynchronize(o.dev.stream));
        std::vector<double> pc(nt);
        for (int j = 0; j < nt; ++j) pc[j] = f + ((double)pred[j + 1] - (double)pred[0]);
        std::vector<int> order(nt);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return pc[i] < pc[j]; });
        for (int c = 0; c < std::min(p.max_screened, nt); ++c) {
          const int j = order[c];
          if (!(pc[j] <= f + p.c1 * as[j] * d0)) break;
          HIP_CHECK(hipMemcpyAsync(xt.p(), (double*)cand_x.p + (size_t)j * n, (size_t)n * 8, hipMemcpyDeviceToDevice,
                                   o.dev.stream));
          double ft;
          o.evaluate(xt.p(), &ft, gt.p());
          const double dt = o.dot(gt.p(), pd.p());
          if (ft <= f + p.c1 * as[j] * d0 && std::fabs(dt) <= -p.c2 * d0) {
            accepted = true;
            screened = 1;
            a_acc = as[j];
            f_acc = ft;
            break;
          }
        }
      }
      if (!accepted) {
        if (!line_search(o, x.p(), f, pd.p(), d0, a_init, xt.p(), gt.p(), xb.p(), gb.p(), a_acc, f_acc)) {
          if (S.empty()) break;
          // a failed search along a quasi-Newton direction: forget the curvature
          // pairs and retry this iteration along -g
          S.clear(); Y.clear(); rho.clear();
          --k;
          continue;
        }
      }
      // s = xt - x, y = gt - g
      Vec s(&o.dev, n), y(&o.dev, n);
      HIP_CHECK(hipMemcpyAsync(s.p(), xt.p(), (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
      HIP_CHECK(optk::launch_axpby(-1.0, x.p(), 1.0, s.p(), n, o.dev.stream));
      HIP_CHECK(hipMemcpyAsync(y.p(), gt.p(), (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
      HIP_CHECK(optk::launch_axpby(-1.0, g.p(), 1.0, y.p(), n, o.dev.stream));
      const double sy = o.dot(s.p(), y.p());
      if (sy > 0.0) {
        S.push_back(std::move(s));
        Y.push_back(std::move(y));
        rho.push_back(1.0 / sy);
        if ((int)S.size() > p.history) {
          S.erase(S.begin());
          Y.erase(Y.begin());
          rho.erase(rho.begin());
        }
      }
      HIP_CHECK(hipMemcpyAsync(x.p(), xt.p(), (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
      HIP_CHECK(hipMemcpyAsync(g.p(), gt.p(), (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
      f = f_acc;
      iters = k;
      if (trace && k - 1 < capacity) {
        ctm_lbfgs_record& r = trace[k - 1];
        r.iter = k;
        r.evals = o.evals;
        r.screened = screened;
        r.f = f;
        r.gmax = o.absmax(g.p());
        r.step = a_acc;
      }
      if (o.sur && k >= p.sur_start - 1 && (k - (p.sur_start - 1)) % p.refit_every == 0) {
        float loss = 0;
        const int64_t use = p.window > 0 ? std::min<int64_t>(p.window, o.count) : o.count;
        int rc = sur_train(o.sur, (const float*)o.dX.p + (o.count - use) * n, (const float*)o.dF.p + (o.count - use),
                           (int)use, p.refit_steps, p.lr, &loss);
        if (rc != CTM_OK) throw Error(rc, std::string("surrogate: ") + sur_last_error(o.sur));
        trained = true;
      }
    }
    if (!converged && iters == p.max_iter) converged = o.absmax(g.p()) < p.gtol;
    HIP_CHECK(hipMemcpyAsync(x_io, x.p(), (size_t)n * 8, hipMemcpyDeviceToDevice, o.dev.stream));
    HIP_CHECK(hipStreamSynchronize(o.dev.stream));
    if (n_iter) *n_iter = iters;
    return converged ? CTM_OK : CTM_ENOTCONV;
  } catch (const Error& e) {
    g_opt_error = e.what();
    if (n_iter) *n_iter = iters;
    return e.code;
  }
}

int ctm_energy_objective_fn(void* user, const double* x, double* f, double* g) {
  ctm_energy_objective* ob = (ctm_energy_objective*)user;
  if (!ob || !ob->ctx) return CTM_EINVAL;
  int rc = ctm_set_tensors(ob->ctx, x);
  if (rc != CTM_OK) return rc;
  if (ob->conv_sweeps > 0) {
    int done = 0;
    double delta = 0;
    rc = ctm_sweep(ob->ctx, ob->conv_sweeps, ob->conv_tol, &done, &delta);
    if (rc < 0) return rc;
  }
  return ctm_energy_grad(ob->ctx, nullptr, ob->grad_sweeps, ob->H_bond, ob->n_terms, ob->terms, f, g);
}

const char* ctm_lbfgs_last_error(void) { return g_opt_error.c_str(); }

}  // extern "C"
