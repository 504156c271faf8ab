// Learned line-search surrogate: a two-hidden-layer GELU perceptron in
// float32 whose matrix products run on the MFMA contraction kernel and whose
// elementwise steps, loss and Adam update are the kernels of opt_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/ctm_opt.h"
#include "engine.h"
#include "opt_kernels.h"
#include "surrogate.h"

using namespace ctm;

namespace {

thread_local std::string g_sur_error;

struct Acts {
  DBuf Z1, A1, Z2, A2, y;
};

TRef f32(void* p, const std::vector<int64_t>& d, const std::string& lab) { return view(p, T_F32, d, lab); }

void forward(sur_net* s, const float* X, int64_t B, Acts& a) {
  Dev& dev = s->dev;
  const int64_t w = s->width, n = s->n_in;
  const int m = ctmk::MODE_F32;
  a.Z1 = DBuf(&dev, (size_t)B * w * 4);
  a.A1 = DBuf(&dev, (size_t)B * w * 4);
  a.Z2 = DBuf(&dev, (size_t)B * w * 4);
  a.A2 = DBuf(&dev, (size_t)B * w * 4);
  a.y = DBuf(&dev, (size_t)B * 4);
  contract(dev, m, f32(a.Z1.p, {B, w}, "bw"), f32((void*)X, {B, n}, "bi"), f32(s->P(s->oW1), {w, n}, "wi"));
  HIP_CHECK(optk::launch_bias_act((float*)a.Z1.p, s->P(s->ob1), (float*)a.A1.p, B, w, dev.stream));
  contract(dev, m, f32(a.Z2.p, {B, w}, "bv"), f32(a.A1.p, {B, w}, "bw"), f32(s->P(s->oW2), {w, w}, "vw"));
  HIP_CHECK(optk::launch_bias_act((float*)a.Z2.p, s->P(s->ob2), (float*)a.A2.p, B, w, dev.stream));
  contract(dev, m, f32(a.y.p, {B}, "b"), f32(a.A2.p, {B, w}, "bw"), f32(s->P(s->oW3), {w}, "w"));
  HIP_CHECK(optk::launch_bias_act((float*)a.y.p, s->P(s->ob3), nullptr, B, 1, dev.stream));
}

// Gradient of the loss with respect to all parameters, from dy = dL/dy.
void backward(sur_net* s, const float* X, int64_t B, const Acts& a, const float* dy, float* g) {
  Dev& dev = s->dev;
  const int64_t w = s->width, n = s->n_in;
  const int m = ctmk::MODE_F32;
  contract(dev, m, f32(g + s->oW3, {w}, "w"), f32((void*)dy, {B}, "b"), f32(a.A2.p, {B, w}, "bw"));
  HIP_CHECK(optk::launch_colsum(dy, B, 1, g + s->ob3, dev.stream));
  DBuf dA(&dev, (size_t)B * w * 4), dZ(&dev, (size_t)B * w * 4);
  contract(dev, m, f32(dA.p, {B, w}, "bw"), f32((void*)dy, {B}, "b"), f32(s->P(s->oW3), {w}, "w"));
  HIP_CHECK(optk::launch_gelu_backward((const float*)a.Z2.p, (const float*)dA.p, (float*)dZ.p, B * w, dev.stream));
  contract(dev, m, f32(g + s->oW2, {w, w}, "vw"), f32(dZ.p, {B, w}, "bv"), f32(a.A1.p, {B, w}, "bw"));
  HIP_CHECK(optk::launch_colsum((const float*)dZ.p, B, w, g + s->ob2, dev.stream));
  contract(dev, m, f32(dA.p, {B, w}, "bw"), f32(dZ.p, {B, w}, "bv"), f32(s->P(s->oW2), {w, w}, "vw"));
  HIP_CHECK(optk::launch_gelu_backward((const float*)a.Z1.p, (const float*)dA.p, (float*)dZ.p, B * w, dev.stream));
  contract(dev, m, f32(g + s->oW1, {w, n}, "wi"), f32(dZ.p, {B, w}, "bw"), f32((void*)X, {B, n}, "bi"));
  HIP_CHECK(optk::launch_colsum((const float*)dZ.p, B, w, g + s->ob1, dev.stream));
}

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

int sfail(sur_net* s, const Error& e) {
  if (s) s->err = e.what();
  else g_sur_error = e.what();
  return e.code;
}

}  // namespace

namespace ctm {

void sur_predict_impl(sur_net* s, const float* X, int64_t batch, float* y) {
  Acts a;
  forward(s, X, batch, a);
  HIP_CHECK(hipMemcpyAsync(y, a.y.p, (size_t)batch * 4, hipMemcpyDeviceToDevice, s->dev.stream));
  HIP_CHECK(optk::launch_destandardize(y, (int)batch, (const float*)s->stats.p, s->dev.stream));
}

// The blocks forward() takes, in its order: Z1, A1, the partials of
// X W1^T, Z2, A2, those of A1 W2^T, y, those of A2 W3.
int64_t sur_predict_workspace_bytes(int64_t n_in, int64_t width, int64_t batch) {
  const int64_t act = round256(batch * width * 4);
  return 4 * act + round256(batch * 4) + round256(split_workspace_bytes(batch, width, n_in, 1, 4)) +
         round256(split_workspace_bytes(batch, width, width, 1, 4)) +
         round256(split_workspace_bytes(batch, 1, width, 1, 4));
}

}  // namespace ctm

extern "C" {

int sur_init(sur_net** out, int n_in, int width, uint64_t seed, void* stream) {
  if (!out) return CTM_EINVAL;
  *out = nullptr;
  sur_net* s = nullptr;
  try {
    if (n_in < 1 || width < 1) throw Error(CTM_EINVAL, "n_in and width must be positive");
    s = new sur_net();
    s->dev.stream = (hipStream_t)stream;
    s->n_in = n_in;
    s->width = width;
    const int64_t n = n_in, w = width;
    s->oW1 = 0;
    s->ob1 = s->oW1 + w * n;
    s->oW2 = s->ob1 + w;
    s->ob2 = s->oW2 + w * w;
    s->oW3 = s->ob2 + w;
    s->ob3 = s->oW3 + w;
    s->np = s->ob3 + 1;
    s->params = DBuf(&s->dev, (size_t)s->np * 4);
    s->stats = DBuf(&s->dev, 8);
    const int64_t off[7] = {s->oW1, s->ob1, s->oW2, s->ob2, s->oW3, s->ob3, s->np};
    const double fan[6] = {(double)n, (double)n, (double)w, (double)w, (double)w, (double)w};
    for (int k = 0; k < 6; ++k)
      HIP_CHECK(optk::launch_uniform_init(s->P(off[k]), off[k + 1] - off[k], seed, off[k], 1.0 / std::sqrt(fan[k]),
                                          s->dev.stream));
    float st[2] = {0.0f, 1.0f};
    HIP_CHECK(hipMemcpyAsync(s->stats.p, st, 8, hipMemcpyHostToDevice, s->dev.stream));
    HIP_CHECK(hipStreamSynchronize(s->dev.stream));
    // the scratch of sur_predict_noalloc on this device
    HIP_CHECK((hipError_t)sur_scratch_setup());
    *out = s;
    return CTM_OK;
  } catch (const Error& e) {
    g_sur_error = e.what();
    delete s;
    return e.code;
  }
}

int64_t sur_param_count(const sur_net* s) { return s ? s->np : 0; }

int sur_get_params(sur_net* s, float* params) {
  if (!s || !params) return CTM_EINVAL;
  try {
    HIP_CHECK(hipMemcpyAsync(params, s->params.p, (size_t)s->np * 4, hipMemcpyDeviceToDevice, s->dev.stream));
    HIP_CHECK(hipStreamSynchronize(s->dev.stream));
    return CTM_OK;
  } catch (const Error& e) { return sfail(s, e); }
}

int sur_set_params(sur_net* s, const float* params) {
  if (!s || !params) return CTM_EINVAL;
  try {
    HIP_CHECK(hipMemcpyAsync(s->params.p, params, (size_t)s->np * 4, hipMemcpyDeviceToDevice, s->dev.stream));
    return CTM_OK;
  } catch (const Error& e) { return sfail(s, e); }
}

int sur_predict(sur_net* s, const float* X, int batch, float* y) {
  if (!s || !X || !y || batch < 1) return CTM_EINVAL;
  try {
    sur_predict_impl(s, X, batch, y);
    return CTM_OK;
  } catch (const Error& e) { return sfail(s, e); }
}

int sur_loss_grad(sur_net* s, const float* X, const float* t, int n, float* loss, float* grad) {
  if (!s || !X || !t || !grad || n < 1) return CTM_EINVAL;
  try {
    Acts a;
    forward(s, X, n, a);
    DBuf dy(&s->dev, (size_t)n * 4), l(&s->dev, 8);
    HIP_CHECK(optk::launch_mse((const float*)a.y.p, t, n, nullptr, (float*)dy.p, (float*)l.p, s->dev.stream));
    backward(s, X, n, a, (const float*)dy.p, grad);
    if (loss) HIP_CHECK(hipMemcpyAsync(loss, l.p, 4, hipMemcpyDeviceToHost, s->dev.stream));
    HIP_CHECK(hipStreamSynchronize(s->dev.stream));
    return CTM_OK;
  } catch (const Error& e) { return sfail(s, e); }
}

int sur_train(sur_net* s, const float* X, const float* t, int n, int steps, float lr, float* loss) {
  if (!s || !X || !t || n < 1 || steps < 0) return CTM_EINVAL;
  try {
    Dev& dev = s->dev;
    HIP_CHECK(optk::launch_mean_std(t, n, (float*)s->stats.p, dev.stream));
    DBuf g(&dev, (size_t)s->np * 4), m(&dev, (size_t)s->np * 4), v(&dev, (size_t)s->np * 4), dy(&dev, (size_t)n * 4),
        l(&dev, 8);
    fill(dev, view(m.p, T_F32, {s->np}, "q"), 0.0);
    fill(dev, view(v.p, T_F32, {s->np}, "q"), 0.0);
    for (int k = 1; k <= steps; ++k) {
      Acts a;
      forward(s, X, n, a);
      HIP_CHECK(optk::launch_mse((const float*)a.y.p, t, n, (const float*)s->stats.p, (float*)dy.p, (float*)l.p,
                                 dev.stream));
      backward(s, X, n, a, (const float*)dy.p, (float*)g.p);
      HIP_CHECK(optk::launch_adam((float*)s->params.p, (const float*)g.p, (float*)m.p, (float*)v.p, s->np, lr, 0.9f,
                                  0.999f, 1e-8f, k, dev.stream));
    }
    if (loss) {
      *loss = 0.0f;
      if (steps > 0) HIP_CHECK(hipMemcpyAsync(loss, l.p, 4, hipMemcpyDeviceToHost, dev.stream));
    }
    HIP_CHECK(hipStreamSynchronize(dev.stream));
    return CTM_OK;
  } catch (const Error& e) { return sfail(s, e); }
}

const char* sur_last_error(const sur_net* s) { return s ? s->err.c_str() : g_sur_error.c_str(); }

void sur_free(sur_net* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->dev.stream);
  s->params.reset();
  s->stats.reset();
  s->dev.release();
  (void)hipStreamSynchronize(s->dev.stream);
  delete s;
}

}  // extern "C"
