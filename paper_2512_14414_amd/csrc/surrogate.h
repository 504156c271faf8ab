// Internal interface of the surrogate network (surrogate.cpp) shared with the
// allocation-free entry point (sur_noalloc.hip).  Not part of the C ABI.
#pragma once
#include <string>

#include "engine.h"

struct sur_net {
  ctm::Dev dev;
  int n_in = 0, width = 0;
  int64_t np = 0;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  ctm::DBuf params, stats;
  std::string err;
  float* P(int64_t off) { return (float*)params.p + off; }
};

namespace ctm {

// Forward pass of ``batch`` inputs and the de-standardised predictions in y
// (the body of sur_predict); its workspaces come from s->dev.
void sur_predict_impl(sur_net* s, const float* X, int64_t batch, float* y);
// Device bytes the workspaces of sur_predict_impl take, each rounded up to
// 256 bytes, for a network of n_in inputs and width ``width``.
int64_t sur_predict_workspace_bytes(int64_t n_in, int64_t width, int64_t batch);
// Resolves the allocation-free entry point's scratch on the current device
// (sur_noalloc.hip); called by sur_init.  Returns a HIP status.
int sur_scratch_setup();

}  // namespace ctm
