// Proposal network state (csrc/nullnet.hip).
#pragma once

#include "mg_internal.h"

struct mgdwf_ctx;

namespace mgdwf {

struct NullNet {
  int ch[5];         // channels: input, three hidden, output (= 4 x proposals)
  double lam = 1.0;  // weight of the Gram (anti-collapse) term
  DevBuf w, wb, m, v, g;  // FP32 master weights, BF16 copy, Adam moments, gradient
  long long step = 0;
  long long nweights() const;
  long long woff(int layer) const;
  void init(unsigned long long seed);
  void set_weights(const float* host, hipStream_t st);
};

void net_propose(NullNet& net, mgdwf_ctx* c, const double2* eta, double2* V_canon);
double net_grad(NullNet& net, mgdwf_ctx* c, const double2* eta);
double net_train_step(NullNet& net, mgdwf_ctx* c, const double2* eta, double lr);

}  // namespace mgdwf
