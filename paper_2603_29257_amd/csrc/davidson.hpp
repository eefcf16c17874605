// Block Davidson on the device.
#pragma once

#include <functional>
#include <vector>

#include "factors.hpp"

namespace risp {

// sigma_fn(m, X_dev, S_dev): S = A X for m rows stored in the trial-vector type (FP64 for FP64
// factors, FP32 otherwise). Must be stream-ordered on the context stream.
using SigmaFn = std::function<void(int m, const void* X, void* S)>;

struct DavOptions {
  int nstates = 5;
  int block = 0;
  int max_space = 0;
  int max_iter = 200;
  double tol = 1e-5;
  const double* x0_dev = nullptr;  // optional initial vectors [nx0][ov] FP64 on the device
  int nx0 = 0;
  // stop early when the largest residual has not dropped below 0.7 of its best value for this many
  // iterations (0: never); used for the BF16 stage, whose products limit the attainable residual
  int stall_iters = 0;
};

struct DavResult {
  std::vector<double> energies;  // [nstates]
  DevBuf X;                      // [k][ov] FP64 Ritz vectors of the last iteration (k = krows)
  int krows = 0;
  int iters = 0, restarts = 0, sigma_vectors = 0;
  bool converged = false;
  bool stalled = false;
  double t_sigma = 0.0, t_subspace = 0.0, sigma_flops = 0.0;
  std::vector<double> resid_hist;  // max residual over the nstates per iteration
};

void davidson(risp_factors* f, const DavOptions& o, const SigmaFn& sigma_fn, DavResult& res);

}  // namespace risp
