// Block Davidson on the device.
#pragma once

#include <chrono>
#include <functional>
#include <vector>

#include "factors.hpp"

namespace risp {

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double sec() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

// sigma_fn(m, X_dev, S_dev): S = A X for m rows stored in the trial-vector type (FP64 for FP64
// factors, FP32 otherwise). Must be stream-ordered on the context stream.
using SigmaFn = std::function<void(int m, const void* X, void* S)>;

// default tolerance of the BF16 stage before the correction pass of BF16 factors
constexpr double kBf16StageTol = 1e-3;

struct DavOptions {
  int nstates = 5;
  int block = 0;
  int max_space = 0;
  int max_iter = 200;
  double tol = 1e-5;
  const double* x0_dev = nullptr;  // optional initial vectors [nx0][ov] FP64 on the device
  int nx0 = 0;
  // stop early when the largest residual has not dropped below 0.9 of its best value for this many
  // iterations (0: never) once that best value is at most stall_below; used for the BF16 stage,
  // whose products limit the attainable residual (slow progress far above that floor is not a stall)
  int stall_iters = 0;
  double stall_below = 1e300;
  const char* log_tag = nullptr;  // print one line per iteration to stderr under this tag
  int max_corr = 0;  // corrections only for the lowest max_corr Ritz pairs (0: all `block`)
  bool spill = false;  // subspace vectors V and products W in pinned host memory
  // Olsen's correction t = (D - theta)^-1 (r - eps x) with eps such that t is orthogonal to x (D the
  // diagonal of A); false: t = (D - theta)^-1 r
  bool olsen = false;
  // rows stored for a product are rounded to BF16 values (FP32 trial vectors only), so split-BF16
  // products can skip the vector's lo half; the basis is then orthonormal only to about 2^-9 and the
  // Rayleigh-Ritz solves H c = theta S c with the projected overlap S = V^T V
  bool bf16_basis = false;
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

// One Davidson solve as a resumable state machine: next() names the sigma block it needs (rows of
// V to multiply into the same rows of W), complete() consumes it and advances. Everything except
// the sigma products runs inside complete() on the run's stream.
class DavidsonRun {
 public:
  struct Request {
    int r0 = 0, n = 0;
    void* X = nullptr;  // device rows of V
    void* S = nullptr;  // device rows of W to fill
  };
  DavidsonRun(risp_factors* f, const DavOptions& o, hipStream_t s);
  bool next(Request& rq) const;  // false when finished
  void complete();
  bool done() const { return state_ == State::Done; }
  bool bf16_basis() const { return o_.bf16_basis; }
  DavResult& result() { return res_; }

 private:
  enum class State { Init, Append, Done };
  void* vrow(DevBuf& b, int r);
  void update_H(int nall, int n0, int nn);
  void update_S(int nall, int n0, int nn);
  void generalized_eig(int kk);
  void row_norms(const double* R, int k, double* out_dev);
  void combine_rows(const double* Cm, int ldcm, int nsub, int k, const void* Vsrc, double* out, double alpha,
                    double beta);
  int orth_block(int nt, bool unit_ref);
  void project_out(int nsub, int nt);
  void store_T(int r0, int n);
  void iterate(Timer& tsub);
  void append_corrections(int nt, Timer& tsub);
  void finish(Timer& tsub);
  void thick_restart(int keep);

  risp_factors* f_;
  DavOptions o_;
  hipStream_t s_;
  int64_t ov_ = 0;
  bool fp64_ = false;
  DType tvec_ = DType::F32;
  size_t vsz_ = 4;
  int nstates_ = 0, block_ = 0, max_space_ = 0, cap_ = 0, ld_ = 0, max_iter_ = 0, nblk_ = 1;
  int nsub_ = 0, best_it_ = 0;
  double best_r_ = 1e300;
  double drop_ = 1e-6;
  State state_ = State::Init;
  Request rq_;
  DavResult res_;
  std::vector<double> hnorm_, htheta_;
  DevBuf V_, W_, H_, Hw_, Zs_, eigws_, theta_, AX_, T_, T2_, Cmix_, G_, Cf_, partial_, norms_, eps_, kept_,
      src_, Hn_, split_, Rv_, Rw_;
  DevBuf S_, Ls_, Li_, T1_, Y_;  // bf16_basis: overlap, its Cholesky factor and inverse, products
};

void davidson(risp_factors* f, const DavOptions& o, const SigmaFn& sigma_fn, DavResult& res);

// Full TDDFT-risp (eq. tddft with eq. hessian): the lowest nstates excitation energies and X + Y,
// X - Y by a Davidson-like solver on one subspace V for both (A + B) and (A - B) (section on
// Davidson settings): with Pm = V^T (A + B) V and Mm = V^T (A - B) V (FP64) and Mm = L L^T, the
// symmetric problem L^T Pm L c = Omega^2 c gives X + Y = V L c / sqrt(Omega) and
// X - Y = V L^-T c sqrt(Omega); residuals (A + B)(X + Y) - Omega (X - Y) and
// (A - B)(X - Y) - Omega (X + Y); both preconditioned by 1/(Omega - diag A) and added to V.
struct FullResult {
  std::vector<double> omega;  // [nstates]
  DevBuf XpY, XmY;            // [nstates][ov] FP64
  int iters = 0, restarts = 0, sigma_vectors = 0;
  bool converged = false;
  double t_sigma = 0.0, t_subspace = 0.0, sigma_flops = 0.0;
  std::vector<double> resid_hist;  // max residual over the states per iteration
};
void davidson_full(risp_factors* f, const DavOptions& o, FullResult& res);

}  // namespace risp
