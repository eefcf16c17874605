// Obara-Saika integral kernels (FP64, gfx950) and the shell/pair data they read.
#pragma once

#include "common.hpp"

namespace risp {

// Boys-function table for Taylor interpolation: F_n(T_g) for n < kBoysCols at T_g = g * kBoysDT.
constexpr int kBoysCols = 13;       // orders 0..12: F_m for m <= 4 plus 8 Taylor terms
constexpr double kBoysDT = 0.1;
constexpr double kBoysTMax = 40.0;  // above: asymptotic F_0 and upward recursion
constexpr int kBoysRows = 402;
void boys_table_host(std::vector<double>& tab);  // kBoysRows * kBoysCols values

// Device-resident shells (SoA). cn = coef * normalisation of the primitive (per Cartesian
// component; the same for the three p components).
struct DevShells {
  int n = 0;
  int nfunc = 0;
  DevBuf x, y, z, ex, cn;  // double [n]
  DevBuf l, off, atom;     // int [n]
};
void upload_shells(DevShells& d, const double* coords, const risp_shell* sh, int n, hipStream_t s);
int shell_functions(const risp_shell* sh, int n);

// Range-separated operator coefficients: alpha / r + beta erf(omega r) / r.
struct Operator {
  double alpha = 1.0, beta = 0.0, omega = 0.0;
};

// Screened shell pairs, grouped by class (s s), (p s), (p p); within a class ascending (A, B) with
// A >= B in the original numbering, stored with the p shell first for the (p s) class.
struct PairList {
  int n = 0;
  int cls_begin[4] = {0, 0, 0, 0};  // class c occupies [cls_begin[c], cls_begin[c+1])
  DevBuf a, b;                      // int [n]
};

// Kept pairs on the device. If `canonical`, one group in ascending (A, B) order (cls_begin[1..3] = n).
void screen_pairs(const DevShells& ao, double qaux, double tau, bool canonical, PairList& out,
                  hipStream_t s);

// max_P (P|P) over the auxiliary functions (FP64, returned to the host).
double aux_diag_max(const DevShells& aux, const double* boys_tab, hipStream_t s);

// (P|Q) with the given operator: out dev [naux][naux].
void int2c(const DevShells& aux, const Operator& op, const double* boys_tab, double* out,
           hipStream_t s);

// Packed output of int3c over per-atom partner lists. AO functions fall into groups (runs of
// consecutive shells on one atom); group g owns functions [mu0_g, mu0_g + n_g) and a sorted list of
// partner functions (every function of a shell that forms a kept pair with a shell of the group),
// padded with zeros to kp_g entries. The chunk is stored group after group, each group as
// [f][mu - mu0_g][position of nu in its list] for the nf_stride auxiliary functions f of the chunk:
// element (f, mu, nu) lives at nf_stride * voff[mu] + (f * ng[mu] + ml[mu]) * kp[mu] + pos(nu).
// pos(nu) for a kept pair (A, B) (the pair list's own order and orientation) is cab[pair] + (nu -
// first function of B) when mu is a function of A, and cba[pair] + (nu - first function of A) in
// the mirrored position.
struct PackMap {
  const int64_t* voff = nullptr;  // [nao] elements per auxiliary function before the group of mu
  const int* ng = nullptr;        // [nao] functions of the group of mu
  const int* kp = nullptr;        // [nao] padded partner count of the group of mu
  const int* ml = nullptr;        // [nao] mu - mu0 of its group
  const int* cab = nullptr;       // [npair] list position of B's first function in A's group
  const int* cba = nullptr;       // [npair] list position of A's first function in B's group
  int nf_stride = 0;
  int64_t elems = 0;              // elements of one chunk (nf_stride * sum_g n_g kp_g)
  // > 0: function-major instead, element (f, mu, nu) at f * f_stride + voff[mu] + ml[mu] * kp[mu] +
  // pos(nu) (f_stride = sum_g n_g kp_g: one contiguous row per auxiliary function)
  int64_t f_stride = 0;
};

// (mu nu|P) with the given operator for auxiliary shells [s0, s1): out dev
// [nf][nao][nao] (nf = functions of those shells), zeroed first; or, with pack, the packed layout
// above (zeroed first; nf must not exceed pack->nf_stride).
void int3c(const DevShells& ao, const PairList& pairs, const DevShells& aux, int s0, int s1,
           const Operator& op, const double* boys_tab, double* out, hipStream_t s,
           const PackMap* pack = nullptr);

// Window predicate on the device: flags[k] = 1 for kept orbitals; counts via compaction.
void window_sets(const double* mo_energy_dev, int nmo, int nocc, double window_ev, int mode,
                 int* occ_out, int* nocc_k, int* vir_out, int* nvir_k, hipStream_t s);

}  // namespace risp
