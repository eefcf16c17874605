// The factor object, the factor build and the sigma product.
#pragma once

#include "common.hpp"
#include "gemm.hpp"
#include "integrals.hpp"

#include <set>

struct risp_factors;

namespace risp {
struct Server;
// Per-atom partner lists of the kept shell pairs: the first transform G[P][i][mu] =
// sum_nu C[i][nu] (mu nu|P) only needs, for the functions mu of one atom, the functions nu that
// form a kept pair with one of that atom's shells (on the 1000-atom molecule 14.5 % of nao^2 instead
// of every nu), so it runs as one small dense product per atom over its partners; the AO-density
// Coulomb route contracts the integrals in the same packed layout.
struct Partners {
  int ngroups = 0;
  int64_t S = 0;   // elements of one auxiliary function in the packed layout: sum_g n_g kp_g
  std::vector<int> mu0, n, kp;
  std::vector<int64_t> voff, koff;  // per group: sum over earlier groups of n kp, of kp
  DevBuf idx;                       // [sum kp] partner functions, -1 = padding
  DevBuf gkoff, gkp;                // per group (device copies of koff, kp)
  DevBuf fvoff, fng, fkp, fml;      // per AO function: its group's voff, n, kp, and its index in the group
  DevBuf cab, cba;                  // per kept pair (device list order), see PackMap
  DevBuf prow, pcol;                // per packed position of one function: mu and nu (-1 = padding)
  // group-major chunk [group][f][mu][partner] for nf_stride functions
  PackMap map(int nf_stride) const {
    PackMap m;
    m.voff = fvoff.as<int64_t>();
    m.ng = fng.as<int>();
    m.kp = fkp.as<int>();
    m.ml = fml.as<int>();
    m.cab = cab.as<int>();
    m.cba = cba.as<int>();
    m.nf_stride = nf_stride;
    m.elems = (int64_t)nf_stride * S;
    return m;
  }
  // function-major chunk [f][group][mu][partner] (one contiguous row of S per function)
  PackMap map_fmajor(int nf) const {
    PackMap m = map(nf);
    m.f_stride = S;
    return m;
  }
};

// Event-timed launches of one sigma phase.
struct PhaseLog {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  int64_t launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};
}  // namespace risp

struct risp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  risp::DevBuf boys;                // Boys-function Taylor table
  void* scratch = nullptr;          // this device's copy of the library's fixed scratch array
  std::set<risp_factors*> factors;  // live factor objects (detached when the context goes away)
  bool profiling = false;
  risp::PhaseLog phase[RISP_NPHASE_SLOTS];
  // serving
  risp::Server* server = nullptr;
  hipStream_t serve_stream = nullptr;
  int64_t serve_budget = 0;
  int serve_max_active = 0;
  int serve_graphs = 1;
  void resolve_phases();  // fold pending events into ms (synchronises)
  void clear_phases();
};

namespace risp {
// Records HIP events around the launches issued during its lifetime when profiling is on.
class PhaseScope {
 public:
  PhaseScope(risp_ctx* c, hipStream_t s, int ph, double flops, double bytes);
  ~PhaseScope() noexcept(false);

 private:
  risp_ctx* c_;
  hipStream_t s_;
  int ph_;
  hipEvent_t a_ = nullptr;
};
}  // namespace risp

struct risp_factors {
  risp_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;  // stream of this object's work (the context stream, or a job stream)
  int nao = 0, nmo = 0, nocc = 0, nvir = 0;
  int naux_j = 0, naux_k = 0, nok = 0, nvk = 0, npair = 0;
  int64_t ld_ia = 0;     // row stride of T_ia (nocc*nvir padded to a multiple of 8)
  int nokp = 0, nvkp = 0;  // row strides of T_ij and T_ab (window sizes padded to multiples of 8)
  int precision = RISP_FP32;
  bool has_f32 = false;  // BF16 mode: the correction-pass operands below are kept
  risp::DevBuf t_ia, t_ij, t_ab;           // stored precision
  // BF16 mode, for the correction pass: FP32 copy of T_ia (Coulomb) and the BF16 rounding
  // remainders of T_ij and T_ab (exchange as three BF16 products, hi*hi + lo*hi + hi*lo)
  risp::DevBuf t_ia32, t_ij_lo, t_ab_lo;
  // full TDDFT-risp: the windowed exchange factor over (i, a) pairs in the stored precision (FP64 or
  // FP32), as Tx [naux_k][nocc_k][ld_ab] (b contiguous) and Txt [nvir_k][naux_k][ld_ij] ((P, j) contiguous)
  bool full = false;
  bool coul32 = false;  // BF16 mode: the Coulomb term of every sigma from t_ia32
  risp::DevBuf t_x, t_xt;
  risp::DevBuf scale_ia, scale_ia2, scale_k;  // BF16 power-of-two scales (s_P, s_P^2, s_ij s_ab)
  risp::DevBuf occ_k, vir_k, pos_o, pos_v; // window index sets and inverse maps
  risp::DevBuf de64, de32;                 // e_a - e_i
  // FP64 diagonal of A from the FP64 factors (Davidson guess and preconditioner): e_a - e_i
  // + 2 sum_P B_ia^2 - [window] sum_P Bx_ii Bx_aa (no Coulomb part on the AO route)
  risp::DevBuf diag64;
  // sigma workspaces, sized for ws_m trial vectors
  int ws_m = 0;
  int ws_csz = 0;  // bytes per element of the compute type the workspaces were sized for
  risp::DevBuf ws_y, ws_ybf, ws_xbf, ws_xw, ws_mt, ws_k, ws_split;
  // AO-density Coulomb route (RISP_J_AO_DIRECT): what regenerating (mu nu|P) needs, and workspaces
  int j_mode = RISP_J_MO;
  risp::DevShells ao_sh, auxj_sh;
  risp::PairList pairs;
  risp::Operator j_op;
  risp::DevBuf linv_j, co_t, cv_t;  // FP64 L^-1 of the Coulomb metric, C_occ^T [nocc][nao], C_vir^T
  risp::DevBuf co;                  // C_occ [nao][nocc] (FP64)
  std::vector<int> ao_s0, ao_f0;     // auxiliary shell / function start of each integral chunk (+ end)
  int ao_max_f = 0;                  // functions of the largest chunk
  int ao_mg = 0;                     // trial vectors per group (dense D_m / U_m slices)
  // workspaces: G [ao_mg][nao][nocc] / H [ao_mg][nocc][nao], D / U [ao_mg][nao][nao], packed (mu nu|P) chunk [f][S],
  // R and L^-1 R
  risp::DevBuf ws_ao_t, ws_ao_d, ws_ao_v, ws_ao_r;
  risp::Partners ao_partners;  // packed layout of the regenerated integrals
  risp::DevBuf ws_ao_p;        // D_m / U_m in the packed layout [ao_mg][S]
  double t_build = 0.0;  // seconds spent in the factor build
  int64_t bytes() const;
};

namespace risp {

// largest AO basis of the AO Coulomb route: one dense FP64 (mu nu|P) slice is at most 2 GiB

// precision of the sigma arithmetic: FP64 factors -> FP64, FP32 -> FP32, BF16 -> BF16 with FP32
// accumulation; `use_f32` selects the correction-pass arithmetic of BF16 factors: the Coulomb term
// from the FP32 copy of T_ia and the exchange from split BF16 operands (factor and vector each as
// hi + lo BF16 parts, three BF16 products per contraction, FP32 accumulation, the intermediate kept
// as hi + lo), about 2^-16 relative. x_bf16 (with use_f32): every element of X is a BF16 value, so
// the vector's lo part is zero and the first exchange contraction skips its (hi, lo) product.
void sigma(risp_factors* f, int m, const void* X, void* sig, bool use_f32, hipStream_t s, bool x_bf16 = false);

// sigma in the stored precision with every workspace taken from [scratch, scratch + cap): no
// allocation. Throws RISP_E_SHAPE when m vectors do not fit (sigma_scratch_need gives the bytes of
// the smallest layout, 0 when it fits). The stored-factor Coulomb route only.
void sigma_scratch(risp_factors* f, int m, const void* X, void* sig, void* scratch, size_t cap, hipStream_t s);
size_t sigma_scratch_need(const risp_factors* f, int m, size_t cap);

// Full TDDFT-risp products for m vectors V [m][nocc][nvir] (FP64 or FP32 factors built with
// full_tddft): P = (A + B) V = de V + 4 J V - KA V - KB V and M = (A - B) V = de V - KA V + KB V, where
// KA is the exchange term of A and KB V_ia = sum_(P, j, b) Tx_ib Tx_ja V_jb over the window.
void sigma_full(risp_factors* f, int m, const void* V, void* P, void* M, hipStream_t s);

// size the sigma workspaces for m vectors ahead of a graph capture (their allocation synchronises)
void sigma_prepare(risp_factors* f, int m, bool use_f32);

// algorithmic flops of one sigma block of m vectors
double sigma_flops(const risp_factors* f, int m);

// Builds on `stream` (the context stream when null); f->stream is set to it.
void build_factors(risp_ctx* ctx, const risp_system* sys, const risp_params* prm, risp_factors* f,
                   hipStream_t stream = nullptr);

void validate_system(const risp_system* sys);
void select_aux(const risp_system* sys, const risp_params* prm, std::vector<risp_shell>& J,
                std::vector<risp_shell>& K);

}  // namespace risp
