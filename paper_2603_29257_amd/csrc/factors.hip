// Factor build (auxiliary basis, window, screening, metric Cholesky, 3-centre integrals, MO
// transforms, metric application, storage precision) and the sigma product A X.
#include <algorithm>
#include <cmath>
#include <optional>

#include "coulomb.hpp"
#include "factors.hpp"
#include "linalg.hpp"

static size_t shell_bytes(const risp::DevShells& d) {
  return d.x.bytes() + d.y.bytes() + d.z.bytes() + d.ex.bytes() + d.cn.bytes() + d.l.bytes() + d.off.bytes() +
         d.atom.bytes();
}

int64_t risp_factors::bytes() const {
  return (int64_t)(t_ia.bytes() + t_ij.bytes() + t_ab.bytes() + t_ia32.bytes() + t_ij_lo.bytes() +
                   t_ab_lo.bytes() + scale_ia.bytes() + scale_ia2.bytes() + scale_k.bytes() + occ_k.bytes() +
                   vir_k.bytes() + pos_o.bytes() + pos_v.bytes() + de64.bytes() + de32.bytes() + diag64.bytes() +
                   ws_y.bytes() + ws_ybf.bytes() + ws_xbf.bytes() + ws_xw.bytes() + ws_mt.bytes() +
                   ws_k.bytes() + ws_split.bytes() + shell_bytes(ao_sh) + shell_bytes(auxj_sh) + pairs.a.bytes() +
                   pairs.b.bytes() + linv_j.bytes() + co_t.bytes() + cv_t.bytes() + co.bytes() + ws_ao_t.bytes() +
                   ws_ao_d.bytes() + ws_ao_v.bytes() + ws_ao_r.bytes() + ws_ao_p.bytes());
}

void risp_ctx::resolve_phases() {
  for (auto& p : phase) {
    for (auto& ev : p.pending) {
      float ms = 0.f;
      RISP_HIP(hipEventSynchronize(ev.second));
      RISP_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
      p.ms += ms;
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
    p.pending.clear();
  }
}

void risp_ctx::clear_phases() {
  resolve_phases();
  for (auto& p : phase) p = risp::PhaseLog();
}

namespace risp {

PhaseScope::PhaseScope(risp_ctx* c, hipStream_t s, int ph, double flops, double bytes) : c_(c), s_(s), ph_(ph) {
  if (!c_->profiling) return;
  RISP_HIP(hipEventCreate(&a_));
  RISP_HIP(hipEventRecord(a_, s_));
  PhaseLog& p = c_->phase[ph_];
  p.launches += 1;
  p.flops += flops;
  p.bytes += bytes;
}

PhaseScope::~PhaseScope() noexcept(false) {
  if (!a_) return;
  hipEvent_t b = nullptr;
  RISP_HIP(hipEventCreate(&b));
  RISP_HIP(hipEventRecord(b, s_));
  c_->phase[ph_].pending.emplace_back(a_, b);
}

void validate_system(const risp_system* sys) {
  RISP_CHECK(sys != nullptr, RISP_E_ARG, "system is NULL");
  RISP_CHECK(sys->natm > 0 && sys->coords && sys->Z && sys->aux_radius, RISP_E_ARG,
             "system: atoms, coordinates, charges and radii are required");
  RISP_CHECK(sys->nshell > 0 && sys->shells, RISP_E_ARG, "system: AO shells are required");
  RISP_CHECK(sys->mo_coeff && sys->mo_energy, RISP_E_ARG, "system: MO coefficients and energies are required");
  int nf = 0;
  for (int k = 0; k < sys->nshell; ++k) {
    const risp_shell& s = sys->shells[k];
    RISP_CHECK(s.l == 0 || s.l == 1, RISP_E_ARG, "only s and p shells are supported");
    RISP_CHECK(s.atom >= 0 && s.atom < sys->natm, RISP_E_ARG, "shell atom index out of range");
    RISP_CHECK(s.exponent > 0.0 && std::isfinite(s.exponent), RISP_E_ARG, "shell exponent must be positive");
    nf += s.l == 0 ? 1 : 3;
  }
  RISP_CHECK(nf == sys->nao, RISP_E_SHAPE, "nao does not match the shells");
  RISP_CHECK(sys->nmo > 0 && sys->nmo <= sys->nao, RISP_E_SHAPE, "need 0 < nmo <= nao");
  RISP_CHECK(sys->nocc > 0 && sys->nocc < sys->nmo, RISP_E_SHAPE, "need 0 < nocc < nmo");
  for (int a = 0; a < sys->natm; ++a)
    RISP_CHECK(sys->aux_radius[a] > 0.0, RISP_E_ARG, "auxiliary radius must be positive");
}

void select_aux(const risp_system* sys, const risp_params* prm, std::vector<risp_shell>& J,
                std::vector<risp_shell>& K) {
  J.clear();
  K.clear();
  for (int a = 0; a < sys->natm; ++a) {
    if (sys->Z[a] == 1 && !prm->h_in_aux) continue;
    const double r = sys->aux_radius[a];
    const double e = prm->theta / (r * r);
    J.push_back({a, 0, e, 1.0});
    J.push_back({a, 1, e, 1.0});
    K.push_back({a, 0, e, 1.0});
  }
}

// Non-owning view of device memory: a sigma workspace (a DevBuf of the factor object, or a piece of
// a fixed scratch buffer) or a piece of the build's arena.
struct WsView {
  void* p = nullptr;
  size_t n = 0;
  void* get() const { return p; }
  template <typename T> T* as() const { return static_cast<T*>(p); }
  size_t bytes() const { return n; }
};

// One device allocation that the build's large temporaries are carved from (bump allocation,
// released back to a mark). Device memory that was used and then freed is cleared by the driver
// before it is handed out again (measured at tens of GB/s), so freeing and reallocating large
// temporaries between the build's phases costs seconds on the large molecules; the arena is
// allocated once.
class Arena {
 public:
  static size_t round(size_t b) { return (b + 255) / 256 * 256; }
  void reserve(size_t bytes) {
    buf_.alloc(std::max<size_t>(bytes, 256));
    off_ = 0;
  }
  WsView take(size_t bytes) {
    const size_t b = round(std::max<size_t>(bytes, 1));
    RISP_CHECK(off_ + b <= buf_.bytes(), RISP_E_STATE, "build arena exhausted");
    WsView v{static_cast<char*>(buf_.get()) + off_, b};
    off_ += b;
    return v;
  }
  size_t mark() const { return off_; }
  void release_to(size_t m) { off_ = m; }

 private:
  DevBuf buf_;
  size_t off_ = 0;
};

static Gemm g64(int M, int N, int K) {
  Gemm g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.tin = g.tout = DType::F64;
  return g;
}

constexpr int64_t kIntChunk = 16ll << 30;    // bytes of one chunk of dense (mu nu|P) slices in the build

// T <- Linv T in place for T [n][cols] (row stride cols), through column panels of at most ~1 GiB
// (tmp holds one panel, two for long contractions: metric_panel_bytes)
static int64_t metric_panel_cols(int n, int64_t cols) {
  return std::max<int64_t>(8, std::min<int64_t>(cols, ((1ll << 30) / (8 * (int64_t)std::max(n, 1))) / 8 * 8));
}
// auxiliary functions from which the panel product writes a contiguous transposed result (measured
// on the 1000-atom build: 2400 functions 8.3 against 10.2 ms per panel with the transposes; 600
// functions 3.7 against 2.5 ms, where the in-place form's row tiles of 128 fit L^-1 better)
constexpr int kMetricTransposedFrom = 1536;
static size_t metric_panel_bytes(int n, int64_t cols) {
  const size_t one = Arena::round((size_t)std::max(n, 1) * metric_panel_cols(n, cols) * 8);
  return n >= kMetricTransposedFrom ? 2 * one : one;
}
static void metric_apply_inplace(const double* Linv, int n, double* T, int64_t cols, const WsView& tmp, hipStream_t s) {
  if (n == 0 || cols == 0) return;
  const int64_t w = metric_panel_cols(n, cols);
  const size_t one = Arena::round((size_t)n * w * 8);
  const bool tr = n >= kMetricTransposedFrom;
  RISP_CHECK(tmp.bytes() >= (tr ? 2 : 1) * one, RISP_E_STATE, "metric panel buffer too small");
  double* Pt = tmp.as<double>();  // panel^T [col][Q]
  double* Bt = tr ? reinterpret_cast<double*>(static_cast<char*>(tmp.get()) + one) : nullptr;  // result^T [col][P]
  // each panel transposed to [col][Q] (contraction-contiguous), then on the NT MFMA kernel either
  // T[:, panel] = L^-1 panel straight into T, or (tr) result^T = panel^T L^-T into a contiguous
  // buffer that is transposed back into T; L^-1 is lower triangular, so each output tile stops its
  // contraction at its last auxiliary function. An odd n (no 16-byte contraction rows) keeps the
  // generic form.
  Gemm nt = tr ? g64((int)std::min<int64_t>(w, cols), n, n) : g64(n, (int)std::min<int64_t>(w, cols), n);
  nt.A = tr ? Pt : Linv;
  nt.lda = n;
  nt.B = tr ? Linv : Pt;
  nt.ldb = n;
  nt.a_lower = !tr;
  nt.b_lower = tr;
  nt.C = tr ? Bt : T;
  nt.ldc = tr ? n : cols;
  const bool use_nt = gemm_bf16_nt_eligible(nt);
  for (int64_t c0 = 0; c0 < cols; c0 += w) {
    const int nc = (int)std::min<int64_t>(w, cols - c0);
    if (use_nt) {
      transpose64(T + c0, cols, n, nc, Pt, n, s);
      if (tr) {
        nt.M = nc;
        gemm(nt, nullptr, s);
        transpose64(Bt, n, nc, n, T + c0, cols, s);
      } else {
        nt.N = nc;
        nt.C = T + c0;
        gemm(nt, nullptr, s);
      }
      continue;
    }
    Gemm g = g64(n, nc, n);
    g.A = Linv;
    g.lda = n;
    g.B = T + c0;  // B[j][k] = T[k][c0 + j]
    g.ldb = cols;
    g.b_kc = false;
    g.C = Pt;
    g.ldc = nc;
    gemm(g, nullptr, s);
    store_block(Pt, DType::F64, nc, 0, T + c0, DType::F64, cols, 0, 1, n, nc, s);
  }
}

// rows of FP64 B [rows][cols] into the preallocated stored factor (row stride ldd, zero padding; BF16
// rows divided by the power-of-two scale (row / div) % mod, remainder into lo when given)
static void store_factor(const double* B, int64_t rows, int64_t cols, int64_t ldd, int precision,
                         const float* scale, int64_t div, int64_t mod, DevBuf& main, DevBuf* lo, hipStream_t s) {
  const int64_t n = std::max<int64_t>(rows * ldd, 1);
  const DType td = precision == RISP_FP64 ? DType::F64 : (precision == RISP_FP32 ? DType::F32 : DType::BF16);
  RISP_CHECK(main.bytes() >= (size_t)n * dtype_size(td) && (!lo || lo->bytes() >= (size_t)n * 2), RISP_E_STATE,
             "stored factor buffer too small");
  store_rows_padded(B, DType::F64, cols, rows, cols, main.get(), td, ldd, td == DType::BF16 ? scale : nullptr,
                    div, mod, s);
  if (td == DType::BF16 && lo)
    store_rows_padded_lo(B, DType::F64, cols, rows, cols, main.get(), lo->get(), ldd, scale, div, mod, s);
}

// power-of-two scales of `slices` contiguous FP64 slices of `len` values (ones when disabled)
static void slice_scales(const double* B, int slices, int64_t len, bool enabled, DevBuf& out, hipStream_t s) {
  out.alloc(std::max(slices, 1) * sizeof(float));
  if (enabled) {
    row_pow2_scales(B, slices, len, out.as<float>(), s);
  } else {
    std::vector<float> ones(std::max(slices, 1), 1.0f);
    RISP_HIP(hipMemcpyAsync(out.get(), ones.data(), ones.size() * 4, hipMemcpyHostToDevice, s));
    RISP_HIP(hipStreamSynchronize(s));
  }
}

__global__ void k_mul_scales(const float* a, const float* b, float* c, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) c[t] = a[t] * b[t];
}

// T~[P][p][q] = C_l^T (mu nu|P) C_r over auxiliary shells, chunked; V = (mu nu|op|P) FP64.
// CLT [nl][nao], CRT [nr][nao] (transposed MO coefficient blocks). Out: FP64 [nfunc][nl][nr].
static void transformed_3c(risp_ctx* ctx, hipStream_t s, const DevShells& ao, const PairList& pairs,
                           const DevShells& aux, const Operator& op, const double* CLT, int nl,
                           const double* CRT, int nr, double* out) {
  const int nao = ao.nfunc;
  // auxiliary shell chunks (the batch of the transform products): enough functions for ~2048 output
  // tiles of the first product, within kIntChunk bytes of FP64 integrals
  const int64_t per_func = (int64_t)nao * nao * 8;
  const int64_t tiles_per_func = (int64_t)((nl + 127) / 128) * ((nao + 255) / 256);
  const int max_f = (int)std::max<int64_t>(
      3, std::min<int64_t>({256, kIntChunk / per_func, (2048 + tiles_per_func - 1) / tiles_per_func}));
  std::vector<int> l(aux.n);
  RISP_HIP(hipMemcpyAsync(l.data(), aux.l.get(), aux.n * sizeof(int), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  DevBuf V((size_t)max_f * nao * nao * 8 + 8);
  DevBuf G((size_t)max_f * std::max(nl, 1) * nao * 8 + 8);
  int f0 = 0;
  for (int s0 = 0; s0 < aux.n;) {
    int s1 = s0, nf = 0;
    while (s1 < aux.n && nf + (l[s1] == 0 ? 1 : 3) <= max_f) nf += l[s1++] == 0 ? 1 : 3;
    int3c(ao, pairs, aux, s0, s1, op, ctx->boys.as<double>(), V.as<double>(), s);
    // G[P][i][mu] = sum_nu CLT[i][nu] V[P][mu][nu]   (V symmetric in mu, nu)
    Gemm g = g64(nl, nao, nao);
    g.A = CLT;
    g.lda = nao;
    g.B = V.get();
    g.ldb = nao;
    g.C = G.get();
    g.ldc = nao;
    g.nb2 = nf;
    g.sb2 = (int64_t)nao * nao;
    g.sc2 = (int64_t)nl * nao;
    gemm(g, nullptr, s);
    // out[P][i][a] = sum_mu G[P][i][mu] CRT[a][mu]
    Gemm h = g64(nl, nr, nao);
    h.A = G.get();
    h.lda = nao;
    h.sa2 = (int64_t)nl * nao;
    h.B = CRT;
    h.ldb = nao;
    h.C = out + (int64_t)f0 * nl * nr;
    h.ldc = nr;
    h.sc2 = (int64_t)nl * nr;
    h.nb2 = nf;
    gemm(h, nullptr, s);
    f0 += nf;
    s0 = s1;
  }
  RISP_HIP(hipStreamSynchronize(s));
}

static void build_partners(const risp_system* sys, const PairList& pairs, Partners& P, hipStream_t s) {
  const int nsh = sys->nshell;
  std::vector<int> shoff(nsh + 1, 0);
  for (int k = 0; k < nsh; ++k) shoff[k + 1] = shoff[k] + (sys->shells[k].l == 0 ? 1 : 3);
  const int nao = shoff[nsh];
  // groups: runs of consecutive shells on one atom (their functions are contiguous)
  std::vector<int> gsh(nsh), first;
  for (int k = 0; k < nsh; ++k) {
    if (k == 0 || sys->shells[k].atom != sys->shells[k - 1].atom) first.push_back(k);
    gsh[k] = (int)first.size() - 1;
  }
  const int ng = (int)first.size();
  first.push_back(nsh);
  std::vector<int> pa(pairs.n), pb(pairs.n);
  if (pairs.n > 0) {
    RISP_HIP(hipMemcpyAsync(pa.data(), pairs.a.get(), pairs.n * sizeof(int), hipMemcpyDeviceToHost, s));
    RISP_HIP(hipMemcpyAsync(pb.data(), pairs.b.get(), pairs.n * sizeof(int), hipMemcpyDeviceToHost, s));
  }
  RISP_HIP(hipStreamSynchronize(s));
  std::vector<std::vector<int>> part(ng), spos(ng);
  for (int ip = 0; ip < pairs.n; ++ip) {
    const int A = pa[ip], B = pb[ip];
    part[gsh[A]].push_back(B);
    if (A != B) part[gsh[B]].push_back(A);
  }
  P.ngroups = ng;
  P.mu0.resize(ng);
  P.n.resize(ng);
  P.kp.resize(ng);
  P.voff.resize(ng);
  P.koff.resize(ng);
  std::vector<int> hidx;
  std::vector<int64_t> hfvoff(nao);
  std::vector<int> hfng(nao), hfkp(nao), hfml(nao);
  int64_t voff = 0, koff = 0;
  for (int g = 0; g < ng; ++g) {
    auto& pl = part[g];
    std::sort(pl.begin(), pl.end());
    pl.erase(std::unique(pl.begin(), pl.end()), pl.end());
    int pos = 0;
    for (int t : pl) {
      spos[g].push_back(pos);
      for (int q = shoff[t]; q < shoff[t + 1]; ++q) hidx.push_back(q);
      pos += shoff[t + 1] - shoff[t];
    }
    const int kp = std::max<int>(8, (int)pad8(pos));
    for (int q = pos; q < kp; ++q) hidx.push_back(-1);
    P.mu0[g] = shoff[first[g]];
    P.n[g] = shoff[first[g + 1]] - shoff[first[g]];
    P.kp[g] = kp;
    P.voff[g] = voff;
    P.koff[g] = koff;
    for (int mu = P.mu0[g]; mu < P.mu0[g] + P.n[g]; ++mu) {
      hfvoff[mu] = voff;
      hfng[mu] = P.n[g];
      hfkp[mu] = kp;
      hfml[mu] = mu - P.mu0[g];
    }
    voff += (int64_t)P.n[g] * kp;
    koff += kp;
  }
  P.S = voff;
  auto where = [&](int g, int t) {
    const auto& pl = part[g];
    const auto it = std::lower_bound(pl.begin(), pl.end(), t);
    RISP_CHECK(it != pl.end() && *it == t, RISP_E_STATE, "partner list misses a kept pair");
    return spos[g][it - pl.begin()];
  };
  // row and partner function of every packed position (group, mu, k) of one auxiliary function
  std::vector<int> hrow((size_t)P.S), hcol((size_t)P.S);
  for (int g = 0; g < ng; ++g)
    for (int ml = 0; ml < P.n[g]; ++ml)
      for (int k = 0; k < P.kp[g]; ++k) {
        const size_t q = (size_t)P.voff[g] + (size_t)ml * P.kp[g] + k;
        hrow[q] = P.mu0[g] + ml;
        hcol[q] = hidx[(size_t)P.koff[g] + k];
      }
  std::vector<int> hcab(pairs.n), hcba(pairs.n);
  for (int ip = 0; ip < pairs.n; ++ip) {
    hcab[ip] = where(gsh[pa[ip]], pb[ip]);
    hcba[ip] = where(gsh[pb[ip]], pa[ip]);
  }
  P.idx = upload(hidx.data(), hidx.size(), s);
  P.gkoff = upload(P.koff.data(), P.koff.size(), s);
  P.gkp = upload(P.kp.data(), P.kp.size(), s);
  P.fvoff = upload(hfvoff.data(), hfvoff.size(), s);
  P.fng = upload(hfng.data(), hfng.size(), s);
  P.fkp = upload(hfkp.data(), hfkp.size(), s);
  P.fml = upload(hfml.data(), hfml.size(), s);
  P.cab = upload(hcab.data(), hcab.size(), s);
  P.cba = upload(hcba.data(), hcba.size(), s);
  P.prow = upload(hrow.data(), hrow.size(), s);
  P.pcol = upload(hcol.data(), hcol.size(), s);
  RISP_HIP(hipStreamSynchronize(s));  // the host arrays die at return
}

// Cg[g][i][k] = CLT[i][idx[koff_g + k]] (0 for padding) for the groups g0 + blockIdx.y, stored group after
// group from group g0 on (nl rows of kp_g values each)
__global__ void k_gather_partner_cols(const double* __restrict__ CLT, int nao, int nl, const int* __restrict__ idx,
                                      const int64_t* __restrict__ koff, const int* __restrict__ kp, int g0,
                                      double* __restrict__ out) {
  const int g = g0 + blockIdx.y;
  const int64_t ko = koff[g], base = (ko - koff[g0]) * nl;
  const int K = kp[g];
  const int64_t total = (int64_t)nl * K;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / K), k = (int)(t % K);
    const int nu = idx[ko + k];
    out[base + t] = nu >= 0 ? CLT[(int64_t)i * nao + nu] : 0.0;
  }
}

// transformed_3c over the partner lists: the integrals of each auxiliary chunk go straight into the
// packed per-atom layout, and the first product runs as one grouped launch of per-atom products
// (rows i, columns (f, mu) of the atom, K = its padded partner count) writing G[f][i][mu]; the
// second product is the dense one of transformed_3c.
constexpr int kPartnerChunkF = 51;             // functions per chunk: groups of 5 and 9 fill 256-wide tiles
constexpr int64_t kPartnerG = 16ll << 30;      // bytes of G per chunk
constexpr int64_t kPartnerPack = 8ll << 30;    // bytes of the packed integrals per chunk
constexpr int64_t kPartnerCg = 6ll << 30;      // bytes of gathered C columns per batch of atoms

// Buffers of one transformed_3c_partners call for nl left orbitals: functions per auxiliary chunk,
// batches of consecutive groups (gathered C columns within kPartnerCg, unless one group alone is
// larger) and the bytes taken from the arena.
struct PartnerPlan {
  int max_f = 0;
  std::vector<int> bstart;
  int64_t cg_elems = 0;
  size_t bytes = 0;
};
static PartnerPlan partner_plan(const Partners& P, int nl, int nao) {
  PartnerPlan pl;
  const int64_t per_g = (int64_t)std::max(nl, 1) * nao * 8;
  pl.max_f = (int)std::max<int64_t>(
      3, std::min<int64_t>({kPartnerChunkF, kPartnerG / per_g, kPartnerPack / std::max<int64_t>(P.S * 8, 1)}));
  pl.bstart.push_back(0);
  int64_t acc = 0;
  for (int g = 0; g < P.ngroups; ++g) {
    if (acc > 0 && (int64_t)nl * (acc + P.kp[g]) * 8 > kPartnerCg) {
      pl.bstart.push_back(g);
      acc = 0;
    }
    acc += P.kp[g];
    pl.cg_elems = std::max<int64_t>(pl.cg_elems, (int64_t)nl * acc);
  }
  pl.bstart.push_back(P.ngroups);
  pl.bytes = Arena::round((size_t)pl.max_f * P.S * 8) + Arena::round((size_t)pl.max_f * std::max(nl, 1) * nao * 8) +
             Arena::round((size_t)pl.cg_elems * 8 + 8);
  return pl;
}

static void transformed_3c_partners(risp_ctx* ctx, hipStream_t s, const DevShells& ao, const PairList& pairs,
                                    const Partners& P, const DevShells& aux, const Operator& op, const double* CLT,
                                    int nl, const double* CRT, int nr, double* out, Arena& ar, bool upper) {
  const int nao = ao.nfunc;
  RISP_CHECK(!upper || nr >= nl, RISP_E_STATE, "upper transform: the right orbitals must include the left ones");
  const PartnerPlan pl = partner_plan(P, nl, nao);
  const int max_f = pl.max_f;
  const std::vector<int>& bstart = pl.bstart;
  std::vector<int> l(aux.n);
  RISP_HIP(hipMemcpyAsync(l.data(), aux.l.get(), aux.n * sizeof(int), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  const int nb = (int)bstart.size() - 1;
  // descriptors and tile numbering of every batch (fixed over the chunks: the packed layout and G
  // use max_f functions; the rows of a narrower last chunk are zero)
  const int tiles_m = (nl + 127) / 128;
  std::vector<GemmGroup> hd(P.ngroups);
  std::vector<int> ht;  // per batch: tile0 of its groups, then the total
  std::vector<int> toff(nb), ttot(nb);
  for (int b = 0; b < nb; ++b) {
    const int g0 = bstart[b], g1 = bstart[b + 1];
    toff[b] = (int)ht.size();
    int64_t tiles = 0;
    for (int g = g0; g < g1; ++g) {
      GemmGroup& d = hd[g];
      d.a_off = (int64_t)nl * (P.koff[g] - P.koff[g0]);
      d.b_off = (int64_t)max_f * P.voff[g];
      d.c_off = P.mu0[g];
      d.K = P.kp[g];
      d.ld = P.kp[g];
      d.N = max_f * P.n[g];
      d.n_inner = P.n[g];
      ht.push_back((int)tiles);
      tiles += (int64_t)tiles_m * ((d.N + 255) / 256);
    }
    RISP_CHECK(tiles < (1ll << 31), RISP_E_SHAPE, "partner product grid too large");
    ht.push_back((int)tiles);
    ttot[b] = (int)tiles;
  }
  DevBuf dd = upload(hd.data(), hd.size(), s), dt = upload(ht.data(), ht.size(), s);
  const size_t m0 = ar.mark();
  const WsView Vp = ar.take((size_t)max_f * P.S * 8), G = ar.take((size_t)max_f * std::max(nl, 1) * nao * 8),
               Cg = ar.take((size_t)pl.cg_elems * 8 + 8);
  const PackMap pm = P.map(max_f);
  auto gather = [&](int b) {
    const int g0 = bstart[b], g1 = bstart[b + 1];
    k_gather_partner_cols<<<dim3(64, g1 - g0), 256, 0, s>>>(CLT, nao, nl, P.idx.as<int>(), P.gkoff.as<int64_t>(),
                                                          P.gkp.as<int>(), g0, Cg.as<double>());
    RISP_LAUNCHED();
  };
  if (nb == 1) gather(0);
  int f0 = 0;
  for (int s0 = 0; s0 < aux.n;) {
    int s1 = s0, nf = 0;
    while (s1 < aux.n && nf + (l[s1] == 0 ? 1 : 3) <= max_f) nf += l[s1++] == 0 ? 1 : 3;
    int3c(ao, pairs, aux, s0, s1, op, ctx->boys.as<double>(), Vp.as<double>(), s, &pm);
    for (int b = 0; b < nb; ++b) {
      if (nb > 1) gather(b);
      Gemm g = g64(nl, 0, 0);
      g.A = Cg.get();
      g.B = Vp.get();
      g.C = G.get();
      g.ldc = nao;
      g.sc_outer = (int64_t)nl * nao;
      gemm_f64_grouped(g, dd.as<GemmGroup>() + bstart[b], dt.as<int>() + toff[b], bstart[b + 1] - bstart[b], ttot[b],
                       s);
    }
    // out[P][i][a] = sum_mu G[P][i][mu] CRT[a][mu]; upper: the right orbitals start with the left
    // ones and only a >= i is needed, so each 128-row band starts at its own first row
    const int band = upper ? 128 : nl;
    for (int r0 = 0; r0 < nl; r0 += band) {
      Gemm h = g64(std::min(band, nl - r0), nr - (upper ? r0 : 0), nao);
      h.A = G.as<double>() + (size_t)r0 * nao;
      h.lda = nao;
      h.sa2 = (int64_t)nl * nao;
      h.B = CRT + (upper ? (size_t)r0 * nao : 0);
      h.ldb = nao;
      h.C = out + (int64_t)f0 * nl * nr + (int64_t)r0 * nr + (upper ? r0 : 0);
      h.ldc = nr;
      h.sc2 = (int64_t)nl * nr;
      h.nb2 = nf;
      gemm(h, nullptr, s);
    }
    f0 += nf;
    s0 = s1;
  }
  RISP_HIP(hipStreamSynchronize(s));
  ar.release_to(m0);
}

// B = L^-1 T~ over the auxiliary index: T~ [n][cols] -> B [n][cols] (FP64), in ov-column chunks.
// Txt[a][P][j] = Bx[P][j][a] (FP64 source, FP64 or FP32 destination, row stride ldj)
template <typename TD>
__global__ void k_permute_x(const double* __restrict__ Bx, int nP, int no, int nv, TD* __restrict__ out, int ldj) {
  const int64_t total = (int64_t)nP * no * nv;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t % nv);
    const int j = (int)((t / nv) % no);
    const int P = (int)(t / ((int64_t)nv * no));
    out[((int64_t)a * nP + P) * ldj + j] = (TD)Bx[t];
  }
}

static void permute_x_to_xt(const double* Bx, int nP, int no, int nv, void* out, DType td, int ldj, hipStream_t s) {
  const int64_t total = (int64_t)nP * no * nv;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 16);
  if (td == DType::F64) k_permute_x<double><<<grid, 256, 0, s>>>(Bx, nP, no, nv, static_cast<double*>(out), ldj);
  else k_permute_x<float><<<grid, 256, 0, s>>>(Bx, nP, no, nv, static_cast<float*>(out), ldj);
  RISP_LAUNCHED();
}

static void metric_apply(const double* Linv, int n, const double* T, int64_t cols, double* B, hipStream_t s) {
  const int64_t chunk = 1ll << 24;
  for (int64_t c0 = 0; c0 < cols; c0 += chunk) {
    const int nc = (int)std::min<int64_t>(chunk, cols - c0);
    Gemm g = g64(n, nc, n);
    g.A = Linv;
    g.lda = n;
    g.B = T + c0;  // B[j][k] = T[k][c0 + j]
    g.ldb = cols;
    g.b_kc = false;
    g.C = B + c0;
    g.ldc = cols;
    gemm(g, nullptr, s);
  }
}

static void metric_inverse_cholesky(risp_ctx* ctx, hipStream_t s, const DevShells& aux, const Operator& op,
                                    DevBuf& Linv) {
  const int n = aux.nfunc;
  DevBuf V((size_t)n * n * 8);
  int2c(aux, op, ctx->boys.as<double>(), V.as<double>(), s);
  cholesky(V.as<double>(), n, s);
  Linv.alloc((size_t)n * n * 8);
  tri_inverse(V.as<double>(), Linv.as<double>(), n, s);
  RISP_HIP(hipStreamSynchronize(s));
}

void build_factors(risp_ctx* ctx, const risp_system* sys, const risp_params* prm, risp_factors* f,
                   hipStream_t stream) {
  validate_system(sys);
  RISP_CHECK(prm != nullptr, RISP_E_ARG, "params is NULL");
  RISP_CHECK(prm->precision >= RISP_FP64 && prm->precision <= RISP_BF16, RISP_E_ARG, "bad precision");
  RISP_CHECK(prm->rsh_mode == RISP_RSH_COMBINED || prm->rsh_mode == RISP_RSH_SPLIT, RISP_E_ARG, "bad rsh_mode");
  RISP_CHECK(prm->window_mode == RISP_WIN_ABSOLUTE || prm->window_mode == RISP_WIN_FRONTIER, RISP_E_ARG,
             "bad window_mode");
  RISP_CHECK(prm->theta > 0.0 && prm->schwarz_tau >= 0.0 && prm->omega >= 0.0, RISP_E_ARG,
             "theta must be positive, tau and omega non-negative");
  RISP_CHECK(prm->beta == 0.0 || prm->omega > 0.0, RISP_E_ARG, "beta != 0 needs omega > 0");
  RISP_CHECK(prm->j_mode == RISP_J_MO || prm->j_mode == RISP_J_AO_DIRECT, RISP_E_ARG, "bad j_mode");
  RISP_CHECK(!prm->full_tddft || (prm->precision != RISP_BF16 && prm->rsh_mode == RISP_RSH_COMBINED &&
                                   prm->j_mode == RISP_J_MO),
             RISP_E_ARG, "full TDDFT-risp factors: FP64 or FP32 storage, combined exchange, stored Coulomb route");
  hipStream_t s = stream ? stream : ctx->stream;
  const int nao = sys->nao, nmo = sys->nmo, nocc = sys->nocc, nvir = nmo - nocc;
  f->ctx = ctx;
  f->stream = s;
  f->nao = nao;
  f->nmo = nmo;
  f->nocc = nocc;
  f->nvir = nvir;
  f->precision = prm->precision;
  f->has_f32 = prm->precision == RISP_BF16;
  f->j_mode = prm->j_mode;
  f->full = prm->full_tddft != 0;
  f->coul32 = prm->precision == RISP_BF16 && prm->bf16_coulomb_fp32 != 0;

  // auxiliary bases (section on exchange-space truncation: H omitted, J = s + p, K = s)
  std::vector<risp_shell> auxJ, auxK;
  select_aux(sys, prm, auxJ, auxK);
  RISP_CHECK(!auxJ.empty(), RISP_E_ARG, "no auxiliary functions (all atoms are hydrogen)");

  DevShells ao, aj, ak;
  upload_shells(ao, sys->coords, sys->shells, sys->nshell, s);
  upload_shells(aj, sys->coords, auxJ.data(), (int)auxJ.size(), s);
  upload_shells(ak, sys->coords, auxK.data(), (int)auxK.size(), s);
  f->naux_j = aj.nfunc;

  DevBuf C = upload(sys->mo_coeff, (size_t)nao * nmo, s);
  DevBuf E = upload(sys->mo_energy, (size_t)nmo, s);

  // window
  f->occ_k.alloc(std::max(nocc, 1) * sizeof(int));
  f->vir_k.alloc(std::max(nvir, 1) * sizeof(int));
  window_sets(E.as<double>(), nmo, nocc, prm->window_ev, prm->window_mode, f->occ_k.as<int>(), &f->nok,
              f->vir_k.as<int>(), &f->nvk, s);
  f->pos_o.alloc(std::max(nocc, 1) * sizeof(int));
  f->pos_v.alloc(std::max(nvir, 1) * sizeof(int));
  window_positions(f->occ_k.as<int>(), f->nok, nocc, f->pos_o.as<int>(), s);
  window_positions(f->vir_k.as<int>(), f->nvk, nvir, f->pos_v.as<int>(), s);

  // screening against the Coulomb auxiliary basis
  const double qaux = std::sqrt(aux_diag_max(aj, ctx->boys.as<double>(), s));
  PairList pairs;
  screen_pairs(ao, qaux, prm->schwarz_tau, false, pairs, s);
  f->npair = pairs.n;
  // first transforms over the per-atom partner lists of the kept pairs, or over dense slabs
  Partners partners;
  const bool sparse_t = prm->dense_transform == 0;
  if (sparse_t || prm->j_mode == RISP_J_AO_DIRECT) build_partners(sys, pairs, partners, s);
  Arena ar;
  // upper: CRT starts with the nl orbitals of CLT and only out[P][i][a] with a >= i is needed (the
  // partner path skips most of the rest; the dense path computes everything)
  auto t3c = [&](const DevShells& aux, const Operator& op, const double* CLT, int nl, const double* CRT, int nr,
                 double* out, bool upper = false) {
    if (sparse_t) transformed_3c_partners(ctx, s, ao, pairs, partners, aux, op, CLT, nl, CRT, nr, out, ar, upper);
    else transformed_3c(ctx, s, ao, pairs, aux, op, CLT, nl, CRT, nr, out);
  };
  // arena bytes of one t3c call with nl left orbitals (the dense path allocates its own buffers)
  auto t3c_bytes = [&](int nl) -> size_t { return sparse_t ? partner_plan(partners, nl, nao).bytes : 0; };

  // transposed MO blocks
  DevBuf CoT((size_t)nocc * nao * 8), CvT((size_t)nvir * nao * 8);
  gather_transpose(C.as<double>(), nmo, nao, nullptr, 0, nocc, CoT.as<double>(), s);
  gather_transpose(C.as<double>(), nmo, nao, nullptr, nocc, nvir, CvT.as<double>(), s);

  // exchange operator blocks (combined reading: one; split reading: 1/r and erf(omega r)/r)
  std::vector<Operator> blocks;
  if (prm->c_x != 0.0 || prm->beta != 0.0) {
    if (prm->rsh_mode == RISP_RSH_COMBINED) {
      blocks.push_back({prm->c_x, prm->beta, prm->omega});
    } else {
      if (prm->c_x != 0.0) blocks.push_back({prm->c_x, 0.0, 0.0});
      if (prm->beta != 0.0) blocks.push_back({0.0, prm->beta, prm->omega});
    }
  }
  const int nks = ak.nfunc;
  const int nok = f->nok, nvk = f->nvk;
  f->naux_k = (int)blocks.size() * nks;
  const bool exch = f->naux_k > 0 && nok > 0 && nvk > 0;
  if (!exch) f->naux_k = 0;
  const int nK = f->naux_k;
  const bool jmo = f->j_mode != RISP_J_AO_DIRECT;
  const int nJ = aj.nfunc;
  const int64_t ov = (int64_t)nocc * nvir;
  f->ld_ia = pad8(ov);
  f->nokp = (int)pad8(nok);
  f->nvkp = (int)pad8(nvk);

  // ---- stored factors, allocated before any temporary ----
  // BF16 factors also keep the FP32 copy of T_ia and the BF16 remainders of T_ij and T_ab (the
  // correction pass); T_ia goes through its FP32 copy (the per-slice scales need the maximum over
  // every chunk) and T_ab through an FP32 staging block in the arena.
  const bool bf = prm->precision == RISP_BF16;
  const DType tdst = prm->precision == RISP_FP64 ? DType::F64 : DType::F32;
  const size_t dsz = dtype_size(tdst);
  const size_t esz = bf ? 2 : dsz;  // stored element
  f->diag64.alloc((size_t)std::max<int64_t>(ov, 1) * 8);
  fill_zero(f->diag64.get(), f->diag64.bytes(), s);
  if (jmo) {
    DevBuf& dst = bf ? f->t_ia32 : f->t_ia;
    dst.alloc((size_t)std::max<int64_t>((int64_t)nJ * f->ld_ia, 1) * dsz);
    fill_zero(dst.get(), dst.bytes(), s);  // zero padding columns
    if (bf) f->t_ia.alloc((size_t)std::max<int64_t>((int64_t)nJ * f->ld_ia, 1) * 2);
  }
  const size_t n_ab = (size_t)std::max<int64_t>((int64_t)nK * nvk * f->nvkp, 1);
  const size_t n_ij = (size_t)std::max<int64_t>((int64_t)nok * nK * f->nokp, 1);
  if (exch) {
    // written chunk by chunk, padding stays zero; BF16 factors stage the FP32 values as their two
    // 16-bit halves in t_ab and t_ab_lo and convert them in place once the slice scales are known
    f->t_ab.alloc(n_ab * esz);
    fill_zero(f->t_ab.get(), f->t_ab.bytes(), s);
    if (bf) {
      f->t_ab_lo.alloc(n_ab * 2);
      fill_zero(f->t_ab_lo.get(), f->t_ab_lo.bytes(), s);
    }
    f->t_ij.alloc(n_ij * esz);
    if (bf) f->t_ij_lo.alloc(n_ij * 2);
    if (f->full) {
      f->t_x.alloc((size_t)std::max<int64_t>((int64_t)nks * nok * f->nvkp, 1) * dsz);
      f->t_xt.alloc((size_t)std::max<int64_t>((int64_t)nvk * nks * f->nokp, 1) * dsz);
      fill_zero(f->t_xt.get(), f->t_xt.bytes(), s);
    }
  }

  // ---- the arena: chunk sizes planned against the free device memory ----
  RISP_CHECK(prm->build_chunk_kib >= 0, RISP_E_ARG, "build_chunk_kib must be non-negative");
  size_t fr = 0, tot = 0;
  RISP_HIP(hipMemGetInfo(&fr, &tot));
  // room left for the small allocations of the build, for the dense-slab path's own buffers, and for
  // a following Davidson solve (default block of 30 and subspace of 270 vectors with their products,
  // Ritz and correction rows, sigma workspaces): its allocations then find device memory that no
  // earlier allocation used, which the driver does not have to clear first
  const int64_t vsz = prm->precision == RISP_FP64 ? 8 : 4, blk = 30, cap = 9 * blk;
  const int64_t dav = 2 * cap * ov * vsz + 4 * blk * ov * 8 + 4 * blk * ov * vsz + blk * f->ld_ia * 4 +
                      (exch ? std::min<int64_t>(4ll << 30, (int64_t)nK * blk * nvk * f->nokp * 4) +
                                  blk * (int64_t)f->nokp * f->nvkp * 4 + 5 * blk * (int64_t)nok * nvk * 4
                            : 0);
  const int64_t keep = (2ll << 30) + (int64_t)(0.02 * (double)tot) + (sparse_t ? 0 : (20ll << 30));
  const int64_t budget = std::max<int64_t>(1ll << 30, (int64_t)fr - keep - dav);
  // FP64 chunk of transformed integrals: build_chunk_kib when given
  const int64_t chunk_cap = prm->build_chunk_kib > 0 ? ((int64_t)prm->build_chunk_kib << 10) : budget;
  // rows per chunk: all when they fit, else the largest multiple of 128 (the transforms' row tile)
  auto plan_rows = [&](int n, int64_t per_row, auto&& bytes_for) -> int {
    auto fits = [&](int r) { return r * per_row <= chunk_cap && (int64_t)bytes_for(r) <= budget; };
    if (fits(n)) return std::max(n, 1);
    int r = std::max(1, (int)std::min<int64_t>(n, chunk_cap / std::max<int64_t>(per_row, 1)));
    if (r >= 128) r = r / 128 * 128;
    while (r > 128 && !fits(r)) r -= 128;
    while (r > 1 && !fits(r)) r = r > 128 ? r - 128 : r / 2;
    return r;
  };
  int ni = 0, na = 0;
  size_t need_j = 0, need_k = 0, k_persist = 0;
  if (jmo) {
    const int64_t per_row = (int64_t)nJ * std::max(nvir, 1) * 8;
    auto bytes_j = [&](int r) {
      return Arena::round((size_t)per_row * r) + metric_panel_bytes(nJ, (int64_t)r * nvir) + t3c_bytes(r);
    };
    ni = plan_rows(nocc, per_row, bytes_j);
    need_j = bytes_j(ni);
  }
  if (exch) {
    k_persist = Arena::round((size_t)nK * nok * nok * 8) + Arena::round((size_t)nK * nvk * 8);
    const size_t step_ij = Arena::round((size_t)nks * nok * nok * 8) + t3c_bytes(nok);
    const size_t step_x = f->full ? 2 * Arena::round((size_t)nks * nok * nvk * 8) + t3c_bytes(nok) : 0;
    const size_t after = Arena::round((size_t)nK * nok * nok * 8);  // T_ij in [i][P][j] order (FP64)
    const int64_t per_row = (int64_t)nks * nvk * 8;
    auto bytes_k = [&](int r) {
      const size_t tab = Arena::round((size_t)per_row * r) + metric_panel_bytes(nks, (int64_t)r * nvk) + t3c_bytes(r);
      return k_persist + std::max({step_ij, step_x, tab, after});
    };
    na = plan_rows(nvk, per_row, bytes_k);
    need_k = bytes_k(na);
  }
  ar.reserve(std::max(need_j, need_k));

  // ---- Coulomb factor T_ia ----
  // Built in chunks of ni occupied orbitals: transformed integrals (Q|ia), the metric applied in
  // place, then stored rows.
  if (!jmo) {
    // no stored T_ia: keep the metric factor and plan the auxiliary chunks of the per-sigma integral
    // passes (packed (mu nu|P) over the kept pairs, at most ~2 GiB per chunk, whole shells)
    Operator coul;
    metric_inverse_cholesky(ctx, s, aj, coul, f->linv_j);
    f->j_op = coul;
    const int64_t per_func = std::max<int64_t>(partners.S * 8, 8);
    const int max_f = (int)std::max<int64_t>(3, std::min<int64_t>(256, (2ll << 30) / per_func));
    const int ns = (int)auxJ.size();
    f->ao_s0.clear();
    f->ao_f0.clear();
    f->ao_max_f = 0;
    int fo = 0;
    for (int s0 = 0; s0 < ns;) {
      int s1 = s0, nf = 0;
      while (s1 < ns && nf + (auxJ[s1].l == 0 ? 1 : 3) <= max_f) nf += auxJ[s1++].l == 0 ? 1 : 3;
      f->ao_s0.push_back(s0);
      f->ao_f0.push_back(fo);
      f->ao_max_f = std::max(f->ao_max_f, nf);
      fo += nf;
      s0 = s1;
    }
    f->ao_s0.push_back(ns);
    f->ao_f0.push_back(fo);
    RISP_CHECK(fo == aj.nfunc, RISP_E_STATE, "auxiliary chunk plan does not cover the basis");
    // trial vectors per group (each group regenerates the integrals twice): as many as a quarter of
    // the memory left after the factors holds (at least 4 GiB) with their dense D_m / U_m, packed
    // D_m and half-transformed block; the rest stays for the Davidson subspace and the exchange
    const int64_t per_vec = ((int64_t)nao * nao + (int64_t)nocc * nao + partners.S) * 8;
    const int64_t ao_budget = std::max<int64_t>(4ll << 30, (int64_t)(fr / 4));
    f->ao_mg = (int)std::max<int64_t>(1, std::min<int64_t>(64, ao_budget / per_vec));
  } else {
    Operator coul;  // 1/r
    DevBuf Linv;
    metric_inverse_cholesky(ctx, s, aj, coul, Linv);
    DevBuf& dst = bf ? f->t_ia32 : f->t_ia;
    DevBuf mx((size_t)std::max(nJ, 1) * 8);
    const size_t m0 = ar.mark();
    const WsView Tt = ar.take((size_t)nJ * ni * std::max(nvir, 1) * 8);
    const WsView tmp = ar.take(metric_panel_bytes(nJ, (int64_t)ni * nvir));
    for (int i0 = 0; i0 < nocc; i0 += ni) {
      const int nic = std::min(ni, nocc - i0);
      const int64_t cols = (int64_t)nic * nvir;
      t3c(aj, coul, CoT.as<double>() + (size_t)i0 * nao, nic, CvT.as<double>(), nvir, Tt.as<double>());
      metric_apply_inplace(Linv.as<double>(), nJ, Tt.as<double>(), cols, tmp, s);
      col_sumsq(Tt.as<double>(), nJ, cols, cols, 2.0, f->diag64.as<double>() + (size_t)i0 * nvir, s);
      if (bf) row_absmax(Tt.as<double>(), nJ, cols, cols, mx.as<double>(), i0 > 0, s);
      store_block(Tt.get(), DType::F64, cols, 0, static_cast<char*>(dst.get()) + (size_t)i0 * nvir * dsz, tdst,
                  f->ld_ia, 0, 1, nJ, cols, s);
    }
    if (bf) {
      f->scale_ia.alloc((size_t)std::max(nJ, 1) * sizeof(float));
      pow2_from_max(mx.as<double>(), nJ, prm->bf16_scale != 0, f->scale_ia.as<float>(), s);
      store_rows_padded(f->t_ia32.get(), DType::F32, f->ld_ia, nJ, f->ld_ia, f->t_ia.get(), DType::BF16, f->ld_ia,
                        f->scale_ia.as<float>(), 1, std::max(nJ, 1), s);
      f->scale_ia2.alloc((size_t)std::max(nJ, 1) * sizeof(float));
      k_mul_scales<<<ceil_div(std::max(nJ, 1), 256), 256, 0, s>>>(f->scale_ia.as<float>(), f->scale_ia.as<float>(),
                                                                   f->scale_ia2.as<float>(), nJ);
      RISP_LAUNCHED();
    }
    RISP_HIP(hipStreamSynchronize(s));  // mx and Linv die at the end of this scope
    ar.release_to(m0);
  }

  // ---- exchange factors T_ij, T_ab in the J^ metric ----
  if (exch) {
    DevBuf CoKT((size_t)nok * nao * 8), CvKT((size_t)nvk * nao * 8);
    gather_transpose(C.as<double>(), nmo, nao, f->occ_k.as<int>(), 0, nok, CoKT.as<double>(), s);
    // virtual window columns are nocc + vir_k[b]: gather through a shifted index list
    {
      std::vector<int> hv(nvk);
      RISP_HIP(hipMemcpyAsync(hv.data(), f->vir_k.get(), nvk * sizeof(int), hipMemcpyDeviceToHost, s));
      RISP_HIP(hipStreamSynchronize(s));
      for (int& v : hv) v += nocc;
      DevBuf dv = upload(hv.data(), hv.size(), s);
      gather_transpose(C.as<double>(), nmo, nao, dv.as<int>(), 0, nvk, CvKT.as<double>(), s);
      RISP_HIP(hipStreamSynchronize(s));
    }
    // T_ij stored [i][P][j] (j padded) for the second exchange product; T_ab [P][a][b] (b padded),
    // written chunk by chunk of window virtuals a (BF16 factors: into an FP32 staging block until
    // the slice scales are known)
    const size_t m0 = ar.mark();
    const WsView Bij = ar.take((size_t)nK * nok * nok * 8);
    const WsView Baa = ar.take((size_t)nK * nvk * 8);  // Bx^P_aa, for the diagonal of A
    DevBuf mxab((size_t)std::max(nK, 1) * 8);
    for (size_t blk = 0; blk < blocks.size(); ++blk) {
      DevBuf Linv;
      metric_inverse_cholesky(ctx, s, ak, blocks[blk], Linv);
      {
        const size_t mk = ar.mark();
        const WsView Tij = ar.take((size_t)nks * nok * nok * 8);
        t3c(ak, blocks[blk], CoKT.as<double>(), nok, CoKT.as<double>(), nok, Tij.as<double>());
        metric_apply(Linv.as<double>(), nks, Tij.as<double>(), (int64_t)nok * nok,
                     Bij.as<double>() + blk * (size_t)nks * nok * nok, s);
        RISP_HIP(hipStreamSynchronize(s));
        ar.release_to(mk);
      }
      if (f->full) {
        // full TDDFT-risp: the exchange factor over the window's (i, a) pairs, FP64 [P][i][b], stored
        // as Tx [P][i][b] (b padded) and Txt [a][P][j] (j padded)
        const size_t mk = ar.mark();
        const WsView Tx = ar.take((size_t)nks * nok * nvk * 8), Bx = ar.take((size_t)nks * nok * nvk * 8);
        t3c(ak, blocks[blk], CoKT.as<double>(), nok, CvKT.as<double>(), nvk, Tx.as<double>());
        metric_apply(Linv.as<double>(), nks, Tx.as<double>(), (int64_t)nok * nvk, Bx.as<double>(), s);
        store_rows_padded(Bx.get(), DType::F64, nvk, (int64_t)nks * nok, nvk, f->t_x.get(), tdst, f->nvkp, nullptr, 1,
                          1, s);
        permute_x_to_xt(Bx.as<double>(), nks, nok, nvk, f->t_xt.get(), tdst, f->nokp, s);
        RISP_HIP(hipStreamSynchronize(s));
        ar.release_to(mk);
      }
      const size_t mk = ar.mark();
      const WsView Tab = ar.take((size_t)nks * na * nvk * 8);
      const WsView tmp = ar.take(metric_panel_bytes(nks, (int64_t)na * nvk));
      // T^P_ab is symmetric in (a, b): a chunk of rows a0 <= a < a0 + nac forms the columns b >= a0
      // only (its transform skips most b < a), stores what it formed with b >= a0, and the strict
      // lower triangle is mirrored from the upper one once every chunk is stored
      for (int a0 = 0; a0 < nvk; a0 += na) {
        const int nac = std::min(na, nvk - a0), nb = nvk - a0;
        const int64_t cols = (int64_t)nac * nb;
        const double* Ca = CvKT.as<double>() + (size_t)a0 * nao;
        t3c(ak, blocks[blk], Ca, nac, Ca, nb, Tab.as<double>(), true);
        metric_apply_inplace(Linv.as<double>(), nks, Tab.as<double>(), cols, tmp, s);
        // chunk element (p, a, a) is Bx^P_aa of window virtual a0 + a
        gather_strided(Tab.as<double>(), nks, nac, cols, nb + 1, Baa.as<double>() + (size_t)blk * nks * nvk + a0, nvk,
                       s);
        if (bf) row_absmax_upper(Tab.as<double>(), nks, nac, nb, mxab.as<double>() + blk * nks, a0 > 0, s);
        // chunk element (p, a, b) -> stored row (blk * nks + p) * nvk + a0 + a, column a0 + b
        const size_t r0 = ((size_t)blk * nks * nvk + a0) * f->nvkp + a0;
        if (bf)
          store_block_split(Tab.as<double>(), nb, nac, f->t_ab.as<uint16_t>() + r0, f->t_ab_lo.as<uint16_t>() + r0,
                            f->nvkp, nvk, nks, nac, nb, s);
        else
          store_block(Tab.get(), DType::F64, nb, nac, static_cast<char*>(f->t_ab.get()) + r0 * dsz, tdst, f->nvkp,
                      nvk, nks, nac, nb, s);
      }
      RISP_HIP(hipStreamSynchronize(s));
      ar.release_to(mk);
    }
    {
      // exchange part of the diagonal: K_ia = sum_P Bx^P_ii Bx^P_aa inside the window
      DevBuf Bii((size_t)nK * nok * 8), Kd((size_t)nok * nvk * 8);
      gather_strided(Bij.as<double>(), nK, nok, (int64_t)nok * nok, nok + 1, Bii.as<double>(), nok, s);
      Gemm g = g64(nok, nvk, nK);  // Kd[i][a] = sum_P Bii[P][i] Baa[P][a]
      g.A = Bii.get();
      g.lda = nok;
      g.a_kc = false;
      g.B = Baa.get();
      g.ldb = nvk;
      g.b_kc = false;
      g.C = Kd.get();
      g.ldc = nvk;
      gemm(g, nullptr, s);
      scatter_sub_window(Kd.as<double>(), nok, nvk, f->occ_k.as<int>(), f->vir_k.as<int>(), nvir,
                         f->diag64.as<double>(), s);
      RISP_HIP(hipStreamSynchronize(s));
    }
    // the strict lower triangle of every T^P_ab from its upper triangle (BF16: both staged halves)
    mirror_lower(f->t_ab.get(), bf ? 2 : (int)dsz, nK, nvk, f->nvkp, (int64_t)nvk * f->nvkp, s);
    if (bf) mirror_lower(f->t_ab_lo.get(), 2, nK, nvk, f->nvkp, (int64_t)nvk * f->nvkp, s);
    DevBuf sij, sab;
    if (bf) {
      slice_scales(Bij.as<double>(), nK, (int64_t)nok * nok, prm->bf16_scale != 0, sij, s);
      sab.alloc((size_t)std::max(nK, 1) * sizeof(float));
      pow2_from_max(mxab.as<double>(), nK, prm->bf16_scale != 0, sab.as<float>(), s);
      split_to_bf16_pair(f->t_ab.get(), f->t_ab_lo.get(), (int64_t)nK * nvk, f->nvkp, sab.as<float>(), nvk, nK, s);
      RISP_HIP(hipStreamSynchronize(s));
    }
    {
      const WsView Bp = ar.take((size_t)nK * nok * nok * 8);  // FP64 [i][P][j]
      permute_pij_ipj(Bij.as<double>(), nK, nok, nok, 8, Bp.get(), s);
      store_factor(Bp.as<double>(), (int64_t)nok * nK, nok, f->nokp, prm->precision, sij.as<float>(), 1, nK, f->t_ij,
                   bf ? &f->t_ij_lo : nullptr, s);
      RISP_HIP(hipStreamSynchronize(s));
    }
    if (bf) {
      f->scale_k.alloc(nK * sizeof(float));
      k_mul_scales<<<ceil_div(nK, 256), 256, 0, s>>>(sij.as<float>(), sab.as<float>(), f->scale_k.as<float>(), nK);
      RISP_LAUNCHED();
    }
    RISP_HIP(hipStreamSynchronize(s));
    ar.release_to(m0);
  }

  // orbital gaps
  f->de64.alloc((size_t)nocc * nvir * 8);
  f->de32.alloc((size_t)nocc * nvir * 4);
  orbital_gaps(E.as<double>(), nocc, nvir, f->de64.as<double>(), f->de32.as<float>(), s);
  add_inplace(f->diag64.as<double>(), f->de64.as<double>(), (int64_t)nocc * nvir, s);
  RISP_HIP(hipStreamSynchronize(s));
  if (f->j_mode == RISP_J_AO_DIRECT) {
    f->ao_sh = std::move(ao);
    f->auxj_sh = std::move(aj);
    f->pairs = std::move(pairs);
    f->co_t = std::move(CoT);
    f->cv_t = std::move(CvT);
    f->co.alloc((size_t)nao * nocc * 8);  // C_occ [mu][i]
    RISP_HIP(hipMemcpy2DAsync(f->co.get(), (size_t)nocc * 8, C.get(), (size_t)nmo * 8, (size_t)nocc * 8, nao,
                              hipMemcpyDeviceToDevice, s));
    RISP_HIP(hipStreamSynchronize(s));
    f->ao_partners = std::move(partners);
  }
}

// -------------------------------------------------------------------------------------------
// sigma = A X
// -------------------------------------------------------------------------------------------
double sigma_flops(const risp_factors* f, int m) {
  const double ov = (double)f->nocc * f->nvir;
  double fl = ov * m;
  if (f->j_mode == RISP_J_AO_DIRECT) {
    // D_m and the back transform (two products each way), both integral contractions, the metric
    const double nao = f->nao, nJ = f->naux_j;
    fl += 4.0 * m * (ov * nao + f->nocc * nao * nao + nJ * nao * nao + nJ * nJ);
  } else {
    fl += 4.0 * ov * f->naux_j * m;
  }
  if (f->naux_k > 0)
    fl += 2.0 * f->naux_k * (double)f->nok * f->nvk * m * (double)(f->nok + f->nvk);
  return fl;
}

constexpr int kMaxSplit = 1024;
constexpr int kMaxSplitK = 4;                 // split-K of the second exchange product
constexpr int64_t kMtBudget = 4ll << 30;      // bytes of the exchange intermediate per P-chunk

// Workspaces are sized for the largest block and the widest compute type seen so far (BF16
// factors also run FP32 products in the correction pass).
static int64_t pad_to(int64_t n, int64_t q) { return (n + q - 1) / q * q; }

// auxiliary functions per exchange chunk for element size c: the intermediate stays within the budget
static int64_t mt_chunk(int64_t nK, int64_t per_p, int64_t c, int64_t budget = kMtBudget) {
  return std::max<int64_t>(1, std::min<int64_t>(nK, budget / (per_p * c)));
}

static void ensure_workspace(risp_factors* f, int m, DType tc, hipStream_t s) {
  const int csz = tc == DType::F64 ? 8 : (tc == DType::F32 ? 4 : 2);
  if (m <= f->ws_m && csz <= f->ws_csz) return;
  RISP_HIP(hipStreamSynchronize(s));  // workspaces may be in use by queued work
  m = std::max(m, f->ws_m);
  const int cs = std::max(csz, f->ws_csz);
  const size_t acc = cs == 8 ? 8 : 4;
  size_t split_bytes = 0;
  if (f->j_mode == RISP_J_AO_DIRECT) {
    const size_t mg = std::min(m, f->ao_mg), nao = f->nao, S = (size_t)f->ao_partners.S;
    f->ws_ao_t.alloc(mg * f->nocc * nao * 8);
    f->ws_ao_d.alloc(mg * nao * nao * 8);
    f->ws_ao_v.alloc((size_t)f->ao_max_f * S * 8);
    f->ws_ao_p.alloc(mg * S * 8);
    f->ws_ao_r.alloc(2 * (size_t)f->naux_j * mg * 8);
    split_bytes = (size_t)kMaxSplit * f->ao_max_f * mg * 8;
  } else {
    f->ws_y.alloc((size_t)f->naux_j * m * acc);
    // Coulomb passes of BF16 and FP32 factors: X with the row stride of T_ia, Yt [64][nJp]
    const size_t xe = (cs >= 4 || f->coul32) ? 4 : 2;
    f->ws_ybf.alloc((size_t)kCoulombMaxM * pad_to(f->naux_j, 32) * xe + 16);
    f->ws_xbf.alloc((size_t)m * f->ld_ia * xe + 16);
    split_bytes = std::max((size_t)kMaxSplit * f->naux_j * m * acc,
                           coulomb_y_workspace(f->naux_j, std::min(m, kCoulombMaxM), f->ld_ia));
  }
  if (f->naux_k > 0 && f->nok > 0 && f->nvk > 0) {
    const int64_t per_p = (int64_t)m * f->nvk * f->nokp;
    // room for the chunk of every compute type up to cs bytes per element and every block size up to
    // m: a chunk holds at most max(one function, min(all functions, the budget))
    int64_t mt = 0;
    for (int64_t c = 2; c <= cs; c *= 2)
      mt = std::max(mt, std::max(per_p * c, std::min<int64_t>(f->naux_k * per_p * c, kMtBudget)));
    f->ws_xw.alloc((size_t)m * f->nokp * f->nvkp * cs);
    f->ws_mt.alloc((size_t)mt);
    f->ws_k.alloc((size_t)m * f->nok * f->nvk * acc);
    split_bytes = std::max(split_bytes, (size_t)kMaxSplitK * m * f->nok * f->nvk * acc);
  }
  f->ws_split.alloc(split_bytes);
  f->ws_m = m;
  f->ws_csz = cs;
}

void sigma_prepare(risp_factors* f, int m, bool use_f32) {
  const bool bf = f->precision == RISP_BF16 && !use_f32;
  const DType tc = f->precision == RISP_FP64 ? DType::F64 : (bf ? DType::BF16 : DType::F32);
  ensure_workspace(f, m, tc, f->stream);
}

static void need(const DevBuf& b, size_t bytes, const char* what) {
  RISP_CHECK(b.bytes() >= bytes, RISP_E_STATE, std::string("sigma workspace too small: ") + what);
}

static void need(const WsView& b, size_t bytes, const char* what) {
  RISP_CHECK(b.bytes() >= bytes, RISP_E_STATE, std::string("sigma workspace too small: ") + what);
}
// The workspaces of one sigma call and the byte budget of one exchange chunk (which fixes the
// auxiliary functions per chunk, hence the summation order).
struct SigmaWs {
  WsView y, ybf, xbf, xw, mt, k, split;
  int64_t mt_budget = kMtBudget;
};

static unsigned grid_1d(int64_t n) { return (unsigned)std::min<int64_t>(ceil_div(n, 256), 1 << 16); }

// Dp[m][q] = D[m][prow[q]][pcol[q]] (0 for padding): dense AO matrices gathered into the packed
// order of one auxiliary function's integrals
__global__ void k_pack_dense(const double* __restrict__ D, int nao, const int* __restrict__ prow,
                             const int* __restrict__ pcol, int64_t S, int mg, double* __restrict__ Dp) {
  const int64_t n2 = (int64_t)nao * nao, total = (int64_t)mg * S;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(t / S);
    const int64_t q = t % S;
    const int nu = pcol[q];
    Dp[t] = nu >= 0 ? D[m * n2 + (int64_t)prow[q] * nao + nu] : 0.0;
  }
}

// U[m][prow[q]][pcol[q]] = Up[m][q] for the packed positions that hold a pair; every kept pair (mu, nu)
// has exactly one position (in mu's group), the other elements of U are zero beforehand
__global__ void k_unpack_dense(const double* __restrict__ Up, int nao, const int* __restrict__ prow,
                               const int* __restrict__ pcol, int64_t S, int mg, double* __restrict__ U) {
  const int64_t n2 = (int64_t)nao * nao, total = (int64_t)mg * S;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(t / S);
    const int64_t q = t % S;
    const int nu = pcol[q];
    if (nu >= 0) U[m * n2 + (int64_t)prow[q] * nao + nu] = Up[t];
  }
}

// Coulomb term by the AO-density route (section on on-the-fly Coulomb evaluation), FP64 throughout,
// for groups of mg trial vectors:
//   D_m = C_occ X_m C_vir^T;  R_Q = sum_(mu nu) (mu nu|Q) D_m,mu nu;  R~ = L^-T L^-1 R;
//   U_m = sum_P (mu nu|P) R~_P;  sigma_m = 2 C_occ^T U_m C_vir.
// (mu nu|P) is regenerated over the screened pairs in each of the two passes; it is symmetric in
// (mu, nu), so D_m needs no symmetrisation. int3c synchronises the stream.
static void coulomb_ao(risp_factors* f, int m, const void* X, DType tv, void* sig, int pb, hipStream_t s) {
  const int nao = f->nao, nocc = f->nocc, nvir = f->nvir, nJ = f->naux_j;
  const int64_t ov = (int64_t)nocc * nvir, n2 = (int64_t)nao * nao;
  const size_t vsz = dtype_size(tv);
  const int nchunk = (int)f->ao_s0.size() - 1;
  const int mgmax = std::min(m, f->ao_mg);
  need(f->ws_ao_t, (size_t)mgmax * nocc * nao * 8, "AO half-transformed block");
  need(f->ws_ao_d, (size_t)mgmax * n2 * 8, "AO densities");
  const Partners& pk = f->ao_partners;
  const int64_t S = pk.S;
  need(f->ws_ao_v, (size_t)f->ao_max_f * S * 8, "AO integral chunk");
  need(f->ws_ao_p, (size_t)mgmax * S * 8, "packed AO densities");
  need(f->ws_ao_r, 2 * (size_t)nJ * mgmax * 8, "AO auxiliary vectors");
  double* Dp = f->ws_ao_p.as<double>();  // packed D_m in pass 1, packed U_m in pass 2
  double* G = f->ws_ao_t.as<double>();
  double* D = f->ws_ao_d.as<double>();  // D_m in pass 1, U_m in pass 2
  double* V = f->ws_ao_v.as<double>();
  double* R = f->ws_ao_r.as<double>();  // [nJ][mg]
  double* Yr = R + (size_t)nJ * mgmax;  // [nJ][mg]
  const double* Linv = f->linv_j.as<double>();
  for (int g0 = 0; g0 < m; g0 += mgmax) {
    const int mg = std::min(mgmax, m - g0);
    {
      PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_Y,
                    2.0 * mg * ((double)ov * nao + (double)nocc * n2 + (double)nJ * S + 2.0 * nJ * nJ),
                    (double)vsz * mg * ov + 8.0 * ((double)nJ * S + 2.0 * mg * S + mg * n2 + (double)nJ * nJ));
      // G[m][nu][i] = sum_a C_vir[nu][a] X[m][i][a]
      Gemm a = g64(nao, nocc, nvir);
      a.A = f->cv_t.get();
      a.lda = nao;
      a.a_kc = false;
      a.mem_b = tv;
      a.B = static_cast<const char*>(X) + (size_t)g0 * ov * vsz;
      a.ldb = nvir;
      a.sb2 = ov;
      a.C = G;
      a.ldc = nocc;
      a.sc2 = (int64_t)nao * nocc;
      a.nb2 = mg;
      gemm(a, nullptr, s);
      // D[m][mu][nu] = sum_i C_occ[mu][i] G[m][nu][i] (both operands contiguous along i)
      Gemm b = g64(nao, nao, nocc);
      b.A = f->co.get();
      b.lda = nocc;
      b.B = G;
      b.ldb = nocc;
      b.sb2 = (int64_t)nao * nocc;
      b.C = D;
      b.ldc = nao;
      b.sc2 = n2;
      b.nb2 = mg;
      gemm(b, nullptr, s);
      // D_m in the packed order of the integrals (each kept pair (mu, nu) once per orientation)
      k_pack_dense<<<grid_1d((int64_t)mg * S), 256, 0, s>>>(D, nao, pk.prow.as<int>(), pk.pcol.as<int>(), S, mg,
                                                          Dp);
      RISP_LAUNCHED();
      // R[Q][m] = sum_(mu nu) (mu nu|Q) D[m][mu nu] over the kept pairs, chunk by chunk
      for (int c = 0; c < nchunk; ++c) {
        const int nf = f->ao_f0[c + 1] - f->ao_f0[c];
        const PackMap pm = pk.map_fmajor(nf);
        int3c(f->ao_sh, f->pairs, f->auxj_sh, f->ao_s0[c], f->ao_s0[c + 1], f->j_op, f->ctx->boys.as<double>(), V, s,
              &pm);
        Gemm r = g64(nf, mg, (int)std::min<int64_t>(S, INT32_MAX));
        RISP_CHECK(S < INT32_MAX, RISP_E_SHAPE, "packed integrals of one auxiliary function exceed 2^31 elements");
        r.A = V;
        r.lda = S;
        r.B = Dp;
        r.ldb = S;
        r.C = R + (size_t)f->ao_f0[c] * mg;
        r.ldc = mg;
        r.ksplit = std::min(kMaxSplit, gemm_auto_split(r));
        if (r.ksplit > 1) need(f->ws_split, gemm_workspace_bytes(r), "split-K (AO Coulomb)");
        gemm(r, r.ksplit > 1 ? f->ws_split.get() : nullptr, s);
      }
      // R~ = L^-T (L^-1 R)
      Gemm l1 = g64(nJ, mg, nJ);
      l1.A = Linv;
      l1.lda = nJ;
      l1.B = R;
      l1.ldb = mg;
      l1.b_kc = false;
      l1.C = Yr;
      l1.ldc = mg;
      gemm(l1, nullptr, s);
      Gemm l2 = g64(nJ, mg, nJ);
      l2.A = Linv;
      l2.lda = nJ;
      l2.a_kc = false;
      l2.B = Yr;
      l2.ldb = mg;
      l2.b_kc = false;
      l2.C = R;
      l2.ldc = mg;
      gemm(l2, nullptr, s);
    }
    PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_J,
                  2.0 * mg * ((double)nJ * S + (double)nocc * n2 + (double)ov * nao),
                  8.0 * ((double)nJ * S + 2.0 * mg * S + mg * n2) + (double)vsz * mg * ov);
    // U[m][mu nu] = sum_P R~[P][m] (mu nu|P) over the kept pairs, chunk by chunk in the packed order,
    // then into the dense U (which overwrites D; the screened-out elements are zero)
    for (int c = 0; c < nchunk; ++c) {
      const int nf = f->ao_f0[c + 1] - f->ao_f0[c];
      const PackMap pm = pk.map_fmajor(nf);
      int3c(f->ao_sh, f->pairs, f->auxj_sh, f->ao_s0[c], f->ao_s0[c + 1], f->j_op, f->ctx->boys.as<double>(), V, s,
            &pm);
      Gemm u = g64(mg, (int)S, nf);
      u.A = R + (size_t)f->ao_f0[c] * mg;
      u.lda = mg;
      u.a_kc = false;
      u.B = V;
      u.ldb = S;
      u.b_kc = false;
      u.C = Dp;
      u.ldc = S;
      u.beta = c > 0 ? 1.0 : 0.0;
      gemm(u, nullptr, s);
    }
    fill_zero(D, (size_t)mg * n2 * 8, s);
    k_unpack_dense<<<grid_1d((int64_t)mg * S), 256, 0, s>>>(Dp, nao, pk.prow.as<int>(), pk.pcol.as<int>(), S, mg,
                                                            D);
    RISP_LAUNCHED();
    // H[m][i][nu] = sum_mu C_occ[mu][i] U[m][mu][nu], U read as U[m][nu][mu] (symmetric: both
    // orientations of a kept pair hold the same integrals and coefficients), so both operands are
    // contiguous along mu
    Gemm h = g64(nocc, nao, nao);
    h.A = f->co_t.get();
    h.lda = nao;
    h.B = D;
    h.ldb = nao;
    h.sb2 = n2;
    h.C = G;
    h.ldc = nao;
    h.sc2 = (int64_t)nocc * nao;
    h.nb2 = mg;
    gemm(h, nullptr, s);
    // sigma[m][i][a] = 2 sum_nu H[m][i][nu] C_vir[nu][a]
    Gemm j = g64(nocc, nvir, nao);
    j.tout = tv;
    j.A = G;
    j.lda = nao;
    j.sa2 = (int64_t)nocc * nao;
    j.B = f->cv_t.get();
    j.ldb = nao;
    j.C = static_cast<char*>(sig) + (size_t)g0 * ov * vsz;
    j.ldc = nvir;
    j.sc2 = ov;
    j.nb2 = mg;
    j.alpha = 2.0;
    gemm(j, nullptr, s);
  }
}

// coulomb_only: stop after the Coulomb term (sig = 2 J X, no diagonal, no exchange)
static void sigma_run(risp_factors* f, int m, const void* X, void* sig, bool use_f32, hipStream_t s, const SigmaWs& w,
                      bool coulomb_only = false, bool x_bf16 = false) {
  const bool bf = f->precision == RISP_BF16 && !use_f32;
  const DType tc = f->precision == RISP_FP64 ? DType::F64 : (bf ? DType::BF16 : DType::F32);
  const DType tv = f->precision == RISP_FP64 ? DType::F64 : DType::F32;  // X / sigma type
  const DType tacc = tc == DType::F64 ? DType::F64 : DType::F32;
  const int pb = RISP_NPHASE * (bf ? RISP_BF16 : (tc == DType::F32 ? RISP_FP32 : RISP_FP64));  // profile slots
  const int64_t ov = (int64_t)f->nocc * f->nvir;
  const int nJ = f->naux_j;
  const int64_t ldt = f->ld_ia;  // padded row stride of T_ia
  // correction-pass arithmetic of BF16 factors: FP32 Coulomb, split-BF16 exchange; coul32: the BF16
  // stage forms its Coulomb term from the FP32 copy of T_ia as well
  const bool split = f->precision == RISP_BF16 && use_f32;
  const bool c32 = split || (bf && f->coul32);
  const void* Tia = c32 ? f->t_ia32.get() : f->t_ia.get();
  const void* Tij = f->t_ij.get();
  const void* Tab = f->t_ab.get();
  const size_t esz = dtype_size(tc);
  if (f->j_mode == RISP_J_AO_DIRECT) {
    coulomb_ao(f, m, X, tv, sig, pb, s);
  } else if (bf && !c32) {
    need(w.xbf, (size_t)m * ldt * 2, "X (BF16)");
    need(w.ybf, (size_t)kCoulombMaxM * pad_to(nJ, 32) * 2, "Yt (BF16)");
    // BF16 copy of X with the row stride of T_ia (zero padding), then the two skinny passes
    {
      PhaseScope po(f->ctx, s, pb + RISP_PHASE_OTHER, 0.0, 6.0 * m * ov);
      store_rows_padded(X, DType::F32, ov, m, ov, w.xbf.get(), DType::BF16, ldt, nullptr, 1, 1, s);
    }
    const int nJp = (int)pad_to(nJ, 32);
    for (int g0 = 0; g0 < m; g0 += kCoulombMaxM) {
      const int mg = std::min(kCoulombMaxM, m - g0);
      {
        // pass 1: Yt[m][P] = s_P^2 sum_ia T_ia[P][ia] X[m][ia]   (s_P^2 undoes the storage scale)
        PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_Y, 2.0 * nJ * (double)ov * mg,
                      2.0 * ((double)nJ * ov + (double)mg * ov) + 4.0 * nJ * mg);
        coulomb_y_bf16(static_cast<const uint16_t*>(Tia), nJ, ldt,
                       static_cast<const uint16_t*>(w.xbf.get()) + (size_t)g0 * ldt, mg,
                       f->scale_ia2.as<float>(), w.split.as<float>(), w.split.bytes(),
                       static_cast<uint16_t*>(w.ybf.get()), nJp, s);
      }
      {
        // pass 2: sigma[m][ia] = 2 sum_P Yt[m][P] T_ia[P][ia]
        PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_J, 2.0 * nJ * (double)ov * mg,
                      2.0 * (double)nJ * ov + 4.0 * (double)mg * ov);
        coulomb_j_bf16(static_cast<const uint16_t*>(Tia), nJ, ldt, ov,
                       static_cast<const uint16_t*>(w.ybf.get()), nJp, mg, 2.0f,
                       static_cast<float*>(sig) + (size_t)g0 * ov, s);
      }
    }
  } else if (tc == DType::F32 || c32) {
    // FP32 copy of X with the row stride of T_ia (zero padding), then the two skinny FP32 passes
    need(w.xbf, (size_t)m * ldt * 4, "X (padded)");
    need(w.ybf, (size_t)kCoulombMaxM * pad_to(nJ, 32) * 4, "Yt");
    {
      PhaseScope po(f->ctx, s, pb + RISP_PHASE_OTHER, 0.0, 8.0 * m * ov);
      store_rows_padded(X, DType::F32, ov, m, ov, w.xbf.get(), DType::F32, ldt, nullptr, 1, 1, s);
    }
    const int nJp = (int)pad_to(nJ, 32);
    for (int g0 = 0; g0 < m; g0 += kCoulombMaxM) {
      const int mg = std::min(kCoulombMaxM, m - g0);
      {
        PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_Y, 2.0 * nJ * (double)ov * mg,
                      4.0 * ((double)nJ * ov + (double)mg * ov) + 4.0 * nJ * mg);
        coulomb_y_f32(static_cast<const float*>(Tia), nJ, ldt, w.xbf.as<float>() + (size_t)g0 * ldt, mg,
                      w.split.as<float>(), w.split.bytes(), w.ybf.as<float>(), nJp, s);
      }
      {
        PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_J, 2.0 * nJ * (double)ov * mg,
                      4.0 * (double)nJ * ov + 4.0 * (double)mg * ov);
        coulomb_j_f32(static_cast<const float*>(Tia), nJ, ldt, ov, w.ybf.as<float>(), nJp, mg, 2.0f,
                      static_cast<float*>(sig) + (size_t)g0 * ov, s);
      }
    }
  } else {
    need(w.y, (size_t)nJ * m * dtype_size(tacc), "Y");
    // Coulomb pass 1: Y[P][m] = sum_ia T_ia[P][ia] X[m][ia]   (split over ia)
    {
      PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_Y, 2.0 * nJ * (double)ov * m,
                    (double)esz * ((double)nJ * ov + (double)m * ov) + 4.0 * nJ * m);
      Gemm g;
      g.M = nJ;
      g.N = m;
      g.K = (int)ov;
      RISP_CHECK(ov < (1ll << 31), RISP_E_SHAPE, "nocc*nvir too large");
      g.tin = tc;
      g.tout = tacc;
      g.A = Tia;
      g.lda = ldt;
      g.B = X;
      g.ldb = ov;
      g.C = w.y.get();
      g.ldc = m;
      g.ksplit = std::min(kMaxSplit, gemm_auto_split(g));
      while (g.ksplit > 1 && gemm_workspace_bytes(g) > w.split.bytes()) --g.ksplit;
      need(w.split, gemm_workspace_bytes(g), "split-K");
      gemm(g, w.split.get(), s);
    }
    // Coulomb pass 2: sigma[m][ia] = 2 sum_P Y[P][m] T_ia[P][ia]
    {
      PhaseScope ps(f->ctx, s, pb + RISP_PHASE_COULOMB_J, 2.0 * nJ * (double)ov * m,
                    (double)esz * ((double)nJ * ov + (double)nJ * m) + (double)dtype_size(tv) * m * ov);
      Gemm g;
      g.M = m;
      g.N = (int)ov;
      g.K = nJ;
      g.tin = tc;
      g.tout = tv;
      g.A = w.y.get();  // A[mm][P] = Y[P][mm]
      g.lda = m;
      g.a_kc = false;
      g.B = Tia;  // B[ia][P] = T[P][ia]
      g.ldb = ldt;
      g.b_kc = false;
      g.C = sig;
      g.ldc = ov;
      g.alpha = 2.0;
      gemm(g, nullptr, s);
    }
  }
  if (coulomb_only) return;
  // exchange inside the window
  const int nK = f->naux_k, nok = f->nok, nvk = f->nvk;
  const bool exch = nK > 0 && nok > 0 && nvk > 0;
  if (exch) {
    const int nokp = f->nokp, nvkp = f->nvkp;
    const size_t csz = dtype_size(tc);
    // P-chunk from the budget rule alone (not from the workspace capacity, which depends on earlier
    // calls), so the summation order depends only on the inputs
    const int64_t per_p = (int64_t)m * nvk * nokp;
    const int pc = (int)mt_chunk(nK, per_p, (int64_t)csz, w.mt_budget);
    need(w.mt, (size_t)per_p * pc * csz, "exchange intermediate");
    need(w.xw, (size_t)m * nokp * nvkp * csz, "Xw");
    need(w.k, (size_t)m * nok * nvk * dtype_size(tacc), "K");
    const size_t nxw = (size_t)m * nokp * nvkp;  // elements of one window block
    const size_t fsz = split ? 2 : csz;  // bytes per stored factor element (split: the BF16 hi part)
    {
      // window block of X, rows and columns padded with zeros ([m][nokp][nvkp]); split mode: hi and
      // lo BF16 blocks one after the other
      PhaseScope po(f->ctx, s, pb + RISP_PHASE_OTHER, 0.0,
                    (double)m * nok * nvk * dtype_size(tv) + (double)m * nokp * nvkp * csz);
      if (split)
        gather_window_split(static_cast<const float*>(X), m, f->nocc, f->nvir, f->occ_k.as<int>(), nok,
                            f->vir_k.as<int>(), nvk, w.xw.get(), w.xw.as<uint16_t>() + nxw, nokp, nvkp, s);
      else
        gather_window(X, tv, m, f->nocc, f->nvir, f->occ_k.as<int>(), nok, f->vir_k.as<int>(), nvk,
                      w.xw.get(), tc, nokp, nvkp, s);
    }
    for (int P0 = 0; P0 < nK; P0 += pc) {
      const int np = std::min(pc, nK - P0);
      // product 1, one GEMM per auxiliary function P over all trial vectors at once:
      //   Mt[m][a][p][j] = s_P sum_b T_ab[P][a][b] Xw[m][j][b]   (rows a, columns (m, j))
      std::optional<PhaseScope> ps1(std::in_place, f->ctx, s, pb + RISP_PHASE_EXCHANGE_M,
                                    2.0 * m * np * (double)nvk * nvk * nok,
                                    (double)csz * ((double)np * nvk * nvk + (double)m * nok * nvk +
                                                   (double)m * np * nvk * nok));
      Gemm g1;
      g1.M = nvk;
      g1.N = m * nokp;
      g1.K = nvkp;  // the padding columns of T_ab and Xw are zero
      g1.tin = split ? DType::BF16 : tc;
      g1.tout = split ? DType::BF16 : tc;
      g1.A = static_cast<const char*>(Tab) + (size_t)P0 * nvk * nvkp * fsz;
      g1.lda = nvkp;
      g1.B = w.xw.get();
      g1.ldb = nvkp;
      g1.C = w.mt.get();
      g1.ldc = (int64_t)np * nokp;
      g1.nb2 = np;
      g1.sa2 = (int64_t)nvk * nvkp;
      g1.sc2 = nokp;
      g1.n_inner = nokp;
      g1.sc_outer = (int64_t)nvk * np * nokp;
      g1.batch_scale = (bf || split) ? f->scale_k.as<float>() + P0 : nullptr;
      if (split) {
        // (hi, hi) + (lo, hi) + (hi, lo) in one accumulation; the intermediate as hi + lo halves (BF16
        // valued X: its lo block is zero and the third pair is left out)
        g1.npair = x_bf16 ? 2 : 3;
        g1.A2 = static_cast<const uint16_t*>(f->t_ab_lo.get()) + (size_t)P0 * nvk * nvkp;
        g1.A3 = g1.A;
        g1.B2 = g1.B;
        g1.B3 = w.xw.as<uint16_t>() + nxw;
        g1.C_lo = w.mt.as<uint16_t>() + (size_t)per_p * pc;
      }
      gemm(g1, nullptr, s);
      ps1.reset();
      // product 2, one GEMM over the chunk: K[m][i][a] (+)= sum_(p, j) T_ij[i][P0 + p][j] Mt[m][a][p][j]
      // (rows i, columns (m, a); padding terms are zero)
      PhaseScope ps2(f->ctx, s, pb + RISP_PHASE_EXCHANGE_K, 2.0 * m * (double)nok * np * nok * nvk,
                     (double)csz * ((double)nok * np * nok + (double)m * np * nvk * nok) +
                         (double)dtype_size(tacc) * m * nok * nvk * (P0 > 0 ? 2.0 : 1.0));
      Gemm g2;
      g2.M = nok;
      g2.N = m * nvk;
      g2.K = np * nokp;
      g2.tin = split ? DType::BF16 : tc;
      g2.tout = tacc;
      g2.A = static_cast<const char*>(Tij) + (size_t)P0 * nokp * fsz;
      g2.lda = (int64_t)nK * nokp;
      g2.B = w.mt.get();
      g2.ldb = (int64_t)np * nokp;
      g2.C = w.k.get();
      g2.ldc = nvk;
      g2.n_inner = nvk;
      g2.sc_outer = (int64_t)nok * nvk;
      g2.beta = P0 > 0 ? 1.0 : 0.0;
      if (split) {
        g2.npair = 3;
        g2.A2 = static_cast<const uint16_t*>(f->t_ij_lo.get()) + (size_t)P0 * nokp;
        g2.A3 = g2.A;
        g2.B2 = g2.B;
        g2.B3 = w.mt.as<uint16_t>() + (size_t)per_p * pc;
      }
      g2.ksplit = std::max(1, std::min(kMaxSplitK, gemm_auto_split(g2)));
      while (g2.ksplit > 1 && gemm_workspace_bytes(g2) > w.split.bytes()) --g2.ksplit;
      if (g2.ksplit > 1) need(w.split, gemm_workspace_bytes(g2), "split-K (exchange)");
      gemm(g2, g2.ksplit > 1 ? w.split.get() : nullptr, s);
    }
  }
  PhaseScope po(f->ctx, s, pb + RISP_PHASE_OTHER, (double)m * ov * 3.0,
                (double)m * ov * dtype_size(tv) * 3.0 + (double)m * nok * nvk * dtype_size(tacc));
  combine_sigma(sig, X, tv, f->de64.as<double>(), f->de32.as<float>(), m, f->nocc, f->nvir,
                exch ? w.k.get() : nullptr, tacc, f->pos_o.as<int>(), f->pos_v.as<int>(), nok, nvk, s);
}


void sigma(risp_factors* f, int m, const void* X, void* sig, bool use_f32, hipStream_t s, bool x_bf16) {
  if (m <= 0) return;
  const bool bf = f->precision == RISP_BF16 && !use_f32;
  const DType tc = f->precision == RISP_FP64 ? DType::F64 : (bf ? DType::BF16 : DType::F32);
  ensure_workspace(f, m, tc, s);
  SigmaWs w;
  w.y = {f->ws_y.get(), f->ws_y.bytes()};
  w.ybf = {f->ws_ybf.get(), f->ws_ybf.bytes()};
  w.xbf = {f->ws_xbf.get(), f->ws_xbf.bytes()};
  w.xw = {f->ws_xw.get(), f->ws_xw.bytes()};
  w.mt = {f->ws_mt.get(), f->ws_mt.bytes()};
  w.k = {f->ws_k.get(), f->ws_k.bytes()};
  w.split = {f->ws_split.get(), f->ws_split.bytes()};
  sigma_run(f, m, X, sig, use_f32, s, w, false, x_bf16 && use_f32);
}

// P = A V + 2 J V - KB V and M = A V - 2 J V + KB V, where on entry P holds A V and M holds 2 J V
template <typename T>
__global__ void k_combine_full(T* __restrict__ P, T* __restrict__ M, const T* __restrict__ KB, int m, int nocc,
                               int nvir, const int* __restrict__ po, const int* __restrict__ pv, int nok, int nvk) {
  const int64_t ov = (int64_t)nocc * nvir, total = (int64_t)m * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ia = t % ov;
    const int mm = (int)(t / ov);
    const int i = (int)(ia / nvir), a = (int)(ia % nvir);
    T kb = (T)0;
    if (KB) {
      const int ik = po[i], ak = pv[a];
      if (ik >= 0 && ak >= 0) kb = KB[((int64_t)mm * nok + ik) * nvk + ak];
    }
    const T av = P[t], j2 = M[t];
    P[t] = av + j2 - kb;
    M[t] = av - j2 + kb;
  }
}

void sigma_full(risp_factors* f, int m, const void* V, void* P, void* M, hipStream_t s) {
  RISP_CHECK(f->full, RISP_E_STATE, "factors were built without the full-TDDFT exchange factor");
  RISP_CHECK(f->precision == RISP_FP64 || f->precision == RISP_FP32, RISP_E_ARG, "full TDDFT: FP64 or FP32 factors");
  if (m <= 0) return;
  const DType tc = f->precision == RISP_FP64 ? DType::F64 : DType::F32;
  const size_t csz = dtype_size(tc);
  // P = A V (leaves the window block of V in ws_xw), M = 2 J V
  sigma(f, m, V, P, false, s);
  {
    SigmaWs w;
    w.y = {f->ws_y.get(), f->ws_y.bytes()};
    w.ybf = {f->ws_ybf.get(), f->ws_ybf.bytes()};
    w.xbf = {f->ws_xbf.get(), f->ws_xbf.bytes()};
    w.split = {f->ws_split.get(), f->ws_split.bytes()};
    sigma_run(f, m, V, M, false, s, w, true);
  }
  const int nK = f->naux_k, nok = f->nok, nvk = f->nvk, nokp = f->nokp, nvkp = f->nvkp;
  const bool exch = nK > 0 && nok > 0 && nvk > 0;
  if (exch) {
    // KB[m][i][a] = sum_(P, j) H[m][i][P][j] Txt[a][P][j] with H[m][i][P][j] = sum_b Tx[P][i][b] Vw[m][j][b]
    const int64_t per_h = (int64_t)m * nok * nokp;  // elements of H per auxiliary function
    const int pc = (int)mt_chunk(nK, per_h, (int64_t)csz);
    DevBuf H((size_t)per_h * pc * csz);
    need(f->ws_xw, (size_t)m * nokp * nvkp * csz, "Xw");
    need(f->ws_k, (size_t)m * nok * nvk * csz, "KB");
    for (int P0 = 0; P0 < nK; P0 += pc) {
      const int np = std::min(pc, nK - P0);
      Gemm g1;  // rows i, columns (m, j), one product per auxiliary function
      g1.M = nok;
      g1.N = m * nokp;
      g1.K = nvkp;
      g1.tin = g1.tout = tc;
      g1.A = static_cast<const char*>(f->t_x.get()) + (size_t)P0 * nok * nvkp * csz;
      g1.lda = nvkp;
      g1.sa2 = (int64_t)nok * nvkp;
      g1.B = f->ws_xw.get();
      g1.ldb = nvkp;
      g1.C = H.get();
      g1.ldc = (int64_t)np * nokp;
      g1.nb2 = np;
      g1.sc2 = nokp;
      g1.n_inner = nokp;
      g1.sc_outer = (int64_t)nok * np * nokp;
      gemm(g1, nullptr, s);
      Gemm g2;  // rows (m, i), columns a, contraction over (p, j) of the chunk
      g2.M = m * nok;
      g2.N = nvk;
      g2.K = np * nokp;
      g2.tin = g2.tout = tc;
      g2.A = H.get();
      g2.lda = (int64_t)np * nokp;
      g2.B = static_cast<const char*>(f->t_xt.get()) + (size_t)P0 * nokp * csz;
      g2.ldb = (int64_t)nK * nokp;
      g2.C = f->ws_k.get();
      g2.ldc = nvk;
      g2.beta = P0 > 0 ? 1.0 : 0.0;
      gemm(g2, nullptr, s);
    }
  }
  const int64_t total = (int64_t)m * f->nocc * f->nvir;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 16);
  if (tc == DType::F64)
    k_combine_full<double><<<grid, 256, 0, s>>>(static_cast<double*>(P), static_cast<double*>(M),
                                                exch ? f->ws_k.as<double>() : nullptr, m, f->nocc, f->nvir,
                                                f->pos_o.as<int>(), f->pos_v.as<int>(), nok, nvk);
  else
    k_combine_full<float><<<grid, 256, 0, s>>>(static_cast<float*>(P), static_cast<float*>(M),
                                               exch ? f->ws_k.as<float>() : nullptr, m, f->nocc, f->nvir,
                                               f->pos_o.as<int>(), f->pos_v.as<int>(), nok, nvk);
  RISP_LAUNCHED();
  RISP_HIP(hipStreamSynchronize(s));  // H dies at return
}

// Lays the sigma workspaces of m vectors (stored-precision products) out in [base, base + cap),
// each piece 256-byte aligned: Y or (Yt, padded X); the window block and the exchange accumulator;
// then, of what is left, three quarters for the exchange intermediate (whole auxiliary functions,
// at least one) and the rest for split-K partial sums (at least what the Coulomb pass needs).
// Returns 0 when it fits, else the bytes of the smallest layout.
static size_t carve_scratch(const risp_factors* f, int m, SigmaWs& w, char* base, size_t cap) {
  const DType tc = f->precision == RISP_FP64 ? DType::F64 : (f->precision == RISP_BF16 ? DType::BF16 : DType::F32);
  const size_t csz = dtype_size(tc), acc = tc == DType::F64 ? 8 : 4;
  const int nJ = f->naux_j;
  auto up = [](size_t n) { return (n + 255) / 256 * 256; };
  size_t off = 0;
  auto take = [&](WsView& v, size_t bytes) {
    v = {base && bytes ? base + off : nullptr, bytes};
    off += up(bytes);
  };
  size_t split_min = 0;
  if (tc == DType::F64) {
    take(w.y, (size_t)nJ * m * acc);
  } else {
    const size_t xe = (tc == DType::BF16 && !f->coul32) ? 2 : 4;
    take(w.ybf, (size_t)kCoulombMaxM * pad_to(nJ, 32) * xe + 16);
    take(w.xbf, (size_t)m * f->ld_ia * xe + 16);
    split_min = coulomb_y_workspace(nJ, std::min(m, kCoulombMaxM), f->ld_ia);
  }
  const bool exch = f->naux_k > 0 && f->nok > 0 && f->nvk > 0;
  const size_t per_p = exch ? (size_t)m * f->nvk * f->nokp * csz : 0;  // intermediate bytes per function
  if (exch) {
    take(w.xw, (size_t)m * f->nokp * f->nvkp * csz);
    take(w.k, (size_t)m * f->nok * f->nvk * acc);
  }
  const size_t smallest = off + up(per_p) + up(split_min);
  if (smallest > cap) return smallest;
  size_t rest = cap - off;
  if (exch) {
    const size_t share = std::max(per_p, (rest - up(split_min)) / 4 * 3);
    const int64_t pc = std::min<int64_t>(f->naux_k, (int64_t)(share / per_p));
    take(w.mt, (size_t)pc * per_p);
    w.mt_budget = (int64_t)(pc * per_p);
    rest = cap - off;
  }
  w.split = {base ? base + off : nullptr, rest};
  return 0;
}

size_t sigma_scratch_need(const risp_factors* f, int m, size_t cap) {
  SigmaWs w;
  return carve_scratch(f, m, w, nullptr, cap);
}

void sigma_scratch(risp_factors* f, int m, const void* X, void* sig, void* base, size_t cap, hipStream_t s) {
  if (m <= 0) return;
  RISP_CHECK(f->j_mode == RISP_J_MO, RISP_E_ARG,
             "the scratch-buffer sigma supports the stored-factor Coulomb route only");
  SigmaWs w;
  const size_t need_bytes = carve_scratch(f, m, w, static_cast<char*>(base), cap);
  RISP_CHECK(need_bytes == 0, RISP_E_SHAPE,
             "sigma of " + std::to_string(m) + " vectors needs at least " + std::to_string(need_bytes) +
                 " bytes of scratch; the fixed scratch holds " + std::to_string(cap));
  sigma_run(f, m, X, sig, false, s, w);
}

}  // namespace risp
