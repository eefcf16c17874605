// C ABI of librisp (declared in include/risp.h): argument checks, status codes, context and
// factor objects, and the stage entry points used for validation.
#include <chrono>
#include <map>
#include <mutex>
#include <cstring>
#include <string>

#include "davidson.hpp"
#include "factors.hpp"
#include "integrals.hpp"
#include "linalg.hpp"
#include "properties.hpp"
#include "serve.hpp"

namespace risp {
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace risp

using namespace risp;

namespace {

template <typename Fn>
risp_status guarded(Fn&& fn) {
  try {
    set_last_error("");
    return fn();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return RISP_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return RISP_E_HIP;
  } catch (...) {
    set_last_error("unknown failure");
    return RISP_E_HIP;
  }
}

void use_ctx(const risp_ctx* ctx) {
  RISP_CHECK(ctx != nullptr, RISP_E_ARG, "context is NULL");
  RISP_HIP(hipSetDevice(ctx->device));
}

// Fixed scratch array of the allocation-free sigma entry point. Each device holds its own copy
// (allocated when the code object is loaded, kept until the process ends); host code reaches it only
// through the per-device address from hipGetSymbolAddress, never through the array's name.
__device__ __align__(256) unsigned char scratch[RISP_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of its copy

// address of this device's scratch copy (the device must be current)
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  RISP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  RISP_CHECK(p != nullptr, RISP_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_addr[device] = p;
  return p;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct risp_factors_ext {
  double t_build = 0.0;
};

extern "C" {

const char* risp_last_error(void) { return g_last_error.c_str(); }

risp_status risp_ctx_create(int32_t device, void* hip_stream, risp_ctx** out) {
  return guarded([&]() -> risp_status {
    RISP_CHECK(out != nullptr, RISP_E_ARG, "out is NULL");
    int ndev = 0;
    RISP_HIP(hipGetDeviceCount(&ndev));
    RISP_CHECK(device >= 0 && device < ndev, RISP_E_ARG, "device index out of range");
    RISP_HIP(hipSetDevice(device));
    auto* c = new risp_ctx();
    c->device = device;
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete c;
        throw Error(RISP_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
      }
      c->own_stream = true;
    }
    try {
      std::vector<double> tab;
      boys_table_host(tab);
      c->boys = upload(tab.data(), tab.size(), c->stream);
      RISP_HIP(hipStreamSynchronize(c->stream));
      c->scratch = scratch_address(device);
    } catch (...) {
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      delete c;
      throw;
    }
    *out = c;
    return RISP_OK;
  });
}

risp_status risp_ctx_destroy(risp_ctx* ctx) {
  return guarded([&]() -> risp_status {
    if (!ctx) return RISP_OK;
    (void)hipSetDevice(ctx->device);
    stop_server(ctx);  // finishes resident jobs, drops queued ones
    (void)hipStreamSynchronize(ctx->stream);
    try {
      ctx->clear_phases();
    } catch (...) {
    }
    for (risp_factors* f : ctx->factors) f->ctx = nullptr;  // factors outlive their context detached
    ctx->factors.clear();
    ctx->boys.release();
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return RISP_OK;
  });
}

risp_status risp_ctx_profile(risp_ctx* ctx, int32_t enable, int32_t reset, risp_phase_stat* out) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_HIP(hipStreamSynchronize(ctx->stream));
    ctx->resolve_phases();
    if (out) {
      for (int p = 0; p < RISP_NPHASE_SLOTS; ++p) {
        out[p].launches = ctx->phase[p].launches;
        out[p].ms = ctx->phase[p].ms;
        out[p].flops = ctx->phase[p].flops;
        out[p].bytes = ctx->phase[p].bytes;
      }
    }
    if (reset) ctx->clear_phases();
    ctx->profiling = enable != 0;
    return RISP_OK;
  });
}

risp_status risp_select_aux(const risp_system* sys, const risp_params* prm, int32_t cap, risp_shell* aux_j,
                            int32_t* n_j, risp_shell* aux_k, int32_t* n_k) {
  return guarded([&]() -> risp_status {
    RISP_CHECK(sys && prm && n_j && n_k, RISP_E_ARG, "NULL argument");
    RISP_CHECK(sys->natm > 0 && sys->Z && sys->aux_radius, RISP_E_ARG, "atoms, charges and radii are required");
    RISP_CHECK(prm->theta > 0.0, RISP_E_ARG, "theta must be positive");
    for (int a = 0; a < sys->natm; ++a)
      RISP_CHECK(sys->aux_radius[a] > 0.0, RISP_E_ARG, "auxiliary radius must be positive");
    std::vector<risp_shell> J, K;
    select_aux(sys, prm, J, K);
    RISP_CHECK((int)J.size() <= cap && (int)K.size() <= cap, RISP_E_SHAPE, "cap too small for the auxiliary shells");
    if (aux_j) std::memcpy(aux_j, J.data(), J.size() * sizeof(risp_shell));
    if (aux_k) std::memcpy(aux_k, K.data(), K.size() * sizeof(risp_shell));
    *n_j = (int32_t)J.size();
    *n_k = (int32_t)K.size();
    return RISP_OK;
  });
}

risp_status risp_window(risp_ctx* ctx, int32_t nmo, int32_t nocc, const double* mo_energy, double window_ev,
                        int32_t window_mode, int32_t* occ_k, int32_t* nocc_k, int32_t* vir_k, int32_t* nvir_k) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(mo_energy && occ_k && nocc_k && vir_k && nvir_k, RISP_E_ARG, "NULL argument");
    RISP_CHECK(nocc > 0 && nocc < nmo, RISP_E_SHAPE, "need 0 < nocc < nmo");
    RISP_CHECK(window_mode == RISP_WIN_ABSOLUTE || window_mode == RISP_WIN_FRONTIER, RISP_E_ARG, "bad window_mode");
    hipStream_t s = ctx->stream;
    DevBuf e = upload(mo_energy, nmo, s);
    DevBuf o(nocc * sizeof(int)), v((nmo - nocc) * sizeof(int));
    int no = 0, nv = 0;
    window_sets(e.as<double>(), nmo, nocc, window_ev, window_mode, o.as<int>(), &no, v.as<int>(), &nv, s);
    RISP_HIP(hipMemcpyAsync(occ_k, o.get(), no * sizeof(int), hipMemcpyDeviceToHost, s));
    RISP_HIP(hipMemcpyAsync(vir_k, v.get(), nv * sizeof(int), hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    *nocc_k = no;
    *nvir_k = nv;
    return RISP_OK;
  });
}

static void check_shells(const risp_system* sys, int naux, const risp_shell* aux) {
  RISP_CHECK(sys && sys->natm > 0 && sys->coords && sys->nshell > 0 && sys->shells, RISP_E_ARG,
             "system: atoms and shells are required");
  RISP_CHECK(naux >= 0 && (naux == 0 || aux), RISP_E_ARG, "auxiliary shells missing");
  auto chk = [&](const risp_shell& s) {
    RISP_CHECK(s.l == 0 || s.l == 1, RISP_E_ARG, "only s and p shells are supported");
    RISP_CHECK(s.atom >= 0 && s.atom < sys->natm, RISP_E_ARG, "shell atom index out of range");
    RISP_CHECK(s.exponent > 0.0, RISP_E_ARG, "shell exponent must be positive");
  };
  for (int k = 0; k < sys->nshell; ++k) chk(sys->shells[k]);
  for (int k = 0; k < naux; ++k) chk(aux[k]);
}

risp_status risp_screen(risp_ctx* ctx, const risp_system* sys, int32_t naux_shell, const risp_shell* aux,
                        double tau, int32_t cap, int32_t* pairs, int32_t* npair) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    check_shells(sys, naux_shell, aux);
    RISP_CHECK(naux_shell > 0 && npair && tau >= 0.0, RISP_E_ARG, "bad screening arguments");
    hipStream_t s = ctx->stream;
    DevShells ao, ax;
    upload_shells(ao, sys->coords, sys->shells, sys->nshell, s);
    upload_shells(ax, sys->coords, aux, naux_shell, s);
    const double qaux = std::sqrt(aux_diag_max(ax, ctx->boys.as<double>(), s));
    PairList pl;
    screen_pairs(ao, qaux, tau, true, pl, s);
    *npair = pl.n;
    RISP_CHECK(pl.n <= cap, RISP_E_SHAPE, "cap too small for the kept pairs");
    if (pairs && pl.n > 0) {
      std::vector<int> a(pl.n), b(pl.n);
      RISP_HIP(hipMemcpyAsync(a.data(), pl.a.get(), pl.n * sizeof(int), hipMemcpyDeviceToHost, s));
      RISP_HIP(hipMemcpyAsync(b.data(), pl.b.get(), pl.n * sizeof(int), hipMemcpyDeviceToHost, s));
      RISP_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < pl.n; ++k) {
        pairs[2 * k] = a[k];
        pairs[2 * k + 1] = b[k];
      }
    }
    return RISP_OK;
  });
}

risp_status risp_int2c(risp_ctx* ctx, const risp_system* sys, int32_t naux_shell, const risp_shell* aux,
                       double omega, double* out) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    check_shells(sys, naux_shell, aux);
    RISP_CHECK(out && naux_shell > 0, RISP_E_ARG, "bad arguments");
    hipStream_t s = ctx->stream;
    DevShells ax;
    upload_shells(ax, sys->coords, aux, naux_shell, s);
    Operator op;
    if (omega > 0.0) op = Operator{0.0, 1.0, omega};
    DevBuf V((size_t)ax.nfunc * ax.nfunc * 8);
    int2c(ax, op, ctx->boys.as<double>(), V.as<double>(), s);
    RISP_HIP(hipMemcpyAsync(out, V.get(), V.bytes(), hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    return RISP_OK;
  });
}

risp_status risp_int3c(risp_ctx* ctx, const risp_system* sys, int32_t naux_shell, const risp_shell* aux,
                       int32_t aux_begin, int32_t aux_end, double omega, double tau, double* out) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    check_shells(sys, naux_shell, aux);
    RISP_CHECK(out && naux_shell > 0 && tau >= 0.0, RISP_E_ARG, "bad arguments");
    RISP_CHECK(0 <= aux_begin && aux_begin < aux_end && aux_end <= naux_shell, RISP_E_ARG, "bad auxiliary range");
    hipStream_t s = ctx->stream;
    DevShells ao, ax;
    upload_shells(ao, sys->coords, sys->shells, sys->nshell, s);
    upload_shells(ax, sys->coords, aux, naux_shell, s);
    const double qaux = std::sqrt(aux_diag_max(ax, ctx->boys.as<double>(), s));
    PairList pl;
    screen_pairs(ao, qaux, tau, false, pl, s);
    Operator op;
    if (omega > 0.0) op = Operator{0.0, 1.0, omega};
    int nf = 0;
    for (int k = aux_begin; k < aux_end; ++k) nf += aux[k].l == 0 ? 1 : 3;
    const size_t n = (size_t)nf * ao.nfunc * ao.nfunc;
    DevBuf V(n * 8);
    int3c(ao, pl, ax, aux_begin, aux_end, op, ctx->boys.as<double>(), V.as<double>(), s);
    RISP_HIP(hipMemcpyAsync(out, V.get(), n * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    return RISP_OK;
  });
}

risp_status risp_build_factors(risp_ctx* ctx, const risp_system* sys, const risp_params* prm, risp_factors** out) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(out != nullptr, RISP_E_ARG, "out is NULL");
    auto t0 = std::chrono::steady_clock::now();
    auto* f = new risp_factors();
    try {
      build_factors(ctx, sys, prm, f);
    } catch (...) {
      delete f;
      throw;
    }
    f->t_build = seconds_since(t0);
    ctx->factors.insert(f);
    *out = f;
    return RISP_OK;
  });
}

risp_status risp_factors_query(const risp_factors* f, risp_factors_desc* d) {
  return guarded([&]() -> risp_status {
    RISP_CHECK(f && d, RISP_E_ARG, "NULL argument");
    std::memset(d, 0, sizeof(*d));
    d->nao = f->nao;
    d->nmo = f->nmo;
    d->nocc = f->nocc;
    d->nvir = f->nvir;
    d->naux_j = f->naux_j;
    d->naux_k = f->naux_k;
    d->nocc_k = f->nok;
    d->nvir_k = f->nvk;
    d->npair = f->npair;
    d->precision = f->precision;
    d->bytes = f->bytes();
    d->t_ia = f->t_ia.get();
    d->t_ij = f->naux_k ? f->t_ij.get() : nullptr;
    d->t_ab = f->naux_k ? f->t_ab.get() : nullptr;
    d->t_ij_lo = (f->precision == RISP_BF16 && f->naux_k) ? f->t_ij_lo.get() : nullptr;
    d->t_ab_lo = (f->precision == RISP_BF16 && f->naux_k) ? f->t_ab_lo.get() : nullptr;
    d->scale_ia = f->precision == RISP_BF16 ? f->scale_ia.as<float>() : nullptr;
    d->scale_k = (f->precision == RISP_BF16 && f->naux_k) ? f->scale_k.as<float>() : nullptr;
    d->occ_k = f->occ_k.as<int32_t>();
    d->vir_k = f->vir_k.as<int32_t>();
    d->ld_ia = f->ld_ia;
    d->ld_ij = f->nokp;
    d->ld_ab = f->nvkp;
    d->diag_a = f->diag64.as<double>();
    return RISP_OK;
  });
}

risp_status risp_factors_free(risp_factors* f) {
  return guarded([&]() -> risp_status {
    if (!f) return RISP_OK;
    if (f->ctx) {
      (void)hipSetDevice(f->ctx->device);
      (void)hipStreamSynchronize(f->ctx->stream);
      f->ctx->factors.erase(f);
    }
    delete f;
    return RISP_OK;
  });
}

risp_status risp_sigma(risp_ctx* ctx, const risp_factors* fc, int32_t m, const void* X_dev, void* sigma_dev,
                       int32_t dtype) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(fc != nullptr, RISP_E_ARG, "factors are NULL");
    RISP_CHECK(fc->ctx == ctx, RISP_E_STATE, "factors belong to another context");
    RISP_CHECK(m >= 0, RISP_E_ARG, "m must be non-negative");
    RISP_CHECK(m == 0 || (X_dev && sigma_dev), RISP_E_ARG, "NULL device buffer");
    const int want = fc->precision == RISP_FP64 ? RISP_FP64 : RISP_FP32;
    RISP_CHECK(dtype == want, RISP_E_ARG,
               want == RISP_FP64 ? "FP64 factors take FP64 vectors" : "FP32/BF16 factors take FP32 vectors");
    sigma(const_cast<risp_factors*>(fc), m, X_dev, sigma_dev, false, fc->stream);
    return RISP_OK;
  });
}

risp_status risp_sigma_noalloc(risp_ctx* ctx, const risp_factors* fc, int32_t m, const void* X_dev,
                               void* sigma_dev, int32_t dtype) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(fc != nullptr, RISP_E_ARG, "factors are NULL");
    RISP_CHECK(fc->ctx == ctx, RISP_E_STATE, "factors belong to another context");
    RISP_CHECK(m >= 0, RISP_E_ARG, "m must be non-negative");
    RISP_CHECK(m == 0 || (X_dev && sigma_dev), RISP_E_ARG, "NULL device buffer");
    const int want = fc->precision == RISP_FP64 ? RISP_FP64 : RISP_FP32;
    RISP_CHECK(dtype == want, RISP_E_ARG,
               want == RISP_FP64 ? "FP64 factors take FP64 vectors" : "FP32/BF16 factors take FP32 vectors");
    RISP_CHECK(ctx->scratch != nullptr, RISP_E_STATE, "context has no scratch address");
    // no phase events either: event creation is left out of this path
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    try {
      sigma_scratch(const_cast<risp_factors*>(fc), m, X_dev, sigma_dev, ctx->scratch, RISP_SCRATCH_BYTES,
                    fc->stream);
    } catch (...) {
      ctx->profiling = prof;
      throw;
    }
    ctx->profiling = prof;
    return RISP_OK;
  });
}

risp_status risp_sigma_full(risp_ctx* ctx, const risp_factors* fc, int32_t m, const void* V_dev, void* P_dev,
                            void* M_dev, int32_t dtype) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(fc != nullptr, RISP_E_ARG, "factors are NULL");
    RISP_CHECK(fc->ctx == ctx, RISP_E_STATE, "factors belong to another context");
    RISP_CHECK(m >= 0, RISP_E_ARG, "m must be non-negative");
    RISP_CHECK(m == 0 || (V_dev && P_dev && M_dev), RISP_E_ARG, "NULL device buffer");
    const int want = fc->precision == RISP_FP64 ? RISP_FP64 : RISP_FP32;
    RISP_CHECK(dtype == want, RISP_E_ARG, want == RISP_FP64 ? "FP64 factors take FP64 vectors"
                                                              : "FP32 factors take FP32 vectors");
    sigma_full(const_cast<risp_factors*>(fc), m, V_dev, P_dev, M_dev, fc->stream);
    return RISP_OK;
  });
}

risp_status risp_davidson_full(risp_ctx* ctx, const risp_factors* fc, const risp_dav_opts* opts, double* energies,
                               float* xpy, float* xmy, risp_dav_info* info) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(fc && opts && energies, RISP_E_ARG, "NULL argument");
    RISP_CHECK(fc->ctx == ctx, RISP_E_STATE, "factors belong to another context");
    RISP_CHECK(opts->nx0 == 0, RISP_E_ARG, "initial vectors are not supported by the full-TDDFT solver");
    risp_factors* f = const_cast<risp_factors*>(fc);
    const int64_t ov = (int64_t)f->nocc * f->nvir;
    DavOptions o;
    o.nstates = opts->nstates;
    o.block = opts->block;
    o.max_space = opts->max_space;
    o.max_iter = opts->max_iter > 0 ? opts->max_iter : 200;
    o.tol = opts->tol;
    o.log_tag = (opts->flags & RISP_DAV_VERBOSE) ? "full" : nullptr;
    FullResult r;
    davidson_full(f, o, r);
    const int n = (int)std::min<size_t>(opts->nstates, r.omega.size());
    for (int k = 0; k < n; ++k) energies[k] = r.omega[k];
    for (float* dst : {xpy, xmy}) {
      if (!dst || n == 0) continue;
      std::vector<double> h((size_t)n * ov);
      RISP_HIP(hipMemcpy(h.data(), (dst == xpy ? r.XpY : r.XmY).get(), h.size() * 8, hipMemcpyDeviceToHost));
      for (size_t t = 0; t < h.size(); ++t) dst[t] = (float)h[t];
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iters = r.iters;
      info->restarts = r.restarts;
      info->sigma_vectors = r.sigma_vectors;
      info->converged = r.converged ? 1 : 0;
      info->t_build = f->t_build;
      info->t_sigma = r.t_sigma;
      info->t_subspace = r.t_subspace;
      info->sigma_flops = r.sigma_flops;
      info->hbm_bytes = f->bytes();
      for (size_t k = 0; k < std::min<size_t>(256, r.resid_hist.size()); ++k) info->resid_hist[k] = r.resid_hist[k];
    }
    return r.converged ? RISP_OK : RISP_E_NOTCONV;
  });
}

risp_status risp_properties(risp_ctx* ctx, const risp_system* sys, const double* origin, int32_t nstates,
                            const double* energies, const void* X_dev, double* mu, double* mdip, double* f,
                            double* R) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    validate_system(sys);
    RISP_CHECK(nstates >= 0, RISP_E_ARG, "nstates must be non-negative");
    RISP_CHECK(nstates == 0 || (energies && X_dev && f && R), RISP_E_ARG, "NULL argument");
    hipStream_t s = ctx->stream;
    const double O[3] = {origin ? origin[0] : 0.0, origin ? origin[1] : 0.0, origin ? origin[2] : 0.0};
    DevShells ao;
    upload_shells(ao, sys->coords, sys->shells, sys->nshell, s);
    DevBuf C = upload(sys->mo_coeff, (size_t)sys->nao * sys->nmo, s);
    const int n = nstates;
    DevBuf w = upload(energies ? energies : O, (size_t)std::max(n, 1), s);
    DevBuf T((size_t)std::max(n, 1) * 6 * 8), fd((size_t)std::max(n, 1) * 8), Rd((size_t)std::max(n, 1) * 8);
    transition_properties(ao, C.as<double>(), sys->nao, sys->nmo, sys->nocc, O, n, w.as<double>(),
                          static_cast<const float*>(X_dev), T.as<double>(), fd.as<double>(), Rd.as<double>(), s);
    if (n > 0) {
      std::vector<double> t((size_t)n * 6);
      RISP_HIP(hipMemcpy(t.data(), T.get(), t.size() * 8, hipMemcpyDeviceToHost));
      RISP_HIP(hipMemcpy(f, fd.get(), (size_t)n * 8, hipMemcpyDeviceToHost));
      RISP_HIP(hipMemcpy(R, Rd.get(), (size_t)n * 8, hipMemcpyDeviceToHost));
      for (int k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) {
          if (mu) mu[3 * k + c] = t[6 * k + c];
          if (mdip) mdip[3 * k + c] = t[6 * k + 3 + c];
        }
    }
    return RISP_OK;
  });
}

risp_status risp_spectrum(risp_ctx* ctx, int32_t nstates, const double* energies, const double* strengths,
                          double hwhm, double e0, double de, int32_t npts, double* out) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(nstates >= 0 && npts >= 0, RISP_E_ARG, "negative size");
    RISP_CHECK(hwhm > 0.0, RISP_E_ARG, "hwhm must be positive");
    RISP_CHECK((nstates == 0 || (energies && strengths)) && (npts == 0 || out), RISP_E_ARG, "NULL argument");
    if (npts == 0) return RISP_OK;
    hipStream_t s = ctx->stream;
    const double zero = 0.0;
    DevBuf w = upload(nstates ? energies : &zero, (size_t)std::max(nstates, 1), s);
    DevBuf st = upload(nstates ? strengths : &zero, (size_t)std::max(nstates, 1), s);
    DevBuf o((size_t)npts * 8);
    lorentz_spectrum(w.as<double>(), st.as<double>(), nstates, hwhm, e0, de, npts, o.as<double>(), s);
    RISP_HIP(hipMemcpyAsync(out, o.get(), (size_t)npts * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    return RISP_OK;
  });
}

risp_status risp_davidson(risp_ctx* ctx, const risp_factors* fc, const risp_dav_opts* opts, double* energies,
                          float* vectors, risp_dav_info* info) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(fc && opts && energies, RISP_E_ARG, "NULL argument");
    RISP_CHECK(opts->ncorr >= 0 && opts->correction_ncorr >= 0, RISP_E_ARG, "ncorr must be non-negative");
    RISP_CHECK(fc->ctx == ctx, RISP_E_STATE, "factors belong to another context");
    risp_factors* f = const_cast<risp_factors*>(fc);
    const int64_t ov = (int64_t)f->nocc * f->nvir;
    hipStream_t s = f->stream;
    DavOptions o;
    o.nstates = opts->nstates;
    o.block = opts->block;
    o.max_space = opts->max_space;
    o.max_iter = opts->max_iter > 0 ? opts->max_iter : 200;
    o.tol = opts->tol;
    o.max_corr = opts->ncorr > 0 ? opts->ncorr : opts->nstates;
    o.spill = (opts->flags & RISP_DAV_SPILL) != 0;
    o.olsen = (opts->flags & RISP_DAV_OLSEN) != 0;
    DevBuf x0;
    if (opts->nx0 > 0) {
      RISP_CHECK(opts->x0 != nullptr, RISP_E_ARG, "x0 is NULL");
      std::vector<double> h((size_t)opts->nx0 * ov);
      for (size_t t = 0; t < h.size(); ++t) h[t] = (double)opts->x0[t];
      x0 = upload(h.data(), h.size(), s);
      RISP_HIP(hipStreamSynchronize(s));
      o.x0_dev = x0.as<double>();
      o.nx0 = opts->nx0;
    }
    SigmaFn native = [&](int m, const void* X, void* S) { sigma(f, m, X, S, false, s); };
    const bool correct = f->precision == RISP_BF16 && opts->correction_pass;
    if (opts->flags & RISP_DAV_VERBOSE) o.log_tag = f->precision == RISP_BF16 ? "bf16" : (f->precision == RISP_FP32 ? "fp32" : "fp64");
    DavOptions ob = o;
    if (f->precision == RISP_BF16) {
      // BF16 products bound the attainable residual: stop at the stage tolerance or on a stall
      const double bt = opts->bf16_tol > 0.0 ? opts->bf16_tol : kBf16StageTol;
      if (correct) ob.tol = std::max(o.tol, bt);
      ob.stall_iters = 2;
      ob.stall_below = 10.0 * bt;
    }
    DavResult r;
    davidson(f, ob, native, r);
    int corr_iters = 0;
    double t_corr = 0.0;
    DavResult rc;
    DavResult* fin = &r;
    if (correct && r.krows > 0) {
      // FP32 products from the BF16-converged Ritz vectors: Rayleigh-Ritz, then at most
      // correction_steps FP32 Davidson steps
      auto t0 = std::chrono::steady_clock::now();
      DavOptions oc = o;
      if (oc.log_tag) oc.log_tag = "fp32 correction";
      oc.x0_dev = r.X.as<double>();
      oc.nx0 = r.krows;
      oc.max_iter = 1 + (opts->correction_steps > 0 ? opts->correction_steps : 16);
      oc.max_corr = opts->correction_ncorr > 0 ? opts->correction_ncorr : opts->nstates;
      // BF16-valued basis rows: the split products skip the vector's lo half
      oc.bf16_basis = (opts->flags & RISP_DAV_FP32_BASIS) == 0;
      const bool xb = oc.bf16_basis;
      SigmaFn f32 = [&](int m, const void* X, void* S) { sigma(f, m, X, S, true, s, xb); };
      davidson(f, oc, f32, rc);
      corr_iters = rc.iters;
      t_corr = seconds_since(t0);
      fin = &rc;
    }
    const int ns = std::min<int>(opts->nstates, (int)fin->energies.size());
    for (int k = 0; k < ns; ++k) energies[k] = fin->energies[k];
    if (vectors && ns > 0) {
      std::vector<double> h((size_t)ns * ov);
      RISP_HIP(hipMemcpyAsync(h.data(), fin->X.get(), h.size() * 8, hipMemcpyDeviceToHost, s));
      RISP_HIP(hipStreamSynchronize(s));
      for (size_t t = 0; t < h.size(); ++t) vectors[t] = (float)h[t];
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iters = r.iters;
      info->restarts = r.restarts + rc.restarts;
      info->sigma_vectors = r.sigma_vectors;
      info->converged = fin->converged ? 1 : 0;
      info->correction_iters = corr_iters;
      info->correction_vectors = rc.sigma_vectors;
      info->t_build = f->t_build;
      info->t_sigma = r.t_sigma;
      info->t_subspace = r.t_subspace;
      info->t_correct = t_corr;
      info->t_sigma_correct = rc.t_sigma;
      info->sigma_flops = r.sigma_flops;
      info->sigma_flops_correct = rc.sigma_flops;
      info->hbm_bytes = f->bytes();
      // residual history of the main stage followed by that of the correction stage
      std::vector<double> hist = r.resid_hist;
      hist.insert(hist.end(), rc.resid_hist.begin(), rc.resid_hist.end());
      const size_t nh = std::min<size_t>(256, hist.size());
      for (size_t k = 0; k < nh; ++k) info->resid_hist[k] = hist[k];
    }
    if (!fin->converged) {
      set_last_error("Davidson did not converge within max_iter");
      return (risp_status)RISP_E_NOTCONV;
    }
    return RISP_OK;
  });
}

risp_status risp_serve_config(risp_ctx* ctx, const risp_serve_opts* opts) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(opts != nullptr, RISP_E_ARG, "opts is NULL");
    RISP_CHECK(ctx->server == nullptr, RISP_E_STATE, "serving already started");
    RISP_CHECK(opts->hbm_budget_bytes >= 0 && opts->max_active >= 0, RISP_E_ARG, "negative serving limits");
    ctx->serve_budget = opts->hbm_budget_bytes;
    ctx->serve_max_active = opts->max_active;
    ctx->serve_graphs = opts->use_graphs;
    return RISP_OK;
  });
}

risp_status risp_job_footprint(const risp_system* sys, const risp_params* prm, const risp_dav_opts* opts,
                               int64_t* bytes) {
  return guarded([&]() -> risp_status {
    validate_system(sys);
    RISP_CHECK(prm && bytes, RISP_E_ARG, "NULL argument");
    *bytes = job_footprint(sys, prm, opts);
    return RISP_OK;
  });
}

risp_status risp_submit(risp_ctx* ctx, const risp_system* sys, const risp_params* prm, const risp_dav_opts* opts,
                        uint64_t* job_id) {
  return guarded([&]() -> risp_status {
    use_ctx(ctx);
    RISP_CHECK(job_id != nullptr, RISP_E_ARG, "job_id is NULL");
    *job_id = submit_job(ctx, sys, prm, opts);
    return RISP_OK;
  });
}

risp_status risp_poll(risp_ctx* ctx, uint64_t job_id, risp_result* out) {
  return guarded([&]() -> risp_status {
    RISP_CHECK(ctx && out, RISP_E_ARG, "NULL argument");
    return poll_job(ctx, job_id, out);
  });
}

risp_status risp_device_usage(int64_t* live_bytes, int64_t* peak_bytes, int32_t reset_peak) {
  return guarded([&]() -> risp_status {
    RISP_CHECK(live_bytes && peak_bytes, RISP_E_ARG, "NULL argument");
    if (reset_peak) g_device_usage.peak.store(g_device_usage.live.load());
    *live_bytes = g_device_usage.live.load();
    *peak_bytes = g_device_usage.peak.load();
    return RISP_OK;
  });
}

risp_status risp_serve_stats_get(risp_ctx* ctx, risp_serve_stats* out) {
  return guarded([&]() -> risp_status {
    RISP_CHECK(ctx && out, RISP_E_ARG, "NULL argument");
    serve_stats(ctx, out);
    return RISP_OK;
  });
}

}  // extern "C"
