// Transition properties of the excited states (eq. oscillator_strength, eq. rotator_strength,
// eq. transition, eq. transition_magnetic, dipole-length form, TDA amplitudes) and Lorentzian
// spectra.
//
// AO integrals <mu| r - O |nu> and <mu| (r - O) x nabla |nu> by one-dimensional Obara-Saika
// recurrences (one thread per shell pair, consecutive threads on consecutive ket shells so a row of
// each output matrix is written contiguously); FP64 MFMA products for the MO transform
// r_ia = C_occ^T P C_vir; one split-K product for the transition moments of all states at once
// (sqrt(2) sum_ia r_ia X_nia, the singlet of unit-normalised X); a small kernel for
// f = 2/3 Omega |mu|^2 and R = 1/2 mu . m; one thread per grid point for the spectra.
#include <cmath>

#include "gemm.hpp"
#include "properties.hpp"

namespace risp {

namespace {

// one Cartesian direction of a primitive pair (powers i <= 1 on A, j <= 1 on B): overlap S(i, j),
// moment <i| x - O |j> and ket derivative <i| d/dx |j>, without the Gaussian prefactor
struct Dir {
  double S, M, D;
};
__device__ __forceinline__ Dir dir1(int i, int j, double A, double B, double a, double b, double O) {
  const double p = a + b, P = (a * A + b * B) / p, xa = P - A, xb = P - B, h = 0.5 / p;
  // horizontal recurrence S(i+1, j) = xa S(i, j) + (i S(i-1, j) + j S(i, j-1)) / (2p), same on j
  const double s00 = 1.0, s01 = xb, s02 = xb * xb + h;
  const double s10 = xa, s11 = xa * xb + h, s12 = xa * s02 + 2.0 * h * xb;
  const double sij = i == 0 ? (j == 0 ? s00 : s01) : (j == 0 ? s10 : s11);
  const double sij1 = i == 0 ? (j == 0 ? s01 : s02) : (j == 0 ? s11 : s12);  // S(i, j + 1)
  const double sijm = j == 0 ? 0.0 : (i == 0 ? s00 : s10);                   // S(i, j - 1)
  Dir d;
  d.S = sij;
  d.M = sij1 + (B - O) * sij;  // x - O = (x - B) + (B - O)
  d.D = (double)j * sijm - 2.0 * b * sij1;
  return d;
}

// out [6][nao][nao]: components 0..2 dipole x, y, z; 3..5 (r - O) x nabla x, y, z
__global__ __launch_bounds__(256) void k_prop_ao(const double* __restrict__ sx, const double* __restrict__ sy,
                                                 const double* __restrict__ sz, const double* __restrict__ ex,
                                                 const double* __restrict__ cn, const int* __restrict__ sl,
                                                 const int* __restrict__ soff, int nsh, int64_t nao, double ox,
                                                 double oy, double oz, double* __restrict__ out) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  const int A = blockIdx.y;
  if (B >= nsh) return;
  const double a = ex[A], b = ex[B];
  const double Ac[3] = {sx[A], sy[A], sz[A]}, Bc[3] = {sx[B], sy[B], sz[B]}, Oc[3] = {ox, oy, oz};
  const double p = a + b, mu = a * b / p;
  double r2 = 0.0;
  for (int d = 0; d < 3; ++d) r2 += (Ac[d] - Bc[d]) * (Ac[d] - Bc[d]);
  const double pre = exp(-mu * r2) * (M_PI / p) * sqrt(M_PI / p) * cn[A] * cn[B];
  const int la = sl[A], lb = sl[B];
  const int na = la ? 3 : 1, nb = lb ? 3 : 1;
  const int64_t n2 = nao * nao;
  for (int ia = 0; ia < na; ++ia)
    for (int ib = 0; ib < nb; ++ib) {
      Dir t[3];
      for (int d = 0; d < 3; ++d) {
        const int i = (la && ia == d) ? 1 : 0, j = (lb && ib == d) ? 1 : 0;
        t[d] = dir1(i, j, Ac[d], Bc[d], a, b, Oc[d]);
      }
      double* o = out + (int64_t)(soff[A] + ia) * nao + soff[B] + ib;
      o[0] = pre * t[0].M * t[1].S * t[2].S;
      o[n2] = pre * t[0].S * t[1].M * t[2].S;
      o[2 * n2] = pre * t[0].S * t[1].S * t[2].M;
      // (r x nabla)_x = y d/dz - z d/dy, and cyclic
      o[3 * n2] = pre * t[0].S * (t[1].M * t[2].D - t[1].D * t[2].M);
      o[4 * n2] = pre * t[1].S * (t[2].M * t[0].D - t[2].D * t[0].M);
      o[5 * n2] = pre * t[2].S * (t[0].M * t[1].D - t[0].D * t[1].M);
    }
}

// f_n = 2/3 Omega_n |mu_n|^2, R_n = 1/2 mu_n . m_n from T [n][6] (sqrt(2) already applied)
__global__ void k_strengths(const double* __restrict__ T, const double* __restrict__ omega, int n,
                            double* __restrict__ f, double* __restrict__ R) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double* t = T + 6 * k;
  f[k] = 2.0 / 3.0 * omega[k] * (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  R[k] = 0.5 * (t[0] * t[3] + t[1] * t[4] + t[2] * t[5]);
}

__global__ void k_lorentz(const double* __restrict__ w, const double* __restrict__ s, int n, double g, double e0,
                          double de, int npts, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npts) return;
  const double E = e0 + de * q;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const double x = E - w[k];
    acc += s[k] * (g / M_PI) / (x * x + g * g);
  }
  out[q] = acc;
}

}  // namespace

void transition_properties(const DevShells& ao, const double* C_dev, int nao, int nmo, int nocc, const double* origin,
                           int n, const double* omega_dev, const float* X_dev, double* T_dev, double* f_dev,
                           double* R_dev, hipStream_t s) {
  const int nvir = nmo - nocc;
  const int64_t ov = (int64_t)nocc * nvir, n2 = (int64_t)nao * nao;
  RISP_CHECK(ao.nfunc == nao, RISP_E_SHAPE, "AO shells and nao disagree");
  RISP_CHECK(ao.n < 65536, RISP_E_SHAPE, "more than 65535 AO shells");
  // AO integrals, then r_c[i][a] = sum C[mu][i] P_c[mu][nu] C[nu][nocc + a] for the six operators
  DevBuf P((size_t)6 * n2 * 8), H((size_t)nocc * nao * 8), Rmo((size_t)6 * ov * 8);
  {
    const dim3 grid(ceil_div(ao.n, 256), ao.n);
    k_prop_ao<<<grid, 256, 0, s>>>(ao.x.as<double>(), ao.y.as<double>(), ao.z.as<double>(), ao.ex.as<double>(),
                                   ao.cn.as<double>(), ao.l.as<int>(), ao.off.as<int>(), ao.n, nao, origin[0],
                                   origin[1], origin[2], P.as<double>());
    RISP_LAUNCHED();
  }
  for (int c = 0; c < 6; ++c) {
    Gemm h;  // H[i][nu] = sum_mu C[mu][i] P_c[mu][nu]
    h.M = nocc;
    h.N = nao;
    h.K = nao;
    h.tin = h.tout = DType::F64;
    h.A = C_dev;
    h.lda = nmo;
    h.a_kc = false;
    h.B = P.as<double>() + (size_t)c * n2;
    h.ldb = nao;
    h.b_kc = false;
    h.C = H.get();
    h.ldc = nao;
    gemm(h, nullptr, s);
    Gemm r;  // r_c[i][a] = sum_nu H[i][nu] C[nu][nocc + a]
    r.M = nocc;
    r.N = nvir;
    r.K = nao;
    r.tin = r.tout = DType::F64;
    r.A = H.get();
    r.lda = nao;
    r.B = C_dev + nocc;
    r.ldb = nmo;
    r.b_kc = false;
    r.C = Rmo.as<double>() + (size_t)c * ov;
    r.ldc = nvir;
    gemm(r, nullptr, s);
  }
  if (n > 0) {
    // T[k][c] = sqrt(2) sum_ia X[k][ia] r_c[ia] for all states and the six operators in one product
    Gemm t;
    t.M = n;
    t.N = 6;
    t.K = (int)ov;
    t.tin = t.tout = DType::F64;
    t.mem_a = DType::F32;
    t.A = X_dev;
    t.lda = ov;
    t.B = Rmo.get();
    t.ldb = ov;
    t.C = T_dev;
    t.ldc = 6;
    t.alpha = std::sqrt(2.0);
    t.ksplit = std::min(512, gemm_auto_split(t));
    DevBuf work(gemm_workspace_bytes(t));
    gemm(t, work.get(), s);
    k_strengths<<<ceil_div(n, 64), 64, 0, s>>>(T_dev, omega_dev, n, f_dev, R_dev);
    RISP_LAUNCHED();
  }
  RISP_HIP(hipStreamSynchronize(s));  // the workspaces die at return
}

void lorentz_spectrum(const double* omega_dev, const double* s_dev, int n, double hwhm, double e0, double de, int npts,
                      double* out_dev, hipStream_t s) {
  if (npts <= 0) return;
  k_lorentz<<<ceil_div(npts, 256), 256, 0, s>>>(omega_dev, s_dev, n, hwhm, e0, de, npts, out_dev);
  RISP_LAUNCHED();
}

}  // namespace risp
