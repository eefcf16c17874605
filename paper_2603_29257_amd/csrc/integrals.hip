// Integral kernels of the factor build: Boys function, Schwarz screening with stream compaction,
// 2-centre metric and 3-centre (mu nu|P) integrals by Obara-Saika recurrences, energy window.
#include <cmath>

#include "integrals.hpp"
#include "os.hpp"

namespace risp {

// -------------------------------------------------------------------------------------------
// Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt
// -------------------------------------------------------------------------------------------
// Host table: the convergent series F_n(T) = exp(-T) sum_k (2T)^k / ((2n+1)(2n+3)...(2n+2k+1))
// summed in long double on the grid T_g = g * 0.1.
void boys_table_host(std::vector<double>& tab) {
  tab.assign((size_t)kBoysRows * kBoysCols, 0.0);
  for (int g = 0; g < kBoysRows; ++g) {
    long double T = (long double)g * (long double)kBoysDT;
    for (int n = 0; n < kBoysCols; ++n) {
      long double term = 1.0L / (2 * n + 1), sum = term;
      for (int k = 1; k < 2000; ++k) {
        term *= 2.0L * T / (long double)(2 * n + 2 * k + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
      }
      tab[(size_t)g * kBoysCols + n] = (double)(expl(-T) * sum);
    }
  }
}

// F_0..F_L at T: 8-term Taylor expansion of F_L about the nearest grid point, then the stable
// downward recurrence F_m = (2T F_{m+1} + e^-T)/(2m+1); beyond the table F_0 = sqrt(pi/T)/2 and the
// upward recurrence F_{m+1} = ((2m+1) F_m - e^-T)/(2T).
template <int L>
__device__ __forceinline__ void boys(double T, const double* __restrict__ tab, double* F) {
  if (T < kBoysTMax) {
    const int g = (int)rint(T * (1.0 / kBoysDT));
    const double x = g * kBoysDT - T;
    const double* r = tab + g * kBoysCols + L;
    double f = r[7];
    f = r[6] + f * x * (1.0 / 7.0);
    f = r[5] + f * x * (1.0 / 6.0);
    f = r[4] + f * x * (1.0 / 5.0);
    f = r[3] + f * x * (1.0 / 4.0);
    f = r[2] + f * x * (1.0 / 3.0);
    f = r[1] + f * x * (1.0 / 2.0);
    f = r[0] + f * x;
    F[L] = f;
    const double e = exp(-T);
#pragma unroll
    for (int m = L - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) * (1.0 / (2 * m + 1));
  } else {
    const double inv = 1.0 / T;
    F[0] = 0.5 * sqrt(M_PI * inv);
    const double e = exp(-T);
#pragma unroll
    for (int m = 0; m < L; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * 0.5 * inv;
  }
}

// S[m] = K (alpha F_m(T) + beta kappa^(m+1/2) F_m(kappa T)), kappa = omega^2 / (omega^2 + rho).
template <int L>
__device__ __forceinline__ void base_terms(double K, double T, double rho, double alpha, double beta,
                                           double omega, const double* tab, double* S) {
#pragma unroll
  for (int m = 0; m <= L; ++m) S[m] = 0.0;
  if (alpha != 0.0) {
    double F[L + 1];
    boys<L>(T, tab, F);
#pragma unroll
    for (int m = 0; m <= L; ++m) S[m] = alpha * K * F[m];
  }
  if (beta != 0.0) {
    const double w2 = omega * omega;
    const double kap = w2 / (w2 + rho);
    double F[L + 1];
    boys<L>(kap * T, tab, F);
    double kp = beta * K * sqrt(kap);
#pragma unroll
    for (int m = 0; m <= L; ++m) {
      S[m] += kp * F[m];
      kp *= kap;
    }
  }
}

// -------------------------------------------------------------------------------------------
// Shells
// -------------------------------------------------------------------------------------------
int shell_functions(const risp_shell* sh, int n) {
  int f = 0;
  for (int k = 0; k < n; ++k) f += sh[k].l == 0 ? 1 : 3;
  return f;
}

void upload_shells(DevShells& d, const double* coords, const risp_shell* sh, int n, hipStream_t s) {
  std::vector<double> x(n), y(n), z(n), ex(n), cn(n);
  std::vector<int> l(n), off(n), atom(n);
  int f = 0;
  for (int k = 0; k < n; ++k) {
    const double a = sh[k].exponent;
    x[k] = coords[3 * sh[k].atom + 0];
    y[k] = coords[3 * sh[k].atom + 1];
    z[k] = coords[3 * sh[k].atom + 2];
    ex[k] = a;
    double ns = std::pow(2.0 * a / M_PI, 0.75);
    cn[k] = sh[k].coef * (sh[k].l == 0 ? ns : ns * 2.0 * std::sqrt(a));
    l[k] = sh[k].l;
    off[k] = f;
    atom[k] = sh[k].atom;
    f += sh[k].l == 0 ? 1 : 3;
  }
  d.n = n;
  d.nfunc = f;
  d.x = upload(x.data(), n, s);
  d.y = upload(y.data(), n, s);
  d.z = upload(z.data(), n, s);
  d.ex = upload(ex.data(), n, s);
  d.cn = upload(cn.data(), n, s);
  d.l = upload(l.data(), n, s);
  d.off = upload(off.data(), n, s);
  d.atom = upload(atom.data(), n, s);
  // the host vectors die at return: make the copies complete first
  RISP_HIP(hipStreamSynchronize(s));
}

struct ShellView {
  const double *x, *y, *z, *ex, *cn;
  const int *l, *off;
};
static ShellView view(const DevShells& d) {
  return {d.x.as<double>(), d.y.as<double>(), d.z.as<double>(), d.ex.as<double>(),
          d.cn.as<double>(), d.l.as<int>(), d.off.as<int>()};
}

// -------------------------------------------------------------------------------------------
// Schwarz screening: Q_AB = max sqrt((mu nu|mu nu)); keep (A >= B) if Q_AB * qaux >= tau
// -------------------------------------------------------------------------------------------
template <int LA, int LB>
__device__ double schwarz_q(const ShellView& S, int A, int B) {
  const double a = S.ex[A], b = S.ex[B];
  const double Ax = S.x[A], Ay = S.y[A], Az = S.z[A];
  const double AB[3] = {Ax - S.x[B], Ay - S.y[B], Az - S.z[B]};
  const double p = a + b;
  const double K = exp(-a * b / p * (AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2]));
  OSCtx c;
  const double PA[3] = {-b / p * AB[0], -b / p * AB[1], -b / p * AB[2]};  // P - A
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c.PA[d] = PA[d];
    c.QC[d] = PA[d];
    c.WP[d] = 0.0;
    c.WQ[d] = 0.0;
  }
  c.i2p = 0.5 / p;
  c.i2q = 0.5 / p;
  c.i2pq = 0.25 / p;
  c.rp = 0.5;
  c.rq = 0.5;
  const double pref = 2.0 * pow(M_PI, 2.5) / (p * p * sqrt(2.0 * p)) * K * K;
#pragma unroll
  for (int m = 0; m < 5; ++m) c.S[m] = pref / (2 * m + 1);  // F_m(0) = 1/(2m+1)
  const double n2 = S.cn[A] * S.cn[A] * S.cn[B] * S.cn[B];
  double best = 0.0;
  static_for<0, ncart(LA)>([&](auto ka) {
    static_for<0, ncart(LB)>([&](auto kb) {
      double v = os4c_diag<LA, decltype(ka)::value, LB, decltype(kb)::value>(c, AB) * n2;
      best = fmax(best, sqrt(fmax(v, 0.0)));
    });
  });
  return best;
}

// Lower-triangle pair index t -> (A, B), A >= B, t = A (A + 1) / 2 + B.
__device__ __forceinline__ void tri_decode(int64_t t, int& A, int& B) {
  int64_t a = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > t) --a;
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  A = (int)a;
  B = (int)(t - a * (a + 1) / 2);
}

// key[t] = -1 (dropped) or the group of the kept pair (its class, or 0 when canonical).
__global__ void k_screen_keys(ShellView S, int64_t npt, double qaux, double tau, int canonical,
                              int8_t* __restrict__ key) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < npt;
       t += (int64_t)gridDim.x * blockDim.x) {
    int A, B;
    tri_decode(t, A, B);
    const int la = S.l[A], lb = S.l[B];
    double q;
    if (la == 0 && lb == 0) q = schwarz_q<0, 0>(S, A, B);
    else if (la == 1 && lb == 0) q = schwarz_q<1, 0>(S, A, B);
    else if (la == 0 && lb == 1) q = schwarz_q<1, 0>(S, B, A);
    else q = schwarz_q<1, 1>(S, A, B);
    const bool keep = q * qaux >= tau;
    key[t] = keep ? (int8_t)(canonical ? 0 : la + lb) : (int8_t)-1;
  }
}

// ---- stable compaction by group key (k < NG), 1024 items per block ----
constexpr int kCompactItems = 1024;

template <int NG>
__global__ void k_group_count(const int8_t* __restrict__ key, int64_t n, int* __restrict__ counts) {
  __shared__ int c[NG];
  if (threadIdx.x < NG) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kCompactItems;
  for (int i = threadIdx.x; i < kCompactItems; i += blockDim.x) {
    const int64_t t = base + i;
    if (t < n) {
      const int k = key[t];
      if (k >= 0) atomicAdd(&c[k], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < NG) counts[(int64_t)blockIdx.x * NG + threadIdx.x] = c[threadIdx.x];
}

// Single block: exclusive scan of the per-block counts per group, groups laid out one after another.
template <int NG>
__global__ void k_group_scan(int* __restrict__ counts, int nblk, int* __restrict__ totals) {
  __shared__ int run[NG];
  __shared__ int tot[NG];
  if (threadIdx.x < NG) tot[threadIdx.x] = 0;
  __syncthreads();
  // pass 1: totals per group
  for (int g = 0; g < NG; ++g) {
    int s = 0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += counts[(int64_t)b * NG + g];
    atomicAdd(&tot[g], s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int g = 0; g < NG; ++g) {
      run[g] = acc;
      totals[g] = tot[g];
      acc += tot[g];
    }
    totals[NG] = acc;
    // sequential exclusive scan (nblk is modest: one entry per 1024 pairs)
    for (int g = 0; g < NG; ++g) {
      int r = run[g];
      for (int b = 0; b < nblk; ++b) {
        const int v = counts[(int64_t)b * NG + g];
        counts[(int64_t)b * NG + g] = r;
        r += v;
      }
    }
  }
}

// Scatter kept pairs to out_a/out_b at their stable positions. The (p s) class stores the p shell
// first (key 1 with la = 0 means the original B is the p shell).
template <int NG>
__global__ __launch_bounds__(256) void k_group_scatter(const int8_t* __restrict__ key, int64_t n,
                                                       const int* __restrict__ offs,
                                                       const int* __restrict__ lsh,
                                                       int* __restrict__ out_a,
                                                       int* __restrict__ out_b) {
  constexpr int PER = kCompactItems / 256;  // consecutive items per thread
  __shared__ int scan[NG][256];
  const int64_t base = (int64_t)blockIdx.x * kCompactItems + (int64_t)threadIdx.x * PER;
  int cnt[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) cnt[g] = 0;
  int8_t k[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int64_t t = base + i;
    k[i] = t < n ? key[t] : (int8_t)-1;
#pragma unroll
    for (int g = 0; g < NG; ++g) cnt[g] += (k[i] == g);
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) scan[g][threadIdx.x] = cnt[g];
  __syncthreads();
  // inclusive Hillis-Steele scan per group over the 256 threads
  for (int d = 1; d < 256; d <<= 1) {
    int v[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) v[g] = threadIdx.x >= d ? scan[g][threadIdx.x - d] : 0;
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NG; ++g) scan[g][threadIdx.x] += v[g];
    __syncthreads();
  }
  int pos[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) pos[g] = offs[(int64_t)blockIdx.x * NG + g] + scan[g][threadIdx.x] - cnt[g];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int g = k[i];
    if (g < 0) continue;
    const int64_t t = base + i;
    int A, B;
    tri_decode(t, A, B);
    if (NG > 1 && lsh[A] < lsh[B]) {
      const int tmp = A;
      A = B;
      B = tmp;
    }
    int p = 0;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg)
      if (gg == g) p = pos[gg]++;
    out_a[p] = A;
    out_b[p] = B;
  }
}

template <int NG>
static void compact_groups(const int8_t* key, int64_t n, const int* lsh, PairList& out, hipStream_t s) {
  const int nblk = (int)((n + kCompactItems - 1) / kCompactItems);
  DevBuf counts((size_t)std::max(nblk, 1) * NG * sizeof(int));
  DevBuf totals((NG + 1) * sizeof(int));
  if (nblk > 0) {
    k_group_count<NG><<<nblk, 256, 0, s>>>(key, n, counts.as<int>());
    RISP_LAUNCHED();
  }
  k_group_scan<NG><<<1, 256, 0, s>>>(counts.as<int>(), nblk, totals.as<int>());
  RISP_LAUNCHED();
  int tot[NG + 1];
  RISP_HIP(hipMemcpyAsync(tot, totals.get(), sizeof(tot), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  out.n = tot[NG];
  out.cls_begin[0] = 0;
  for (int g = 1; g <= 3; ++g) out.cls_begin[g] = g <= NG ? out.cls_begin[g - 1] + tot[g - 1] : out.n;
  out.a.alloc((size_t)std::max(out.n, 1) * sizeof(int));
  out.b.alloc((size_t)std::max(out.n, 1) * sizeof(int));
  if (nblk > 0) {
    k_group_scatter<NG><<<nblk, 256, 0, s>>>(key, n, counts.as<int>(), lsh, out.a.as<int>(), out.b.as<int>());
    RISP_LAUNCHED();
  }
  RISP_HIP(hipStreamSynchronize(s));  // counts/totals die at return
}

void screen_pairs(const DevShells& ao, double qaux, double tau, bool canonical, PairList& out,
                  hipStream_t s) {
  const int64_t npt = (int64_t)ao.n * (ao.n + 1) / 2;
  DevBuf key((size_t)std::max<int64_t>(npt, 1));
  if (npt > 0) {
    const unsigned grid = std::min<int64_t>(ceil_div(npt, 256), 65536);
    k_screen_keys<<<grid, 256, 0, s>>>(view(ao), npt, qaux, tau, canonical ? 1 : 0, key.as<int8_t>());
    RISP_LAUNCHED();
  }
  if (canonical)
    compact_groups<1>(key.as<int8_t>(), npt, ao.l.as<int>(), out, s);
  else
    compact_groups<3>(key.as<int8_t>(), npt, ao.l.as<int>(), out, s);
}

// -------------------------------------------------------------------------------------------
// Two-centre integrals (P|Q)
// -------------------------------------------------------------------------------------------
// Block of (P|Q) for shells P (LP) and Q (LQ): blk[kp * ncart(LQ) + kq].
template <int LP, int LQ>
__device__ void int2c_block(const ShellView& S, int P, int Q, Operator op, const double* tab,
                            double* blk) {
  const double p = S.ex[P], q = S.ex[Q];
  const double PQ[3] = {S.x[P] - S.x[Q], S.y[P] - S.y[Q], S.z[P] - S.z[Q]};
  const double rho = p * q / (p + q);
  const double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
  OSCtx c;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double WP = -q * PQ[d] / (p + q);  // W - P
    c.PA[d] = 0.0;                           // one Gaussian on each side: P = A, Q = C
    c.QC[d] = 0.0;
    c.WP[d] = WP;
    c.WQ[d] = WP + PQ[d];  // W - Q
  }
  c.i2p = 0.5 / p;
  c.i2q = 0.5 / q;
  c.i2pq = 0.5 / (p + q);
  c.rp = rho / p;
  c.rq = rho / q;
  const double K = 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q));
  base_terms<LP + LQ>(K, T, rho, op.alpha, op.beta, op.omega, tab, c.S);
  const double nrm = S.cn[P] * S.cn[Q];
  const double zero[3] = {0.0, 0.0, 0.0};
  static_for<0, ncart(LP)>([&](auto kp) {
    static_for<0, ncart(LQ)>([&](auto kq) {
      blk[decltype(kp)::value * ncart(LQ) + decltype(kq)::value] =
          os3c<LP, decltype(kp)::value, 0, 0, LQ, decltype(kq)::value>(c, zero) * nrm;
    });
  });
}

template <int LP, int LQ>
__device__ void int2c_pair(const ShellView& S, int P, int Q, Operator op, const double* tab,
                           double* out, int nf) {
  double blk[9];
  int2c_block<LP, LQ>(S, P, Q, op, tab, blk);
  for (int kp = 0; kp < ncart(LP); ++kp)
    for (int kq = 0; kq < ncart(LQ); ++kq)
      out[(int64_t)(S.off[P] + kp) * nf + S.off[Q] + kq] = blk[kp * ncart(LQ) + kq];
}

__global__ void k_int2c(ShellView S, int n, int nf, Operator op, const double* __restrict__ tab,
                        double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int P = t / n, Q = t % n;
  const int lp = S.l[P], lq = S.l[Q];
  if (lp == 0 && lq == 0) int2c_pair<0, 0>(S, P, Q, op, tab, out, nf);
  else if (lp == 1 && lq == 0) int2c_pair<1, 0>(S, P, Q, op, tab, out, nf);
  else if (lp == 0 && lq == 1) int2c_pair<0, 1>(S, P, Q, op, tab, out, nf);
  else int2c_pair<1, 1>(S, P, Q, op, tab, out, nf);
}

void int2c(const DevShells& aux, const Operator& op, const double* boys_tab, double* out,
           hipStream_t s) {
  const int n = aux.n;
  if (n == 0) return;
  k_int2c<<<ceil_div((int64_t)n * n, 128), 128, 0, s>>>(view(aux), n, aux.nfunc, op, boys_tab, out);
  RISP_LAUNCHED();
}

// largest diagonal element (P|P) of each auxiliary shell (Coulomb operator)
__global__ void k_aux_diag(ShellView S, int n, const double* __restrict__ tab, double* __restrict__ out) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= n) return;
  Operator op;
  double blk[9];
  if (S.l[P] == 0) {
    int2c_block<0, 0>(S, P, P, op, tab, blk);
    out[P] = blk[0];
  } else {
    int2c_block<1, 1>(S, P, P, op, tab, blk);
    out[P] = fmax(blk[0], fmax(blk[4], blk[8]));
  }
}

double aux_diag_max(const DevShells& aux, const double* boys_tab, hipStream_t s) {
  if (aux.n == 0) return 0.0;
  DevBuf d((size_t)aux.n * sizeof(double));
  k_aux_diag<<<ceil_div(aux.n, 64), 64, 0, s>>>(view(aux), aux.n, boys_tab, d.as<double>());
  RISP_LAUNCHED();
  std::vector<double> h(aux.n);
  RISP_HIP(hipMemcpyAsync(h.data(), d.get(), aux.n * sizeof(double), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  double m = 0.0;
  for (double x : h) m = std::max(m, x);
  return m;
}

// -------------------------------------------------------------------------------------------
// Three-centre integrals (mu nu|P) over the screened pair list, one thread per (pair, aux shell)
// -------------------------------------------------------------------------------------------
template <int LA, int LB, int LC>
__global__ __launch_bounds__(256) void k_int3c(ShellView AO, ShellView AX, const int* __restrict__ pa,
                                               const int* __restrict__ pb, int npair,
                                               const int* __restrict__ auxlist, int naux_cls, int f0,
                                               int nao, Operator op, const double* __restrict__ tab,
                                               double* __restrict__ out, PackMap pk, int pair0) {
  const int64_t total = (int64_t)npair * naux_cls;
  const int64_t nao2 = (int64_t)nao * nao;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int ip = (int)(t % npair);
    const int C = auxlist[t / npair];
    const int A = pa[ip], B = pb[ip];
    const double a = AO.ex[A], b = AO.ex[B], q = AX.ex[C];
    const double Ax = AO.x[A], Ay = AO.y[A], Az = AO.z[A];
    const double AB[3] = {Ax - AO.x[B], Ay - AO.y[B], Az - AO.z[B]};
    const double p = a + b;
    const double ip_ = 1.0 / p;
    const double Kab = exp(-a * b * ip_ * (AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2]));
    const double P[3] = {Ax - b * ip_ * AB[0], Ay - b * ip_ * AB[1], Az - b * ip_ * AB[2]};
    const double Cc[3] = {AX.x[C], AX.y[C], AX.z[C]};
    const double ipq = 1.0 / (p + q);
    const double rho = p * q * ipq;
    OSCtx c;
    double PC2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double W = (p * P[d] + q * Cc[d]) * ipq;
      c.PA[d] = P[d] - (d == 0 ? Ax : (d == 1 ? Ay : Az));
      c.WP[d] = W - P[d];
      c.QC[d] = 0.0;
      c.WQ[d] = W - Cc[d];
      PC2 += (P[d] - Cc[d]) * (P[d] - Cc[d]);
    }
    c.i2p = 0.5 * ip_;
    c.i2q = 0.5 / q;
    c.i2pq = 0.5 * ipq;
    c.rp = rho * ip_;
    c.rq = rho / q;
    const double K = 2.0 * pow(M_PI, 2.5) * ip_ / (q * sqrt(p + q)) * Kab;
    base_terms<LA + LB + LC>(K, rho * PC2, rho, op.alpha, op.beta, op.omega, tab, c.S);
    const double nrm = AO.cn[A] * AO.cn[B] * AX.cn[C];
    const int oa = AO.off[A], ob = AO.off[B];
    const bool same = (A == B);
    if (pk.voff) {
      // packed: row mu of A's group at column cab + kb, mirrored row nu of B's group at cba + ka
      const int fc = AX.off[C] - f0;
      const int cab = pk.cab[pair0 + ip], cba = pk.cba[pair0 + ip];
      const int nga = pk.ng[oa], ngb = pk.ng[ob], kpa = pk.kp[oa], kpb = pk.kp[ob];
      const int mla = pk.ml[oa], mlb = pk.ml[ob];
      // offset of row (f, mu) for the first function mu of A's / B's shell: group-major or
      // function-major layout
      auto row_a = [&](int f) -> int64_t {
        return pk.f_stride ? f * pk.f_stride + pk.voff[oa] + (int64_t)mla * kpa
                           : pk.nf_stride * pk.voff[oa] + ((int64_t)f * nga + mla) * kpa;
      };
      auto row_b = [&](int f) -> int64_t {
        return pk.f_stride ? f * pk.f_stride + pk.voff[ob] + (int64_t)mlb * kpb
                           : pk.nf_stride * pk.voff[ob] + ((int64_t)f * ngb + mlb) * kpb;
      };
      static_for<0, ncart(LA)>([&](auto ka) {
        static_for<0, ncart(LB)>([&](auto kb) {
          static_for<0, ncart(LC)>([&](auto kc) {
            const double v = os3c<LA, decltype(ka)::value, LB, decltype(kb)::value, LC,
                                  decltype(kc)::value>(c, AB) * nrm;
            const int f = fc + decltype(kc)::value;
            out[row_a(f) + (int64_t)decltype(ka)::value * kpa + cab + decltype(kb)::value] = v;
            if (!same) out[row_b(f) + (int64_t)decltype(kb)::value * kpb + cba + decltype(ka)::value] = v;
          });
        });
      });
    } else {
      double* o = out + (int64_t)(AX.off[C] - f0) * nao2;
      static_for<0, ncart(LA)>([&](auto ka) {
        static_for<0, ncart(LB)>([&](auto kb) {
          static_for<0, ncart(LC)>([&](auto kc) {
            const double v = os3c<LA, decltype(ka)::value, LB, decltype(kb)::value, LC,
                                  decltype(kc)::value>(c, AB) * nrm;
            const int mu = oa + decltype(ka)::value, nu = ob + decltype(kb)::value;
            double* oc = o + (int64_t)decltype(kc)::value * nao2;
            oc[(int64_t)mu * nao + nu] = v;
            if (!same) oc[(int64_t)nu * nao + mu] = v;
          });
        });
      });
    }
  }
}

void int3c(const DevShells& ao, const PairList& pairs, const DevShells& aux, int s0, int s1,
           const Operator& op, const double* boys_tab, double* out, hipStream_t s, const PackMap* pack) {
  // auxiliary shells of each angular momentum in [s0, s1) (host copy of l and offsets)
  std::vector<int> l(aux.n), off(aux.n);
  RISP_HIP(hipMemcpyAsync(l.data(), aux.l.get(), aux.n * sizeof(int), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipMemcpyAsync(off.data(), aux.off.get(), aux.n * sizeof(int), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  std::vector<int> byl[2];
  for (int k = s0; k < s1; ++k) byl[l[k]].push_back(k);
  const int f0 = s0 < aux.n ? off[s0] : 0;
  const int f1 = s1 < aux.n ? off[s1] : aux.nfunc;
  const int nao = ao.nfunc;
  PackMap pk;
  if (pack) {
    RISP_CHECK(f1 - f0 <= pack->nf_stride, RISP_E_STATE, "int3c: chunk wider than the packed layout");
    pk = *pack;
    RISP_HIP(hipMemsetAsync(out, 0, (size_t)pk.elems * sizeof(double), s));
  } else {
    RISP_HIP(hipMemsetAsync(out, 0, (size_t)(f1 - f0) * nao * nao * sizeof(double), s));
  }
  DevBuf lists[2];
  for (int lc = 0; lc < 2; ++lc) lists[lc] = upload(byl[lc].data(), byl[lc].size(), s);
  const ShellView A = view(ao), X = view(aux);
  const int* pa = pairs.a.as<int>();
  const int* pb = pairs.b.as<int>();
  for (int cls = 0; cls < 3; ++cls) {
    const int b0 = pairs.cls_begin[cls], np = pairs.cls_begin[cls + 1] - b0;
    if (np <= 0) continue;
    for (int lc = 0; lc < 2; ++lc) {
      const int na = (int)byl[lc].size();
      if (na == 0) continue;
      const int64_t total = (int64_t)np * na;
      const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 20);
      const int* la = lists[lc].as<int>();
#define RISP_LAUNCH3C(LA_, LB_, LC_)                                                                 \
  k_int3c<LA_, LB_, LC_><<<grid, 256, 0, s>>>(A, X, pa + b0, pb + b0, np, la, na, f0, nao, op,       \
                                              boys_tab, out, pk, b0)
      if (cls == 0 && lc == 0) RISP_LAUNCH3C(0, 0, 0);
      else if (cls == 0 && lc == 1) RISP_LAUNCH3C(0, 0, 1);
      else if (cls == 1 && lc == 0) RISP_LAUNCH3C(1, 0, 0);
      else if (cls == 1 && lc == 1) RISP_LAUNCH3C(1, 0, 1);
      else if (cls == 2 && lc == 0) RISP_LAUNCH3C(1, 1, 0);
      else RISP_LAUNCH3C(1, 1, 1);
#undef RISP_LAUNCH3C
      RISP_LAUNCHED();
    }
  }
  RISP_HIP(hipStreamSynchronize(s));  // the shell lists die at return
}

// -------------------------------------------------------------------------------------------
// Exchange window
// -------------------------------------------------------------------------------------------
__global__ void k_window_keys(const double* __restrict__ e, int nmo, int nocc, double win, int mode,
                              int8_t* __restrict__ key_o, int8_t* __restrict__ key_v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nmo) return;
  const double h2ev = 27.211386245988;
  if (k < nocc) {
    const bool keep = mode == RISP_WIN_ABSOLUTE ? (e[k] * h2ev > -win) : ((e[nocc] - e[k]) * h2ev < win);
    key_o[k] = keep ? 0 : -1;
  } else {
    const bool keep = mode == RISP_WIN_ABSOLUTE ? (e[k] * h2ev < win) : ((e[k] - e[nocc - 1]) * h2ev < win);
    key_v[k - nocc] = keep ? 0 : -1;
  }
}

// Compact a key array into indices t with key == 0 (stable), single block.
__global__ void k_compact_index(const int8_t* __restrict__ key, int n, int* __restrict__ idx,
                                int* __restrict__ count) {
  __shared__ int s[256];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += 256) {
    const int t = c0 + threadIdx.x;
    const int f = (t < n && key[t] == 0) ? 1 : 0;
    s[threadIdx.x] = f;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const int v = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) idx[base + s[threadIdx.x] - 1] = t;
    __syncthreads();
    if (threadIdx.x == 255) base += s[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

void window_sets(const double* e, int nmo, int nocc, double win, int mode, int* occ_out,
                 int* nocc_k, int* vir_out, int* nvir_k, hipStream_t s) {
  DevBuf ko(std::max(nocc, 1)), kv(std::max(nmo - nocc, 1)), cnt(2 * sizeof(int));
  k_window_keys<<<ceil_div(nmo, 256), 256, 0, s>>>(e, nmo, nocc, win, mode, ko.as<int8_t>(),
                                                   kv.as<int8_t>());
  RISP_LAUNCHED();
  k_compact_index<<<1, 256, 0, s>>>(ko.as<int8_t>(), nocc, occ_out, cnt.as<int>());
  RISP_LAUNCHED();
  k_compact_index<<<1, 256, 0, s>>>(kv.as<int8_t>(), nmo - nocc, vir_out, cnt.as<int>() + 1);
  RISP_LAUNCHED();
  int h[2];
  RISP_HIP(hipMemcpyAsync(h, cnt.get(), sizeof(h), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  *nocc_k = h[0];
  *nvir_k = h[1];
}

}  // namespace risp
