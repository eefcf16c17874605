// Lowest eigenpairs of the FP64 Davidson subspace matrix in one workgroup:
// Householder reduction to tridiagonal form, multisection on Sturm counts for the k lowest
// eigenvalues, inverse iteration (tridiagonal LU with partial pivoting, factored once per eigenvalue)
// with Gram-Schmidt inside clusters of close eigenvalues, and back-transformation by the stored
// reflectors.
#include <cfloat>

#include "subspace.hpp"

namespace risp {

namespace {

constexpr int kThreads = 1024;

__device__ double wave_sum(double v) {  // full sum in every lane of the wave
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kMaxN = 1024;  // largest subspace (LDS vectors below)

// number of eigenvalues of the tridiagonal (d, e^2 = e2) below x (Sturm sequence of LDL^T pivots)
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// LU factorisation with partial pivoting of T - lam I (tridiagonal d, e) for one eigenvalue. The
// factors of the k eigenvalues are interleaved, element i of eigenvalue t at [i * k + t], so a wave's
// threads touch neighbouring addresses at every step.
__device__ void tri_factor(const double* d, const double* e, int n, double lam, double tiny, int k, double* D,
                           double* DL, double* DU, double* DU2, int* sw) {
  double di = d[0] - lam;  // running diagonal of the current row
  double ui = n > 1 ? e[0] : 0.0;  // running superdiagonal of the current row
  for (int i = 0; i + 1 < n; ++i) {
    const double l = e[i];               // subdiagonal below row i
    const double dn = d[i + 1] - lam;    // diagonal of row i + 1
    const double un = i + 2 < n ? e[i + 1] : 0.0;
    if (fabs(di) >= fabs(l)) {
      const double dd = di == 0.0 ? tiny : di;
      const double f = l / dd;
      D[i * k] = dd;
      DU[i * k] = ui;
      DU2[i * k] = 0.0;
      DL[i * k] = f;
      sw[i * k] = 0;
      di = dn - f * ui;
      ui = un;
    } else {
      const double f = di / l;
      D[i * k] = l;
      DU[i * k] = dn;
      DU2[i * k] = un;
      DL[i * k] = f;
      sw[i * k] = 1;
      di = ui - f * dn;
      ui = -f * un;
    }
  }
  D[(n - 1) * k] = di == 0.0 ? tiny : di;
  for (int i = 0; i < n; ++i) {
    const double v = D[i * k];
    if (fabs(v) < tiny) D[i * k] = v < 0.0 ? -tiny : tiny;
  }
}

// solve with the factors above, y (stride k) in place
__device__ void tri_solve(int n, int k, const double* D, const double* DL, const double* DU, const double* DU2,
                          const int* sw, double* y) {
  double yi = y[0];
  for (int i = 0; i + 1 < n; ++i) {
    const double yn = y[(i + 1) * k];
    if (sw[i * k]) {
      y[i * k] = yn;
      yi = yi - DL[i * k] * yn;
    } else {
      y[i * k] = yi;
      yi = yn - DL[i * k] * yi;
    }
  }
  y[(n - 1) * k] = yi;
  double y2 = 0.0, y1 = yi / D[(n - 1) * k];
  y[(n - 1) * k] = y1;
  if (n > 1) {
    const double v = (y[(n - 2) * k] - DU[(n - 2) * k] * y1) / D[(n - 2) * k];
    y[(n - 2) * k] = v;
    y2 = y1;
    y1 = v;
  }
  for (int i = n - 3; i >= 0; --i) {
    const double v = (y[i * k] - DU[i * k] * y1 - DU2[i * k] * y2) / D[i * k];
    y[i * k] = v;
    y2 = y1;
    y1 = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_syev_lowest(double* __restrict__ H, int n, int ld, int k,
                                                          double* __restrict__ w, double* __restrict__ Z,
                                                          double* __restrict__ ws) {
  __shared__ double sv[kMaxN], sp[kMaxN];  // current reflector and b A v; later d and e^2
  __shared__ double se[kMaxN];             // e (off-diagonal) for the bisection / inverse iteration
  __shared__ int scnt[kThreads];
  __shared__ double sh_beta, sh_alpha;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  double* V = ws;                      // reflectors: row j holds v_j[0..n-j-2]
  double* d = V + (size_t)n * n;       // diagonal
  double* e = d + n;                   // off-diagonal
  double* beta = e + n;                // reflector scales
  double* p = beta + n;                // work vector (length n >= k)
  double* Y = p + n;                   // [n][k] eigenvectors of the tridiagonal
  double* S = Y + (size_t)n * k;       // LU factors, 4 arrays [n][k]
  int* piv = reinterpret_cast<int*>(S + (size_t)4 * n * k);  // [n][k] row interchanges

  // ---- Householder tridiagonalisation (full symmetric storage, lower reflectors) ----
  // per step: wave 0 forms the reflector, all waves form p = b A22 v, then every wave forms
  // K = b v.p / 2 itself and applies A22 -= v q^T + q v^T with q = p - K v
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const double* x = H + (size_t)j * ld + j + 1;  // row j right of the diagonal = column j below
    if (wave == 0) {
      double s = 0.0;
      for (int c = lane; c < m; c += 64) s += x[c] * x[c];
      s = wave_sum(s);
      const double x0 = x[0];
      const double rest = s - x0 * x0;
      double b = 0.0, alpha = x0;
      if (rest > 0.0) {
        alpha = x0 >= 0.0 ? -sqrt(s) : sqrt(s);
        const double v0 = x0 - alpha;
        b = 2.0 / (rest + v0 * v0);
      }
      for (int c = lane; c < m; c += 64) {
        const double vc = c == 0 ? x0 - alpha : x[c];
        sv[c] = vc;
        V[(size_t)j * n + c] = vc;
      }
      if (lane == 0) {
        sh_beta = b;
        sh_alpha = alpha;
        d[j] = H[(size_t)j * ld + j];
        e[j] = alpha;
        beta[j] = b;
      }
    }
    __syncthreads();
    const double b = sh_beta;
    if (b == 0.0) {  // uniform; the barrier keeps wave 0 from overwriting sh_beta before all read it
      __syncthreads();
      continue;
    }
    for (int r = wave; r < m; r += nwave) {
      const double* row = H + (size_t)(j + 1 + r) * ld + j + 1;
      double acc = 0.0;
      for (int c = lane; c < m; c += 64) acc += row[c] * sv[c];
      acc = wave_sum(acc);
      if (lane == 0) sp[r] = b * acc;
    }
    __syncthreads();
    double kk = 0.0;
    for (int c = lane; c < m; c += 64) kk += sv[c] * sp[c];
    const double K = 0.5 * b * wave_sum(kk);
    for (int r = wave; r < m; r += nwave) {
      double* row = H + (size_t)(j + 1 + r) * ld + j + 1;
      const double vr = sv[r], qr = sp[r] - K * sv[r];
      for (int c = lane; c < m; c += 64) row[c] -= vr * (sp[c] - K * sv[c]) + qr * sv[c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = H[(size_t)(n - 2) * ld + n - 2];
      e[n - 2] = H[(size_t)(n - 1) * ld + n - 2];
    }
    d[n - 1] = H[(size_t)(n - 1) * ld + n - 1];
    if (n >= 2) beta[n - 2] = 0.0;
    beta[n - 1] = 0.0;
  }
  __syncthreads();
  // tridiagonal into LDS: sv = d, sp = e^2, se = e
  for (int i = tid; i < n; i += nt) {
    sv[i] = d[i];
    const double ei = i + 1 < n ? e[i] : 0.0;
    se[i] = ei;
    sp[i] = ei * ei;
  }
  __syncthreads();
  const double* dd = sv;
  const double* e2 = sp;
  const double* ee = se;

  // ---- multisection for the k lowest eigenvalues ----
  // G threads per eigenvalue evaluate Sturm counts at G interior points of its interval and the
  // interval shrinks to the subinterval where the count passes the eigenvalue's index
  double tnorm = 0.0, emax2 = 0.0;
  double lo = dd[0], hi = dd[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
    lo = fmin(lo, dd[i] - r);
    hi = fmax(hi, dd[i] + r);
    tnorm = fmax(tnorm, fabs(dd[i]) + r);
    if (i + 1 < n) emax2 = fmax(emax2, e2[i]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double eps = DBL_EPSILON;
  const double span = fmax(hi - lo, tnorm * eps);
  lo -= 2.0 * eps * span + pivmin;
  hi += 2.0 * eps * span + pivmin;
  const int G = nt / k;  // >= 1 (k <= kThreads)
  const int t_ev = tid / G, g = tid % G;
  const bool act = t_ev < k;
  double a = lo, bnd = hi;
  for (int it = 0; it < 100; ++it) {
    // every thread of a group holds the same interval; the stop test is uniform per group
    const bool open = act && !(bnd - a <= 2.0 * eps * fmax(fabs(a), fabs(bnd)) + pivmin);
    if (open) scnt[tid] = sturm_count(dd, e2, n, a + (bnd - a) * (double)(g + 1) / (double)(G + 1), pivmin);
    __syncthreads();
    int any = 0;
    if (open) {
      // first point whose count exceeds the index: the eigenvalue lies below it
      int q = G;
      for (int u = 0; u < G; ++u)
        if (scnt[t_ev * G + u] > t_ev) {
          q = u;
          break;
        }
      const double na = q == 0 ? a : a + (bnd - a) * (double)q / (double)(G + 1);
      const double nb = q == G ? bnd : a + (bnd - a) * (double)(q + 1) / (double)(G + 1);
      a = na;
      bnd = nb;
      any = 1;
    }
    if (!__syncthreads_or(any)) break;
  }
  if (act && g == 0) w[t_ev] = 0.5 * (a + bnd);
  __syncthreads();

  // ---- inverse iteration: one factorisation per eigenvalue, three solves ----
  const double tiny = eps * fmax(tnorm, DBL_MIN);
  const double ortol = 1e-3 * tnorm;
  double* fD = S;
  double* fDL = S + (size_t)n * k;
  double* fDU = S + (size_t)2 * n * k;
  double* fDU2 = S + (size_t)3 * n * k;
  if (tid < k) {
    tri_factor(dd, ee, n, w[tid], tiny, k, fD + tid, fDL + tid, fDU + tid, fDU2 + tid, piv + tid);
    for (int i = 0; i < n; ++i) Y[(size_t)i * k + tid] = 1.0 + 0.25 * sin(0.7 * (i + 1) * (tid + 1));
  }
  for (int round = 0; round < 3; ++round) {
    if (tid < k) {
      double* yy = Y + tid;  // column tid, stride k
      tri_solve(n, k, fD + tid, fDL + tid, fDU + tid, fDU2 + tid, piv + tid, yy);
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += yy[(size_t)i * k] * yy[(size_t)i * k];
      nrm = sqrt(nrm);
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = 0; i < n; ++i) yy[(size_t)i * k] *= inv;
    }
    __syncthreads();
    // Gram-Schmidt inside clusters of close eigenvalues (in ascending order), by the first wave
    // alone: lanes over rows, wave reductions, no block barriers inside the loops
    if (wave == 0) {
      for (int t = 1; t < k; ++t) {
        bool touched = false;
        for (int s = 0; s < t; ++s) {
          if (fabs(w[t] - w[s]) >= ortol) continue;
          touched = true;
          double dot = 0.0;
          for (int i = lane; i < n; i += 64) dot += Y[(size_t)i * k + s] * Y[(size_t)i * k + t];
          dot = wave_sum(dot);
          for (int i = lane; i < n; i += 64) Y[(size_t)i * k + t] -= dot * Y[(size_t)i * k + s];
        }
        if (!touched) continue;
        double nn = 0.0;
        for (int i = lane; i < n; i += 64) nn += Y[(size_t)i * k + t] * Y[(size_t)i * k + t];
        nn = wave_sum(nn);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int i = lane; i < n; i += 64) Y[(size_t)i * k + t] *= inv;
      }
    }
    __syncthreads();
  }

  // ---- back-transformation: Z = H_0 H_1 ... H_{n-3} Y ----
  for (int j = n - 3; j >= 0; --j) {
    const double b = beta[j];
    if (b == 0.0) continue;
    const int m = n - j - 1;
    const double* v = V + (size_t)j * n;
    // gamma_t = b v . Y[j+1:, t] for each column t (one wave per column)
    for (int t = wave; t < k; t += nwave) {
      double acc = 0.0;
      for (int c = lane; c < m; c += 64) acc += v[c] * Y[(size_t)(j + 1 + c) * k + t];
      acc = wave_sum(acc);
      if (lane == 0) p[t] = b * acc;
    }
    __syncthreads();
    for (int c = wave; c < m; c += nwave) {
      const double vc = v[c];
      double* yr = Y + (size_t)(j + 1 + c) * k;
      for (int t = lane; t < k; t += 64) yr[t] -= p[t] * vc;
    }
    __syncthreads();
  }
  for (int r = wave; r < n; r += nwave)
    for (int t = lane; t < k; t += 64) Z[(size_t)r * ld + t] = Y[(size_t)r * k + t];
}

}  // namespace

size_t subspace_eig_workspace(int n, int k) {
  return sizeof(double) * ((size_t)n * n + 4 * (size_t)n + (size_t)n * k + 4 * (size_t)n * k) +
         sizeof(int) * (size_t)n * k + 64;
}

void subspace_eig(double* H, int n, int ld, int k, double* w, double* Z, double* ws, hipStream_t s) {
  RISP_CHECK(n >= 1 && k >= 1 && k <= n && k <= kThreads && n <= kMaxN && ld >= n, RISP_E_ARG,
             "subspace_eig: bad sizes");
  k_syev_lowest<<<1, kThreads, 0, s>>>(H, n, ld, k, w, Z, ws);
  RISP_LAUNCHED();
}

}  // namespace risp
