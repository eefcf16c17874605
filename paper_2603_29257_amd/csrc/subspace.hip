// Lowest eigenpairs of the FP64 Davidson subspace matrix in one workgroup:
// Householder reduction to tridiagonal form, bisection on Sturm counts for the k lowest eigenvalues,
// inverse iteration (tridiagonal LU with partial pivoting) with Gram-Schmidt inside clusters of
// close eigenvalues, and back-transformation by the stored reflectors.
#include <cfloat>

#include "subspace.hpp"

namespace risp {

namespace {

constexpr int kThreads = 1024;

__device__ double block_sum(double v, double* red) {
  // wave64 reduction, then across the 16 waves
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

__device__ double wave_sum(double v) {  // full sum in every lane of the wave
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence of LDL^T pivots)
__device__ int sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// One inverse-iteration solve (T - lam I) y = y in place, tridiagonal LU with partial pivoting.
// Scratch: D, DL, DU, DU2 of length n (one set per thread).
__device__ void tri_solve(const double* d, const double* e, int n, double lam, double tiny, double* D,
                          double* DL, double* DU, double* DU2, int* piv_swap, double* y) {
  for (int i = 0; i < n; ++i) D[i] = d[i] - lam;
  for (int i = 0; i + 1 < n; ++i) {
    DL[i] = e[i];
    DU[i] = e[i];
  }
  for (int i = 0; i + 1 < n; ++i) {
    DU2[i] = 0.0;
    if (fabs(D[i]) >= fabs(DL[i])) {
      if (D[i] == 0.0) D[i] = tiny;
      const double f = DL[i] / D[i];
      DL[i] = f;
      D[i + 1] -= f * DU[i];
      piv_swap[i] = 0;
    } else {
      const double f = D[i] / DL[i];
      D[i] = DL[i];
      DL[i] = f;
      const double t = DU[i];
      DU[i] = D[i + 1];
      D[i + 1] = t - f * D[i + 1];
      if (i + 2 < n) {
        DU2[i] = DU[i + 1];
        DU[i + 1] = -f * DU[i + 1];
      }
      piv_swap[i] = 1;
    }
  }
  if (D[n - 1] == 0.0) D[n - 1] = tiny;
  for (int i = 0; i < n; ++i)
    if (fabs(D[i]) < tiny) D[i] = D[i] < 0.0 ? -tiny : tiny;
  // forward: L with row interchanges
  for (int i = 0; i + 1 < n; ++i) {
    if (piv_swap[i]) {
      const double t = y[i];
      y[i] = y[i + 1];
      y[i + 1] = t - DL[i] * y[i];
    } else {
      y[i + 1] -= DL[i] * y[i];
    }
  }
  // back substitution with the upper factor (diagonals D, DU, DU2)
  y[n - 1] /= D[n - 1];
  if (n > 1) y[n - 2] = (y[n - 2] - DU[n - 2] * y[n - 1]) / D[n - 2];
  for (int i = n - 3; i >= 0; --i) y[i] = (y[i] - DU[i] * y[i + 1] - DU2[i] * y[i + 2]) / D[i];
}

__global__ __launch_bounds__(kThreads) void k_syev_lowest(double* __restrict__ H, int n, int ld, int k,
                                                          double* __restrict__ w, double* __restrict__ Z,
                                                          double* __restrict__ ws) {
  __shared__ double red[kThreads / 64];
  __shared__ double sh_beta, sh_alpha, sh_K;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  double* V = ws;                      // reflectors: row j holds v_j[0..n-j-2]
  double* d = V + (size_t)n * n;       // diagonal
  double* e = d + n;                   // off-diagonal
  double* beta = e + n;                // reflector scales
  double* p = beta + n;                // work vector (length n >= k)
  double* Y = p + n;                   // [n][k] eigenvectors of the tridiagonal
  double* S = Y + (size_t)n * k;       // per-eigenvalue scratch: 5 n doubles each
  int* piv = reinterpret_cast<int*>(S + (size_t)5 * n * k);  // per-eigenvalue n ints

  // ---- Householder tridiagonalisation (full symmetric storage, lower reflectors) ----
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const double* x = H + (size_t)j * ld + j + 1;  // row j right of the diagonal = column j below
    double s = 0.0;
    for (int c = tid; c < m; c += nt) s += x[c] * x[c];
    s = block_sum(s, red);
    if (tid == 0) {
      const double x0 = x[0];
      const double rest = s - x0 * x0;
      if (rest <= 0.0) {  // already reduced
        sh_beta = 0.0;
        sh_alpha = x0;
      } else {
        const double alpha = x0 >= 0.0 ? -sqrt(s) : sqrt(s);
        const double v0 = x0 - alpha;
        sh_beta = 2.0 / (rest + v0 * v0);
        sh_alpha = alpha;
      }
      d[j] = H[(size_t)j * ld + j];
      e[j] = sh_alpha;
      beta[j] = sh_beta;
    }
    __syncthreads();
    const double b = sh_beta;
    double* v = V + (size_t)j * n;
    for (int c = tid; c < m; c += nt) v[c] = (c == 0) ? x[0] - sh_alpha : x[c];
    __syncthreads();
    if (b == 0.0) continue;
    // p = b A22 v (one wave per row, lanes over columns)
    for (int r = wave; r < m; r += nwave) {
      const double* row = H + (size_t)(j + 1 + r) * ld + j + 1;
      double acc = 0.0;
      for (int c = lane; c < m; c += 64) acc += row[c] * v[c];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
      if (lane == 0) p[r] = b * acc;
    }
    __syncthreads();
    double kk = 0.0;
    for (int r = tid; r < m; r += nt) kk += v[r] * p[r];
    kk = block_sum(kk, red);
    if (tid == 0) sh_K = 0.5 * b * kk;
    __syncthreads();
    const double K = sh_K;
    for (int r = tid; r < m; r += nt) p[r] -= K * v[r];  // q
    __syncthreads();
    // A22 -= v q^T + q v^T  (one wave per row)
    for (int r = wave; r < m; r += nwave) {
      double* row = H + (size_t)(j + 1 + r) * ld + j + 1;
      const double vr = v[r], pr = p[r];
      for (int c = lane; c < m; c += 64) row[c] -= vr * p[c] + pr * v[c];
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

  // ---- bisection for the k lowest eigenvalues ----
  double tnorm = 0.0, emax2 = 0.0;
  double lo = 0.0, hi = 0.0;
  {
    lo = d[0];
    hi = d[0];
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      tnorm = fmax(tnorm, fabs(d[i]) + r);
      if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
    }
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double eps = DBL_EPSILON;
  const double span = fmax(hi - lo, tnorm * eps);
  lo -= 2.0 * eps * span + pivmin;
  hi += 2.0 * eps * span + pivmin;
  if (tid < k) {
    double a = lo, bnd = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + bnd);
      if (bnd - a <= 2.0 * eps * fmax(fabs(a), fabs(bnd)) + pivmin) break;
      if (sturm_count(d, e, n, mid, pivmin) > tid) bnd = mid;
      else a = mid;
    }
    w[tid] = 0.5 * (a + bnd);
  }
  __syncthreads();

  // ---- inverse iteration ----
  const double tiny = eps * fmax(tnorm, DBL_MIN);
  const double ortol = 1e-3 * tnorm;
  for (int round = 0; round < 3; ++round) {
    if (tid < k) {
      double* sD = S + (size_t)5 * n * tid;
      double* sDL = sD + n;
      double* sDU = sD + 2 * n;
      double* sDU2 = sD + 3 * n;
      double* col = sD + 4 * n;
      double* yy = Y + tid;  // column tid, stride k
      if (round == 0) {
        for (int i = 0; i < n; ++i) col[i] = 1.0 + 0.25 * sin(0.7 * (i + 1) * (tid + 1));
      } else {
        for (int i = 0; i < n; ++i) col[i] = yy[(size_t)i * k];
      }
      tri_solve(d, e, n, w[tid], tiny, sD, sDL, sDU, sDU2, piv + (size_t)n * tid, col);
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += col[i] * col[i];
      nrm = sqrt(nrm);
      for (int i = 0; i < n; ++i) yy[(size_t)i * k] = nrm > 0.0 ? col[i] / nrm : 0.0;
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
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
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
  return sizeof(double) * ((size_t)n * n + 4 * (size_t)n + (size_t)n * k + 5 * (size_t)n * k) +
         sizeof(int) * (size_t)n * k + 64;
}

void subspace_eig(double* H, int n, int ld, int k, double* w, double* Z, double* ws, hipStream_t s) {
  RISP_CHECK(n >= 1 && k >= 1 && k <= n && k <= kThreads && ld >= n, RISP_E_ARG, "subspace_eig: bad sizes");
  k_syev_lowest<<<1, kThreads, 0, s>>>(H, n, ld, k, w, Z, ws);
  RISP_LAUNCHED();
}

}  // namespace risp
