// Block Davidson for the lowest eigenpairs of A (section on large-system Davidson diagonalisation):
// sigma blocks on MFMA; FP64 subspace matrix, Gram-Schmidt and a one-workgroup Jacobi eigensolver on
// the device; trial vectors stored in the sigma precision (FP32, or FP64 for FP64 factors); restart
// from the current Ritz vectors with their products recomputed when the subspace is full.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "davidson.hpp"
#include "linalg.hpp"

namespace risp {

// ---------------------------------------------------------------------------------------------
// Jacobi eigensolver: one workgroup, parallel (round-robin) ordering of disjoint rotations
// ---------------------------------------------------------------------------------------------
constexpr int kJacobiMaxN = 1024;

__global__ __launch_bounds__(1024) void k_jacobi(double* __restrict__ H, int n, int ld,
                                                 double* __restrict__ Z, double* __restrict__ w,
                                                 double* __restrict__ Zs, int max_sweeps) {
  __shared__ double cs[kJacobiMaxN / 2], sn[kJacobiMaxN / 2];
  __shared__ int pp[kJacobiMaxN / 2], qq[kJacobiMaxN / 2];
  __shared__ double red[1024];
  __shared__ int stop;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t t = tid; t < (int64_t)n * n; t += nt) {
    const int i = (int)(t / n), j = (int)(t % n);
    Z[(int64_t)i * ld + j] = i == j ? 1.0 : 0.0;
  }
  const int m = n + (n & 1);  // players; index n (if odd) is a dummy
  const int half = m / 2;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal Frobenius norm against the full norm
    double off = 0.0, all = 0.0;
    for (int64_t t = tid; t < (int64_t)n * n; t += nt) {
      const int i = (int)(t / n), j = (int)(t % n);
      const double v = H[(int64_t)i * ld + j];
      all += v * v;
      if (i != j) off += v * v;
    }
    red[tid] = off;
    __syncthreads();
    for (int d = nt / 2; d > 0; d >>= 1) {
      if (tid < d) red[tid] += red[tid + d];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = all;
    __syncthreads();
    for (int d = nt / 2; d > 0; d >>= 1) {
      if (tid < d) red[tid] += red[tid + d];
      __syncthreads();
    }
    if (tid == 0) stop = (offs <= 1e-30 * red[0] || offs == 0.0) ? 1 : 0;
    __syncthreads();
    if (stop) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int k = tid; k < half; k += nt) {
        int p, q;
        if (k == 0) {
          p = r;
          q = m - 1;
        } else {
          p = (r + k) % (m - 1);
          q = (r - k + (m - 1)) % (m - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = H[(int64_t)p * ld + q];
          if (apq != 0.0) {
            const double app = H[(int64_t)p * ld + p], aqq = H[(int64_t)q * ld + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pp[k] = p;
        qq[k] = q;
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // rows p, q  <-  J^T H
      for (int64_t t = tid; t < (int64_t)half * n; t += nt) {
        const int k = (int)(t / n), j = (int)(t % n);
        const int p = pp[k], q = qq[k];
        if (q >= n || sn[k] == 0.0) continue;
        const double c = cs[k], s = sn[k];
        const double hp = H[(int64_t)p * ld + j], hq = H[(int64_t)q * ld + j];
        H[(int64_t)p * ld + j] = c * hp - s * hq;
        H[(int64_t)q * ld + j] = s * hp + c * hq;
      }
      __syncthreads();
      // columns p, q  <-  H J ; eigenvectors Z J
      for (int64_t t = tid; t < (int64_t)half * n; t += nt) {
        const int k = (int)(t / n), i = (int)(t % n);
        const int p = pp[k], q = qq[k];
        if (q >= n || sn[k] == 0.0) continue;
        const double c = cs[k], s = sn[k];
        double hp = H[(int64_t)i * ld + p], hq = H[(int64_t)i * ld + q];
        H[(int64_t)i * ld + p] = c * hp - s * hq;
        H[(int64_t)i * ld + q] = s * hp + c * hq;
        hp = Z[(int64_t)i * ld + p];
        hq = Z[(int64_t)i * ld + q];
        Z[(int64_t)i * ld + p] = c * hp - s * hq;
        Z[(int64_t)i * ld + q] = s * hp + c * hq;
      }
      __syncthreads();
    }
  }
  // sort ascending (rank by value, ties by index); Zs[:, rank] = Z[:, i]
  for (int i = tid; i < n; i += nt) {
    const double v = H[(int64_t)i * ld + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = H[(int64_t)j * ld + j];
      rank += (u < v) || (u == v && j < i);
    }
    w[rank] = v;
    for (int r = 0; r < n; ++r) Zs[(int64_t)r * ld + rank] = Z[(int64_t)r * ld + i];
  }
}

// ---------------------------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_unit_rows(T* V, int64_t ov, const int* idx, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) V[(int64_t)r * ov + idx[r]] = (T)1;
}

// Per-row sums of squares of R [k][ov] (FP64) in a fixed order: partial[row][blk]
__global__ __launch_bounds__(256) void k_row_sumsq(const double* __restrict__ R, int64_t ov,
                                                   double* __restrict__ partial) {
  __shared__ double red[256];
  const int row = blockIdx.y;
  const int64_t per = (ov + gridDim.x - 1) / gridDim.x;
  const int64_t b = blockIdx.x * per, e = min(ov, b + per);
  double s = 0.0;
  for (int64_t t = b + threadIdx.x; t < e; t += blockDim.x) {
    const double v = R[(int64_t)row * ov + t];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)row * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_finish_norms(const double* partial, int nblk, int k, double* norms) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= k) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)r * nblk + b];
  norms[r] = sqrt(s);
}

// R = AX - theta X (in place in AX)
__global__ void k_residual(double* __restrict__ AX, const double* __restrict__ X, const double* __restrict__ theta,
                           int k, int64_t ov) {
  const int64_t total = (int64_t)k * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x)
    AX[t] -= theta[t / ov] * X[t];
}

// T[r][ia] = R[src[r]][ia] / (theta[src[r]] - de[ia]), |denominator| floored at 1e-8 (sign kept)
__global__ void k_precond(const double* __restrict__ R, const double* __restrict__ theta,
                          const double* __restrict__ de, const int* __restrict__ src, int nt, int64_t ov,
                          double* __restrict__ T) {
  const int64_t total = (int64_t)nt * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / ov);
    const int64_t ia = t % ov;
    const int k = src[r];
    double d = theta[k] - de[ia];
    if (fabs(d) < 1e-8) d = d < 0.0 ? -1e-8 : 1e-8;
    T[t] = R[(int64_t)k * ov + ia] / d;
  }
}

__global__ void k_scale_rows(double* T, int nt, int64_t ov, const double* norms) {
  const int64_t total = (int64_t)nt * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double n = norms[t / ov];
    T[t] = n > 0.0 ? T[t] / n : 0.0;
  }
}

// Gram-Schmidt in coefficient space on one block: given G = T T^T (nt x nt), build the
// coefficients Q = Cf T of an orthonormal basis of span(T), dropping vectors whose remaining norm is
// below drop * (norm of the input vector). Cf is [nt][nt] (rows of kept vectors first), count out.
__global__ void k_block_mgs(const double* __restrict__ G, int nt, double drop, double* __restrict__ Cf,
                            int* __restrict__ kept) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int nk = 0;
  for (int j = 0; j < nt; ++j) {
    // candidate c = e_j - sum_q (q . t_j) q,  q . t_j = sum_i Cf[q][i] G[i][j]
    double c[64];
    for (int i = 0; i < nt; ++i) c[i] = (i == j) ? 1.0 : 0.0;
    for (int q = 0; q < nk; ++q) {
      double dot = 0.0;
      for (int i = 0; i < nt; ++i) dot += Cf[q * nt + i] * G[i * nt + j];
      for (int i = 0; i < nt; ++i) c[i] -= dot * Cf[q * nt + i];
    }
    double n2 = 0.0;
    for (int a = 0; a < nt; ++a) {
      double s = 0.0;
      for (int b = 0; b < nt; ++b) s += G[a * nt + b] * c[b];
      n2 += c[a] * s;
    }
    const double tj = sqrt(fmax(G[j * nt + j], 0.0));
    const double nn = sqrt(fmax(n2, 0.0));
    if (nn > drop * tj && nn > 0.0) {
      for (int i = 0; i < nt; ++i) Cf[nk * nt + i] = c[i] / nn;
      ++nk;
    }
  }
  *kept = nk;
}

// eigenvalue copy for the residual kernel
template <typename TS>
__global__ void k_store_rows(const double* __restrict__ T, int64_t n, TS* __restrict__ dst) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = (TS)T[t];
}

__global__ void k_sym_update(double* H, int ld, const double* Hn, int nall, int n0, int nn) {
  // Hn [nall][nn] = V[0:nall] . W[n0:n0+nn]^T ; H[i][n0+j] = H[n0+j][i] = Hn[i][j]
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nall * nn) return;
  const int i = (int)(t / nn), j = (int)(t % nn);
  const double v = Hn[t];
  H[(int64_t)i * ld + n0 + j] = v;
  H[(int64_t)(n0 + j) * ld + i] = v;
}

__global__ void k_symmetrize_block(double* H, int ld, int n0, int nn) {
  // average the new-new block so H stays exactly symmetric
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn * nn) return;
  const int i = t / nn, j = t % nn;
  if (j <= i) return;
  double* a = H + (int64_t)(n0 + i) * ld + n0 + j;
  double* b = H + (int64_t)(n0 + j) * ld + n0 + i;
  const double v = 0.5 * (*a + *b);
  *a = v;
  *b = v;
}

__global__ void k_copy_sub(const double* H, int ld, int n, double* out, int ldo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  out[(int64_t)i * ldo + j] = H[(int64_t)i * ld + j];
}

// ---------------------------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------------------------
namespace {

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double sec() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(ceil_div(n, 256), 65536); }

}  // namespace

void davidson(risp_factors* f, const DavOptions& o, const SigmaFn& sigma_fn, DavResult& res) {
  risp_ctx* ctx = f->ctx;
  hipStream_t s = ctx->stream;
  const int64_t ov = (int64_t)f->nocc * f->nvir;
  const bool fp64 = f->precision == RISP_FP64;
  const DType tvec = fp64 ? DType::F64 : DType::F32;  // storage of V and W
  const size_t vsz = fp64 ? 8 : 4;
  const int nstates = o.nstates;
  RISP_CHECK(nstates > 0 && nstates <= ov, RISP_E_ARG, "nstates out of range");
  RISP_CHECK(o.tol > 0.0, RISP_E_ARG, "tol must be positive");
  int block = o.block > 0 ? o.block : std::min(2 * nstates, 30);
  block = (int)std::min<int64_t>(std::max(block, nstates), ov);
  RISP_CHECK(block <= 64, RISP_E_ARG, "block is limited to 64 trial vectors");
  int max_space = o.max_space > 0 ? o.max_space : std::max(8 * block, nstates + 2 * block);
  max_space = (int)std::min<int64_t>(max_space, ov);
  RISP_CHECK(max_space >= block, RISP_E_ARG, "max_space must hold at least one block");
  RISP_CHECK(max_space + block <= kJacobiMaxN, RISP_E_ARG, "max_space too large for the subspace solver");
  RISP_CHECK(ov < (1ll << 31), RISP_E_SHAPE, "nocc*nvir too large");
  const int cap = max_space + block;  // rows of V and W
  const int ld = cap;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;

  DevBuf V((size_t)cap * ov * vsz), W((size_t)cap * ov * vsz);
  DevBuf H((size_t)ld * ld * 8), Hw((size_t)ld * ld * 8), Z((size_t)ld * ld * 8), Zs((size_t)ld * ld * 8);
  DevBuf theta((size_t)ld * 8);
  res.X.alloc((size_t)block * ov * 8);
  DevBuf AX((size_t)block * ov * 8), T((size_t)block * ov * 8), T2((size_t)block * ov * 8);
  DevBuf Tsave((size_t)block * ov * 8);
  DevBuf Cmix((size_t)cap * block * 8), G((size_t)block * block * 8), Cf((size_t)block * block * 8);
  const int nblk = (int)std::min<int64_t>(64, std::max<int64_t>(1, ov / 4096));
  DevBuf partial((size_t)std::max(cap, block) * nblk * 8), norms((size_t)std::max(cap, block) * 8);
  DevBuf kept(sizeof(int)), src((size_t)block * sizeof(int)), Hn((size_t)cap * block * 8);
  double* X = res.X.as<double>();
  auto vrow = [&](DevBuf& b, int r) { return static_cast<char*>(b.get()) + (size_t)r * ov * vsz; };

  auto run_sigma = [&](int r0, int n) {
    RISP_HIP(hipStreamSynchronize(s));
    Timer t;
    sigma_fn(n, vrow(V, r0), vrow(W, r0));
    RISP_HIP(hipStreamSynchronize(s));
    res.t_sigma += t.sec();
    res.sigma_vectors += n;
    res.sigma_flops += sigma_flops(f, n);
  };
  // H[0:nall][n0:n0+nn] and its transpose from V . W^T (FP64 products)
  auto update_H = [&](int nall, int n0, int nn) {
    Gemm g;
    g.M = nall;
    g.N = nn;
    g.K = (int)ov;
    g.tin = DType::F64;
    g.tout = DType::F64;
    g.mem_a = tvec;
    g.mem_b = tvec;
    g.A = V.get();
    g.lda = ov;
    g.B = vrow(W, n0);
    g.ldb = ov;
    g.C = Hn.get();
    g.ldc = nn;
    g.ksplit = gemm_auto_split(g);
    DevBuf work(gemm_workspace_bytes(g));
    gemm(g, work.get(), s);
    k_sym_update<<<ceil_div((int64_t)nall * nn, 256), 256, 0, s>>>(H.as<double>(), ld, Hn.as<double>(), nall, n0, nn);
    RISP_LAUNCHED();
    k_symmetrize_block<<<ceil_div(nn * nn, 256), 256, 0, s>>>(H.as<double>(), ld, n0, nn);
    RISP_LAUNCHED();
    RISP_HIP(hipStreamSynchronize(s));  // work dies at return
  };
  auto row_norms = [&](const double* R, int k, double* out_dev) {
    k_row_sumsq<<<dim3(nblk, k), 256, 0, s>>>(R, ov, partial.as<double>());
    RISP_LAUNCHED();
    k_finish_norms<<<ceil_div(k, 64), 64, 0, s>>>(partial.as<double>(), nblk, k, out_dev);
    RISP_LAUNCHED();
  };
  // Y = Cm^T Vsrc: rows [0:k) of the FP64 result from the columns of Cm [nsub][ldcm] and rows of
  // Vsrc (tvec). out [k][ov] FP64; alpha, beta as in the product.
  auto combine_rows = [&](const double* Cm, int ldcm, int nsub, int k, const void* Vsrc, double* out,
                          double alpha, double beta) {
    Gemm g;
    g.M = k;
    g.N = (int)ov;
    g.K = nsub;
    g.tin = DType::F64;
    g.tout = DType::F64;
    g.mem_a = DType::F64;
    g.mem_b = tvec;
    g.A = Cm;  // A[i][s] = Cm[s][i]
    g.lda = ldcm;
    g.a_kc = false;
    g.B = Vsrc;  // B[ia][s] = V[s][ia]
    g.ldb = ov;
    g.b_kc = false;
    g.C = out;
    g.ldc = ov;
    g.alpha = alpha;
    g.beta = beta;
    gemm(g, nullptr, s);
  };
  // orthonormalise the nt FP64 rows of T within the block (coefficient-space Gram-Schmidt run twice);
  // result in T, returns the number of rows kept
  auto orth_block = [&](int nt) -> int {
    int nk = nt;
    for (int pass = 0; pass < 2 && nk > 0; ++pass) {
      Gemm g;
      g.M = nk;
      g.N = nk;
      g.K = (int)ov;
      g.tin = g.tout = DType::F64;
      g.A = T.get();
      g.lda = ov;
      g.B = T.get();
      g.ldb = ov;
      g.C = G.get();
      g.ldc = nk;
      g.ksplit = gemm_auto_split(g);
      DevBuf work(gemm_workspace_bytes(g));
      gemm(g, work.get(), s);
      k_block_mgs<<<1, 64, 0, s>>>(G.as<double>(), nk, 1e-6, Cf.as<double>(), kept.as<int>());
      RISP_LAUNCHED();
      int h = 0;
      RISP_HIP(hipMemcpyAsync(&h, kept.get(), sizeof(int), hipMemcpyDeviceToHost, s));
      RISP_HIP(hipStreamSynchronize(s));
      if (h == 0) return 0;
      // T2 = Cf T ; T <- T2
      Gemm c;
      c.M = h;
      c.N = (int)ov;
      c.K = nk;
      c.tin = c.tout = DType::F64;
      c.A = Cf.get();
      c.lda = nk;
      c.B = T.get();  // B[ia][t] = T[t][ia]
      c.ldb = ov;
      c.b_kc = false;
      c.C = T2.get();
      c.ldc = ov;
      gemm(c, nullptr, s);
      RISP_HIP(hipMemcpyAsync(T.get(), T2.get(), (size_t)h * ov * 8, hipMemcpyDeviceToDevice, s));
      nk = h;
    }
    return nk;
  };
  // project the nt FP64 rows of T off V[0:nsub] (classical Gram-Schmidt, two passes)
  auto project_out = [&](int nsub, int nt) {
    for (int pass = 0; pass < 2 && nsub > 0; ++pass) {
      Gemm g;  // Cmix[r][t] = V[r] . T[t]
      g.M = nsub;
      g.N = nt;
      g.K = (int)ov;
      g.tin = g.tout = DType::F64;
      g.mem_a = tvec;
      g.mem_b = DType::F64;
      g.A = V.get();
      g.lda = ov;
      g.B = T.get();
      g.ldb = ov;
      g.C = Cmix.get();
      g.ldc = nt;
      g.ksplit = gemm_auto_split(g);
      DevBuf work(gemm_workspace_bytes(g));
      gemm(g, work.get(), s);
      combine_rows(Cmix.as<double>(), nt, nsub, nt, V.get(), T.as<double>(), -1.0, 1.0);
      RISP_HIP(hipStreamSynchronize(s));
    }
  };
  auto store_T = [&](int r0, int n) {
    if (fp64)
      k_store_rows<double><<<grid_for((int64_t)n * ov), 256, 0, s>>>(T.as<double>(), (int64_t)n * ov,
                                                                    reinterpret_cast<double*>(vrow(V, r0)));
    else
      k_store_rows<float><<<grid_for((int64_t)n * ov), 256, 0, s>>>(T.as<double>(), (int64_t)n * ov,
                                                                   reinterpret_cast<float*>(vrow(V, r0)));
    RISP_LAUNCHED();
  };

  // ---- initial subspace ----
  int nsub = 0;
  if (o.nx0 > 0 && o.x0_dev) {
    const int n0 = std::min(o.nx0, block);
    RISP_HIP(hipMemcpyAsync(T.get(), o.x0_dev, (size_t)n0 * ov * 8, hipMemcpyDeviceToDevice, s));
    const int nk = orth_block(n0);
    RISP_CHECK(nk > 0, RISP_E_ARG, "initial vectors are zero or dependent");
    store_T(0, nk);
    nsub = nk;
  } else {
    // unit vectors at the lowest e_a - e_i, ties broken by (i, a)
    std::vector<double> de(ov);
    RISP_HIP(hipMemcpyAsync(de.data(), f->de64.get(), ov * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    std::vector<int> idx(ov);
    std::iota(idx.begin(), idx.end(), 0);
    std::partial_sort(idx.begin(), idx.begin() + block, idx.end(),
                      [&](int a, int b) { return de[a] < de[b] || (de[a] == de[b] && a < b); });
    DevBuf di = upload(idx.data(), block, s);
    RISP_HIP(hipMemsetAsync(V.get(), 0, (size_t)block * ov * vsz, s));
    if (fp64) k_unit_rows<double><<<1, 64, 0, s>>>(V.as<double>(), ov, di.as<int>(), block);
    else k_unit_rows<float><<<1, 64, 0, s>>>(V.as<float>(), ov, di.as<int>(), block);
    RISP_LAUNCHED();
    RISP_HIP(hipStreamSynchronize(s));
    nsub = block;
  }
  run_sigma(0, nsub);
  update_H(nsub, 0, nsub);

  std::vector<double> hnorm(block), htheta(ld);
  double best_r = 1e300;
  int best_it = 0;
  for (int it = 1; it <= max_iter; ++it) {
    Timer tsub;
    res.iters = it;
    // Rayleigh-Ritz on the subspace
    k_copy_sub<<<ceil_div((int64_t)nsub * nsub, 256), 256, 0, s>>>(H.as<double>(), ld, nsub, Hw.as<double>(), ld);
    RISP_LAUNCHED();
    k_jacobi<<<1, 1024, 0, s>>>(Hw.as<double>(), nsub, ld, Z.as<double>(), theta.as<double>(), Zs.as<double>(), 50);
    RISP_LAUNCHED();
    const int k = std::min(block, nsub);
    combine_rows(Zs.as<double>(), ld, nsub, k, V.get(), X, 1.0, 0.0);
    combine_rows(Zs.as<double>(), ld, nsub, k, W.get(), AX.as<double>(), 1.0, 0.0);
    k_residual<<<grid_for((int64_t)k * ov), 256, 0, s>>>(AX.as<double>(), X, theta.as<double>(), k, ov);
    RISP_LAUNCHED();
    row_norms(AX.as<double>(), k, norms.as<double>());
    RISP_HIP(hipMemcpyAsync(hnorm.data(), norms.get(), k * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipMemcpyAsync(htheta.data(), theta.get(), k * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    res.krows = k;
    double rmax = 0.0;
    for (int j = 0; j < std::min(nstates, k); ++j) rmax = std::max(rmax, hnorm[j]);
    res.resid_hist.push_back(rmax);
    res.energies.assign(htheta.begin(), htheta.begin() + std::min(nstates, k));
    if (k >= nstates && rmax < o.tol) {
      res.converged = true;
      res.t_subspace += tsub.sec();
      break;
    }
    if (rmax < 0.7 * best_r) {
      best_r = rmax;
      best_it = it;
    } else if (o.stall_iters > 0 && it - best_it >= o.stall_iters) {
      res.stalled = true;
      res.t_subspace += tsub.sec();
      break;
    }
    if (it == max_iter) {
      res.t_subspace += tsub.sec();
      break;
    }
    // corrections for the Ritz pairs not yet converged
    std::vector<int> todo;
    for (int j = 0; j < k; ++j)
      if (hnorm[j] >= o.tol) todo.push_back(j);
    const int nt = (int)todo.size();
    RISP_HIP(hipMemcpyAsync(src.get(), todo.data(), nt * sizeof(int), hipMemcpyHostToDevice, s));
    k_precond<<<grid_for((int64_t)nt * ov), 256, 0, s>>>(AX.as<double>(), theta.as<double>(), f->de64.as<double>(),
                                                        src.as<int>(), nt, ov, T.as<double>());
    RISP_LAUNCHED();
    row_norms(T.as<double>(), nt, norms.as<double>());
    k_scale_rows<<<grid_for((int64_t)nt * ov), 256, 0, s>>>(T.as<double>(), nt, ov, norms.as<double>());
    RISP_LAUNCHED();
    if (nsub + nt > max_space) {
      // restart: the current Ritz vectors become the subspace; their products are recomputed
      RISP_HIP(hipMemcpyAsync(Tsave.get(), T.get(), (size_t)nt * ov * 8, hipMemcpyDeviceToDevice, s));
      RISP_HIP(hipMemcpyAsync(T.get(), X, (size_t)k * ov * 8, hipMemcpyDeviceToDevice, s));
      const int nk = orth_block(k);
      store_T(0, nk);
      res.t_subspace += tsub.sec();
      run_sigma(0, nk);
      tsub = Timer();
      update_H(nk, 0, nk);
      nsub = nk;
      ++res.restarts;
      RISP_HIP(hipMemcpyAsync(T.get(), Tsave.get(), (size_t)nt * ov * 8, hipMemcpyDeviceToDevice, s));
    }
    project_out(nsub, nt);
    const int nk = orth_block(nt);
    if (nk == 0) {
      res.t_subspace += tsub.sec();
      break;  // no new direction: the subspace cannot grow
    }
    store_T(nsub, nk);
    res.t_subspace += tsub.sec();
    run_sigma(nsub, nk);
    update_H(nsub + nk, nsub, nk);
    nsub += nk;
  }
  RISP_HIP(hipStreamSynchronize(s));
}

}  // namespace risp
