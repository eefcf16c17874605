// Block Davidson for the lowest eigenpairs of A (section on large-system Davidson diagonalisation):
// sigma blocks on MFMA; FP64 subspace matrix, Gram-Schmidt and a one-workgroup eigensolver
// (Householder tridiagonalisation, bisection, inverse iteration) on the device; trial vectors stored in the sigma precision (FP32, or FP64 for FP64 factors); restart
// from the current Ritz vectors with their products recomputed when the subspace is full.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include <cstdio>

#include "davidson.hpp"
#include "linalg.hpp"
#include "subspace.hpp"

namespace risp {

constexpr int kSubspaceMaxN = 1024;

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

__device__ __forceinline__ double precond_den(double theta, double de) {
  double d = theta - de;
  if (fabs(d) < 1e-8) d = d < 0.0 ? -1e-8 : 1e-8;
  return d;
}

// T[r][ia] = (R[k][ia] - eps[r] X[k][ia]) / (theta[k] - de[ia]) for k = src[r], with de the diagonal
// of A, |denominator| floored at 1e-8 (sign kept); eps = nullptr: plain Davidson correction
__global__ void k_precond(const double* __restrict__ R, const double* __restrict__ theta,
                          const double* __restrict__ de, const int* __restrict__ src, int nt, int64_t ov,
                          const double* __restrict__ X, const double* __restrict__ eps, double* __restrict__ T) {
  const int64_t total = (int64_t)nt * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / ov);
    const int64_t ia = t % ov;
    const int k = src[r];
    double v = R[(int64_t)k * ov + ia];
    if (eps) v -= eps[r] * X[(int64_t)k * ov + ia];
    T[t] = v / precond_den(theta[k], de[ia]);
  }
}

// Olsen's correction: the two sums x.(D - theta)^-1 r and x.(D - theta)^-1 x per corrected pair, in a
// fixed order (partial[2][nt][nblk], then eps = first / second)
__global__ __launch_bounds__(256) void k_olsen_partial(const double* __restrict__ R, const double* __restrict__ X,
                                                       const double* __restrict__ theta,
                                                       const double* __restrict__ de, const int* __restrict__ src,
                                                       int nt, int64_t ov, double* __restrict__ partial) {
  __shared__ double red[2][256];
  const int r = blockIdx.y, k = src[r];
  const int64_t per = (ov + gridDim.x - 1) / gridDim.x;
  const int64_t b = blockIdx.x * per, e = min(ov, b + per);
  const double th = theta[k];
  double sa = 0.0, sb = 0.0;
  for (int64_t t = b + threadIdx.x; t < e; t += blockDim.x) {
    const double x = X[(int64_t)k * ov + t], inv = 1.0 / precond_den(th, de[t]);
    sa += x * R[(int64_t)k * ov + t] * inv;
    sb += x * x * inv;
  }
  red[0][threadIdx.x] = sa;
  red[1][threadIdx.x] = sb;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) {
      red[0][threadIdx.x] += red[0][threadIdx.x + d];
      red[1][threadIdx.x] += red[1][threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[((int64_t)0 * nt + r) * gridDim.x + blockIdx.x] = red[0][0];
    partial[((int64_t)1 * nt + r) * gridDim.x + blockIdx.x] = red[1][0];
  }
}

__global__ void k_olsen_eps(const double* partial, int nblk, int nt, double* eps) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nt) return;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nblk; ++q) {
    a += partial[(int64_t)r * nblk + q];
    b += partial[((int64_t)nt + r) * nblk + q];
  }
  eps[r] = fabs(b) > 1e-300 ? a / b : 0.0;
}

__global__ void k_scale_rows(double* T, int nt, int64_t ov, const double* norms) {
  const int64_t total = (int64_t)nt * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double n = norms[t / ov];
    T[t] = n > 0.0 ? T[t] / n : 0.0;
  }
}

// Gram-Schmidt in coefficient space on one block: given G = T T^T (nt x nt, nt <= 64), build the
// coefficients Q = Cf T of an orthonormal basis of span(T), dropping vectors whose remaining norm is
// below drop * ref, where ref is 1 when unit_ref (rows that had unit length before an earlier
// projection against the subspace, so a row that the projection reduced to rounding noise is
// dropped too) and otherwise the row's own norm sqrt(G_jj). Cf is [nt][nt] (rows of kept vectors
// first), count out. One wave: lane i holds component i of the candidate; G and the kept rows sit
// in LDS.
__global__ __launch_bounds__(64) void k_block_mgs(const double* __restrict__ G, int nt, double drop, int unit_ref,
                                                  double* __restrict__ Cf, int* __restrict__ kept) {
  __shared__ double sG[64 * 64];
  __shared__ double sQ[64 * 64];
  const int lane = threadIdx.x;
  for (int t = lane; t < nt * nt; t += 64) sG[t] = G[t];
  __syncthreads();
  auto wsum = [](double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
  };
  int nk = 0;
  for (int j = 0; j < nt; ++j) {
    // candidate c = e_j - sum_q (q . t_j) q,  q . t_j = sum_i Q[q][i] G[i][j]
    double c = (lane == j) ? 1.0 : 0.0;
    const double gij = lane < nt ? sG[lane * nt + j] : 0.0;
    for (int q = 0; q < nk; ++q) {
      const double qi = lane < nt ? sQ[q * 64 + lane] : 0.0;
      const double dot = wsum(qi * gij);
      c -= dot * qi;
    }
    // |c|^2 in the metric G: sum_a c_a (G c)_a
    double gc = 0.0;
    for (int b = 0; b < nt; ++b) gc += (lane < nt ? sG[lane * nt + b] : 0.0) * __shfl(c, b, 64);
    const double n2 = wsum(lane < nt ? c * gc : 0.0);
    const double tj = unit_ref ? 1.0 : sqrt(fmax(sG[j * nt + j], 0.0));
    const double nn = sqrt(fmax(n2, 0.0));
    if (nn > drop * tj && nn > 0.0) {
      if (lane < nt) sQ[nk * 64 + lane] = c / nn;
      ++nk;
    }
    __syncthreads();
  }
  for (int q = 0; q < nk; ++q)
    if (lane < nt) Cf[q * nt + lane] = sQ[q * 64 + lane];
  if (lane == 0) *kept = nk;
}

// eigenvalue copy for the residual kernel
template <typename TS>
__global__ void k_store_rows(const double* __restrict__ T, int64_t n, TS* __restrict__ dst) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = (TS)T[t];
}

// Hn [nall][nn] = V[0:nall] . W[n0:n0+nn]^T. Columns n0.. of H (and rows, by symmetry) take Hn; the
// new-new block takes the average of Hn and its transpose, so H is exactly symmetric and every cell
// has exactly one writer.
// FP64 rows -> FP32 storage of their BF16 roundings (round to nearest even)
__global__ void k_store_rows_bf16(const double* __restrict__ T, int64_t n, float* __restrict__ dst) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t u = __float_as_uint((float)T[t]);
    u += 0x7FFFu + ((u >> 16) & 1u);
    dst[t] = __uint_as_float(u & 0xFFFF0000u);
  }
}

// S[i][j] = (i == j) for i, j < n
__global__ void k_set_eye(double* S, int ld, int n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  S[(int64_t)i * ld + j] = i == j ? 1.0 : 0.0;
}

__global__ void k_sym_update(double* H, int ld, const double* Hn, int nall, int n0, int nn) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nall * nn) return;
  const int i = (int)(t / nn), j = (int)(t % nn);
  if (i < n0) {
    const double v = Hn[t];
    H[(int64_t)i * ld + n0 + j] = v;
    H[(int64_t)(n0 + j) * ld + i] = v;
  } else {
    const int a = i - n0;
    H[(int64_t)i * ld + n0 + j] = 0.5 * (Hn[t] + Hn[(int64_t)(n0 + j) * nn + a]);
  }
}

// H[i][j] = (i == j) ? theta[i] : 0 for i, j < n
__global__ void k_diag_H(double* H, int ld, int n, const double* theta) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  H[(int64_t)i * ld + j] = i == j ? theta[i] : 0.0;
}

__global__ void k_copy_sub(const double* H, int ld, int n, double* out, int ldo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  out[(int64_t)i * ldo + j] = H[(int64_t)i * ld + j];
}

// ---------------------------------------------------------------------------------------------
// driver: a resumable state machine, so a scheduler can interleave the sigma blocks of many runs
// ---------------------------------------------------------------------------------------------
namespace {

inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(ceil_div(n, 256), 65536); }

constexpr int kDavSplit = 512;  // split-K factor cap of the subspace products

}  // namespace

DavidsonRun::DavidsonRun(risp_factors* f, const DavOptions& o, hipStream_t s) : f_(f), o_(o), s_(s) {
  ov_ = (int64_t)f->nocc * f->nvir;
  fp64_ = f->precision == RISP_FP64;
  tvec_ = fp64_ ? DType::F64 : DType::F32;
  vsz_ = fp64_ ? 8 : 4;
  // drop threshold of the Gram-Schmidt: a few times above the rounding of the stored subspace
  drop_ = fp64_ ? 1e-6 : 1e-5;
  nstates_ = o.nstates;
  RISP_CHECK(nstates_ > 0 && nstates_ <= ov_, RISP_E_ARG, "nstates out of range");
  RISP_CHECK(o.tol > 0.0, RISP_E_ARG, "tol must be positive");
  int block = o.block > 0 ? o.block : std::min(2 * nstates_, 30);
  block_ = (int)std::min<int64_t>(std::max(block, nstates_), ov_);
  RISP_CHECK(block_ <= 64, RISP_E_ARG, "block is limited to 64 trial vectors");
  int ms = o.max_space > 0 ? o.max_space : std::max(8 * block_, nstates_ + 2 * block_);
  max_space_ = (int)std::min<int64_t>(ms, ov_);
  RISP_CHECK(max_space_ >= block_, RISP_E_ARG, "max_space must hold at least one block");
  RISP_CHECK(max_space_ + block_ <= kSubspaceMaxN, RISP_E_ARG, "max_space too large for the subspace solver");
  RISP_CHECK(ov_ < (1ll << 31), RISP_E_SHAPE, "nocc*nvir too large");
  cap_ = max_space_ + block_;
  ld_ = cap_;
  max_iter_ = o.max_iter > 0 ? o.max_iter : 200;
  const int64_t ov = ov_;
  if (o.spill) {
    V_.alloc_pinned((size_t)cap_ * ov * vsz_);
    W_.alloc_pinned((size_t)cap_ * ov * vsz_);
  } else {
    V_.alloc((size_t)cap_ * ov * vsz_);
    W_.alloc((size_t)cap_ * ov * vsz_);
  }
  H_.alloc((size_t)ld_ * ld_ * 8);
  Hw_.alloc((size_t)ld_ * ld_ * 8);
  Zs_.alloc((size_t)ld_ * ld_ * 8);
  eigws_.alloc(subspace_eig_workspace(cap_, std::min(2 * block_, cap_)));
  theta_.alloc((size_t)ld_ * 8);
  res_.X.alloc((size_t)block_ * ov * 8);
  AX_.alloc((size_t)block_ * ov * 8);
  T_.alloc((size_t)block_ * ov * 8);
  T2_.alloc((size_t)block_ * ov * 8);
  Cmix_.alloc((size_t)cap_ * block_ * 8);
  G_.alloc((size_t)block_ * block_ * 8);
  Cf_.alloc((size_t)block_ * block_ * 8);
  nblk_ = (int)std::min<int64_t>(64, std::max<int64_t>(1, ov / 4096));
  partial_.alloc((size_t)cap_ * nblk_ * 8);
  norms_.alloc((size_t)cap_ * 8);
  eps_.alloc((size_t)block_ * 8);
  kept_.alloc(sizeof(int));
  src_.alloc((size_t)block_ * sizeof(int));
  Hn_.alloc((size_t)cap_ * block_ * 8);
  split_.alloc((size_t)kDavSplit * cap_ * block_ * 8);
  if (o.bf16_basis) {
    RISP_CHECK(!fp64_, RISP_E_ARG, "a BF16-valued basis needs FP32 trial vectors");
    S_.alloc((size_t)ld_ * ld_ * 8);
    Ls_.alloc((size_t)cap_ * cap_ * 8);
    Li_.alloc((size_t)cap_ * cap_ * 8);
    T1_.alloc((size_t)cap_ * cap_ * 8);
    Y_.alloc((size_t)ld_ * ld_ * 8);
  }
  hnorm_.assign(block_, 0.0);
  htheta_.assign(ld_, 0.0);

  // ---- initial subspace ----
  if (o.nx0 > 0 && o.x0_dev) {
    const int n0 = std::min(o.nx0, block_);
    RISP_HIP(hipMemcpyAsync(T_.get(), o.x0_dev, (size_t)n0 * ov * 8, hipMemcpyDeviceToDevice, s_));
    const int nk = orth_block(n0, false);
    RISP_CHECK(nk > 0, RISP_E_ARG, "initial vectors are zero or dependent");
    store_T(0, nk);
    rq_ = {0, nk};
  } else {
    // unit vectors at the lowest diagonal elements of A, ties broken by (i, a)
    std::vector<double> de(ov);
    RISP_HIP(hipMemcpyAsync(de.data(), f->diag64.get() ? f->diag64.get() : f->de64.get(), ov * 8,
                            hipMemcpyDeviceToHost, s_));
    RISP_HIP(hipStreamSynchronize(s_));
    std::vector<int> idx(ov);
    std::iota(idx.begin(), idx.end(), 0);
    std::partial_sort(idx.begin(), idx.begin() + block_, idx.end(),
                      [&](int a, int b) { return de[a] < de[b] || (de[a] == de[b] && a < b); });
    RISP_HIP(hipMemcpyAsync(src_.get(), idx.data(), block_ * sizeof(int), hipMemcpyHostToDevice, s_));
    RISP_HIP(hipMemsetAsync(V_.get(), 0, (size_t)block_ * ov * vsz_, s_));
    if (fp64_) k_unit_rows<double><<<1, 64, 0, s_>>>(V_.as<double>(), ov, src_.as<int>(), block_);
    else k_unit_rows<float><<<1, 64, 0, s_>>>(V_.as<float>(), ov, src_.as<int>(), block_);
    RISP_LAUNCHED();
    RISP_HIP(hipStreamSynchronize(s_));  // the host index list dies at return
    rq_ = {0, block_};
  }
  state_ = State::Init;
}

void* DavidsonRun::vrow(DevBuf& b, int r) { return static_cast<char*>(b.get()) + (size_t)r * ov_ * vsz_; }

bool DavidsonRun::next(Request& rq) const {
  if (state_ == State::Done) return false;
  rq.r0 = rq_.r0;
  rq.n = rq_.n;
  rq.X = const_cast<DavidsonRun*>(this)->vrow(const_cast<DevBuf&>(V_), rq_.r0);
  rq.S = const_cast<DavidsonRun*>(this)->vrow(const_cast<DevBuf&>(W_), rq_.r0);
  return true;
}

void DavidsonRun::update_H(int nall, int n0, int nn) {
  Gemm g;
  g.M = nall;
  g.N = nn;
  g.K = (int)ov_;
  g.tin = DType::F64;
  g.tout = DType::F64;
  g.mem_a = tvec_;
  g.mem_b = tvec_;
  g.A = V_.get();
  g.lda = ov_;
  g.B = vrow(W_, n0);
  g.ldb = ov_;
  g.C = Hn_.get();
  g.ldc = nn;
  g.ksplit = std::min(kDavSplit, gemm_auto_split(g));
  gemm(g, split_.get(), s_);
  k_sym_update<<<ceil_div((int64_t)nall * nn, 256), 256, 0, s_>>>(H_.as<double>(), ld_, Hn_.as<double>(), nall, n0, nn);
  RISP_LAUNCHED();
}

// S rows / columns n0 .. n0 + nn of V^T V (bf16_basis)
void DavidsonRun::update_S(int nall, int n0, int nn) {
  Gemm g;
  g.M = nall;
  g.N = nn;
  g.K = (int)ov_;
  g.tin = DType::F64;
  g.tout = DType::F64;
  g.mem_a = tvec_;
  g.mem_b = tvec_;
  g.A = V_.get();
  g.lda = ov_;
  g.B = vrow(V_, n0);
  g.ldb = ov_;
  g.C = Hn_.get();
  g.ldc = nn;
  g.ksplit = std::min(kDavSplit, gemm_auto_split(g));
  gemm(g, split_.get(), s_);
  k_sym_update<<<ceil_div((int64_t)nall * nn, 256), 256, 0, s_>>>(S_.as<double>(), ld_, Hn_.as<double>(), nall, n0, nn);
  RISP_LAUNCHED();
}

// Lowest kk pairs of H c = theta S c (H in Hw_): S = L L^T, L^-1 H L^-T y = theta y, c = L^-T y (Zs_)
void DavidsonRun::generalized_eig(int kk) {
  const int n = nsub_;
  k_copy_sub<<<ceil_div((int64_t)n * n, 256), 256, 0, s_>>>(S_.as<double>(), ld_, n, Ls_.as<double>(), n);
  RISP_LAUNCHED();
  try {
    cholesky(Ls_.as<double>(), n, s_);
  } catch (const Error&) {
    throw Error(RISP_E_STATE, "Davidson: the projected overlap of the BF16-valued basis is not positive definite");
  }
  tri_inverse(Ls_.as<double>(), Li_.as<double>(), n, s_);
  Gemm g;  // T1 = H L^-T: T1[i][j] = sum_t H[i][t] Li[j][t]
  g.M = n;
  g.N = n;
  g.K = n;
  g.tin = g.tout = DType::F64;
  g.A = Hw_.get();
  g.lda = ld_;
  g.B = Li_.get();
  g.ldb = n;
  g.C = T1_.get();
  g.ldc = n;
  gemm(g, nullptr, s_);
  Gemm h = g;  // Hw = L^-1 T1: Hw[i][j] = sum_t Li[i][t] T1[t][j]
  h.A = Li_.get();
  h.lda = n;
  h.B = T1_.get();
  h.ldb = n;
  h.b_kc = false;
  h.C = Hw_.get();
  h.ldc = ld_;
  gemm(h, nullptr, s_);
  subspace_eig(Hw_.as<double>(), n, ld_, kk, theta_.as<double>(), Y_.as<double>(), eigws_.as<double>(), s_);
  Gemm z;  // Zs = L^-T Y: Zs[r][q] = sum_t Li[t][r] Y[t][q]
  z.M = n;
  z.N = kk;
  z.K = n;
  z.tin = z.tout = DType::F64;
  z.A = Li_.get();
  z.lda = n;
  z.a_kc = false;
  z.B = Y_.get();
  z.ldb = ld_;
  z.b_kc = false;
  z.C = Zs_.get();
  z.ldc = ld_;
  gemm(z, nullptr, s_);
}

void DavidsonRun::row_norms(const double* R, int k, double* out_dev) {
  k_row_sumsq<<<dim3(nblk_, k), 256, 0, s_>>>(R, ov_, partial_.as<double>());
  RISP_LAUNCHED();
  k_finish_norms<<<ceil_div(k, 64), 64, 0, s_>>>(partial_.as<double>(), nblk_, k, out_dev);
  RISP_LAUNCHED();
}

// out [k][ov] (FP64) = alpha Cm^T Vsrc + beta out, Cm [nsub][ldcm], Vsrc rows in the vector type
void DavidsonRun::combine_rows(const double* Cm, int ldcm, int nsub, int k, const void* Vsrc, double* out,
                               double alpha, double beta) {
  Gemm g;
  g.M = k;
  g.N = (int)ov_;
  g.K = nsub;
  g.tin = DType::F64;
  g.tout = DType::F64;
  g.mem_a = DType::F64;
  g.mem_b = tvec_;
  g.A = Cm;  // A[i][s] = Cm[s][i]
  g.lda = ldcm;
  g.a_kc = false;
  g.B = Vsrc;  // B[ia][s] = V[s][ia]
  g.ldb = ov_;
  g.b_kc = false;
  g.C = out;
  g.ldc = ov_;
  g.alpha = alpha;
  g.beta = beta;
  gemm(g, nullptr, s_);
}

// orthonormalise the nt FP64 rows of T within the block (coefficient-space Gram-Schmidt, twice).
// unit_ref: the rows had unit length before they were projected off the subspace, and the drop test
// compares with that length (first pass; the second pass sees rows of unit length anyway)
int DavidsonRun::orth_block(int nt, bool unit_ref) {
  RISP_CHECK(nt <= 64, RISP_E_ARG, "block orthonormalisation handles at most 64 vectors");
  int nk = nt;
  for (int pass = 0; pass < 2 && nk > 0; ++pass) {
    Gemm g;
    g.M = nk;
    g.N = nk;
    g.K = (int)ov_;
    g.tin = g.tout = DType::F64;
    g.A = T_.get();
    g.lda = ov_;
    g.B = T_.get();
    g.ldb = ov_;
    g.C = G_.get();
    g.ldc = nk;
    g.ksplit = std::min(kDavSplit, gemm_auto_split(g));
    gemm(g, split_.get(), s_);
    k_block_mgs<<<1, 64, 0, s_>>>(G_.as<double>(), nk, drop_, (unit_ref || pass > 0) ? 1 : 0, Cf_.as<double>(),
                                  kept_.as<int>());
    RISP_LAUNCHED();
    int h = 0;
    RISP_HIP(hipMemcpyAsync(&h, kept_.get(), sizeof(int), hipMemcpyDeviceToHost, s_));
    RISP_HIP(hipStreamSynchronize(s_));
    if (h == 0) return 0;
    Gemm c;  // T2 = Cf T ; T <- T2
    c.M = h;
    c.N = (int)ov_;
    c.K = nk;
    c.tin = c.tout = DType::F64;
    c.A = Cf_.get();
    c.lda = nk;
    c.B = T_.get();  // B[ia][t] = T[t][ia]
    c.ldb = ov_;
    c.b_kc = false;
    c.C = T2_.get();
    c.ldc = ov_;
    gemm(c, nullptr, s_);
    RISP_HIP(hipMemcpyAsync(T_.get(), T2_.get(), (size_t)h * ov_ * 8, hipMemcpyDeviceToDevice, s_));
    nk = h;
  }
  return nk;
}

// project the nt FP64 rows of T off V[0:nsub] (classical Gram-Schmidt, two passes)
void DavidsonRun::project_out(int nsub, int nt) {
  for (int pass = 0; pass < 2 && nsub > 0; ++pass) {
    Gemm g;  // Cmix[r][t] = V[r] . T[t]
    g.M = nsub;
    g.N = nt;
    g.K = (int)ov_;
    g.tin = g.tout = DType::F64;
    g.mem_a = tvec_;
    g.mem_b = DType::F64;
    g.A = V_.get();
    g.lda = ov_;
    g.B = T_.get();
    g.ldb = ov_;
    g.C = Cmix_.get();
    g.ldc = nt;
    g.ksplit = std::min(kDavSplit, gemm_auto_split(g));
    gemm(g, split_.get(), s_);
    combine_rows(Cmix_.as<double>(), nt, nsub, nt, V_.get(), T_.as<double>(), -1.0, 1.0);
  }
}

void DavidsonRun::store_T(int r0, int n) {
  if (o_.bf16_basis) {
    k_store_rows_bf16<<<grid_for((int64_t)n * ov_), 256, 0, s_>>>(T_.as<double>(), (int64_t)n * ov_,
                                                                  reinterpret_cast<float*>(vrow(V_, r0)));
    RISP_LAUNCHED();
    return;
  }
  if (fp64_)
    k_store_rows<double><<<grid_for((int64_t)n * ov_), 256, 0, s_>>>(T_.as<double>(), (int64_t)n * ov_,
                                                                    reinterpret_cast<double*>(vrow(V_, r0)));
  else
    k_store_rows<float><<<grid_for((int64_t)n * ov_), 256, 0, s_>>>(T_.as<double>(), (int64_t)n * ov_,
                                                                   reinterpret_cast<float*>(vrow(V_, r0)));
  RISP_LAUNCHED();
}

// Called after the requested sigma rows are in W. Advances to the next request or finishes.
void DavidsonRun::complete() {
  Timer tsub;
  res_.sigma_vectors += rq_.n;
  res_.sigma_flops += sigma_flops(f_, rq_.n);
  if (state_ == State::Init) {
    nsub_ = rq_.n;
    update_H(nsub_, 0, nsub_);
    if (o_.bf16_basis) update_S(nsub_, 0, nsub_);
  } else if (state_ == State::Append) {
    update_H(nsub_ + rq_.n, nsub_, rq_.n);
    if (o_.bf16_basis) update_S(nsub_ + rq_.n, nsub_, rq_.n);
    nsub_ += rq_.n;
  }
  iterate(tsub);
}

void DavidsonRun::finish(Timer& tsub) {
  RISP_HIP(hipStreamSynchronize(s_));
  res_.t_subspace += tsub.sec();
  state_ = State::Done;
}

// project, orthonormalise and append the nt corrections in T, then request their sigma
void DavidsonRun::append_corrections(int nt, Timer& tsub) {
  project_out(nsub_, nt);
  const int nk = orth_block(nt, true);
  if (nk == 0) {  // no new direction: the subspace cannot grow
    finish(tsub);
    return;
  }
  store_T(nsub_, nk);
  RISP_HIP(hipStreamSynchronize(s_));
  res_.t_subspace += tsub.sec();
  rq_ = {nsub_, nk};
  state_ = State::Append;
}

void DavidsonRun::iterate(Timer& tsub) {
  const int64_t ov = ov_;
  const int it = ++res_.iters;
  double* X = res_.X.as<double>();
  // Rayleigh-Ritz on the subspace
  k_copy_sub<<<ceil_div((int64_t)nsub_ * nsub_, 256), 256, 0, s_>>>(H_.as<double>(), ld_, nsub_, Hw_.as<double>(), ld_);
  RISP_LAUNCHED();
  const int k = std::min(block_, nsub_);
  // Ritz pairs kept by a thick restart; computed only when this iteration may restart
  const int kk = nsub_ + block_ > max_space_ ? std::min(2 * block_, nsub_) : k;
  if (o_.bf16_basis) generalized_eig(kk);
  else subspace_eig(Hw_.as<double>(), nsub_, ld_, kk, theta_.as<double>(), Zs_.as<double>(), eigws_.as<double>(), s_);
  combine_rows(Zs_.as<double>(), ld_, nsub_, k, V_.get(), X, 1.0, 0.0);
  combine_rows(Zs_.as<double>(), ld_, nsub_, k, W_.get(), AX_.as<double>(), 1.0, 0.0);
  k_residual<<<grid_for((int64_t)k * ov), 256, 0, s_>>>(AX_.as<double>(), X, theta_.as<double>(), k, ov);
  RISP_LAUNCHED();
  row_norms(AX_.as<double>(), k, norms_.as<double>());
  RISP_HIP(hipMemcpyAsync(hnorm_.data(), norms_.get(), k * 8, hipMemcpyDeviceToHost, s_));
  RISP_HIP(hipMemcpyAsync(htheta_.data(), theta_.get(), k * 8, hipMemcpyDeviceToHost, s_));
  RISP_HIP(hipStreamSynchronize(s_));
  res_.krows = k;
  double rmax = 0.0;
  for (int j = 0; j < std::min(nstates_, k); ++j) rmax = std::max(rmax, hnorm_[j]);
  res_.resid_hist.push_back(rmax);
  if (o_.log_tag) {
    std::fprintf(stderr, "risp davidson %s: iteration %d, subspace %d, max residual %.3e\n", o_.log_tag, it, nsub_,
                 rmax);
    std::fflush(stderr);
  }
  res_.energies.assign(htheta_.begin(), htheta_.begin() + std::min(nstates_, k));
  if (k >= nstates_ && rmax < o_.tol) {
    res_.converged = true;
    finish(tsub);
    return;
  }
  if (rmax < 0.9 * best_r_) {
    best_r_ = rmax;
    best_it_ = it;
  } else if (o_.stall_iters > 0 && it - best_it_ >= o_.stall_iters && best_r_ <= o_.stall_below) {
    res_.stalled = true;
    finish(tsub);
    return;
  }
  if (it >= max_iter_) {
    finish(tsub);
    return;
  }
  // corrections for the Ritz pairs not yet converged
  std::vector<int> todo;
  const int kc = o_.max_corr > 0 ? std::min(k, std::max(o_.max_corr, nstates_)) : k;
  for (int j = 0; j < kc; ++j)
    if (hnorm_[j] >= o_.tol) todo.push_back(j);
  const int nt = (int)todo.size();
  RISP_HIP(hipMemcpyAsync(src_.get(), todo.data(), nt * sizeof(int), hipMemcpyHostToDevice, s_));
  const double* dg = f_->diag64.get() ? f_->diag64.as<double>() : f_->de64.as<double>();
  if (o_.olsen && nt > 0) {
    k_olsen_partial<<<dim3(nblk_, nt), 256, 0, s_>>>(AX_.as<double>(), X, theta_.as<double>(), dg, src_.as<int>(),
                                                     nt, ov, partial_.as<double>());
    RISP_LAUNCHED();
    k_olsen_eps<<<ceil_div(nt, 64), 64, 0, s_>>>(partial_.as<double>(), nblk_, nt, eps_.as<double>());
    RISP_LAUNCHED();
  }
  k_precond<<<grid_for((int64_t)nt * ov), 256, 0, s_>>>(AX_.as<double>(), theta_.as<double>(), dg,
                                                        src_.as<int>(), nt, ov, X,
                                                        o_.olsen ? eps_.as<double>() : nullptr, T_.as<double>());
  RISP_LAUNCHED();
  row_norms(T_.as<double>(), nt, norms_.as<double>());
  k_scale_rows<<<grid_for((int64_t)nt * ov), 256, 0, s_>>>(T_.as<double>(), nt, ov, norms_.as<double>());
  RISP_LAUNCHED();
  if (nsub_ + nt > max_space_) {
    // thick restart: the lowest `keep` Ritz vectors become the subspace; their products are the same
    // combination of W (no sigma), and the projected matrix is diag(theta)
    const int keep = std::max(1, std::min({kk, cap_ - nt, nsub_}));
    thick_restart(keep);
    ++res_.restarts;
  }
  append_corrections(nt, tsub);
}

// V[0:keep] <- V Z[:, 0:keep], W[0:keep] <- W Z[:, 0:keep] (FP64 products, stored in the vector type),
// H <- diag(theta[0:keep])
void DavidsonRun::thick_restart(int keep) {
  const int64_t ov = ov_;
  const size_t bytes = (size_t)keep * ov * vsz_;
  if (Rv_.bytes() < bytes) Rv_.alloc(bytes);
  if (Rw_.bytes() < bytes) Rw_.alloc(bytes);
  for (int w = 0; w < 2; ++w) {
    Gemm g;  // out[i][ia] = sum_s Z[s][i] src[s][ia]
    g.M = keep;
    g.N = (int)ov;
    g.K = nsub_;
    g.tin = DType::F64;
    g.tout = tvec_;
    g.mem_a = DType::F64;
    g.mem_b = tvec_;
    g.A = Zs_.get();
    g.lda = ld_;
    g.a_kc = false;
    g.B = w == 0 ? V_.get() : W_.get();
    g.ldb = ov;
    g.b_kc = false;
    g.C = w == 0 ? Rv_.get() : Rw_.get();
    g.ldc = ov;
    gemm(g, nullptr, s_);
  }
  RISP_HIP(hipMemcpyAsync(V_.get(), Rv_.get(), bytes, hipMemcpyDefault, s_));
  RISP_HIP(hipMemcpyAsync(W_.get(), Rw_.get(), bytes, hipMemcpyDefault, s_));
  k_diag_H<<<ceil_div((int64_t)keep * keep, 256), 256, 0, s_>>>(H_.as<double>(), ld_, keep, theta_.as<double>());
  RISP_LAUNCHED();
  if (o_.bf16_basis) {  // V Z is S-orthonormal: Z^T S Z = I
    k_set_eye<<<ceil_div((int64_t)keep * keep, 256), 256, 0, s_>>>(S_.as<double>(), ld_, keep);
    RISP_LAUNCHED();
  }
  nsub_ = keep;
}

void davidson(risp_factors* f, const DavOptions& o, const SigmaFn& sigma_fn, DavResult& res) {
  hipStream_t s = f->stream;
  DavidsonRun run(f, o, s);
  DavidsonRun::Request rq;
  double t_sigma = 0.0;
  while (run.next(rq)) {
    RISP_HIP(hipStreamSynchronize(s));
    Timer t;
    sigma_fn(rq.n, rq.X, rq.S);
    RISP_HIP(hipStreamSynchronize(s));
    t_sigma += t.sec();
    run.complete();
  }
  res = std::move(run.result());
  res.t_sigma = t_sigma;
}

}  // namespace risp

// ---------------------------------------------------------------------------------------------
// full TDDFT-risp
// ---------------------------------------------------------------------------------------------
namespace risp {

namespace {

// A[r][c] *= sc[c] for r < rows, c < cols (row stride ld)
__global__ void k_scale_cols(double* A, int rows, int cols, int ld, const double* sc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int r = (int)(t / cols), c = (int)(t % cols);
  A[(int64_t)r * ld + c] *= sc[c];
}

}  // namespace

void davidson_full(risp_factors* f, const DavOptions& o, FullResult& res) {
  hipStream_t s = f->stream;
  const int64_t ov = (int64_t)f->nocc * f->nvir;
  const bool fp64 = f->precision == RISP_FP64;
  const DType tvec = fp64 ? DType::F64 : DType::F32;
  const size_t vsz = fp64 ? 8 : 4;
  const int n = o.nstates;
  RISP_CHECK(n > 0 && n <= ov && 2 * n <= 64, RISP_E_ARG, "full TDDFT: 1 <= nstates <= 32 and <= nocc*nvir");
  RISP_CHECK(o.tol > 0.0, RISP_E_ARG, "tol must be positive");
  RISP_CHECK(ov < (1ll << 31), RISP_E_SHAPE, "nocc*nvir too large");
  const int blk = (int)std::min<int64_t>(std::max(n, o.block > 0 ? o.block : std::min(2 * n, 30)), ov);
  RISP_CHECK(blk <= 64, RISP_E_ARG, "block is limited to 64 trial vectors");
  const int nnew = 2 * n;  // corrections per iteration at most (two per state)
  const int max_space = (int)std::min<int64_t>(o.max_space > 0 ? o.max_space : std::max(8 * blk, 4 * nnew), ov);
  RISP_CHECK(max_space >= std::max(blk, nnew), RISP_E_ARG, "max_space too small");
  const int cap = max_space + nnew;
  RISP_CHECK(cap <= 1024, RISP_E_ARG, "max_space too large for the subspace solver");
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  const int wmax = std::max(blk, nnew);
  DevBuf V((size_t)cap * ov * vsz), WP((size_t)cap * ov * vsz), WM((size_t)cap * ov * vsz);
  DevBuf Pm((size_t)cap * cap * 8), Mm((size_t)cap * cap * 8), Hn((size_t)cap * wmax * 8);
  DevBuf split((size_t)512 * cap * wmax * 8);
  DevBuf L((size_t)cap * cap * 8), Li((size_t)cap * cap * 8), T1((size_t)cap * cap * 8), Sm((size_t)cap * cap * 8);
  DevBuf Zc((size_t)cap * cap * 8), theta((size_t)cap * 8), eigws(subspace_eig_workspace(cap, n));
  DevBuf Ac((size_t)cap * n * 8), Bc((size_t)cap * n * 8), om((size_t)n * 8), sc1((size_t)n * 8), sc2((size_t)n * 8);
  res.XpY.alloc((size_t)n * ov * 8);
  res.XmY.alloc((size_t)n * ov * 8);
  DevBuf R1((size_t)n * ov * 8), R2((size_t)n * ov * 8), T((size_t)nnew * ov * 8), T2((size_t)nnew * ov * 8);
  DevBuf Cmix((size_t)cap * nnew * 8), G(64 * 64 * 8), Cf(64 * 64 * 8), kept(sizeof(int)), src((size_t)nnew * sizeof(int));
  const int nblk = (int)std::min<int64_t>(64, std::max<int64_t>(1, ov / 4096));
  DevBuf partial((size_t)nnew * nblk * 8), norms((size_t)nnew * 8);
  const double* dg = f->diag64.get() ? f->diag64.as<double>() : f->de64.as<double>();
  auto vrow = [&](DevBuf& b, int r) { return static_cast<char*>(b.get()) + (size_t)r * ov * vsz; };

  auto products = [&](int r0, int nn) {
    RISP_HIP(hipStreamSynchronize(s));
    Timer t;
    sigma_full(f, nn, vrow(V, r0), vrow(WP, r0), vrow(WM, r0), s);
    RISP_HIP(hipStreamSynchronize(s));
    res.t_sigma += t.sec();
    res.sigma_vectors += nn;
    const double nK = f->naux_k, no = f->nok, nv = f->nvk;
    res.sigma_flops += sigma_flops(f, nn) + 4.0 * (double)ov * f->naux_j * nn + 4.0 * nK * no * no * nv * nn;
  };
  // columns [n0, n0 + nn) of Msub = V^T W for rows [0, nall)
  auto update = [&](DevBuf& Msub, DevBuf& W, int nall, int n0, int nn) {
    Gemm g;
    g.M = nall;
    g.N = nn;
    g.K = (int)ov;
    g.tin = g.tout = DType::F64;
    g.mem_a = tvec;
    g.mem_b = tvec;
    g.A = V.get();
    g.lda = ov;
    g.B = vrow(W, n0);
    g.ldb = ov;
    g.C = Hn.get();
    g.ldc = nn;
    g.ksplit = std::min(512, gemm_auto_split(g));
    gemm(g, split.get(), s);
    k_sym_update<<<ceil_div((int64_t)nall * nn, 256), 256, 0, s>>>(Msub.as<double>(), cap, Hn.as<double>(), nall, n0,
                                                                   nn);
    RISP_LAUNCHED();
  };
  // out [k][ov] (FP64) = alpha Cm^T Vsrc + beta out, Cm [nsub][ldcm] FP64
  auto combine = [&](const double* Cm, int ldcm, int nsub, int k, const void* Vsrc, double* out, double alpha,
                     double beta) {
    Gemm g;
    g.M = k;
    g.N = (int)ov;
    g.K = nsub;
    g.tin = g.tout = DType::F64;
    g.mem_a = DType::F64;
    g.mem_b = tvec;
    g.A = Cm;
    g.lda = ldcm;
    g.a_kc = false;
    g.B = Vsrc;
    g.ldb = ov;
    g.b_kc = false;
    g.C = out;
    g.ldc = ov;
    g.alpha = alpha;
    g.beta = beta;
    gemm(g, nullptr, s);
  };
  auto row_norms = [&](const double* Rr, int k, std::vector<double>& out) {
    k_row_sumsq<<<dim3(nblk, k), 256, 0, s>>>(Rr, ov, partial.as<double>());
    RISP_LAUNCHED();
    k_finish_norms<<<ceil_div(k, 64), 64, 0, s>>>(partial.as<double>(), nblk, k, norms.as<double>());
    RISP_LAUNCHED();
    out.assign(k, 0.0);
    RISP_HIP(hipMemcpyAsync(out.data(), norms.get(), k * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
  };
  // orthonormalise the nt FP64 rows of B within the block (coefficient-space Gram-Schmidt, twice)
  auto orth = [&](DevBuf& B, int nt, bool unit_ref) {
    int nk = nt;
    for (int pass = 0; pass < 2 && nk > 0; ++pass) {
      Gemm g;
      g.M = nk;
      g.N = nk;
      g.K = (int)ov;
      g.tin = g.tout = DType::F64;
      g.A = B.get();
      g.lda = ov;
      g.B = B.get();
      g.ldb = ov;
      g.C = G.get();
      g.ldc = nk;
      g.ksplit = std::min(512, gemm_auto_split(g));
      gemm(g, split.get(), s);
      k_block_mgs<<<1, 64, 0, s>>>(G.as<double>(), nk, fp64 ? 1e-6 : 1e-5, (unit_ref || pass > 0) ? 1 : 0,
                                    Cf.as<double>(), kept.as<int>());
      RISP_LAUNCHED();
      int h = 0;
      RISP_HIP(hipMemcpyAsync(&h, kept.get(), sizeof(int), hipMemcpyDeviceToHost, s));
      RISP_HIP(hipStreamSynchronize(s));
      if (h == 0) return 0;
      Gemm c;  // T2 = Cf B ; B <- T2
      c.M = h;
      c.N = (int)ov;
      c.K = nk;
      c.tin = c.tout = DType::F64;
      c.A = Cf.get();
      c.lda = nk;
      c.B = B.get();
      c.ldb = ov;
      c.b_kc = false;
      c.C = T2.get();
      c.ldc = ov;
      gemm(c, nullptr, s);
      RISP_HIP(hipMemcpyAsync(B.get(), T2.get(), (size_t)h * ov * 8, hipMemcpyDeviceToDevice, s));
      nk = h;
    }
    return nk;
  };
  // project the nt FP64 rows of B off V[0:nsub] (classical Gram-Schmidt, two passes)
  auto project = [&](DevBuf& B, int nsub, int nt) {
    for (int pass = 0; pass < 2 && nsub > 0; ++pass) {
      Gemm g;  // Cmix[r][t] = V[r] . B[t]
      g.M = nsub;
      g.N = nt;
      g.K = (int)ov;
      g.tin = g.tout = DType::F64;
      g.mem_a = tvec;
      g.mem_b = DType::F64;
      g.A = V.get();
      g.lda = ov;
      g.B = B.get();
      g.ldb = ov;
      g.C = Cmix.get();
      g.ldc = nt;
      g.ksplit = std::min(512, gemm_auto_split(g));
      gemm(g, split.get(), s);
      combine(Cmix.as<double>(), nt, nsub, nt, V.get(), B.as<double>(), -1.0, 1.0);
    }
  };
  auto store = [&](DevBuf& B, int r0, int nn) {
    if (fp64)
      k_store_rows<double><<<grid_for((int64_t)nn * ov), 256, 0, s>>>(B.as<double>(), (int64_t)nn * ov,
                                                                      reinterpret_cast<double*>(vrow(V, r0)));
    else
      k_store_rows<float><<<grid_for((int64_t)nn * ov), 256, 0, s>>>(B.as<double>(), (int64_t)nn * ov,
                                                                     reinterpret_cast<float*>(vrow(V, r0)));
    RISP_LAUNCHED();
  };

  // ---- guess: unit vectors at the lowest diagonal elements of A, ties by (i, a) ----
  {
    std::vector<double> d(ov);
    RISP_HIP(hipMemcpyAsync(d.data(), dg, ov * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    std::vector<int> idx(ov);
    std::iota(idx.begin(), idx.end(), 0);
    std::partial_sort(idx.begin(), idx.begin() + blk, idx.end(),
                      [&](int a, int b) { return d[a] < d[b] || (d[a] == d[b] && a < b); });
    DevBuf srcg((size_t)blk * sizeof(int));
    RISP_HIP(hipMemcpyAsync(srcg.get(), idx.data(), blk * sizeof(int), hipMemcpyHostToDevice, s));
    RISP_HIP(hipMemsetAsync(V.get(), 0, (size_t)blk * ov * vsz, s));
    if (fp64) k_unit_rows<double><<<1, 64, 0, s>>>(V.as<double>(), ov, srcg.as<int>(), blk);
    else k_unit_rows<float><<<1, 64, 0, s>>>(V.as<float>(), ov, srcg.as<int>(), blk);
    RISP_LAUNCHED();
    RISP_HIP(hipStreamSynchronize(s));
  }
  int nsub = blk;
  products(0, nsub);
  update(Pm, WP, nsub, 0, nsub);
  update(Mm, WM, nsub, 0, nsub);

  std::vector<double> hth, hom(n), r1, r2;
  for (int it = 1;; ++it) {
    Timer tsub;
    const int k = nsub, nw = std::min(n, k);
    // Mm = L L^T, S = L^T Pm L, S c = Omega^2 c
    k_copy_sub<<<ceil_div((int64_t)k * k, 256), 256, 0, s>>>(Mm.as<double>(), cap, k, L.as<double>(), k);
    RISP_LAUNCHED();
    try {
      cholesky(L.as<double>(), k, s);
    } catch (const Error&) {
      throw Error(RISP_E_STATE, "full TDDFT: the projected A - B is not positive definite (unstable ground state)");
    }
    tri_inverse(L.as<double>(), Li.as<double>(), k, s);
    {
      Gemm g;  // T1 = Pm L
      g.M = k;
      g.N = k;
      g.K = k;
      g.tin = g.tout = DType::F64;
      g.A = Pm.get();
      g.lda = cap;
      g.B = L.get();  // B[j][t] = L[t][j]
      g.ldb = k;
      g.b_kc = false;
      g.C = T1.get();
      g.ldc = k;
      gemm(g, nullptr, s);
      Gemm h;  // S = L^T T1
      h.M = k;
      h.N = k;
      h.K = k;
      h.tin = h.tout = DType::F64;
      h.A = L.get();  // A[i][t] = L[t][i]
      h.lda = k;
      h.a_kc = false;
      h.B = T1.get();  // B[j][t] = T1[t][j]
      h.ldb = k;
      h.b_kc = false;
      h.C = Sm.get();
      h.ldc = k;
      gemm(h, nullptr, s);
    }
    subspace_eig(Sm.as<double>(), k, k, nw, theta.as<double>(), Zc.as<double>(), eigws.as<double>(), s);
    hth.assign(nw, 0.0);
    RISP_HIP(hipMemcpyAsync(hth.data(), theta.get(), nw * 8, hipMemcpyDeviceToHost, s));
    RISP_HIP(hipStreamSynchronize(s));
    std::vector<double> h1(nw), h2(nw);
    for (int q = 0; q < nw; ++q) {
      RISP_CHECK(hth[q] > 0.0, RISP_E_STATE, "full TDDFT: non-positive Omega^2 in the subspace");
      hom[q] = std::sqrt(hth[q]);
      h1[q] = 1.0 / std::sqrt(hom[q]);
      h2[q] = std::sqrt(hom[q]);
    }
    RISP_HIP(hipMemcpyAsync(om.get(), hom.data(), nw * 8, hipMemcpyHostToDevice, s));
    RISP_HIP(hipMemcpyAsync(sc1.get(), h1.data(), nw * 8, hipMemcpyHostToDevice, s));
    RISP_HIP(hipMemcpyAsync(sc2.get(), h2.data(), nw * 8, hipMemcpyHostToDevice, s));
    {
      Gemm a;  // Ac[s][q] = sum_t L[s][t] c[t][q]
      a.M = k;
      a.N = nw;
      a.K = k;
      a.tin = a.tout = DType::F64;
      a.A = L.get();
      a.lda = k;
      a.B = Zc.get();  // B[q][t] = Z[t][q]
      a.ldb = k;
      a.b_kc = false;
      a.C = Ac.get();
      a.ldc = nw;
      gemm(a, nullptr, s);
      Gemm b = a;  // Bc[s][q] = sum_t Li[t][s] c[t][q]
      b.A = Li.get();
      b.a_kc = false;
      b.C = Bc.get();
      gemm(b, nullptr, s);
      k_scale_cols<<<ceil_div((int64_t)k * nw, 256), 256, 0, s>>>(Ac.as<double>(), k, nw, nw, sc1.as<double>());
      RISP_LAUNCHED();
      k_scale_cols<<<ceil_div((int64_t)k * nw, 256), 256, 0, s>>>(Bc.as<double>(), k, nw, nw, sc2.as<double>());
      RISP_LAUNCHED();
    }
    double* xp = res.XpY.as<double>();
    double* xm = res.XmY.as<double>();
    combine(Ac.as<double>(), nw, k, nw, V.get(), xp, 1.0, 0.0);
    combine(Bc.as<double>(), nw, k, nw, V.get(), xm, 1.0, 0.0);
    combine(Ac.as<double>(), nw, k, nw, WP.get(), R1.as<double>(), 1.0, 0.0);
    combine(Bc.as<double>(), nw, k, nw, WM.get(), R2.as<double>(), 1.0, 0.0);
    k_residual<<<grid_for((int64_t)nw * ov), 256, 0, s>>>(R1.as<double>(), xm, om.as<double>(), nw, ov);
    RISP_LAUNCHED();
    k_residual<<<grid_for((int64_t)nw * ov), 256, 0, s>>>(R2.as<double>(), xp, om.as<double>(), nw, ov);
    RISP_LAUNCHED();
    row_norms(R1.as<double>(), nw, r1);
    row_norms(R2.as<double>(), nw, r2);
    res.iters = it;
    res.omega.assign(hom.begin(), hom.begin() + nw);
    double rmax = 0.0;
    std::vector<int> todo;
    for (int q = 0; q < nw; ++q) {
      rmax = std::max(rmax, std::max(r1[q], r2[q]));
      if (std::max(r1[q], r2[q]) >= o.tol) todo.push_back(q);
    }
    res.resid_hist.push_back(rmax);
    if (o.log_tag) {
      std::fprintf(stderr, "risp davidson %s: iteration %d, subspace %d, max residual %.3e\n", o.log_tag, it, nsub,
                   rmax);
      std::fflush(stderr);
    }
    if (nw >= n && todo.empty()) {
      res.converged = true;
      res.t_subspace += tsub.sec();
      break;
    }
    if (it >= max_iter) {
      res.t_subspace += tsub.sec();
      break;
    }
    // corrections t = r / (Omega - diag A) for both residuals of the unconverged states
    const int nq = (int)todo.size();
    RISP_HIP(hipMemcpyAsync(src.get(), todo.data(), nq * sizeof(int), hipMemcpyHostToDevice, s));
    k_precond<<<grid_for((int64_t)nq * ov), 256, 0, s>>>(R1.as<double>(), om.as<double>(), dg, src.as<int>(), nq, ov,
                                                         nullptr, nullptr, T.as<double>());
    RISP_LAUNCHED();
    k_precond<<<grid_for((int64_t)nq * ov), 256, 0, s>>>(R2.as<double>(), om.as<double>(), dg, src.as<int>(), nq, ov,
                                                         nullptr, nullptr, T.as<double>() + (size_t)nq * ov);
    RISP_LAUNCHED();
    int nt = 2 * nq;
    {
      std::vector<double> tn;
      row_norms(T.as<double>(), nt, tn);
      RISP_HIP(hipMemcpyAsync(norms.get(), tn.data(), nt * 8, hipMemcpyHostToDevice, s));
      k_scale_rows<<<grid_for((int64_t)nt * ov), 256, 0, s>>>(T.as<double>(), nt, ov, norms.as<double>());
      RISP_LAUNCHED();
    }
    if (nsub + nt > max_space) {
      // restart: the subspace becomes X + Y and X - Y of the current states, products recomputed
      DevBuf Rb((size_t)2 * nw * ov * 8);
      RISP_HIP(hipMemcpyAsync(Rb.get(), xp, (size_t)nw * ov * 8, hipMemcpyDeviceToDevice, s));
      RISP_HIP(hipMemcpyAsync(Rb.as<double>() + (size_t)nw * ov, xm, (size_t)nw * ov * 8, hipMemcpyDeviceToDevice, s));
      // orthonormalise through T2 (which orth uses as its product buffer): copy in, orthonormalise, store
      DevBuf Tb((size_t)2 * nw * ov * 8);
      RISP_HIP(hipMemcpyAsync(Tb.get(), Rb.get(), (size_t)2 * nw * ov * 8, hipMemcpyDeviceToDevice, s));
      const int nr = orth(Tb, 2 * nw, false);
      RISP_CHECK(nr > 0, RISP_E_STATE, "full TDDFT: restart basis vanished");
      store(Tb, 0, nr);
      nsub = nr;
      products(0, nsub);
      update(Pm, WP, nsub, 0, nsub);
      update(Mm, WM, nsub, 0, nsub);
      ++res.restarts;
    }
    project(T, nsub, nt);
    const int nk = orth(T, nt, true);
    if (nk == 0) {  // no new direction: the subspace cannot grow
      res.t_subspace += tsub.sec();
      break;
    }
    store(T, nsub, nk);
    res.t_subspace += tsub.sec();
    products(nsub, nk);
    update(Pm, WP, nsub + nk, nsub, nk);
    update(Mm, WM, nsub + nk, nsub, nk);
    nsub += nk;
  }
  RISP_HIP(hipStreamSynchronize(s));
}

}  // namespace risp
