// Blocked FP64 Cholesky and triangular inverse (panel kernels + MFMA GEMM updates), and the small
// gather / convert / scale kernels of the factor build and the sigma product.
#include <algorithm>
#include <cmath>

#include "linalg.hpp"

namespace risp {

constexpr int kNB = 32;  // panel width

__device__ __forceinline__ uint16_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f_(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---- Cholesky ----
__global__ void k_potrf_diag(double* A, int n, int j0, int jb, int* info) {
  __shared__ double a[kNB][kNB + 1];
  for (int t = threadIdx.x; t < jb * jb; t += blockDim.x) {
    const int i = t / jb, j = t % jb;
    a[i][j] = j <= i ? A[(int64_t)(j0 + i) * n + j0 + j] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < jb; ++k) {
    if (threadIdx.x == 0) {
      const double d = a[k][k];
      if (!(d > 0.0)) {
        if (*info == 0) *info = j0 + k + 1;
        a[k][k] = 1.0;  // keep going with a harmless pivot; the host reports the failure
      } else {
        a[k][k] = sqrt(d);
      }
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < jb; i += blockDim.x) a[i][k] /= a[k][k];
    __syncthreads();
    for (int t = threadIdx.x; t < jb * jb; t += blockDim.x) {
      const int i = t / jb, j = t % jb;
      if (j > k && j <= i) a[i][j] -= a[i][k] * a[j][k];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < jb * jb; t += blockDim.x) {
    const int i = t / jb, j = t % jb;
    A[(int64_t)(j0 + i) * n + j0 + j] = j <= i ? a[i][j] : 0.0;
  }
}

// rows r >= j0 + jb: A[r][j0:j0+jb] <- A[r][j0:j0+jb] L_kk^-T (forward substitution per row)
__global__ void k_trsm_panel(double* A, int n, int j0, int jb) {
  __shared__ double L[kNB][kNB + 1];
  for (int t = threadIdx.x; t < jb * jb; t += blockDim.x) {
    const int i = t / jb, j = t % jb;
    L[i][j] = A[(int64_t)(j0 + i) * n + j0 + j];
  }
  __syncthreads();
  const int r = j0 + jb + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double x[kNB];
  double* row = A + (int64_t)r * n + j0;
  for (int c = 0; c < jb; ++c) {
    double v = row[c];
    for (int t = 0; t < c; ++t) v -= x[t] * L[c][t];
    x[c] = v / L[c][c];
  }
  for (int c = 0; c < jb; ++c) row[c] = x[c];
}

__global__ void k_zero_upper(double* A, int n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  if (j > i) A[t] = 0.0;
}

void cholesky(double* A, int n, hipStream_t s) {
  DevBuf info(sizeof(int));
  RISP_HIP(hipMemsetAsync(info.get(), 0, sizeof(int), s));
  for (int j0 = 0; j0 < n; j0 += kNB) {
    const int jb = std::min(kNB, n - j0);
    k_potrf_diag<<<1, 256, 0, s>>>(A, n, j0, jb, info.as<int>());
    RISP_LAUNCHED();
    const int r0 = j0 + jb, nr = n - r0;
    if (nr <= 0) break;
    k_trsm_panel<<<ceil_div(nr, 64), 64, 0, s>>>(A, n, j0, jb);
    RISP_LAUNCHED();
    Gemm g;
    g.M = nr;
    g.N = nr;
    g.K = jb;
    g.tin = g.tout = DType::F64;
    g.A = A + (int64_t)r0 * n + j0;
    g.lda = n;
    g.a_kc = true;
    g.B = g.A;
    g.ldb = n;
    g.b_kc = true;
    g.C = A + (int64_t)r0 * n + r0;
    g.ldc = n;
    g.alpha = -1.0;
    g.beta = 1.0;
    gemm(g, nullptr, s);
  }
  k_zero_upper<<<ceil_div((int64_t)n * n, 256), 256, 0, s>>>(A, n);
  RISP_LAUNCHED();
  int h = 0;
  RISP_HIP(hipMemcpyAsync(&h, info.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  RISP_HIP(hipStreamSynchronize(s));
  RISP_CHECK(h == 0, RISP_E_ARG,
             "auxiliary metric is not positive definite (pivot " + std::to_string(h) + ")");
}

// ---- triangular inverse ----
// X[k0:k0+kb][0:k0+kb] <- identity block (ones on the diagonal of the kb x kb block)
__global__ void k_set_rhs(double* X, int n, int k0, int kb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int ncol = k0 + kb;
  if (t >= (int64_t)kb * ncol) return;
  const int r = (int)(t / ncol), c = (int)(t % ncol);
  X[(int64_t)(k0 + r) * n + c] = (c == k0 + r) ? 1.0 : 0.0;
}

// solve L_kk Y = X[k0:k0+kb][c] for each column c < k0 + kb (one thread per column)
__global__ void k_trsv_block(const double* L, double* X, int n, int k0, int kb) {
  __shared__ double Lk[kNB][kNB + 1];
  for (int t = threadIdx.x; t < kb * kb; t += blockDim.x) {
    const int i = t / kb, j = t % kb;
    Lk[i][j] = L[(int64_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k0 + kb) return;
  double y[kNB];
  for (int r = 0; r < kb; ++r) {
    double v = X[(int64_t)(k0 + r) * n + c];
    for (int t = 0; t < r; ++t) v -= Lk[r][t] * y[t];
    y[r] = v / Lk[r][r];
  }
  for (int r = 0; r < kb; ++r) X[(int64_t)(k0 + r) * n + c] = y[r];
}

void tri_inverse(const double* L, double* X, int n, hipStream_t s) {
  RISP_HIP(hipMemsetAsync(X, 0, (size_t)n * n * sizeof(double), s));
  for (int k0 = 0; k0 < n; k0 += kNB) {
    const int kb = std::min(kNB, n - k0);
    k_set_rhs<<<ceil_div((int64_t)kb * (k0 + kb), 256), 256, 0, s>>>(X, n, k0, kb);
    RISP_LAUNCHED();
    if (k0 > 0) {
      // X[k0:k0+kb][0:k0] -= L[k0:k0+kb][0:k0] X[0:k0][0:k0]
      Gemm g;
      g.M = kb;
      g.N = k0;
      g.K = k0;
      g.tin = g.tout = DType::F64;
      g.A = L + (int64_t)k0 * n;
      g.lda = n;
      g.a_kc = true;
      g.B = X;  // B[j][k] = X[k][j]
      g.ldb = n;
      g.b_kc = false;
      g.C = X + (int64_t)k0 * n;
      g.ldc = n;
      g.alpha = -1.0;
      g.beta = 1.0;
      gemm(g, nullptr, s);
    }
    k_trsv_block<<<ceil_div(k0 + kb, 64), 64, 0, s>>>(L, X, n, k0, kb);
    RISP_LAUNCHED();
  }
}

// ---- data movement ----
__global__ void k_gather_transpose(const double* __restrict__ C, int64_t ldc, int nao,
                                   const int* __restrict__ cols, int col0, int nr,
                                   double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nr * nao) return;
  const int r = (int)(t / nao), mu = (int)(t % nao);
  const int c = cols ? cols[r] : col0 + r;
  out[t] = C[(int64_t)mu * ldc + c];
}

void gather_transpose(const double* C, int64_t ldc, int nao, const int* cols, int col0, int nr,
                      double* out, hipStream_t s) {
  if ((int64_t)nr * nao == 0) return;
  k_gather_transpose<<<ceil_div((int64_t)nr * nao, 256), 256, 0, s>>>(C, ldc, nao, cols, col0, nr, out);
  RISP_LAUNCHED();
}

template <typename TS, typename TD> __device__ __forceinline__ TD cvt(TS v) { return (TD)v; }
template <> __device__ __forceinline__ uint16_t cvt<double, uint16_t>(double v) { return f2bf_rne((float)v); }
template <> __device__ __forceinline__ uint16_t cvt<float, uint16_t>(float v) { return f2bf_rne(v); }
template <> __device__ __forceinline__ uint16_t cvt<uint16_t, uint16_t>(uint16_t v) { return v; }

template <typename TS, typename TD>
__global__ void k_convert(const TS* __restrict__ a, TD* __restrict__ b, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = cvt<TS, TD>(a[t]);
}

void convert(const void* src, DType ts, void* dst, DType td, int64_t n, hipStream_t s) {
  if (n == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 1 << 16);
  if (ts == DType::F64 && td == DType::F32)
    k_convert<double, float><<<grid, 256, 0, s>>>((const double*)src, (float*)dst, n);
  else if (ts == DType::F64 && td == DType::BF16)
    k_convert<double, uint16_t><<<grid, 256, 0, s>>>((const double*)src, (uint16_t*)dst, n);
  else if (ts == DType::F32 && td == DType::BF16)
    k_convert<float, uint16_t><<<grid, 256, 0, s>>>((const float*)src, (uint16_t*)dst, n);
  else if (ts == DType::F32 && td == DType::F64)
    k_convert<float, double><<<grid, 256, 0, s>>>((const float*)src, (double*)dst, n);
  else if (ts == td)
    RISP_HIP(hipMemcpyAsync(dst, src, n * dtype_size(ts), hipMemcpyDeviceToDevice, s));
  else
    throw Error(RISP_E_ARG, "convert: unsupported type pair");
  RISP_LAUNCHED();
}

__global__ __launch_bounds__(256) void k_row_pow2(const double* __restrict__ A, int64_t cols,
                                                  float* __restrict__ scale) {
  __shared__ double red[256];
  const double* a = A + (int64_t)blockIdx.x * cols;
  double m = 0.0;
  for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) m = fmax(m, fabs(a[c]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = red[0];
    double sc = 1.0;
    if (mx > 0.0) {
      int e;
      const double f = frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
      sc = ldexp(1.0, f == 0.5 ? e - 1 : e);  // smallest power of two >= mx
    }
    scale[blockIdx.x] = (float)sc;
  }
}

void row_pow2_scales(const double* A, int rows, int64_t cols, float* scale, hipStream_t s) {
  if (rows == 0) return;
  k_row_pow2<<<rows, 256, 0, s>>>(A, cols, scale);
  RISP_LAUNCHED();
}

// out[r] = max(out[r] (if acc), max_c |A[r * lda + c]|), one block per row
__global__ __launch_bounds__(256) void k_row_absmax(const double* __restrict__ A, int64_t cols, int64_t lda,
                                                    double* __restrict__ out, int acc) {
  __shared__ double red[256];
  const double* a = A + (int64_t)blockIdx.x * lda;
  double m = 0.0;
  for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) m = fmax(m, fabs(a[c]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = acc ? fmax(out[blockIdx.x], red[0]) : red[0];
}

// out[p] = max(out[p] (if acc), max |A[p][i][j]| over j >= i) for A [np][nr][nc], one block per p
__global__ __launch_bounds__(256) void k_row_absmax_upper(const double* __restrict__ A, int nr, int nc,
                                                          double* __restrict__ out, int acc) {
  __shared__ double red[256];
  const int64_t n = (int64_t)nr * nc;
  const double* a = A + (int64_t)blockIdx.x * n;
  double m = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x)
    if (t % nc >= t / nc) m = fmax(m, fabs(a[t]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = acc ? fmax(out[blockIdx.x], red[0]) : red[0];
}

void row_absmax_upper(const double* A, int np, int nr, int nc, double* out, bool accumulate, hipStream_t s) {
  if (np == 0 || (int64_t)nr * nc == 0) return;
  k_row_absmax_upper<<<np, 256, 0, s>>>(A, nr, nc, out, accumulate ? 1 : 0);
  RISP_LAUNCHED();
}

// X[p][r][c] = X[p][c][r] for c < r < n (row stride ld, slice stride sp): the strict lower triangle
// of each slice from its upper triangle, through 32 x 32 tiles in LDS. Block (bx, by, p) writes the
// tile of rows by and columns bx (bx <= by) from the mirrored tile of rows bx and columns by.
template <typename T>
__global__ __launch_bounds__(256) void k_mirror_lower(T* __restrict__ X, int n, int64_t ld, int64_t sp) {
  const int bx = blockIdx.x, by = blockIdx.y;
  if (bx > by) return;
  T* S = X + (int64_t)blockIdx.z * sp;
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int row = bx * 32 + r, col = by * 32 + tx;
    if (row < n && col < n) tile[r][tx] = S[(int64_t)row * ld + col];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int row = by * 32 + r, col = bx * 32 + tx;
    if (row < n && col < row) S[(int64_t)row * ld + col] = tile[tx][r];
  }
}

void mirror_lower(void* X, int esz, int np, int n, int64_t ld, int64_t sp, hipStream_t s) {
  if (np <= 0 || n <= 1) return;
  RISP_CHECK(esz == 2 || esz == 4 || esz == 8, RISP_E_ARG, "mirror_lower: element size must be 2, 4 or 8 bytes");
  RISP_CHECK(ceil_div(n, 32) <= 65535, RISP_E_SHAPE, "mirror_lower: slices too large");
  for (int p0 = 0; p0 < np; p0 += 65535) {  // at most 65535 slices per launch (grid z)
    const dim3 grid(ceil_div(n, 32), ceil_div(n, 32), std::min(np - p0, 65535));
    char* Xp = static_cast<char*>(X) + (size_t)p0 * sp * esz;
    if (esz == 2) k_mirror_lower<uint16_t><<<grid, 256, 0, s>>>(reinterpret_cast<uint16_t*>(Xp), n, ld, sp);
    else if (esz == 4) k_mirror_lower<float><<<grid, 256, 0, s>>>(reinterpret_cast<float*>(Xp), n, ld, sp);
    else k_mirror_lower<double><<<grid, 256, 0, s>>>(reinterpret_cast<double*>(Xp), n, ld, sp);
    RISP_LAUNCHED();
  }
}

void row_absmax(const double* A, int rows, int64_t cols, int64_t lda, double* out, bool accumulate, hipStream_t s) {
  if (rows == 0) return;
  k_row_absmax<<<rows, 256, 0, s>>>(A, cols, lda, out, accumulate ? 1 : 0);
  RISP_LAUNCHED();
}

// scale[r] = smallest power of two >= mx[r] (1 for 0 or when disabled)
__global__ void k_pow2_from_max(const double* __restrict__ mx, int n, int enabled, float* __restrict__ scale) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double sc = 1.0;
  if (enabled && mx[r] > 0.0) {
    int e;
    const double f = frexp(mx[r], &e);  // mx = f 2^e, f in [0.5, 1)
    sc = ldexp(1.0, f == 0.5 ? e - 1 : e);
  }
  scale[r] = (float)sc;
}

void pow2_from_max(const double* mx, int n, bool enabled, float* scale, hipStream_t s) {
  if (n == 0) return;
  k_pow2_from_max<<<ceil_div(n, 256), 256, 0, s>>>(mx, n, enabled ? 1 : 0, scale);
  RISP_LAUNCHED();
}

template <typename TS, typename TD>
__global__ void k_store_block(const TS* __restrict__ src, int64_t lds, int64_t sps, TD* __restrict__ dst,
                              int64_t ldd, int64_t dps, int64_t nr, int64_t nc, int64_t total) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t % nc, r = (t / nc) % nr, p = t / (nc * nr);
    dst[(p * dps + r) * ldd + c] = cvt<TS, TD>(src[(p * sps + r) * lds + c]);
  }
}

void store_block(const void* src, DType ts, int64_t lds, int64_t sps, void* dst, DType td, int64_t ldd, int64_t dps,
                 int64_t np, int64_t nr, int64_t nc, hipStream_t s) {
  const int64_t total = np * nr * nc;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 18);
  if (ts == DType::F64 && td == DType::F64)
    k_store_block<double, double><<<grid, 256, 0, s>>>((const double*)src, lds, sps, (double*)dst, ldd, dps, nr, nc,
                                                       total);
  else if (ts == DType::F64 && td == DType::F32)
    k_store_block<double, float><<<grid, 256, 0, s>>>((const double*)src, lds, sps, (float*)dst, ldd, dps, nr, nc,
                                                      total);
  else
    throw Error(RISP_E_ARG, "store_block: unsupported type pair");
  RISP_LAUNCHED();
}

// out[c][r] = A[r][c] for r < rows, c < cols (FP64; A row stride lda, out row stride ldo), through
// 32 x 32 tiles in LDS so both the reads and the writes are coalesced
__global__ __launch_bounds__(256) void k_transpose64(const double* __restrict__ A, int64_t lda, int rows, int cols,
                                                     double* __restrict__ out, int64_t ldo) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = A[(int64_t)r * lda + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (c < cols && r < rows) out[(int64_t)c * ldo + r] = tile[tx][k];
  }
}

void transpose64(const double* A, int64_t lda, int rows, int cols, double* out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  RISP_CHECK(ceil_div(rows, 32) <= 65535, RISP_E_SHAPE, "transpose64: too many rows");
  k_transpose64<<<dim3(ceil_div(cols, 32), ceil_div(rows, 32)), 256, 0, s>>>(A, lda, rows, cols, out, ldo);
  RISP_LAUNCHED();
}

// FP64 block -> FP32 values kept as their upper and lower 16-bit halves in two arrays (the two BF16
// arrays of a split factor used as FP32 staging), same indexing as k_store_block
__global__ void k_store_block_split(const double* __restrict__ src, int64_t lds, int64_t sps, uint16_t* __restrict__ hi,
                                    uint16_t* __restrict__ lo, int64_t ldd, int64_t dps, int64_t nr, int64_t nc,
                                    int64_t total) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t % nc, r = (t / nc) % nr, p = t / (nc * nr);
    const uint32_t u = __float_as_uint(cvt<double, float>(src[(p * sps + r) * lds + c]));
    const int64_t d = (p * dps + r) * ldd + c;
    hi[d] = (uint16_t)(u >> 16);
    lo[d] = (uint16_t)(u & 0xFFFFu);
  }
}

void store_block_split(const double* src, int64_t lds, int64_t sps, void* hi, void* lo, int64_t ldd, int64_t dps,
                       int64_t np, int64_t nr, int64_t nc, hipStream_t s) {
  const int64_t total = np * nr * nc;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 18);
  k_store_block_split<<<grid, 256, 0, s>>>(src, lds, sps, static_cast<uint16_t*>(hi), static_cast<uint16_t*>(lo), ldd,
                                          dps, nr, nc, total);
  RISP_LAUNCHED();
}

// In place: the FP32 value staged as halves (hi, lo) becomes its scaled BF16 rounding in hi and the
// BF16 rounding of the remainder in lo, exactly as store_rows_padded + store_rows_padded_lo from an
// FP32 source (zeros stay zeros)
__global__ void k_split_to_bf16_pair(uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int64_t total, int64_t ldd,
                                     const float* __restrict__ scale, int64_t div, int64_t mod) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const float x = __uint_as_float(((uint32_t)hi[t] << 16) | (uint32_t)lo[t]);
    double v = (double)x;
    if (scale) v /= (double)scale[((t / ldd) / div) % mod];  // exact: powers of two
    const uint16_t h = cvt<double, uint16_t>(v);
    hi[t] = h;
    lo[t] = f2bf_rne((float)(v - (double)bf2f_(h)));
  }
}

void split_to_bf16_pair(void* hi, void* lo, int64_t rows, int64_t ldd, const float* scale, int64_t div, int64_t mod,
                        hipStream_t s) {
  const int64_t total = rows * ldd;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 18);
  k_split_to_bf16_pair<<<grid, 256, 0, s>>>(static_cast<uint16_t*>(hi), static_cast<uint16_t*>(lo), total, ldd, scale,
                                           div, mod);
  RISP_LAUNCHED();
}

template <typename TS, typename TD>
__global__ void k_store_padded(const TS* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                               TD* __restrict__ dst, int64_t ldd, const float* __restrict__ scale, int64_t div,
                               int64_t mod) {
  const int64_t total = rows * ldd;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / ldd, c = t % ldd;
    double v = 0.0;
    if (c < cols) {
      v = (double)src[r * lds + c];
      if (scale) v /= (double)scale[(r / div) % mod];  // exact: powers of two
    }
    dst[t] = cvt<double, TD>(v);
  }
}

void store_rows_padded(const void* src, DType ts, int64_t lds, int64_t rows, int64_t cols, void* dst, DType td,
                       int64_t ldd, const float* scale, int64_t div, int64_t mod, hipStream_t s) {
  const int64_t total = rows * ldd;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 18);
#define RISP_SP(TS_, TD_) \
  k_store_padded<TS_, TD_><<<grid, 256, 0, s>>>((const TS_*)src, lds, rows, cols, (TD_*)dst, ldd, scale, div, mod)
  if (ts == DType::F64 && td == DType::F64) RISP_SP(double, double);
  else if (ts == DType::F64 && td == DType::F32) RISP_SP(double, float);
  else if (ts == DType::F64 && td == DType::BF16) RISP_SP(double, uint16_t);
  else if (ts == DType::F32 && td == DType::BF16) RISP_SP(float, uint16_t);
  else if (ts == DType::F32 && td == DType::F32) RISP_SP(float, float);
  else throw Error(RISP_E_ARG, "store_rows_padded: unsupported type pair");
#undef RISP_SP
  RISP_LAUNCHED();
}

// BF16 remainder of a padded BF16 store: lo = bf16(v / scale - hi), where hi holds the rounded
// values written by store_rows_padded with the same layout and scales (zero in the padding)
template <typename TS>
__global__ void k_store_padded_lo(const TS* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                                  const uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int64_t ldd,
                                  const float* __restrict__ scale, int64_t div, int64_t mod) {
  const int64_t total = rows * ldd;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / ldd, c = t % ldd;
    double v = 0.0;
    if (c < cols) {
      v = (double)src[r * lds + c];
      if (scale) v /= (double)scale[(r / div) % mod];
    }
    lo[t] = f2bf_rne((float)(v - (double)bf2f_(hi[t])));
  }
}

void store_rows_padded_lo(const void* src, DType ts, int64_t lds, int64_t rows, int64_t cols, const void* hi,
                          void* lo, int64_t ldd, const float* scale, int64_t div, int64_t mod, hipStream_t s) {
  const int64_t total = rows * ldd;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 18);
  if (ts == DType::F64)
    k_store_padded_lo<double><<<grid, 256, 0, s>>>((const double*)src, lds, rows, cols, (const uint16_t*)hi,
                                                   (uint16_t*)lo, ldd, scale, div, mod);
  else if (ts == DType::F32)
    k_store_padded_lo<float><<<grid, 256, 0, s>>>((const float*)src, lds, rows, cols, (const uint16_t*)hi,
                                                  (uint16_t*)lo, ldd, scale, div, mod);
  else
    throw Error(RISP_E_ARG, "store_rows_padded_lo: FP64 or FP32 source");
  RISP_LAUNCHED();
}

__global__ void k_fill_zero16(uint4* p, int64_t n16) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n16; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = make_uint4(0, 0, 0, 0);
}
__global__ void k_fill_zero1(uint8_t* p, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = 0;
}

void fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  const int64_t n16 = (reinterpret_cast<uintptr_t>(p) % 16 == 0) ? (int64_t)(bytes / 16) : 0;
  if (n16 > 0) {
    k_fill_zero16<<<(unsigned)std::min<int64_t>(ceil_div(n16, 256), 1 << 16), 256, 0, s>>>((uint4*)p, n16);
    RISP_LAUNCHED();
  }
  const int64_t rest = (int64_t)bytes - n16 * 16;
  if (rest > 0) {
    k_fill_zero1<<<(unsigned)std::min<int64_t>(ceil_div(rest, 256), 1 << 16), 256, 0, s>>>((uint8_t*)p + n16 * 16,
                                                                                           rest);
    RISP_LAUNCHED();
  }
}

template <typename T>
__global__ void k_permute(const T* __restrict__ a, T* __restrict__ b, int nP, int ni, int nj) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nP * ni * nj;
  if (t >= total) return;
  // t indexes the output [i][P][j]
  const int j = (int)(t % nj);
  const int P = (int)((t / nj) % nP);
  const int i = (int)(t / ((int64_t)nj * nP));
  b[t] = a[((int64_t)P * ni + i) * nj + j];
}

void permute_pij_ipj(const void* T, int nP, int ni, int nj, size_t esz, void* out, hipStream_t s) {
  const int64_t total = (int64_t)nP * ni * nj;
  if (total == 0) return;
  const unsigned grid = ceil_div(total, 256);
  if (esz == 8) k_permute<double><<<grid, 256, 0, s>>>((const double*)T, (double*)out, nP, ni, nj);
  else if (esz == 4) k_permute<float><<<grid, 256, 0, s>>>((const float*)T, (float*)out, nP, ni, nj);
  else k_permute<uint16_t><<<grid, 256, 0, s>>>((const uint16_t*)T, (uint16_t*)out, nP, ni, nj);
  RISP_LAUNCHED();
}

__global__ void k_gaps(const double* __restrict__ e, int nocc, int nvir, double* de64, float* de32) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nocc * nvir) return;
  const int i = (int)(t / nvir), a = (int)(t % nvir);
  const double d = e[nocc + a] - e[i];
  de64[t] = d;
  de32[t] = (float)d;
}

void orbital_gaps(const double* e, int nocc, int nvir, double* de64, float* de32, hipStream_t s) {
  k_gaps<<<ceil_div((int64_t)nocc * nvir, 256), 256, 0, s>>>(e, nocc, nvir, de64, de32);
  RISP_LAUNCHED();
}

// out[c] += alpha sum_r T[r][c]^2 (threads over columns, rows in a loop: coalesced rows)
__global__ void k_col_sumsq(const double* __restrict__ T, int rows, int64_t cols, int64_t ld, double alpha,
                            double* __restrict__ out) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < rows; ++r) {
      const double v = T[(int64_t)r * ld + c];
      acc += v * v;
    }
    out[c] += alpha * acc;
  }
}

void col_sumsq(const double* T, int rows, int64_t cols, int64_t ld, double alpha, double* out, hipStream_t s) {
  if (cols <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(cols, 256), 1 << 16);
  k_col_sumsq<<<grid, 256, 0, s>>>(T, rows, cols, ld, alpha, out);
  RISP_LAUNCHED();
}

__global__ void k_gather_strided(const double* __restrict__ src, int np, int nt, int64_t sp, int64_t st,
                                 double* __restrict__ out, int64_t ldo) {
  const int64_t n = (int64_t)np * nt;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = x / nt, t = x % nt;
    out[p * ldo + t] = src[p * sp + t * st];
  }
}

void gather_strided(const double* src, int np, int nt, int64_t sp, int64_t st, double* out, int64_t ldo,
                    hipStream_t s) {
  if ((int64_t)np * nt <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div((int64_t)np * nt, 256), 1 << 16);
  k_gather_strided<<<grid, 256, 0, s>>>(src, np, nt, sp, st, out, ldo);
  RISP_LAUNCHED();
}

__global__ void k_scatter_sub_window(const double* __restrict__ K, int nok, int nvk, const int* __restrict__ occ,
                                     const int* __restrict__ vir, int nvir, double* __restrict__ diag) {
  const int64_t n = (int64_t)nok * nvk;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(x / nvk), a = (int)(x % nvk);
    diag[(int64_t)occ[i] * nvir + vir[a]] -= K[x];
  }
}

void scatter_sub_window(const double* K, int nok, int nvk, const int* occ, const int* vir, int nvir, double* diag,
                        hipStream_t s) {
  if ((int64_t)nok * nvk <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div((int64_t)nok * nvk, 256), 1 << 16);
  k_scatter_sub_window<<<grid, 256, 0, s>>>(K, nok, nvk, occ, vir, nvir, diag);
  RISP_LAUNCHED();
}

__global__ void k_add_inplace(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    y[t] += x[t];
}

void add_inplace(double* y, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 1 << 16);
  k_add_inplace<<<grid, 256, 0, s>>>(y, x, n);
  RISP_LAUNCHED();
}

__global__ void k_fill_neg(int* p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = -1;
}
__global__ void k_positions(const int* idx, int n, int* pos) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) pos[idx[t]] = t;
}

void window_positions(const int* idx, int n, int len, int* pos, hipStream_t s) {
  if (len > 0) {
    k_fill_neg<<<ceil_div(len, 256), 256, 0, s>>>(pos, len);
    RISP_LAUNCHED();
  }
  if (n > 0) {
    k_positions<<<ceil_div(n, 256), 256, 0, s>>>(idx, n, pos);
    RISP_LAUNCHED();
  }
}

template <typename TS, typename TD>
__global__ void k_gather_window(const TS* __restrict__ X, int m, int nocc, int nvir,
                                const int* __restrict__ occ, int nok, const int* __restrict__ vir,
                                int nvk, TD* __restrict__ Xw, int nokp, int nvkp) {
  const int64_t total = (int64_t)m * nokp * nvkp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t % nvkp);
    const int j = (int)((t / nvkp) % nokp);
    const int mm = (int)(t / ((int64_t)nvkp * nokp));
    Xw[t] = (j < nok && b < nvk) ? cvt<TS, TD>(X[((int64_t)mm * nocc + occ[j]) * nvir + vir[b]]) : cvt<double, TD>(0.0);
  }
}

// window block of FP32 X split into BF16 parts: hi = bf16(x), lo = bf16(x - hi), zero padding
__global__ void k_gather_window_split(const float* __restrict__ X, int m, int nocc, int nvir,
                                      const int* __restrict__ occ, int nok, const int* __restrict__ vir, int nvk,
                                      uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int nokp, int nvkp) {
  const int64_t total = (int64_t)m * nokp * nvkp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t % nvkp);
    const int j = (int)((t / nvkp) % nokp);
    const int mm = (int)(t / ((int64_t)nvkp * nokp));
    const float x = (j < nok && b < nvk) ? X[((int64_t)mm * nocc + occ[j]) * nvir + vir[b]] : 0.0f;
    const uint16_t h = f2bf_rne(x);
    hi[t] = h;
    lo[t] = f2bf_rne(x - bf2f_(h));
  }
}

void gather_window_split(const float* X, int m, int nocc, int nvir, const int* occ, int nok, const int* vir, int nvk,
                         void* hi, void* lo, int nokp, int nvkp, hipStream_t s) {
  const int64_t total = (int64_t)m * nokp * nvkp;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 16);
  k_gather_window_split<<<grid, 256, 0, s>>>(X, m, nocc, nvir, occ, nok, vir, nvk, (uint16_t*)hi, (uint16_t*)lo, nokp,
                                             nvkp);
  RISP_LAUNCHED();
}

void gather_window(const void* X, DType ts, int m, int nocc, int nvir, const int* occ, int nok,
                   const int* vir, int nvk, void* Xw, DType td, int nokp, int nvkp, hipStream_t s) {
  const int64_t total = (int64_t)m * nokp * nvkp;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 16);
  if (ts == DType::F64 && td == DType::F64)
    k_gather_window<double, double><<<grid, 256, 0, s>>>((const double*)X, m, nocc, nvir, occ, nok, vir, nvk, (double*)Xw, nokp, nvkp);
  else if (ts == DType::F32 && td == DType::F32)
    k_gather_window<float, float><<<grid, 256, 0, s>>>((const float*)X, m, nocc, nvir, occ, nok, vir, nvk, (float*)Xw, nokp, nvkp);
  else if (ts == DType::F32 && td == DType::BF16)
    k_gather_window<float, uint16_t><<<grid, 256, 0, s>>>((const float*)X, m, nocc, nvir, occ, nok, vir, nvk, (uint16_t*)Xw, nokp, nvkp);
  else
    throw Error(RISP_E_ARG, "gather_window: unsupported type pair");
  RISP_LAUNCHED();
}

template <typename T, typename TK, typename TD>
__global__ void k_combine(T* __restrict__ sig, const T* __restrict__ X, const TD* __restrict__ de,
                          int m, int nocc, int nvir, const TK* __restrict__ K,
                          const int* __restrict__ po, const int* __restrict__ pv, int nok, int nvk) {
  const int64_t ov = (int64_t)nocc * nvir;
  const int64_t total = (int64_t)m * ov;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ia = t % ov;
    const int mm = (int)(t / ov);
    const int i = (int)(ia / nvir), a = (int)(ia % nvir);
    T v = sig[t] + (T)de[ia] * X[t];
    if (K) {
      const int ik = po[i], ak = pv[a];
      if (ik >= 0 && ak >= 0) v -= (T)K[((int64_t)mm * nok + ik) * nvk + ak];
    }
    sig[t] = v;
  }
}

void combine_sigma(void* sigma, const void* X, DType t, const double* de64, const float* de32, int m,
                   int nocc, int nvir, const void* K, DType tk, const int* pos_o, const int* pos_v,
                   int nok, int nvk, hipStream_t s) {
  const int64_t total = (int64_t)m * nocc * nvir;
  if (total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 16);
  if (t == DType::F64) {
    RISP_CHECK(tk == DType::F64, RISP_E_ARG, "combine: FP64 sigma needs FP64 exchange");
    k_combine<double, double, double><<<grid, 256, 0, s>>>((double*)sigma, (const double*)X, de64, m, nocc,
                                                           nvir, (const double*)K, pos_o, pos_v, nok, nvk);
  } else {
    RISP_CHECK(tk == DType::F32, RISP_E_ARG, "combine: FP32 sigma needs FP32 exchange");
    k_combine<float, float, float><<<grid, 256, 0, s>>>((float*)sigma, (const float*)X, de32, m, nocc, nvir,
                                                        (const float*)K, pos_o, pos_v, nok, nvk);
  }
  RISP_LAUNCHED();
}

}  // namespace risp
