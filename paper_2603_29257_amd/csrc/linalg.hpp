// FP64 dense linear algebra on the device for the auxiliary metric, and small data-movement kernels.
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace risp {

// In-place lower Cholesky factor of the SPD matrix A [n][n] (row-major): A = L L^T; the upper
// triangle is zeroed. Throws RISP_E_ARG if a pivot is not positive.
void cholesky(double* A, int n, hipStream_t s);

// X = L^-1 for lower-triangular L [n][n]; X is lower triangular.
void tri_inverse(const double* L, double* X, int n, hipStream_t s);

// out[r][mu] = C[mu][cols[r]] for r < nr (cols may be null: cols[r] = col0 + r); C is [nao][ldc].
void gather_transpose(const double* C, int64_t ldc, int nao, const int* cols, int col0, int nr,
                      double* out, hipStream_t s);

// dst[i] = (type) src[i] (FP64/FP32 -> FP64/FP32/BF16), n elements.
void convert(const void* src, DType ts, void* dst, DType td, int64_t n, hipStream_t s);

// zero `bytes` bytes with a kernel (safe inside graph capture, unlike a memset node)
void fill_zero(void* p, size_t bytes, hipStream_t s);

// scale[r] = 2^ceil(log2 max_c |A[r][c]|) (1 for a zero row) of an FP64 matrix [rows][cols]
void row_pow2_scales(const double* A, int rows, int64_t cols, float* scale, hipStream_t s);

// dst[r][c] = (td)(src[r][c] / scale[(r / div) % mod]) for c < cols and 0 for cols <= c < ldd;
// src is FP64 or FP32 [rows][lds]; scale may be null (no scaling).
void store_rows_padded(const void* src, DType ts, int64_t lds, int64_t rows, int64_t cols, void* dst, DType td,
                       int64_t ldd, const float* scale, int64_t div, int64_t mod, hipStream_t s);

inline int64_t pad8(int64_t n) { return (n + 7) / 8 * 8; }

// out[r] = max_c |A[r * lda + c]| over c < cols (max with the previous out[r] when accumulate)
void row_absmax(const double* A, int rows, int64_t cols, int64_t lda, double* out, bool accumulate, hipStream_t s);
// out[p] = max(out[p] (if accumulate), max |A[p][i][j]| over j >= i) for A [np][nr][nc]
void row_absmax_upper(const double* A, int np, int nr, int nc, double* out, bool accumulate, hipStream_t s);
// X[p][r][c] = X[p][c][r] for c < r < n in each of np slices (element size esz = 2, 4 or 8 bytes,
// row stride ld, slice stride sp elements)
void mirror_lower(void* X, int esz, int np, int n, int64_t ld, int64_t sp, hipStream_t s);

// scale[r] = smallest power of two >= mx[r] (1 where mx[r] = 0, or everywhere when not enabled)
void pow2_from_max(const double* mx, int n, bool enabled, float* scale, hipStream_t s);

// dst[(p * dps + r) * ldd + c] = (td) src[(p * sps + r) * lds + c] for p < np, r < nr, c < nc (FP64
// source; FP64 or FP32 destination); nothing outside those positions is written
void store_block(const void* src, DType ts, int64_t lds, int64_t sps, void* dst, DType td, int64_t ldd, int64_t dps,
                 int64_t np, int64_t nr, int64_t nc, hipStream_t s);

// out[c][r] = A[r][c] (FP64), rows x cols, row strides lda and ldo
void transpose64(const double* A, int64_t lda, int rows, int cols, double* out, int64_t ldo, hipStream_t s);

// store_block of an FP64 source into FP32 values kept as upper / lower 16-bit halves in hi and lo
void store_block_split(const double* src, int64_t lds, int64_t sps, void* hi, void* lo, int64_t ldd, int64_t dps,
                       int64_t np, int64_t nr, int64_t nc, hipStream_t s);
// in place: staged halves -> BF16 rows scaled by scale[(row / div) % mod] in hi, the remainder in lo
void split_to_bf16_pair(void* hi, void* lo, int64_t rows, int64_t ldd, const float* scale, int64_t div, int64_t mod,
                        hipStream_t s);

// T [P][i][j] -> out [i][P][j]  (element size esz bytes)
void permute_pij_ipj(const void* T, int nP, int ni, int nj, size_t esz, void* out, hipStream_t s);

// de[i][a] = e[nocc + a] - e[i] (FP64 and FP32 copies)
void orbital_gaps(const double* e, int nocc, int nvir, double* de64, float* de32, hipStream_t s);

// pieces of the diagonal of A: out[c] += alpha sum_r T[r][c]^2 over rows of stride ld;
// out[p][t] (row stride ldo) = src[p sp + t st]; diag[occ[i] nvir + vir[a]] -= K[i][a]; y += x
void col_sumsq(const double* T, int rows, int64_t cols, int64_t ld, double alpha, double* out, hipStream_t s);
void gather_strided(const double* src, int np, int nt, int64_t sp, int64_t st, double* out, int64_t ldo,
                    hipStream_t s);
void scatter_sub_window(const double* K, int nok, int nvk, const int* occ, const int* vir, int nvir, double* diag,
                        hipStream_t s);
void add_inplace(double* y, const double* x, int64_t n, hipStream_t s);

// window position maps: pos[k] = index of k in idx[0..n) or -1 (length len)
void window_positions(const int* idx, int n, int len, int* pos, hipStream_t s);

// Xw[m][j][b] = X[m][occ[j]][vir[b]] with conversion from ts to td for j < nok, b < nvk; Xw is
// [m][nokp][nvkp] and its padding (j >= nok or b >= nvk) is written with zeros
// BF16 remainder lo = bf16(v / scale - hi) of a store_rows_padded BF16 store hi (same layout)
void store_rows_padded_lo(const void* src, DType ts, int64_t lds, int64_t rows, int64_t cols, const void* hi,
                          void* lo, int64_t ldd, const float* scale, int64_t div, int64_t mod, hipStream_t s);
// window block of FP32 X as two BF16 parts, hi = bf16(x), lo = bf16(x - hi), layout as gather_window
void gather_window_split(const float* X, int m, int nocc, int nvir, const int* occ, int nok, const int* vir, int nvk,
                         void* hi, void* lo, int nokp, int nvkp, hipStream_t s);
void gather_window(const void* X, DType ts, int m, int nocc, int nvir, const int* occ, int nok,
                   const int* vir, int nvk, void* Xw, DType td, int nokp, int nvkp, hipStream_t s);

// sigma[m][i][a] += de[i][a] X[m][i][a] - (i, a in window ? K[m][pos_o[i]][pos_v[a]] : 0)
void combine_sigma(void* sigma, const void* X, DType t, const double* de64, const float* de32, int m,
                   int nocc, int nvir, const void* K, DType tk, const int* pos_o, const int* pos_v,
                   int nok, int nvk, hipStream_t s);

}  // namespace risp
