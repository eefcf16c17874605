// Batched MFMA matrix products for gfx950: C = alpha * s_b * r_i * (A . B^T) + beta * C.
//
// A is M x K and B is N x K (the contraction index k is shared). Each operand is stored either
// k-contiguous (A[i][k] at A + i*lda + k) or mn-contiguous (A[i][k] at A + k*lda + i); C is
// row-major M x N. Batches are two-level, b = b1 * nb2 + b2, with separate strides for each level.
// Products are FP64 (v_mfma_f64_16x16x4f64; operands stored as FP64 or FP32), FP32
// (v_mfma_f32_16x16x4f32) or BF16 (v_mfma_f32_16x16x32_bf16); accumulation is FP64 for FP64
// products and FP32 otherwise. Optional
// factors: r_i (row_scale[i], FP32) and s_b (batch_scale[b2], FP32). Split-K writes partial sums to
// a workspace and reduces them in a fixed order, so results do not depend on scheduling.
#pragma once

#include "common.hpp"

namespace risp {

// Same: the operand is stored in the product type.
enum class DType : int { F64 = 0, F32 = 1, BF16 = 2, Same = 3 };

inline size_t dtype_size(DType t) { return t == DType::F64 ? 8 : (t == DType::F32 ? 4 : 2); }

struct Gemm {
  int M = 0, N = 0, K = 0;
  DType tin = DType::F32;  // type the products are formed in
  DType tout = DType::F32; // type of C
  // storage of A and B when it differs from tin (FP64 products of FP32 data, subspace algebra)
  DType mem_a = DType::Same, mem_b = DType::Same;
  const void* A = nullptr;
  int64_t lda = 0;
  bool a_kc = true;
  const void* B = nullptr;
  int64_t ldb = 0;
  bool b_kc = true;
  void* C = nullptr;
  int64_t ldc = 0;
  int nb1 = 1, nb2 = 1;
  int64_t sa1 = 0, sa2 = 0, sb1 = 0, sb2 = 0, sc1 = 0, sc2 = 0;
  double alpha = 1.0, beta = 0.0;
  const float* row_scale = nullptr;
  const float* batch_scale = nullptr;
  int ksplit = 1;  // > 1 splits K over blocks (uses workspace)
  // A or B is lower triangular (A[i][k] = 0 for k > i, B[j][k] = 0 for k > j): a kernel may skip
  // those k (the FP64 NT kernel does; the sums keep their order, only exact zero terms are left out)
  bool a_lower = false, b_lower = false;
  // column split of C: when n_inner > 0, column n is stored at (n / n_inner) * sc_outer + n % n_inner
  // within its row (lets one product write an interleaved [outer][row][inner] layout)
  int n_inner = 0;
  int64_t sc_outer = 0;
  // BF16 products only: npair (1..3) operand pairs (A, B), (A2, B2), (A3, B3) with the same strides
  // concatenated along K, i.e. C = A B^T + A2 B2^T + A3 B3^T in one accumulation; and, for BF16 C,
  // an optional second output C_lo that receives the rounding remainder of each element
  // (C = bf16(v), C_lo = bf16(v - C), beta must be 0)
  int npair = 1;
  const void* A2 = nullptr;
  const void* B2 = nullptr;
  const void* A3 = nullptr;
  const void* B3 = nullptr;
  void* C_lo = nullptr;
};

// Launch on stream s. `work` must hold ksplit * nb1 * nb2 * M * N accumulator elements when
// ksplit > 1 (gemm_workspace_bytes).
size_t gemm_workspace_bytes(const Gemm& g);
void gemm(const Gemm& g, void* work, hipStream_t s);

// Tuned kernel for contraction-contiguous operands (used by gemm() when eligible: BF16 products
// with F32/BF16 output, FP32 products of FP32 data, FP64 products of FP64 data with FP64/FP32
// output; 16-byte aligned operands, strides and K multiples of 16 bytes).
bool gemm_bf16_nt_eligible(const Gemm& g);
int gemm_bf16_nt_tile(const Gemm& g);  // rows of the output tile it would use (128, 192, 256)
void gemm_bf16_nt(const Gemm& g, void* work, hipStream_t s);
void gemm_f64_nt(const Gemm& g, void* work, hipStream_t s);  // FP64 operands (gemm_bf16_nt forwards them)

// One product of a grouped FP64 launch: (C + c_off)[r][col(c)] = alpha (A + a_off)[r][:] . (B + b_off)[c][:]
// (+ beta C) over K values, with both operands at row stride ld (a multiple of 2, offsets even) and
// N output columns split by n_inner as in Gemm (n_inner <= 0: no split).
struct GemmGroup {
  int64_t a_off = 0, b_off = 0, c_off = 0;  // element offsets from the launch's A, B and C
  int K = 0, ld = 0, N = 0, n_inner = 0;
};
// Runs ngroups FP64 products of M rows in one launch (A, B, C, M, ldc, sc_outer, alpha, beta from g;
// FP64 output, no batches, no split-K). tile0 [ngroups + 1] (device) numbers the 128 x 256 output
// tiles: product k owns tiles [tile0[k], tile0[k + 1]) with at least ceil(M / 128) * ceil(N_k / 256)
// of them, row tile fastest; total_tiles = tile0[ngroups].
void gemm_f64_grouped(const Gemm& g, const GemmGroup* groups, const int* tile0, int ngroups, int total_tiles,
                      hipStream_t s);

// Choose a split-K factor so that the grid covers the chip for products with few output tiles;
// returns 1 when tiles alone suffice.
int gemm_auto_split(const Gemm& g);

}  // namespace risp
