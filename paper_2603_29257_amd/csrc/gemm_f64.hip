// FP64 products with both operands stored contraction-contiguous (C = A . B^T): the MO transforms and
// metric products of the factor build, and the grouped per-atom first transforms. Same loader, LDS
// stages, XCD renumbering and tile order as the BF16 / FP32 kernels (gemm_bf16.hip).
#include "gemm.hpp"
#include "gemm_tile.hpp"

namespace risp {

namespace {

using namespace tile;

// FP64 products (factor build): the same loader, LDS stages and XCD renumbering with a 128 x 256
// tile; each wave owns a 64 x 64 sub-tile of 4 x 4 v_mfma_f64_16x16x4_f64 accumulators. A 128-byte
// slice holds 16 k values; lane group q = lane / 16 reads chunk 4 s + q (two k values) in step
// s = 0, 1 and feeds them to two consecutive MFMAs, so the k values of one MFMA are 8 s + 2 q + e
// for e = 0, 1 (a permutation of the slice, the same for A and B).
typedef double d4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int uni32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// GROUPED: one launch runs many independent products that share M, the output row stride and the
// column-split stride (gemm_f64_grouped); block L belongs to the product g with
// tile0[g] <= L < tile0[g + 1], whose tiles are numbered row tile fastest.
template <typename TO, bool GROUPED>
__global__ __launch_bounds__(NT, 1) void k_gemm_nt64(Gemm g, int tiles_m, int tiles_n, double* __restrict__ work,
                                                     const GemmGroup* __restrict__ groups,
                                                     const int* __restrict__ tile0, int ngroups) {
  constexpr int ES = 8, BK = ROWB / ES, EPC = 2;
  constexpr int BM = 128, ROWS = BM + BN, NLD = ROWS / RSTEP, STAGE = ROWS * ROWB;
  constexpr int FM = BM / 2 / 16, FN = WN / 16;
  __shared__ __attribute__((aligned(16))) char lds[2 * STAGE];

  // runs of 32 consecutive tiles (one XCD's resident blocks) dealt to the XCDs in turn: hardware
  // block w runs on XCD w % 8 as its (w / 8)-th block; a last partial round keeps the hardware order
  // (1000-atom build: 13.58 -> 13.14 s against one contiguous range of tiles per XCD)
  constexpr int SEG = 32;
  const int W = gridDim.x, w = blockIdx.x;
  const int full = W / (8 * SEG) * (8 * SEG);
  int L = w;
  if (w < full) {
    const int x = w % 8, qb8 = w / 8;
    L = ((qb8 / SEG) * 8 + x) * SEG + qb8 % SEG;
  }
  int tm, tn, split = 0, b2 = 0, K, N, n_inner = g.n_inner;
  int64_t lda, ldb, zoff = 0;
  const double* A;
  const double* B;
  TO* Cb;
  if constexpr (GROUPED) {
    int lo = 0, hi = ngroups;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (uni32(tile0[mid]) <= L) lo = mid;
      else hi = mid;
    }
    const GemmGroup& gd = groups[lo];
    const int t = L - uni32(tile0[lo]);
    tm = t % tiles_m;
    tn = t / tiles_m;
    K = uni32(gd.K);
    N = uni32(gd.N);
    n_inner = uni32(gd.n_inner);
    lda = ldb = uni32(gd.ld);
    A = static_cast<const double*>(g.A) + uni64(gd.a_off);
    B = static_cast<const double*>(g.B) + uni64(gd.b_off);
    Cb = static_cast<TO*>(g.C) + uni64(gd.c_off);
  } else {
    const int tiles = tiles_m * tiles_n;
    const int zb = L / tiles, t = L % tiles;
    grouped_tile(t, tiles_m, tiles_n, tm, tn);
    // lower-triangular A (B): row (column) tile t costs ~t slices, and each XCD runs a contiguous
    // range of tiles; alternating light and heavy tiles (0, last, 1, last - 1, ...) evens them out
    if (g.a_lower) tm = (tm & 1) ? tiles_m - 1 - (tm >> 1) : (tm >> 1);
    if (g.b_lower) tn = (tn & 1) ? tiles_n - 1 - (tn >> 1) : (tn >> 1);
    split = zb % g.ksplit;
    const int b = zb / g.ksplit;
    const int b1 = b / g.nb2;
    b2 = b % g.nb2;
    zoff = b;
    K = g.K;
    N = g.N;
    lda = g.lda;
    ldb = g.ldb;
    A = static_cast<const double*>(g.A) + b1 * g.sa1 + b2 * g.sa2;
    B = static_cast<const double*>(g.B) + b1 * g.sb1 + b2 * g.sb2;
    Cb = static_cast<TO*>(g.C) + b1 * g.sc1 + b2 * g.sc2;
  }
  const int m0 = tm * BM, n0 = tn * BN;
  int kbeg = 0, kend = K;
  if (!GROUPED && g.ksplit > 1) {
    const int kchunk = ((K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    kbeg = split * kchunk;
    kend = min(K, kbeg + kchunk);
  }
  // lower-triangular A (B): the tile's rows (columns) end at m0 + BM (n0 + BN), so no later k
  // contributes
  if (!GROUPED && g.a_lower) kend = min(kend, m0 + BM);
  if (!GROUPED && g.b_lower) kend = min(kend, n0 + BN);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int r_t = tid >> 3, c_t = tid & 7;
  const int st_off = r_t * ROWB + 16 * (c_t ^ ((r_t >> 1) & 7));
  const int rows_a = max(0, min(BM, g.M - m0)), rows_b = max(0, min(BN, N - n0));
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + (int64_t)m0 * lda, (int)((int64_t)rows_a * lda * ES));
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(B + (int64_t)n0 * ldb, (int)((int64_t)rows_b * ldb * ES));
  const uint32_t va = (uint32_t)((r_t * lda + EPC * c_t) * ES), vb = (uint32_t)((r_t * ldb + EPC * c_t) * ES);
  const uint32_t qa = (uint32_t)(RSTEP * lda * ES), qbs = (uint32_t)(RSTEP * ldb * ES);

  uint4 reg[NLD];
  auto gload = [&](int kt) {
    const int k0 = kbeg + kt * BK;
    const bool kin = k0 + EPC * c_t < kend;
#pragma unroll
    for (int qq = 0; qq < NLD; ++qq) {
      const bool isA = qq < BM / RSTEP;
      const uint32_t off = isA ? va + qq * qa + ES * k0 : vb + (qq - BM / RSTEP) * qbs + ES * k0;
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(isA ? ra : rb, kin ? off : 0x80000000u, 0, 0);
      __builtin_memcpy(&reg[qq], &v, 16);
    }
  };
  auto sstore = [&](int stage) {
    char* base = lds + stage * STAGE + st_off;
#pragma unroll
    for (int qq = 0; qq < NLD; ++qq) *reinterpret_cast<uint4*>(base + qq * RSTEP * ROWB) = reg[qq];
  };

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * WN;
  const int l16 = lane & 15, q = lane >> 4, swz = (l16 >> 1) & 7;
  const int a_off = (wm + l16) * ROWB, b_off = (BM + wn + l16) * ROWB;

  d4v acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

  if (nk > 0) {
    gload(0);
    sstore(0);
    if (nk > 1) gload(1);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const char* buf = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int chunk = 16 * ((4 * st + q) ^ swz);
      double2 a[FM], bb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const double2*>(buf + a_off + i * 16 * ROWB + chunk);
#pragma unroll
      for (int j = 0; j < FN; ++j) bb[j] = *reinterpret_cast<const double2*>(buf + b_off + j * 16 * ROWB + chunk);
      // all first-k MFMAs, then all second-k ones: consecutive MFMAs use different accumulators
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, bb[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, bb[j].y, acc[i][j], 0, 0, 0);
      if (st == 0) {
        if (kt + 1 < nk) sstore((kt + 1) & 1);
        if (kt + 2 < nk) gload(kt + 2);
      }
    }
    __syncthreads();
  }

  // accumulator element r of lane l: row l / 16 + 4 r, column l % 16 of its 16 x 16 fragment
  if (!GROUPED && g.ksplit > 1) {
    double* Wp = work + (zoff * g.ksplit + split) * g.M * N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + q + 4 * r;
        if (row >= g.M) continue;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = n0 + wn + j * 16 + l16;
          if (col < N) Wp[(int64_t)row * N + col] = acc[i][j][r];
        }
      }
    return;
  }
  TO* C = Cb;
  const double bs = g.alpha * (g.batch_scale ? (double)g.batch_scale[b2] : 1.0);
  int64_t coff[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int col = n0 + wn + j * 16 + l16;
    coff[j] = col >= N ? -1 : (n_inner <= 0 ? col : (int64_t)(col / n_inner) * g.sc_outer + col % n_inner);
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm + i * 16 + q + 4 * r;
      if (row >= g.M) continue;
      const double rs = g.row_scale ? bs * (double)g.row_scale[row] : bs;
      TO* crow = C + (int64_t)row * g.ldc;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if (coff[j] < 0) continue;
        TO* cp = crow + coff[j];
        double v = rs * acc[i][j][r];
        if (g.beta != 0.0) v += g.beta * (double)*cp;
        *cp = (TO)v;
      }
    }
}

}  // namespace

void gemm_f64_nt(const Gemm& g, void* work, hipStream_t s) {
  const int tm = (g.M + 127) / 128, tn = (g.N + BN - 1) / BN;
  const int64_t blocks = (int64_t)tm * tn * g.nb1 * g.nb2 * g.ksplit;
  RISP_CHECK(blocks < (1ll << 31), RISP_E_SHAPE, "gemm grid too large");
  double* w = static_cast<double*>(work);
  if (g.tout == DType::F64)
    k_gemm_nt64<double, false><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w, nullptr, nullptr, 0);
  else k_gemm_nt64<float, false><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w, nullptr, nullptr, 0);
  RISP_LAUNCHED();
}

void gemm_f64_grouped(const Gemm& g, const GemmGroup* groups, const int* tile0, int ngroups, int total_tiles,
                      hipStream_t s) {
  RISP_CHECK(g.tin == DType::F64 && (g.mem_a == DType::Same || g.mem_a == DType::F64) &&
                 (g.mem_b == DType::Same || g.mem_b == DType::F64) && g.tout == DType::F64 && g.ksplit <= 1 &&
                 g.nb1 == 1 && g.nb2 == 1 && g.a_kc && g.b_kc && !g.row_scale && !g.batch_scale,
             RISP_E_ARG, "gemm_f64_grouped: FP64 contraction-contiguous products without batches or split-K");
  RISP_CHECK(reinterpret_cast<uintptr_t>(g.A) % 16 == 0 && reinterpret_cast<uintptr_t>(g.B) % 16 == 0,
             RISP_E_ARG, "gemm_f64_grouped: operand bases must be 16-byte aligned");
  if (total_tiles <= 0 || ngroups <= 0 || g.M <= 0) return;
  const int tm = (g.M + 127) / 128;
  k_gemm_nt64<double, true><<<(unsigned)total_tiles, NT, 0, s>>>(g, tm, 0, nullptr, groups, tile0, ngroups);
  RISP_LAUNCHED();
}

}  // namespace risp
