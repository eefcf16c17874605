// Products with both operands stored contraction-contiguous (C = A . B^T), BF16 or FP32 operands:
// the exchange products of sigma and the plain FP32 path (FP64 operands: gemm_f64.hip).
//
// One 512-thread block (8 wave64s in a 2 x 4 grid, two per SIMD) computes a BM x 256 tile,
// BM = 64 * TI (128, 192 or 256); each wave owns a (BM/2) x 64 sub-tile of TI x 2 32x32 MFMA
// accumulators. K advances in slices of 128 bytes per row (64 BF16 or 32 FP32 values) through two
// LDS stages: while the MFMAs consume one stage, the next slice (already in registers) is written
// to the other stage halfway through the slice's MFMAs and the slice after it is then requested
// from memory, so one barrier per slice suffices; with two waves per SIMD, one wave's memory phase
// overlaps the other's MFMAs. LDS rows
// are 128 bytes with the 16-byte chunks XOR-swizzled by (row / 2) mod 8, which makes both the
// 16-byte fragment reads and the row-slice writes conflict-free without padding. Blocks are
// renumbered so that runs of 32 consecutive tiles land on one XCD (the dispatcher deals workgroups
// round-robin over the 8 XCDs) and ordered in groups of row tiles, which lets neighbouring tiles
// share operand panels in that XCD's L2.
//
// BF16: v_mfma_f32_32x32x16_bf16, a lane's 16-byte chunk is its 8 consecutive k. FP32:
// v_mfma_f32_32x32x2_f32 takes one k per lane and half-wave; the contraction order is permuted
// (step s of a chunk pair uses k = 8q + 4h + s for half-wave h), so a lane's 16-byte chunk again
// holds the k values of four consecutive MFMAs. The sum over k does not depend on its order.
#include "gemm.hpp"
#include "gemm_tile.hpp"

namespace risp {

namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

using namespace tile;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <typename TO> __device__ __forceinline__ void store_out(TO* p, float v);
template <> __device__ __forceinline__ void store_out<float>(float* p, float v) { *p = v; }
template <> __device__ __forceinline__ void store_out<uint16_t>(uint16_t* p, float v) { *p = f2bf(v); }
template <typename TO> __device__ __forceinline__ float load_out(const TO* p);
template <> __device__ __forceinline__ float load_out<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float load_out<uint16_t>(const uint16_t* p) { return bf2f(*p); }

// element offset of output column `col` (column split: col -> (col / n_inner, col % n_inner))
__device__ __forceinline__ int64_t col_offset(const Gemm& g, int col) {
  if (g.n_inner <= 0) return col;
  return (int64_t)(col / g.n_inner) * g.sc_outer + col % g.n_inner;
}


// one 16-byte chunk of A and of B: the MFMAs of that chunk's k values
template <typename TE> __device__ __forceinline__ f16v mfma_chunk(uint4 a, uint4 b, f16v c);
template <> __device__ __forceinline__ f16v mfma_chunk<uint16_t>(uint4 a, uint4 b, f16v c) {
  bf8v av, bv;
  __builtin_memcpy(&av, &a, 16);
  __builtin_memcpy(&bv, &b, 16);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
}

__device__ __forceinline__ float chunk_elt(uint4 v, int e) {
  return __uint_as_float(e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w)));
}

// NPAIR > 1: up to NPAIR operand pairs concatenated along K (g.npair of them) and the optional split
// BF16 output; NPAIR = 1 is the plain product.
template <typename TE, int TI, typename TO, int NPAIR>
__global__ __launch_bounds__(NT, 1) void k_gemm_nt(Gemm g, int tiles_m, int tiles_n, float* __restrict__ work) {
  constexpr int ES = sizeof(TE), BK = ROWB / ES, EPC = 16 / ES;  // element size, K slice, elements per chunk
  constexpr int BM = 64 * TI, ROWS = BM + BN, NLD = ROWS / RSTEP, STAGE = ROWS * ROWB;
  __shared__ __attribute__((aligned(16))) char lds[2 * STAGE];

  // XCD-aware renumbering: hardware block w runs on XCD w % 8 as that XCD's (w / 8)-th block. The
  // logical tiles are dealt to the XCDs in segments of 32 consecutive tiles (one XCD's resident
  // blocks), segment s to XCD s % 8: within an XCD neighbouring tiles share operand panels in its
  // L2, and the eight XCDs work on neighbouring segments of the same product at the same time, so
  // the panels they fetch overlap in the memory-side cache (1000-atom exchange product: 2.4 % faster
  // than one contiguous range of tiles per XCD). A last partial round keeps the hardware order.
  constexpr int SEG = 32;
  const int W = gridDim.x, w = blockIdx.x;
  const int full = W / (8 * SEG) * (8 * SEG);
  int L = w;
  if (w < full) {
    const int x = w % 8, q = w / 8;
    L = ((q / SEG) * 8 + x) * SEG + q % SEG;
  }
  const int tiles = tiles_m * tiles_n;
  const int zb = L / tiles, t = L % tiles;
  int tm, tn;
  grouped_tile(t, tiles_m, tiles_n, tm, tn);
  const int split = zb % g.ksplit, b = zb / g.ksplit;
  const int b1 = b / g.nb2, b2 = b % g.nb2;
  const int64_t aoff = b1 * g.sa1 + b2 * g.sa2, boff = b1 * g.sb1 + b2 * g.sb2;
  const TE* A = static_cast<const TE*>(g.A) + aoff;
  const TE* B = static_cast<const TE*>(g.B) + boff;
  const int m0 = tm * BM, n0 = tn * BN;
  int kbeg = 0, kend = g.K;
  if (g.ksplit > 1) {
    const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    kbeg = split * kchunk;
    kend = min(g.K, kbeg + kchunk);
  }
  const int nk1 = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;  // K slices per operand pair
  const int npair = NPAIR > 1 ? g.npair : 1;
  const int nk = nk1 * npair;

  // loader: thread loads 16-byte chunk c_t of rows r_t + RSTEP q (q < NLD; the first BM / RSTEP
  // are A rows) through buffer descriptors limited to the tile's valid rows, so rows past M or N and
  // chunks past K (offset forced out of range) read as zero without branches
  const int tid = threadIdx.x;
  const int r_t = tid >> 3, c_t = tid & 7;
  const int st_off = r_t * ROWB + 16 * (c_t ^ ((r_t >> 1) & 7));  // + q * RSTEP * ROWB
  const int rows_a = max(0, min(BM, g.M - m0)), rows_b = max(0, min(BN, g.N - n0));
  const int bytes_a = (int)((int64_t)rows_a * g.lda * ES), bytes_b = (int)((int64_t)rows_b * g.ldb * ES);
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + (int64_t)m0 * g.lda, bytes_a);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(B + (int64_t)n0 * g.ldb, bytes_b);
  // the other operand pairs (same strides), when the product concatenates several along K
  // tile bases of the other operand pairs; their descriptors are built per slice from the base the
  // slice's pair selects (scalar pointers, so the descriptors stay in scalar registers)
  const TE* pa2 = nullptr;
  const TE* pb2 = nullptr;
  const TE* pa3 = nullptr;
  const TE* pb3 = nullptr;
  if constexpr (NPAIR > 1) {
    pa2 = static_cast<const TE*>(g.A2) + aoff + (int64_t)m0 * g.lda;
    pb2 = static_cast<const TE*>(g.B2) + boff + (int64_t)n0 * g.ldb;
    pa3 = static_cast<const TE*>(g.A3 ? g.A3 : g.A2) + aoff + (int64_t)m0 * g.lda;
    pb3 = static_cast<const TE*>(g.B3 ? g.B3 : g.B2) + boff + (int64_t)n0 * g.ldb;
  }
  const uint32_t va = (uint32_t)((r_t * g.lda + EPC * c_t) * ES), vb = (uint32_t)((r_t * g.ldb + EPC * c_t) * ES);
  const uint32_t qa = (uint32_t)(RSTEP * g.lda * ES), qb = (uint32_t)(RSTEP * g.ldb * ES);

  uint4 reg[NLD];
  auto gload = [&](int kt) {
    // operand pair of slice kt (wave-uniform; made scalar so the descriptor choice stays scalar)
    const int pr = NPAIR > 1 ? __builtin_amdgcn_readfirstlane(kt / nk1) : 0;
    const int k0 = kbeg + (kt - pr * nk1) * BK;
    const bool kin = k0 + EPC * c_t < kend;
    __amdgpu_buffer_rsrc_t rA = ra, rB = rb;
    if constexpr (NPAIR > 1) {
      if (pr > 0) {
        rA = make_rsrc(pr == 1 ? pa2 : pa3, bytes_a);
        rB = make_rsrc(pr == 1 ? pb2 : pb3, bytes_b);
      }
    }
#pragma unroll
    for (int qq = 0; qq < NLD; ++qq) {
      const bool isA = qq < BM / RSTEP;
      const uint32_t off = isA ? va + qq * qa + ES * k0 : vb + (qq - BM / RSTEP) * qb + ES * k0;
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(isA ? rA : rB, kin ? off : 0x80000000u, 0, 0);
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
  const int lr = lane & 31, hi = lane >> 5, swz = (lr >> 1) & 7;
  const int a_off = (wm + lr) * ROWB, b_off = (BM + wn + lr) * ROWB;

  f16v acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  if (nk > 0) {
    gload(0);
    sstore(0);
    if (nk > 1) gload(1);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const char* buf = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {  // chunk pairs: half-wave h reads chunk 2 ks + h
      const int chunk = 16 * ((2 * ks + hi) ^ swz);
      uint4 a[TI], bb[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) a[i] = *reinterpret_cast<const uint4*>(buf + a_off + i * 32 * ROWB + chunk);
#pragma unroll
      for (int j = 0; j < TJ; ++j) bb[j] = *reinterpret_cast<const uint4*>(buf + b_off + j * 32 * ROWB + chunk);
      if constexpr (sizeof(TE) == 4) {
        // the four MFMAs of each chunk in turn over all accumulators: consecutive MFMAs never share
        // an accumulator (each accumulator still sums its k values in the same order)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(chunk_elt(a[i], e), chunk_elt(bb[j], e), acc[i][j],
                                                               0, 0, 0);
      } else {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) acc[i][j] = mfma_chunk<TE>(a[i], bb[j], acc[i][j]);
      }
      if (ks == 1) {
        // the next slice goes to the other stage (last read before the previous barrier) while this
        // slice's remaining MFMAs run, then the slice after it is requested into the freed registers
        if (kt + 1 < nk) sstore((kt + 1) & 1);
        if (kt + 2 < nk) gload(kt + 2);
      }
    }
    __syncthreads();
  }

  // accumulator element r of lane l: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
  if (g.ksplit > 1) {
    float* Wp = work + ((int64_t)b * g.ksplit + split) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
        if (row >= g.M) continue;
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          const int col = n0 + wn + j * 32 + lr;
          if (col < g.N) Wp[(int64_t)row * g.N + col] = acc[i][j][r];
        }
      }
    return;
  }
  TO* C = static_cast<TO*>(g.C) + b1 * g.sc1 + b2 * g.sc2;
  uint16_t* Clo = (NPAIR > 1 && g.C_lo) ? static_cast<uint16_t*>(g.C_lo) + b1 * g.sc1 + b2 * g.sc2 : nullptr;
  const float bs = (float)g.alpha * (g.batch_scale ? g.batch_scale[b2] : 1.f);
  const float beta = (float)g.beta;
  int64_t coff[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int col = n0 + wn + j * 32 + lr;
    coff[j] = col < g.N ? col_offset(g, col) : -1;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
      if (row >= g.M) continue;
      const float rs = g.row_scale ? bs * g.row_scale[row] : bs;
      TO* crow = C + (int64_t)row * g.ldc;
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        if (coff[j] < 0) continue;
        TO* cp = crow + coff[j];
        float v = rs * acc[i][j][r];
        if constexpr (sizeof(TO) == 2 && NPAIR > 1) {
          if (Clo) {  // split output: the remainder of the BF16 rounding goes to C_lo
            const uint16_t h = f2bf(v);
            *reinterpret_cast<uint16_t*>(cp) = h;
            Clo[(int64_t)row * g.ldc + coff[j]] = f2bf(v - bf2f(h));
            continue;
          }
        }
        if (beta != 0.f) v += beta * load_out<TO>(cp);
        store_out<TO>(cp, v);
      }
    }
}

template <int TI>
void launch_ti(const Gemm& g, void* work, hipStream_t s) {
  constexpr int BM = 64 * TI;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  const int64_t nz = (int64_t)g.nb1 * g.nb2 * g.ksplit;
  const int64_t blocks = (int64_t)tm * tn * nz;
  RISP_CHECK(blocks < (1ll << 31), RISP_E_SHAPE, "gemm grid too large");
  float* w = static_cast<float*>(work);
  const bool multi = g.npair > 1 || g.C_lo != nullptr;
  if (g.tin == DType::F32)
    k_gemm_nt<float, TI, float, 1><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w);
  else if (g.tout == DType::F32 && !multi)
    k_gemm_nt<uint16_t, TI, float, 1><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w);
  else if (g.tout == DType::F32)
    k_gemm_nt<uint16_t, TI, float, 3><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w);
  else if (!multi)
    k_gemm_nt<uint16_t, TI, uint16_t, 1><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w);
  else
    k_gemm_nt<uint16_t, TI, uint16_t, 3><<<(unsigned)blocks, NT, 0, s>>>(g, tm, tn, w);
  RISP_LAUNCHED();
}

}  // namespace

bool gemm_bf16_nt_eligible(const Gemm& g) {
  const DType ma = g.mem_a == DType::Same ? g.tin : g.mem_a, mb = g.mem_b == DType::Same ? g.tin : g.mem_b;
  const bool bf = g.tin == DType::BF16 && (g.tout == DType::F32 || g.tout == DType::BF16);
  const bool f32 = g.tin == DType::F32 && ma == DType::F32 && mb == DType::F32 && g.tout == DType::F32;
  const bool f64 = g.tin == DType::F64 && ma == DType::F64 && mb == DType::F64 &&
                   (g.tout == DType::F64 || g.tout == DType::F32);
  if (!(bf || f32 || f64) || !g.a_kc || !g.b_kc) return false;
  const int64_t es = bf ? 2 : (f32 ? 4 : 8), epc = 16 / es;  // element bytes, elements per 16-byte chunk
  const bool aligned = (reinterpret_cast<uintptr_t>(g.A) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0);
  const bool strides = g.lda % epc == 0 && g.ldb % epc == 0 && g.sa1 % epc == 0 && g.sa2 % epc == 0 &&
                       g.sb1 % epc == 0 && g.sb2 % epc == 0 && g.K % epc == 0;
  // buffer offsets within one tile (256 rows) stay below 2^31 bytes
  const bool small = (int64_t)BN * g.lda * es < (1ll << 31) && (int64_t)BN * g.ldb * es < (1ll << 31) &&
                     g.K <= g.lda && g.K <= g.ldb;
  const bool pairs_ok = g.npair == 1 ||
                        (bf && g.npair <= 3 && reinterpret_cast<uintptr_t>(g.A2) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(g.B2) % 16 == 0 &&
                         (g.npair < 3 || (reinterpret_cast<uintptr_t>(g.A3) % 16 == 0 &&
                                          reinterpret_cast<uintptr_t>(g.B3) % 16 == 0)));
  const bool lo_ok = g.C_lo == nullptr || (bf && g.tout == DType::BF16 && g.beta == 0.0 && g.ksplit <= 1);
  return aligned && strides && small && pairs_ok && lo_ok;
}

int gemm_bf16_nt_tile(const Gemm& g) {
  if (g.tin == DType::F64) return 128;
  // pick BM in {256, 192, 128}: fraction of useful rows x fill of the last wave of blocks x
  // relative per-tile throughput of the narrower tiles (fewer MFMAs per LDS byte)
  const int64_t nz = (int64_t)g.nb1 * g.nb2 * g.ksplit;
  const int64_t tn = (g.N + BN - 1) / BN;
  double best = -1.0;
  int best_ti = 4;
  for (int ti = 4; ti >= 2; --ti) {
    const int bm = 64 * ti;
    const int64_t tm = (g.M + bm - 1) / bm;
    const int64_t blocks = tm * tn * nz;
    const double rows = (double)g.M / (double)(tm * bm);
    const double fill = (double)blocks / (double)(((blocks + 255) / 256) * 256);
    const double speed = ti == 4 ? 1.0 : (ti == 3 ? 0.98 : 0.8);
    const double score = rows * fill * speed;
    if (score > best + 1e-9) {
      best = score;
      best_ti = ti;
    }
  }
  return 64 * best_ti;
}

void gemm_bf16_nt(const Gemm& g, void* work, hipStream_t s) {
  if (g.tin == DType::F64) {
    gemm_f64_nt(g, work, s);
    return;
  }
  switch (gemm_bf16_nt_tile(g)) {
    case 256: launch_ti<4>(g, work, s); break;
    case 192: launch_ti<3>(g, work, s); break;
    default: launch_ti<2>(g, work, s); break;
  }
}

}  // namespace risp
