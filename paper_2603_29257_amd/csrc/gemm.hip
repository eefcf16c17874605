// Batched MFMA products (see gemm.hpp). One 256-thread block (4 wave64s in a 2 x 2 grid) computes a
// BM x BN tile; the K loop stages BK-deep slices of A and B through LDS. FP64/FP32 slices are kept
// mn-major in LDS ([k][row], one element per lane per MFMA), BF16 slices k-major ([row][k], eight
// consecutive k per lane, one 16-byte LDS read).
#include <algorithm>

#include "gemm.hpp"

namespace risp {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef uint16_t bfs;  // BF16 storage

__device__ __forceinline__ float bf2f(bfs h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ bfs f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bfs)(u >> 16);
}

template <typename T> struct MF;
template <> struct MF<double> {
  static constexpr int KSTEP = 4, KPL = 1, VEC = 2, BM = 64, BN = 64, BK = 16;
  using Acc = double;
  using AccV = d4v;
};
template <> struct MF<float> {
  static constexpr int KSTEP = 4, KPL = 1, VEC = 4, BM = 128, BN = 128, BK = 32;
  using Acc = float;
  using AccV = f4v;
};
template <> struct MF<bfs> {
  static constexpr int KSTEP = 32, KPL = 8, VEC = 8, BM = 128, BN = 128, BK = 64;
  using Acc = float;
  using AccV = f4v;
};

template <typename T> __device__ __forceinline__ T zero_val() { return T(0); }

// element offset of output column `col` within its row (see Gemm::n_inner)
__device__ __forceinline__ int64_t col_offset(const Gemm& g, int col) {
  if (g.n_inner <= 0) return col;
  return (int64_t)(col / g.n_inner) * g.sc_outer + col % g.n_inner;
}

template <typename TO> __device__ __forceinline__ TO to_out(double v);
template <> __device__ __forceinline__ double to_out<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_out<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bfs to_out<bfs>(double v) { return f2bf((float)v); }
template <typename TO> __device__ __forceinline__ double from_out(TO v) { return (double)v; }
template <> __device__ __forceinline__ double from_out<bfs>(bfs v) { return (double)bf2f(v); }

// LDS tile geometry per input type
template <typename T> struct Tile {
  using M = MF<T>;
  static constexpr bool KMAJOR = M::KPL > 1;
  static constexpr int PAD = KMAJOR ? 8 : (16 / (int)sizeof(T));
  // A tile: KMAJOR ? [BM][BK+PAD] : [BK][BM+PAD]
  static constexpr int A_ELEMS = KMAJOR ? M::BM * (M::BK + PAD) : M::BK * (M::BM + PAD);
  static constexpr int B_ELEMS = KMAJOR ? M::BN * (M::BK + PAD) : M::BK * (M::BN + PAD);
};

// Copy a rows x BK slice (rows r0.., k k0..) of one operand to LDS.
template <typename T, typename TM, int ROWS>
__device__ __forceinline__ void load_tile(T* __restrict__ lds, const TM* __restrict__ src, int64_t ld,
                                          bool kc, bool vec_ok, int nrows, int K, int r0, int k0) {
  using M = MF<T>;
  using TL = Tile<T>;
  constexpr int BK = M::BK;
  constexpr int VEC = 16 / (int)sizeof(TM);  // one 16-byte global load
  constexpr bool SAME = sizeof(T) == sizeof(TM);
  constexpr int LDR = TL::KMAJOR ? (BK + TL::PAD) : (ROWS + TL::PAD);  // LDS row length
  if (kc) {
    // vectors along k
    constexpr int NV = ROWS * BK / VEC;
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
      const int row = v / (BK / VEC), kk = (v % (BK / VEC)) * VEC;
      const int gr = r0 + row, gk = k0 + kk;
      TM val[VEC];
      if (vec_ok && gr < nrows && gk + VEC <= K) {
        *reinterpret_cast<uint4*>(val) = *reinterpret_cast<const uint4*>(src + gr * ld + gk);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          val[e] = (gr < nrows && gk + e < K) ? src[gr * ld + gk + e] : zero_val<TM>();
      }
      if constexpr (TL::KMAJOR && SAME) {
        *reinterpret_cast<uint4*>(lds + row * LDR + kk) = *reinterpret_cast<uint4*>(val);
      } else if constexpr (TL::KMAJOR) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) lds[row * LDR + kk + e] = (T)val[e];
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) lds[(kk + e) * LDR + row] = (T)val[e];
      }
    }
  } else {
    // vectors along the rows
    constexpr int NV = BK * ROWS / VEC;
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
      const int kk = v / (ROWS / VEC), row = (v % (ROWS / VEC)) * VEC;
      const int gr = r0 + row, gk = k0 + kk;
      TM val[VEC];
      if (vec_ok && gk < K && gr + VEC <= nrows) {
        *reinterpret_cast<uint4*>(val) = *reinterpret_cast<const uint4*>(src + gk * ld + gr);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          val[e] = (gk < K && gr + e < nrows) ? src[gk * ld + gr + e] : zero_val<TM>();
      }
      if constexpr (TL::KMAJOR) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) lds[(row + e) * LDR + kk] = (T)val[e];
      } else if constexpr (SAME) {
        *reinterpret_cast<uint4*>(lds + kk * LDR + row) = *reinterpret_cast<uint4*>(val);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) lds[kk * LDR + row + e] = (T)val[e];
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ typename MF<T>::AccV mfma(const T* a, const T* b, typename MF<T>::AccV c);
template <>
__device__ __forceinline__ d4v mfma<double>(const double* a, const double* b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(*a, *b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f4v mfma<float>(const float* a, const float* b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f4v mfma<bfs>(const bfs* a, const bfs* b, f4v c) {
  bf8v av, bv;
  __builtin_memcpy(&av, a, 16);
  __builtin_memcpy(&bv, b, 16);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

// row of accumulator element r held by lane l (column is l % 16)
template <typename T> __device__ __forceinline__ int acc_row(int l, int r) {
  if constexpr (sizeof(T) == 8) return l / 16 + 4 * r;
  else return 4 * (l / 16) + r;
}

template <typename TMA, typename TMB, typename TI, typename TO>
__global__ __launch_bounds__(256) void k_gemm(Gemm g, int batch0, void* __restrict__ work) {
  using M = MF<TI>;
  using TL = Tile<TI>;
  using Acc = typename M::Acc;
  constexpr int BM = M::BM, BN = M::BN, BK = M::BK, KSTEP = M::KSTEP, KPL = M::KPL;
  constexpr int FM = BM / 32, FN = BN / 32;  // 16x16 fragments per wave in each direction
  __shared__ __attribute__((aligned(16))) TI As[TL::A_ELEMS];
  __shared__ __attribute__((aligned(16))) TI Bs[TL::B_ELEMS];

  const int tiles_m = (g.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int zb = blockIdx.y + batch0;
  const int split = zb % g.ksplit;
  const int b = zb / g.ksplit;
  const int b1 = b / g.nb2, b2 = b % g.nb2;
  const TMA* A = static_cast<const TMA*>(g.A) + b1 * g.sa1 + b2 * g.sa2;
  const TMB* B = static_cast<const TMB*>(g.B) + b1 * g.sb1 + b2 * g.sb2;
  const int m0 = tm * BM, n0 = tn * BN;
  constexpr int VECA = 16 / (int)sizeof(TMA), VECB = 16 / (int)sizeof(TMB);
  const bool avec = (g.lda % VECA == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool bvec = (g.ldb % VECB == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);

  int kbeg = 0, kend = g.K;
  if (g.ksplit > 1) {
    const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    kbeg = split * kchunk;
    kend = min(g.K, kbeg + kchunk);
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
  typename M::AccV acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    load_tile<TI, TMA, BM>(As, A, g.lda, g.a_kc, avec, g.M, kend, m0, k0);
    load_tile<TI, TMB, BN>(Bs, B, g.ldb, g.b_kc, bvec, g.N, kend, n0, k0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += KSTEP) {
      TI af[FM][KPL], bfr[FN][KPL];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int row = wm + i * 16 + (lane & 15);
        if constexpr (TL::KMAJOR) {
          const TI* p = As + row * (BK + TL::PAD) + kk + KPL * (lane >> 4);
          *reinterpret_cast<uint4*>(af[i]) = *reinterpret_cast<const uint4*>(p);
        } else {
          af[i][0] = As[(kk + (lane >> 4)) * (BM + TL::PAD) + row];
        }
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int row = wn + j * 16 + (lane & 15);
        if constexpr (TL::KMAJOR) {
          const TI* p = Bs + row * (BK + TL::PAD) + kk + KPL * (lane >> 4);
          *reinterpret_cast<uint4*>(bfr[j]) = *reinterpret_cast<const uint4*>(p);
        } else {
          bfr[j][0] = Bs[(kk + (lane >> 4)) * (BN + TL::PAD) + row];
        }
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma<TI>(af[i], bfr[j], acc[i][j]);
    }
    __syncthreads();
  }

  if (g.ksplit > 1) {
    Acc* W = static_cast<Acc*>(work) + ((int64_t)b * g.ksplit + split) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + acc_row<TI>(lane, r);
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < g.M && col < g.N) W[(int64_t)row * g.N + col] = acc[i][j][r];
        }
    return;
  }
  TO* C = static_cast<TO*>(g.C) + b1 * g.sc1 + b2 * g.sc2;
  const double bs = g.batch_scale ? (double)g.batch_scale[b2] : 1.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + acc_row<TI>(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < g.M && col < g.N) {
          double v = g.alpha * bs * (double)acc[i][j][r];
          if (g.row_scale) v *= (double)g.row_scale[row];
          TO* cp = C + (int64_t)row * g.ldc + col_offset(g, col);
          if (g.beta != 0.0) v += g.beta * from_out<TO>(*cp);
          *cp = to_out<TO>(v);
        }
      }
}

// Fixed-order reduction of split-K partial sums with the epilogue.
template <typename Acc, typename TO>
__global__ void k_gemm_reduce(Gemm g, const Acc* __restrict__ work, int nbatch) {
  const int64_t total = (int64_t)nbatch * g.M * g.N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t / ((int64_t)g.M * g.N));
    const int64_t rc = t % ((int64_t)g.M * g.N);
    const int row = (int)(rc / g.N), col = (int)(rc % g.N);
    const Acc* w = work + (int64_t)b * g.ksplit * g.M * g.N + rc;
    Acc s = 0;
    for (int sp = 0; sp < g.ksplit; ++sp) s += w[(int64_t)sp * g.M * g.N];
    const int b1 = b / g.nb2, b2 = b % g.nb2;
    double v = g.alpha * (double)s;
    if (g.batch_scale) v *= (double)g.batch_scale[b2];
    if (g.row_scale) v *= (double)g.row_scale[row];
    TO* cp = static_cast<TO*>(g.C) + b1 * g.sc1 + b2 * g.sc2 + (int64_t)row * g.ldc + col_offset(g, col);
    if (g.beta != 0.0) v += g.beta * from_out<TO>(*cp);
    *cp = to_out<TO>(v);
  }
}

template <typename Acc, typename TO>
static void reduce_split(const Gemm& g, void* work, hipStream_t s) {
  const int64_t total = (int64_t)g.nb1 * g.nb2 * g.M * g.N;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 1 << 16);
  k_gemm_reduce<Acc, TO><<<grid, 256, 0, s>>>(g, static_cast<const Acc*>(work), g.nb1 * g.nb2);
  RISP_LAUNCHED();
}

template <typename TI> static int tile_m() { return MF<TI>::BM; }
template <typename TI> static int tile_n() { return MF<TI>::BN; }

size_t gemm_workspace_bytes(const Gemm& g) {
  if (g.ksplit <= 1) return 0;
  const size_t acc = g.tin == DType::F64 ? 8 : 4;
  return acc * (size_t)g.ksplit * g.nb1 * g.nb2 * g.M * g.N;
}

int gemm_auto_split(const Gemm& g) {
  const bool f64 = g.tin == DType::F64;
  if (f64 && gemm_bf16_nt_eligible(g)) {
    // 128 x 256 tiles, one block per CU: aim for at least two waves of blocks over 256 CUs
    const int64_t tiles = (int64_t)((g.M + 127) / 128) * ((g.N + 255) / 256) * g.nb1 * g.nb2;
    if (tiles >= 512) return 1;
    int64_t split = (512 + tiles - 1) / tiles;
    split = std::min<int64_t>(split, std::max(1, g.K / (8 * 16)));
    return (int)std::max<int64_t>(1, std::min<int64_t>(split, 4096));
  }
  if (gemm_bf16_nt_eligible(g)) {
    // large tiles, one block per CU: aim for at least four waves of blocks over 256 CUs
    Gemm h = g;
    h.ksplit = 1;
    const int bm = gemm_bf16_nt_tile(h);
    const int64_t tiles = (int64_t)((g.M + bm - 1) / bm) * ((g.N + 255) / 256) * g.nb1 * g.nb2;
    if (tiles >= 1024) return 1;
    int64_t split = (1024 + tiles - 1) / tiles;
    split = std::min<int64_t>(split, std::max(1, g.K / (8 * 64)));
    return (int)std::max<int64_t>(1, std::min<int64_t>(split, 4096));
  }
  const int bm = f64 ? 64 : 128, bn = bm;
  const int64_t tiles = (int64_t)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * g.nb1 * g.nb2;
  if (tiles >= 1024) return 1;
  const int bk = f64 ? 16 : (g.tin == DType::F32 ? 32 : 64);
  int64_t split = (2048 + tiles - 1) / tiles;
  split = std::min<int64_t>(split, std::max(1, g.K / (8 * bk)));  // keep >= 8 K-slices per split
  return (int)std::max<int64_t>(1, std::min<int64_t>(split, 4096));
}

template <typename TMA, typename TMB, typename TI, typename TO>
static void launch(const Gemm& g, void* work, hipStream_t s) {
  const int tm = (g.M + tile_m<TI>() - 1) / tile_m<TI>();
  const int tn = (g.N + tile_n<TI>() - 1) / tile_n<TI>();
  const int64_t nz = (int64_t)g.nb1 * g.nb2 * g.ksplit;
  RISP_CHECK((int64_t)tm * tn < (1ll << 31), RISP_E_SHAPE, "gemm grid too large");
  for (int64_t z0 = 0; z0 < nz; z0 += 65535) {
    const unsigned zc = (unsigned)std::min<int64_t>(65535, nz - z0);
    k_gemm<TMA, TMB, TI, TO><<<dim3(tm * tn, zc), 256, 0, s>>>(g, (int)z0, work);
    RISP_LAUNCHED();
  }
  if (g.ksplit > 1) reduce_split<typename MF<TI>::Acc, TO>(g, work, s);
}

void gemm(const Gemm& g, void* work, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 <= 0 || g.nb2 <= 0) return;
  RISP_CHECK(g.K >= 0, RISP_E_SHAPE, "gemm: negative K");
  RISP_CHECK(g.ksplit <= 1 || work != nullptr, RISP_E_ARG, "gemm: split-K needs a workspace");
  if (g.npair != 1 || g.C_lo) {
    // concatenated operand pairs and split outputs exist only in the BF16 NT kernel
    RISP_CHECK(g.tin == DType::BF16 && gemm_bf16_nt_eligible(g), RISP_E_ARG,
               "gemm: operand pairs / split output need an eligible BF16 NT product");
  }
  const DType ma = g.mem_a == DType::Same ? g.tin : g.mem_a;
  const DType mb = g.mem_b == DType::Same ? g.tin : g.mem_b;
  if (g.tin == DType::F64) {
    RISP_CHECK((ma == DType::F64 || ma == DType::F32) && (mb == DType::F64 || mb == DType::F32), RISP_E_ARG,
               "gemm: FP64 products read FP64 or FP32 operands");
    RISP_CHECK(g.tout == DType::F64 || g.tout == DType::F32, RISP_E_ARG, "gemm: FP64 products write FP64/FP32");
    const bool o64 = g.tout == DType::F64;
    if (gemm_bf16_nt_eligible(g)) {
      gemm_bf16_nt(g, work, s);
      if (g.ksplit > 1) {
        if (o64) reduce_split<double, double>(g, work, s);
        else reduce_split<double, float>(g, work, s);
      }
      return;
    }
    if (ma == DType::F64 && mb == DType::F64) {
      if (o64) launch<double, double, double, double>(g, work, s);
      else launch<double, double, double, float>(g, work, s);
    } else if (ma == DType::F32 && mb == DType::F32) {
      if (o64) launch<float, float, double, double>(g, work, s);
      else launch<float, float, double, float>(g, work, s);
    } else if (ma == DType::F32) {
      if (o64) launch<float, double, double, double>(g, work, s);
      else launch<float, double, double, float>(g, work, s);
    } else {
      if (o64) launch<double, float, double, double>(g, work, s);
      else launch<double, float, double, float>(g, work, s);
    }
  } else {
    RISP_CHECK(ma == g.tin && mb == g.tin, RISP_E_ARG, "gemm: FP32/BF16 products read their own type");
    if (gemm_bf16_nt_eligible(g)) {
      gemm_bf16_nt(g, work, s);
      if (g.ksplit > 1) {
        if (g.tout == DType::F32) reduce_split<float, float>(g, work, s);
        else reduce_split<float, bfs>(g, work, s);
      }
      return;
    }
    if (g.tin == DType::F32) {
      if (g.tout == DType::F32) launch<float, float, float, float>(g, work, s);
      else if (g.tout == DType::F64) launch<float, float, float, double>(g, work, s);
      else launch<float, float, float, bfs>(g, work, s);
    } else {
      if (g.tout == DType::F32) launch<bfs, bfs, bfs, float>(g, work, s);
      else if (g.tout == DType::BF16) launch<bfs, bfs, bfs, bfs>(g, work, s);
      else launch<bfs, bfs, bfs, double>(g, work, s);
    }
  }
}

}  // namespace risp
