// BF16 products with both operands stored contraction-contiguous (C = A . B^T), the form of the
// exchange and Coulomb-Y products of sigma. 128 x 256 output tile per 256-thread block (4 wave64s,
// each 64 x 128 with v_mfma_f32_32x32x16_bf16), K in slices of 64 staged through LDS; the next
// slice's global loads are issued before the current slice's MFMAs so their latency is hidden.
#include "gemm.hpp"

namespace risp {

namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 256, BK = 64, LDK = BK + 8;  // LDS row stride in elements (144 bytes)

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <typename TO> __device__ __forceinline__ void store_out(TO* p, double v);
template <> __device__ __forceinline__ void store_out<float>(float* p, double v) { *p = (float)v; }
template <> __device__ __forceinline__ void store_out<uint16_t>(uint16_t* p, double v) { *p = f2bf((float)v); }
template <typename TO> __device__ __forceinline__ double load_out(const TO* p);
template <> __device__ __forceinline__ double load_out<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ double load_out<uint16_t>(const uint16_t* p) { return bf2f(*p); }

// rows x 64 slice starting at (r0, k0) of a k-contiguous BF16 operand into registers (16-byte
// vectors; out-of-range elements are zero)
template <int ROWS>
__device__ __forceinline__ void gload(uint4 (&r)[ROWS / 32], const uint16_t* __restrict__ src, int64_t ld,
                                      int nrows, int kend, int r0, int k0) {
#pragma unroll
  for (int q = 0; q < ROWS / 32; ++q) {
    const int v = threadIdx.x + 256 * q;
    const int row = v >> 3, kv = (v & 7) * 8;
    const int gr = r0 + row, gk = k0 + kv;
    if (gr < nrows && gk + 8 <= kend) {
      r[q] = *reinterpret_cast<const uint4*>(src + gr * ld + gk);
    } else {
      uint16_t t[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = (gr < nrows && gk + e < kend) ? src[gr * ld + gk + e] : (uint16_t)0;
      r[q] = *reinterpret_cast<uint4*>(t);
    }
  }
}

template <int ROWS>
__device__ __forceinline__ void sstore(uint16_t* lds, const uint4 (&r)[ROWS / 32]) {
#pragma unroll
  for (int q = 0; q < ROWS / 32; ++q) {
    const int v = threadIdx.x + 256 * q;
    const int row = v >> 3, kv = (v & 7) * 8;
    *reinterpret_cast<uint4*>(lds + row * LDK + kv) = r[q];
  }
}

template <typename TO>
__global__ __launch_bounds__(256, 1) void k_gemm_bf16_nt(Gemm g, int batch0, float* __restrict__ work) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDK];
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int zb = blockIdx.y + batch0;
  const int split = zb % g.ksplit;
  const int b = zb / g.ksplit;
  const int b1 = b / g.nb2, b2 = b % g.nb2;
  const uint16_t* A = static_cast<const uint16_t*>(g.A) + b1 * g.sa1 + b2 * g.sa2;
  const uint16_t* B = static_cast<const uint16_t*>(g.B) + b1 * g.sb1 + b2 * g.sb2;
  const int m0 = tm * BM, n0 = tn * BN;
  int kbeg = 0, kend = g.K;
  if (g.ksplit > 1) {
    const int kchunk = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    kbeg = split * kchunk;
    kend = min(g.K, kbeg + kchunk);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 128;
  f16v acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  uint4 ra[BM / 32], rb[BN / 32];
  if (kbeg < kend) {
    gload<BM>(ra, A, g.lda, g.M, kend, m0, kbeg);
    gload<BN>(rb, B, g.ldb, g.N, kend, n0, kbeg);
    sstore<BM>(As, ra);
    sstore<BN>(Bs, rb);
  }
  __syncthreads();
  const int lr = lane & 31, lk = 8 * (lane >> 5);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      gload<BM>(ra, A, g.lda, g.M, kend, m0, k0 + BK);
      gload<BN>(rb, B, g.ldb, g.N, kend, n0, k0 + BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf8v a[2], bb[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf8v*>(As + (wm + i * 32 + lr) * LDK + ks + lk);
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = *reinterpret_cast<const bf8v*>(Bs + (wn + j * 32 + lr) * LDK + ks + lk);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      __syncthreads();
      sstore<BM>(As, ra);
      sstore<BN>(Bs, rb);
      __syncthreads();
    }
  }

  if (g.ksplit > 1) {
    float* W = work + ((int64_t)b * g.ksplit + split) * g.M * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int col = n0 + wn + j * 32 + lr;
          if (row < g.M && col < g.N) W[(int64_t)row * g.N + col] = acc[i][j][r];
        }
    return;
  }
  TO* C = static_cast<TO*>(g.C) + b1 * g.sc1 + b2 * g.sc2;
  const double bs = g.alpha * (g.batch_scale ? (double)g.batch_scale[b2] : 1.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (row >= g.M) continue;
      const double rs = g.row_scale ? bs * (double)g.row_scale[row] : bs;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn + j * 32 + lr;
        if (col < g.N) {
          TO* cp = C + (int64_t)row * g.ldc + col;
          double v = rs * (double)acc[i][j][r];
          if (g.beta != 0.0) v += g.beta * load_out<TO>(cp);
          store_out<TO>(cp, v);
        }
      }
    }
}

}  // namespace

bool gemm_bf16_nt_eligible(const Gemm& g) {
  const bool aligned = (reinterpret_cast<uintptr_t>(g.A) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0);
  const bool strides = g.lda % 8 == 0 && g.ldb % 8 == 0 && g.sa1 % 8 == 0 && g.sa2 % 8 == 0 &&
                       g.sb1 % 8 == 0 && g.sb2 % 8 == 0;
  return g.tin == DType::BF16 && g.a_kc && g.b_kc && aligned && strides &&
         (g.tout == DType::F32 || g.tout == DType::BF16);
}

void gemm_bf16_nt(const Gemm& g, void* work, hipStream_t s) {
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  const int64_t nz = (int64_t)g.nb1 * g.nb2 * g.ksplit;
  RISP_CHECK((int64_t)tm * tn < (1ll << 31), RISP_E_SHAPE, "gemm grid too large");
  for (int64_t z0 = 0; z0 < nz; z0 += 65535) {
    const unsigned zc = (unsigned)std::min<int64_t>(65535, nz - z0);
    if (g.tout == DType::F32)
      k_gemm_bf16_nt<float><<<dim3(tm * tn, zc), 256, 0, s>>>(g, (int)z0, static_cast<float*>(work));
    else
      k_gemm_bf16_nt<uint16_t><<<dim3(tm * tn, zc), 256, 0, s>>>(g, (int)z0, static_cast<float*>(work));
    RISP_LAUNCHED();
  }
}

}  // namespace risp
