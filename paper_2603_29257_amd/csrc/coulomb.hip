// Coulomb passes of sigma for BF16 and FP32 factors (the 2 T_ia (T_jb^T X) term). Both passes stream the
// whole of T_ia [naux_J][ld] once and are bound by HBM bandwidth, so they get their own skinny
// MFMA kernels instead of the square-tile products:
//
//   pass Y:  Y[P][m] = s_P^2 sum_c T[P][c] X[m][c]     (c = (i, a), contraction over the long axis)
//   pass J:  sigma[m][c] = alpha sum_P Yt[m][P] T[P][c]  (contraction over the auxiliary axis)
//
// Pass Y splits c into chunks over blocks (128 P rows x up to 64 trial vectors per block) and
// reduces the chunk partial sums in a fixed order; the reduction applies s_P^2, rounds to BF16
// and transposes, giving Yt [64][nJp] (zero rows past m, zero columns past naux_J). Pass J gives
// each block 256 consecutive c and all trial vectors; T slices of 32 auxiliary rows are read as
// 16-byte row pieces and transposed into LDS as (P, P+1) pairs so the MFMA operands are
// contraction-contiguous. Addressing is 64-bit throughout (T_ia reaches tens of GB).
#include "coulomb.hpp"

namespace risp {

namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int YP = 128, YK = 64, YROWB = 128;  // pass Y: P rows per block, K slice, LDS row bytes

// one 16-byte piece, zero when out of range
__device__ __forceinline__ uint4 ld16(const uint16_t* p, bool ok) {
  return ok ? *reinterpret_cast<const uint4*>(p) : make_uint4(0, 0, 0, 0);
}

template <int MT>
__global__ __launch_bounds__(256) void k_coul_y(const uint16_t* __restrict__ T, int nJ, int64_t ld,
                                                const uint16_t* __restrict__ X, int m, int64_t chunk,
                                                float* __restrict__ part) {
  constexpr int ROWS = YP + 32 * MT, NLD = ROWS / 32, STAGE = ROWS * YROWB;
  __shared__ __attribute__((aligned(16))) char lds[2 * STAGE];
  const int P0 = blockIdx.x * YP;
  const int64_t kbeg = (int64_t)blockIdx.y * chunk, kend = min(ld, kbeg + chunk);
  const int nk = kend > kbeg ? (int)((kend - kbeg + YK - 1) / YK) : 0;
  const int tid = threadIdx.x, r_t = tid >> 3, c_t = tid & 7;
  const int st_off = r_t * YROWB + 16 * (c_t ^ ((r_t >> 1) & 7));
  uint4 reg[NLD];
  auto gload = [&](int kt) {
    const int64_t k = kbeg + (int64_t)kt * YK + 8 * c_t;
    const bool kin = k < kend;
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int row = r_t + 32 * q;
      if (row < YP) {
        const int P = P0 + row;
        reg[q] = ld16(T + (int64_t)min(P, nJ - 1) * ld + k, kin && P < nJ);
      } else {
        const int mm = row - YP;
        reg[q] = ld16(X + (int64_t)min(mm, m - 1) * ld + k, kin && mm < m);
      }
    }
  };
  auto sstore = [&](int stage) {
    char* base = lds + stage * STAGE + st_off;
#pragma unroll
    for (int q = 0; q < NLD; ++q) *reinterpret_cast<uint4*>(base + q * 32 * YROWB) = reg[q];
  };
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, hi = lane >> 5, swz = (lr >> 1) & 7;
  const int a_off = (32 * wave + lr) * YROWB, b_off = (YP + lr) * YROWB;
  f16v acc[MT];
#pragma unroll
  for (int j = 0; j < MT; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
  if (nk > 0) {
    gload(0);
    sstore(0);
    if (nk > 1) gload(1);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const char* buf = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int ks = 0; ks < YK / 16; ++ks) {
      const int chunk16 = 16 * ((2 * ks + hi) ^ swz);
      const bf8v a = *reinterpret_cast<const bf8v*>(buf + a_off + chunk16);
#pragma unroll
      for (int j = 0; j < MT; ++j) {
        const bf8v b = *reinterpret_cast<const bf8v*>(buf + b_off + j * 32 * YROWB + chunk16);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) sstore((kt + 1) & 1);
    if (kt + 2 < nk) gload(kt + 2);
    __syncthreads();
  }
  // part[chunk][P][mm]
  float* out = part + (int64_t)blockIdx.y * nJ * m;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int P = P0 + 32 * wave + 8 * (r >> 2) + 4 * hi + (r & 3);
    if (P >= nJ) continue;
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      const int mm = 32 * j + lr;
      if (mm < m) out[(int64_t)P * m + mm] = acc[j][r];
    }
  }
}

// Yt[mm][P] = bf16(s2[P] * sum_chunks part[chunk][P][mm]) for mm < 32 * MT rows, P < nJp columns
__global__ void k_coul_y_reduce(const float* __restrict__ part, int nch, int nJ, int m, const float* __restrict__ s2,
                                int rows, int nJp, uint16_t* __restrict__ Yt) {
  const int64_t total = (int64_t)rows * nJp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int mm = (int)(t / nJp), P = (int)(t % nJp);
    float v = 0.f;
    if (mm < m && P < nJ) {
      for (int c = 0; c < nch; ++c) v += part[((int64_t)c * nJ + P) * m + mm];
      if (s2) v *= s2[P];
    }
    Yt[t] = f2bf(v);
  }
}

constexpr int JC = 256, JK = 32, JROW = JK + 8;  // pass J: columns per block, P slice, LDS row (elements)

template <int MT>
__global__ __launch_bounds__(256) void k_coul_j(const uint16_t* __restrict__ T, int nJ, int64_t ld, int64_t ov,
                                                const uint16_t* __restrict__ Yt, int nJp, int m, float alpha,
                                                float* __restrict__ sig) {
  __shared__ __attribute__((aligned(16))) uint16_t Bs[JC * JROW];
  const int64_t c0 = (int64_t)blockIdx.x * JC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pp = tid & 15, cq = tid >> 4;  // loader: P pair (2 pp, 2 pp + 1), 8-column pieces cq, cq + 16
  const int nslices = nJp / JK;
  uint4 reg[4];
  auto gload = [&](int sl) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int P = sl * JK + 2 * pp + e;
        const int64_t c = c0 + 8 * (cq + 16 * h);
        const bool ok = P < nJ && c < ld;
        reg[2 * h + e] = ld16(T + (int64_t)min(P, nJ - 1) * ld + min(c, ld - 8), ok);
      }
  };
  auto sstore = [&]() {
    uint32_t* B32 = reinterpret_cast<uint32_t*>(Bs);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint16_t* lo = reinterpret_cast<const uint16_t*>(&reg[2 * h]);
      const uint16_t* hi = reinterpret_cast<const uint16_t*>(&reg[2 * h + 1]);
      const int cb = 8 * (cq + 16 * h);
#pragma unroll
      for (int e = 0; e < 8; ++e) B32[((cb + e) * JROW) / 2 + pp] = (uint32_t)lo[e] | ((uint32_t)hi[e] << 16);
    }
  };
  const int lr = lane & 31, hi = lane >> 5;
  f16v acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  if (nslices > 0) gload(0);
  for (int sl = 0; sl < nslices; ++sl) {
    __syncthreads();  // previous slice fully consumed
    sstore();
    __syncthreads();
    if (sl + 1 < nslices) gload(sl + 1);
#pragma unroll
    for (int ks = 0; ks < JK / 16; ++ks) {
      bf8v a[MT], b[2];
#pragma unroll
      for (int i = 0; i < MT; ++i)
        a[i] = *reinterpret_cast<const bf8v*>(Yt + (int64_t)(32 * i + lr) * nJp + sl * JK + 16 * ks + 8 * hi);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf8v*>(Bs + (64 * wave + 32 * j + lr) * JROW + 16 * ks + 8 * hi);
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int mm = 32 * i + 8 * (r >> 2) + 4 * hi + (r & 3);
      if (mm >= m) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t c = c0 + 64 * wave + 32 * j + lr;
        if (c < ov) sig[(int64_t)mm * ov + c] = alpha * acc[i][j][r];
      }
    }
}

// ---- FP32 factors (plain FP32 path and the FP32 correction pass) ----
// Same structure with 128-byte rows of 32 floats. v_mfma_f32_32x32x2_f32 takes one k per lane and
// half-wave, so a lane's 16-byte chunk (four consecutive k) feeds four MFMAs: MFMA e of chunk pair
// ks contracts k = 8 ks + e (half-wave 0) and 8 ks + 4 + e (half-wave 1), the same for both
// operands; the sum over k does not depend on its order.
constexpr int YK32 = 32;  // pass Y: K slice (floats per 128-byte row)

__device__ __forceinline__ uint4 ld16f(const float* p, bool ok) {
  return ok ? *reinterpret_cast<const uint4*>(p) : make_uint4(0, 0, 0, 0);
}
__device__ __forceinline__ float elt(uint4 v, int e) {
  return __uint_as_float(e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w)));
}

template <int MT>
__global__ __launch_bounds__(256) void k_coul_y32(const float* __restrict__ T, int nJ, int64_t ld,
                                                  const float* __restrict__ X, int m, int64_t chunk,
                                                  float* __restrict__ part) {
  constexpr int ROWS = YP + 32 * MT, NLD = ROWS / 32, STAGE = ROWS * YROWB;
  __shared__ __attribute__((aligned(16))) char lds[2 * STAGE];
  const int P0 = blockIdx.x * YP;
  const int64_t kbeg = (int64_t)blockIdx.y * chunk, kend = min(ld, kbeg + chunk);
  const int nk = kend > kbeg ? (int)((kend - kbeg + YK32 - 1) / YK32) : 0;
  const int tid = threadIdx.x, r_t = tid >> 3, c_t = tid & 7;
  const int st_off = r_t * YROWB + 16 * (c_t ^ ((r_t >> 1) & 7));
  uint4 reg[NLD];
  auto gload = [&](int kt) {
    const int64_t k = kbeg + (int64_t)kt * YK32 + 4 * c_t;
    const bool kin = k < kend;
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int row = r_t + 32 * q;
      if (row < YP) {
        const int P = P0 + row;
        reg[q] = ld16f(T + (int64_t)min(P, nJ - 1) * ld + k, kin && P < nJ);
      } else {
        const int mm = row - YP;
        reg[q] = ld16f(X + (int64_t)min(mm, m - 1) * ld + k, kin && mm < m);
      }
    }
  };
  auto sstore = [&](int stage) {
    char* base = lds + stage * STAGE + st_off;
#pragma unroll
    for (int q = 0; q < NLD; ++q) *reinterpret_cast<uint4*>(base + q * 32 * YROWB) = reg[q];
  };
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, hi = lane >> 5, swz = (lr >> 1) & 7;
  const int a_off = (32 * wave + lr) * YROWB, b_off = (YP + lr) * YROWB;
  f16v acc[MT];
#pragma unroll
  for (int j = 0; j < MT; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
  if (nk > 0) {
    gload(0);
    sstore(0);
    if (nk > 1) gload(1);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const char* buf = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int ks = 0; ks < YK32 / 8; ++ks) {
      const int chunk16 = 16 * ((2 * ks + hi) ^ swz);
      const uint4 a = *reinterpret_cast<const uint4*>(buf + a_off + chunk16);
      uint4 b[MT];
#pragma unroll
      for (int j = 0; j < MT; ++j) b[j] = *reinterpret_cast<const uint4*>(buf + b_off + j * 32 * YROWB + chunk16);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int j = 0; j < MT; ++j)
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(elt(a, e), elt(b[j], e), acc[j], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore((kt + 1) & 1);
    if (kt + 2 < nk) gload(kt + 2);
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.y * nJ * m;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int P = P0 + 32 * wave + 8 * (r >> 2) + 4 * hi + (r & 3);
    if (P >= nJ) continue;
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      const int mm = 32 * j + lr;
      if (mm < m) out[(int64_t)P * m + mm] = acc[j][r];
    }
  }
}

// Yt[mm][P] = sum_chunks part[chunk][P][mm] (FP32) for mm < 32 * MT rows, P < nJp columns
__global__ void k_coul_y_reduce32(const float* __restrict__ part, int nch, int nJ, int m, int rows, int nJp,
                                  float* __restrict__ Yt) {
  const int64_t total = (int64_t)rows * nJp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int mm = (int)(t / nJp), P = (int)(t % nJp);
    float v = 0.f;
    if (mm < m && P < nJ)
      for (int c = 0; c < nch; ++c) v += part[((int64_t)c * nJ + P) * m + mm];
    Yt[t] = v;
  }
}

constexpr int JROW32 = JK + 4;  // pass J (FP32): LDS row of one column, in floats

template <int MT>
__global__ __launch_bounds__(256) void k_coul_j32(const float* __restrict__ T, int nJ, int64_t ld, int64_t ov,
                                                  const float* __restrict__ Yt, int nJp, int m, float alpha,
                                                  float* __restrict__ sig) {
  __shared__ __attribute__((aligned(16))) float Bs[JC * JROW32];
  const int64_t c0 = (int64_t)blockIdx.x * JC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pl = tid & 31, cq = tid >> 5;  // loader: auxiliary row pl of the slice, 4-column pieces cq + 8 h
  const int nslices = nJp / JK;
  uint4 reg[8];
  auto gload = [&](int sl) {
    const int P = sl * JK + pl;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int64_t c = c0 + 4 * (cq + 8 * h);
      reg[h] = ld16f(T + (int64_t)min(P, nJ - 1) * ld + min(c, ld - 4), P < nJ && c < ld);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int cb = 4 * (cq + 8 * h);
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[(cb + e) * JROW32 + pl] = elt(reg[h], e);
    }
  };
  const int lr = lane & 31, hi = lane >> 5;
  f16v acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  if (nslices > 0) gload(0);
  for (int sl = 0; sl < nslices; ++sl) {
    __syncthreads();  // previous slice fully consumed
    sstore();
    __syncthreads();
    if (sl + 1 < nslices) gload(sl + 1);
#pragma unroll
    for (int ks = 0; ks < JK / 8; ++ks) {
      uint4 a[MT], b[2];
#pragma unroll
      for (int i = 0; i < MT; ++i)
        a[i] = *reinterpret_cast<const uint4*>(Yt + (int64_t)(32 * i + lr) * nJp + sl * JK + 8 * ks + 4 * hi);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const uint4*>(Bs + (64 * wave + 32 * j + lr) * JROW32 + 8 * ks + 4 * hi);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(elt(a[i], e), elt(b[j], e), acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int mm = 32 * i + 8 * (r >> 2) + 4 * hi + (r & 3);
      if (mm >= m) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t c = c0 + 64 * wave + 32 * j + lr;
        if (c < ov) sig[(int64_t)mm * ov + c] = alpha * acc[i][j][r];
      }
    }
}

}  // namespace

int coulomb_y_chunks(int nJ, int64_t ld) {
  const int ptiles = (nJ + YP - 1) / YP;
  const int64_t slices = (ld + YK - 1) / YK;
  const int64_t want = (1024 + ptiles - 1) / ptiles;  // about four blocks per CU
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, slices));
}

size_t coulomb_y_workspace(int nJ, int m, int64_t ld) {
  return sizeof(float) * (size_t)coulomb_y_chunks(nJ, ld) * nJ * std::min(m, kCoulombMaxM);
}

void coulomb_y_f32(const float* T, int nJ, int64_t ld, const float* X, int m, float* part, size_t part_bytes,
                   float* Yt, int nJp, hipStream_t s) {
  RISP_CHECK(m >= 1 && m <= kCoulombMaxM, RISP_E_ARG, "coulomb pass Y: 1..64 trial vectors per call");
  RISP_CHECK(ld % 8 == 0 && nJp % 32 == 0 && nJp >= nJ, RISP_E_ARG, "coulomb pass Y: bad strides");
  if (nJ == 0) return;
  const int nch = coulomb_y_chunks(nJ, ld);
  RISP_CHECK(part_bytes >= sizeof(float) * (size_t)nch * nJ * m, RISP_E_STATE, "coulomb pass Y: workspace too small");
  const int64_t slices = (ld + YK32 - 1) / YK32;
  const int64_t chunk = ((slices + nch - 1) / nch) * YK32;
  const dim3 grid((nJ + YP - 1) / YP, nch);
  if (m <= 32) k_coul_y32<1><<<grid, 256, 0, s>>>(T, nJ, ld, X, m, chunk, part);
  else k_coul_y32<2><<<grid, 256, 0, s>>>(T, nJ, ld, X, m, chunk, part);
  RISP_LAUNCHED();
  const int rows = m <= 32 ? 32 : 64;
  const int64_t total = (int64_t)rows * nJp;
  k_coul_y_reduce32<<<(unsigned)std::min<int64_t>((total + 255) / 256, 1 << 16), 256, 0, s>>>(part, nch, nJ, m, rows,
                                                                                              nJp, Yt);
  RISP_LAUNCHED();
}

void coulomb_j_f32(const float* T, int nJ, int64_t ld, int64_t ov, const float* Yt, int nJp, int m, float alpha,
                   float* sig, hipStream_t s) {
  RISP_CHECK(m >= 1 && m <= kCoulombMaxM, RISP_E_ARG, "coulomb pass J: 1..64 trial vectors per call");
  RISP_CHECK(ld % 8 == 0 && ld >= ov && nJp % 32 == 0 && nJp >= nJ, RISP_E_ARG, "coulomb pass J: bad strides");
  if (ov == 0) return;
  const unsigned grid = (unsigned)((ov + JC - 1) / JC);
  if (m <= 32) k_coul_j32<1><<<grid, 256, 0, s>>>(T, nJ, ld, ov, Yt, nJp, m, alpha, sig);
  else k_coul_j32<2><<<grid, 256, 0, s>>>(T, nJ, ld, ov, Yt, nJp, m, alpha, sig);
  RISP_LAUNCHED();
}

void coulomb_y_bf16(const uint16_t* T, int nJ, int64_t ld, const uint16_t* Xb, int m, const float* s2, float* part,
                    size_t part_bytes, uint16_t* Yt, int nJp, hipStream_t s) {
  RISP_CHECK(m >= 1 && m <= kCoulombMaxM, RISP_E_ARG, "coulomb pass Y: 1..64 trial vectors per call");
  RISP_CHECK(ld % 8 == 0 && nJp % 32 == 0 && nJp >= nJ, RISP_E_ARG, "coulomb pass Y: bad strides");
  if (nJ == 0) return;
  const int nch = coulomb_y_chunks(nJ, ld);
  RISP_CHECK(part_bytes >= sizeof(float) * (size_t)nch * nJ * m, RISP_E_STATE, "coulomb pass Y: workspace too small");
  const int64_t slices = (ld + YK - 1) / YK;
  const int64_t chunk = ((slices + nch - 1) / nch) * YK;
  const dim3 grid((nJ + YP - 1) / YP, nch);
  if (m <= 32) k_coul_y<1><<<grid, 256, 0, s>>>(T, nJ, ld, Xb, m, chunk, part);
  else k_coul_y<2><<<grid, 256, 0, s>>>(T, nJ, ld, Xb, m, chunk, part);
  RISP_LAUNCHED();
  const int rows = m <= 32 ? 32 : 64;
  const int64_t total = (int64_t)rows * nJp;
  k_coul_y_reduce<<<(unsigned)std::min<int64_t>((total + 255) / 256, 1 << 16), 256, 0, s>>>(part, nch, nJ, m, s2,
                                                                                            rows, nJp, Yt);
  RISP_LAUNCHED();
}

void coulomb_j_bf16(const uint16_t* T, int nJ, int64_t ld, int64_t ov, const uint16_t* Yt, int nJp, int m, float alpha,
                    float* sig, hipStream_t s) {
  RISP_CHECK(m >= 1 && m <= kCoulombMaxM, RISP_E_ARG, "coulomb pass J: 1..64 trial vectors per call");
  RISP_CHECK(ld % 8 == 0 && ld >= ov && nJp % 32 == 0 && nJp >= nJ, RISP_E_ARG, "coulomb pass J: bad strides");
  if (ov == 0) return;
  const unsigned grid = (unsigned)((ov + JC - 1) / JC);
  if (m <= 32) k_coul_j<1><<<grid, 256, 0, s>>>(T, nJ, ld, ov, Yt, nJp, m, alpha, sig);
  else k_coul_j<2><<<grid, 256, 0, s>>>(T, nJ, ld, ov, Yt, nJp, m, alpha, sig);
  RISP_LAUNCHED();
}

}  // namespace risp
