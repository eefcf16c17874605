// Tile geometry and device helpers shared by the contraction-contiguous product kernels
// (gemm_bf16.hip: BF16 and FP32 operands; gemm_f64.hip: FP64 operands).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace risp {
namespace tile {

constexpr int BN = 256, ROWB = 128;            // tile width, LDS bytes per row (one K slice)
constexpr int NW = 8, NT = 64 * NW;            // waves and threads per block
constexpr int WN = BN / (NW / 2), TJ = WN / 32;  // wave tile width, MFMA tiles across it
constexpr int RSTEP = NT / 8;                  // rows covered by one pass of the loader

// raw buffer descriptor (stride 0, num_records bytes); the fields are made wave-uniform so the
// descriptor lives in scalar registers
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const int n = __builtin_amdgcn_readfirstlane(bytes);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, n,
                                           0x00020000);
}

// Output tile of logical index t within one product: groups of kGroupM row tiles, the group's
// columns in turn, rows fastest. The blocks that run together on one XCD (consecutive logical
// indices) then share a few A row panels and a few B column panels in that XCD's L2 instead of
// every A panel of the product: on the 1000-atom exchange product (4259 x 45120 x 4264, 11
// auxiliary functions) the L2 misses fall from 45 to 35 GB per launch and the rate rises by 13 %.
constexpr int kGroupM = 6;
__device__ __forceinline__ void grouped_tile(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int gsz = kGroupM * tiles_n, grp = t / gsz, r0 = grp * kGroupM, gm = min(kGroupM, tiles_m - r0), u = t % gsz;
  tm = r0 + u % gm;
  tn = u / gm;
}

}  // namespace tile
}  // namespace risp
