// Coulomb passes of sigma for BF16 and FP32 factors: skinny MFMA kernels that stream T_ia once per pass.
#pragma once

#include "common.hpp"

namespace risp {

constexpr int kCoulombMaxM = 64;  // trial vectors per call of either pass

// number of c-chunks pass Y splits the contraction into, and its partial-sum workspace (bytes)
int coulomb_y_chunks(int nJ, int64_t ld);
size_t coulomb_y_workspace(int nJ, int m, int64_t ld);

// Yt[mm][P] = bf16(s2[P] * sum_c T[P][c] Xb[mm][c]) for mm < m, P < nJ; rows mm in [m, 32 ceil(m/32))
// and columns P in [nJ, nJp) are written as zero. T [nJ][ld] and Xb [m][ld] are BF16 with zero
// padding past the nocc*nvir columns; s2 may be null; part is the workspace (part_bytes bytes).
void coulomb_y_bf16(const uint16_t* T, int nJ, int64_t ld, const uint16_t* Xb, int m, const float* s2, float* part,
                    size_t part_bytes, uint16_t* Yt, int nJp, hipStream_t s);

// sig[mm][c] = alpha * sum_P Yt[mm][P] T[P][c] for mm < m, c < ov (sig FP32 [m][ov]).
void coulomb_j_bf16(const uint16_t* T, int nJ, int64_t ld, int64_t ov, const uint16_t* Yt, int nJp, int m, float alpha,
                    float* sig, hipStream_t s);

// The same passes for FP32 factors: X [m][ld] FP32 with zero padding, Yt FP32 [32 ceil(m/32)][nJp]
// (no scales).
void coulomb_y_f32(const float* T, int nJ, int64_t ld, const float* X, int m, float* part, size_t part_bytes,
                   float* Yt, int nJp, hipStream_t s);
void coulomb_j_f32(const float* T, int nJ, int64_t ld, int64_t ov, const float* Yt, int nJp, int m, float alpha,
                   float* sig, hipStream_t s);

}  // namespace risp
