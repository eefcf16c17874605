// Obara-Saika recurrences for primitive Cartesian Gaussians with l <= 1 on gfx950 (FP64 VALU).
//
// Vertical recurrence (Obara & Saika 1986, written for [e 0|f 0]^(m) with product centres P, Q and
// W = (p P + q Q)/(p + q), rho = p q/(p + q)):
//   [e+1_i|f]^(m) = PA_i [e|f]^(m) + WP_i [e|f]^(m+1)
//                 + e_i/(2p) ([e-1_i|f]^(m) - rho/p [e-1_i|f]^(m+1)) + f_i/(2(p+q)) [e|f-1_i]^(m+1)
//   [e|f+1_i]^(m) = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
//                 + f_i/(2q) ([e|f-1_i]^(m) - rho/q [e|f-1_i]^(m+1)) + e_i/(2(p+q)) [e-1_i|f]^(m+1)
// and horizontal transfer (a, b+1_j| = (a+1_j, b| + AB_j (a, b|.
// The base [0|0]^(m) is linear in the operator, so alpha/r + beta erf(omega r)/r enters only
// through S[m] = K (alpha F_m(T) + beta kappa^(m+1/2) F_m(kappa T)), kappa = omega^2/(omega^2+rho):
// the attenuated operator is the Coulomb potential of a Gaussian of exponent omega^2.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace risp {

struct OSCtx {
  double PA[3], WP[3], QC[3], WQ[3];
  double i2p, i2q, i2pq, rp, rq;  // 1/(2p), 1/(2q), 1/(2(p+q)), rho/p, rho/q
  double S[5];
};

__host__ __device__ constexpr int pick(int v0, int v1, int v2, int i) {
  return i == 0 ? v0 : (i == 1 ? v1 : v2);
}
__host__ __device__ constexpr int first_nz(int v0, int v1, int v2) {
  return v0 > 0 ? 0 : (v1 > 0 ? 1 : 2);
}

template <int e0, int e1, int e2, int f0, int f1, int f2, int m>
__device__ __forceinline__ double vrr(const OSCtx& c) {
  if constexpr (e0 < 0 || e1 < 0 || e2 < 0 || f0 < 0 || f1 < 0 || f2 < 0) {
    return 0.0;
  } else if constexpr (e0 + e1 + e2 == 0 && f0 + f1 + f2 == 0) {
    return c.S[m];
  } else if constexpr (e0 + e1 + e2 > 0) {
    constexpr int i = first_nz(e0, e1, e2);
    constexpr int a0 = e0 - (i == 0), a1 = e1 - (i == 1), a2 = e2 - (i == 2);  // e - 1_i
    constexpr int ai = pick(a0, a1, a2, i);
    constexpr int fi = pick(f0, f1, f2, i);
    double v = c.PA[i] * vrr<a0, a1, a2, f0, f1, f2, m>(c) +
               c.WP[i] * vrr<a0, a1, a2, f0, f1, f2, m + 1>(c);
    if constexpr (ai > 0) {
      v += ai * c.i2p *
           (vrr<a0 - (i == 0), a1 - (i == 1), a2 - (i == 2), f0, f1, f2, m>(c) -
            c.rp * vrr<a0 - (i == 0), a1 - (i == 1), a2 - (i == 2), f0, f1, f2, m + 1>(c));
    }
    if constexpr (fi > 0) {
      v += fi * c.i2pq * vrr<a0, a1, a2, f0 - (i == 0), f1 - (i == 1), f2 - (i == 2), m + 1>(c);
    }
    return v;
  } else {
    // bra is s: build the ket
    constexpr int i = first_nz(f0, f1, f2);
    constexpr int g0 = f0 - (i == 0), g1 = f1 - (i == 1), g2 = f2 - (i == 2);  // f - 1_i
    constexpr int gi = pick(g0, g1, g2, i);
    double v = c.QC[i] * vrr<0, 0, 0, g0, g1, g2, m>(c) + c.WQ[i] * vrr<0, 0, 0, g0, g1, g2, m + 1>(c);
    if constexpr (gi > 0) {
      v += gi * c.i2q *
           (vrr<0, 0, 0, g0 - (i == 0), g1 - (i == 1), g2 - (i == 2), m>(c) -
            c.rq * vrr<0, 0, 0, g0 - (i == 0), g1 - (i == 1), g2 - (i == 2), m + 1>(c));
    }
    return v;
  }
}

// Cartesian component k of a shell with angular momentum L (L <= 1): exponent along direction d.
__host__ __device__ constexpr int cart(int L, int k, int d) { return (L == 1 && k == d) ? 1 : 0; }
__host__ __device__ constexpr int ncart(int L) { return L == 0 ? 1 : 3; }

template <int F, int... I, typename Fn>
__device__ __forceinline__ void static_for_impl(Fn&& fn, std::integer_sequence<int, I...>) {
  (fn(std::integral_constant<int, F + I>{}), ...);
}
template <int F, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  static_for_impl<F>(fn, std::make_integer_sequence<int, N - F>{});
}

// (a b | c) for components ka of shell LA at A, kb of LB at B, kc of LC (the auxiliary Gaussian).
template <int LA, int ka, int LB, int kb, int LC, int kc>
__device__ __forceinline__ double os3c(const OSCtx& c, const double AB[3]) {
  constexpr int a0 = cart(LA, ka, 0), a1 = cart(LA, ka, 1), a2 = cart(LA, ka, 2);
  constexpr int c0 = cart(LC, kc, 0), c1 = cart(LC, kc, 1), c2 = cart(LC, kc, 2);
  if constexpr (LB == 0) {
    return vrr<a0, a1, a2, c0, c1, c2, 0>(c);
  } else {
    constexpr int j = kb;
    return vrr<a0 + (j == 0), a1 + (j == 1), a2 + (j == 2), c0, c1, c2, 0>(c) +
           AB[j] * vrr<a0, a1, a2, c0, c1, c2, 0>(c);
  }
}

// (a b | a b) for the diagonal of the 4-centre integrals, bra and ket both (A, B).
template <int LA, int ka, int LB, int kb>
__device__ __forceinline__ double os4c_diag(const OSCtx& c, const double AB[3]) {
  constexpr int a0 = cart(LA, ka, 0), a1 = cart(LA, ka, 1), a2 = cart(LA, ka, 2);
  if constexpr (LB == 0) {
    return vrr<a0, a1, a2, a0, a1, a2, 0>(c);
  } else {
    constexpr int j = kb;
    constexpr int b0 = a0 + (j == 0), b1 = a1 + (j == 1), b2 = a2 + (j == 2);
    // (a+1_j + AB_j a | a+1_j + AB_j a)
    return vrr<b0, b1, b2, b0, b1, b2, 0>(c) + AB[j] * vrr<a0, a1, a2, b0, b1, b2, 0>(c) +
           AB[j] * vrr<b0, b1, b2, a0, a1, a2, 0>(c) + AB[j] * AB[j] * vrr<a0, a1, a2, a0, a1, a2, 0>(c);
  }
}

}  // namespace risp
