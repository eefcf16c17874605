// Transition properties and spectra of the excited states.
#pragma once

#include "common.hpp"
#include "integrals.hpp"

namespace risp {

// For n states with energies omega_dev [n] (FP64, device) and unit-normalised amplitudes X_dev
// [n][nocc][nvir] (FP32, device): T_dev [n][6] = sqrt(2) (r_ia, (r x nabla)_ia) . X (transition
// electric dipole mu_0n and magnetic term m_0n about `origin` (host [3])), f_dev [n] oscillator and
// R_dev [n] rotatory strengths. C_dev: MO coefficients [nao][nmo] FP64 on the device. Synchronises s.
void transition_properties(const DevShells& ao, const double* C_dev, int nao, int nmo, int nocc, const double* origin,
                           int n, const double* omega_dev, const float* X_dev, double* T_dev, double* f_dev,
                           double* R_dev, hipStream_t s);

// out_dev [npts]: sum_k s_k (g / pi) / ((e0 + q de - omega_k)^2 + g^2), g = hwhm.
void lorentz_spectrum(const double* omega_dev, const double* s_dev, int n, double hwhm, double e0, double de, int npts,
                      double* out_dev, hipStream_t s);

}  // namespace risp
