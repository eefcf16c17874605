// FP64 symmetric eigensolver for the small Davidson subspace matrix (one workgroup on the device).
#pragma once

#include "common.hpp"

namespace risp {

// Lowest k eigenpairs of the symmetric n x n matrix H (row stride ld, destroyed): eigenvalues
// ascending in w[0..k), eigenvectors in the columns 0..k-1 of Z (row stride ld). ws must hold
// subspace_eig_workspace(n, k) bytes.
size_t subspace_eig_workspace(int n, int k);
void subspace_eig(double* H, int n, int ld, int k, double* w, double* Z, double* ws, hipStream_t s);

}  // namespace risp
