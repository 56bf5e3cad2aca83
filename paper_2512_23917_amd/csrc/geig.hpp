// General (non-Hermitian) eigendecomposition kernels (see geig.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace tci {

// Largest matrix order of the one-workgroup Hessenberg / Schur kernels.
constexpr int GEIG_MAX_N = 1024;
// QR sweeps allowed per eigenvalue before the iteration reports failure.
constexpr int GEIG_MAX_SWEEPS = 60;

// H (n x n complex128, row-major) -> its complex Schur form T in place, Q ->
// the unitary Z with A = Z T Z^H (Q is overwritten; no input needed).
// status[0] = 1 when the QR iteration did not converge; fro[0] = ||T||_F.
hipError_t geig_schur(cd* H, cd* Q, int n, int* status, double* fro, hipStream_t s);
// w[k] = T[k, k]
hipError_t geig_diag(const cd* T, int n, cd* w, hipStream_t s);
// X (n x n): eigenvectors of the upper triangular T by back substitution.
hipError_t geig_triangular_vectors(const cd* T, cd* X, int n, const double* fro, hipStream_t s);
// out[:, k] = V[:, perm[k]] scaled to unit 2-norm, its largest-modulus entry
// (the first on exact ties) made real positive.
hipError_t geig_finish(const cd* V, const int* perm, int n, cd* out, hipStream_t s);

}  // namespace tci
