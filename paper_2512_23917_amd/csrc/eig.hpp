// Batched FP64 Hermitian eigensolver pieces (see eig.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace tci {

constexpr int TRIDIAG_NB = 32;
// The reduction reads G only at entries with col - row < TRIDIAG_BAND (the
// lower triangle and the 64 x 64 diagonal tiles); producers may skip the rest.
constexpr int TRIDIAG_BAND = 64;

// Layout per problem (row-major unless stated), problems strided by s*:
//   G    n x n, ld ldg      the Hermitian matrix; read (and overwritten) only at col - row < TRIDIAG_BAND
//   Vt   n x n, ld n        Vt[c * n + r] = reflector c at row r (0 for r <= c, 1 at r = c+1)
//   Wp   n x NB, ld NB      panel W of the blocked reduction
//   y    n                  Hermitian matrix-vector product
//   d, e (real), tau        tridiagonal diagonal / off-diagonal, reflector scalars (dtype)
struct TriArgs {
  int n;
  void* G; long long ldg, sG;
  double* d; double* e; long long sde;
  void* tau; long long stau;
  void* Vt; long long sVt;
  void* Wp; long long sWp;
  void* y; long long sy;
  void* ws; long long sws;   // per-problem workspace of tridiag_ws_bytes(n) bytes
};

// Bytes of the per-problem workspace of the reduction (zero-fill before use).
size_t tridiag_ws_bytes(int dtype, int n);

// G = Q T Q^H (dtype C128 or F64).
hipError_t tridiagonalize(int dtype, const TriArgs& a, int batch, hipStream_t s);
// lam[b][j], j < kmax: the j-th largest eigenvalue of tridiag(d, e).  e2: scratch like e.
hipError_t tridiag_eigvals_top(const double* d, const double* e, double* e2, long long sde, int n,
                               int kmax, double* lam, long long slam, int batch, hipStream_t s);
// Z[b] (n x kmax, ld ldz, real): unit eigenvectors of tridiag(d, e) for lam[b][j], j < chi[b]
// (chi may be null = kmax).  work: 4 * batch * n * ldz doubles.
hipError_t tridiag_invit(const double* d, const double* e, long long sde, int n, const double* lam,
                         long long slam, const int* chi, int kmax, double* Z, long long ldz, long long sZ,
                         double* work, int batch, hipStream_t s);
// U[b] (n x kmax, ld ldu, dtype) <- Q U[b].  Tf: per problem
// tridiag_backtransform_tf_elems(n) elements of dtype (stride sTf); work:
// tridiag_backtransform_work_bytes(dtype, kmax, batch) bytes (the reflector
// products plus the split-K scratch of the thin products).
size_t tridiag_backtransform_tf_elems(int n);
size_t tridiag_backtransform_work_bytes(int dtype, int kmax, int batch);
hipError_t tridiag_backtransform(int dtype, const TriArgs& a, void* Tf, long long sTf, void* U,
                                 long long ldu, long long sU, int kmax, void* work, int batch,
                                 hipStream_t s);

}  // namespace tci
