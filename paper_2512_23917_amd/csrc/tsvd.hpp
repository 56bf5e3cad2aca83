// Batched truncated-SVD engine (host orchestration of the device kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <vector>

#include "eig.hpp"
#include "linalg.hpp"
#include "runtime.hpp"

namespace tci {

// Result of a batched truncated SVD of nb matrices theta_b (m x n, FP64
// working type), all on the device inside the context arena.
struct TsvdOut {
  int kz = 0;                // max kept chi over the batch (leading dim of U)
  int kmax = 0;              // eigenvalues computed per problem (stride of s arrays)
  void* U = nullptr;         // nb x m x kz (ld kz): left singular vectors, gauge fixed
  void* Vh = nullptr;        // nb x kz x n (ld n): right singular vectors (rows), orthonormalised
  int* chi = nullptr;        // device, nb
  double* s = nullptr;       // device, nb x kmax: kept singular values (0 beyond chi)
  double* sn = nullptr;      // device, nb x kmax: s / ||s_kept||
  double* total = nullptr;   // device, nb: ||theta||_F^2
  std::vector<int> chi_h;
  std::vector<double> err_h, disc_h, total_h;
};

// theta: nb x m x n contiguous (working dtype wdt = F64 or C128); consumed
// only for reading.  The rule of trunc_svd form (2) selects chi per problem.
tci_status tsvd_run(tci_context ctx, int wdt, int nb, int m, int n, const void* theta,
                    const TruncParams& tp, TsvdOut& out);

// The two halves of tsvd_run, for callers that choose chi themselves (the
// block-sparse update truncates across sectors).  tsvd_eigvals: total weight,
// Gram matrix, tridiagonal reduction and the kmax largest Gram eigenvalues
// (descending, st.lam, stride kmax).  tsvd_vectors: for chi[b] <= kz kept
// values with 1/s in sinv (stride kmax), U (m x kz) and V^H (kz x n).  Zin
// (optional, device, used as workspace): the tridiagonal eigenvectors of the
// kept values, as tsvd_vectors would compute them (ng x kz per problem, ld
// kz); null = compute them here.
struct TsvdStage {
  int wdt = 0, nb = 0, m = 0, n = 0, ng = 0, kmax = 0;
  bool left = true;
  const void* theta = nullptr;
  TriArgs ta{};
  double *d = nullptr, *e = nullptr, *e2 = nullptr, *lam = nullptr, *total = nullptr;
};
tci_status tsvd_eigvals(tci_context ctx, int wdt, int nb, int m, int n, const void* theta, int kmax,
                        TsvdStage& st);
tci_status tsvd_vectors(tci_context ctx, const TsvdStage& st, const int* chi, int kz, const double* sinv,
                        TsvdOut& out, double* Zin = nullptr);

}  // namespace tci

namespace tci {
// Randomized truncated SVD of nb problems (see sketch.cpp).
tci_status sketch_run(tci_context ctx, int dt_lo, int wdt, int prec, int nb, int m, int n, const void* th_lo,
                      const void* th64, const TruncParams& tp, const std::vector<int>& kvec, int q, uint64_t seed,
                      const std::vector<uint32_t>& streams, TsvdOut& out, std::vector<double>& resid_h);
// Sketch rank per problem (0 = plain SVD) for TCI_SVD_RANDOMIZED / TCI_SVD_LEARNED.
tci_status choose_sketch_ranks(tci_context ctx, const tci_update_params& p, int nb, int first, int ng, int chi_max,
                               int d, std::vector<int>& kvec);
}  // namespace tci
