// Batched truncated-SVD engine (host orchestration of the device kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <vector>

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

}  // namespace tci

extern "C" tci_status tci_two_site_update_sketched(tci_context ctx, int nupd, const tci_tensor* A,
                                                   const tci_tensor* B, const tci_tensor* gates,
                                                   const tci_update_params* p, tci_tensor* A_out,
                                                   tci_tensor* s_out, tci_tensor* B_out,
                                                   tci_update_info* infos);
