// Batched linear-algebra / elementwise kernels (see linalg.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace tci {

// Truncation rule parameters (trunc_svd form 2; form 1 = chi_min 1, target 0).
struct TruncParams {
  int chi_min, chi_max;
  double target, s_min;
};

// Cholesky-QR workspace for one call, per problem: G (k x k), RI (nblk * 32 * 32),
// diag0 (k), mask (k) -- strided by problem.
struct CholWork {
  void* G;        // batch * k * k elements
  void* RI;       // batch * nblk * 32 * 32 elements
  double* diag0;  // batch * k
  double* mask;   // batch * k
  void* kws;      // optional split-K scratch of the products (null: none)
  size_t kws_bytes;
};
size_t cholqr_work_elems(int k);  // G + RI elements per problem

hipError_t sumsq_batched(int dtype, const void* x, long long n, long long sx, double* out,
                         double* partial, int batch, hipStream_t s);
constexpr int SUMSQ_PARTIALS = 128;

hipError_t gate_apply(int dtype, void* theta, long long stheta, const void* gate, long long sgate,
                      int chi_l, int d, int chi_r, int batch, hipStream_t s);

hipError_t trunc_select(const double* lam, long long slam, int kmax, const double* total,
                        const TruncParams& p, int* chi, double* err, double* disc, double* s,
                        double* sinv, double* sn, long long ss, int batch, hipStream_t st,
                        bool sv_input = false);

hipError_t gauge_columns(int dtype, void* U, long long ldu, long long sU, int m, int ncol,
                         const int* chi, int batch, hipStream_t s);

hipError_t real_to_complex(const double* z, void* u, long long n, long long sz, long long su, int batch,
                           hipStream_t s);

hipError_t compact_columns(int dtype, const void* in, long long ldin, long long sin_, void* out,
                           long long sout, int rows, int maxchi, const int* chi, const double* cs,
                           long long scs, int batch, hipStream_t s);
hipError_t scale_rows(int dtype, const void* in, long long sin_, void* out, long long sout, long long ncols,
                      int maxchi, const int* chi, const double* rs, long long srs, int batch, hipStream_t s);

// x[i] /= lam[(i / div) % mod], i < n (Vidal-form inverse bond weights).
hipError_t inv_scale_axis(int dtype, void* x, long long n, long long div, long long mod, const double* lam,
                          hipStream_t s);

hipError_t permute(int dtype, const void* in, void* out, int order, const long long* shape,
                   const int* perm, hipStream_t s);

// mode 0: columns of Y (m x k) orthonormalised; mode 1: rows of X (k x m).
// Y is consumed as workspace.  Q receives the result (dropped columns/rows zero).
// have_gram: w.G already holds the Gram matrix of Y (ortho_defect).
hipError_t cholqr(int dtype, int mode, void* Y, long long ldy, long long sY, int m, int k, void* Q,
                  long long ldq, long long sQ, CholWork w, double tau, int batch, hipStream_t s,
                  bool have_gram = false);
// Gram matrix of the columns (mode 0) or rows (mode 1) of Y into G (k x k per
// problem), then out[0] = max over problems of ||G - I||_F^2 restricted to the
// non-zero vectors (part: batch * ORTHO_DEFECT_PARTS doubles).  C128 / F64.
constexpr int ORTHO_DEFECT_PARTS = 64;
hipError_t ortho_defect(int dtype, int mode, const void* Y, long long ldy, long long sY, int m, int k, void* G,
                        double* part, double* out, int batch, hipStream_t s, void* kws = nullptr,
                        size_t kws_bytes = 0);
// Cholesky QR to first order for G = I + E with small E: R = I + M + O(E^2)
// with M = strict upper triangle of E + diag(E) / 2, so that
// X = Y - Y M (mode 0) or X = Y - M^H Y (mode 1).  G (from ortho_defect) is
// overwritten by M; X must hold a copy of Y on entry and must not alias it.
hipError_t first_order_orthonormalise(int dtype, int mode, const void* Y, long long ldy, long long sY, int m, int k,
                                      void* G, void* X, int batch, hipStream_t s, void* kws = nullptr,
                                      size_t kws_bytes = 0);
// The same to second order: R = I + M + N + O(E^3) with N = -(strict upper
// triangle of M^H M + diag(M^H M) / 2), R^-1 = I - C + O(E^3), C = M + N - M M;
// X = Y - Y C (mode 0) or Y - C^H Y (mode 1).  PS: workspace of 2 batch k x k
// matrices.  Leaves an orthogonality defect of order ||E||^3.
hipError_t second_order_orthonormalise(int dtype, int mode, const void* Y, long long ldy, long long sY, int m,
                                       int k, void* G, void* PS, void* X, int batch, hipStream_t s,
                                       void* kws = nullptr, size_t kws_bytes = 0);

}  // namespace tci
