// Truncated SVD, QR, eigh and the two-site update composites.
//
// Plain truncated SVD of theta (m x n), TCI-spec appendix "trunc_svd":
//   W = ||theta||_F^2; G = theta theta^H (m <= n) or theta^H theta (m > n);
//   G = Q T Q^H (Householder, FP64); top eigenvalues of T by bisection;
//   truncation rule a-c on s_j = sqrt(lambda_j) with eps measured against W;
//   eigenvectors by inverse iteration, Cholesky-QR2 (FP64), U = Q Z;
//   V^H = diag(1/s) U^H theta re-orthonormalised by row Cholesky-QR2.
// The two-site update wraps it (Application A listing): theta = A.B, gate,
// trunc_svd, renormalise s, write the new site tensors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "bf16x3.hpp"
#include "common.hpp"
#include "eig.hpp"
#include "gaussjordan.hpp"
#include "geig.hpp"
#include "gemm.hpp"
#include "jacobi.hpp"
#include "linalg.hpp"
#include "prof.hpp"
#include "runtime.hpp"
#include "subtensor.hpp"
#include "tsvd.hpp"
#include "vecops.hpp"

namespace tci {

static constexpr double CHOL_DROP_TAU = 1e-12;

static int work_dtype(int dt) { return dt == C64 ? C128 : dt == F32 ? F64 : dt; }

#define ARENA(ptr, type, count)                                                        \
  type* ptr = static_cast<type*>(ctx->arena.get(sizeof(type) * (size_t)(count)));      \
  if (!ptr) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace allocation failed: " #ptr)

// Squared Frobenius bound on ||G - I|| below which one first-order Cholesky-QR
// step leaves an orthogonality defect of order ||G - I||^2, below rounding.
static constexpr double FIRST_ORDER_DEFECT2 = 1e-16;
// The same for one second-order step (defect of order ||G - I||^3): V^H =
// diag(1/s) U^H theta arrives with squared defects of 1e-14 .. 1e-11 on
// power-law bonds, which the second-order step takes in place of a full
// Cholesky-QR pass and a first-order step.
static constexpr double SECOND_ORDER_DEFECT2 = 1e-10;

static tci_status cholqr2(tci_context ctx, int wdt, int mode, void* X, long long ldx, long long sX, int m,
                          int k, void* tmp, int nb) {
  // X (column mode m x k, or row mode k x m) is orthonormalised in place; tmp is
  // a buffer of the same size.  Cholesky-QR passes until the Gram matrix is
  // within FIRST_ORDER_DEFECT2 of the identity, then one first-order step
  // (at most two full passes, as in CholeskyQR2).
  hipStream_t s = ctx->stream;
  const size_t es = elem_bytes(wdt);
  // elements of one problem: the stride, or for a single problem given with
  // stride 0 the extent of its matrix (m rows, or k rows in row mode, of ldx)
  const size_t per = sX > 0 ? (size_t)sX : (size_t)(mode == 0 ? m : k) * (size_t)ldx;
  const size_t bytes = es * per * nb;
  CholWork w{};
  w.G = ctx->arena.get(es * cholqr_work_elems(k) * nb);
  w.RI = static_cast<char*>(w.G) + es * (size_t)k * k * nb;
  w.diag0 = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  w.mask = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  double* part = static_cast<double*>(ctx->arena.get(sizeof(double) * ((size_t)nb * ORTHO_DEFECT_PARTS + 1)));
  w.kws = ctx->arena.get(GEMM_SPLITK_WS_BYTES);
  w.kws_bytes = GEMM_SPLITK_WS_BYTES;
  if (!w.G || !w.diag0 || !w.mask || !part || !w.kws) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "cholqr workspace");
  double* dout = part + (size_t)nb * ORTHO_DEFECT_PARTS;
  auto defect = [&](const void* Y, double& d) -> tci_status {
    TCI_CHECK_HIP(ortho_defect(wdt, mode, Y, ldx, sX, m, k, w.G, part, dout, nb, s, w.kws, w.kws_bytes));
    TCI_CHECK_HIP(hipMemcpyAsync(&d, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    TCI_CHECK_HIP(hipStreamSynchronize(s));
    return TCI_OK;
  };
  // first-order step from Y (Gram in w.G) into X
  auto finish = [&](const void* Y) -> tci_status {
    TCI_CHECK_HIP(hipMemcpyAsync(X, Y, bytes, hipMemcpyDeviceToDevice, s));
    TCI_CHECK_HIP(first_order_orthonormalise(wdt, mode, Y, ldx, sX, m, k, w.G, X, nb, s, w.kws, w.kws_bytes));
    return TCI_OK;
  };
  double d = 0.0;
  TCI_TRY(defect(X, d));
  if (d <= FIRST_ORDER_DEFECT2) {   // X already holds the copy the step updates
    TCI_CHECK_HIP(hipMemcpyAsync(tmp, X, bytes, hipMemcpyDeviceToDevice, s));
    TCI_CHECK_HIP(first_order_orthonormalise(wdt, mode, tmp, ldx, sX, m, k, w.G, X, nb, s, w.kws, w.kws_bytes));
    return TCI_OK;
  }
  if (d <= SECOND_ORDER_DEFECT2) {
    void* ps = ctx->arena.get(es * (size_t)k * k * nb * 2);
    if (!ps) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "cholqr workspace");
    TCI_CHECK_HIP(hipMemcpyAsync(tmp, X, bytes, hipMemcpyDeviceToDevice, s));
    TCI_CHECK_HIP(second_order_orthonormalise(wdt, mode, tmp, ldx, sX, m, k, w.G, ps, X, nb, s, w.kws,
                                              w.kws_bytes));
    return TCI_OK;
  }
  TCI_CHECK_HIP(cholqr(wdt, mode, X, ldx, sX, m, k, tmp, ldx, sX, w, CHOL_DROP_TAU, nb, s, true));
  TCI_TRY(defect(tmp, d));
  if (d <= FIRST_ORDER_DEFECT2) return finish(tmp);
  TCI_CHECK_HIP(cholqr(wdt, mode, tmp, ldx, sX, m, k, X, ldx, sX, w, CHOL_DROP_TAU, nb, s, true));
  return TCI_OK;
}

tci_status tsvd_eigvals(tci_context ctx, int wdt, int nb, int m, int n, const void* theta, int kmax,
                        TsvdStage& st) {
  hipStream_t s = ctx->stream;
  const size_t es = elem_bytes(wdt);
  const int ng = std::min(m, n);
  st.wdt = wdt; st.nb = nb; st.m = m; st.n = n; st.ng = ng; st.kmax = kmax;
  st.left = (m <= n);
  st.theta = theta;
  const long long smn = (long long)m * n;

  // total weight
  ARENA(total, double, nb);
  ARENA(partial, double, (size_t)nb * SUMSQ_PARTIALS);
  TCI_CHECK_HIP(sumsq_batched(wdt, theta, smn, smn, total, partial, nb, s));
  st.total = total;

  // Gram matrix
  ARENA(Gm, char, es * (size_t)ng * ng * nb);
  const long long sG = (long long)ng * ng;
  {
    ProfTag tag("svd_gram");
    GemmArgs g = st.left ? gemm_args(ng, ng, n, OP_N, OP_C, theta, n, theta, n, Gm, ng)
                         : gemm_args(ng, ng, m, OP_C, OP_N, theta, n, theta, n, Gm, ng);
    g.sA = smn; g.sB = smn; g.sC = sG; g.batch = nb;
    g.lower_band = TRIDIAG_BAND;   // the reduction reads the lower triangle and the diagonal tiles
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  // tridiagonal reduction
  ARENA(d, double, (size_t)ng * nb);
  ARENA(e, double, (size_t)ng * nb);
  ARENA(e2, double, (size_t)ng * nb);
  ARENA(tau, char, es * (size_t)ng * nb);
  ARENA(Vt, char, es * (size_t)ng * ng * nb);
  ARENA(Wp, char, es * (size_t)ng * TRIDIAG_NB * nb);
  ARENA(y, char, es * (size_t)ng * nb);
  TriArgs& ta = st.ta;
  ta = TriArgs{};
  ta.n = ng;
  ta.G = Gm; ta.ldg = ng; ta.sG = sG;
  ta.d = d; ta.e = e; ta.sde = ng;
  ta.tau = tau; ta.stau = ng;
  ta.Vt = Vt; ta.sVt = (long long)ng * ng;
  ta.Wp = Wp; ta.sWp = (long long)ng * TRIDIAG_NB;
  ta.y = y; ta.sy = ng;
  ta.sws = (long long)tridiag_ws_bytes(wdt, ng);
  ta.ws = ctx->arena.get((size_t)ta.sws * nb);
  if (!ta.ws) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(zero_fill(e, sizeof(double) * (size_t)ng * nb, s));
  {
    ProfTag tag("svd_tridiag");
    TCI_CHECK_HIP(tridiagonalize(wdt, ta, nb, s));
  }
  st.d = d; st.e = e; st.e2 = e2;
  // top eigenvalues
  ARENA(lam, double, (size_t)kmax * nb);
  TCI_CHECK_HIP(tridiag_eigvals_top(d, e, e2, ng, ng, kmax, lam, kmax, nb, s));
  st.lam = lam;
  return TCI_OK;
}

tci_status tsvd_vectors(tci_context ctx, const TsvdStage& st, const int* chi, int kz, const double* sinv,
                        TsvdOut& out, double* Zin) {
  hipStream_t s = ctx->stream;
  const int wdt = st.wdt, nb = st.nb, m = st.m, n = st.n, ng = st.ng, kmax = st.kmax;
  const size_t es = elem_bytes(wdt);
  const bool cplx = is_complex(wdt);
  const long long smn = (long long)m * n;
  const void* theta = st.theta;
  out.kz = kz;
  // eigenvectors of T (real), orthonormalised
  const long long sZ = (long long)ng * kz;
  double* Z = Zin;
  if (!Z) {
    Z = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)sZ * nb));
    ARENA(iw, double, (size_t)4 * ng * kz * nb);
    if (!Z) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    TCI_CHECK_HIP(zero_fill(Z, sizeof(double) * (size_t)sZ * nb, s));
    TCI_CHECK_HIP(tridiag_invit(st.d, st.e, ng, ng, st.lam, kmax, chi, kz, Z, kz, sZ, iw, nb, s));
  }
  ARENA(Z2, double, (size_t)ng * kz * nb);
  {
    ProfTag tag("svd_zqr");
    TCI_TRY(cholqr2(ctx, F64, 0, Z, kz, sZ, ng, kz, Z2, nb));
  }
  // back-transformation to eigenvectors of G
  void* Ev;
  if (cplx) {
    Ev = ctx->arena.get(es * (size_t)sZ * nb);
    if (!Ev) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    TCI_CHECK_HIP(real_to_complex(Z, Ev, sZ, sZ, sZ, nb, s));
  } else {
    Ev = Z;
  }
  const size_t tfe = tridiag_backtransform_tf_elems(ng);
  ARENA(Tf, char, es * tfe * nb);
  ARENA(btw, char, tridiag_backtransform_work_bytes(wdt, kz, nb));
  ARENA(kws, char, GEMM_SPLITK_WS_BYTES);
  {
    ProfTag tag("svd_backtr");
    TCI_CHECK_HIP(tridiag_backtransform(wdt, st.ta, Tf, (long long)tfe, Ev, kz, sZ, kz, btw, nb, s));
  }
  ProfTag tag_uv("svd_uv");
  // left factor U (m x kz)
  const long long sU = (long long)m * kz;
  void* U;
  if (st.left) {
    U = Ev;  // m == ng
  } else {
    // U = theta V diag(1/s), then orthonormalise its columns
    U = ctx->arena.get(es * (size_t)sU * nb);
    void* Ut = ctx->arena.get(es * (size_t)sU * nb);
    if (!U || !Ut) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    GemmArgs g = gemm_args(m, kz, n, OP_N, OP_N, theta, n, Ev, kz, U, kz);
    g.sA = smn; g.sB = sZ; g.sC = sU; g.batch = nb;
    g.cs = sinv; g.s_cs = kmax;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
    TCI_TRY(cholqr2(ctx, wdt, 0, U, kz, sU, m, kz, Ut, nb));
  }
  TCI_CHECK_HIP(gauge_columns(wdt, U, kz, sU, m, kz, chi, nb, s));
  // V^H = diag(1/s) U^H theta, rows orthonormalised
  const long long sV = (long long)kz * n;
  void* Vh = ctx->arena.get(es * (size_t)sV * nb);
  void* Vt2 = ctx->arena.get(es * (size_t)sV * nb);
  if (!Vh || !Vt2) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  {
    GemmArgs g = gemm_args(kz, n, m, OP_C, OP_N, U, kz, theta, n, Vh, n);
    g.sA = sU; g.sB = smn; g.sC = sV; g.batch = nb;
    g.rs = sinv; g.s_rs = kmax;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  ProfTag tag_vqr("svd_vqr");
  TCI_TRY(cholqr2(ctx, wdt, 1, Vh, n, sV, n, kz, Vt2, nb));
  out.U = U;
  out.Vh = Vh;
  return TCI_OK;
}

tci_status tsvd_run(tci_context ctx, int wdt, int nb, int m, int n, const void* theta, const TruncParams& tp,
                    TsvdOut& out) {
  hipStream_t s = ctx->stream;
  const int ng = std::min(m, n);
  const int kmax = std::max(1, std::min(tp.chi_max, ng));
  out.kmax = kmax;
  TsvdStage st;
  TCI_TRY(tsvd_eigvals(ctx, wdt, nb, m, n, theta, kmax, st));
  out.total = st.total;
  // the truncation rule
  ARENA(chi, int, nb);
  ARENA(err, double, nb);
  ARENA(disc, double, nb);
  ARENA(sv, double, (size_t)kmax * nb);
  ARENA(sinv, double, (size_t)kmax * nb);
  ARENA(sn, double, (size_t)kmax * nb);
  TCI_CHECK_HIP(trunc_select(st.lam, kmax, kmax, st.total, tp, chi, err, disc, sv, sinv, sn, kmax, nb, s));
  out.chi = chi; out.s = sv; out.sn = sn;
  out.chi_h.resize(nb); out.err_h.resize(nb); out.disc_h.resize(nb); out.total_h.resize(nb);
  TCI_CHECK_HIP(hipMemcpyAsync(out.chi_h.data(), chi, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.err_h.data(), err, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.disc_h.data(), disc, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.total_h.data(), st.total, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < nb; ++b)
    if (!std::isfinite(out.total_h[b])) TCI_RET(TCI_ERR_NUMERIC, "non-finite entries in theta");
  int kz = 1;
  for (int b = 0; b < nb; ++b) kz = std::max(kz, out.chi_h[b]);
  return tsvd_vectors(ctx, st, chi, kz, sinv, out);
}

// trunc_svd of nb small matrices (min(m, n) <= JACOBI_MAX_K, problem b at
// theta + b*m*n) by one-sided Jacobi rotations on the matrices themselves, so
// that singular values far below the largest are resolved (the Gram route
// squares the condition number).  Fills every field of `out` that
// store_outputs and tci_trunc_svd read: U (m x k per problem, ld k), Vh
// (k x n), s, sn, chi, total and the host copies, with kmax = kz = k.
static tci_status tsvd_small(tci_context ctx, int wdt, int nb, int m, int n, const void* theta,
                             const TruncParams& tp, TsvdOut& out) {
  hipStream_t s = ctx->stream;
  const size_t es = elem_bytes(wdt);
  const int k = std::min(m, n);
  const long long smn = (long long)m * n;
  ARENA(work, char, es * jacobi_work_elems(std::max(m, n), k) * nb);
  ARENA(U, char, es * (size_t)m * k * nb);
  ARENA(Vh, char, es * (size_t)k * n * nb);
  ARENA(sraw, double, (size_t)k * nb);
  ARENA(sweeps, int, nb);
  ARENA(total, double, nb);
  ARENA(partial, double, (size_t)SUMSQ_PARTIALS * nb);
  TCI_CHECK_HIP(sumsq_batched(wdt, theta, smn, smn, total, partial, nb, s));
  TCI_CHECK_HIP(jacobi_svd(wdt, theta, n, smn, m, n, work, U, (long long)m * k, Vh, (long long)k * n, sraw, k, sweeps,
                           nb, s));
  ARENA(chi, int, nb);
  ARENA(err, double, nb);
  ARENA(disc, double, nb);
  ARENA(sv, double, (size_t)k * nb);
  ARENA(sinv, double, (size_t)k * nb);
  ARENA(sn, double, (size_t)k * nb);
  TCI_CHECK_HIP(trunc_select(sraw, k, k, total, tp, chi, err, disc, sv, sinv, sn, k, nb, s, true));
  std::vector<int> sw(nb);
  out.chi_h.resize(nb); out.err_h.resize(nb); out.disc_h.resize(nb); out.total_h.resize(nb);
  TCI_CHECK_HIP(hipMemcpyAsync(out.chi_h.data(), chi, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.err_h.data(), err, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.disc_h.data(), disc, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.total_h.data(), total, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(sw.data(), sweeps, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < nb; ++b) {
    if (!std::isfinite(out.total_h[b])) TCI_RET(TCI_ERR_NUMERIC, "non-finite entries in the matrix");
    if (sw[b] < 0) TCI_RET(TCI_ERR_NOT_CONVERGED, "Jacobi SVD did not converge in 80 sweeps");
  }
  out.kmax = k; out.kz = k;
  out.U = U; out.Vh = Vh;
  out.chi = chi; out.s = sv; out.sn = sn; out.total = total;
  return TCI_OK;
}

static tci_status matricize(tci_tensor a, int k_rows, int64_t& rows, int64_t& cols) {
  if (k_rows < 1 || k_rows >= a->order) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need 1 <= k_rows < order");
  rows = 1;
  cols = 1;
  for (int i = 0; i < k_rows; ++i) rows *= a->shape[i];
  for (int i = k_rows; i < a->order; ++i) cols *= a->shape[i];
  if (rows > (1LL << 30) || cols > (1LL << 30)) TCI_RET(TCI_ERR_UNSUPPORTED, "matrix too large");
  return TCI_OK;
}

// Working copy of a tensor in FP64 (promoting F32/C64).
static tci_status working_copy(tci_context ctx, tci_tensor a, int& wdt, const void*& w) {
  wdt = a->dtype == C64 ? C128 : a->dtype == F32 ? F64 : a->dtype;
  if (wdt == a->dtype) {
    w = a->data;
    return TCI_OK;
  }
  void* p = ctx->arena.get(elem_bytes(wdt) * (size_t)tsize(a));
  if (!p) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(convert(a->dtype, a->data, wdt, p, tsize(a), ctx->stream));
  w = p;
  return TCI_OK;
}

// Copy device data of working type into an output tensor of dtype odt.
static tci_status store_as(tci_context ctx, int wdt, const void* src, tci_tensor out) {
  const long long n = tsize(out);
  if (n == 0) return TCI_OK;
  if (out->dtype == wdt)
    TCI_CHECK_HIP(hipMemcpyAsync(out->data, src, (size_t)n * elem_bytes(wdt), hipMemcpyDeviceToDevice, ctx->stream));
  else
    TCI_CHECK_HIP(convert(wdt, src, out->dtype, out->data, n, ctx->stream));
  return TCI_OK;
}

// Write the factors of the local problems listed in `idx` (local index ->
// output slot) from a TsvdOut: A' = U (s), B' = (s) V^H with s renormalised.
static tci_status store_outputs(tci_context ctx, int dt, int wdt, int chil, int d, int chir, const TsvdOut& o,
                                const std::vector<int>& idx, const tci_update_params& p, tci_tensor* A_out,
                                tci_tensor* s_out, tci_tensor* B_out, tci_update_info* infos,
                                const std::vector<double>* resid, bool fallback, const std::vector<int>* krank) {
  hipStream_t s = ctx->stream;
  const int m = chil * d, n = d * chir, nb = (int)idx.size();
  const size_t wes = elem_bytes(wdt);
  const int kz = o.kz;
  ARENA(Ucmp, char, wes * (size_t)m * kz * nb);
  ARENA(Vcmp, char, wes * (size_t)kz * n * nb);
  const bool right = p.direction == TCI_DIR_RIGHT, left = p.direction == TCI_DIR_LEFT;
  const bool vidal = p.direction == TCI_DIR_VIDAL;
  TCI_CHECK_HIP(compact_columns(wdt, o.U, kz, (long long)m * kz, Ucmp, (long long)m * kz, m, kz, o.chi,
                                right ? o.sn : nullptr, o.kmax, nb, s));
  TCI_CHECK_HIP(scale_rows(wdt, o.Vh, (long long)kz * n, Vcmp, (long long)kz * n, n, kz, o.chi,
                           left ? o.sn : nullptr, o.kmax, nb, s));
  for (int i = 0; i < nb; ++i) {
    const int g = idx[i];
    const int64_t chi = o.chi_h[i];
    const int64_t ash[3] = {chil, d, chi}, bsh[3] = {chi, d, chir}, ssh[1] = {chi};
    TCI_TRY(ensure_shape(ctx, A_out[g], dt, 3, ash));
    TCI_TRY(ensure_shape(ctx, B_out[g], dt, 3, bsh));
    TCI_TRY(ensure_shape(ctx, s_out[g], F64, 1, ssh));
    TCI_TRY(store_as(ctx, wdt, Ucmp + wes * (size_t)m * kz * i, A_out[g]));
    TCI_TRY(store_as(ctx, wdt, Vcmp + wes * (size_t)kz * n * i, B_out[g]));
    if (vidal) {
      // Gamma_A = diag(1/lambda_l) U, Gamma_B = V^H diag(1/lambda_r)
      TCI_CHECK_HIP(inv_scale_axis(dt, A_out[g]->data, (long long)chil * d * chi, (long long)d * chi, chil,
                                   static_cast<const double*>(p.lambda_left[g]->data), s));
      TCI_CHECK_HIP(inv_scale_axis(dt, B_out[g]->data, chi * d * (long long)chir, 1, chir,
                                   static_cast<const double*>(p.lambda_right[g]->data), s));
    }
    TCI_CHECK_HIP(hipMemcpyAsync(s_out[g]->data, o.sn + (size_t)o.kmax * i, sizeof(double) * chi,
                                 hipMemcpyDeviceToDevice, s));
    if (infos) {
      tci_update_info& inf = infos[g];
      std::memset(&inf, 0, sizeof(inf));
      inf.chi = chi;
      inf.trunc_err = o.err_h[i];
      inf.discarded_abs = o.disc_h[i];
      inf.norm2 = o.total_h[i];
      inf.used_fallback = fallback ? 1 : 0;
      inf.sketch_rank = krank ? (*krank)[g] : 0;
      inf.max_residual = resid ? (*resid)[i] : 0.0;
    }
  }
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  return TCI_OK;
}

// Gather problems `idx` of a strided batch (stride elems) into a new buffer.
static tci_status gather(tci_context ctx, int dt, const void* src, long long stride, const std::vector<int>& idx,
                         const void** out) {
  const size_t es = elem_bytes(dt);
  char* dst = static_cast<char*>(ctx->arena.get(es * (size_t)stride * idx.size()));
  if (!dst) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  for (size_t i = 0; i < idx.size(); ++i)
    TCI_CHECK_HIP(hipMemcpyAsync(dst + es * stride * i, static_cast<const char*>(src) + es * stride * idx[i],
                                 es * stride, hipMemcpyDeviceToDevice, ctx->stream));
  *out = dst;
  return TCI_OK;
}

// Direction and Vidal weights of an update batch: lambda_left[i] / lambda_right[i]
// F64 vectors of chil / chir finite positive entries (checked on the host).
static tci_status check_direction(tci_context ctx, const tci_update_params& p, int nupd, int64_t chil,
                                  int64_t chir) {
  if (p.direction != TCI_DIR_LEFT && p.direction != TCI_DIR_RIGHT && p.direction != TCI_DIR_VIDAL)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad direction");
  if (p.direction != TCI_DIR_VIDAL) return TCI_OK;
  if (!p.lambda_left || !p.lambda_right) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "TCI_DIR_VIDAL needs lambda_left/right");
  std::vector<double> h;
  for (int i = 0; i < nupd; ++i) {
    for (int side = 0; side < 2; ++side) {
      const tci_tensor l = side ? p.lambda_right[i] : p.lambda_left[i];
      const int64_t want = side ? chir : chil;
      if (!l || l->empty) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null Vidal weight tensor");
      if (l->dtype != TCI_F64 || l->order != 1 || l->shape[0] != want)
        TCI_RET(TCI_ERR_SHAPE, "Vidal weights must be F64 vectors of the outer bond dimensions");
      h.resize((size_t)want);
      TCI_CHECK_HIP(hipMemcpyAsync(h.data(), l->data, sizeof(double) * want, hipMemcpyDeviceToHost, ctx->stream));
      TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
      for (double x : h)
        if (!(x > 0.0) || !std::isfinite(x)) TCI_RET(TCI_ERR_NUMERIC, "Vidal weights must be finite and positive");
    }
  }
  return TCI_OK;
}

// Plain truncated SVD of nb matrices theta (FP64 working type) and the
// write-back to the output slots gslot[i].  Gram matrices, reductions,
// eigenvalues and the truncation rule run for the whole batch; the vector
// stage then runs per group of similar kept chi (ascending chi, the largest
// at most 5/4 of the smallest), each group on gathered copies of its
// problems' reduction data, so that no problem's eigenvectors, back-
// transformation and factor products are padded to the batch's largest chi.
// The plain truncated SVD in two halves, so that the first (Gram matrices,
// reductions, eigenvalues, truncation rule: no host synchronisation) can run
// on a second stream while other work of the same call proceeds.
struct PlainPending {
  int nb = 0, m = 0, n = 0, ng = 0, kmax = 0;
  const void* theta = nullptr;
  TsvdStage st;
  int* chi = nullptr;
  double *err = nullptr, *disc = nullptr, *sv = nullptr, *sinv = nullptr, *sn = nullptr;
};

static tci_status tsvd_plain_begin(tci_context ctx, int wdt, int nb, int m, int n, const void* theta,
                                   const TruncParams& tp, PlainPending& pp) {
  hipStream_t s = ctx->stream;
  pp.nb = nb; pp.m = m; pp.n = n; pp.ng = std::min(m, n);
  pp.kmax = std::max(1, std::min(tp.chi_max, pp.ng));
  pp.theta = theta;
  const int kmax = pp.kmax;
  TCI_TRY(tsvd_eigvals(ctx, wdt, nb, m, n, theta, kmax, pp.st));
  ARENA(chi, int, nb);
  ARENA(err, double, nb);
  ARENA(disc, double, nb);
  ARENA(sv, double, (size_t)kmax * nb);
  ARENA(sinv, double, (size_t)kmax * nb);
  ARENA(sn, double, (size_t)kmax * nb);
  TCI_CHECK_HIP(trunc_select(pp.st.lam, kmax, kmax, pp.st.total, tp, chi, err, disc, sv, sinv, sn, kmax, nb, s));
  pp.chi = chi; pp.err = err; pp.disc = disc; pp.sv = sv; pp.sinv = sinv; pp.sn = sn;
  return TCI_OK;
}

// The vector stage and the write-back of a begun plain batch, on the
// context stream (the caller has made the begun work visible to it).
static tci_status tsvd_plain_finish(tci_context ctx, int dt, int wdt, int chil, int d, int chir, const PlainPending& pp,
                                    const std::vector<int>& gslot, const tci_update_params& p, tci_tensor* A_out,
                                    tci_tensor* s_out, tci_tensor* B_out, tci_update_info* infos, bool fallback,
                                    const std::vector<int>* krank) {
  hipStream_t s = ctx->stream;
  const int nb = pp.nb, m = pp.m, n = pp.n, ng = pp.ng, kmax = pp.kmax;
  const void* theta = pp.theta;
  const TsvdStage& st = pp.st;
  int* chi = pp.chi;
  double *sv = pp.sv, *sinv = pp.sinv, *sn = pp.sn;
  const double *err = pp.err, *disc = pp.disc;
  std::vector<int> chi_h(nb);
  std::vector<double> err_h(nb), disc_h(nb), total_h(nb);
  TCI_CHECK_HIP(hipMemcpyAsync(chi_h.data(), chi, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(err_h.data(), err, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(disc_h.data(), disc, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(total_h.data(), st.total, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < nb; ++b)
    if (!std::isfinite(total_h[b])) TCI_RET(TCI_ERR_NUMERIC, "non-finite entries in theta");
  std::vector<int> ord(nb);
  for (int i = 0; i < nb; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return chi_h[x] < chi_h[y] || (chi_h[x] == chi_h[y] && x < y); });
  const size_t es = elem_bytes(wdt);
  const long long smn = (long long)m * n, sG = (long long)ng * ng;
  // Inverse iteration of every problem in one launch: its sequential
  // recurrences make a launch latency-bound, whatever the number of vectors.
  int kzall = 1;
  for (int b = 0; b < nb; ++b) kzall = std::max(kzall, chi_h[b]);
  const long long sZall = (long long)ng * kzall;
  ARENA(Zall, double, (size_t)sZall * nb);
  {
    const std::vector<size_t> before = ctx->arena.used_state();
    ARENA(iw, double, (size_t)4 * sZall * nb);
    TCI_CHECK_HIP(zero_fill(Zall, sizeof(double) * (size_t)sZall * nb, s));
    TCI_CHECK_HIP(tridiag_invit(st.d, st.e, ng, ng, st.lam, kmax, chi, kzall, Zall, kzall, sZall, iw, nb, s));
    ctx->arena.restore(before);   // iw is dead once the stream has run the launches above
  }
  for (int g0 = 0; g0 < nb;) {
    int g1 = g0 + 1;
    while (g1 < nb && 4 * chi_h[ord[g1]] <= 5 * chi_h[ord[g0]]) ++g1;
    const std::vector<int> loc(ord.begin() + g0, ord.begin() + g1);
    g0 = g1;
    const int ngp = (int)loc.size();
    int kz = 1;
    for (int i : loc) kz = std::max(kz, chi_h[i]);
    const std::vector<size_t> mark = ctx->arena.used_state();
    TsvdOut o;
    o.kmax = kmax;
    bool identity = ngp == nb;
    for (int i = 0; identity && i < ngp; ++i) identity = loc[i] == i;
    // the group's eigenvectors of T: columns 0 .. kz of its problems' Zall
    double* Zg = Zall;
    if (!(identity && kz == kzall)) {
      ARENA(zg, double, (size_t)ng * kz * ngp);
      for (int i = 0; i < ngp; ++i)
        TCI_CHECK_HIP(hipMemcpy2DAsync(zg + (size_t)ng * kz * i, sizeof(double) * kz, Zall + (size_t)sZall * loc[i],
                                       sizeof(double) * kzall, sizeof(double) * kz, ng, hipMemcpyDeviceToDevice, s));
      Zg = zg;
    }
    if (identity) {
      TCI_TRY(tsvd_vectors(ctx, st, chi, kz, sinv, o, Zg));
      o.chi = chi; o.s = sv; o.sn = sn; o.total = st.total;
    } else {
      TsvdStage sg = st;
      sg.nb = ngp;
      const void* ptr = nullptr;
      TCI_TRY(gather(ctx, wdt, theta, smn, loc, &ptr));
      sg.theta = ptr;
      TCI_TRY(gather(ctx, F64, st.d, ng, loc, &ptr));
      sg.d = const_cast<double*>(static_cast<const double*>(ptr));
      TCI_TRY(gather(ctx, F64, st.e, ng, loc, &ptr));
      sg.e = const_cast<double*>(static_cast<const double*>(ptr));
      TCI_TRY(gather(ctx, F64, st.lam, kmax, loc, &ptr));
      sg.lam = const_cast<double*>(static_cast<const double*>(ptr));
      TCI_TRY(gather(ctx, wdt, st.ta.Vt, sG, loc, &ptr));
      sg.ta.Vt = const_cast<void*>(ptr);
      TCI_TRY(gather(ctx, wdt, st.ta.tau, st.ta.stau, loc, &ptr));
      sg.ta.tau = const_cast<void*>(ptr);
      TCI_TRY(gather(ctx, F32, chi, 1, loc, &ptr));     // 4-byte elements
      int* chi_g = const_cast<int*>(static_cast<const int*>(ptr));
      TCI_TRY(gather(ctx, F64, sinv, kmax, loc, &ptr));
      const double* sinv_g = static_cast<const double*>(ptr);
      TCI_TRY(gather(ctx, F64, sn, kmax, loc, &ptr));
      double* sn_g = const_cast<double*>(static_cast<const double*>(ptr));
      TCI_TRY(tsvd_vectors(ctx, sg, chi_g, kz, sinv_g, o, Zg));
      o.chi = chi_g; o.sn = sn_g; o.s = nullptr;
    }
    std::vector<int> slots;
    for (int i : loc) {
      o.chi_h.push_back(chi_h[i]);
      o.err_h.push_back(err_h[i]);
      o.disc_h.push_back(disc_h[i]);
      o.total_h.push_back(total_h[i]);
      slots.push_back(gslot[i]);
    }
    // store_outputs synchronises the stream, so the group's workspace is free after it
    TCI_TRY(store_outputs(ctx, dt, wdt, chil, d, chir, o, slots, p, A_out, s_out, B_out, infos, nullptr, fallback,
                          krank));
    ctx->arena.restore(mark);
  }
  return TCI_OK;
}

static tci_status tsvd_store_grouped(tci_context ctx, int dt, int wdt, int nb, int chil, int d, int chir,
                                     const void* theta, const TruncParams& tp, const std::vector<int>& gslot,
                                     const tci_update_params& p, tci_tensor* A_out, tci_tensor* s_out,
                                     tci_tensor* B_out, tci_update_info* infos, bool fallback,
                                     const std::vector<int>* krank) {
  PlainPending pp;
  TCI_TRY(tsvd_plain_begin(ctx, wdt, nb, chil * d, d * chir, theta, tp, pp));
  return tsvd_plain_finish(ctx, dt, wdt, chil, d, chir, pp, gslot, p, A_out, s_out, B_out, infos, fallback, krank);
}

// trunc_svd of nb matrices theta ((chil*d) x (d*chir)): th_lo in the storage
// dtype dt, thw its FP64 working copy (the same pointer when dt is FP64);
// plain, randomized or learned per params; then renormalised s and the
// write-back.  `first` is the global index of problem 0 (sketch stream id).
static tci_status split_and_store(tci_context ctx, int dt, int wdt, int nb, int chil, int d, int chir,
                                  const void* th_lo, const void* thw, const tci_update_params& p, int first,
                                  tci_tensor* A_out, tci_tensor* s_out, tci_tensor* B_out, tci_update_info* infos) {
  const int m = chil * d, n = d * chir, ng = std::min(m, n);
  TruncParams tp{(int)std::min<int64_t>(p.chi_min, ng), (int)std::min<int64_t>(p.chi_max, ng), p.target_trunc_err,
                 p.s_min};
  if (tp.chi_min > tp.chi_max) tp.chi_min = tp.chi_max;
  const long long smn = (long long)m * n;
  std::vector<int> plain_idx, sk_idx, kvec(nb, 0);
  if (p.svd_mode == TCI_SVD_PLAIN) {
    for (int i = 0; i < nb; ++i) plain_idx.push_back(i);
  } else {
    TCI_TRY(choose_sketch_ranks(ctx, p, nb, first, ng, tp.chi_max, d, kvec));
    for (int i = 0; i < nb; ++i) {
      if (kvec[i] > 0 && kvec[i] < ng) sk_idx.push_back(i);
      else plain_idx.push_back(i);
    }
  }
  // The problems sent to the plain SVD from the start begin their eigenvalue
  // stage on the second stream, so that their reductions (bound by HBM and
  // launch latency) overlap the sketches (bound by the FP64 matrix cores).
  PlainPending early;
  std::vector<int> early_idx;
  struct AuxJoin {   // no return leaves work of this call running on the second stream
    hipStream_t st = nullptr;
    ~AuxJoin() { if (st) (void)hipStreamSynchronize(st); }
  } aux_join;
  if (!plain_idx.empty() && !sk_idx.empty() && ng > JACOBI_MAX_K) {
    early_idx = plain_idx;
    plain_idx.clear();
    const void* hi = thw;
    if ((int)early_idx.size() != nb) TCI_TRY(gather(ctx, wdt, thw, smn, early_idx, &hi));
    if (!ctx->aux) TCI_CHECK_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    if (!ctx->aux_ev) TCI_CHECK_HIP(hipEventCreateWithFlags(&ctx->aux_ev, hipEventDisableTiming));
    TCI_CHECK_HIP(hipEventRecord(ctx->aux_ev, ctx->stream));
    TCI_CHECK_HIP(hipStreamWaitEvent(ctx->aux, ctx->aux_ev, 0));
    aux_join.st = ctx->aux;
    const hipStream_t main_stream = ctx->stream;
    ctx->stream = ctx->aux;
    const tci_status sb = tsvd_plain_begin(ctx, wdt, (int)early_idx.size(), m, n, hi, tp, early);
    ctx->stream = main_stream;
    TCI_TRY(sb);
  }
  // Sketched problems run in groups of similar rank (ascending k, the
  // largest at most twice the smallest): no problem's products are padded
  // far beyond its own rank, and the groups stay large enough to fill the
  // chip (measured on the TEBD batch: groups within 5/4 ran 1.8% slower, one
  // group for all as fast as within 2).
  std::sort(sk_idx.begin(), sk_idx.end(), [&](int x, int y) { return kvec[x] < kvec[y] || (kvec[x] == kvec[y] && x < y); });
  for (size_t g0 = 0; g0 < sk_idx.size();) {
    size_t g1 = g0 + 1;
    while (g1 < sk_idx.size() && kvec[sk_idx[g1]] <= 2 * kvec[sk_idx[g0]]) ++g1;
    std::vector<int> grp(sk_idx.begin() + g0, sk_idx.begin() + g1);
    g0 = g1;
    const void* lo = th_lo;
    const void* hi = thw;
    bool identity = (int)grp.size() == nb;
    for (size_t i = 0; identity && i < grp.size(); ++i) identity = grp[i] == (int)i;
    if (!identity) {
      TCI_TRY(gather(ctx, dt, th_lo, smn, grp, &lo));
      hi = lo;
      if (thw != th_lo) TCI_TRY(gather(ctx, wdt, thw, smn, grp, &hi));
    }
    std::vector<int> ks;
    std::vector<uint32_t> streams;
    for (int i : grp) {
      ks.push_back(kvec[i]);
      streams.push_back((uint32_t)(first + i));
    }
    TsvdOut o;
    std::vector<double> resid;
    const int q = p.power_iters < 0 ? 2 : p.power_iters;
    const int prec = is_double(dt) ? PREC_FP64 : p.precision;
    TCI_TRY(sketch_run(ctx, dt, wdt, prec, (int)grp.size(), m, n, lo, hi, tp, ks, q, p.seed, streams, o, resid));
    const double cert = p.cert_tol > 0 ? p.cert_tol : 1e-7;
    std::vector<int> acc_local, acc_global;
    for (size_t i = 0; i < grp.size(); ++i) {
      if (o.err_h[i] <= p.target_trunc_err && resid[i] <= cert) {
        acc_local.push_back((int)i);
        acc_global.push_back(grp[i]);
      } else {
        plain_idx.push_back(grp[i]);
      }
    }
    if (acc_local.size() == grp.size()) {
      TCI_TRY(store_outputs(ctx, dt, wdt, chil, d, chir, o, acc_global, p, A_out, s_out, B_out, infos, &resid, false,
                            &kvec));
    } else if (!acc_local.empty()) {
      // store the accepted ones one at a time (their TsvdOut rows are strided)
      for (size_t a = 0; a < acc_local.size(); ++a) {
        TsvdOut one = o;
        const int i = acc_local[a];
        const size_t ew = elem_bytes(wdt);
        one.U = static_cast<char*>(o.U) + ew * (size_t)m * o.kz * i;
        one.Vh = static_cast<char*>(o.Vh) + ew * (size_t)o.kz * n * i;
        one.chi = o.chi + i;
        one.sn = o.sn + (size_t)o.kmax * i;
        one.s = o.s + (size_t)o.kmax * i;
        one.chi_h = {o.chi_h[i]};
        one.err_h = {o.err_h[i]};
        one.disc_h = {o.disc_h[i]};
        one.total_h = {o.total_h[i]};
        std::vector<double> r1 = {resid[i]};
        TCI_TRY(store_outputs(ctx, dt, wdt, chil, d, chir, one, {acc_global[a]}, p, A_out, s_out, B_out, infos, &r1,
                              false, &kvec));
      }
    }
  }
  if (!early_idx.empty()) {
    TCI_CHECK_HIP(hipStreamSynchronize(ctx->aux));
    TCI_TRY(tsvd_plain_finish(ctx, dt, wdt, chil, d, chir, early, early_idx, p, A_out, s_out, B_out, infos,
                              p.svd_mode != TCI_SVD_PLAIN, &kvec));
  }
  if (!plain_idx.empty()) {
    std::sort(plain_idx.begin(), plain_idx.end());
    const void* hi = thw;
    if ((int)plain_idx.size() != nb) TCI_TRY(gather(ctx, wdt, thw, smn, plain_idx, &hi));
    if (ng <= JACOBI_MAX_K) {
      TsvdOut o;
      TCI_TRY(tsvd_small(ctx, wdt, (int)plain_idx.size(), m, n, hi, tp, o));
      TCI_TRY(store_outputs(ctx, dt, wdt, chil, d, chir, o, plain_idx, p, A_out, s_out, B_out, infos, nullptr,
                            p.svd_mode != TCI_SVD_PLAIN, &kvec));
    } else {
      TCI_TRY(tsvd_store_grouped(ctx, dt, wdt, (int)plain_idx.size(), chil, d, chir, hi, tp, plain_idx, p, A_out,
                                 s_out, B_out, infos, p.svd_mode != TCI_SVD_PLAIN, &kvec));
    }
  }
  return TCI_OK;
}

}  // namespace tci

using namespace tci;

extern "C" {

tci_status tci_trunc_svd(tci_context ctx, tci_tensor a, int k_rows, tci_tensor u, tci_tensor s, tci_tensor vdag,
                         double* trunc_err, int64_t chi_min, int64_t chi_max, double target_trunc_err,
                         double s_min) try {
  if (!ctx || !a || !u || !s || !vdag) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  if (a->empty) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "moved-from tensor");
  if (chi_min < 1 || chi_max < 1 || chi_min > chi_max) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need 1 <= chi_min <= chi_max");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(a, k_rows, rows, cols));
  Trace tr(ctx, "trunc_svd", std::to_string(rows) + "x" + std::to_string(cols));
  ctx->arena.reset();
  int wdt;
  const void* w;
  TCI_TRY(working_copy(ctx, a, wdt, w));
  const int64_t kap = std::min(rows, cols);
  TruncParams tp{(int)std::min<int64_t>(chi_min, kap), (int)std::min<int64_t>(chi_max, kap), target_trunc_err, s_min};
  if (tp.chi_min > tp.chi_max) tp.chi_min = tp.chi_max;
  TsvdOut o;
  bool done = false;
  // Context svd mode RANDOMIZED: sketch of rank chi_max + 64 (q = 2), kept
  // when the discarded weight meets the target and the residual certificate
  // holds; otherwise the plain truncated SVD below decides.
  const int k_sk = (int)std::min<int64_t>(kap, 32 * ((tp.chi_max + 64 + 31) / 32));
  if (ctx->svd_mode == TCI_SVD_RANDOMIZED && kap > JACOBI_MAX_K && target_trunc_err > 0.0 && k_sk < kap) {
    std::vector<double> resid;
    const int prec = is_double(a->dtype) ? PREC_FP64 : ctx->precision;
    TCI_TRY(sketch_run(ctx, a->dtype, wdt, prec, 1, (int)rows, (int)cols, a->data, w, tp, {k_sk}, 2, 0, {0u}, o,
                       resid));
    done = o.err_h[0] <= target_trunc_err && resid[0] <= 1e-7;
    tr.info += done ? " randomized k=" + std::to_string(k_sk) : " randomized k=" + std::to_string(k_sk) + " fallback";
  }
  if (!done) {
    o = TsvdOut{};
    if (kap <= JACOBI_MAX_K) TCI_TRY(tsvd_small(ctx, wdt, 1, (int)rows, (int)cols, w, tp, o));
    else TCI_TRY(tsvd_run(ctx, wdt, 1, (int)rows, (int)cols, w, tp, o));
  }
  const int chi = o.chi_h[0];
  // outputs
  int64_t ushape[MAX_ORDER + 1];
  for (int i = 0; i < k_rows; ++i) ushape[i] = a->shape[i];
  ushape[k_rows] = chi;
  int64_t vshape[MAX_ORDER + 1];
  vshape[0] = chi;
  for (int i = k_rows; i < a->order; ++i) vshape[1 + i - k_rows] = a->shape[i];
  const int odt = a->dtype;
  const int rdt = is_double(odt) ? F64 : F32;
  const int order_a = a->order;
  TCI_TRY(ensure_shape(ctx, u, odt, k_rows + 1, ushape));
  TCI_TRY(ensure_shape(ctx, vdag, odt, order_a - k_rows + 1, vshape));
  int64_t sshape[1] = {chi};
  TCI_TRY(ensure_shape(ctx, s, rdt, 1, sshape));
  const size_t es = elem_bytes(wdt);
  void* ucmp = ctx->arena.get(es * (size_t)rows * chi);
  if (!ucmp) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(compact_columns(wdt, o.U, o.kz, (long long)rows * o.kz, ucmp, (long long)rows * chi, (int)rows, chi,
                                o.chi, nullptr, 0, 1, ctx->stream));
  TCI_TRY(store_as(ctx, wdt, ucmp, u));
  TCI_TRY(store_as(ctx, wdt, o.Vh, vdag));  // first chi rows are contiguous
  TCI_TRY(store_as(ctx, F64, o.s, s));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  if (trunc_err) *trunc_err = o.err_h[0];
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_svd(tci_context ctx, tci_tensor a, int k_rows, tci_tensor u, tci_tensor s, tci_tensor vdag) try {
  if (!a) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  int64_t rows, cols;
  TCI_TRY(matricize(a, k_rows, rows, cols));
  const int64_t kap = std::min(rows, cols);
  return tci_trunc_svd(ctx, a, k_rows, u, s, vdag, nullptr, kap, kap, 0.0, 0.0);
} TCI_API_CATCH

// Thin QR of the m x k (m >= k) working-precision matrix at w: Y (m x k)
// receives Q and R (k x k) the triangular factor.  Two Cholesky-QR passes,
// R = R2 R1 with the diagonals of dropped columns zeroed.
static tci_status qr_core(tci_context ctx, int wdt, int m, int k, const void* w, void*& Y, void*& R) {
  const size_t es = elem_bytes(wdt);
  hipStream_t st = ctx->stream;
  Y = ctx->arena.get(es * (size_t)m * k);
  void* Q1 = ctx->arena.get(es * (size_t)m * k);
  if (!Y || !Q1) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(hipMemcpyAsync(Y, w, es * (size_t)m * k, hipMemcpyDeviceToDevice, st));
  CholWork w1{}, w2{};
  for (CholWork* cw : {&w1, &w2}) {
    cw->G = ctx->arena.get(es * cholqr_work_elems(k));
    cw->RI = static_cast<char*>(cw->G) + es * (size_t)k * k;
    cw->diag0 = static_cast<double*>(ctx->arena.get(sizeof(double) * k));
    cw->mask = static_cast<double*>(ctx->arena.get(sizeof(double) * k));
    if (!cw->G || !cw->diag0 || !cw->mask) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  }
  TCI_CHECK_HIP(cholqr(wdt, 0, Y, k, 0, m, k, Q1, k, 0, w1, CHOL_DROP_TAU, 1, st));
  TCI_CHECK_HIP(cholqr(wdt, 0, Q1, k, 0, m, k, Y, k, 0, w2, CHOL_DROP_TAU, 1, st));
  TCI_CHECK_HIP(triu_mask(wdt, w1.G, k, 0, k, w1.mask, 0, 1, st));
  TCI_CHECK_HIP(triu_mask(wdt, w2.G, k, 0, k, w2.mask, 0, 1, st));
  R = ctx->arena.get(es * (size_t)k * k);
  if (!R) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  GemmArgs g = gemm_args(k, k, k, OP_N, OP_N, w2.G, k, w1.G, k, R, k);
  TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, st));
  return TCI_OK;
}

tci_status tci_qr(tci_context ctx, tci_tensor a, int k_rows, tci_tensor q, tci_tensor r) try {
  if (!ctx || !a || !q || !r) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(a, k_rows, rows, cols));
  if (rows < cols) TCI_RET(TCI_ERR_UNSUPPORTED, "qr of a wide matrix (rows < cols) is not supported");
  Trace tr(ctx, "qr", std::to_string(rows) + "x" + std::to_string(cols));
  ctx->arena.reset();
  int wdt;
  const void* w;
  TCI_TRY(working_copy(ctx, a, wdt, w));
  const int m = (int)rows, k = (int)cols;
  void *Y, *R;
  TCI_TRY(qr_core(ctx, wdt, m, k, w, Y, R));
  int64_t qshape[MAX_ORDER + 1], rshape[MAX_ORDER + 1];
  for (int i = 0; i < k_rows; ++i) qshape[i] = a->shape[i];
  qshape[k_rows] = k;
  rshape[0] = k;
  for (int i = k_rows; i < a->order; ++i) rshape[1 + i - k_rows] = a->shape[i];
  const int odt = a->dtype, ord = a->order;
  TCI_TRY(ensure_shape(ctx, q, odt, k_rows + 1, qshape));
  TCI_TRY(ensure_shape(ctx, r, odt, ord - k_rows + 1, rshape));
  TCI_TRY(store_as(ctx, wdt, Y, q));
  TCI_TRY(store_as(ctx, wdt, R, r));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

// Conjugate transpose of a rows x cols working-precision matrix.
static tci_status conj_transpose(tci_context ctx, int wdt, const void* in, int rows, int cols, void* out) {
  const long long shp[2] = {rows, cols};
  const int perm[2] = {1, 0};
  TCI_CHECK_HIP(permute(wdt, in, out, 2, shp, perm, ctx->stream));
  if (is_complex(wdt)) TCI_CHECK_HIP(conjugate(wdt, out, out, (long long)rows * cols, ctx->stream));
  return TCI_OK;
}

tci_status tci_lq(tci_context ctx, tci_tensor a, int k_rows, tci_tensor l, tci_tensor q) try {
  if (!ctx || !a || !l || !q) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(a, k_rows, rows, cols));
  if (rows > cols) TCI_RET(TCI_ERR_UNSUPPORTED, "lq of a tall matrix (rows > cols) is not supported");
  Trace tr(ctx, "lq", std::to_string(rows) + "x" + std::to_string(cols));
  ctx->arena.reset();
  int wdt;
  const void* w;
  TCI_TRY(working_copy(ctx, a, wdt, w));
  const size_t es = elem_bytes(wdt);
  const int m = (int)rows, n = (int)cols;
  // A^H = Q1 R1 (n x m tall), so A = R1^H Q1^H: L = R1^H, Q = Q1^H
  void* Ah = ctx->arena.get(es * (size_t)m * n);
  if (!Ah) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_TRY(conj_transpose(ctx, wdt, w, m, n, Ah));
  void *Y, *R;
  TCI_TRY(qr_core(ctx, wdt, n, m, Ah, Y, R));
  void* Lw = ctx->arena.get(es * (size_t)m * m);
  void* Qw = ctx->arena.get(es * (size_t)m * n);
  if (!Lw || !Qw) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_TRY(conj_transpose(ctx, wdt, R, m, m, Lw));
  TCI_TRY(conj_transpose(ctx, wdt, Y, n, m, Qw));
  int64_t lshape[MAX_ORDER + 1], qshape[MAX_ORDER + 1];
  for (int i = 0; i < k_rows; ++i) lshape[i] = a->shape[i];
  lshape[k_rows] = m;
  qshape[0] = m;
  for (int i = k_rows; i < a->order; ++i) qshape[1 + i - k_rows] = a->shape[i];
  const int odt = a->dtype, ord = a->order;
  TCI_TRY(ensure_shape(ctx, l, odt, k_rows + 1, lshape));
  TCI_TRY(ensure_shape(ctx, q, odt, ord - k_rows + 1, qshape));
  TCI_TRY(store_as(ctx, wdt, Lw, l));
  TCI_TRY(store_as(ctx, wdt, Qw, q));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

// Matrix exponential by scaling and squaring with a Taylor polynomial, in
// FP64 for every dtype: B = A / 2^s with ||B||_F <= 1/2, exp(B) ~ sum_{j <= 18}
// B^j / j! by Horner's rule (P <- I + B P / j for j = 18 .. 1; truncation
// below 2^-19 / 19! ~ 1.6e-23 relative), then s squarings.
tci_status tci_exp(tci_context ctx, tci_tensor in, int k_rows, tci_tensor out) try {
  if (!ctx || !in || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(in, k_rows, rows, cols));
  if (rows != cols) TCI_RET(TCI_ERR_SHAPE, "exp needs equal row and column dimensions");
  Trace tr(ctx, "exp", std::to_string(rows) + "x" + std::to_string(cols));
  ctx->arena.reset();
  int wdt;
  const void* w;
  TCI_TRY(working_copy(ctx, in, wdt, w));
  const int n = (int)rows;
  const size_t es = elem_bytes(wdt);
  const size_t bytes = es * (size_t)n * n;
  hipStream_t st = ctx->stream;
  void* B = ctx->arena.get(bytes);
  void* P = ctx->arena.get(bytes);
  void* T = ctx->arena.get(bytes);
  double* nrm = static_cast<double*>(ctx->arena.get(sizeof(double) * (SUMSQ_PARTIALS + 1)));
  if (!B || !P || !T || !nrm) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(hipMemcpyAsync(B, w, bytes, hipMemcpyDeviceToDevice, st));
  TCI_CHECK_HIP(sumsq_batched(wdt, B, (long long)n * n, 0, nrm + SUMSQ_PARTIALS, nrm, 1, st));
  double fn2 = 0.0;
  TCI_CHECK_HIP(hipMemcpyAsync(&fn2, nrm + SUMSQ_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, st));
  TCI_CHECK_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(fn2)) TCI_RET(TCI_ERR_NUMERIC, "non-finite entries");
  const double fn = std::sqrt(fn2);
  int sq = 0;
  while (fn > 0.5 * std::ldexp(1.0, sq) && sq < 1100) ++sq;
  TCI_CHECK_HIP(scale_inplace(wdt, B, (long long)n * n, std::ldexp(1.0, -sq), 0.0, st));
  constexpr int TAYLOR_DEGREE = 18;
  TCI_CHECK_HIP(fill_value(wdt, P, (long long)n * n, 0.0, 0.0, st));
  TCI_CHECK_HIP(add_diag(wdt, P, n, n, 1.0, st));
  for (int j = TAYLOR_DEGREE; j >= 1; --j) {
    // T = B P / j, then P = I + T
    GemmArgs g = gemm_args(n, n, n, OP_N, OP_N, B, n, P, n, T, n);
    g.alpha_re = 1.0 / j;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, st));
    TCI_CHECK_HIP(add_diag(wdt, T, n, n, 1.0, st));
    std::swap(P, T);
  }
  for (int k = 0; k < sq; ++k) {
    GemmArgs g = gemm_args(n, n, n, OP_N, OP_N, P, n, P, n, T, n);
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, st));
    std::swap(P, T);
  }
  int64_t shape[MAX_ORDER];
  for (int i = 0; i < in->order; ++i) shape[i] = in->shape[i];
  const int odt = in->dtype, ord = in->order;
  TCI_TRY(ensure_shape(ctx, out, odt, ord, shape));
  TCI_TRY(store_as(ctx, wdt, P, out));
  TCI_CHECK_HIP(hipStreamSynchronize(st));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_inverse(tci_context ctx, tci_tensor in, int k_rows, tci_tensor out) try {
  if (!ctx || !in || !out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(in, k_rows, rows, cols));
  if (rows != cols) TCI_RET(TCI_ERR_SHAPE, "inverse needs equal row and column dimensions");
  if (rows > 65536) TCI_RET(TCI_ERR_UNSUPPORTED, "inverse of a matrix above 65536 x 65536");
  Trace tr(ctx, "inverse", std::to_string(rows) + "x" + std::to_string(cols));
  ctx->arena.reset();
  int wdt;
  const void* w;
  TCI_TRY(working_copy(ctx, in, wdt, w));
  const int n = (int)rows;
  const size_t es = elem_bytes(wdt);
  hipStream_t st = ctx->stream;
  void* work = ctx->arena.get(gauss_jordan_work_bytes(wdt, n));
  void* res = ctx->arena.get(es * (size_t)n * n);
  int* status = static_cast<int*>(ctx->arena.get(sizeof(int)));
  double* nrm = static_cast<double*>(ctx->arena.get(sizeof(double) * (SUMSQ_PARTIALS + 1)));
  if (!work || !res || !status || !nrm) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(hipMemsetAsync(status, 0, sizeof(int), st));
  TCI_CHECK_HIP(gauss_jordan_inverse(wdt, w, n, work, status, st));
  // the inverse is the right half of the n x 2n augmented matrix
  TCI_CHECK_HIP(hipMemcpy2DAsync(res, es * n, static_cast<char*>(work) + es * n, es * 2 * n, es * n, n,
                                 hipMemcpyDeviceToDevice, st));
  TCI_CHECK_HIP(sumsq_batched(wdt, res, (long long)n * n, 0, nrm + SUMSQ_PARTIALS, nrm, 1, st));
  int singular = 0;
  double fn2 = 0.0;
  TCI_CHECK_HIP(hipMemcpyAsync(&singular, status, sizeof(int), hipMemcpyDeviceToHost, st));
  TCI_CHECK_HIP(hipMemcpyAsync(&fn2, nrm + SUMSQ_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, st));
  TCI_CHECK_HIP(hipStreamSynchronize(st));
  if (singular) TCI_RET(TCI_ERR_NUMERIC, "singular matrix: no pivot in column " + std::to_string(singular - 1));
  if (!std::isfinite(fn2)) TCI_RET(TCI_ERR_NUMERIC, "non-finite entries");
  int64_t shape[MAX_ORDER];
  for (int i = 0; i < in->order; ++i) shape[i] = in->shape[i];
  const int odt = in->dtype, ord = in->order;
  TCI_TRY(ensure_shape(ctx, out, odt, ord, shape));
  TCI_TRY(store_as(ctx, wdt, res, out));
  TCI_CHECK_HIP(hipStreamSynchronize(st));
  return TCI_OK;
} TCI_API_CATCH

// Spec eigh / eigvalsh: Hermitian eigensolve of the matricised tensor in
// FP64 (single-precision inputs promoted); v == nullptr skips the vectors.
static tci_status eigh_core(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w, tci_tensor v) {
  if (!ctx || !a || !w) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  if (a->empty) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "moved-from tensor");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(a, k_rows, rows, cols));
  if (rows != cols) TCI_RET(TCI_ERR_SHAPE, "eigh needs a square matricisation (I == J)");
  Trace tr(ctx, v ? "eigh" : "eigvalsh", std::to_string(rows));
  ctx->arena.reset();
  const int n = (int)rows, odt = a->dtype;
  int dt;
  const void* src;
  TCI_TRY(working_copy(ctx, a, dt, src));
  const size_t es = elem_bytes(dt);
  hipStream_t s = ctx->stream;
  ARENA(G, char, es * (size_t)n * n);
  TCI_CHECK_HIP(hipMemcpyAsync(G, src, es * (size_t)n * n, hipMemcpyDeviceToDevice, s));
  ARENA(d, double, n);
  ARENA(e, double, n);
  ARENA(e2, double, n);
  ARENA(tau, char, es * n);
  ARENA(Vt, char, es * (size_t)n * n);
  ARENA(Wp, char, es * (size_t)n * TRIDIAG_NB);
  ARENA(y, char, es * n);
  TriArgs ta{};
  ta.n = n; ta.G = G; ta.ldg = n; ta.d = d; ta.e = e; ta.tau = tau; ta.Vt = Vt; ta.Wp = Wp; ta.y = y;
  ta.sws = (long long)tridiag_ws_bytes(dt, n);
  ta.ws = ctx->arena.get((size_t)ta.sws);
  if (!ta.ws) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(hipMemsetAsync(e, 0, sizeof(double) * n, s));
  TCI_CHECK_HIP(tridiagonalize(dt, ta, 1, s));
  ARENA(lam, double, n);
  TCI_CHECK_HIP(tridiag_eigvals_top(d, e, e2, n, n, n, lam, n, 1, s));
  void* Ev = nullptr;
  if (v) {
    ARENA(Z, double, (size_t)n * n);
    ARENA(Z2, double, (size_t)n * n);
    ARENA(iw, double, (size_t)4 * n * n);
    TCI_CHECK_HIP(hipMemsetAsync(Z, 0, sizeof(double) * (size_t)n * n, s));
    TCI_CHECK_HIP(tridiag_invit(d, e, n, n, lam, n, nullptr, n, Z, n, 0, iw, 1, s));
    TCI_TRY(cholqr2(ctx, F64, 0, Z, n, (long long)n * n, n, n, Z2, 1));
    Ev = Z;
    if (is_complex(dt)) {
      Ev = ctx->arena.get(es * (size_t)n * n);
      if (!Ev) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
      TCI_CHECK_HIP(real_to_complex(Z, Ev, (long long)n * n, 0, 0, 1, s));
    }
    const size_t tfe = tridiag_backtransform_tf_elems(n);
    ARENA(Tf, char, es * tfe);
    ARENA(btw, char, tridiag_backtransform_work_bytes(dt, n, 1));
    TCI_CHECK_HIP(tridiag_backtransform(dt, ta, Tf, (long long)tfe, Ev, n, 0, n, btw, 1, s));
    // ascending order: reverse the descending bisection order
    TCI_CHECK_HIP(reverse_columns(dt, Ev, n, n, n, s));
    TCI_CHECK_HIP(gauge_columns(dt, Ev, n, 0, n, n, nullptr, 1, s));
  }
  std::vector<double> lh(n);
  TCI_CHECK_HIP(hipMemcpyAsync(lh.data(), lam, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  std::reverse(lh.begin(), lh.end());
  for (double x : lh)
    if (!std::isfinite(x)) TCI_RET(TCI_ERR_NUMERIC, "non-finite eigenvalues (non-finite input?)");
  const int rdt = is_double(odt) ? F64 : F32;
  int64_t wshape[1] = {n};
  TCI_TRY(ensure_shape(ctx, w, rdt, 1, wshape));
  ARENA(wd, double, n);
  TCI_CHECK_HIP(hipMemcpyAsync(wd, lh.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  TCI_TRY(store_as(ctx, F64, wd, w));
  if (v) {
    int64_t vshape[MAX_ORDER + 1];
    for (int i = 0; i < k_rows; ++i) vshape[i] = a->shape[i];
    vshape[k_rows] = n;
    TCI_TRY(ensure_shape(ctx, v, odt, k_rows + 1, vshape));
    TCI_TRY(store_as(ctx, dt, Ev, v));
  }
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  return TCI_OK;
}

tci_status tci_eigh(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w, tci_tensor v) try {
  if (!v) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  return eigh_core(ctx, a, k_rows, w, v);
} TCI_API_CATCH

tci_status tci_eigvalsh(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w) try {
  return eigh_core(ctx, a, k_rows, w, nullptr);
} TCI_API_CATCH

// Spec eig / eigvals: general eigendecomposition of the matricised tensor in
// complex128 (geig.hip); v == nullptr skips the vectors.  Eigenvalues in
// ascending order of the real part, then of the imaginary part.
static tci_status eig_core(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w, tci_tensor v) {
  if (!ctx || !a || !w) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  if (a->empty) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "moved-from tensor");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int64_t rows, cols;
  TCI_TRY(matricize(a, k_rows, rows, cols));
  if (rows != cols) TCI_RET(TCI_ERR_SHAPE, "eig needs a square matricisation (I == J)");
  if (rows > GEIG_MAX_N)
    TCI_RET(TCI_ERR_UNSUPPORTED, "eig / eigvals: matrix order above " + std::to_string(GEIG_MAX_N));
  Trace tr(ctx, v ? "eig" : "eigvals", std::to_string(rows));
  ctx->arena.reset();
  const int n = (int)rows, odt = a->dtype;
  const int cdt = is_double(odt) ? C128 : C64;   // complex type of the input's precision
  if (n == 0) {
    int64_t z[MAX_ORDER + 1] = {0};
    TCI_TRY(ensure_shape(ctx, w, cdt, 1, z));
    if (v) {
      for (int i = 0; i < k_rows; ++i) z[i] = a->shape[i];
      z[k_rows] = 0;
      TCI_TRY(ensure_shape(ctx, v, cdt, k_rows + 1, z));
    }
    return TCI_OK;
  }
  hipStream_t s = ctx->stream;
  const size_t nn = (size_t)n * n;
  ARENA(H, cd, nn);
  ARENA(Q, cd, nn);
  ARENA(st, int, 1);
  ARENA(fro, double, 1);
  ARENA(wd, cd, n);
  TCI_CHECK_HIP(convert(odt, a->data, C128, H, (long long)nn, s));
  TCI_CHECK_HIP(geig_schur(H, Q, n, st, fro, s));
  TCI_CHECK_HIP(geig_diag(H, n, wd, s));
  int sth = 0;
  std::vector<cd> wh(n);
  TCI_CHECK_HIP(hipMemcpyAsync(&sth, st, sizeof(int), hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(wh.data(), wd, sizeof(cd) * n, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  if (sth) TCI_RET(TCI_ERR_NOT_CONVERGED, "eig: the QR iteration did not converge");
  for (const cd& x : wh)
    if (!std::isfinite(x.x) || !std::isfinite(x.y)) TCI_RET(TCI_ERR_NUMERIC, "non-finite eigenvalues (non-finite input?)");
  // order of the returned values: keys rounded to the output precision, so
  // that the order holds exactly for what the caller reads
  std::vector<double> kr(n), ki(n);
  for (int i = 0; i < n; ++i) {
    kr[i] = cdt == C64 ? (double)(float)wh[i].x : wh[i].x;
    ki[i] = cdt == C64 ? (double)(float)wh[i].y : wh[i].y;
  }
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
    return kr[x] < kr[y] || (kr[x] == kr[y] && ki[x] < ki[y]);
  });
  std::vector<cd> wo(n);
  for (int i = 0; i < n; ++i) wo[i] = wh[perm[i]];
  ARENA(w2, cd, n);
  TCI_CHECK_HIP(hipMemcpyAsync(w2, wo.data(), sizeof(cd) * n, hipMemcpyHostToDevice, s));
  int64_t wshape[1] = {n};
  TCI_TRY(ensure_shape(ctx, w, cdt, 1, wshape));
  TCI_TRY(store_as(ctx, C128, w2, w));
  if (v) {
    ARENA(X, cd, nn);
    ARENA(V, cd, nn);
    ARENA(Vo, cd, nn);
    ARENA(pd, int, n);
    TCI_CHECK_HIP(geig_triangular_vectors(H, X, n, fro, s));
    GemmArgs g = gemm_args(n, n, n, OP_N, OP_N, Q, n, X, n, V, n);
    TCI_CHECK_HIP(gemm(C128, PREC_FP64, g, s));
    TCI_CHECK_HIP(hipMemcpyAsync(pd, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    TCI_CHECK_HIP(geig_finish(V, pd, n, Vo, s));
    int64_t vshape[MAX_ORDER + 1];
    for (int i = 0; i < k_rows; ++i) vshape[i] = a->shape[i];
    vshape[k_rows] = n;
    TCI_TRY(ensure_shape(ctx, v, cdt, k_rows + 1, vshape));
    TCI_TRY(store_as(ctx, C128, Vo, v));
  }
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  return TCI_OK;
}

tci_status tci_eig(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w, tci_tensor v) try {
  if (!v) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  return eig_core(ctx, a, k_rows, w, v);
} TCI_API_CATCH

tci_status tci_eigvals(tci_context ctx, tci_tensor a, int k_rows, tci_tensor w) try {
  return eig_core(ctx, a, k_rows, w, nullptr);
} TCI_API_CATCH

// ----------------------------------------------------------------- two-site update
tci_status tci_two_site_update_batched(tci_context ctx, int nupd, const tci_tensor* A, const tci_tensor* B,
                                       const tci_tensor* gates, const tci_update_params* params,
                                       tci_tensor* A_out, tci_tensor* s_out, tci_tensor* B_out,
                                       tci_update_info* infos) try {
  if (!ctx || nupd < 1 || !A || !B || !A_out || !s_out || !B_out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  tci_update_params p;
  if (params) {
    p = *params;
  } else {
    tci_update_params_default(&p);
    p.svd_mode = ctx->svd_mode;
    if (A[0] && !is_double(A[0]->dtype)) p.precision = ctx->precision;
  }
  if (p.chi_min < 1 || p.chi_max < 1 || p.chi_min > p.chi_max) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need 1 <= chi_min <= chi_max");
  const tci_tensor a0 = A[0], b0 = B[0];
  if (!a0 || !b0 || a0->order != 3 || b0->order != 3) TCI_RET(TCI_ERR_SHAPE, "A and B must be order 3");
  const int dt = a0->dtype;
  const int64_t chil = a0->shape[0], d = a0->shape[1], chim = a0->shape[2], chir = b0->shape[2];
  if (b0->shape[0] != chim || b0->shape[1] != d) TCI_RET(TCI_ERR_SHAPE, "A and B bond mismatch");
  for (int i = 0; i < nupd; ++i) {
    if (!A[i] || !B[i] || !A_out[i] || !s_out[i] || !B_out[i]) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null tensor");
    if (A[i]->dtype != dt || B[i]->dtype != dt) TCI_RET(TCI_ERR_DTYPE, "mixed dtypes in the batch");
    for (int k = 0; k < 3; ++k)
      if (A[i]->shape[k] != a0->shape[k] || B[i]->shape[k] != b0->shape[k])
        TCI_RET(TCI_ERR_SHAPE, "all updates of a batch must have the same shapes");
    if (gates && gates[i]) {
      if (gates[i]->dtype != dt) TCI_RET(TCI_ERR_DTYPE, "gate dtype");
      if (tsize(gates[i]) != d * d * d * d) TCI_RET(TCI_ERR_SHAPE, "gate must have d^4 elements");
    }
  }
  if (gates && d != 2) TCI_RET(TCI_ERR_UNSUPPORTED, "gates are supported for d = 2");
  TCI_TRY(check_direction(ctx, p, nupd, chil, chir));
  const int prec = p.precision;
  if (is_double(dt) != (prec == TCI_PREC_FP64))
    TCI_RET(TCI_ERR_DTYPE, "FP64 precision needs F64/C128 tensors, mixed precisions F32/C64");
  Trace tr(ctx, "two_site_update_batched", std::to_string(nupd) + " x " + std::to_string(chil) + "," +
                                               std::to_string(d) + "," + std::to_string(chir));
  const int m = (int)(chil * d), n = (int)(d * chir), K = (int)chim;
  const int wdt = work_dtype(dt);
  const size_t es = elem_bytes(dt), wes = elem_bytes(wdt);
  hipStream_t s = ctx->stream;
  const int maxb = p.max_batch > 0 ? p.max_batch : 64;
  for (int c0 = 0; c0 < nupd; c0 += maxb) {
    const int nb = std::min(maxb, nupd - c0);
    ctx->arena.reset();
    // gather operands into strided batches
    const size_t szA = (size_t)chil * d * chim, szB = (size_t)chim * d * chir;
    ARENA(Ab, char, es * szA * nb);
    ARENA(Bb, char, es * szB * nb);
    for (int i = 0; i < nb; ++i) {
      TCI_CHECK_HIP(hipMemcpyAsync(Ab + es * szA * i, A[c0 + i]->data, es * szA, hipMemcpyDeviceToDevice, s));
      TCI_CHECK_HIP(hipMemcpyAsync(Bb + es * szB * i, B[c0 + i]->data, es * szB, hipMemcpyDeviceToDevice, s));
    }
    // theta = A . B  (contraction over the shared bond)
    const long long smn = (long long)m * n;
    ARENA(th, char, es * (size_t)smn * nb);
    if (prec == PREC_BF16X3) {
      // split-BF16x3: A and B split once into bf16 hi/lo planes, the batched
      // product runs on the planes
      const size_t pa = planes_bytes(dt, m, K), pb = planes_bytes(dt, n, K);
      ARENA(Ap, char, pa * nb);
      ARENA(Bp, char, pb * nb);
      TCI_CHECK_HIP(split_a(dt, OP_N, Ab, K, (long long)szA, m, K, Ap, nb, s));
      TCI_CHECK_HIP(split_b(dt, OP_N, Bb, n, (long long)szB, K, n, Bp, nb, s));
      PlaneGemmArgs pg{};
      pg.m = m; pg.n = n; pg.k = K;
      pg.Mp = pad_rows(m); pg.Np = pad_rows(n); pg.Kp = pad_k(K);
      pg.Ap = reinterpret_cast<const __bf16*>(Ap); pg.sAp = (long long)(pa / sizeof(__bf16));
      pg.Bp = reinterpret_cast<const __bf16*>(Bp); pg.sBp = (long long)(pb / sizeof(__bf16));
      pg.C = th; pg.ldc = n; pg.sC = smn;
      pg.alpha_re = 1.0;
      pg.batch = nb;
      ProfTag tag("theta");
      TCI_CHECK_HIP(gemm_planes(dt, pg, s));
    } else {
      GemmArgs g = gemm_args(m, n, K, OP_N, OP_N, Ab, K, Bb, n, th, n);
      g.sA = (long long)szA; g.sB = (long long)szB; g.sC = smn; g.batch = nb;
      ProfTag tag("theta");
      TCI_CHECK_HIP(gemm(dt, prec, g, s));
    }
    // gate
    if (gates) {
      const int g2 = (int)(d * d * d * d);
      ARENA(Gb, char, es * (size_t)g2 * nb);
      std::vector<double> eye(2 * 16, 0.0);
      for (int i = 0; i < nb; ++i) {
        if (gates[c0 + i]) {
          TCI_CHECK_HIP(hipMemcpyAsync(Gb + es * g2 * i, gates[c0 + i]->data, es * g2, hipMemcpyDeviceToDevice, s));
        } else {
          // identity in the batch's dtype
          std::vector<char> host(es * g2, 0);
          for (int q = 0; q < 4; ++q) {
            char* p0 = host.data() + es * (q * 4 + q);
            if (dt == C128 || dt == F64) { const double one = 1.0; std::memcpy(p0, &one, 8); }
            else { const float one = 1.0f; std::memcpy(p0, &one, 4); }
          }
          TCI_CHECK_HIP(hipMemcpy(Gb + es * g2 * i, host.data(), es * g2, hipMemcpyHostToDevice));
        }
      }
      TCI_CHECK_HIP(gate_apply(dt, th, smn, Gb, g2, (int)chil, (int)d, (int)chir, nb, s));
    }
    // FP64 working copy for the decomposition
    const void* thw = th;
    if (wdt != dt) {
      ARENA(tw, char, wes * (size_t)smn * nb);
      TCI_CHECK_HIP(convert(dt, th, wdt, tw, smn * nb, s));
      thw = tw;
    }
    tci_update_params pc = p;  // Vidal weights indexed like the outputs of this chunk
    if (pc.lambda_left) pc.lambda_left += c0;
    if (pc.lambda_right) pc.lambda_right += c0;
    TCI_TRY(split_and_store(ctx, dt, wdt, nb, (int)chil, (int)d, (int)chir, th, thw, pc, c0, A_out + c0,
                            s_out + c0, B_out + c0, infos ? infos + c0 : nullptr));
    TCI_CHECK_HIP(hipStreamSynchronize(s));
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_two_site_update(tci_context ctx, tci_tensor A, tci_tensor B, tci_tensor gate,
                               const tci_update_params* params, tci_tensor A_out, tci_tensor s_out, tci_tensor B_out,
                               tci_update_info* info) try {
  return tci_two_site_update_batched(ctx, 1, &A, &B, gate ? &gate : nullptr, params, &A_out, &s_out, &B_out, info);
} TCI_API_CATCH

tci_status tci_split_batched(tci_context ctx, int nupd, const tci_tensor* theta, const tci_update_params* params,
                             tci_tensor* A_out, tci_tensor* s_out, tci_tensor* B_out, tci_update_info* infos) try {
  if (!ctx || nupd < 1 || !theta || !A_out || !s_out || !B_out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  tci_update_params p;
  if (params) {
    p = *params;
  } else {
    tci_update_params_default(&p);
    p.svd_mode = ctx->svd_mode;
  }
  if (p.chi_min < 1 || p.chi_max < 1 || p.chi_min > p.chi_max) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need 1 <= chi_min <= chi_max");
  const tci_tensor t0 = theta[0];
  if (!t0 || t0->order != 4) TCI_RET(TCI_ERR_SHAPE, "theta must be order 4 (chi_l, d, d, chi_r)");
  const int dt = t0->dtype;
  const int64_t chil = t0->shape[0], d = t0->shape[1], chir = t0->shape[3];
  if (t0->shape[2] != d) TCI_RET(TCI_ERR_SHAPE, "theta physical dimensions differ");
  for (int i = 0; i < nupd; ++i) {
    if (!theta[i] || !A_out[i] || !s_out[i] || !B_out[i]) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null tensor");
    if (theta[i]->dtype != dt || theta[i]->order != 4) TCI_RET(TCI_ERR_DTYPE, "mixed dtypes in the batch");
    for (int k = 0; k < 4; ++k)
      if (theta[i]->shape[k] != t0->shape[k]) TCI_RET(TCI_ERR_SHAPE, "all thetas of a batch must have one shape");
  }
  TCI_TRY(check_direction(ctx, p, nupd, chil, chir));
  Trace tr(ctx, "split_batched", std::to_string(nupd) + " x " + std::to_string(chil) + "," + std::to_string(chir));
  const int wdt = work_dtype(dt);
  const size_t es = elem_bytes(dt), wes = elem_bytes(wdt);
  const long long smn = (long long)chil * d * d * chir;
  hipStream_t s = ctx->stream;
  const int maxb = p.max_batch > 0 ? p.max_batch : 64;
  for (int c0 = 0; c0 < nupd; c0 += maxb) {
    const int nb = std::min(maxb, nupd - c0);
    ctx->arena.reset();
    ARENA(tl, char, es * (size_t)smn * nb);
    for (int i = 0; i < nb; ++i)
      TCI_CHECK_HIP(hipMemcpyAsync(tl + es * smn * i, theta[c0 + i]->data, es * smn, hipMemcpyDeviceToDevice, s));
    const void* tw = tl;
    if (wdt != dt) {
      ARENA(t64, char, wes * (size_t)smn * nb);
      TCI_CHECK_HIP(convert(dt, tl, wdt, t64, smn * nb, s));
      tw = t64;
    }
    tci_update_params pc = p;
    if (pc.lambda_left) pc.lambda_left += c0;
    if (pc.lambda_right) pc.lambda_right += c0;
    TCI_TRY(split_and_store(ctx, dt, wdt, nb, (int)chil, (int)d, (int)chir, tl, tw, pc, c0, A_out + c0, s_out + c0,
                            B_out + c0, infos ? infos + c0 : nullptr));
  }
  return TCI_OK;
} TCI_API_CATCH

}  // extern "C"
