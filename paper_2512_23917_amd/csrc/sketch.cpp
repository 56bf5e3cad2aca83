// Randomized truncated SVD with plain fallback, and its learned sketch rank.
//
// Range finder with q power iterations (Halko, Martinsson, Tropp, SIAM Rev. 53,
// 2011, Alg. 4.4): every product with theta runs in the contraction precision
// (FP32 or split-BF16x3 on complex64 storage, or FP64), every
// orthonormalisation is FP64 Cholesky-QR2 with column dropping; then
// B = Q^H theta, the FP64 eigensolve of the small Gram matrix B B^H, the
// truncation rule of trunc_svd with the error measured against the exact
// ||theta||_F^2, U = Q W, V^H = diag(1/s) U^H theta (FP64, rows re-
// orthonormalised) and the residual certificate r_j = ||theta v_j - s_j u_j||.
// A problem is accepted when eps <= target and max_j r_j <= cert * s_1;
// otherwise the plain truncated SVD decides it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "common.hpp"
#include "eig.hpp"
#include "gemm.hpp"
#include "linalg.hpp"
#include "prof.hpp"
#include "runtime.hpp"
#include "sketch_kernels.hpp"
#include "tsvd.hpp"
#include "vecops.hpp"

namespace tci {

#define SK_ARENA(ptr, type, count)                                                     \
  type* ptr = static_cast<type*>(ctx->arena.get(sizeof(type) * (size_t)(count)));      \
  if (!ptr) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace allocation failed: " #ptr)

static tci_status ortho2(tci_context ctx, int wdt, void* X, long long ld, long long sX, int m, int k, int nb,
                             void* kws) {
  const size_t es = elem_bytes(wdt);
  void* tmp = ctx->arena.get(es * (size_t)sX * nb);
  CholWork w{};
  w.G = ctx->arena.get(es * cholqr_work_elems(k) * nb);
  w.diag0 = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  w.mask = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  if (!tmp || !w.G || !w.diag0 || !w.mask) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "cholqr workspace");
  w.RI = static_cast<char*>(w.G) + es * (size_t)k * k * nb;
  w.kws = kws;
  w.kws_bytes = kws ? GEMM_SPLITK_WS_BYTES : 0;
  TCI_CHECK_HIP(cholqr(wdt, 0, X, ld, sX, m, k, tmp, ld, sX, w, 1e-12, nb, ctx->stream));
  TCI_CHECK_HIP(cholqr(wdt, 0, tmp, ld, sX, m, k, X, ld, sX, w, 1e-12, nb, ctx->stream));
  return TCI_OK;
}

// One Cholesky-QR pass: enough between the power steps of the range finder,
// where the block only has to stay well conditioned (orthogonality error
// about u cond(X)^2); the range that the last step hands on is
// orthonormalised by ortho2.
static tci_status ortho1(tci_context ctx, int wdt, void* X, long long ld, long long sX, int m, int k, int nb,
                             void* kws) {
  const size_t es = elem_bytes(wdt);
  void* tmp = ctx->arena.get(es * (size_t)sX * nb);
  CholWork w{};
  w.G = ctx->arena.get(es * cholqr_work_elems(k) * nb);
  w.diag0 = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  w.mask = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  if (!tmp || !w.G || !w.diag0 || !w.mask) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "cholqr workspace");
  w.RI = static_cast<char*>(w.G) + es * (size_t)k * k * nb;
  w.kws = kws;
  w.kws_bytes = kws ? GEMM_SPLITK_WS_BYTES : 0;
  TCI_CHECK_HIP(cholqr(wdt, 0, X, ld, sX, m, k, tmp, ld, sX, w, 1e-12, nb, ctx->stream));
  TCI_CHECK_HIP(hipMemcpyAsync(X, tmp, es * (size_t)sX * nb, hipMemcpyDeviceToDevice, ctx->stream));
  return TCI_OK;
}

static tci_status row_ortho2(tci_context ctx, int wdt, void* X, long long ld, long long sX, int m, int k, int nb,
                             void* kws) {
  const size_t es = elem_bytes(wdt);
  void* tmp = ctx->arena.get(es * (size_t)sX * nb);
  CholWork w{};
  w.G = ctx->arena.get(es * cholqr_work_elems(k) * nb);
  w.diag0 = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  w.mask = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)k * nb));
  if (!tmp || !w.G || !w.diag0 || !w.mask) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "cholqr workspace");
  w.RI = static_cast<char*>(w.G) + es * (size_t)k * k * nb;
  w.kws = kws;
  w.kws_bytes = kws ? GEMM_SPLITK_WS_BYTES : 0;
  TCI_CHECK_HIP(cholqr(wdt, 1, X, ld, sX, m, k, tmp, ld, sX, w, 1e-12, nb, ctx->stream));
  TCI_CHECK_HIP(cholqr(wdt, 1, tmp, ld, sX, m, k, X, ld, sX, w, 1e-12, nb, ctx->stream));
  return TCI_OK;
}

// th_lo: nb x m x n in dt_lo (the contraction precision's storage);
// th64: the same in wdt (FP64 working type; may equal th_lo).
tci_status sketch_run(tci_context ctx, int dt_lo, int wdt, int prec, int nb, int m, int n, const void* th_lo,
                      const void* th64, const TruncParams& tp, const std::vector<int>& kvec, int q, uint64_t seed,
                      const std::vector<uint32_t>& streams, TsvdOut& out, std::vector<double>& resid_h) {
  ProfTag tag("sketch");
  hipStream_t s = ctx->stream;
  const size_t el = elem_bytes(dt_lo), ew = elem_bytes(wdt);
  const long long smn = (long long)m * n;
  int kmax = 1;
  for (int k : kvec) kmax = std::max(kmax, k);
  kmax = std::min(kmax, std::min(m, n));
  const int kk = std::max(1, std::min(tp.chi_max, kmax));
  out.kmax = kk;
  auto lo_from = [&](const void* src, void* dst, long long cnt) -> hipError_t {
    return dt_lo == wdt ? hipMemcpyAsync(dst, src, ew * cnt, hipMemcpyDeviceToDevice, s)
                        : convert(wdt, src, dt_lo, dst, cnt, s);
  };
  auto w_from = [&](const void* src, void* dst, long long cnt) -> hipError_t {
    return dt_lo == wdt ? hipMemcpyAsync(dst, src, ew * cnt, hipMemcpyDeviceToDevice, s)
                        : convert(dt_lo, src, wdt, dst, cnt, s);
  };
  SK_ARENA(total, double, nb);
  SK_ARENA(partial, double, (size_t)nb * SUMSQ_PARTIALS);
  TCI_CHECK_HIP(sumsq_batched(wdt, th64, smn, smn, total, partial, nb, s));
  SK_ARENA(kws, char, GEMM_SPLITK_WS_BYTES);   // split-K scratch of the FP64 products
  SK_ARENA(kdev, int, nb);
  SK_ARENA(sdev, uint32_t, nb);
  std::vector<int> kc(nb);
  for (int b = 0; b < nb; ++b) kc[b] = std::min(kvec[b], kmax);
  TCI_CHECK_HIP(hipMemcpyAsync(kdev, kc.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
  TCI_CHECK_HIP(hipMemcpyAsync(sdev, streams.data(), sizeof(uint32_t) * nb, hipMemcpyHostToDevice, s));
  // sketch and range finder
  const long long sY = (long long)m * kmax, sZ = (long long)n * kmax;
  SK_ARENA(Om, char, el * (size_t)sZ * nb);
  TCI_CHECK_HIP(sketch_fill(dt_lo, Om, kmax, sZ, n, kdev, kmax, seed, sdev, nb, s));
  SK_ARENA(Ylo, char, el * (size_t)sY * nb);
  SK_ARENA(Y64, char, ew * (size_t)sY * nb);
  SK_ARENA(Zlo, char, el * (size_t)sZ * nb);
  SK_ARENA(Z64, char, ew * (size_t)sZ * nb);
  {
    GemmArgs g = gemm_args(m, kmax, n, OP_N, OP_N, th_lo, n, Om, kmax, Ylo, kmax);
    g.sA = smn; g.sB = sZ; g.sC = sY; g.batch = nb;
    TCI_CHECK_HIP(gemm(dt_lo, prec, g, s));
  }
  TCI_CHECK_HIP(w_from(Ylo, Y64, sY * nb));
  if (q > 0) TCI_TRY(ortho1(ctx, wdt, Y64, kmax, sY, m, kmax, nb, kws));
  else TCI_TRY(ortho2(ctx, wdt, Y64, kmax, sY, m, kmax, nb, kws));
  // Power iterations in the contraction precision; the last product with
  // theta, and B = Q^H theta, in FP64 so that the Rayleigh-Ritz step sees the
  // sketched subspace without the rounding of the mixed products.
  for (int it = 0; it < q; ++it) {
    TCI_CHECK_HIP(lo_from(Y64, Ylo, sY * nb));
    GemmArgs g1 = gemm_args(n, kmax, m, OP_C, OP_N, th_lo, n, Ylo, kmax, Zlo, kmax);
    g1.sA = smn; g1.sB = sY; g1.sC = sZ; g1.batch = nb;
    TCI_CHECK_HIP(gemm(dt_lo, prec, g1, s));
    TCI_CHECK_HIP(w_from(Zlo, Z64, sZ * nb));
    TCI_TRY(ortho1(ctx, wdt, Z64, kmax, sZ, n, kmax, nb, kws));
    if (it + 1 < q) {
      TCI_CHECK_HIP(lo_from(Z64, Zlo, sZ * nb));
      GemmArgs g2 = gemm_args(m, kmax, n, OP_N, OP_N, th_lo, n, Zlo, kmax, Ylo, kmax);
      g2.sA = smn; g2.sB = sZ; g2.sC = sY; g2.batch = nb;
      TCI_CHECK_HIP(gemm(dt_lo, prec, g2, s));
      TCI_CHECK_HIP(w_from(Ylo, Y64, sY * nb));
      TCI_TRY(ortho1(ctx, wdt, Y64, kmax, sY, m, kmax, nb, kws));
    } else {
      GemmArgs g2 = gemm_args(m, kmax, n, OP_N, OP_N, th64, n, Z64, kmax, Y64, kmax);
      g2.sA = smn; g2.sB = sZ; g2.sC = sY; g2.batch = nb;
      g2.kws = kws; g2.kws_bytes = GEMM_SPLITK_WS_BYTES;
      TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g2, s));
      TCI_TRY(ortho2(ctx, wdt, Y64, kmax, sY, m, kmax, nb, kws));
    }
  }
  // B = Q^H theta (FP64), Gram B B^H (FP64)
  const long long sB = (long long)kmax * n;
  SK_ARENA(B64, char, ew * (size_t)sB * nb);
  {
    GemmArgs g = gemm_args(kmax, n, m, OP_C, OP_N, Y64, kmax, th64, n, B64, n);
    g.sA = sY; g.sB = smn; g.sC = sB; g.batch = nb;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  const long long sG = (long long)kmax * kmax;
  SK_ARENA(Gk, char, ew * (size_t)sG * nb);
  {
    GemmArgs g = gemm_args(kmax, kmax, n, OP_N, OP_C, B64, n, B64, n, Gk, kmax);
    g.sA = sB; g.sB = sB; g.sC = sG; g.batch = nb;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  // small FP64 eigensolve
  const int ng = kmax;
  SK_ARENA(d, double, (size_t)ng * nb);
  SK_ARENA(e, double, (size_t)ng * nb);
  SK_ARENA(e2, double, (size_t)ng * nb);
  SK_ARENA(tau, char, ew * (size_t)ng * nb);
  SK_ARENA(Vt, char, ew * (size_t)sG * nb);
  SK_ARENA(Wp, char, ew * (size_t)ng * TRIDIAG_NB * nb);
  SK_ARENA(yv, char, ew * (size_t)ng * nb);
  TriArgs ta{};
  ta.n = ng; ta.G = Gk; ta.ldg = ng; ta.sG = sG; ta.d = d; ta.e = e; ta.sde = ng; ta.tau = tau; ta.stau = ng;
  ta.Vt = Vt; ta.sVt = sG; ta.Wp = Wp; ta.sWp = (long long)ng * TRIDIAG_NB; ta.y = yv; ta.sy = ng;
  ta.sws = (long long)tridiag_ws_bytes(wdt, ng);
  ta.ws = ctx->arena.get((size_t)ta.sws * nb);
  if (!ta.ws) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(hipMemsetAsync(e, 0, sizeof(double) * (size_t)ng * nb, s));
  TCI_CHECK_HIP(tridiagonalize(wdt, ta, nb, s));
  SK_ARENA(lam, double, (size_t)kk * nb);
  TCI_CHECK_HIP(tridiag_eigvals_top(d, e, e2, ng, ng, kk, lam, kk, nb, s));
  SK_ARENA(chi, int, nb);
  SK_ARENA(err, double, nb);
  SK_ARENA(disc, double, nb);
  SK_ARENA(sv, double, (size_t)kk * nb);
  SK_ARENA(sinv, double, (size_t)kk * nb);
  SK_ARENA(sn, double, (size_t)kk * nb);
  TCI_CHECK_HIP(trunc_select(lam, kk, kk, total, tp, chi, err, disc, sv, sinv, sn, kk, nb, s));
  out.chi = chi; out.s = sv; out.sn = sn; out.total = total;
  out.chi_h.resize(nb); out.err_h.resize(nb); out.disc_h.resize(nb); out.total_h.resize(nb);
  TCI_CHECK_HIP(hipMemcpyAsync(out.chi_h.data(), chi, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.err_h.data(), err, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.disc_h.data(), disc, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(out.total_h.data(), total, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  int kz = 1;
  for (int b = 0; b < nb; ++b) kz = std::max(kz, out.chi_h[b]);
  out.kz = kz;
  // eigenvectors W (kmax x kz)
  const long long sW = (long long)ng * kz;
  SK_ARENA(Zr, double, (size_t)sW * nb);
  SK_ARENA(Zr2, double, (size_t)sW * nb);
  SK_ARENA(iw, double, (size_t)4 * sW * nb);
  TCI_CHECK_HIP(hipMemsetAsync(Zr, 0, sizeof(double) * (size_t)sW * nb, s));
  TCI_CHECK_HIP(tridiag_invit(d, e, ng, ng, lam, kk, chi, kz, Zr, kz, sW, iw, nb, s));
  {
    CholWork w{};
    w.G = ctx->arena.get(sizeof(double) * cholqr_work_elems(kz) * nb);
    w.diag0 = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)kz * nb));
    w.mask = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)kz * nb));
    if (!w.G || !w.diag0 || !w.mask) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    w.RI = static_cast<char*>(w.G) + sizeof(double) * (size_t)kz * kz * nb;
    w.kws = kws;
    w.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(cholqr(F64, 0, Zr, kz, sW, ng, kz, Zr2, kz, sW, w, 1e-12, nb, s));
    TCI_CHECK_HIP(cholqr(F64, 0, Zr2, kz, sW, ng, kz, Zr, kz, sW, w, 1e-12, nb, s));
  }
  void* Wv = Zr;
  if (is_complex(wdt)) {
    Wv = ctx->arena.get(ew * (size_t)sW * nb);
    if (!Wv) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
    TCI_CHECK_HIP(real_to_complex(Zr, Wv, sW, sW, sW, nb, s));
  }
  const size_t tfe = tridiag_backtransform_tf_elems(ng);
  SK_ARENA(Tf, char, ew * tfe * nb);
  SK_ARENA(btw, char, tridiag_backtransform_work_bytes(wdt, kz, nb));
  TCI_CHECK_HIP(tridiag_backtransform(wdt, ta, Tf, (long long)tfe, Wv, kz, sW, kz, btw, nb, s));
  // U = Q W, gauge, V^H = diag(1/s) U^H theta (rows re-orthonormalised)
  const long long sU = (long long)m * kz, sV = (long long)kz * n;
  void* U = ctx->arena.get(ew * (size_t)sU * nb);
  void* Vh = ctx->arena.get(ew * (size_t)sV * nb);
  void* P = ctx->arena.get(ew * (size_t)sU * nb);
  if (!U || !Vh || !P) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  {
    GemmArgs g = gemm_args(m, kz, kmax, OP_N, OP_N, Y64, kmax, Wv, kz, U, kz);
    g.sA = sY; g.sB = sW; g.sC = sU; g.batch = nb;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  TCI_CHECK_HIP(gauge_columns(wdt, U, kz, sU, m, kz, chi, nb, s));
  {
    GemmArgs g = gemm_args(kz, n, m, OP_C, OP_N, U, kz, th64, n, Vh, n);
    g.sA = sU; g.sB = smn; g.sC = sV; g.batch = nb;
    g.rs = sinv; g.s_rs = kk;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  TCI_TRY(row_ortho2(ctx, wdt, Vh, n, sV, n, kz, nb, kws));
  // residual certificate: P = theta V, r_j = || P_j - s_j U_j ||
  {
    GemmArgs g = gemm_args(m, kz, n, OP_N, OP_C, th64, n, Vh, n, P, kz);
    g.sA = smn; g.sB = sV; g.sC = sU; g.batch = nb;
    g.kws = kws; g.kws_bytes = GEMM_SPLITK_WS_BYTES;
    TCI_CHECK_HIP(gemm(wdt, PREC_FP64, g, s));
  }
  SK_ARENA(rr, double, (size_t)kk * nb);
  TCI_CHECK_HIP(hipMemsetAsync(rr, 0, sizeof(double) * (size_t)kk * nb, s));
  TCI_CHECK_HIP(residual_norms(wdt, P, U, kz, sU, m, kz, sv, kk, chi, rr, nb, s));
  std::vector<double> rh((size_t)kk * nb), s0(nb);
  TCI_CHECK_HIP(hipMemcpyAsync(rh.data(), rr, sizeof(double) * rh.size(), hipMemcpyDeviceToHost, s));
  for (int b = 0; b < nb; ++b)
    TCI_CHECK_HIP(hipMemcpyAsync(&s0[b], sv + (size_t)kk * b, sizeof(double), hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  resid_h.assign(nb, 0.0);
  for (int b = 0; b < nb; ++b) {
    double mx = 0.0;
    for (int j = 0; j < out.chi_h[b]; ++j) mx = std::max(mx, rh[(size_t)kk * b + j]);
    resid_h[b] = s0[b] > 0.0 ? mx / s0[b] : 0.0;
  }
  out.U = U;
  out.Vh = Vh;
  return TCI_OK;
}

}  // namespace tci

namespace tci {

int sketch_model_nparams();
tci_status sketch_predict_dev(tci_context ctx, tci_sketch_model m, const float* X, int n, float* y);
tci_status sketch_features_dev(tci_context ctx, const double* s, long long ss, const int* len, int chi_max, int d,
                               double eps, float* X, int n);

// Sketch rank of the model's prediction y = log2 chi*:
// k = 32 ceil((1.5 * 2^y + 32) / 32); 0 (plain SVD) when y > log2 chi_max or
// when k > n / 4.  The range finder's orthonormalisations cost O(n k^2) in
// FP64 and its products O(n^2 k); measured on 2048 x 2048 complex bonds, a
// sketch of rank n / 3 already costs about as much as the plain SVD.
static int rank_from_prediction(double y, int ng, int chi_max) {
  if (!(y <= std::log2((double)chi_max))) return 0;
  const double want = std::pow(2.0, y) * 1.5 + 32.0;
  const int k = 32 * (int)std::ceil(want / 32.0);
  if (4 * k > ng) return 0;
  return k;
}

tci_status choose_sketch_ranks(tci_context ctx, const tci_update_params& p, int nb, int first, int ng, int chi_max,
                               int d, std::vector<int>& kvec) {
  kvec.assign(nb, 0);
  if (p.svd_mode == TCI_SVD_RANDOMIZED) {
    const int k = p.sketch_rank > 0 ? p.sketch_rank : std::min(ng, chi_max + 64);
    for (int i = 0; i < nb; ++i) kvec[i] = std::min(k, ng);
    return TCI_OK;
  }
  if (p.svd_mode != TCI_SVD_LEARNED) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "unknown svd_mode");
  if (!p.sketch_model) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "TCI_SVD_LEARNED needs params.sketch_model");
  if (!p.prev_spectra) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "TCI_SVD_LEARNED needs params.prev_spectra");
  if (!(p.target_trunc_err > 0.0)) {
    // eps = 0 keeps everything up to chi_max: nothing to predict
    for (int i = 0; i < nb; ++i) kvec[i] = 0;
    return TCI_OK;
  }
  hipStream_t s = ctx->stream;
  int lmax = 1;
  for (int i = 0; i < nb; ++i) {
    const tci_tensor t = p.prev_spectra[first + i];
    if (!t || t->order != 1 || t->dtype != TCI_F64) TCI_RET(TCI_ERR_DTYPE, "prev_spectra must be F64 vectors");
    lmax = std::max<int>(lmax, (int)t->shape[0]);
  }
  double* sp = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)lmax * nb));
  int* len = static_cast<int*>(ctx->arena.get(sizeof(int) * nb));
  float* X = static_cast<float*>(ctx->arena.get(sizeof(float) * 35 * (size_t)nb));
  float* y = static_cast<float*>(ctx->arena.get(sizeof(float) * nb));
  if (!sp || !len || !X || !y) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  std::vector<int> lh(nb);
  for (int i = 0; i < nb; ++i) {
    const tci_tensor t = p.prev_spectra[first + i];
    lh[i] = (int)t->shape[0];
    if (lh[i] > 0)
      TCI_CHECK_HIP(hipMemcpyAsync(sp + (size_t)lmax * i, t->data, sizeof(double) * lh[i], hipMemcpyDeviceToDevice, s));
  }
  TCI_CHECK_HIP(hipMemcpyAsync(len, lh.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
  TCI_TRY(sketch_features_dev(ctx, sp, lmax, len, chi_max, d, p.target_trunc_err, X, nb));
  TCI_TRY(sketch_predict_dev(ctx, static_cast<tci_sketch_model>(p.sketch_model), X, nb, y));
  std::vector<float> yh(nb);
  TCI_CHECK_HIP(hipMemcpyAsync(yh.data(), y, sizeof(float) * nb, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < nb; ++i) kvec[i] = rank_from_prediction(yh[i], ng, chi_max);
  return TCI_OK;
}

}  // namespace tci

extern "C" tci_status tci_philox_blocks(tci_context ctx, uint64_t seed, uint32_t stream, uint64_t first, int64_t n,
                                        uint32_t* out) try {
  if (!ctx || !out || n < 0) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  if (n == 0) return TCI_OK;
  TCI_CHECK_HIP(tci::philox_blocks(seed, stream, first, n, out, ctx->stream));
  return TCI_OK;
} TCI_API_CATCH
