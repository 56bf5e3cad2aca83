// Two-site DMRG pieces: the effective-Hamiltonian matvec and the Lanczos
// ground-state step.  The matvec is three matrix-core GEMMs:
//   X1[(a,w),(s1',s2',b')]  = sum_a'   L[(a,w),a'] x[a',(s1',s2',b')]
//   X2[a][(s1,s2,w''),b']   = sum_{w,s1',s2'} W12[(w,s1',s2'),(s1,s2,w'')] X1[a][(w,s1',s2'),b']
//   y[(a,s1,s2),b]          = sum_{w'',b'} X2[(a,s1,s2),(w'',b')] R[b,(w'',b')]
// with W12 = sum_w' W1[w,w',s1,s1'] W2[w',w'',s2,s2'] formed once per call.
// In the split-BF16x3 precision the environments are split into bf16 planes
// once per call; x and X2 are split once per matvec, and the two large
// products run on the pre-split planes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "common.hpp"
#include "eig.hpp"
#include "bf16x3.hpp"
#include "gemm.hpp"
#include "linalg.hpp"
#include "runtime.hpp"
#include "vecops.hpp"
#include "prof.hpp"

namespace tci {

struct HeffPlan {
  int dt, prec;
  int chil, chir, w, d;
  const void *L, *R;
  void* W12;  // (w d d) x (d d w)
  void* X1;   // chil * w * d * d * chir
  void* X2;   // chil * d * d * w * chir
  bool planes;               // split-BF16x3 on pre-split planes
  void *Lp, *Rp, *Xp, *X2p;  // planes of L', R', x', X2'
};

static tci_status heff_check(tci_tensor L, tci_tensor W1, tci_tensor W2, tci_tensor R, tci_tensor x, int& chil,
                             int& chir, int& wd, int& d) {
  for (tci_tensor t : {L, W1, W2, R, x})
    if (!t || t->empty) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null tensor");
  if (L->order != 3 || W1->order != 4 || W2->order != 4 || R->order != 3 || x->order != 4)
    TCI_RET(TCI_ERR_SHAPE, "heff operand orders must be 3, 4, 4, 3, 4");
  const int dt = L->dtype;
  for (tci_tensor t : {W1, W2, R, x})
    if (t->dtype != dt) TCI_RET(TCI_ERR_DTYPE, "heff operands must share one dtype");
  chil = (int)L->shape[0];
  wd = (int)L->shape[1];
  d = (int)W1->shape[2];
  chir = (int)R->shape[0];
  if (L->shape[2] != chil || R->shape[2] != chir || R->shape[1] != wd) TCI_RET(TCI_ERR_SHAPE, "environment shapes");
  for (tci_tensor t : {W1, W2})
    if (t->shape[0] != wd || t->shape[1] != wd || t->shape[2] != d || t->shape[3] != d)
      TCI_RET(TCI_ERR_SHAPE, "MPO shapes");
  if (x->shape[0] != chil || x->shape[1] != d || x->shape[2] != d || x->shape[3] != chir)
    TCI_RET(TCI_ERR_SHAPE, "theta shape");
  return TCI_OK;
}

// Bump allocation inside a caller-provided device region (the fixed scratch
// of the allocation-free matvec); regions are 256-byte aligned like the arena's.
struct Bump {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (!base || bytes > cap - used) return nullptr;
    void* p = base + used;
    used += bytes;
    return p;
  }
};

static size_t round256(size_t b) { return b == 0 ? 256 : (b + 255) & ~size_t(255); }

// Device bytes that heff_prepare takes for these shapes (W12, X1, X2 and, in
// the split-BF16x3 precision, the four operand plane sets).
static size_t heff_workspace_bytes(int dt, int prec, int chil, int chir, int wd, int d) {
  const size_t es = elem_bytes(dt);
  const int kw = wd * d * d, dd = d * d;
  size_t b = round256(es * (size_t)kw * kw) + 2 * round256(es * (size_t)chil * kw * chir);
  if ((dt == C64 || dt == F32) && prec == PREC_BF16X3)
    b += round256(planes_bytes(dt, chil * wd, chil)) + round256(planes_bytes(dt, chir, wd * chir)) +
         round256(planes_bytes(dt, dd * chir, chil)) + round256(planes_bytes(dt, chil * dd, wd * chir));
  return b;
}

// ws == nullptr: workspace from the context's arena; otherwise from ws.
static tci_status heff_prepare(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2, tci_tensor R, int chil,
                               int chir, int wd, int d, HeffPlan& p, Bump* ws = nullptr) {
  auto get = [&](size_t bytes) -> void* { return ws ? ws->get(bytes) : ctx->arena.get(bytes); };
  p.dt = L->dtype;
  p.prec = is_double(p.dt) ? PREC_FP64 : ctx->precision;
  p.chil = chil; p.chir = chir; p.w = wd; p.d = d;
  p.L = L->data; p.R = R->data;
  const size_t es = elem_bytes(p.dt);
  const int kw = wd * d * d;
  p.W12 = get(es * (size_t)kw * kw);
  p.X1 = get(es * (size_t)chil * kw * chir);
  p.X2 = get(es * (size_t)chil * kw * chir);
  if (!p.W12 || !p.X1 || !p.X2) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "heff workspace");
  TCI_CHECK_HIP(mpo_pair(p.dt, W1->data, W2->data, p.W12, wd, d, ctx->stream));
  p.planes = (p.dt == C64 || p.dt == F32) && p.prec == PREC_BF16X3;
  if (p.planes) {
    const int dd = d * d;
    p.Lp = get(planes_bytes(p.dt, chil * wd, chil));
    p.Rp = get(planes_bytes(p.dt, chir, wd * chir));
    p.Xp = get(planes_bytes(p.dt, dd * chir, chil));
    p.X2p = get(planes_bytes(p.dt, chil * dd, wd * chir));
    if (!p.Lp || !p.Rp || !p.Xp || !p.X2p) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "heff plane workspace");
    // L' = L[(a,w),a'] as op(A) of the first product; R'^T as op(B) of the last
    TCI_CHECK_HIP(split_a(p.dt, OP_N, L->data, chil, 0, chil * wd, chil, p.Lp, 1, ctx->stream));
    TCI_CHECK_HIP(split_b(p.dt, OP_T, R->data, (long long)wd * chir, 0, wd * chir, chir, p.Rp, 1, ctx->stream));
    // the fused middle step writes only the valid part of the X2' planes
    TCI_CHECK_HIP(zero_fill(p.X2p, planes_bytes(p.dt, chil * dd, wd * chir), ctx->stream));
  }
  return TCI_OK;
}

static PlaneGemmArgs plane_args(int m, int n, int k, const void* Ap, const void* Bp, void* C, long long ldc) {
  PlaneGemmArgs a{};
  a.m = m; a.n = n; a.k = k;
  a.Mp = pad_rows(m); a.Np = pad_rows(n); a.Kp = pad_k(k);
  a.Ap = static_cast<const __bf16*>(Ap); a.Bp = static_cast<const __bf16*>(Bp);
  a.C = C; a.ldc = ldc;
  a.alpha_re = 1.0;
  a.batch = 1;
  return a;
}

static tci_status heff_apply(tci_context ctx, const HeffPlan& p, const void* x, void* y) {
  const int kw = p.w * p.d * p.d;
  hipStream_t s = ctx->stream;
  // X1 = L' x'
  ProfTag t1("heff_L");
  const int dd = p.d * p.d;
  if (p.planes) {
    TCI_CHECK_HIP(split_b(p.dt, OP_N, x, (long long)dd * p.chir, 0, p.chil, dd * p.chir, p.Xp, 1, s));
    TCI_CHECK_HIP(gemm_planes(p.dt, plane_args(p.chil * p.w, dd * p.chir, p.chil, p.Lp, p.Xp, p.X1, dd * p.chir), s));
  } else {
    GemmArgs g1 = gemm_args(p.chil * p.w, dd * p.chir, p.chil, OP_N, OP_N, p.L, p.chil, x, dd * p.chir, p.X1,
                            dd * p.chir);
    TCI_CHECK_HIP(gemm(p.dt, p.prec, g1, s));
  }
  // X2[a] = W12^T X1[a]
  ProfTag t2("heff_W12");
  if (p.planes && kw == 20) {
    // fused with the split of X2' for the R-step
    TCI_CHECK_HIP(w12_to_planes(p.dt, p.X1, p.W12, p.chil, kw, p.chir, p.w, p.X2p, pad_rows(p.chil * dd),
                                pad_k(p.w * p.chir), s));
    ProfTag t3("heff_R");
    TCI_CHECK_HIP(gemm_planes(p.dt, plane_args(p.chil * dd, p.chir, p.w * p.chir, p.X2p, p.Rp, y, p.chir), s));
    return TCI_OK;
  }
  GemmArgs g2 = gemm_args(kw, p.chir, kw, OP_T, OP_N, p.W12, kw, p.X1, p.chir, p.X2, p.chir);
  g2.sA = 0; g2.sB = (long long)kw * p.chir; g2.sC = (long long)kw * p.chir; g2.batch = p.chil;
  TCI_CHECK_HIP(gemm(p.dt, p.prec, g2, s));
  // y = X2' R'^T
  ProfTag t3("heff_R");
  if (p.planes) {
    TCI_CHECK_HIP(split_a(p.dt, OP_N, p.X2, (long long)p.w * p.chir, 0, p.chil * dd, p.w * p.chir, p.X2p, 1, s));
    TCI_CHECK_HIP(gemm_planes(p.dt, plane_args(p.chil * dd, p.chir, p.w * p.chir, p.X2p, p.Rp, y, p.chir), s));
    return TCI_OK;
  }
  GemmArgs g3 = gemm_args(p.chil * p.d * p.d, p.chir, p.w * p.chir, OP_N, OP_T, p.X2, (long long)p.w * p.chir, p.R,
                          (long long)p.w * p.chir, y, p.chir);
  TCI_CHECK_HIP(gemm(p.dt, p.prec, g3, s));
  return TCI_OK;
}

// Fixed device scratch of the allocation-free matvec.  In host code the
// array's name is only a host-side stand-in: its device address, one per
// device, comes from hipGetSymbolAddress at context creation (with that
// device current) and is the only form in which host code hands the array to
// kernels.
static __device__ __align__(256) unsigned char scratch[HEFF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

tci_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "device id beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return TCI_OK;
  void* ptr = nullptr;
  TCI_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) TCI_RET(TCI_ERR_DEVICE, "hipGetSymbolAddress returned a null scratch address");
  g_scratch_ptr[device] = ptr;
  return TCI_OK;
}

static void* noalloc_scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace tci

using namespace tci;

extern "C" {

tci_status tci_heff_matvec(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2, tci_tensor R, tci_tensor x,
                           tci_tensor y) try {
  if (!ctx || !y) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int chil, chir, wd, d;
  TCI_TRY(heff_check(L, W1, W2, R, x, chil, chir, wd, d));
  if (y == x) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "y must not alias x");
  Trace tr(ctx, "heff_matvec", std::to_string(chil) + "," + std::to_string(wd) + "," + std::to_string(chir));
  ctx->arena.reset();
  HeffPlan p{};
  TCI_TRY(heff_prepare(ctx, L, W1, W2, R, chil, chir, wd, d, p));
  const int64_t ysh[4] = {chil, d, d, chir};
  TCI_TRY(ensure_shape(ctx, y, L->dtype, 4, ysh));
  TCI_TRY(heff_apply(ctx, p, x->data, y->data));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_heff_matvec_noalloc(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2, tci_tensor R,
                                   tci_tensor x, tci_tensor y) try {
  if (!ctx || !y) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int chil, chir, wd, d;
  TCI_TRY(heff_check(L, W1, W2, R, x, chil, chir, wd, d));
  if (y == x) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "y must not alias x");
  const int dt = L->dtype;
  const int prec = is_double(dt) ? PREC_FP64 : ctx->precision;
  const size_t need = heff_workspace_bytes(dt, prec, chil, chir, wd, d);
  if (need > HEFF_NOALLOC_SCRATCH_BYTES)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "heff_matvec_noalloc: these shapes need " + std::to_string(need) +
                                          " bytes of workspace, above the fixed scratch of " +
                                          std::to_string(HEFF_NOALLOC_SCRATCH_BYTES) + " bytes");
  if (y->dtype != dt) TCI_RET(TCI_ERR_DTYPE, "heff_matvec_noalloc: y must have the operands' dtype");
  const size_t ybytes = (size_t)chil * d * d * chir * elem_bytes(dt);
  if (y->empty || !y->data || y->cap < ybytes)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "heff_matvec_noalloc: y must hold chi_l*d*d*chi_r elements already");
  void* ptr = noalloc_scratch_ptr(ctx->device);
  if (!ptr) TCI_RET(TCI_ERR_DEVICE, "no scratch address for this device (context not created by tci_create_context)");
  Trace tr(ctx, "heff_matvec_noalloc",
           ctx->verbose ? std::to_string(chil) + "," + std::to_string(wd) + "," + std::to_string(chir) : std::string());
  Bump ws;
  ws.base = static_cast<char*>(ptr);
  ws.cap = HEFF_NOALLOC_SCRATCH_BYTES;
  HeffPlan p{};
  TCI_TRY(heff_prepare(ctx, L, W1, W2, R, chil, chir, wd, d, p, &ws));
  y->order = 4;
  y->shape[0] = chil; y->shape[1] = d; y->shape[2] = d; y->shape[3] = chir;
  y->nlabels = 0;
  TCI_TRY(heff_apply(ctx, p, x->data, y->data));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_lanczos_ground(tci_context ctx, tci_tensor L, tci_tensor W1, tci_tensor W2, tci_tensor R,
                              tci_tensor theta, int n_matvec, double* energy) try {
  if (!ctx || !theta || !energy) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  if (n_matvec < 1 || n_matvec > 32) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "n_matvec must be in [1, 32]");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  int chil, chir, wd, d;
  TCI_TRY(heff_check(L, W1, W2, R, theta, chil, chir, wd, d));
  Trace tr(ctx, "lanczos_ground", std::to_string(chil) + "," + std::to_string(chir) + " m=" + std::to_string(n_matvec));
  ctx->arena.reset();
  hipStream_t s = ctx->stream;
  HeffPlan p{};
  TCI_TRY(heff_prepare(ctx, L, W1, W2, R, chil, chir, wd, d, p));
  const int dt = L->dtype;
  const long long N = (long long)chil * d * d * chir;
  const size_t es = elem_bytes(dt);
  // Krylov scalars, the working vector and all arithmetic in complex128.  The
  // basis is stored in complex128, or in complex64 for complex64 operands:
  // there each stored vector is the operand of its matvec, and the sweeps
  // over the basis move half the bytes.
  const bool c64 = dt == C64;
  const int vdt = c64 ? C64 : C128;
  const size_t ves = c64 ? sizeof(cf) : sizeof(cd);
  char* basis = static_cast<char*>(ctx->arena.get(ves * (size_t)N * (n_matvec + 1)));
  cd* w = static_cast<cd*>(ctx->arena.get(sizeof(cd) * (size_t)N));
  cd* th = static_cast<cd*>(ctx->arena.get(sizeof(cd) * (size_t)N));
  void* xin = ctx->arena.get(es * (size_t)N);
  void* yout = ctx->arena.get(es * (size_t)N);
  double* part = static_cast<double*>(ctx->arena.get(sizeof(double) * MULTIDOT_PARTIAL_DOUBLES));
  double* coef = static_cast<double*>(ctx->arena.get(sizeof(double) * 3 * 128));
  double* nrm = static_cast<double*>(ctx->arena.get(sizeof(double) * (SUMSQ_PARTIALS + 1)));
  if (!basis || !w || !th || !xin || !yout || !part || !coef || !nrm) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(convert(dt, theta->data, C128, th, N, s));
  auto norm2 = [&](const cd* v, double& out) -> tci_status {
    TCI_CHECK_HIP(sumsq_batched(C128, v, N, 0, nrm + SUMSQ_PARTIALS, nrm, 1, s));
    TCI_CHECK_HIP(hipMemcpyAsync(&out, nrm + SUMSQ_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, s));
    TCI_CHECK_HIP(hipStreamSynchronize(s));
    return TCI_OK;
  };
  double n0 = 0.0;
  TCI_TRY(norm2(th, n0));
  n0 = std::sqrt(n0);
  if (!(n0 > 0.0) || !std::isfinite(n0)) TCI_RET(TCI_ERR_NUMERIC, "starting vector has zero or non-finite norm");
  if (c64) TCI_CHECK_HIP(scale_to_c64(th, 1.0 / n0, 0.0, basis, N, s));
  else TCI_CHECK_HIP(scale_copy(th, 1.0 / n0, 0.0, basis, N, s));
  std::vector<double> alpha, beta;
  double tmax = 0.0;
  for (int j = 0; j < n_matvec; ++j) {
    const void* vj = basis + ves * (size_t)N * j;
    // w = H v_j (in the operands' dtype / precision)
    const void* xv = vj;
    if (dt != C128 && !c64) {
      TCI_CHECK_HIP(convert(C128, vj, dt, xin, N, s));
      xv = xin;
    }
    TCI_TRY(heff_apply(ctx, p, xv, dt == C128 ? (void*)w : yout));
    // alpha_j = Re <v_j, w> (coef[0], read by the recurrence sweep on the device)
    if (c64) {
      TCI_CHECK_HIP(widen_multidot_c64(yout, vj, w, N, part, coef, s, vdt));
    } else {
      if (dt != C128) TCI_CHECK_HIP(convert(dt, yout, C128, w, N, s));
      TCI_CHECK_HIP(multidot(vj, 1, w, N, part, coef, s));
    }
    if (j == n_matvec - 1) {   // the last residual enters neither T nor psi
      double hc[2];
      TCI_CHECK_HIP(hipMemcpyAsync(hc, coef, sizeof(hc), hipMemcpyDeviceToHost, s));
      TCI_CHECK_HIP(hipStreamSynchronize(s));
      alpha.push_back(hc[0]);
      break;
    }
    // w -= alpha v_j + beta_{j-1} v_{j-1}, then classical Gram-Schmidt
    // against v_0..v_j.  The first sweep subtracts the three-term part and
    // forms c = V^H w; the second subtracts V c and returns ||w||^2.  A second
    // Gram-Schmidt pass (one more dot sweep and one more subtraction sweep)
    // runs only when the first removed more than half of the norm,
    // ||w_after||^2 < ||c||^2 (the criterion of Daniel, Gragg, Kaufman and
    // Stewart, 1976, with ||w_before||^2 = ||w_after||^2 + ||c||^2); in exact
    // arithmetic the second pass subtracts zero.
    std::vector<double> c1(2 * (j + 1) + 1, 0.0), hc(2, 0.0);
    // bytes of one stored basis vector and of the working vector
    const double vbytes = (double)ves * (double)N, wbytes = (double)sizeof(cd) * (double)N;
    ProfTag tag("lanczos");
    {
      ProfScope ps(s, vbytes * (j + 1) + 2 * wbytes, "sweep_dot");
      TCI_CHECK_HIP(three_term_multidot(basis, j + 1, coef, j > 0 ? beta[j - 1] : 0.0, w, N, part, coef + 128, s, vdt));
    }
    {
      ProfScope ps(s, vbytes * (j + 1) + 2 * wbytes, "sweep_axpy");
      TCI_CHECK_HIP(multiaxpy_norm2(basis, j + 1, coef + 128, -1.0, w, N, part, coef + 128 + 2 * (j + 1), s, vdt));
    }
    TCI_CHECK_HIP(hipMemcpyAsync(hc.data(), coef, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    TCI_CHECK_HIP(hipMemcpyAsync(c1.data(), coef + 128, sizeof(double) * c1.size(), hipMemcpyDeviceToHost, s));
    TCI_CHECK_HIP(hipStreamSynchronize(s));
    const double a = hc[0];
    alpha.push_back(a);
    tmax = std::max(tmax, std::fabs(a));
    double b2 = c1[2 * (j + 1)], cn2 = 0.0;
    for (int q = 0; q < 2 * (j + 1); ++q) cn2 += c1[q] * c1[q];
    if (b2 < cn2) {
      {
        ProfScope ps(s, vbytes * (j + 1) + wbytes, "reorth2_dot");
        TCI_CHECK_HIP(multidot(basis, j + 1, w, N, part, coef + 256, s, vdt));
      }
      {
        ProfScope ps(s, vbytes * (j + 1) + 2 * wbytes, "reorth2_axpy");
        TCI_CHECK_HIP(multiaxpy_norm2(basis, j + 1, coef + 256, -1.0, w, N, part, nrm + SUMSQ_PARTIALS, s, vdt));
      }
      TCI_CHECK_HIP(hipMemcpyAsync(&b2, nrm + SUMSQ_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, s));
      TCI_CHECK_HIP(hipStreamSynchronize(s));
    }
    const double b = std::sqrt(b2);
    tmax = std::max(tmax, b);
    if (b <= 1e-13 * tmax) break;
    beta.push_back(b);
    void* vnext = basis + ves * (size_t)N * (j + 1);
    if (c64) TCI_CHECK_HIP(scale_to_c64(w, 1.0 / b, 0.0, vnext, N, s));
    else TCI_CHECK_HIP(scale_copy(w, 1.0 / b, 0.0, vnext, N, s));
  }
  const int m = (int)alpha.size();
  // lowest eigenpair of T = tridiag(alpha, beta): top eigenpair of -T on the device
  double* dd = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* ee = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* e2 = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* lam = static_cast<double*>(ctx->arena.get(sizeof(double) * 8));
  double* z = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* iw = static_cast<double*>(ctx->arena.get(sizeof(double) * 4 * 64));
  if (!dd || !ee || !e2 || !lam || !z || !iw) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  std::vector<double> hd(m), he(std::max(m, 1), 0.0);
  for (int i = 0; i < m; ++i) hd[i] = -alpha[i];
  for (int i = 0; i + 1 < m; ++i) he[i] = -beta[i];
  TCI_CHECK_HIP(hipMemcpyAsync(dd, hd.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
  TCI_CHECK_HIP(hipMemcpyAsync(ee, he.data(), sizeof(double) * he.size(), hipMemcpyHostToDevice, s));
  TCI_CHECK_HIP(tridiag_eigvals_top(dd, ee, e2, m, m, 1, lam, 1, 1, s));
  TCI_CHECK_HIP(hipMemsetAsync(z, 0, sizeof(double) * m, s));
  TCI_CHECK_HIP(tridiag_invit(dd, ee, m, m, lam, 1, nullptr, 1, z, 1, 0, iw, 1, s));
  std::vector<double> hz(m);
  double hl = 0.0;
  TCI_CHECK_HIP(hipMemcpyAsync(hz.data(), z, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(&hl, lam, sizeof(double), hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  // psi = sum_i y_i v_i
  std::vector<double> cy(2 * m, 0.0);
  for (int i = 0; i < m; ++i) cy[2 * i] = hz[i];
  TCI_CHECK_HIP(hipMemsetAsync(w, 0, sizeof(cd) * (size_t)N, s));
  TCI_CHECK_HIP(hipMemcpyAsync(coef, cy.data(), sizeof(double) * 2 * m, hipMemcpyHostToDevice, s));
  TCI_CHECK_HIP(multiaxpy(basis, m, coef, 1.0, w, N, s, vdt));
  double pn2 = 0.0;
  TCI_TRY(norm2(w, pn2));
  const double pn = std::sqrt(pn2);
  // phase: <theta, psi> real positive
  double ov[2];
  TCI_CHECK_HIP(multidot(th, 1, w, N, part, coef, s));
  TCI_CHECK_HIP(hipMemcpyAsync(ov, coef, sizeof(ov), hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  const double om = std::hypot(ov[0], ov[1]);
  double pr = 1.0 / pn, pi = 0.0;
  if (om > 0.0) {
    pr = ov[0] / om / pn;
    pi = -ov[1] / om / pn;
  }
  if (c64) {
    TCI_CHECK_HIP(scale_to_c64(w, pr, pi, theta->data, N, s));
  } else {
    TCI_CHECK_HIP(scale_copy(w, pr, pi, th, N, s));
    TCI_CHECK_HIP(convert(C128, th, dt, theta->data, N, s));
  }
  TCI_CHECK_HIP(hipStreamSynchronize(s));
  *energy = -hl;
  return TCI_OK;
} TCI_API_CATCH

}  // extern "C"
