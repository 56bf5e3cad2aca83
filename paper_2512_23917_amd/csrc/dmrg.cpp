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

// Krylov state of the Lanczos solve, kept on the device so that the
// recurrence runs without host round trips (doubles):
//   [LZ_ALPHA, +32) alpha_j   [LZ_BETA, +32) beta_j
//   LZ_TMAX  running max of |alpha| and beta (scale of the breakdown test)
//   LZ_STOP  1 after an invariant subspace was found (later steps are void)
//   LZ_M     number of recorded alpha (the order of T)
//   LZ_FLAG  1 when the step needs the second Gram-Schmidt pass
//   LZ_B2    ||w||^2 after the first pass, LZ_RB2 after the second
//   LZ_SCALE complex factor of the next basis vector: 1/||theta|| for v_0,
//            1/beta_j after step j (0 after a breakdown); at the end the
//            phase and normalisation of psi
//   LZ_NREORTH count of second passes
//   LZ_START 1 when theta has a finite nonzero norm, LZ_VALID 1 when the
//            Ritz vector is finite and nonzero (theta is written only then)
enum {
  LZ_ALPHA = 0, LZ_BETA = 32, LZ_TMAX = 64, LZ_STOP, LZ_M, LZ_FLAG, LZ_B2, LZ_RB2,
  LZ_SCALE = 72, LZ_NREORTH = 74, LZ_START, LZ_VALID, LZ_WORDS = 80
};

// Clears the state and sets the factor that normalises the start vector
// (zero when its squared norm n2 is zero or not finite).
__global__ void lz_init_kernel(double* k, const double* n2) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < LZ_WORDS; ++i) k[i] = 0.0;
  const double n0 = sqrt(*n2);
  const bool ok = n0 > 0.0 && isfinite(n0);
  k[LZ_START] = ok ? 1.0 : 0.0;
  k[LZ_SCALE] = ok ? 1.0 / n0 : 0.0;
}

// After the first Gram-Schmidt pass of step j: record alpha_j = Re coef[0],
// take ||w||^2 and the projections c = coef[128 ..) of the pass, and ask for
// a second pass when it removed more than half of the norm, ||w||^2 < ||c||^2
// (Daniel, Gragg, Kaufman and Stewart, 1976).
__global__ void lz_decide_kernel(double* k, const double* coef, int j) {
  if (threadIdx.x != 0) return;
  if (k[LZ_STOP] != 0.0) {
    k[LZ_FLAG] = 0.0;
    return;
  }
  const double a = coef[0];
  k[LZ_ALPHA + j] = a;
  k[LZ_M] = j + 1;
  k[LZ_TMAX] = fmax(k[LZ_TMAX], fabs(a));
  const double* c1 = coef + 128;
  double cn2 = 0.0;
  for (int q = 0; q < 2 * (j + 1); ++q) cn2 += c1[q] * c1[q];
  const double b2 = c1[2 * (j + 1)];
  k[LZ_B2] = b2;
  k[LZ_FLAG] = b2 < cn2 ? 1.0 : 0.0;
}

// beta_j = ||w|| after the passes; stop when it falls below 1e-13 of the
// largest entry of T seen so far (the Krylov space is invariant).
__global__ void lz_beta_kernel(double* k, int j) {
  if (threadIdx.x != 0) return;
  k[LZ_SCALE + 1] = 0.0;
  if (k[LZ_STOP] != 0.0) {
    k[LZ_SCALE] = 0.0;
    return;
  }
  const bool second = k[LZ_FLAG] != 0.0;
  if (second) k[LZ_NREORTH] += 1.0;
  const double b = sqrt(second ? k[LZ_RB2] : k[LZ_B2]);
  const double tmax = fmax(k[LZ_TMAX], b);
  k[LZ_TMAX] = tmax;
  if (b <= 1e-13 * tmax) {
    k[LZ_STOP] = 1.0;
    k[LZ_SCALE] = 0.0;
  } else {
    k[LZ_BETA + j] = b;
    k[LZ_SCALE] = 1.0 / b;
  }
}

// Last step: its residual enters neither T nor psi, only alpha_j is kept.
__global__ void lz_last_kernel(double* k, const double* coef, int j) {
  if (threadIdx.x != 0 || k[LZ_STOP] != 0.0) return;
  const double a = coef[0];
  k[LZ_ALPHA + j] = a;
  k[LZ_M] = j + 1;
  k[LZ_TMAX] = fmax(k[LZ_TMAX], fabs(a));
}

// -T as (d, e) of order n for the top-eigenpair solver, and zeroed
// eigenvector storage.  T has order m <= n (m < n after a breakdown); the
// remaining n - m diagonal entries are set to -4 max|T|, below every
// eigenvalue of -T (Gershgorin: |alpha|, beta <= max|T|), with zero coupling,
// so the top eigenpair is the one of the order-m block.  The Krylov vectors
// beyond m are zero, so the padding never reaches psi.
__global__ void lz_tridiag_kernel(const double* k, int n, double* d, double* e, double* z) {
  const int m = (int)k[LZ_M];
  const double pad = -4.0 * k[LZ_TMAX];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    d[i] = i < m ? -k[LZ_ALPHA + i] : (i < n ? pad : 0.0);
    e[i] = i + 1 < m ? -k[LZ_BETA + i] : 0.0;
    z[i] = 0.0;
  }
}

// complex coefficients (z_i, 0) of psi = sum_i z_i v_i
__global__ void lz_coef_kernel(const double* z, int m, double* c) {
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    c[2 * i] = z[i];
    c[2 * i + 1] = 0.0;
  }
}

// Factor that normalises psi and makes <theta, psi> real and positive:
// conj(ov) / (|ov| ||psi||), or 1 / ||psi|| when the overlap vanishes.
__global__ void lz_phase_kernel(double* k, const double* pn2, const double* ov) {
  if (threadIdx.x != 0) return;
  const double pn = sqrt(*pn2);
  const double om = hypot(ov[0], ov[1]);
  if (om > 0.0) {
    k[LZ_SCALE] = ov[0] / om / pn;
    k[LZ_SCALE + 1] = -ov[1] / om / pn;
  } else {
    k[LZ_SCALE] = 1.0 / pn;
    k[LZ_SCALE + 1] = 0.0;
  }
  const bool ok = k[LZ_START] != 0.0 && pn > 0.0 && isfinite(pn) && isfinite(k[LZ_SCALE]) &&
                  isfinite(k[LZ_SCALE + 1]);
  k[LZ_VALID] = ok ? 1.0 : 0.0;
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
  double* kst = static_cast<double*>(ctx->arena.get(sizeof(double) * LZ_WORDS));
  if (!basis || !w || !th || !xin || !yout || !part || !coef || !nrm || !kst)
    TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  TCI_CHECK_HIP(convert(dt, theta->data, C128, th, N, s));
  TCI_CHECK_HIP(sumsq_batched(C128, th, N, 0, nrm + SUMSQ_PARTIALS, nrm, 1, s));
  hipLaunchKernelGGL(lz_init_kernel, dim3(1), dim3(64), 0, s, kst, nrm + SUMSQ_PARTIALS);
  TCI_CHECK_HIP(hipGetLastError());
  if (c64) TCI_CHECK_HIP(scale_to_c64_dev(th, kst + LZ_SCALE, basis, N, s));
  else TCI_CHECK_HIP(scale_copy_dev(th, kst + LZ_SCALE, basis, N, s));
  // The whole solve is queued without waiting for the device: alpha, beta,
  // the reorthogonalisation decision, the breakdown test and the final
  // scaling live in kst, and the host reads them once, at the end.  After a
  // breakdown (or from a zero start vector) the remaining steps run on zero
  // vectors and record nothing.
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
      hipLaunchKernelGGL(lz_last_kernel, dim3(1), dim3(64), 0, s, kst, coef, j);
      TCI_CHECK_HIP(hipGetLastError());
      break;
    }
    // w -= alpha v_j + beta_{j-1} v_{j-1}, then classical Gram-Schmidt
    // against v_0..v_j.  The first sweep subtracts the three-term part and
    // forms c = V^H w; the second subtracts V c and returns ||w||^2.  A second
    // Gram-Schmidt pass (one more dot sweep and one more subtraction sweep)
    // is launched every step but does its work only when the device decided
    // that the first removed more than half of the norm; in exact arithmetic
    // it subtracts zero.
    // bytes of one stored basis vector and of the working vector
    const double vbytes = (double)ves * (double)N, wbytes = (double)sizeof(cd) * (double)N;
    ProfTag tag("lanczos");
    {
      ProfScope ps(s, vbytes * (j + 1) + 2 * wbytes, "sweep_dot");
      TCI_CHECK_HIP(three_term_multidot(basis, j + 1, coef, j > 0 ? kst + LZ_BETA + j - 1 : nullptr, w, N, part,
                                        coef + 128, s, vdt));
    }
    {
      ProfScope ps(s, vbytes * (j + 1) + 2 * wbytes, "sweep_axpy");
      TCI_CHECK_HIP(multiaxpy_norm2(basis, j + 1, coef + 128, -1.0, w, N, part, coef + 128 + 2 * (j + 1), s, vdt));
    }
    hipLaunchKernelGGL(lz_decide_kernel, dim3(1), dim3(64), 0, s, kst, coef, j);
    TCI_CHECK_HIP(hipGetLastError());
    TCI_CHECK_HIP(multidot(basis, j + 1, w, N, part, coef + 256, s, vdt, kst + LZ_FLAG));
    TCI_CHECK_HIP(multiaxpy_norm2(basis, j + 1, coef + 256, -1.0, w, N, part, kst + LZ_RB2, s, vdt, kst + LZ_FLAG));
    hipLaunchKernelGGL(lz_beta_kernel, dim3(1), dim3(64), 0, s, kst, j);
    TCI_CHECK_HIP(hipGetLastError());
    void* vnext = basis + ves * (size_t)N * (j + 1);
    if (c64) TCI_CHECK_HIP(scale_to_c64_dev(w, kst + LZ_SCALE, vnext, N, s));
    else TCI_CHECK_HIP(scale_copy_dev(w, kst + LZ_SCALE, vnext, N, s));
  }
  // lowest eigenpair of T = tridiag(alpha, beta): top eigenpair of -T on the device
  const int n = n_matvec;
  double* dd = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* ee = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* e2 = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* lam = static_cast<double*>(ctx->arena.get(sizeof(double) * 8));
  double* z = static_cast<double*>(ctx->arena.get(sizeof(double) * 64));
  double* iw = static_cast<double*>(ctx->arena.get(sizeof(double) * 4 * 64));
  if (!dd || !ee || !e2 || !lam || !z || !iw) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "workspace");
  hipLaunchKernelGGL(lz_tridiag_kernel, dim3(1), dim3(64), 0, s, kst, n, dd, ee, z);
  TCI_CHECK_HIP(hipGetLastError());
  TCI_CHECK_HIP(tridiag_eigvals_top(dd, ee, e2, n, n, 1, lam, 1, 1, s));
  TCI_CHECK_HIP(tridiag_invit(dd, ee, n, n, lam, 1, nullptr, 1, z, 1, 0, iw, 1, s));
  // psi = sum_i z_i v_i
  hipLaunchKernelGGL(lz_coef_kernel, dim3(1), dim3(64), 0, s, z, n, coef);
  TCI_CHECK_HIP(hipGetLastError());
  TCI_CHECK_HIP(hipMemsetAsync(w, 0, sizeof(cd) * (size_t)N, s));
  TCI_CHECK_HIP(multiaxpy(basis, n, coef, 1.0, w, N, s, vdt));
  TCI_CHECK_HIP(sumsq_batched(C128, w, N, 0, nrm + SUMSQ_PARTIALS, nrm, 1, s));
  // normalise, with the phase that makes <theta, psi> real and positive;
  // theta is left as it was when the solve failed (th still holds its
  // complex128 copy then)
  TCI_CHECK_HIP(multidot(th, 1, w, N, part, coef + 256, s));
  hipLaunchKernelGGL(lz_phase_kernel, dim3(1), dim3(64), 0, s, kst, nrm + SUMSQ_PARTIALS, coef + 256);
  TCI_CHECK_HIP(hipGetLastError());
  if (c64) {
    TCI_CHECK_HIP(scale_to_c64_dev(w, kst + LZ_SCALE, theta->data, N, s, kst + LZ_VALID));
  } else {
    TCI_CHECK_HIP(scale_copy_dev(w, kst + LZ_SCALE, th, N, s, kst + LZ_VALID));
    TCI_CHECK_HIP(convert(C128, th, dt, theta->data, N, s));
  }
  double hk[LZ_WORDS], hl = 0.0;
  TCI_CHECK_HIP(hipMemcpyAsync(hk, kst, sizeof(hk), hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipMemcpyAsync(&hl, lam, sizeof(double), hipMemcpyDeviceToHost, s));
  TCI_CHECK_HIP(hipStreamSynchronize(s));   // the solve's only host synchronisation
  if (ctx->verbose > 0)
    tr.info += " krylov=" + std::to_string((int)hk[LZ_M]) + " reorth=" + std::to_string((int)hk[LZ_NREORTH]) +
               " host_syncs=1";
  if (hk[LZ_START] == 0.0) TCI_RET(TCI_ERR_NUMERIC, "starting vector has zero or non-finite norm");
  if (hk[LZ_VALID] == 0.0 || !std::isfinite(hl) || !std::isfinite(hk[LZ_TMAX]))
    TCI_RET(TCI_ERR_NUMERIC, "Lanczos recurrence produced a non-finite or zero Ritz vector");
  *energy = -hl;
  return TCI_OK;
} TCI_API_CATCH

}  // extern "C"
