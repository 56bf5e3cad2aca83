// Batched FP64 Hermitian eigensolver for the Gram matrix of the truncated SVD.
//
// The truncated SVD (paper, TCI-spec appendix, linear algebra: svd and
// trunc_svd) of theta (m x n) is taken from the Gram matrix G = theta theta^dagger:
// G = U diag(s^2) U^dagger.  Only the largest kmax eigenpairs are needed.
//
//   1. Householder reduction to real symmetric tridiagonal form,
//      G = Q T Q^dagger, blocked in panels of NB columns: per column one
//      Hermitian matrix-vector product with the trailing matrix (the only
//      O(n^2) step, memory bound) and one small fused kernel; per panel a
//      rank-2NB update of the trailing matrix on the matrix cores.
//   2. Bisection with Sturm counts for the top eigenvalues of T (one thread
//      per eigenvalue).
//   3. Inverse iteration (tridiagonal LU with partial pivoting, two solves
//      from a fixed pseudo-random start) for their eigenvectors Z (one
//      thread per vector).
//   4. Back-transformation U = Q Z with the compact-WY form of each panel's
//      reflectors, on the matrix cores.
// Every kernel takes the whole batch of same-size problems at once.
#include "common.hpp"
#include "gemm.hpp"
#include "eig.hpp"
#include "prof.hpp"

namespace tci {

template <typename T> struct EigT;
template <> struct EigT<double> {
  static constexpr int dtype = F64;
  __host__ __device__ static double zero() { return 0.0; }
  __host__ __device__ static double one() { return 1.0; }
};
template <> struct EigT<cd> {
  static constexpr int dtype = C128;
  __host__ __device__ static cd zero() { return cd{0.0, 0.0}; }
  __host__ __device__ static cd one() { return cd{1.0, 0.0}; }
};

__device__ inline double cj(double a) { return a; }
__device__ inline cd cj(cd a) { return conjg(a); }
__device__ inline double re(double a) { return a; }
__device__ inline double re(cd a) { return a.x; }
__device__ inline double im(double) { return 0.0; }
__device__ inline double im(cd a) { return a.y; }
__device__ inline double nrm2(double a) { return a * a; }
__device__ inline double nrm2(cd a) { return a.x * a.x + a.y * a.y; }
__device__ inline double mulr(double a, double b) { return a * b; }
__device__ inline cd mulr(cd a, cd b) { return a * b; }
__device__ inline double scl(double s, double a) { return s * a; }
__device__ inline cd scl(double s, cd a) { return s * a; }
__device__ inline double add(double a, double b) { return a + b; }
__device__ inline cd add(cd a, cd b) { return a + b; }
__device__ inline double sub(double a, double b) { return a - b; }
__device__ inline cd sub(cd a, cd b) { return a - b; }
__device__ inline double wsum(double v) { return wave_sum(v); }
__device__ inline cd wsum(cd v) { return cd{wave_sum(v.x), wave_sum(v.y)}; }
__device__ inline double bsum(double v, double* sh) { return block_sum(v, sh); }
__device__ inline cd bsum(cd v, double* sh) {
  const double a = block_sum(v.x, sh);
  const double b = block_sum(v.y, sh);
  return cd{a, b};
}

// w_ip = tau (y - V t2' ...) for panel column pp = ip - j0 (see LAPACK's
// latrd):  t1 = W(ip+1:n, 0:pp)^H v,  t2 = V(ip+1:n, 0:pp)^H v,
//          w = tau (y - V t1 - W t2),  w += (-tau/2 w^H v) v.
template <typename T, int NB>
__device__ void finish_w(const TriArgs& a, int b, int ip, int j0, double* sh, T* s_t1, T* s_t2) {
  const int n = a.n;
  const T* V = reinterpret_cast<const T*>(a.Vt) + b * a.sVt;
  T* W = reinterpret_cast<T*>(a.Wp) + b * a.sWp;
  const T* Y = reinterpret_cast<const T*>(a.y) + b * a.sy;
  const T taup = reinterpret_cast<const T*>(a.tau)[b * a.stau + ip];
  const int pp = ip - j0, tid = threadIdx.x;
  const T* v = V + (long)ip * n;
  for (int q = 0; q < pp; ++q) {
    T p1 = EigT<T>::zero(), p2 = EigT<T>::zero();
    const T* vq = V + (long)(j0 + q) * n;
    for (int r = ip + 1 + tid; r < n; r += 256) {
      p1 = add(p1, mulr(cj(W[(long)r * NB + q]), v[r]));
      p2 = add(p2, mulr(cj(vq[r]), v[r]));
    }
    p1 = bsum(p1, sh);
    p2 = bsum(p2, sh);
    if (tid == 0) { s_t1[q] = p1; s_t2[q] = p2; }
  }
  __syncthreads();
  T dotp = EigT<T>::zero();
  for (int r = ip + 1 + tid; r < n; r += 256) {
    T acc = Y[r];
    for (int q = 0; q < pp; ++q) {
      acc = sub(acc, mulr(V[(long)(j0 + q) * n + r], s_t1[q]));
      acc = sub(acc, mulr(W[(long)r * NB + q], s_t2[q]));
    }
    acc = mulr(taup, acc);
    W[(long)r * NB + pp] = acc;
    dotp = add(dotp, mulr(cj(acc), v[r]));
  }
  dotp = bsum(dotp, sh);
  const T alpha = mulr(scl(-0.5, taup), dotp);
  for (int r = ip + 1 + tid; r < n; r += 256)
    W[(long)r * NB + pp] = add(W[(long)r * NB + pp], mulr(alpha, v[r]));
  for (int r = tid; r <= ip && r < n; r += 256) W[(long)r * NB + pp] = EigT<T>::zero();
  __syncthreads();
}

// Column i: a(i:n, i) -= V(i:n, j0:i) conj(W(i, 0:p)) + W(i:n, 0:p) conj(V(i, j0:i)),
// d_i = Re a(i,i), then the reflector that maps a(i+1:n, i) to beta e_1 (beta
// real, LAPACK larfg convention: H = I - tau v v^H, v(i+1) = 1).
template <typename T, int NB>
__device__ void column_reflect(const TriArgs& a, int b, int i, int j0, double* sh, T* s_vrow,
                               T* s_wrow, T* s_scal) {
  const int n = a.n, tid = threadIdx.x;
  T* G = reinterpret_cast<T*>(a.G) + b * a.sG;
  T* V = reinterpret_cast<T*>(a.Vt) + b * a.sVt;
  const T* W = reinterpret_cast<const T*>(a.Wp) + b * a.sWp;
  T* tau = reinterpret_cast<T*>(a.tau) + b * a.stau;
  double* d = a.d + b * a.sde;
  double* e = a.e + b * a.sde;
  const long ldg = a.ldg;
  const int p = i - j0;
  if (tid < p) {
    s_vrow[tid] = V[(long)(j0 + tid) * n + i];
    s_wrow[tid] = W[(long)i * NB + tid];
  }
  __syncthreads();
  double xn2 = 0.0;
  for (int r = i + tid; r < n; r += 256) {
    T acc = G[(long)r * ldg + i];
    for (int q = 0; q < p; ++q) {
      acc = sub(acc, mulr(V[(long)(j0 + q) * n + r], cj(s_wrow[q])));
      acc = sub(acc, mulr(W[(long)r * NB + q], cj(s_vrow[q])));
    }
    G[(long)r * ldg + i] = acc;
    if (r >= i + 2) xn2 += nrm2(acc);
  }
  xn2 = block_sum(xn2, sh);
  if (tid == 0) {
    d[i] = re(G[(long)i * ldg + i]);
    if (i + 1 < n) {
      const T alpha = G[(long)(i + 1) * ldg + i];
      const double ar = re(alpha), ai = im(alpha);
      T tv = EigT<T>::zero(), scal = EigT<T>::zero();
      double beta;
      if (xn2 == 0.0 && ai == 0.0) {
        beta = ar;  // nothing to annihilate: H = I
      } else {
        const double nrm = sqrt(ar * ar + ai * ai + xn2);
        beta = ar >= 0.0 ? -nrm : nrm;
        // tau = (beta - alpha) / beta,  scal = 1 / (alpha - beta)
        if constexpr (sizeof(T) == sizeof(double)) {
          tv = (beta - ar) / beta;
          scal = 1.0 / (ar - beta);
        } else {
          tv = cd{(beta - ar) / beta, -ai / beta};
          const double xr = ar - beta, xi = ai, den = xr * xr + xi * xi;
          scal = cd{xr / den, -xi / den};
        }
      }
      e[i] = beta;
      tau[i] = tv;
      *s_scal = scal;
    } else {
      tau[i] = EigT<T>::zero();
    }
  }
  __syncthreads();
  if (i + 1 < n) {
    const T scal = *s_scal;
    T* v = V + (long)i * n;
    for (int r = tid; r < n; r += 256) {
      T val;
      if (r <= i) val = EigT<T>::zero();
      else if (r == i + 1) val = EigT<T>::one();
      else val = mulr(G[(long)r * ldg + i], scal);
      v[r] = val;
    }
  }
}

// One workgroup per problem: finish w of column i_fin (if >= 0), then update
// and reflect column i_col (if >= 0).
template <typename T, int NB>
__global__ __launch_bounds__(256) void tri_small_kernel(TriArgs a, int i_fin, int i_col, int j0) {
  __shared__ double sh[16];
  __shared__ T s_t1[NB], s_t2[NB], s_vrow[NB], s_wrow[NB], s_scal;
  const int b = blockIdx.x;
  if (i_fin >= 0) finish_w<T, NB>(a, b, i_fin, j0, sh, s_t1, s_t2);
  if (i_col >= 0) column_reflect<T, NB>(a, b, i_col, j0, sh, s_vrow, s_wrow, &s_scal);
}

// y(r) = sum_{c > i} G(r, c) v_i(c) for r > i: full Hermitian storage of the
// trailing matrix as it stood at the start of the panel.  One wave per row,
// lanes stride over the (contiguous) columns.
template <typename T>
__global__ __launch_bounds__(256) void tri_hemv_kernel(TriArgs a, int i) {
  const int b = blockIdx.y, n = a.n;
  const T* G = reinterpret_cast<const T*>(a.G) + b * a.sG;
  const T* v = reinterpret_cast<const T*>(a.Vt) + b * a.sVt + (long)i * n;
  T* Y = reinterpret_cast<T*>(a.y) + b * a.sy;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int r = i + 1 + blockIdx.x * 16 + wid * 4 + rr;
    if (r >= n) break;
    T acc = EigT<T>::zero();
    const T* grow = G + (long)r * a.ldg;
    for (int c = i + 1 + lane; c < n; c += 64) acc = add(acc, mulr(grow[c], v[c]));
    acc = wsum(acc);
    if (lane == 0) Y[r] = acc;
  }
}

template <typename T, int NB>
static hipError_t tridiag_impl(const TriArgs& a, int batch, hipStream_t s) {
  const int n = a.n;
  const size_t es = sizeof(T);
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int pe = min(NB, n - j0);
    for (int p = 0; p < pe; ++p) {
      const int i = j0 + p;
      hipLaunchKernelGGL((tri_small_kernel<T, NB>), dim3(batch), dim3(256), 0, s, a,
                         p > 0 ? i - 1 : -1, i, j0);
      if (i + 1 < n) {
        dim3 grid((n - i - 1 + 15) / 16, batch);
        // algorithmic bytes: the trailing matrix read once per problem
        ProfScope ps(s, (double)(n - i - 1) * (n - i - 1) * sizeof(T) * batch, "hemv");
        hipLaunchKernelGGL(tri_hemv_kernel<T>, grid, dim3(256), 0, s, a, i);
      }
    }
    const int t = j0 + pe;
    if (t < n) {
      // finish w of the panel's last column (no column update: i = t is the next panel's)
      hipLaunchKernelGGL((tri_small_kernel<T, NB>), dim3(batch), dim3(256), 0, s, a, t - 1, -1, j0);
      // G(t:n, t:n) -= V W^H + W V^H over the panel columns
      const int m = n - t;
      char* G = reinterpret_cast<char*>(a.G);
      char* V = reinterpret_cast<char*>(a.Vt);
      char* W = reinterpret_cast<char*>(a.Wp);
      GemmArgs g = gemm_args(m, m, pe, OP_T, OP_C, V + ((long)j0 * n + t) * es, n,
                             W + (long)t * NB * es, NB, G + ((long)t * a.ldg + t) * es, a.ldg);
      g.sA = a.sVt; g.sB = a.sWp; g.sC = a.sG;
      g.alpha_re = -1.0; g.beta_re = 1.0; g.batch = batch;
      hipError_t err = gemm(EigT<T>::dtype, PREC_FP64, g, s);
      if (err != hipSuccess) return err;
      GemmArgs h = gemm_args(m, m, pe, OP_N, OP_R, W + (long)t * NB * es, NB,
                             V + ((long)j0 * n + t) * es, n, G + ((long)t * a.ldg + t) * es, a.ldg);
      h.sA = a.sWp; h.sB = a.sVt; h.sC = a.sG;
      h.alpha_re = -1.0; h.beta_re = 1.0; h.batch = batch;
      err = gemm(EigT<T>::dtype, PREC_FP64, h, s);
      if (err != hipSuccess) return err;
    }
  }
  return hipGetLastError();
}

hipError_t tridiagonalize(int dtype, const TriArgs& a, int batch, hipStream_t s) {
  if (dtype == C128) return tridiag_impl<cd, TRIDIAG_NB>(a, batch, s);
  if (dtype == F64) return tridiag_impl<double, TRIDIAG_NB>(a, batch, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Bisection: lam[b][j] = j-th largest eigenvalue of the symmetric tridiagonal
// (d, e), j < kmax.  Sturm count: number of negative pivots of the LDL^T
// factorisation of T - x I equals the number of eigenvalues below x.
// ---------------------------------------------------------------------------
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

__global__ void e2_kernel(const double* e, double* e2, long long sde, int n, int batch) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)batch * n) return;
  const int b = (int)(idx / n), i = (int)(idx % n);
  const double v = (i < n - 1) ? e[b * sde + i] : 0.0;
  e2[b * sde + i] = v * v;
}

__global__ __launch_bounds__(256) void bisect_kernel(const double* d, const double* e, const double* e2,
                                                     long long sde, int n, int kmax, double* lam,
                                                     long long slam, int batch) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kmax || b >= batch) return;
  const double* db = d + b * sde;
  const double* eb = e + b * sde;
  const double* e2b = e2 + b * sde;
  double lo = db[0], hi = db[0], emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(eb[i - 1]) : 0.0) + (i < n - 1 ? fabs(eb[i]) : 0.0);
    lo = fmin(lo, db[i] - r);
    hi = fmax(hi, db[i] + r);
    if (i < n - 1) emax2 = fmax(emax2, e2b[i]);
  }
  const double scale = fmax(fabs(lo), fabs(hi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2) * 64.0;
  lo -= 4.0 * 2.220446049250313e-16 * scale + pivmin;
  hi += 4.0 * 2.220446049250313e-16 * scale + pivmin;
  const int t = n - 1 - j;  // ascending index of the wanted eigenvalue
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    if (sturm_count(db, e2b, n, mid, pivmin) <= t) lo = mid;
    else hi = mid;
  }
  lam[b * slam + j] = 0.5 * (lo + hi);
}

hipError_t tridiag_eigvals_top(const double* d, const double* e, double* e2, long long sde, int n,
                               int kmax, double* lam, long long slam, int batch, hipStream_t s) {
  if (kmax <= 0 || batch <= 0) return hipSuccess;
  const long tot = (long)batch * n;
  hipLaunchKernelGGL(e2_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, e, e2, sde, n, batch);
  hipLaunchKernelGGL(bisect_kernel, dim3((kmax + 63) / 64, batch), dim3(64), 0, s, d, e, e2, sde, n,
                     kmax, lam, slam, batch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverse iteration.  Thread (b, j) with j < chi[b] factorises
// P (T - lam_j I) = L U (partial pivoting; U has two super-diagonals) and
// solves twice, starting from a fixed pseudo-random vector; the result is
// normalised to unit 2-norm.  Workspace arrays and Z share the layout
// [b][i][j] (row i of an n x ldz matrix) so that neighbouring threads touch
// neighbouring addresses.
// ---------------------------------------------------------------------------
__device__ inline double hash_uniform(unsigned b, unsigned j, unsigned i) {
  unsigned h = b * 0x9E3779B1u ^ (j * 0x85EBCA77u + 0x165667B1u) ^ (i * 0xC2B2AE3Du);
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)h + 0.5) * (2.0 / 4294967296.0) - 1.0;
}

__global__ __launch_bounds__(64) void invit_kernel(const double* d, const double* e, long long sde, int n,
                                                   const double* lam, long long slam, const int* chi,
                                                   int kmax, double* Z, long long ldz, long long sZ,
                                                   double* w_du1, double* w_du, double* w_du2,
                                                   double* w_dl, long long sw, int batch) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || j >= kmax) return;
  const int cb = chi ? chi[b] : kmax;
  if (j >= cb) return;
  const double* db = d + b * sde;
  const double* eb = e + b * sde;
  double* du1 = w_du1 + b * sw;
  double* du = w_du + b * sw;
  double* du2 = w_du2 + b * sw;
  double* dl = w_dl + b * sw;
  double* z = Z + b * sZ;
  const long ld = ldz;
  const double lamj = lam[b * slam + j];
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) tnorm = fmax(tnorm, fabs(db[i]) + (i > 0 ? fabs(eb[i - 1]) : 0.0) + (i < n - 1 ? fabs(eb[i]) : 0.0));
  const double tiny = fmax(tnorm, 1e-300) * 2.220446049250313e-16;

  // Elimination keeps one "active" row (entries a_i, c_i in columns i, i+1)
  // and meets original row i+1 (e_i, d_{i+1} - lam, e_{i+1}).  U row i is
  // stored as (du1, du, du2); the multiplier goes to dl, offset by +-4 when
  // the rows were interchanged (|multiplier| <= 1 in both cases).
  double a_i = db[0] - lamj;       // current diagonal entry of the active row i
  double c_i = (n > 1) ? eb[0] : 0.0;  // super-diagonal of active row
  for (int i = 0; i < n - 1; ++i) {
    const double sub = eb[i];                 // entry (i+1, i)
    const double a_n = db[i + 1] - lamj;      // entry (i+1, i+1)
    const double c_n = (i + 1 < n - 1) ? eb[i + 1] : 0.0;  // entry (i+1, i+2)
    if (fabs(a_i) >= fabs(sub)) {
      double piv = a_i;
      if (fabs(piv) < tiny) piv = (piv >= 0 ? tiny : -tiny);
      const double m = sub / piv;
      du1[(long)i * ld + j] = piv;
      du[(long)i * ld + j] = c_i;
      du2[(long)i * ld + j] = 0.0;
      dl[(long)i * ld + j] = m;
      a_i = a_n - m * c_i;
      c_i = c_n;
    } else {
      // interchange rows i and i+1
      const double m = a_i / sub;
      du1[(long)i * ld + j] = sub;
      du[(long)i * ld + j] = a_n;
      du2[(long)i * ld + j] = c_n;
      dl[(long)i * ld + j] = m + (m >= 0 ? 4.0 : -4.0);  // |stored| >= 4 marks an interchange
      const double na = c_i - m * a_n;
      a_i = na;
      c_i = -m * c_n;
    }
  }
  {
    double piv = a_i;
    if (fabs(piv) < tiny) piv = (piv >= 0 ? tiny : -tiny);
    du1[(long)(n - 1) * ld + j] = piv;
    du[(long)(n - 1) * ld + j] = 0.0;
    du2[(long)(n - 1) * ld + j] = 0.0;
  }
  // two solves
  double scale = 1.0;
  for (int it = 0; it < 2; ++it) {
    // forward: b <- L^-1 P b, writing the intermediate into z
    double bi = (it == 0) ? hash_uniform(b, j, 0) : z[0 * ld + j] * scale;
    for (int i = 0; i < n - 1; ++i) {
      double bn = (it == 0) ? hash_uniform(b, j, i + 1) : z[(long)(i + 1) * ld + j] * scale;
      const double s = dl[(long)i * ld + j];
      if (fabs(s) >= 4.0) {
        const double m = s - (s >= 0 ? 4.0 : -4.0);
        z[(long)i * ld + j] = bn;
        bi = bi - m * bn;
      } else {
        z[(long)i * ld + j] = bi;
        bi = bn - s * bi;
      }
    }
    z[(long)(n - 1) * ld + j] = bi;
    // backward: U x = b
    double x1 = 0.0, x2 = 0.0, amax = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double x = (z[(long)i * ld + j] - du[(long)i * ld + j] * x1 - du2[(long)i * ld + j] * x2) /
                       du1[(long)i * ld + j];
      z[(long)i * ld + j] = x;
      x2 = x1;
      x1 = x;
      amax = fmax(amax, fabs(x));
    }
    scale = amax > 0.0 ? 1.0 / amax : 1.0;
  }
  // normalise to unit 2-norm (after the last max-scaling)
  double nn = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = z[(long)i * ld + j] * scale;
    nn += x * x;
  }
  const double inv = scale / sqrt(nn);
  for (int i = 0; i < n; ++i) z[(long)i * ld + j] *= inv;
}

hipError_t tridiag_invit(const double* d, const double* e, long long sde, int n, const double* lam,
                         long long slam, const int* chi, int kmax, double* Z, long long ldz, long long sZ,
                         double* work, int batch, hipStream_t s) {
  if (kmax <= 0 || batch <= 0) return hipSuccess;
  const long long sw = (long long)n * ldz;  // each workspace array: n x ldz per problem
  double* du1 = work;
  double* du = work + sw * batch;
  double* du2 = work + 2 * sw * batch;
  double* dl = work + 3 * sw * batch;
  hipLaunchKernelGGL(invit_kernel, dim3((kmax + 63) / 64, batch), dim3(64), 0, s, d, e, sde, n, lam,
                     slam, chi, kmax, Z, ldz, sZ, du1, du, du2, dl, sw, batch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compact-WY factor of each panel (LAPACK larft, forward, columnwise):
// H_{j0} ... H_{j0+pe-1} = I - V T V^H, T upper triangular pe x pe with
// T(i,i) = tau_i and T(0:i, i) = -tau_i T(0:i, 0:i) (V(:, 0:i)^H v_i).
// One workgroup per (panel, problem).
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(256) void larft_kernel(TriArgs a, void* Tf, long long sTf) {
  __shared__ T S[NB][NB];
  __shared__ T Tl[NB][NB];
  __shared__ double sh[16];
  const int panel = blockIdx.x, b = blockIdx.y, n = a.n;
  const int j0 = panel * NB;
  if (j0 >= n - 1) return;
  const int pe = min(NB, n - 1 - j0);  // reflectors exist for columns < n-1
  const T* V = reinterpret_cast<const T*>(a.Vt) + b * a.sVt;
  const T* tau = reinterpret_cast<const T*>(a.tau) + b * a.stau;
  T* Tout = reinterpret_cast<T*>(Tf) + b * sTf + (long)panel * NB * NB;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // S[q][i] = v_q^H v_i for q < i (one wave per pair, round robin)
  for (int pair = wid; pair < pe * pe; pair += 4) {
    const int q = pair / pe, i = pair % pe;
    if (q >= i) continue;
    const T* vq = V + (long)(j0 + q) * n;
    const T* vi = V + (long)(j0 + i) * n;
    T acc = EigT<T>::zero();
    for (int r = j0 + 1 + lane; r < n; r += 64) acc = add(acc, mulr(cj(vq[r]), vi[r]));
    acc = wsum(acc);
    if (lane == 0) S[q][i] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < pe; ++i) {
      const T ti = tau[j0 + i];
      for (int q = 0; q < i; ++q) {
        T acc = EigT<T>::zero();
        for (int r = q; r < i; ++r) acc = add(acc, mulr(Tl[q][r], S[r][i]));
        Tl[q][i] = mulr(scl(-1.0, ti), acc);
      }
      Tl[i][i] = ti;
      for (int q = i + 1; q < NB; ++q) Tl[q][i] = EigT<T>::zero();
    }
  }
  __syncthreads();
  (void)sh;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx / NB, c = idx % NB;
    Tout[idx] = (r < pe && c < pe && r <= c) ? Tl[r][c] : EigT<T>::zero();
  }
}

// U (n x kmax) <- Q U with Q = H_0 ... H_{n-2}: panels applied last to first,
// U <- U - V_p (T_p (V_p^H U)).  work: per problem NB x kmax twice.
template <typename T, int NB>
static hipError_t backtransform_impl(const TriArgs& a, void* Tf, long long sTf, void* U, long long ldu,
                                     long long sU, int kmax, const int* dims, void* work, int batch,
                                     hipStream_t s) {
  const int n = a.n;
  const int npanels = (n - 1 + NB - 1) / NB;
  if (npanels <= 0 || kmax <= 0) return hipSuccess;
  hipLaunchKernelGGL((larft_kernel<T, NB>), dim3(npanels, batch), dim3(256), 0, s, a, Tf, sTf);
  const size_t es = sizeof(T);
  char* W1 = reinterpret_cast<char*>(work);
  char* W2 = W1 + (size_t)batch * NB * kmax * es;
  char* V = reinterpret_cast<char*>(a.Vt);
  char* Uc = reinterpret_cast<char*>(U);
  char* Tc = reinterpret_cast<char*>(Tf);
  (void)dims;
  for (int p = npanels - 1; p >= 0; --p) {
    const int j0 = p * NB;
    const int pe = min(NB, n - 1 - j0);
    const int rows = n - j0 - 1;
    // W1 = V_p^H U(j0+1:n, :)
    GemmArgs g1 = gemm_args(pe, kmax, rows, OP_R, OP_N, V + ((long)j0 * n + j0 + 1) * es, n,
                            Uc + (long)(j0 + 1) * ldu * es, ldu, W1, kmax);
    g1.sA = a.sVt; g1.sB = sU; g1.sC = (long long)NB * kmax; g1.batch = batch;
    hipError_t err = gemm(EigT<T>::dtype, PREC_FP64, g1, s);
    if (err != hipSuccess) return err;
    // W2 = T_p W1
    GemmArgs g2 = gemm_args(pe, kmax, pe, OP_N, OP_N, Tc + (long)p * NB * NB * es, NB, W1, kmax, W2, kmax);
    g2.sA = sTf; g2.sB = (long long)NB * kmax; g2.sC = (long long)NB * kmax; g2.batch = batch;
    err = gemm(EigT<T>::dtype, PREC_FP64, g2, s);
    if (err != hipSuccess) return err;
    // U(j0+1:n, :) -= V_p W2
    GemmArgs g3 = gemm_args(rows, kmax, pe, OP_T, OP_N, V + ((long)j0 * n + j0 + 1) * es, n, W2, kmax,
                            Uc + (long)(j0 + 1) * ldu * es, ldu);
    g3.sA = a.sVt; g3.sB = (long long)NB * kmax; g3.sC = sU;
    g3.alpha_re = -1.0; g3.beta_re = 1.0; g3.batch = batch;
    err = gemm(EigT<T>::dtype, PREC_FP64, g3, s);
    if (err != hipSuccess) return err;
  }
  return hipGetLastError();
}

hipError_t tridiag_backtransform(int dtype, const TriArgs& a, void* Tf, long long sTf, void* U,
                                 long long ldu, long long sU, int kmax, void* work, int batch,
                                 hipStream_t s) {
  if (dtype == C128)
    return backtransform_impl<cd, TRIDIAG_NB>(a, Tf, sTf, U, ldu, sU, kmax, nullptr, work, batch, s);
  if (dtype == F64)
    return backtransform_impl<double, TRIDIAG_NB>(a, Tf, sTf, U, ldu, sU, kmax, nullptr, work, batch, s);
  return hipErrorInvalidValue;
}

}  // namespace tci
