// General (non-Hermitian) eigendecomposition of one square complex128 matrix
// (Spec, eig / eigvals):
//   1. Householder reduction to upper Hessenberg form, A = Q H Q^H;
//   2. single-shift QR iteration with Wilkinson shifts and deflation of
//      negligible subdiagonal entries, the rotations accumulated into Q, to
//      the complex Schur form H = Z T Z^H (T upper triangular);
//   3. eigenvectors of T by back substitution (x_k[k] = 1), one thread per
//      eigenvector; V = (Q Z) X is then a library GEMM;
//   4. columns of V scaled to unit 2-norm with their largest-modulus entry
//      real positive, in the order of the eigenvalues the caller chose.
// Steps 1 and 2 are one workgroup per matrix: every rotation of the QR
// iteration depends on the previous one, so the iteration is bound by the
// workgroup's barrier latency, not by HBM or the matrix cores.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "geig.hpp"

namespace tci {

namespace {

constexpr int HT = 1024;   // threads of the Hessenberg / Schur workgroup
constexpr double UNIT_ROUNDOFF = 1.1102230246251565e-16;   // 2^-53

__device__ inline double cabs(cd a) { return hypot(a.x, a.y); }
__device__ inline cd cdiv(cd a, cd b) {
  // a / b by Smith's scaling
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return cd{(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  }
  const double r = b.x / b.y, den = b.y + b.x * r;
  return cd{(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}
__device__ inline cd csqrt_principal(cd z) {
  const double r = cabs(z);
  const double re = sqrt(0.5 * (r + z.x));
  const double im = sqrt(0.5 * (r - z.x));
  return cd{re, signbit(z.y) ? -im : im};
}

__device__ inline double block_sum_all(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Householder reduction of H (n x n, row-major, in place) to upper Hessenberg
// form; Q (n x n) receives the accumulated reflectors.  One workgroup.
__global__ __launch_bounds__(HT) void hessenberg_kernel(cd* __restrict__ H, cd* __restrict__ Q, int n) {
  __shared__ cd v[GEIG_MAX_N];
  __shared__ double red[HT / 64];
  const int t = threadIdx.x, nt = blockDim.x;
  const int lane = t & 63, wid = t >> 6, nw = nt >> 6;
  for (long long idx = t; idx < (long long)n * n; idx += nt)
    Q[idx] = (idx / n == idx % n) ? cd{1.0, 0.0} : cd{0.0, 0.0};
  __syncthreads();
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;   // x = H[j+1 .., j]
    double part = 0.0;
    for (int r = t; r < m; r += nt) part += abs2(H[(long long)(j + 1 + r) * n + j]);
    const double a2 = block_sum_all(part, red);
    if (a2 == 0.0) continue;
    const double alpha = sqrt(a2);
    const cd x0 = H[(long long)(j + 1) * n + j];
    const double ax0 = cabs(x0);
    const cd ph = ax0 > 0.0 ? cd{x0.x / ax0, x0.y / ax0} : cd{1.0, 0.0};
    // v = x + e^{i arg x0} ||x|| e_1, ||v||^2 = ||x||^2 - |x0|^2 + (|x0| + ||x||)^2
    const double vn = sqrt(a2 - ax0 * ax0 + (ax0 + alpha) * (ax0 + alpha));
    for (int r = t; r < m; r += nt) {
      cd xr = H[(long long)(j + 1 + r) * n + j];
      if (r == 0) xr = xr + alpha * ph;
      v[r] = (1.0 / vn) * xr;
    }
    __syncthreads();
    // left: H[j+1.., c] -= 2 v (v^H H[j+1.., c]) for c >= j, one thread per column
    for (int c = j + t; c < n; c += nt) {
      cd w{0.0, 0.0};
      for (int r = 0; r < m; ++r) w = w + conjg(v[r]) * H[(long long)(j + 1 + r) * n + c];
      w = 2.0 * w;
      for (int r = 0; r < m; ++r) {
        cd* p = &H[(long long)(j + 1 + r) * n + c];
        *p = *p - v[r] * w;
      }
    }
    __syncthreads();
    // right: M[r, j+1..] -= 2 (M[r, j+1..] v) v^H for M = H and Q, one wave per row
    for (int row = wid; row < 2 * n; row += nw) {
      cd* M = row < n ? H + (long long)row * n : Q + (long long)(row - n) * n;
      cd y{0.0, 0.0};
      for (int c = lane; c < m; c += 64) y = y + M[j + 1 + c] * v[c];
      y = cd{wave_sum(y.x), wave_sum(y.y)};
      y = 2.0 * y;
      for (int c = lane; c < m; c += 64) M[j + 1 + c] = M[j + 1 + c] - y * conjg(v[c]);
    }
    __syncthreads();
    for (int r = 2 + t; r <= m; r += nt) H[(long long)(j + r) * n + j] = cd{0.0, 0.0};
    __syncthreads();
  }
}

// c (real) and s with [[c, s], [-conj(s), c]] (a, b)^T = (r, 0)^T.
__device__ inline void givens(cd a, cd b, double& c, cd& s) {
  if (b.x == 0.0 && b.y == 0.0) { c = 1.0; s = cd{0.0, 0.0}; return; }
  if (a.x == 0.0 && a.y == 0.0) {
    const double nb = cabs(b);
    c = 0.0; s = cd{b.x / nb, -b.y / nb};
    return;
  }
  const double na = cabs(a), r = hypot(na, cabs(b));
  c = na / r;
  s = (1.0 / r) * (cd{a.x / na, a.y / na} * conjg(b));
}

// Single-shift QR iteration on the Hessenberg T (in place) to the complex
// Schur form; Z (in: Q of the reduction) accumulates the rotations.
// status[0] = 0 on success, 1 when an eigenvalue needed more than
// max_sweeps sweeps; fro[0] = ||T||_F of the result.  One workgroup.
__global__ __launch_bounds__(HT) void schur_kernel(cd* __restrict__ T, cd* __restrict__ Z, int n, int max_sweeps,
                                                   int* status, double* fro) {
  __shared__ int s_lo, s_hi, s_done;
  __shared__ cd s_g, s_x, s_y;
  __shared__ double s_c;
  __shared__ double red[HT / 64];
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) { s_hi = n - 1; s_done = 0; status[0] = 0; }
  __syncthreads();
  int sweeps = 0;
  while (true) {
    if (t == 0) {
      int hi = s_hi;
      int lo = hi;
      while (hi > 0) {
        lo = hi;
        while (lo > 0) {
          cd* sub = &T[(long long)lo * n + lo - 1];
          if (cabs(*sub) <= UNIT_ROUNDOFF * (cabs(T[(long long)(lo - 1) * n + lo - 1]) + cabs(T[(long long)lo * n + lo]))) {
            *sub = cd{0.0, 0.0};
            break;
          }
          --lo;
        }
        if (lo == hi) { --hi; sweeps = 0; continue; }
        break;
      }
      s_hi = hi;
      s_lo = lo;
      if (hi <= 0) {
        s_done = 1;
      } else {
        ++sweeps;
        if (sweeps > max_sweeps) {
          status[0] = 1;
          s_done = 1;
        } else {
          // Wilkinson shift: eigenvalue of the trailing 2 x 2 block nearer T[hi, hi]
          const cd a = T[(long long)(hi - 1) * n + hi - 1], b = T[(long long)(hi - 1) * n + hi];
          const cd c = T[(long long)hi * n + hi - 1], d = T[(long long)hi * n + hi];
          const cd tr = a + d, det = a * d - b * c;
          const cd q = 0.25 * (tr * tr);
          const cd disc = csqrt_principal(cd{q.x - det.x, q.y - det.y});
          const cd half = 0.5 * tr;
          const cd l1 = half + disc, l2 = cd{half.x - disc.x, half.y - disc.y};
          cd mu = cabs(cd{l1.x - d.x, l1.y - d.y}) < cabs(cd{l2.x - d.x, l2.y - d.y}) ? l1 : l2;
          if (sweeps % 11 == 10) mu = cd{d.x + cabs(c), d.y};   // exceptional shift against cycling
          const cd tl = T[(long long)lo * n + lo];
          s_x = cd{tl.x - mu.x, tl.y - mu.y};
          s_y = T[(long long)(lo + 1) * n + lo];
        }
      }
    }
    __syncthreads();
    if (s_done) break;
    const int lo = s_lo, hi = s_hi;
    for (int k = lo; k < hi; ++k) {
      if (t == 0) {
        double c;
        cd s;
        givens(s_x, s_y, c, s);
        s_c = c;
        s_g = s;
      }
      __syncthreads();
      const double c = s_c;
      const cd s = s_g;
      // rows k, k+1 of T from column max(lo, k-1): [c s; -conj(s) c]
      const int c0 = k - 1 > lo ? k - 1 : lo;
      for (int col = c0 + t; col < n; col += nt) {
        cd* p0 = &T[(long long)k * n + col];
        cd* p1 = &T[(long long)(k + 1) * n + col];
        const cd u0 = *p0, u1 = *p1;
        *p0 = c * u0 + s * u1;
        *p1 = c * u1 - conjg(s) * u0;
      }
      __syncthreads();
      // columns k, k+1 of T (rows 0 .. min(hi, k+2)) and of Z (all rows): times G^H
      const int r1 = k + 2 < hi ? k + 2 : hi;
      for (int row = t; row <= r1 + n; row += nt) {
        cd* M = row <= r1 ? T + (long long)row * n : Z + (long long)(row - r1 - 1) * n;
        const cd u0 = M[k], u1 = M[k + 1];
        M[k] = c * u0 + conjg(s) * u1;
        M[k + 1] = c * u1 - s * u0;
      }
      __syncthreads();
      if (t == 0 && k + 1 < hi) {
        s_x = T[(long long)(k + 1) * n + k];
        s_y = T[(long long)(k + 2) * n + k];
      }
    }
    __syncthreads();
  }
  // exact zeros below the diagonal, and ||T||_F
  double part = 0.0;
  for (long long idx = t; idx < (long long)n * n; idx += nt) {
    const int r = (int)(idx / n), c = (int)(idx % n);
    if (r > c) T[idx] = cd{0.0, 0.0};
    else part += abs2(T[idx]);
  }
  const double f = block_sum_all(part, red);
  if (t == 0) fro[0] = sqrt(f);
}

// X[:, k]: T x = t_kk x with x[k] = 1 and zeros below k, one thread per k.
// A denominator smaller than u ||T||_F (a repeated eigenvalue) is replaced by it.
__global__ __launch_bounds__(256) void triangular_eigvecs_kernel(const cd* __restrict__ T, cd* __restrict__ X, int n,
                                                                 const double* fro) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double small = UNIT_ROUNDOFF * fmax(fro[0], 2.2250738585072014e-308);
  const cd lam = T[(long long)k * n + k];
  for (int i = n - 1; i > k; --i) X[(long long)i * n + k] = cd{0.0, 0.0};
  X[(long long)k * n + k] = cd{1.0, 0.0};
  for (int i = k - 1; i >= 0; --i) {
    cd acc = cd{-T[(long long)i * n + k].x, -T[(long long)i * n + k].y};
    for (int j = i + 1; j < k; ++j) acc = acc - T[(long long)i * n + j] * X[(long long)j * n + k];
    cd den = cd{T[(long long)i * n + i].x - lam.x, T[(long long)i * n + i].y - lam.y};
    if (cabs(den) < small) den = cd{small, 0.0};
    X[(long long)i * n + k] = cdiv(acc, den);
  }
}

// out[:, k] = V[:, perm[k]] / ||.||, times the phase that makes its
// largest-modulus entry (the first on exact ties) real positive.  One
// workgroup per column.
__global__ __launch_bounds__(256) void eig_finish_kernel(const cd* __restrict__ V, const int* __restrict__ perm,
                                                         int n, cd* __restrict__ out) {
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ double red[4];
  const int k = blockIdx.x, t = threadIdx.x;
  const int src = perm[k];
  double best = -1.0, part = 0.0;
  int bi = n;
  for (int r = t; r < n; r += 256) {
    const double a = abs2(V[(long long)r * n + src]);
    part += a;
    if (a > best) { best = a; bi = r; }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      const double b2 = sv[t + off];
      const int i2 = si[t + off];
      if (b2 > sv[t] || (b2 == sv[t] && i2 < si[t])) { sv[t] = b2; si[t] = i2; }
    }
    __syncthreads();
  }
  const double nrm = sqrt(block_sum_all(part, red));
  const cd piv = V[(long long)si[0] * n + src];
  const double ap = cabs(piv);
  // phase |piv| / piv, then 1 / ||v||
  const cd ph = ap > 0.0 ? cd{piv.x / ap, -piv.y / ap} : cd{1.0, 0.0};
  const double sc = nrm > 0.0 ? 1.0 / nrm : 1.0;
  for (int r = t; r < n; r += 256) out[(long long)r * n + k] = sc * (V[(long long)r * n + src] * ph);
}

__global__ void diag_kernel(const cd* __restrict__ T, int n, cd* __restrict__ w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) w[k] = T[(long long)k * n + k];
}

}  // namespace

hipError_t geig_schur(cd* H, cd* Q, int n, int* status, double* fro, hipStream_t s) {
  if (n < 1 || n > GEIG_MAX_N) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hessenberg_kernel, dim3(1), dim3(HT), 0, s, H, Q, n);
  hipLaunchKernelGGL(schur_kernel, dim3(1), dim3(HT), 0, s, H, Q, n, GEIG_MAX_SWEEPS, status, fro);
  return hipGetLastError();
}

hipError_t geig_diag(const cd* T, int n, cd* w, hipStream_t s) {
  hipLaunchKernelGGL(diag_kernel, dim3((n + 255) / 256), dim3(256), 0, s, T, n, w);
  return hipGetLastError();
}

hipError_t geig_triangular_vectors(const cd* T, cd* X, int n, const double* fro, hipStream_t s) {
  hipLaunchKernelGGL(triangular_eigvecs_kernel, dim3((n + 255) / 256), dim3(256), 0, s, T, X, n, fro);
  return hipGetLastError();
}

hipError_t geig_finish(const cd* V, const int* perm, int n, cd* out, hipStream_t s) {
  hipLaunchKernelGGL(eig_finish_kernel, dim3(n), dim3(256), 0, s, V, perm, n, out);
  return hipGetLastError();
}

}  // namespace tci
