// Thin SVD of small matrices by one-sided (Hestenes) Jacobi rotations,
// the decomposition of the Spec's svd / trunc_svd for matrices whose
// smaller dimension is at most JACOBI_MAX_K.
//
// The Gram-matrix route of the large path squares the condition number, so
// singular values below about 1e-8 of the largest are not resolved there.
// One-sided Jacobi works on the columns of the matrix itself: every column
// pair (p, q) is rotated until |<a_p, a_q>| <= m 2^-53 ||a_p|| ||a_q||, and
// the singular values are the column norms.  They carry an absolute error of
// a few ulps of the largest one, which resolves the small values that the
// truncation of message products and of tiny bonds decides on.
//
// One workgroup (256 threads, four waves) per problem; the matrix lives in a
// column-major workspace (columns contiguous) in global memory, which stays
// in the CU's caches at these sizes.  Pairs are scheduled by the round-robin
// (circle) ordering: n/2 disjoint pairs per step, n - 1 steps per sweep, one
// wave per pair, a workgroup barrier between steps.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"
#include "jacobi.hpp"

namespace tci {

namespace {

__device__ inline double cj(double a) { return a; }
__device__ inline cd cj(cd a) { return cd{a.x, -a.y}; }
__device__ inline double sq(double a) { return a * a; }
__device__ inline double sq(cd a) { return a.x * a.x + a.y * a.y; }
__device__ inline double mulr(double a, double b) { return a * b; }
__device__ inline cd mulr(cd a, cd b) { return a * b; }
__device__ inline double scl(double s, double a) { return s * a; }
__device__ inline cd scl(double s, cd a) { return cd{s * a.x, s * a.y}; }
__device__ inline double addv(double a, double b) { return a + b; }
__device__ inline cd addv(cd a, cd b) { return a + b; }
__device__ inline double zero_of(double) { return 0.0; }
__device__ inline cd zero_of(cd) { return cd{0.0, 0.0}; }
__device__ inline double one_of(double) { return 1.0; }
__device__ inline cd one_of(cd) { return cd{1.0, 0.0}; }

__device__ inline double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wsum_re(double v) { return wsum(v); }
__device__ inline cd wsum_c(cd v) { return cd{wsum(v.x), wsum(v.y)}; }
__device__ inline double wsum_c(double v) { return wsum(v); }

// unit-modulus phase of z (1 for z = 0) and its modulus
__device__ inline void polar(double z, double& r, double& ph) {
  r = fabs(z);
  ph = z < 0.0 ? -1.0 : 1.0;
}
__device__ inline void polar(cd z, double& r, cd& ph) {
  r = sqrt(z.x * z.x + z.y * z.y);
  ph = r > 0.0 ? cd{z.x / r, z.y / r} : cd{1.0, 0.0};
}

// Orthonormal completion of vector r of the set vec(q)[i] = P[q*vs + i*is]
// (q < r already orthonormal, length len): the first unit vector e_t whose
// component orthogonal to them has norm > 1/2, orthogonalised twice.  Run
// by one wave.
template <typename T>
__device__ void complete_vector(T* P, long long vs, long long is, int len, int r) {
  const int lane = threadIdx.x & 63;
  for (int t = 0; t < len; ++t) {
    // v = e_t - sum_q conj(vec_q[t]) vec_q, twice
    for (int i = lane; i < len; i += 64) P[r * vs + i * is] = (i == t) ? one_of(T{}) : zero_of(T{});
    __threadfence_block();
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < r; ++q) {
        T c = zero_of(T{});
        for (int i = lane; i < len; i += 64) c = addv(c, mulr(cj(P[q * vs + i * is]), P[r * vs + i * is]));
        c = wsum_c(c);
        for (int i = lane; i < len; i += 64)
          P[r * vs + i * is] = addv(P[r * vs + i * is], scl(-1.0, mulr(c, P[q * vs + i * is])));
        __threadfence_block();
      }
    }
    double nn = 0.0;
    for (int i = lane; i < len; i += 64) nn += sq(P[r * vs + i * is]);
    nn = wsum(nn);
    if (nn > 0.25) {
      const double inv = 1.0 / sqrt(nn);
      for (int i = lane; i < len; i += 64) P[r * vs + i * is] = scl(inv, P[r * vs + i * is]);
      __threadfence_block();
      return;
    }
  }
}

// A: problem b at A + b*sA, row-major with leading dimension lda.
// wide == 0: the matrix is A itself (m x n, m >= n).  wide == 1: the matrix
// is the conjugate transpose of A, A being n x m (so again m x n, m >= n).
// W: m x n column-major, Vw: n x n column-major (workspace per problem).
// Outputs of the SVD of the ORIGINAL A (rows x cols, k = n):
//   wide == 0: u (m x k) = W_j / s_j,       vh (k x n) = V^H
//   wide == 1: u (n x k) = V,               vh (k x m) = (W_j / s_j)^H
// s (k) descending; the largest-modulus entry of each u column (first on
// ties) made real positive, the matching vh row scaled by the conjugate
// phase.  sweeps[b] receives the sweep count (-1 if not converged).
template <typename T>
__global__ __launch_bounds__(256) void jacobi_svd_kernel(const T* A, long long lda, long long sA, int m, int n,
                                                         int wide, T* Wk, T* Vk, long long sW, long long sV, T* u,
                                                         long long su, T* vh, long long svh, double* s,
                                                         long long ss, int* sweeps, int max_sweeps) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const T* Ab = A + b * sA;
  T* W = Wk + b * sW;
  T* V = Vk + b * sV;
  __shared__ int rotated;
  __shared__ double sig[JACOBI_MAX_K];
  __shared__ int rank_of[JACOBI_MAX_K];
  // load and V = I
  for (long long e = tid; e < (long long)m * n; e += 256) {
    const int j = (int)(e / m), i = (int)(e % m);
    W[e] = wide ? cj(Ab[(long long)j * lda + i]) : Ab[(long long)i * lda + j];
  }
  for (int e = tid; e < n * n; e += 256) V[e] = (e / n == e % n) ? one_of(T{}) : zero_of(T{});
  __syncthreads();
  const int N = n + (n & 1);            // even player count (column n is a bye when n is odd)
  const double tol = (double)m * 0x1p-53;
  int sweep = 0;
  bool conv = (n < 2);
  for (; !conv && sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      for (int k = wv; k < N / 2; k += 4) {
        const int t1 = k, t2 = N - 1 - k;
        const int p0 = t1 == 0 ? 0 : 1 + (t1 - 1 + r) % (N - 1);
        const int q0 = t2 == 0 ? 0 : 1 + (t2 - 1 + r) % (N - 1);
        const int p = min(p0, q0), q = max(p0, q0);
        if (q >= n) continue;
        T* wp = W + (long long)p * m;
        T* wq = W + (long long)q * m;
        double al = 0.0, be = 0.0;
        T ga = zero_of(T{});
        for (int i = lane; i < m; i += 64) {
          const T x = wp[i], y = wq[i];
          al += sq(x);
          be += sq(y);
          ga = addv(ga, mulr(cj(x), y));
        }
        al = wsum(al);
        be = wsum(be);
        ga = wsum_c(ga);
        double ag;
        T ph;
        polar(ga, ag, ph);
        if (!(ag > tol * sqrt(al) * sqrt(be)) || al == 0.0 || be == 0.0) continue;
        // rotate [w_p, w_q e^{-i phi}] by the real Jacobi rotation of
        // [[al, |g|], [|g|, be]]
        const double zeta = (be - al) / (2.0 * ag);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        const T phc = cj(ph);
        for (int i = lane; i < m; i += 64) {
          const T x = wp[i], y = mulr(wq[i], phc);
          wp[i] = addv(scl(c, x), scl(-sn, y));
          wq[i] = addv(scl(sn, x), scl(c, y));
        }
        T* vp = V + (long long)p * n;
        T* vq = V + (long long)q * n;
        for (int i = lane; i < n; i += 64) {
          const T x = vp[i], y = mulr(vq[i], phc);
          vp[i] = addv(scl(c, x), scl(-sn, y));
          vq[i] = addv(scl(sn, x), scl(c, y));
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    conv = (rotated == 0);
    __syncthreads();
  }
  if (tid == 0) sweeps[b] = conv ? sweep : -1;
  // singular values = column norms, ranks by descending value (stable)
  for (int j = wv; j < n; j += 4) {
    double nn = 0.0;
    for (int i = lane; i < m; i += 64) nn += sq(W[(long long)j * m + i]);
    nn = wsum(nn);
    if (lane == 0) sig[j] = sqrt(nn);
  }
  __syncthreads();
  if (tid < n) {
    int rk = 0;
    const double sj = sig[tid];
    for (int i = 0; i < n; ++i) rk += (sig[i] > sj) || (sig[i] == sj && i < tid);
    rank_of[tid] = rk;
    s[b * ss + rk] = sj;
  }
  __syncthreads();
  T* ub = u + b * su;
  T* vb = vh + b * svh;
  const int k = n;
  // the normalised columns W_j / s_j and the rotations V_j, at rank r
  if (!wide) {
    for (long long e = tid; e < (long long)m * n; e += 256) {
      const int j = (int)(e / m), i = (int)(e % m);
      const double sj = sig[j];
      ub[(long long)i * k + rank_of[j]] = sj > 0.0 ? scl(1.0 / sj, W[e]) : zero_of(T{});
    }
    for (int e = tid; e < n * n; e += 256) {
      const int j = e / n, i = e % n;
      vb[(long long)rank_of[j] * n + i] = cj(V[e]);
    }
  } else {
    for (int e = tid; e < n * n; e += 256) {
      const int j = e / n, i = e % n;
      ub[(long long)i * k + rank_of[j]] = V[e];
    }
    for (long long e = tid; e < (long long)m * n; e += 256) {
      const int j = (int)(e / m), i = (int)(e % m);
      const double sj = sig[j];
      vb[(long long)rank_of[j] * m + i] = sj > 0.0 ? cj(scl(1.0 / sj, W[e])) : zero_of(T{});
    }
  }
  __syncthreads();
  // orthonormal completion of the vectors of zero singular values (they
  // sort last); one wave, in rank order
  if (wv == 0) {
    for (int r = 0; r < k; ++r) {
      if (s[b * ss + r] > 0.0) continue;
      if (!wide) complete_vector(ub, 1, k, m, r);
      else complete_vector(vb, m, 1, m, r);
    }
  }
  __syncthreads();
  // gauge: largest-modulus entry of each u column real positive
  const int urows = wide ? n : m;
  const int vcols = wide ? m : n;
  for (int r = wv; r < k; r += 4) {
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < urows; i += 64) {
      const double a = sq(ub[(long long)i * k + r]);
      if (a > best) { best = a; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    double mod;
    T ph;
    polar(ub[(long long)bi * k + r], mod, ph);
    const T phc = cj(ph);
    for (int i = lane; i < urows; i += 64) ub[(long long)i * k + r] = mulr(ub[(long long)i * k + r], phc);
    for (int i = lane; i < vcols; i += 64) vb[(long long)r * vcols + i] = mulr(vb[(long long)r * vcols + i], ph);
  }
}

}  // namespace

size_t jacobi_work_elems(int m, int n) { return (size_t)m * n + (size_t)n * n; }

hipError_t jacobi_svd(int dtype, const void* A, long long lda, long long sA, int rows, int cols, void* work,
                      void* u, long long su, void* vh, long long svh, double* s, long long ss, int* sweeps,
                      int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const int wide = rows < cols;
  const int m = wide ? cols : rows, n = wide ? rows : cols;
  if (n > JACOBI_MAX_K || n < 1) return hipErrorInvalidValue;
  const size_t es = elem_bytes(dtype);
  const long long sW = (long long)m * n, sV = (long long)n * n;
  char* W = static_cast<char*>(work);
  char* V = W + es * (size_t)sW * batch;
  const int max_sweeps = 80;
  if (dtype == C128)
    hipLaunchKernelGGL(jacobi_svd_kernel<cd>, dim3(batch), dim3(256), 0, st, (const cd*)A, lda, sA, m, n, wide,
                       (cd*)W, (cd*)V, sW, sV, (cd*)u, su, (cd*)vh, svh, s, ss, sweeps, max_sweeps);
  else if (dtype == F64)
    hipLaunchKernelGGL(jacobi_svd_kernel<double>, dim3(batch), dim3(256), 0, st, (const double*)A, lda, sA, m, n,
                       wide, (double*)W, (double*)V, sW, sV, (double*)u, su, (double*)vh, svh, s, ss, sweeps,
                       max_sweeps);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tci
