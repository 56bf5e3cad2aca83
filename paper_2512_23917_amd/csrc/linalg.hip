// Batched linear-algebra and elementwise kernels of the two-site update:
// Frobenius norms (TCI-spec appendix, norm: sum of squared moduli), the
// two-site gate, the truncation rule (trunc_svd rules a-c), gauge fixing,
// write-back of the site tensors with renormalisation (normalize), transpose
// (Sec. II.B transpose equation) and Cholesky-QR with column dropping.
#include "common.hpp"
#include "gemm.hpp"
#include "linalg.hpp"

namespace tci {

template <typename T> struct LT;
template <> struct LT<double> { static constexpr int dtype = F64; };
template <> struct LT<cd> { static constexpr int dtype = C128; };
template <> struct LT<float> { static constexpr int dtype = F32; };
template <> struct LT<cf> { static constexpr int dtype = C64; };

__device__ inline double sqmod(double a) { return a * a; }
__device__ inline double sqmod(float a) { return (double)a * a; }
__device__ inline double sqmod(cd a) { return a.x * a.x + a.y * a.y; }
__device__ inline double sqmod(cf a) { return (double)a.x * a.x + (double)a.y * a.y; }

// ---------------------------------------------------------------------------
// Sum of squared moduli per problem, FP64 accumulation, deterministic
// two-pass reduction (fixed partial order).
// ---------------------------------------------------------------------------
constexpr int NORM_BLOCKS = 128;

template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial_kernel(const T* x, long long n, long long sx,
                                                            double* partial) {
  __shared__ double sh[16];
  const int b = blockIdx.y;
  const T* xb = x + b * sx;
  double acc = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    acc += sqmod(xb[i]);
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[b * NORM_BLOCKS + blockIdx.x] = acc;
}

__global__ void sumsq_final_kernel(const double* partial, double* out, int nparts) {
  const int b = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += partial[b * NORM_BLOCKS + i];
    out[b] = s;
  }
}

hipError_t sumsq_batched(int dtype, const void* x, long long n, long long sx, double* out,
                         double* partial /* batch * NORM_BLOCKS */, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int nb = (int)std::min<long long>(NORM_BLOCKS, std::max<long long>(1, (n + 255) / 256));
  dim3 grid(nb, batch);
  switch (dtype) {
    case C128: hipLaunchKernelGGL(sumsq_partial_kernel<cd>, grid, dim3(256), 0, s, (const cd*)x, n, sx, partial); break;
    case F64: hipLaunchKernelGGL(sumsq_partial_kernel<double>, grid, dim3(256), 0, s, (const double*)x, n, sx, partial); break;
    case C64: hipLaunchKernelGGL(sumsq_partial_kernel<cf>, grid, dim3(256), 0, s, (const cf*)x, n, sx, partial); break;
    case F32: hipLaunchKernelGGL(sumsq_partial_kernel<float>, grid, dim3(256), 0, s, (const float*)x, n, sx, partial); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(sumsq_final_kernel, dim3(batch), dim3(64), 0, s, partial, out, nb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Two-site gate: theta'(a, u, v, b) = sum_{s,t} G[(u v), (s t)] theta(a, s, t, b)
// for theta of shape (chi_l, d, d, chi_r), in place.  One thread per (a, b).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(256) void gate_kernel(T* theta, long long stheta, const T* gate,
                                                   long long sgate, int chi_l, int chi_r) {
  const int bidx = blockIdx.y;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= (long long)chi_l * chi_r) return;
  const int a = (int)(idx / chi_r), bb = (int)(idx % chi_r);
  T* th = theta + bidx * stheta;
  const T* g = gate + bidx * sgate;
  T in[D * D];
#pragma unroll
  for (int p = 0; p < D * D; ++p) in[p] = th[((long long)a * D * D + p) * chi_r + bb];
#pragma unroll
  for (int o = 0; o < D * D; ++o) {
    T acc{};
#pragma unroll
    for (int p = 0; p < D * D; ++p) acc = acc + g[o * D * D + p] * in[p];
    th[((long long)a * D * D + o) * chi_r + bb] = acc;
  }
}

__device__ inline cf operator*(cf a, cd b) { return cf{(float)(a.x * b.x - a.y * b.y), (float)(a.x * b.y + a.y * b.x)}; }

hipError_t gate_apply(int dtype, void* theta, long long stheta, const void* gate, long long sgate,
                      int chi_l, int d, int chi_r, int batch, hipStream_t s) {
  if (d != 2) return hipErrorInvalidValue;
  const long long n = (long long)chi_l * chi_r;
  dim3 grid((unsigned)((n + 255) / 256), batch);
  switch (dtype) {
    case C128: hipLaunchKernelGGL((gate_kernel<cd, 2>), grid, dim3(256), 0, s, (cd*)theta, stheta, (const cd*)gate, sgate, chi_l, chi_r); break;
    case F64: hipLaunchKernelGGL((gate_kernel<double, 2>), grid, dim3(256), 0, s, (double*)theta, stheta, (const double*)gate, sgate, chi_l, chi_r); break;
    case C64: hipLaunchKernelGGL((gate_kernel<cf, 2>), grid, dim3(256), 0, s, (cf*)theta, stheta, (const cf*)gate, sgate, chi_l, chi_r); break;
    case F32: hipLaunchKernelGGL((gate_kernel<float, 2>), grid, dim3(256), 0, s, (float*)theta, stheta, (const float*)gate, sgate, chi_l, chi_r); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Truncation rule (trunc_svd rules a-c) on the top kmax eigenvalues lam
// (descending) of theta theta^dagger, with the total weight W = ||theta||_F^2:
//   s_j = sqrt(max(lam_j, 0));  n_a = #{j : s_j >= s_min}
//   chi = n_a if n_a <= chi_min, else the smallest chi >= chi_min with
//   eps(chi) <= target, capped at min(chi_max, n_a);  chi >= 1;
//   eps(chi) = max(W - sum_{j<chi} s_j^2, 0) / W  (0 when W = 0).
// Outputs per problem: chi, eps, discarded weight eps*W, the kept s_j,
// 1/s_j (0 for s_j = 0) and s_j / ||s_kept||_2.
// ---------------------------------------------------------------------------
// One workgroup per problem.  lam holds the kmax largest Gram eigenvalues in
// descending order, total the squared Frobenius norm W.  The kept weight of
// chi values is the prefix sum of max(lam, 0); thread t owns the contiguous
// chunk [j0, j1) of indices and tests the candidates chi in that chunk.
__global__ __launch_bounds__(256) void trunc_select_kernel(const double* lam, long long slam, int kmax,
                                                           const double* total, TruncParams p, int* chi_out,
                                                           double* err_out, double* disc_out, double* s_out,
                                                           double* sinv_out, double* sn_out, long long ss,
                                                           int batch, int sv_input) {
  __shared__ double s_scan[256];
  __shared__ int s_red[256];
  __shared__ double s_kept;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b >= batch) return;
  const double* l = lam + b * slam;
  const double W = total[b];
  // lam holds eigenvalues of the Gram matrix (s_j^2), or the singular
  // values themselves when sv_input is set
  auto wt = [&](int j) { return sv_input ? l[j] * l[j] : fmax(l[j], 0.0); };
  auto sval = [&](int j) { return sv_input ? l[j] : sqrt(fmax(l[j], 0.0)); };
  auto eps_of = [&](double kept_w) { return W > 0.0 ? fmax(W - kept_w, 0.0) / W : 0.0; };
  auto block_min = [&](int v) {
    __syncthreads();
    s_red[tid] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) s_red[tid] = min(s_red[tid], s_red[tid + off]);
      __syncthreads();
    }
    return s_red[0];
  };
  // n_a: number of leading values with s_j >= s_min
  int bad = kmax;
  for (int j = tid; j < kmax; j += 256)
    if (sval(j) < p.s_min) bad = min(bad, j);
  const int n_a = block_min(bad);
  // exclusive scan of the chunk sums
  const int chunk = (kmax + 255) / 256;
  const int j0 = min(kmax, tid * chunk), j1 = min(kmax, j0 + chunk);
  double loc = 0.0;
  for (int j = j0; j < j1; ++j) loc += wt(j);
  s_scan[tid] = loc;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const double v = tid >= off ? s_scan[tid - off] : 0.0;
    __syncthreads();
    s_scan[tid] += v;
    __syncthreads();
  }
  const double base = s_scan[tid] - loc;
  // kept(c) = sum_{j < c} wt(j); thread t owns c in [j0, j1), the last thread also c = kmax
  auto kept_at = [&](int c) {
    double k = base;
    for (int j = j0; j < c; ++j) k += wt(j);
    return k;
  };
  int chi;
  if (n_a <= p.chi_min) {
    chi = n_a;
  } else {
    const int lim = min(p.chi_max, n_a);
    int cand = lim;
    double k = base;
    const int chi_hi = (j1 == kmax) ? kmax : j1 - 1;
    for (int c = j0; c <= chi_hi; ++c) {
      if (c >= p.chi_min && c <= lim && eps_of(k) <= p.target) {
        cand = c;
        break;
      }
      if (c < j1) k += wt(c);
    }
    chi = block_min(cand);
  }
  if (chi < 1) chi = 1;
  __syncthreads();
  if (j0 < j1 ? (chi >= j0 && chi < j1) || (chi == kmax && j1 == kmax) : false) s_kept = kept_at(chi);
  __syncthreads();
  const double kept = s_kept;
  const double nrm = sqrt(kept);
  if (tid == 0) {
    const double eps = eps_of(kept);
    chi_out[b] = chi;
    err_out[b] = eps;
    disc_out[b] = eps * W;
  }
  for (int j = tid; j < kmax; j += 256) {
    const double sj = j < chi ? sval(j) : 0.0;
    s_out[b * ss + j] = sj;
    sinv_out[b * ss + j] = sj > 0.0 ? 1.0 / sj : 0.0;
    sn_out[b * ss + j] = nrm > 0.0 ? sj / nrm : 0.0;
  }
}

hipError_t trunc_select(const double* lam, long long slam, int kmax, const double* total,
                        const TruncParams& p, int* chi, double* err, double* disc, double* s,
                        double* sinv, double* sn, long long ss, int batch, hipStream_t st, bool sv_input) {
  if (batch <= 0 || kmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(trunc_select_kernel, dim3(batch), dim3(256), 0, st, lam, slam, kmax, total, p, chi, err, disc,
                     s, sinv, sn, ss, batch, sv_input ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gauge: multiply column j < chi of U (m x ncol, ld ldu) by the phase that
// makes its largest-modulus entry (first on ties) real and positive.
// One wave per column.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T scale_phase(T u, double pr, double pi_) {
  if constexpr (sizeof(T) == 16) return T{u.x * pr - u.y * pi_, u.x * pi_ + u.y * pr};
  else if constexpr (sizeof(T) == 8 && !std::is_same<T, double>::value)
    return T{(float)(u.x * pr - u.y * pi_), (float)(u.x * pi_ + u.y * pr)};
  else return (T)(u * pr);
}

// Phase of each column j < chi[b]: the entry of largest modulus (first row on
// ties) is made real positive.  Workgroup (column block, b): lane -> column
// (coalesced rows), four row groups combined through LDS.
template <typename T>
__global__ __launch_bounds__(256) void gauge_cols_kernel(T* U, long long ldu, long long sU, int m, int ncol,
                                                         const int* chi) {
  __shared__ double s_best[4][64];
  __shared__ int s_idx[4][64];
  __shared__ double s_ph[2][64];
  const int b = blockIdx.y, lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int nc = chi ? min(chi[b], ncol) : ncol;
  const bool cj = j < nc;
  T* u = U + b * sU;
  double best = -1.0;
  int bi = 0;
  if (cj)
    for (int r = rg; r < m; r += 4) {
      const double v = sqmod(u[(long long)r * ldu + j]);
      if (v > best) { best = v; bi = r; }
    }
  s_best[rg][lane] = best;
  s_idx[rg][lane] = bi;
  __syncthreads();
  if (rg == 0) {
    for (int g = 1; g < 4; ++g) {
      const double ob = s_best[g][lane];
      const int oi = s_idx[g][lane];
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    double pr = 1.0, pi_ = 0.0;
    if (cj) {
      const T piv = u[(long long)bi * ldu + j];
      if constexpr (sizeof(T) == 16 || (sizeof(T) == 8 && !std::is_same<T, double>::value)) {
        const double md = sqrt((double)piv.x * piv.x + (double)piv.y * piv.y);
        if (md > 0.0) { pr = piv.x / md; pi_ = -piv.y / md; }
      } else {
        if (piv < 0) pr = -1.0;
      }
    }
    s_ph[0][lane] = pr;
    s_ph[1][lane] = pi_;
  }
  __syncthreads();
  if (!cj) return;
  const double pr = s_ph[0][lane], pi_ = s_ph[1][lane];
  if (pr == 1.0 && pi_ == 0.0) return;
  for (int r = rg; r < m; r += 4) u[(long long)r * ldu + j] = scale_phase(u[(long long)r * ldu + j], pr, pi_);
}

hipError_t gauge_columns(int dtype, void* U, long long ldu, long long sU, int m, int ncol,
                         const int* chi, int batch, hipStream_t s) {
  dim3 grid((ncol + 63) / 64, batch);
  switch (dtype) {
    case C128: hipLaunchKernelGGL(gauge_cols_kernel<cd>, grid, dim3(256), 0, s, (cd*)U, ldu, sU, m, ncol, chi); break;
    case F64: hipLaunchKernelGGL(gauge_cols_kernel<double>, grid, dim3(256), 0, s, (double*)U, ldu, sU, m, ncol, chi); break;
    case C64: hipLaunchKernelGGL(gauge_cols_kernel<cf>, grid, dim3(256), 0, s, (cf*)U, ldu, sU, m, ncol, chi); break;
    case F32: hipLaunchKernelGGL(gauge_cols_kernel<float>, grid, dim3(256), 0, s, (float*)U, ldu, sU, m, ncol, chi); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Real -> complex copy (Z of the tridiagonal problem into the complex U).
// ---------------------------------------------------------------------------
__global__ void real_to_cplx_kernel(const double* z, cd* u, long long n, long long sz, long long su) {
  const int b = blockIdx.y;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    u[b * su + i] = cd{z[b * sz + i], 0.0};
}

hipError_t real_to_complex(const double* z, void* u, long long n, long long sz, long long su, int batch,
                           hipStream_t s) {
  dim3 grid((unsigned)std::min<long long>(1024, (n + 255) / 256), batch);
  hipLaunchKernelGGL(real_to_cplx_kernel, grid, dim3(256), 0, s, z, (cd*)u, n, sz, su);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Write-back: out[b] (rows x chi[b], dense, ld chi[b]) = in[b] (rows x ldin)
// columns 0..chi-1, each column j scaled by colscale[b][j] (optional);
// or rows variant: out rows 0..chi-1 (dense, ncols wide) scaled by rowscale.
// Also works in place when out == in and ld matches.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T mul_scalar(T v, double s);
template <> __device__ inline cd mul_scalar(cd v, double s) { return cd{v.x * s, v.y * s}; }
template <> __device__ inline double mul_scalar(double v, double s) { return v * s; }
template <> __device__ inline cf mul_scalar(cf v, double s) { return cf{(float)(v.x * s), (float)(v.y * s)}; }
template <> __device__ inline float mul_scalar(float v, double s) { return (float)(v * s); }

template <typename T>
__global__ void compact_cols_kernel(const T* in, long long ldin, long long sin_, T* out, long long sout,
                                    int rows, const int* chi, const double* cs, long long scs) {
  const int b = blockIdx.y;
  const int c = chi[b];
  const T* src = in + b * sin_;
  T* dst = out + b * sout;
  const long long total = (long long)rows * c;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
    const int r = (int)(idx / c), j = (int)(idx % c);
    T v = src[(long long)r * ldin + j];
    if (cs) v = mul_scalar(v, cs[b * scs + j]);
    dst[idx] = v;
  }
}

template <typename T>
__global__ void scale_rows_kernel(const T* in, long long sin_, T* out, long long sout, long long ncols,
                                  const int* chi, const double* rs, long long srs) {
  const int b = blockIdx.y;
  const int c = chi[b];
  const T* src = in + b * sin_;
  T* dst = out + b * sout;
  const long long total = (long long)c * ncols;
  for (long long idx = blockIdx.x * 256LL + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
    const int r = (int)(idx / ncols);
    T v = src[idx];
    if (rs) v = mul_scalar(v, rs[b * srs + r]);
    dst[idx] = v;
  }
}

hipError_t compact_columns(int dtype, const void* in, long long ldin, long long sin_, void* out,
                           long long sout, int rows, int maxchi, const int* chi, const double* cs,
                           long long scs, int batch, hipStream_t s) {
  dim3 grid((unsigned)std::min<long long>(2048, ((long long)rows * maxchi + 255) / 256), batch);
  switch (dtype) {
    case C128: hipLaunchKernelGGL(compact_cols_kernel<cd>, grid, dim3(256), 0, s, (const cd*)in, ldin, sin_, (cd*)out, sout, rows, chi, cs, scs); break;
    case F64: hipLaunchKernelGGL(compact_cols_kernel<double>, grid, dim3(256), 0, s, (const double*)in, ldin, sin_, (double*)out, sout, rows, chi, cs, scs); break;
    case C64: hipLaunchKernelGGL(compact_cols_kernel<cf>, grid, dim3(256), 0, s, (const cf*)in, ldin, sin_, (cf*)out, sout, rows, chi, cs, scs); break;
    case F32: hipLaunchKernelGGL(compact_cols_kernel<float>, grid, dim3(256), 0, s, (const float*)in, ldin, sin_, (float*)out, sout, rows, chi, cs, scs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t scale_rows(int dtype, const void* in, long long sin_, void* out, long long sout, long long ncols,
                      int maxchi, const int* chi, const double* rs, long long srs, int batch, hipStream_t s) {
  dim3 grid((unsigned)std::min<long long>(2048, ((long long)maxchi * ncols + 255) / 256), batch);
  switch (dtype) {
    case C128: hipLaunchKernelGGL(scale_rows_kernel<cd>, grid, dim3(256), 0, s, (const cd*)in, sin_, (cd*)out, sout, ncols, chi, rs, srs); break;
    case F64: hipLaunchKernelGGL(scale_rows_kernel<double>, grid, dim3(256), 0, s, (const double*)in, sin_, (double*)out, sout, ncols, chi, rs, srs); break;
    case C64: hipLaunchKernelGGL(scale_rows_kernel<cf>, grid, dim3(256), 0, s, (const cf*)in, sin_, (cf*)out, sout, ncols, chi, rs, srs); break;
    case F32: hipLaunchKernelGGL(scale_rows_kernel<float>, grid, dim3(256), 0, s, (const float*)in, sin_, (float*)out, sout, ncols, chi, rs, srs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// x[i] /= lam[(i / div) % mod] for i < n: the inverse bond weights of the
// Vidal form applied along one bond of a row-major tensor (quotient in FP64).
template <typename T>
__device__ inline T div_scalar(T v, double w);
template <>
__device__ inline double div_scalar<double>(double v, double w) { return v / w; }
template <>
__device__ inline float div_scalar<float>(float v, double w) { return (float)((double)v / w); }
template <>
__device__ inline cd div_scalar<cd>(cd v, double w) { return cd{v.x / w, v.y / w}; }
template <>
__device__ inline cf div_scalar<cf>(cf v, double w) { return cf{(float)((double)v.x / w), (float)((double)v.y / w)}; }

template <typename T>
__global__ void inv_scale_axis_kernel(T* x, long long n, long long div, long long mod, const double* lam) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    x[i] = div_scalar(x[i], lam[(i / div) % mod]);
}

hipError_t inv_scale_axis(int dtype, void* x, long long n, long long div, long long mod, const double* lam,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<long long>(2048, (n + 255) / 256));
  switch (dtype) {
    case C128: hipLaunchKernelGGL(inv_scale_axis_kernel<cd>, grid, dim3(256), 0, s, (cd*)x, n, div, mod, lam); break;
    case F64: hipLaunchKernelGGL(inv_scale_axis_kernel<double>, grid, dim3(256), 0, s, (double*)x, n, div, mod, lam); break;
    case C64: hipLaunchKernelGGL(inv_scale_axis_kernel<cf>, grid, dim3(256), 0, s, (cf*)x, n, div, mod, lam); break;
    case F32: hipLaunchKernelGGL(inv_scale_axis_kernel<float>, grid, dim3(256), 0, s, (float*)x, n, div, mod, lam); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transpose of an order-r tensor (r <= 8): out[c] = in[c'] with
// c'[perm[b]] = c[b].  When the last bond stays last, consecutive threads
// read and write consecutive elements; otherwise the innermost output index
// is split into 64-wide chunks staged through LDS so that both the read
// (along the input's last bond) and the write stay coalesced.
// ---------------------------------------------------------------------------
struct PermArgs {
  int order;
  long long out_shape[8];
  long long in_stride_of_out[8];  // input stride of output bond b (= in_stride[perm[b]])
  long long total;
};

template <typename T>
__global__ __launch_bounds__(256) void permute_kernel(const T* in, T* out, PermArgs p) {
  for (long long lin = blockIdx.x * 256LL + threadIdx.x; lin < p.total; lin += (long long)gridDim.x * 256) {
    long long rem = lin, src = 0;
    for (int b = p.order - 1; b >= 0; --b) {
      const long long cb = rem % p.out_shape[b];
      rem /= p.out_shape[b];
      src += cb * p.in_stride_of_out[b];
    }
    out[lin] = in[src];
  }
}

// Tiled variant for permutations that move the input's last bond: treat the
// tensor as in[..., x, ..., y] with y the input's contiguous bond and x the
// output's contiguous bond; 64 x 64 tiles are transposed through LDS.
template <typename T>
__global__ __launch_bounds__(256) void permute_tiled_kernel(const T* in, T* out, PermArgs p, int bx,
                                                            int by, long long ntile_x, long long ntile_y) {
  __shared__ T tile[64][65];
  // bx: output bond index that is contiguous in the output (order-1);
  // by: output bond index whose input stride is 1.
  const long long nx = p.out_shape[bx], ny = p.out_shape[by];
  long long rest = blockIdx.x;
  const long long tx = rest % ntile_x; rest /= ntile_x;
  const long long ty = rest % ntile_y; rest /= ntile_y;
  // decode the remaining bonds (all except bx, by) from `rest`
  long long src_base = 0, dst_base = 0, dst_stride[8];
  {
    long long acc = 1;
    for (int b = p.order - 1; b >= 0; --b) { dst_stride[b] = acc; acc *= p.out_shape[b]; }
  }
  for (int b = p.order - 1; b >= 0; --b) {
    if (b == bx || b == by) continue;
    const long long cb = rest % p.out_shape[b];
    rest /= p.out_shape[b];
    src_base += cb * p.in_stride_of_out[b];
    dst_base += cb * dst_stride[b];
  }
  const int t = threadIdx.x;
  // read: rows along x (input stride sx), columns along y (input stride 1)
  for (int k = t; k < 64 * 64; k += 256) {
    const int ix = k / 64, iy = k % 64;
    const long long gx = tx * 64 + ix, gy = ty * 64 + iy;
    if (gx < nx && gy < ny) tile[ix][iy] = in[src_base + gx * p.in_stride_of_out[bx] + gy];
  }
  __syncthreads();
  for (int k = t; k < 64 * 64; k += 256) {
    const int iy = k / 64, ix = k % 64;
    const long long gx = tx * 64 + ix, gy = ty * 64 + iy;
    if (gx < nx && gy < ny) out[dst_base + gy * dst_stride[by] + gx] = tile[ix][iy];
  }
}

hipError_t permute(int dtype, const void* in, void* out, int order, const long long* shape,
                   const int* perm, hipStream_t s) {
  if (order < 0 || order > 8) return hipErrorInvalidValue;
  PermArgs p{};
  p.order = order;
  long long in_stride[8];
  long long acc = 1;
  for (int b = order - 1; b >= 0; --b) { in_stride[b] = acc; acc *= shape[b]; }
  p.total = acc;
  if (p.total == 0) return hipSuccess;
  for (int b = 0; b < order; ++b) {
    p.out_shape[b] = shape[perm[b]];
    p.in_stride_of_out[b] = in_stride[perm[b]];
  }
  int by = -1;
  for (int b = 0; b < order; ++b) if (perm[b] == order - 1) by = b;
  const bool tiled = order >= 2 && by != order - 1 && p.out_shape[order - 1] >= 16 &&
                     p.out_shape[by] >= 16;
  const size_t es = elem_bytes(dtype);
  if (tiled) {
    const int bx = order - 1;
    const long long ntx = (p.out_shape[bx] + 63) / 64, nty = (p.out_shape[by] + 63) / 64;
    const long long others = p.total / (p.out_shape[bx] * p.out_shape[by]);
    const long long blocks = ntx * nty * others;
    if (blocks < (1LL << 31)) {
#define PT(T) hipLaunchKernelGGL(permute_tiled_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, (const T*)in, (T*)out, p, bx, by, ntx, nty)
      if (es == 16) PT(cd); else if (es == 8) PT(double); else PT(float);
#undef PT
      return hipGetLastError();
    }
  }
  const unsigned grid = (unsigned)std::min<long long>(65536, (p.total + 255) / 256);
  if (es == 16) hipLaunchKernelGGL(permute_kernel<cd>, dim3(grid), dim3(256), 0, s, (const cd*)in, (cd*)out, p);
  else if (es == 8) hipLaunchKernelGGL(permute_kernel<double>, dim3(grid), dim3(256), 0, s, (const double*)in, (double*)out, p);
  else hipLaunchKernelGGL(permute_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)in, (float*)out, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky-QR with column dropping (batched).
//   column mode:  Y (m x k):  G = Y^H Y = R^H R,  Q = Y R^-1
//   row mode:     X (k x m):  G = X X^H = R^H R,  Q = R^-H X
// Column j is dropped when its Cholesky pivot is <= tau * G_jj(original) or
// not positive (it lies numerically in the span of the earlier columns); R
// keeps a unit diagonal and a zero row there and Q a zero column (row).
// Blocked right-looking factorisation with CB x CB diagonal blocks factored
// in LDS, panels and trailing updates on the matrix cores.
// ---------------------------------------------------------------------------
constexpr int CB = 32;

template <typename T> __device__ inline T czero();
template <> __device__ inline cd czero<cd>() { return cd{0, 0}; }
template <> __device__ inline double czero<double>() { return 0.0; }
__device__ inline cd cconj(cd a) { return conjg(a); }
__device__ inline double cconj(double a) { return a; }
__device__ inline double creal_(cd a) { return a.x; }
__device__ inline double creal_(double a) { return a; }
__device__ inline cd cdiv_real(cd a, double r) { return cd{a.x / r, a.y / r}; }
__device__ inline double cdiv_real(double a, double r) { return a / r; }

template <typename T>
__global__ __launch_bounds__(256) void chol_diag_kernel(T* G, long long ldg, long long sG, int jb, int k,
                                                        const double* diag0, long long sdiag,
                                                        T* RI, long long sRI, double* mask, long long smask,
                                                        double tau) {
  __shared__ T A[CB][CB + 1];
  __shared__ T Ri[CB][CB + 1];
  __shared__ double s_keep[CB];
  const int b = blockIdx.x;
  const int cb = min(CB, k - jb);
  T* Gb = G + b * sG;
  const int t = threadIdx.x;
  for (int idx = t; idx < CB * CB; idx += 256) {
    const int r = idx / CB, c = idx % CB;
    T v = czero<T>();
    if (r < cb && c < cb && r <= c) v = Gb[(long long)(jb + r) * ldg + jb + c];
    A[r][c] = v;
  }
  __syncthreads();
  for (int j = 0; j < cb; ++j) {
    if (t == 0) {
      const double piv = creal_(A[j][j]);
      const double orig = diag0[b * sdiag + jb + j];
      const bool keep = (piv > tau * orig) && (piv > 0.0);
      s_keep[j] = keep ? 1.0 : 0.0;
      if constexpr (sizeof(T) == 16) A[j][j] = cd{keep ? sqrt(piv) : 1.0, 0.0};
      else A[j][j] = keep ? sqrt(piv) : 1.0;
    }
    __syncthreads();
    const bool keep = s_keep[j] != 0.0;
    const double rjj = creal_(A[j][j]);
    for (int c = j + 1 + t; c < cb; c += 256) A[j][c] = keep ? cdiv_real(A[j][c], rjj) : czero<T>();
    __syncthreads();
    for (int idx = t; idx < cb * cb; idx += 256) {
      const int r = idx / cb, c = idx % cb;
      if (r > j && c >= r) A[r][c] = A[r][c] - cconj(A[j][r]) * A[j][c];
    }
    __syncthreads();
  }
  // inverse of the upper-triangular block (one column per thread)
  if (t < cb) {
    const int c = t;
    for (int r = 0; r < CB; ++r) Ri[r][c] = czero<T>();
    if constexpr (sizeof(T) == 16) Ri[c][c] = cd{1.0 / creal_(A[c][c]), 0.0};
    else Ri[c][c] = 1.0 / creal_(A[c][c]);
    for (int r = c - 1; r >= 0; --r) {
      T acc = czero<T>();
      for (int q = r + 1; q <= c; ++q) acc = acc + A[r][q] * Ri[q][c];
      Ri[r][c] = cdiv_real(acc, -creal_(A[r][r]));
    }
  }
  __syncthreads();
  for (int idx = t; idx < cb * cb; idx += 256) {
    const int r = idx / cb, c = idx % cb;
    Gb[(long long)(jb + r) * ldg + jb + c] = (r <= c) ? A[r][c] : czero<T>();
    RI[b * sRI + (long long)r * CB + c] = Ri[r][c];
  }
  if (t < cb) mask[b * smask + jb + t] = s_keep[t];
}

template <typename T>
__global__ void diag_copy_kernel(const T* G, long long ldg, long long sG, int k, double* diag0, long long sdiag) {
  const int b = blockIdx.y;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < k; j += gridDim.x * 256)
    diag0[b * sdiag + j] = creal_(G[b * sG + (long long)j * ldg + j]);
}

__device__ inline void ld2(const double* p, long long i, double& r, double& im) { r = p[i]; im = 0.0; }
__device__ inline void ld2(const cd* p, long long i, double& r, double& im) { r = p[i].x; im = p[i].y; }
__device__ inline void st2(double* p, long long i, double r, double) { p[i] = r; }
__device__ inline void st2(cd* p, long long i, double r, double im) { p[i] = cd{r, im}; }

// G = Y^H Y (column mode) or Y Y^H (row mode), k x k per problem
static hipError_t gram_into(int dt, int mode, const void* Y, long long ldy, long long sY, int m, int k, void* G,
                            int batch, hipStream_t s, void* kws, size_t kws_bytes) {
  GemmArgs g = mode == 0 ? gemm_args(k, k, m, OP_C, OP_N, Y, ldy, Y, ldy, G, k)
                         : gemm_args(k, k, m, OP_N, OP_C, Y, ldy, Y, ldy, G, k);
  g.sA = sY; g.sB = sY; g.sC = (long long)k * k; g.batch = batch;
  g.kws = kws; g.kws_bytes = kws_bytes;
  return gemm(dt, PREC_FP64, g, s);
}

// Squared Frobenius distance of G from the identity over the entries whose
// row and column both belong to non-zero vectors (G_ii > 0 and G_jj > 0):
// block (x, b) sums rows x, x + gridDim.x, ... of problem b into
// part[b * gridDim.x + x].
template <typename T>
__global__ __launch_bounds__(256) void ortho_defect_kernel(const T* G, int k, double* part) {
  __shared__ double sh[4];
  const int b = blockIdx.y;
  const T* g = G + (long long)b * k * k;
  double acc = 0.0;
  for (int i = blockIdx.x; i < k; i += gridDim.x) {
    if (!(creal_(g[(long long)i * k + i]) > 0.0)) continue;
    for (int j = threadIdx.x; j < k; j += 256) {
      if (!(creal_(g[(long long)j * k + j]) > 0.0)) continue;
      double re, im;
      ld2(g, (long long)i * k + j, re, im);
      if (i == j) re -= 1.0;
      acc += re * re + im * im;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// out[0] = max over problems of the sum of that problem's nparts partials
// One thread per problem sums its partials in order (the same sum as a serial
// pass), then the workgroup takes the maximum.
__global__ __launch_bounds__(256) void ortho_defect_final_kernel(const double* part, int nparts, int batch,
                                                                 double* out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int b = tid; b < batch; b += 256) {
    double t = 0.0;
    for (int x = 0; x < nparts; ++x) t += part[(long long)b * nparts + x];
    mx = fmax(mx, t);
  }
  red[tid] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  if (tid == 0) out[0] = red[0];
}

// G <- M = strict upper triangle of G + (diag(G) - 1) / 2, lower triangle zero
// (R - I to first order, for the Cholesky factor R of G = I + E)
template <typename T>
__global__ void first_order_factor_kernel(T* G, int k) {
  T* g = G + (long long)blockIdx.y * k * k;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)k * k; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / k), j = (int)(e % k);
    if (i > j) {
      st2(g, e, 0.0, 0.0);
    } else if (i == j) {
      double re, im;
      ld2(g, e, re, im);
      st2(g, e, 0.5 * (re - 1.0), 0.0);
    }
  }
}

hipError_t ortho_defect(int dtype, int mode, const void* Y, long long ldy, long long sY, int m, int k, void* G,
                        double* part, double* out, int batch, hipStream_t s, void* kws, size_t kws_bytes) {
  if (k <= 0 || m <= 0 || batch <= 0) return hipErrorInvalidValue;
  if (dtype != C128 && dtype != F64) return hipErrorInvalidValue;
  hipError_t e = gram_into(dtype, mode, Y, ldy, sY, m, k, G, batch, s, kws, kws_bytes);
  if (e != hipSuccess) return e;
  const int np = ORTHO_DEFECT_PARTS;
  if (dtype == C128)
    hipLaunchKernelGGL(ortho_defect_kernel<cd>, dim3(np, batch), dim3(256), 0, s, (const cd*)G, k, part);
  else
    hipLaunchKernelGGL(ortho_defect_kernel<double>, dim3(np, batch), dim3(256), 0, s, (const double*)G, k, part);
  hipLaunchKernelGGL(ortho_defect_final_kernel, dim3(1), dim3(256), 0, s, part, np, batch, out);
  return hipGetLastError();
}

// G <- C = M + N - M M (upper triangular), with M from first_order_factor_kernel
// in G, P = M^H M and S = M M: N = -(strict upper triangle of P + diag(P) / 2)
// is the second-order term of the Cholesky factor, R = I + M + N + O(E^3),
// and R^-1 = I - C + O(E^3).
template <typename T>
__global__ void second_order_factor_kernel(T* G, const T* P, const T* S, int k) {
  const long long off = (long long)blockIdx.y * k * k;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < (long long)k * k; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / k), j = (int)(e % k);
    if (i > j) continue;
    double mr, mi, pr, pi, sr, si;
    ld2(G + off, e, mr, mi);
    ld2(P + off, e, pr, pi);
    ld2(S + off, e, sr, si);
    if (i == j) { pr *= 0.5; pi = 0.0; }
    st2(G + off, e, mr - pr - sr, mi - pi - si);
  }
}

hipError_t first_order_orthonormalise(int dtype, int mode, const void* Y, long long ldy, long long sY, int m, int k,
                                      void* G, void* X, int batch, hipStream_t s, void* kws, size_t kws_bytes) {
  if (k <= 0 || m <= 0 || batch <= 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min<long long>(1024, ((long long)k * k + 255) / 256);
  if (dtype == C128)
    hipLaunchKernelGGL(first_order_factor_kernel<cd>, dim3(gx, batch), dim3(256), 0, s, (cd*)G, k);
  else if (dtype == F64)
    hipLaunchKernelGGL(first_order_factor_kernel<double>, dim3(gx, batch), dim3(256), 0, s, (double*)G, k);
  else
    return hipErrorInvalidValue;
  // column mode: X = Y - Y M; row mode: X = Y - M^H Y (X holds Y on entry)
  GemmArgs g = mode == 0 ? gemm_args(m, k, k, OP_N, OP_N, Y, ldy, G, k, X, ldy)
                         : gemm_args(k, m, k, OP_C, OP_N, G, k, Y, ldy, X, ldy);
  g.sA = mode == 0 ? sY : (long long)k * k;
  g.sB = mode == 0 ? (long long)k * k : sY;
  g.sC = sY; g.batch = batch;
  g.alpha_re = -1.0; g.beta_re = 1.0;
  g.kws = kws; g.kws_bytes = kws_bytes;
  return gemm(dtype, PREC_FP64, g, s);
}

hipError_t second_order_orthonormalise(int dtype, int mode, const void* Y, long long ldy, long long sY, int m,
                                       int k, void* G, void* PS, void* X, int batch, hipStream_t s, void* kws,
                                       size_t kws_bytes) {
  if (k <= 0 || m <= 0 || batch <= 0) return hipSuccess;
  if (dtype != C128 && dtype != F64) return hipErrorInvalidValue;
  const size_t es = dtype == C128 ? 16 : 8;
  const long long kk = (long long)k * k;
  const unsigned gx = (unsigned)std::min<long long>(1024, (kk + 255) / 256);
  if (dtype == C128)
    hipLaunchKernelGGL(first_order_factor_kernel<cd>, dim3(gx, batch), dim3(256), 0, s, (cd*)G, k);
  else
    hipLaunchKernelGGL(first_order_factor_kernel<double>, dim3(gx, batch), dim3(256), 0, s, (double*)G, k);
  char* P = static_cast<char*>(PS);
  char* S = P + es * (size_t)kk * batch;
  // P = M^H M, S = M M
  GemmArgs gp = gemm_args(k, k, k, OP_C, OP_N, G, k, G, k, P, k);
  gp.sA = kk; gp.sB = kk; gp.sC = kk; gp.batch = batch;
  gp.kws = kws; gp.kws_bytes = kws_bytes;
  hipError_t e = gemm(dtype, PREC_FP64, gp, s);
  if (e != hipSuccess) return e;
  GemmArgs gs = gemm_args(k, k, k, OP_N, OP_N, G, k, G, k, S, k);
  gs.sA = kk; gs.sB = kk; gs.sC = kk; gs.batch = batch;
  gs.kws = kws; gs.kws_bytes = kws_bytes;
  e = gemm(dtype, PREC_FP64, gs, s);
  if (e != hipSuccess) return e;
  if (dtype == C128)
    hipLaunchKernelGGL(second_order_factor_kernel<cd>, dim3(gx, batch), dim3(256), 0, s, (cd*)G, (const cd*)P,
                       (const cd*)S, k);
  else
    hipLaunchKernelGGL(second_order_factor_kernel<double>, dim3(gx, batch), dim3(256), 0, s, (double*)G,
                       (const double*)P, (const double*)S, k);
  // column mode: X = Y - Y C; row mode: X = Y - C^H Y (X holds Y on entry)
  GemmArgs g = mode == 0 ? gemm_args(m, k, k, OP_N, OP_N, Y, ldy, G, k, X, ldy)
                         : gemm_args(k, m, k, OP_C, OP_N, G, k, Y, ldy, X, ldy);
  g.sA = mode == 0 ? sY : kk;
  g.sB = mode == 0 ? kk : sY;
  g.sC = sY; g.batch = batch;
  g.alpha_re = -1.0; g.beta_re = 1.0;
  g.kws = kws; g.kws_bytes = kws_bytes;
  return gemm(dtype, PREC_FP64, g, s);
}

template <typename T>
static hipError_t cholqr_impl(int mode, void* Y, long long ldy, long long sY, int m, int k, void* Q,
                              long long ldq, long long sQ, CholWork w, double tau, int batch, hipStream_t s,
                              bool have_gram) {
  const int dt = LT<T>::dtype;
  const size_t es = sizeof(T);
  char* G = reinterpret_cast<char*>(w.G);
  const long long ldg = k, sG = (long long)k * k;
  hipError_t err = hipSuccess;
  if (!have_gram) {
    err = gram_into(dt, mode, Y, ldy, sY, m, k, G, batch, s, w.kws, w.kws_bytes);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(diag_copy_kernel<T>, dim3((k + 255) / 256, batch), dim3(256), 0, s, (const T*)G, ldg, sG,
                     k, w.diag0, (long long)k);
  const int nblk = (k + CB - 1) / CB;
  char* RI = reinterpret_cast<char*>(w.RI);
  const long long sRI = (long long)nblk * CB * CB;
  for (int ib = 0; ib < nblk; ++ib) {
    const int jb = ib * CB, cb = std::min(CB, k - jb), rest = k - jb - cb;
    hipLaunchKernelGGL(chol_diag_kernel<T>, dim3(batch), dim3(256), 0, s, (T*)G, ldg, sG, jb, k, w.diag0,
                       (long long)k, (T*)(RI + (size_t)ib * CB * CB * es), sRI, w.mask, (long long)k, tau);
    if (rest > 0) {
      // R(jb, jb+cb:) = Rjj^-H G(jb, jb+cb:), dropped rows zeroed
      GemmArgs p = gemm_args(cb, rest, cb, OP_C, OP_N, RI + (size_t)ib * CB * CB * es, CB,
                             G + ((long long)jb * ldg + jb + cb) * es, ldg,
                             G + ((long long)jb * ldg + jb + cb) * es, ldg);
      p.sA = sRI; p.sB = sG; p.sC = sG; p.batch = batch;
      p.rs = w.mask + jb; p.s_rs = k;
      err = gemm(dt, PREC_FP64, p, s);
      if (err != hipSuccess) return err;
      // trailing: G(jb+cb:, jb+cb:) -= R(jb, jb+cb:)^H R(jb, jb+cb:)
      GemmArgs t = gemm_args(rest, rest, cb, OP_C, OP_N, G + ((long long)jb * ldg + jb + cb) * es, ldg,
                             G + ((long long)jb * ldg + jb + cb) * es, ldg,
                             G + ((long long)(jb + cb) * ldg + jb + cb) * es, ldg);
      t.sA = sG; t.sB = sG; t.sC = sG; t.batch = batch;
      t.alpha_re = -1.0; t.beta_re = 1.0;
      err = gemm(dt, PREC_FP64, t, s);
      if (err != hipSuccess) return err;
    }
  }
  // triangular solve, block by block; Y is consumed as workspace.  The
  // updates from earlier blocks are applied per TS_OUTER rows (columns) in one
  // product of full-height tiles, then per CB block from inside the outer block.
  constexpr int TS_OUTER = 128;
  char* Yc = reinterpret_cast<char*>(Y);
  char* Qc = reinterpret_cast<char*>(Q);
  for (int ob = 0; ob < k; ob += TS_OUTER) {
    const int ocb = std::min(TS_OUTER, k - ob);
    if (ob > 0) {
      GemmArgs o = mode == 0
          // Y(:, ob:ob+ocb) -= Q(:, :ob) R(:ob, ob:ob+ocb)
          ? gemm_args(m, ocb, ob, OP_N, OP_N, Qc, ldq, G + (long long)ob * es, ldg, Yc + (long long)ob * es, ldy)
          // X(ob:ob+ocb, :) -= R(:ob, ob:ob+ocb)^H Q(:ob, :)
          : gemm_args(ocb, m, ob, OP_C, OP_N, G + (long long)ob * es, ldg, Qc, ldq,
                      Yc + (long long)ob * ldy * es, ldy);
      o.sA = mode == 0 ? sQ : sG;
      o.sB = mode == 0 ? sG : sQ;
      o.sC = sY; o.batch = batch;
      o.alpha_re = -1.0; o.beta_re = 1.0;
      o.kws = w.kws; o.kws_bytes = w.kws_bytes;
      err = gemm(dt, PREC_FP64, o, s);
      if (err != hipSuccess) return err;
    }
    for (int jb = ob; jb < ob + ocb; jb += CB) {
      const int ib = jb / CB, cb = std::min(CB, k - jb), kin = jb - ob;
      if (mode == 0) {
        if (kin > 0) {
          // Y(:, jb) -= Q(:, ob:jb) R(ob:jb, jb)
          GemmArgs a1 = gemm_args(m, cb, kin, OP_N, OP_N, Qc + (long long)ob * es, ldq,
                                  G + ((long long)ob * ldg + jb) * es, ldg, Yc + (long long)jb * es, ldy);
          a1.sA = sQ; a1.sB = sG; a1.sC = sY; a1.batch = batch;
          a1.alpha_re = -1.0; a1.beta_re = 1.0;
          err = gemm(dt, PREC_FP64, a1, s);
          if (err != hipSuccess) return err;
        }
        // Q(:, jb) = Y(:, jb) Rjj^-1, dropped columns zeroed
        GemmArgs a2 = gemm_args(m, cb, cb, OP_N, OP_N, Yc + (long long)jb * es, ldy, RI + (size_t)ib * CB * CB * es,
                                CB, Qc + (long long)jb * es, ldq);
        a2.sA = sY; a2.sB = sRI; a2.sC = sQ; a2.batch = batch;
        a2.cs = w.mask + jb; a2.s_cs = k;
        err = gemm(dt, PREC_FP64, a2, s);
        if (err != hipSuccess) return err;
      } else {
        if (kin > 0) {
          // X(jb, :) -= R(ob:jb, jb)^H Q(ob:jb, :)
          GemmArgs a1 = gemm_args(cb, m, kin, OP_C, OP_N, G + ((long long)ob * ldg + jb) * es, ldg,
                                  Qc + (long long)ob * ldq * es, ldq, Yc + (long long)jb * ldy * es, ldy);
          a1.sA = sG; a1.sB = sQ; a1.sC = sY; a1.batch = batch;
          a1.alpha_re = -1.0; a1.beta_re = 1.0;
          err = gemm(dt, PREC_FP64, a1, s);
          if (err != hipSuccess) return err;
        }
        // Q(jb, :) = Rjj^-H X(jb, :), dropped rows zeroed
        GemmArgs a2 = gemm_args(cb, m, cb, OP_C, OP_N, RI + (size_t)ib * CB * CB * es, CB,
                                Yc + (long long)jb * ldy * es, ldy, Qc + (long long)jb * ldq * es, ldq);
        a2.sA = sRI; a2.sB = sY; a2.sC = sQ; a2.batch = batch;
        a2.rs = w.mask + jb; a2.s_rs = k;
        err = gemm(dt, PREC_FP64, a2, s);
        if (err != hipSuccess) return err;
      }
    }
  }
  return hipGetLastError();
}

hipError_t cholqr(int dtype, int mode, void* Y, long long ldy, long long sY, int m, int k, void* Q,
                  long long ldq, long long sQ, CholWork w, double tau, int batch, hipStream_t s, bool have_gram) {
  if (k <= 0 || m <= 0 || batch <= 0) return hipSuccess;
  if (dtype == C128) return cholqr_impl<cd>(mode, Y, ldy, sY, m, k, Q, ldq, sQ, w, tau, batch, s, have_gram);
  if (dtype == F64) return cholqr_impl<double>(mode, Y, ldy, sY, m, k, Q, ldq, sQ, w, tau, batch, s, have_gram);
  return hipErrorInvalidValue;
}

size_t cholqr_work_elems(int k) {
  const int nblk = (k + CB - 1) / CB;
  return (size_t)k * k + (size_t)nblk * CB * CB;
}

}  // namespace tci
