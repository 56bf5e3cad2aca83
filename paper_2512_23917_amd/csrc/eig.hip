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
#include "vecops.hpp"
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
__device__ inline double shfl_xor_t(double v, int m) { return __shfl_xor(v, m); }
__device__ inline cd shfl_xor_t(cd v, int m) { return cd{__shfl_xor(v.x, m), __shfl_xor(v.y, m)}; }
__device__ inline double wsum(double v) { return wave_sum(v); }
__device__ inline cd wsum(cd v) { return cd{wave_sum(v.x), wave_sum(v.y)}; }
__device__ inline double bsum(double v, double* sh) { return block_sum(v, sh); }
__device__ inline cd bsum(cd v, double* sh) {
  const double a = block_sum(v.x, sh);
  const double b = block_sum(v.y, sh);
  return cd{a, b};
}

// ---------------------------------------------------------------------------
// Per-column kernels of the blocked reduction (LAPACK latrd organisation,
// lower storage, panel of NB columns starting at j0; p = i - j0):
//
//  colA (row blocks of TT rows over [row0, n)):
//    finish w_ip (ip = i-1): with t1 = W^H v, t2 = V^H v and yv = v^H A22 v
//      (summed here from the chunk partials of the previous colC),  alpha = -|tau|^2/2 (yv - t1^H t2 - t2^H t1),
//      w(r) = tau (y(r) - V(r,:) t1 - W(r,:) t2) + alpha v(r),  y(r) = sum_t P[t][r];
//    update column i: a(r,i) -= V(r,:) conj(W(i,:)) + W(r,:) conj(V(i,:));
//    d_i = Re a(i,i); one partial of ||a(i+2:n,i)||^2 per workgroup.
//  colC (lower-triangle tiles TT x TT of the trailing matrix, CH tiles of a
//    block row per workgroup):
//    reflector of a(i+1:n,i): beta = -sign(Re a) ||.||, tau = (beta - a)/beta,
//    v = [1, x / (a - beta)];  the chunk of tiles (R, cA..cB) adds
//    sum_C A_RC v_C to P[cA][R rows], and each tile with C < R adds A_RC^H v_R
//    to P[R][C rows]; partial quadratic form v^H A v and, with the diagonal
//    tile, t1 = W^H v and t2 = V^H v over its rows, one partial per chunk.
// Every tile of the lower triangle is read once per column.  Partials are
// summed by the kernel that consumes them (colC sums colA's norm partials,
// colA the chunk partials of colC): the kernel boundary makes them visible,
// and no workgroup waits on a device-scope fence, which on this chip writes
// back the L2 of its XCD.
// ---------------------------------------------------------------------------
constexpr int TT = 64;
static_assert(TRIDIAG_BAND >= TT, "the reduction reads whole diagonal tiles");

template <typename T, int NB>
struct TriWs {
  // byte offsets inside one problem's workspace
  __host__ __device__ static size_t xv(int) { return 0; }
  __host__ __device__ static size_t P(int n) { return align(sizeof(T) * (size_t)n); }
  __host__ __device__ static size_t pa(int n) { return P(n) + align(sizeof(T) * (size_t)nbt(n) * n); }
  __host__ __device__ static size_t pc(int n) { return pa(n) + align(sizeof(double) * (size_t)nbt(n)); }
  // [V_panel; W^T] and [W^T; V_panel], 2 NB rows of n each: operands of the
  // fused rank-2NB trailing update
  __host__ __device__ static size_t cat1(int n) { return pc(n) + align(sizeof(T) * (size_t)ntile(n) * (1 + 2 * NB)); }
  __host__ __device__ static size_t cat2(int n) { return cat1(n) + align(sizeof(T) * (size_t)2 * NB * n); }
  __host__ __device__ static size_t bytes(int n) { return cat2(n) + align(sizeof(T) * (size_t)2 * NB * n); }
  __host__ __device__ static int nbt(int n) { return (n + TT - 1) / TT; }
  __host__ __device__ static int ntile(int n) { return nbt(n) * (nbt(n) + 1) / 2; }
  __host__ __device__ static size_t align(size_t x) { return (x + 255) & ~size_t(255); }
};

// Tiles per workgroup of the trailing matvec: band R (rows R*TT ...) is cut
// into chunks of up to CH consecutive tiles C, and one workgroup handles one
// chunk, so that the reflector set-up and the final reduction are paid once
// per chunk.  The row sums of a chunk starting at tile cA go to P[cA][rows];
// the column sums of an off-diagonal tile (R, C) go to P[R][columns of C].
constexpr int CH = 32;

__host__ __device__ inline int tri_chunks(int nact) {
  int k = 0;
  for (int t = 1; t <= nact; ++t) k += (t + CH - 1) / CH;
  return k;
}

// Is P[t][r] written in the column step whose first active block is b0?
__device__ inline bool tri_slot_used(int t, int r, int b0) {
  const int Rr = r / TT;
  return t > Rr || ((t - b0) % CH == 0);
}

// Sum of a per-thread complex / real value over groups of 4 consecutive lanes.
template <typename T>
__device__ inline T quad_sum(T v) {
  if constexpr (sizeof(T) == 16) {
    double r = v.x, i = v.y;
    r += __shfl_xor(r, 1);
    i += __shfl_xor(i, 1);
    r += __shfl_xor(r, 2);
    i += __shfl_xor(i, 2);
    return cd{r, i};
  } else {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    return v;
  }
}

// Reflector scalars from ||x(i+2:n)||^2 and alpha = x(i+1).
template <typename T>
__device__ inline void reflector(T alpha, double xn2, double& beta, T& tau, T& scal) {
  const double ar = re(alpha), ai = im(alpha);
  if (xn2 == 0.0 && ai == 0.0) {
    beta = ar;
    tau = EigT<T>::zero();
    scal = EigT<T>::zero();
    return;
  }
  const double nrm = sqrt(ar * ar + ai * ai + xn2);
  beta = ar >= 0.0 ? -nrm : nrm;
  if constexpr (sizeof(T) == sizeof(double)) {
    tau = (beta - ar) / beta;
    scal = 1.0 / (ar - beta);
  } else {
    tau = cd{(beta - ar) / beta, -ai / beta};
    const double xr = ar - beta, xi = ai, den = xr * xr + xi * xi;
    scal = cd{xr / den, -xi / den};
  }
}

// Sum of one value per thread over a 256-thread block (wave shuffles, then
// the four wave sums through LDS); every thread receives the total.
template <typename T>
__device__ inline T block_sum256(T v, T* sh4) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  return add(add(sh4[0], sh4[1]), add(sh4[2], sh4[3]));
}

// Sum over the four thread groups part = tid >> 6 that share a row
// (tid & 63): the result is valid in part 0.
template <typename T>
__device__ inline T parts_sum(T v, T* sh256) {
  __syncthreads();
  sh256[threadIdx.x] = v;
  __syncthreads();
  T r = v;
  if (threadIdx.x < 64) r = add(add(sh256[threadIdx.x], sh256[threadIdx.x + 64]),
                                add(sh256[threadIdx.x + 128], sh256[threadIdx.x + 192]));
  return r;
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void tri_colA_kernel(TriArgs a, int row0, int icol, int ifin, int j0) {
  __shared__ T s_t1[NB], s_t2[NB], s_vrow[NB], s_wrow[NB];
  __shared__ T s_alpha, s_wi;
  __shared__ T s_fc[1 + 2 * NB];
  __shared__ T s_red[256];
  __shared__ T s_sh4[4];
  __shared__ double red[256];
  const int b = blockIdx.y, n = a.n, tid = threadIdx.x;
  char* ws = reinterpret_cast<char*>(a.ws) + b * a.sws;
  T* xv = reinterpret_cast<T*>(ws + TriWs<T, NB>::xv(n));
  const T* P = reinterpret_cast<const T*>(ws + TriWs<T, NB>::P(n));
  double* pa = reinterpret_cast<double*>(ws + TriWs<T, NB>::pa(n));
  const T* pc_in = reinterpret_cast<const T*>(ws + TriWs<T, NB>::pc(n));
  T* G = reinterpret_cast<T*>(a.G) + b * a.sG;
  T* V = reinterpret_cast<T*>(a.Vt) + b * a.sVt;
  T* W = reinterpret_cast<T*>(a.Wp) + b * a.sWp;
  const T* Y = reinterpret_cast<const T*>(a.y) + b * a.sy;
  const long ldg = a.ldg;
  const int rlo = row0 + blockIdx.x * TT;          // first row of this block
  const int r = rlo + (tid & (TT - 1));            // row of this thread (4 threads per row)
  const int part = tid >> 6;                       // 0..3
  const bool rv = r < n;

  // ---- finish w_ifin (panel column pp = ifin - j0) on rows >= ifin + 1 = row0
  if (ifin >= 0) {
    const int pp = ifin - j0;
    // reduce the chunk partials of the trailing matvec of column ifin (one
    // value per thread; the kernel boundary made them visible)
    if (tid < 1 + 2 * NB) {
      const int nwg = tri_chunks(TriWs<T, NB>::nbt(n) - (ifin + 1) / TT);
      // loads in groups of 8 (one wait per group), sums in chunk order
      T acc = EigT<T>::zero();
      int k = 0;
      for (; k + 8 <= nwg; k += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pc_in[(long)(k + u) * (1 + 2 * NB) + tid];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = add(acc, v[u]);
      }
      for (; k < nwg; ++k) acc = add(acc, pc_in[(long)k * (1 + 2 * NB) + tid]);
      s_fc[tid] = acc;
    }
    __syncthreads();
    if (tid < pp) { s_t1[tid] = s_fc[1 + tid]; s_t2[tid] = s_fc[1 + NB + tid]; }
    __syncthreads();
    if (tid == 0) {
      const T taup = reinterpret_cast<const T*>(a.tau)[b * a.stau + ifin];
      T yv = s_fc[0];
      for (int q = 0; q < pp; ++q) {
        yv = sub(yv, mulr(cj(s_t1[q]), s_t2[q]));
        yv = sub(yv, mulr(cj(s_t2[q]), s_t1[q]));
      }
      s_alpha = scl(-0.5 * nrm2(taup), yv);
    }
    __syncthreads();
    const T taup = reinterpret_cast<const T*>(a.tau)[b * a.stau + ifin];
    const T alpha = s_alpha;
    const int tb0 = (ifin + 1) / TT, nbt = TriWs<T, NB>::nbt(n);
    const T* vfin = V + (long)ifin * n;
    // w for this thread's row (4 threads share a row: each sums a quarter)
    T acc = EigT<T>::zero();
    if (rv) {
      // slots t = tb0 + part, +4, ...: loaded four at a time (every address
      // is valid), the unused ones dropped, sums in slot order
      int t = tb0 + part;
      for (; t + 12 < nbt; t += 16) {
        T pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pv[u] = P[(long)(t + 4 * u) * n + r];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (tri_slot_used(t + 4 * u, r, tb0)) acc = add(acc, pv[u]);
      }
      for (; t < nbt; t += 4)
        if (tri_slot_used(t, r, tb0)) acc = add(acc, P[(long)t * n + r]);
#pragma unroll 4
      for (int q = part; q < pp; q += 4) {
        acc = sub(acc, mulr(V[(long)(j0 + q) * n + r], s_t1[q]));
        acc = sub(acc, mulr(W[(long)r * NB + q], s_t2[q]));
      }
    }
    const T yy = parts_sum(acc, s_red);
    if (part == 0 && rv) {
      const T w = add(mulr(taup, yy), mulr(alpha, vfin[r]));
      W[(long)r * NB + pp] = w;
    }
    // rows above ifin + 1 carry a zero w
    if (blockIdx.x == 0)
      for (int q = tid; q < row0; q += 256) W[(long)q * NB + pp] = EigT<T>::zero();
    __syncthreads();
  }
  if (icol < 0) return;

  // ---- column update of icol (row0 == icol) with p panel columns
  const int i = icol, p = i - j0;
  // row i of V and W (W(i, p-1) was just finished by the workgroup owning row i:
  // recompute it here so that every workgroup has it without a grid-wide wait)
  if (tid < p) {
    s_vrow[tid] = V[(long)(j0 + tid) * n + i];
    if (tid < p - 1 || ifin < 0) s_wrow[tid] = W[(long)i * NB + tid];
  }
  if (ifin >= 0 && p >= 1) {
    // W(i, p-1): same formula as above for row i
    const int pp = p - 1;
    T acc = EigT<T>::zero();
    const int tb0 = (ifin + 1) / TT, nbt = TriWs<T, NB>::nbt(n);
    for (int t = tb0 + tid; t < nbt; t += 256)
      if (tri_slot_used(t, i, tb0)) acc = add(acc, P[(long)t * n + i]);
    if (tid < pp) {
      acc = sub(acc, mulr(V[(long)(j0 + tid) * n + i], s_t1[tid]));
      acc = sub(acc, mulr(W[(long)i * NB + tid], s_t2[tid]));
    }
    const T yy = block_sum256(acc, s_sh4);
    if (tid == 0) {
      const T taup = reinterpret_cast<const T*>(a.tau)[b * a.stau + ifin];
      s_wi = add(mulr(taup, yy), mulr(s_alpha, V[(long)ifin * n + i]));
      s_wrow[pp] = s_wi;
    }
  }
  __syncthreads();
  double xn2 = 0.0;
  {
    // the four groups of a row share the p panel terms
    T acc = (part == 0 && rv) ? G[(long)r * ldg + i] : EigT<T>::zero();
    if (rv) {
#pragma unroll 4
      for (int q = part; q < p; q += 4) {
        acc = sub(acc, mulr(V[(long)(j0 + q) * n + r], cj(s_wrow[q])));
        acc = sub(acc, mulr(W[(long)r * NB + q], cj(s_vrow[q])));
      }
    }
    acc = parts_sum(acc, s_red);
    if (part == 0 && rv) {
      G[(long)r * ldg + i] = acc;
      if (r >= i + 1) xv[r] = acc;
      if (r >= i + 2) xn2 = nrm2(acc);
      if (r == i) a.d[b * a.sde + i] = re(acc);
    }
  }
  // ||x||^2 partial of this block (summed by the next kernel)
  const double xsum = block_sum256(xn2, red);
  if (tid == 0 && i + 1 < n) pa[blockIdx.x] = xsum;
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void tri_colC_kernel(TriArgs a, int i, int j0) {
  __shared__ T s_vR[TT];
  __shared__ T s_q[4];
  __shared__ T s_colsum[2][4][TT];
  __shared__ T s_tt[4][2 * NB];
  static_assert(2 * NB == TT, "t1/t2 thread mapping assumes 2 NB == TT");
  __shared__ T s_scal;
  const int b = blockIdx.x, n = a.n, tid = threadIdx.x;
  const int wg = (int)gridDim.y - 1 - (int)blockIdx.y;   // chunk: largest bands first
  const int p = i - j0;
  char* ws = reinterpret_cast<char*>(a.ws) + b * a.sws;
  const T* xv = reinterpret_cast<const T*>(ws + TriWs<T, NB>::xv(n));
  T* P = reinterpret_cast<T*>(ws + TriWs<T, NB>::P(n));
  T* pc = reinterpret_cast<T*>(ws + TriWs<T, NB>::pc(n));
  const double* pa = reinterpret_cast<const double*>(ws + TriWs<T, NB>::pa(n));
  const T* G = reinterpret_cast<const T*>(a.G) + b * a.sG;
  T* V = reinterpret_cast<T*>(a.Vt) + b * a.sVt;
  const T* W = reinterpret_cast<const T*>(a.Wp) + b * a.sWp;
  // chunk -> (band R, first tile cA, last tile cB)
  const int b0 = (i + 1) / TT;
  int k = wg, R = b0;
  for (;;) {
    const int nch = (R - b0 + CH) / CH;
    if (k < nch) break;
    k -= nch;
    ++R;
  }
  const int cA = b0 + k * CH, cB = min(R, cA + CH - 1);
  const bool has_diag = (cB == R);
  // reflector scalars (every workgroup computes them from the norm partials of
  // the column kernel, one per block of TT rows from row i)
  double xn2 = 0.0;
  if (tid < 64) {
    const int na = (n - i + TT - 1) / TT;
    for (int k = tid; k < na; k += 64) xn2 += pa[k];
    xn2 = wave_sum(xn2);
  }
  if (tid == 0) {
    double beta;
    T tv, sc;
    reflector(xv[i + 1], xn2, beta, tv, sc);
    s_scal = sc;
    if (wg == 0) {
      a.e[b * a.sde + i] = beta;
      reinterpret_cast<T*>(a.tau)[b * a.stau + i] = tv;
    }
  }
  __syncthreads();
  const T scal = s_scal;
  auto vval = [&](int c) -> T {
    if (c <= i || c >= n) return EigT<T>::zero();
    if (c == i + 1) return EigT<T>::one();
    return mulr(xv[c], scal);
  };
  if (tid < TT) s_vR[tid] = vval(R * TT + tid);
  __syncthreads();
  // reflector i into Vt (the chunk holding the diagonal tile owns band R's
  // rows; chunk 0 zeroes the rows above the active blocks)
  if (has_diag && tid < TT) {
    const int rr = R * TT + tid;
    if (rr < n) V[(long)i * n + rr] = s_vR[tid];
  }
  if (wg == 0)
    for (int rr = tid; rr < b0 * TT; rr += 256) V[(long)i * n + rr] = EigT<T>::zero();

  const int cl = tid & 63, rg = tid >> 6;
  // row-sum accumulators of the two row halves (diagonal / off-diagonal tiles)
  T rs_off0 = EigT<T>::zero(), rs_off1 = EigT<T>::zero();
  T rs_dg0 = EigT<T>::zero(), rs_dg1 = EigT<T>::zero();
#pragma unroll 1
  for (int C = cA; C <= cB; ++C) {
    const bool diag = (C == R);
    const int c = C * TT + cl;
    const bool cok = (c > i) && (c < n);
    const T vc = vval(c);
    T colacc = EigT<T>::zero();
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      T ps[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int rl = rg + 4 * (kk + 8 * h);
        const int r = R * TT + rl;
        T g = EigT<T>::zero();
        if (cok && r > i && r < n) g = G[(long)r * a.ldg + c];
        ps[kk] = mulr(g, vc);                           // row-sum term
        colacc = add(colacc, mulr(cj(g), s_vR[rl]));    // column-sum term
      }
      // butterfly over lane bits 5..3 leaves lane l the partial of
      // kk = (l >> 3) & 7 over 8 lanes; bits 2..0 finish the sum
#pragma unroll
      for (int half = 4, bit = 32; half >= 1; half >>= 1, bit >>= 1) {
        const bool hi = (cl & bit) != 0;
#pragma unroll
        for (int t = 0; t < half; ++t) {
          const T mine = hi ? ps[t + half] : ps[t];
          const T other = hi ? ps[t] : ps[t + half];
          ps[t] = add(mine, shfl_xor_t(other, bit));
        }
      }
      T v = add(ps[0], shfl_xor_t(ps[0], 4));
      v = add(v, shfl_xor_t(v, 2));
      v = add(v, shfl_xor_t(v, 1));
      if (diag) {
        if (h == 0) rs_dg0 = add(rs_dg0, v);
        else rs_dg1 = add(rs_dg1, v);
      } else {
        if (h == 0) rs_off0 = add(rs_off0, v);
        else rs_off1 = add(rs_off1, v);
      }
    }
    if (!diag) {
      const int sb = (C - cA) & 1;
      s_colsum[sb][rg][cl] = colacc;
      __syncthreads();
      if (tid < TT) {
        const T cs = add(add(s_colsum[sb][0][tid], s_colsum[sb][1][tid]),
                         add(s_colsum[sb][2][tid], s_colsum[sb][3][tid]));
        const int cc = C * TT + tid;
        if (cc < n) P[(long)R * n + cc] = cs;
      }
    } else {
      // t1 = W^H v and t2 = V^H v over the diagonal tile's rows: thread
      // (q, part), q < NB for W's column q, q >= NB for V's row q - NB
      const int q = tid & 63, part = tid >> 6, qq = q & (NB - 1);
      T acc = EigT<T>::zero();
      if (qq < p) {
#pragma unroll 4
        for (int kk = 0; kk < TT / 4; ++kk) {
          const int rl = part * (TT / 4) + kk, r = R * TT + rl;
          if (r > i && r < n) {
            const T other = q < NB ? W[(long)r * NB + qq] : V[(long)(j0 + qq) * n + r];
            acc = add(acc, mulr(cj(other), s_vR[rl]));
          }
        }
      }
      s_tt[part][q] = acc;
    }
  }
  // row sums of the chunk -> P[cA][rows]; quadratic-form pieces
  T qd = EigT<T>::zero(), qo = EigT<T>::zero();
  if ((cl & 7) == 0) {
    const int rl0 = rg + 4 * ((cl >> 3) & 7), rl1 = rl0 + 32;
    const int r0 = R * TT + rl0, r1 = R * TT + rl1;
    if (r0 < n) P[(long)cA * n + r0] = add(rs_dg0, rs_off0);
    if (r1 < n) P[(long)cA * n + r1] = add(rs_dg1, rs_off1);
    qd = add(mulr(cj(s_vR[rl0]), rs_dg0), mulr(cj(s_vR[rl1]), rs_dg1));
    qo = add(mulr(cj(s_vR[rl0]), rs_off0), mulr(cj(s_vR[rl1]), rs_off1));
  }
  qd = wsum(qd);
  qo = wsum(qo);
  if (cl == 0) s_q[rg] = add(add(qd, qo), cj(qo));
  __syncthreads();
  T* mypc = pc + (long)wg * (1 + 2 * NB);
  if (tid == 0) mypc[0] = add(add(s_q[0], s_q[1]), add(s_q[2], s_q[3]));
  if (tid < 2 * NB)
    mypc[1 + tid] = has_diag ? add(add(s_tt[0][tid], s_tt[1][tid]), add(s_tt[2][tid], s_tt[3][tid]))
                             : EigT<T>::zero();
}

// Operands of the trailing update G -= V W^H + W V^H = [V W] [W V]^H over
// rows and columns >= t: cat1 = [V_panel; W^T], cat2 = [W^T; V_panel] (rows
// q < pe from V_panel = Vt rows j0 .., from W^T = W columns), columns >= t.
template <typename T, int NB>
__global__ __launch_bounds__(256) void tri_cat_kernel(TriArgs a, int j0, int pe, int t) {
  const int b = blockIdx.y, n = a.n;
  char* ws = reinterpret_cast<char*>(a.ws) + b * a.sws;
  T* c1 = reinterpret_cast<T*>(ws + TriWs<T, NB>::cat1(n));
  T* c2 = reinterpret_cast<T*>(ws + TriWs<T, NB>::cat2(n));
  const T* V = reinterpret_cast<const T*>(a.Vt) + b * a.sVt;
  const T* W = reinterpret_cast<const T*>(a.Wp) + b * a.sWp;
  const long long tot = (long long)pe * (n - t);
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int q = (int)(e / (n - t)), r = t + (int)(e % (n - t));
    const T v = V[(long)(j0 + q) * n + r];
    const T w = W[(long)r * NB + q];
    c1[(long)q * n + r] = v;
    c1[(long)(pe + q) * n + r] = w;
    c2[(long)q * n + r] = w;
    c2[(long)(pe + q) * n + r] = v;
  }
}

template <typename T, int NB>
static hipError_t tridiag_impl(const TriArgs& a, int batch, hipStream_t s) {
  const int n = a.n;
  const size_t es = sizeof(T);
  const int nbt = TriWs<T, NB>::nbt(n);
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int pe = min(NB, n - j0);
    for (int p = 0; p < pe; ++p) {
      const int i = j0 + p;
      const int rowsA = n - i;
      hipLaunchKernelGGL((tri_colA_kernel<T, NB>), dim3((rowsA + TT - 1) / TT, batch), dim3(256), 0, s, a, i, i,
                         p > 0 ? i - 1 : -1, j0);
      if (i + 1 < n) {
        const int nact = nbt - (i + 1) / TT;
        // algorithmic bytes: the lower triangle of the trailing matrix read once
        ProfScope ps(s, 0.5 * (double)(n - i - 1) * (n - i) * sizeof(T) * batch, "hemv");
        hipLaunchKernelGGL((tri_colC_kernel<T, NB>), dim3(batch, tri_chunks(nact)), dim3(256), 0, s, a, i, j0);
      }
    }
    const int t = j0 + pe;
    if (t < n) {
      // finish w of the panel's last column, then the trailing update
      hipLaunchKernelGGL((tri_colA_kernel<T, NB>), dim3((n - t + TT - 1) / TT, batch), dim3(256), 0, s, a, t, -1,
                         t - 1, j0);
      const int m = n - t;
      {
        const long long tot = (long long)pe * m;
        const unsigned gx = (unsigned)std::min<long long>(256, (tot + 255) / 256);
        hipLaunchKernelGGL((tri_cat_kernel<T, NB>), dim3(gx, batch), dim3(256), 0, s, a, j0, pe, t);
      }
      // one rank-2pe update: G[t:, t:] -= cat1[:, t:]^T conj(cat2[:, t:])
      char* G = reinterpret_cast<char*>(a.G);
      char* ws = reinterpret_cast<char*>(a.ws);
      GemmArgs g = gemm_args(m, m, 2 * pe, OP_T, OP_R, ws + TriWs<T, NB>::cat1(n) + (size_t)t * es, n,
                             ws + TriWs<T, NB>::cat2(n) + (size_t)t * es, n, G + ((long)t * a.ldg + t) * es, a.ldg);
      g.sA = a.sws / (long long)es; g.sB = a.sws / (long long)es; g.sC = a.sG;
      g.alpha_re = -1.0; g.beta_re = 1.0; g.batch = batch;
      g.lower_band = TRIDIAG_BAND;
      hipError_t err = gemm(EigT<T>::dtype, PREC_FP64, g, s);
      if (err != hipSuccess) return err;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small matrices (n <= TRI_SMALL_N): the unblocked reduction (LAPACK hetd2
// order, lower storage) by one 1024-thread workgroup per matrix, all columns
// in one launch.  The blocked path pays two launches per column, which for
// n of a few hundred is latency, not bandwidth; here the trailing matrix
// (at most 2.4 MB) stays in the caches across columns.  Above 384 one
// compute unit no longer streams the matrix fast enough (measured at
// n = 512 on 15 complex problems: 33 ms against 27 ms blocked).  Per column i:
//   reflector of a(i+1:n, i) (same convention as the blocked path);
//   y = A22 v over the lower triangle: wave w takes rows i+1+w, +16, ...,
//     its lanes the row's columns; row sums by a wave reduction, the
//     transposed terms conj(a_rc) v_r by LDS atomics into y_c;
//   w = tau y - 1/2 |tau|^2 (y^H v) v;  A22 -= v w^H + w v^H (lower triangle).
// Outputs as the blocked path: d, e, tau and the reflector rows of Vt.
// ---------------------------------------------------------------------------
constexpr int TRI_SMALL_N = 384;

template <typename T>
__global__ __launch_bounds__(1024) void tri_small_kernel(TriArgs a) {
  constexpr int NT = 1024, NW = NT / 64;
  __shared__ T s_v[TRI_SMALL_N];
  __shared__ double s_yr[TRI_SMALL_N], s_yi[TRI_SMALL_N];
  __shared__ double s_red[NW], s_red2[NW];
  __shared__ T s_scal, s_tau;
  __shared__ double s_alr, s_ali;
  const int b = blockIdx.x, n = a.n, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  T* G = reinterpret_cast<T*>(a.G) + b * a.sG;
  T* V = reinterpret_cast<T*>(a.Vt) + b * a.sVt;
  T* tau = reinterpret_cast<T*>(a.tau) + b * a.stau;
  double* dd = a.d + b * a.sde;
  double* ee = a.e + b * a.sde;
  const long ldg = a.ldg;
  for (int i = 0; i + 1 < n; ++i) {
    // ||a(i+2:n, i)||^2
    double part = 0.0;
    for (int r = i + 2 + tid; r < n; r += NT) part += nrm2(G[(long)r * ldg + i]);
    part = wave_sum(part);
    if (lane == 0) s_red[wid] = part;
    __syncthreads();
    if (tid == 0) {
      double xn2 = 0.0;
      for (int w = 0; w < NW; ++w) xn2 += s_red[w];
      double beta;
      T tv, sc;
      reflector(G[(long)(i + 1) * ldg + i], xn2, beta, tv, sc);
      s_scal = sc;
      s_tau = tv;
      dd[i] = re(G[(long)i * ldg + i]);
      ee[i] = beta;
      tau[i] = tv;
    }
    __syncthreads();
    const T scal = s_scal;
    for (int c = tid; c < n; c += NT) {
      T v = EigT<T>::zero();
      if (c == i + 1) v = EigT<T>::one();
      else if (c > i + 1) v = mulr(G[(long)c * ldg + i], scal);
      s_v[c] = v;
      V[(long)i * n + c] = v;
      s_yr[c] = 0.0;
      s_yi[c] = 0.0;
    }
    __syncthreads();
    // y = A22 v (all loads of a row issued before its arithmetic: a row has
    // at most TRI_SMALL_N / 64 chunks of 64 columns)
    constexpr int UNR = TRI_SMALL_N / 64;
    for (int r = i + 1 + wid; r < n; r += NW) {
      const T vr = s_v[r];
      T rs = EigT<T>::zero();
      T g[UNR];
#pragma unroll
      for (int m = 0; m < UNR; ++m) {
        const int c = i + 1 + lane + 64 * m;
        g[m] = c <= r ? G[(long)r * ldg + c] : EigT<T>::zero();
      }
#pragma unroll
      for (int m = 0; m < UNR; ++m) {
        const int c = i + 1 + lane + 64 * m;
        if (c <= r) {
          rs = add(rs, mulr(g[m], s_v[c]));
          if (c < r) {
            const T t = mulr(cj(g[m]), vr);
            atomicAdd(&s_yr[c], re(t));
            if constexpr (sizeof(T) == 16) atomicAdd(&s_yi[c], im(t));
          }
        }
      }
      rs = wsum(rs);
      if (lane == 0) {
        atomicAdd(&s_yr[r], re(rs));
        if constexpr (sizeof(T) == 16) atomicAdd(&s_yi[r], im(rs));
      }
    }
    __syncthreads();
    // w = tau y + alpha v with alpha = -1/2 tau (tau y)^H v
    const T tv = s_tau;
    double pr = 0.0, pi = 0.0;
    for (int c = i + 1 + tid; c < n; c += NT) {
      T y;
      if constexpr (sizeof(T) == 16) y = cd{s_yr[c], s_yi[c]};
      else y = s_yr[c];
      const T w = mulr(tv, y);
      const T p = mulr(cj(w), s_v[c]);
      pr += re(p);
      pi += im(p);
    }
    pr = wave_sum(pr);
    pi = wave_sum(pi);
    if (lane == 0) { s_red[wid] = pr; s_red2[wid] = pi; }
    __syncthreads();
    if (tid == 0) {
      double dr = 0.0, di = 0.0;
      for (int w = 0; w < NW; ++w) { dr += s_red[w]; di += s_red2[w]; }
      // alpha = -1/2 tau dot
      if constexpr (sizeof(T) == 16) {
        const cd al = mulr(tv, cd{dr, di});
        s_alr = -0.5 * al.x;
        s_ali = -0.5 * al.y;
      } else {
        s_alr = -0.5 * tv * dr;
        s_ali = 0.0;
      }
    }
    __syncthreads();
    T alpha;
    if constexpr (sizeof(T) == 16) alpha = cd{s_alr, s_ali};
    else alpha = s_alr;
    for (int c = i + 1 + tid; c < n; c += NT) {
      T y;
      if constexpr (sizeof(T) == 16) y = cd{s_yr[c], s_yi[c]};
      else y = s_yr[c];
      const T w = add(mulr(tv, y), mulr(alpha, s_v[c]));
      if constexpr (sizeof(T) == 16) { s_yr[c] = w.x; s_yi[c] = w.y; }
      else s_yr[c] = w;
    }
    __syncthreads();
    // A22 -= v w^H + w v^H on the lower triangle
    for (int r = i + 1 + wid; r < n; r += NW) {
      const T vr = s_v[r];
      T wr;
      if constexpr (sizeof(T) == 16) wr = cd{s_yr[r], s_yi[r]};
      else wr = s_yr[r];
      T g[UNR];
#pragma unroll
      for (int m = 0; m < UNR; ++m) {
        const int c = i + 1 + lane + 64 * m;
        g[m] = c <= r ? G[(long)r * ldg + c] : EigT<T>::zero();
      }
#pragma unroll
      for (int m = 0; m < UNR; ++m) {
        const int c = i + 1 + lane + 64 * m;
        if (c <= r) {
          T wc;
          if constexpr (sizeof(T) == 16) wc = cd{s_yr[c], s_yi[c]};
          else wc = s_yr[c];
          G[(long)r * ldg + c] = sub(g[m], add(mulr(vr, cj(wc)), mulr(wr, cj(s_v[c]))));
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && n > 0) {
    dd[n - 1] = re(G[(long)(n - 1) * ldg + (n - 1)]);
    ee[n - 1] = 0.0;
  }
}

size_t tridiag_ws_bytes(int dtype, int n) {
  return dtype == C128 ? TriWs<cd, TRIDIAG_NB>::bytes(n) : TriWs<double, TRIDIAG_NB>::bytes(n);
}

hipError_t tridiagonalize(int dtype, const TriArgs& a, int batch, hipStream_t s) {
  if (dtype != C128 && dtype != F64) return hipErrorInvalidValue;
  if (a.n <= TRI_SMALL_N) {
    if (a.n <= 0 || batch <= 0) return hipSuccess;
    // work figure: the lower triangle of the trailing matrix, summed over the columns
    const double es = dtype == C128 ? 16.0 : 8.0;
    const double nn = a.n;
    ProfScope ps(s, es * nn * (nn - 1) * (nn + 1) / 6.0 * batch, "tri_small");
    if (dtype == C128) hipLaunchKernelGGL(tri_small_kernel<cd>, dim3(batch), dim3(1024), 0, s, a);
    else hipLaunchKernelGGL(tri_small_kernel<double>, dim3(batch), dim3(1024), 0, s, a);
    return hipGetLastError();
  }
  if (a.sws < (long long)tridiag_ws_bytes(dtype, a.n)) return hipErrorInvalidValue;
  // partial sums and the reflector panel start at zero; the
  // trailing-update operands are written before they are read
  const size_t zb = dtype == C128 ? TriWs<cd, TRIDIAG_NB>::cat1(a.n) : TriWs<double, TRIDIAG_NB>::cat1(a.n);
  if (a.sws % 4 != 0) return hipErrorInvalidValue;
  hipError_t e = zero_fill_rows(a.ws, zb, (size_t)a.sws, batch, s);
  if (e != hipSuccess) return e;
  if (dtype == C128) return tridiag_impl<cd, TRIDIAG_NB>(a, batch, s);
  return tridiag_impl<double, TRIDIAG_NB>(a, batch, s);
}

// ---------------------------------------------------------------------------
// Bisection: lam[b][j] = j-th largest eigenvalue of the symmetric tridiagonal
// (d, e), j < kmax.  Sturm count: number of negative pivots of the LDL^T
// factorisation of T - x I equals the number of eigenvalues below x.
// ---------------------------------------------------------------------------
// The recurrence is one long dependent chain; d and e2 are the same for every
// lane of the wave, so they are read in blocks of STURM_BLK entries ahead of
// their use (one memory wait per block instead of one per step).
constexpr int STURM_BLK = 16;
__device__ inline int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n, double x,
                                  double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  int i = 1;
  for (; i + STURM_BLK <= n; i += STURM_BLK) {
    double dd[STURM_BLK], ee[STURM_BLK];
#pragma unroll
    for (int u = 0; u < STURM_BLK; ++u) {
      dd[u] = d[i + u];
      ee[u] = e2[i - 1 + u];
    }
#pragma unroll
    for (int u = 0; u < STURM_BLK; ++u) {
      q = dd[u] - x - ee[u] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
  }
  for (; i < n; ++i) {
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

// Multisection, BIS_L lanes per wanted eigenvalue (64 / BIS_L per wave):
// the lanes of eigenvalue j evaluate the Sturm count at the BIS_L interior
// points that cut its interval [lo, hi] (count(lo) <= t < count(hi), t the
// ascending index) into BIS_L + 1 equal parts, and all of them move to the
// part whose ends keep that invariant (the first point whose count exceeds t
// and the point before it), until the interval is at rounding level
// relative to the eigenvalue itself.  Small eigenvalues are resolved to that
// relative accuracy (more steps than the absolute accuracy of the norm would
// need) because inverse iteration with shifts only absolutely accurate
// leaves the vectors of closely spaced small eigenvalues far from
// orthogonal, which costs a second Cholesky-QR pass.  One lane per
// eigenvalue leaves one wave per SIMD on a 64 x 1024 batch, bound by the
// latency of the recurrence's division chain; BIS_L = 4 gives four waves per
// SIMD to interleave and needs about half the rounds (log2 5 bits each).
constexpr int BIS_L = 4;

__global__ __launch_bounds__(64) void bisect_kernel(const double* d, const double* e, const double* e2,
                                                    long long sde, int n, int kmax, double* lam, long long slam,
                                                    int batch) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x;
  const int sub = lane & (BIS_L - 1);
  const int j = blockIdx.x * (64 / BIS_L) + lane / BIS_L;
  if (b >= batch) return;
  const double* db = d + b * sde;
  const double* eb = e + b * sde;
  const double* e2b = e2 + b * sde;
  double lo = db[0], hi = db[0], emax2 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double r = (i > 0 ? fabs(eb[i - 1]) : 0.0) + (i < n - 1 ? fabs(eb[i]) : 0.0);
    lo = fmin(lo, db[i] - r);
    hi = fmax(hi, db[i] + r);
    if (i < n - 1) emax2 = fmax(emax2, e2b[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    emax2 = fmax(emax2, __shfl_xor(emax2, off));
  }
  const double scale = fmax(fabs(lo), fabs(hi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2) * 64.0;
  lo -= 4.0 * 2.220446049250313e-16 * scale + pivmin;
  hi += 4.0 * 2.220446049250313e-16 * scale + pivmin;
  const int t = n - 1 - min(j, kmax - 1);  // ascending index of this lane group's eigenvalue
  const int q0 = lane & ~(BIS_L - 1);      // first lane of the group
  for (int it = 0; it < 128; ++it) {
    const bool done = hi - lo <= 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin;
    if (__ballot(!done) == 0ull) break;
    const double w = (hi - lo) / (BIS_L + 1);
    const double x = lo + w * (sub + 1);
    const bool below = sturm_count(db, e2b, n, x, pivmin) <= t;
    // the group's flags (bit s: count at point s <= t); c = leading points below
    const unsigned flags = (unsigned)(__ballot(below) >> q0) & ((1u << BIS_L) - 1);
    const int c = __builtin_ctz(~flags);
    if (!done) {
      const double nlo = c > 0 ? lo + w * c : lo;
      const double nhi = c < BIS_L ? lo + w * (c + 1) : hi;
      if (nlo >= lo && nhi <= hi && nlo < nhi) {
        lo = nlo;
        hi = nhi;
      }
    }
  }
  if (sub == 0 && j < kmax) lam[b * slam + j] = 0.5 * (lo + hi);
}

hipError_t tridiag_eigvals_top(const double* d, const double* e, double* e2, long long sde, int n,
                               int kmax, double* lam, long long slam, int batch, hipStream_t s) {
  if (kmax <= 0 || batch <= 0) return hipSuccess;
  const long tot = (long)batch * n;
  hipLaunchKernelGGL(e2_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, e, e2, sde, n, batch);
  hipLaunchKernelGGL(bisect_kernel, dim3((kmax + 64 / BIS_L - 1) / (64 / BIS_L), batch), dim3(64), 0, s, d, e, e2,
                     sde, n, kmax, lam, slam, batch);
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

// The recurrences below are sequential in i, one lane per eigenvector.  Each
// pass walks i in blocks of IV_BLK and issues all loads of a block before the
// block's arithmetic, so that one memory latency is paid per block rather than
// per step (the stores of a step could alias the next step's loads, which
// keeps the compiler from moving them ahead by itself).
constexpr int IV_BLK = 16;

// One solve with the stored factors of column j: z[:, j] <- (T - lam_j)^-1
// (pre * z[:, j]); returns the factor 1 / max|z| for the next right-hand side.
// ru holds the reciprocals of U's diagonal.
__device__ inline double invit_solve(double* z, long ld, int j, int n, const double* ru, const double* du,
                                     const double* du2, const double* dl, double pre) {
  // forward: b <- L^-1 P b, writing the intermediate into z
  double bi = z[j] * pre;
  for (int i0 = 0; i0 < n - 1; i0 += IV_BLK) {
    double zb[IV_BLK], sb[IV_BLK];
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) {
      const int i = i0 + u;
      zb[u] = 0.0;
      sb[u] = 0.0;
      if (i < n - 1) {
        zb[u] = z[(long)(i + 1) * ld + j];
        sb[u] = dl[(long)i * ld + j];
      }
    }
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) {
      const int i = i0 + u;
      if (i < n - 1) {
        const double bn = zb[u] * pre;
        const double sv = sb[u];
        if (fabs(sv) >= 4.0) {
          const double m = sv - (sv >= 0 ? 4.0 : -4.0);
          z[(long)i * ld + j] = bn;
          bi = bi - m * bn;
        } else {
          z[(long)i * ld + j] = bi;
          bi = bn - sv * bi;
        }
      }
    }
  }
  z[(long)(n - 1) * ld + j] = bi;
  // backward: U x = b
  double x1 = 0.0, x2 = 0.0, amax = 0.0;
  for (int i0 = n - 1; i0 >= 0; i0 -= IV_BLK) {
    double zb[IV_BLK], c1[IV_BLK], c2[IV_BLK], r0[IV_BLK];
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) {
      const int i = i0 - u;
      zb[u] = 0.0; c1[u] = 0.0; c2[u] = 0.0; r0[u] = 0.0;
      if (i >= 0) {
        zb[u] = z[(long)i * ld + j];
        c1[u] = du[(long)i * ld + j];
        c2[u] = du2[(long)i * ld + j];
        r0[u] = ru[(long)i * ld + j];
      }
    }
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) {
      const int i = i0 - u;
      if (i >= 0) {
        const double x = (zb[u] - c1[u] * x1 - c2[u] * x2) * r0[u];
        z[(long)i * ld + j] = x;
        x2 = x1;
        x1 = x;
        amax = fmax(amax, fabs(x));
      }
    }
  }
  return amax > 0.0 ? 1.0 / amax : 1.0;
}

__global__ __launch_bounds__(64) void invit_kernel(const double* d, const double* e, long long sde, int n,
                                                   const double* lam, long long slam, const int* chi,
                                                   int kmax, double* Z, long long ldz, long long sZ,
                                                   double* w_ru, double* w_du, double* w_du2,
                                                   double* w_dl, long long sw, int batch) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || j >= kmax) return;
  const int cb = chi ? chi[b] : kmax;
  if (j >= cb) return;
  const double* db = d + b * sde;
  const double* eb = e + b * sde;
  double* ru = w_ru + b * sw;
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
  // stored as (1 / pivot, du, du2); the multiplier goes to dl, offset by +-4
  // when the rows were interchanged (|multiplier| <= 1 in both cases).
  double a_i = db[0] - lamj;       // current diagonal entry of the active row i
  double c_i = (n > 1) ? eb[0] : 0.0;  // super-diagonal of active row
  for (int i0 = 0; i0 < n - 1; i0 += IV_BLK) {
    double ev[IV_BLK + 1], dv[IV_BLK];
#pragma unroll
    for (int u = 0; u <= IV_BLK; ++u) {
      const int i = i0 + u;
      ev[u] = i < n - 1 ? eb[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) {
      const int i = i0 + u;
      dv[u] = i + 1 < n ? db[i + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) {
      const int i = i0 + u;
      if (i < n - 1) {
        const double sub = ev[u];                              // entry (i+1, i)
        const double a_n = dv[u] - lamj;                       // entry (i+1, i+1)
        const double c_n = (i + 1 < n - 1) ? ev[u + 1] : 0.0;  // entry (i+1, i+2)
        if (fabs(a_i) >= fabs(sub)) {
          double piv = a_i;
          if (fabs(piv) < tiny) piv = (piv >= 0 ? tiny : -tiny);
          const double m = sub / piv;
          ru[(long)i * ld + j] = 1.0 / piv;
          du[(long)i * ld + j] = c_i;
          du2[(long)i * ld + j] = 0.0;
          dl[(long)i * ld + j] = m;
          a_i = a_n - m * c_i;
          c_i = c_n;
        } else {
          // interchange rows i and i+1
          const double m = a_i / sub;
          ru[(long)i * ld + j] = 1.0 / sub;
          du[(long)i * ld + j] = a_n;
          du2[(long)i * ld + j] = c_n;
          dl[(long)i * ld + j] = m + (m >= 0 ? 4.0 : -4.0);  // |stored| >= 4 marks an interchange
          const double na = c_i - m * a_n;
          a_i = na;
          c_i = -m * c_n;
        }
      }
    }
  }
  {
    double piv = a_i;
    if (fabs(piv) < tiny) piv = (piv >= 0 ? tiny : -tiny);
    ru[(long)(n - 1) * ld + j] = 1.0 / piv;
    du[(long)(n - 1) * ld + j] = 0.0;
    du2[(long)(n - 1) * ld + j] = 0.0;
  }
  // two solves from a pseudo-random start
  for (int i = 0; i < n; ++i) z[(long)i * ld + j] = hash_uniform(b, j, i);
  double scale = 1.0;
  for (int it = 0; it < 2; ++it) scale = invit_solve(z, ld, j, n, ru, du, du2, dl, scale);
  // normalise to unit 2-norm (after the last max-scaling)
  double nn = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = z[(long)i * ld + j] * scale;
    nn += x * x;
  }
  const double inv = scale / sqrt(nn);
  for (int i0 = 0; i0 < n; i0 += IV_BLK) {
    double zb[IV_BLK];
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u) zb[u] = i0 + u < n ? z[(long)(i0 + u) * ld + j] : 0.0;
#pragma unroll
    for (int u = 0; u < IV_BLK; ++u)
      if (i0 + u < n) z[(long)(i0 + u) * ld + j] = zb[u] * inv;
  }
}

// Tight clusters (consecutive eigenvalues closer than INVIT_CLUSTER_TOL of
// the matrix norm; exact multiplicities among them) make independent inverse
// iterations converge to nearly the same vector.  One wave per problem walks
// its clusters; the members of a cluster (64 at a time, one per lane) are
// iterated together with their own factors, and after every solve they are
// orthonormalised in order against the earlier members (modified
// Gram-Schmidt), as in LAPACK's stein.
// The threshold sits at about 90 u ||T||: for a larger gap g the vectors of
// independent solves overlap by at most about u ||T|| / g < 1/90, which the
// Cholesky-QR2 that follows on all vectors removes.  (Graded spectra, as the
// Gram matrices of power-law bonds, have consecutive gaps between 1e-14 and
// 1e-11 of the norm over hundreds of eigenvalues; treating those as one
// cluster made its serial orthonormalisation dominate the whole update.)
constexpr double INVIT_CLUSTER_TOL = 1e-14;

__device__ inline double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(64) void invit_cluster_kernel(const double* d, const double* e, long long sde, int n,
                                                           const double* lam, long long slam, const int* chi,
                                                           int kmax, double* Z, long long ldz, long long sZ,
                                                           const double* w_ru, const double* w_du,
                                                           const double* w_du2, const double* w_dl, long long sw) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const int cb = chi ? min(chi[b], kmax) : kmax;
  const double* db = d + b * sde;
  const double* eb = e + b * sde;
  const double* lb = lam + b * slam;
  double* z = Z + b * sZ;
  const long ld = ldz;
  double tn = 0.0;
  for (int i = lane; i < n; i += 64)
    tn = fmax(tn, fabs(db[i]) + (i > 0 ? fabs(eb[i - 1]) : 0.0) + (i < n - 1 ? fabs(eb[i]) : 0.0));
  for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_xor(tn, off, 64));
  const double tol = INVIT_CLUSTER_TOL * tn;
  int j0 = 0;
  while (j0 < cb) {
    int j1 = j0;
    while (j1 + 1 < cb && lb[j1] - lb[j1 + 1] <= tol) ++j1;
    if (j1 > j0) {
      for (int c0 = j0; c0 <= j1; c0 += 64) {
        const int cn = min(64, j1 - c0 + 1);
        const int m = c0 + lane;
        double scale = 1.0;
        for (int it = 0; it < 3; ++it) {
          if (lane < cn)
            scale = invit_solve(z, ld, m, n, w_ru + b * sw, w_du + b * sw, w_du2 + b * sw, w_dl + b * sw, scale);
          __syncthreads();
          // members c0 .. c0+cn-1 in order: apply the pending scale, remove the
          // earlier members of the cluster, normalise
          for (int q = c0; q < c0 + cn; ++q) {
            const double sq = __shfl(scale, q - c0, 64);
            for (int i = lane; i < n; i += 64) z[(long)i * ld + q] *= sq;
            for (int r = j0; r < q; ++r) {
              double dot = 0.0;
              for (int i = lane; i < n; i += 64) dot += z[(long)i * ld + r] * z[(long)i * ld + q];
              dot = wave_sum_d(dot);
              for (int i = lane; i < n; i += 64) z[(long)i * ld + q] -= dot * z[(long)i * ld + r];
            }
            double nn = 0.0;
            for (int i = lane; i < n; i += 64) nn += z[(long)i * ld + q] * z[(long)i * ld + q];
            nn = wave_sum_d(nn);
            const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
            for (int i = lane; i < n; i += 64) z[(long)i * ld + q] *= inv;
          }
          scale = 1.0;
          __syncthreads();
        }
      }
    }
    j0 = j1 + 1;
  }
}

hipError_t tridiag_invit(const double* d, const double* e, long long sde, int n, const double* lam,
                         long long slam, const int* chi, int kmax, double* Z, long long ldz, long long sZ,
                         double* work, int batch, hipStream_t s) {
  if (kmax <= 0 || batch <= 0) return hipSuccess;
  const long long sw = (long long)n * ldz;  // each workspace array: n x ldz per problem
  double* ru = work;
  double* du = work + sw * batch;
  double* du2 = work + 2 * sw * batch;
  double* dl = work + 3 * sw * batch;
  hipLaunchKernelGGL(invit_kernel, dim3((kmax + 63) / 64, batch), dim3(64), 0, s, d, e, sde, n, lam,
                     slam, chi, kmax, Z, ldz, sZ, ru, du, du2, dl, sw, batch);
  hipLaunchKernelGGL(invit_cluster_kernel, dim3(batch), dim3(64), 0, s, d, e, sde, n, lam, slam, chi, kmax, Z, ldz,
                     sZ, ru, du, du2, dl, sw);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Back-transformation U <- Q U with Q = H_0 H_1 ... H_{n-2}, applied in groups
// of BT_GB consecutive reflectors (several reduction panels), so that the
// products with the reflector block have 128 rows / inner dimension.
// Compact-WY factor of a group (LAPACK larft, forward, columnwise):
// H_{j0} ... H_{j0+g-1} = I - V T V^H, T upper triangular g x g with
// T(i,i) = tau_i and T(0:i, i) = -tau_i T(0:i, 0:i) S(0:i, i),
// S = V^H V from a GEMM.  T is built column by column in LDS, packed by
// columns (column i holds rows 0..i at offset i(i+1)/2).
// ---------------------------------------------------------------------------
constexpr int BT_GB = 128;

// One workgroup per (problem, group): block (b, grp) reads S of the group at
// Sg + b * sF + grp * BT_GB^2 and writes T at Tg + b * sF + grp * BT_GB^2.
template <typename T>
__global__ __launch_bounds__(BT_GB) void larft_group_kernel(TriArgs a, const void* Sg, void* Tg, long long sF) {
  __shared__ T Tp[BT_GB * (BT_GB + 1) / 2];
  __shared__ T scol[BT_GB];
  const int b = blockIdx.x, grp = blockIdx.y, q = threadIdx.x;
  const int j0 = grp * BT_GB, g = min(BT_GB, a.n - 1 - j0);
  const long long off = b * sF + (long long)grp * BT_GB * BT_GB;
  const T* S = reinterpret_cast<const T*>(Sg) + off;   // g x g, ld BT_GB
  const T* tau = reinterpret_cast<const T*>(a.tau) + b * a.stau;
  T* Tout = reinterpret_cast<T*>(Tg) + off;             // BT_GB x BT_GB, ld BT_GB
  for (int i = 0; i < g; ++i) {
    if (q < i) scol[q] = S[(long)q * BT_GB + i];
    __syncthreads();
    const T ti = tau[j0 + i];
    T* coli = Tp + i * (i + 1) / 2;
    if (q < i) {
      T acc = EigT<T>::zero();
      for (int r = q; r < i; ++r) acc = add(acc, mulr(Tp[r * (r + 1) / 2 + q], scol[r]));
      coli[q] = mulr(scl(-1.0, ti), acc);
    } else if (q == i) {
      coli[i] = ti;
    }
    __syncthreads();
  }
  for (int r = 0; r < BT_GB; ++r) {
    const int c = q;
    Tout[(long)r * BT_GB + c] = (r < g && c < g && r <= c) ? Tp[c * (c + 1) / 2 + r] : EigT<T>::zero();
  }
}

static int bt_groups(int n) { return (n - 1 + BT_GB - 1) / BT_GB; }

template <typename T>
static hipError_t backtransform_impl(const TriArgs& a, void* Tf, long long sTf, void* U, long long ldu,
                                     long long sU, int kmax, void* work, int batch, hipStream_t s) {
  const int n = a.n;
  const int ng = bt_groups(n);
  if (ng <= 0 || kmax <= 0) return hipSuccess;
  const size_t es = sizeof(T);
  const int dt = EigT<T>::dtype;
  char* V = reinterpret_cast<char*>(a.Vt);
  char* Uc = reinterpret_cast<char*>(U);
  char* Tc = reinterpret_cast<char*>(Tf);
  char* Sc = Tc + (size_t)ng * BT_GB * BT_GB * es;   // per-problem S of every group after the T factors
  char* W1 = reinterpret_cast<char*>(work);
  char* W2 = W1 + (size_t)batch * BT_GB * kmax * es;
  char* kws = W2 + (size_t)batch * BT_GB * kmax * es;   // split-K scratch
  const long long sW = (long long)BT_GB * kmax;
  hipError_t err = hipSuccess;
  // S = V_g^H V_g of every group (over rows j0+1 .. n-1; V_g = columns of Vt
  // rows j0 ..), then the T factors of all groups in one launch
  for (int grp = 0; grp < ng; ++grp) {
    const int j0 = grp * BT_GB, g = min(BT_GB, n - 1 - j0), rows = n - j0 - 1;
    GemmArgs gs = gemm_args(g, g, rows, OP_R, OP_T, V + ((long)j0 * n + j0 + 1) * es, n,
                            V + ((long)j0 * n + j0 + 1) * es, n, Sc + (size_t)grp * BT_GB * BT_GB * es, BT_GB);
    gs.sA = a.sVt; gs.sB = a.sVt; gs.sC = sTf; gs.batch = batch;
    gs.kws = kws; gs.kws_bytes = GEMM_SPLITK_WS_BYTES;
    err = gemm(dt, PREC_FP64, gs, s);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(larft_group_kernel<T>, dim3(batch, ng), dim3(BT_GB), 0, s, a, (const void*)Sc, (void*)Tc, sTf);
  // groups applied last to first: U <- U - V_g (T_g (V_g^H U))
  for (int grp = ng - 1; grp >= 0; --grp) {
    const int j0 = grp * BT_GB, g = min(BT_GB, n - 1 - j0), rows = n - j0 - 1;
    GemmArgs g1 = gemm_args(g, kmax, rows, OP_R, OP_N, V + ((long)j0 * n + j0 + 1) * es, n,
                            Uc + (long)(j0 + 1) * ldu * es, ldu, W1, kmax);
    g1.sA = a.sVt; g1.sB = sU; g1.sC = sW; g1.batch = batch;
    g1.kws = kws; g1.kws_bytes = GEMM_SPLITK_WS_BYTES;
    err = gemm(dt, PREC_FP64, g1, s);
    if (err != hipSuccess) return err;
    GemmArgs g2 = gemm_args(g, kmax, g, OP_N, OP_N, Tc + (size_t)grp * BT_GB * BT_GB * es, BT_GB, W1, kmax, W2,
                            kmax);
    g2.sA = sTf; g2.sB = sW; g2.sC = sW; g2.batch = batch;
    err = gemm(dt, PREC_FP64, g2, s);
    if (err != hipSuccess) return err;
    GemmArgs g3 = gemm_args(rows, kmax, g, OP_T, OP_N, V + ((long)j0 * n + j0 + 1) * es, n, W2, kmax,
                            Uc + (long)(j0 + 1) * ldu * es, ldu);
    g3.sA = a.sVt; g3.sB = sW; g3.sC = sU;
    g3.alpha_re = -1.0; g3.beta_re = 1.0; g3.batch = batch;
    err = gemm(dt, PREC_FP64, g3, s);
    if (err != hipSuccess) return err;
  }
  return hipGetLastError();
}

size_t tridiag_backtransform_tf_elems(int n) { return (size_t)2 * std::max(1, bt_groups(n)) * BT_GB * BT_GB; }
size_t tridiag_backtransform_work_bytes(int dtype, int kmax, int batch) {
  const size_t es = dtype == C128 ? sizeof(cd) : sizeof(double);
  return es * 2 * BT_GB * (size_t)kmax * batch + GEMM_SPLITK_WS_BYTES;
}

hipError_t tridiag_backtransform(int dtype, const TriArgs& a, void* Tf, long long sTf, void* U,
                                 long long ldu, long long sU, int kmax, void* work, int batch,
                                 hipStream_t s) {
  if (batch > 1 && sTf < (long long)tridiag_backtransform_tf_elems(a.n)) return hipErrorInvalidValue;
  if (dtype == C128) return backtransform_impl<cd>(a, Tf, sTf, U, ldu, sU, kmax, work, batch, s);
  if (dtype == F64) return backtransform_impl<double>(a, Tf, sTf, U, ldu, sU, kmax, work, batch, s);
  return hipErrorInvalidValue;
}

}  // namespace tci
