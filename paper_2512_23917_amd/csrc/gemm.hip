// Batched GEMM on the CDNA4 matrix cores: C = alpha * op(A) op(B) (* diag scales) + beta * C.
//
// The contraction of two site tensors, the Gram matrices and every
// back-multiplication of the truncated SVD reduce to this one primitive after
// the label planner has permuted operands into matrix form (Sec. II.B
// contraction equations: C_IJ = sum_S A_IS B_SJ).
//
// Three arithmetic modes share the tiling:
//   * FP64:   v_mfma_f64_16x16x4f64, double accumulate (complex by four real products);
//   * FP32:   v_mfma_f32_16x16x4f32, float accumulate;
//   * BF16X3: each float operand is split x = hi + lo with hi = rne_bf16(x),
//             lo = rne_bf16(x - hi); three v_mfma_f32_16x16x32_bf16 products
//             hi*hi + hi*lo + lo*hi accumulate in float.
// Operands are row-major with leading dimensions; op() may transpose or
// conjugate-transpose either side.  A batch may carry its own (m, n, k) per
// problem in device memory so ragged batches run in one launch.
#include "common.hpp"
#include "gemm.hpp"
#include "prof.hpp"

namespace tci {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Workgroup -> tile mapping.  Dispatch places workgroup i on XCD (i mod 8);
// re-number so the tiles that one XCD receives are contiguous in (batch,
// tile_m, tile_n) order and share operand panels in that XCD's L2.
// ---------------------------------------------------------------------------
__device__ inline void tile_coords(int& tm, int& tn, int& b) {
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const long total = (long)gx * gy * gz;
  long lin = blockIdx.x + (long)gx * (blockIdx.y + (long)gy * blockIdx.z);
  if ((total & 7) == 0) {
    const long per = total >> 3;
    lin = (lin & 7) * per + (lin >> 3);
  }
  tn = (int)(lin % gx);
  lin /= gx;
  tm = (int)(lin % gy);
  b = (int)(lin / gy);
}

template <typename T> struct Elem;
template <> struct Elem<double> { static constexpr bool cplx = false; };
template <> struct Elem<float> { static constexpr bool cplx = false; };
template <> struct Elem<cd> { static constexpr bool cplx = true; };
template <> struct Elem<cf> { static constexpr bool cplx = true; };

__device__ inline void ld(const double* p, double& re, double& im) { re = *p; im = 0.0; }
__device__ inline void ld(const cd* p, double& re, double& im) { cd v = *p; re = v.x; im = v.y; }
__device__ inline void ld(const float* p, float& re, float& im) { re = *p; im = 0.f; }
__device__ inline void ld(const cf* p, float& re, float& im) { cf v = *p; re = v.x; im = v.y; }
__device__ inline void st(double* p, double re, double) { *p = re; }
__device__ inline void st(cd* p, double re, double im) { *p = cd{re, im}; }
__device__ inline void st(float* p, float re, float) { *p = re; }
__device__ inline void st(cf* p, float re, float im) { *p = cf{re, im}; }

// Zeros that out-of-range tile elements are loaded from, so that the loads
// need no select afterwards (device code reads it; nothing writes it).
__device__ double g_zero_elem[4] = {0.0, 0.0, 0.0, 0.0};
// Where the epilogue stores the values of out-of-range tile elements, so that
// its stores need no branch (never read).
__device__ double g_sink_elem[4];

// ---------------------------------------------------------------------------
// Staging: a BM x BK tile of op(A) and a BK x BN tile of op(B) are read from
// global memory (each thread 8 consecutive elements along the contiguous
// dimension) and written k-major into LDS planes (re, im).
// ---------------------------------------------------------------------------
template <typename T, typename R, int ROWS, int BK>
__device__ inline void stage_rows_tile(const T* __restrict__ A, long lda, int op, int M, int K,
                                       int m0, int k0, R (*re)[ROWS + 2], R (*im)[ROWS + 2]) {
  // Tile element (r, kk) of op(A) (r < ROWS, kk < BK) goes to re[kk][r].
  const int t = threadIdx.x;
  constexpr int PER = ROWS * BK / 256;  // elements per thread (8 for 128x16)
  if (op == OP_N || op == OP_R) {
    // A stored M x K: contiguous along k.
    constexpr int TPR = BK / PER;  // threads per row
    const int r = t / TPR, kk0 = (t % TPR) * PER;
    const int gm = m0 + r;
    const R sgn = (op == OP_R) ? R(-1) : R(1);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int gk = k0 + kk0 + e;
      R vr, vi;
      ld((gm < M && gk < K) ? A + (long)gm * lda + gk : reinterpret_cast<const T*>(g_zero_elem), vr, vi);
      re[kk0 + e][r] = vr;
      im[kk0 + e][r] = sgn * vi;
    }
  } else {
    // A stored K x M: contiguous along m.
    constexpr int TPK = ROWS / PER;  // threads per k-row
    const int kk = t / TPK, r0 = (t % TPK) * PER;
    const int gk = k0 + kk;
    const R sgn = (op == OP_C) ? R(-1) : R(1);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int gm = m0 + r0 + e;
      R vr, vi;
      ld((gm < M && gk < K) ? A + (long)gk * lda + gm : reinterpret_cast<const T*>(g_zero_elem), vr, vi);
      re[kk][r0 + e] = vr;
      im[kk][r0 + e] = sgn * vi;
    }
  }
}

template <typename T, typename R, int COLS, int BK>
__device__ inline void stage_cols_tile(const T* __restrict__ B, long ldb, int op, int N, int K,
                                       int n0, int k0, R (*re)[COLS + 2], R (*im)[COLS + 2]) {
  // Tile element (kk, c) of op(B) goes to re[kk][c].
  const int t = threadIdx.x;
  constexpr int PER = COLS * BK / 256;
  if (op == OP_N || op == OP_R) {
    // B stored K x N: contiguous along n.
    constexpr int TPK = COLS / PER;
    const int kk = t / TPK, c0 = (t % TPK) * PER;
    const int gk = k0 + kk;
    const R sgn = (op == OP_R) ? R(-1) : R(1);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int gn = n0 + c0 + e;
      R vr, vi;
      ld((gn < N && gk < K) ? B + (long)gk * ldb + gn : reinterpret_cast<const T*>(g_zero_elem), vr, vi);
      re[kk][c0 + e] = vr;
      im[kk][c0 + e] = sgn * vi;
    }
  } else {
    // B stored N x K: contiguous along k.
    constexpr int TPC = BK / PER;
    const int c = t / TPC, kk0 = (t % TPC) * PER;
    const int gn = n0 + c;
    const R sgn = (op == OP_C) ? R(-1) : R(1);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int gk = k0 + kk0 + e;
      R vr, vi;
      ld((gn < N && gk < K) ? B + (long)gn * ldb + gk : reinterpret_cast<const T*>(g_zero_elem), vr, vi);
      re[kk0 + e][c] = vr;
      im[kk0 + e][c] = sgn * vi;
    }
  }
}

// The same staging split in two halves, so that the global loads of the next
// k tile are in flight while the current one is multiplied.  load() only
// issues the loads (out-of-range elements read zeros); store() applies the
// conjugation sign and writes LDS, so nothing waits on the loads before the
// products.
template <typename T, typename R, int ROWS, int BK>
struct RowsStage {
  static constexpr int PER = ROWS * BK / 256;
  R re[PER], im[PER];
  __device__ inline void load(const T* __restrict__ A, long lda, int op, int M, int K, int m0, int k0) {
    const int t = threadIdx.x;
    const T* zero = reinterpret_cast<const T*>(g_zero_elem);
    if (op == OP_N || op == OP_R) {
      constexpr int TPR = BK / PER;
      const int r = t / TPR, kk0 = (t % TPR) * PER;
      const int gm = m0 + r;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int gk = k0 + kk0 + e;
        ld((gm < M && gk < K) ? A + (long)gm * lda + gk : zero, re[e], im[e]);
      }
    } else {
      constexpr int TPK = ROWS / PER;
      const int kk = t / TPK, r0 = (t % TPK) * PER;
      const int gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int gm = m0 + r0 + e;
        ld((gm < M && gk < K) ? A + (long)gk * lda + gm : zero, re[e], im[e]);
      }
    }
  }
  __device__ inline void store(int op, R (*sre)[ROWS + 2], R (*sim)[ROWS + 2]) const {
    const int t = threadIdx.x;
    const R sgn = (op == OP_R || op == OP_C) ? R(-1) : R(1);
    if (op == OP_N || op == OP_R) {
      constexpr int TPR = BK / PER;
      const int r = t / TPR, kk0 = (t % TPR) * PER;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        sre[kk0 + e][r] = re[e];
        sim[kk0 + e][r] = sgn * im[e];
      }
    } else {
      constexpr int TPK = ROWS / PER;
      const int kk = t / TPK, r0 = (t % TPK) * PER;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        sre[kk][r0 + e] = re[e];
        sim[kk][r0 + e] = sgn * im[e];
      }
    }
  }
};

template <typename T, typename R, int COLS, int BK>
struct ColsStage {
  static constexpr int PER = COLS * BK / 256;
  R re[PER], im[PER];
  __device__ inline void load(const T* __restrict__ B, long ldb, int op, int N, int K, int n0, int k0) {
    const int t = threadIdx.x;
    const T* zero = reinterpret_cast<const T*>(g_zero_elem);
    if (op == OP_N || op == OP_R) {
      constexpr int TPK = COLS / PER;
      const int kk = t / TPK, c0 = (t % TPK) * PER;
      const int gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int gn = n0 + c0 + e;
        ld((gn < N && gk < K) ? B + (long)gk * ldb + gn : zero, re[e], im[e]);
      }
    } else {
      constexpr int TPC = BK / PER;
      const int c = t / TPC, kk0 = (t % TPC) * PER;
      const int gn = n0 + c;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int gk = k0 + kk0 + e;
        ld((gn < N && gk < K) ? B + (long)gn * ldb + gk : zero, re[e], im[e]);
      }
    }
  }
  __device__ inline void store(int op, R (*sre)[COLS + 2], R (*sim)[COLS + 2]) const {
    const int t = threadIdx.x;
    const R sgn = (op == OP_R || op == OP_C) ? R(-1) : R(1);
    if (op == OP_N || op == OP_R) {
      constexpr int TPK = COLS / PER;
      const int kk = t / TPK, c0 = (t % TPK) * PER;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        sre[kk][c0 + e] = re[e];
        sim[kk][c0 + e] = sgn * im[e];
      }
    } else {
      constexpr int TPC = BK / PER;
      const int c = t / TPC, kk0 = (t % TPC) * PER;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        sre[kk0 + e][c] = re[e];
        sim[kk0 + e][c] = sgn * im[e];
      }
    }
  }
};

__device__ inline void problem_dims(const GemmArgs& a, int b, int& M, int& N, int& K) {
  if (a.dims) {
    M = min(a.dims[3 * b + 0], a.m);
    N = min(a.dims[3 * b + 1], a.n);
    K = min(a.dims[3 * b + 2], a.k);
  } else {
    M = a.m; N = a.n; K = a.k;
  }
}

// ---------------------------------------------------------------------------
// FP64 matrix-core GEMM.  256 threads = 4 waves in a 2 x 2 grid; each wave
// owns a (BM/2) x (BN/2) sub-tile made of 16x16 MFMA blocks.  For complex T
// the product uses four real MFMAs per block and k-step (re*re - im*im,
// re*im + im*re).  f64 16x16x4 output layout: lane l, register r holds
// row (l/16) + 4r, column l%16 of the block.  The loads of k tile t+1 are
// issued right after tile t is in LDS and land in registers while tile t is
// multiplied (one LDS buffer, two barriers per tile).
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmArgs a) {
  constexpr bool CPLX = Elem<T>::cplx;
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FI = WM / 16, FJ = WN / 16;
  __shared__ double As_re[BK][BM + 2], As_im[BK][BM + 2];
  __shared__ double Bs_re[BK][BN + 2], Bs_im[BK][BN + 2];

  int tm, tn, b;
  tile_coords(tm, tn, b);
  // split-K launches carry the chunk index outermost in the batch dimension
  int split = 0;
  if (a.ksplit > 1) {
    split = b / a.batch;
    b -= split * a.batch;
  }
  int M, N, K;
  problem_dims(a, b, M, N, K);
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;
  if (a.lower_band > 0 && n0 - (m0 + BM - 1) >= a.lower_band) return;
  int kbeg = 0, kend = K;
  if (a.ksplit > 1) {
    const int kc = ((K + a.ksplit - 1) / a.ksplit + BK - 1) / BK * BK;
    kbeg = min(K, split * kc);
    kend = min(K, kbeg + kc);
  }

  const T* A = reinterpret_cast<const T*>(a.A) + (long)b * a.sA;
  const T* B = reinterpret_cast<const T*>(a.B) + (long)b * a.sB;
  T* C = reinterpret_cast<T*>(a.C) + (long)b * a.sC;

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;

  d4 acc_re[FI][FJ], acc_im[CPLX ? FI : 1][CPLX ? FJ : 1];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
      acc_re[i][j] = d4{0, 0, 0, 0};
      if constexpr (CPLX) acc_im[i][j] = d4{0, 0, 0, 0};
    }

  // the next k tile is loaded into registers while this one is multiplied
  RowsStage<T, double, BM, BK> sa;
  ColsStage<T, double, BN, BK> sb;
  if (kbeg < kend) {
    sa.load(A, a.lda, a.opA, M, kend, m0, kbeg);
    sb.load(B, a.ldb, a.opB, N, kend, n0, kbeg);
  }
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    sa.store(a.opA, As_re, As_im);
    sb.store(a.opB, Bs_re, Bs_im);
    __syncthreads();
    if (k0 + BK < kend) {
      sa.load(A, a.lda, a.opA, M, kend, m0, k0 + BK);
      sb.load(B, a.ldb, a.opB, N, kend, n0, k0 + BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double fa_re[FI], fa_im[FI], fb_re[FJ], fb_im[FJ];
#pragma unroll
      for (int i = 0; i < FI; ++i) {
        fa_re[i] = As_re[ks + lk][wm * WM + i * 16 + lr];
        if constexpr (CPLX) fa_im[i] = As_im[ks + lk][wm * WM + i * 16 + lr];
      }
#pragma unroll
      for (int j = 0; j < FJ; ++j) {
        fb_re[j] = Bs_re[ks + lk][wn * WN + j * 16 + lr];
        if constexpr (CPLX) fb_im[j] = Bs_im[ks + lk][wn * WN + j * 16 + lr];
      }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa_re[i], fb_re[j], acc_re[i][j], 0, 0, 0);
          if constexpr (CPLX) {
            acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fa_im[i], fb_im[j], acc_re[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa_re[i], fb_im[j], acc_im[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa_im[i], fb_re[j], acc_im[i][j], 0, 0, 0);
          }
        }
    }
  }

  if (a.ksplit > 1) {
    // raw partial product of this K chunk: slab (split, b), M x N, row-major
    T* P = reinterpret_cast<T*>(a.kws) + ((long)split * a.batch + b) * (long)M * N;
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int j = 0; j < FJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + lk + 4 * r;
          const int col = n0 + wn * WN + j * 16 + lr;
          if (row < M && col < N) {
            double vi = 0.0;
            if constexpr (CPLX) vi = acc_im[i][j][r];
            st(P + (long)row * N + col, acc_re[i][j][r], vi);
          }
        }
    return;
  }

  const double* rs = a.rs ? a.rs + (long)b * a.s_rs : nullptr;
  const double* cs = a.cs ? a.cs + (long)b * a.s_cs : nullptr;
  const bool beta0 = (a.beta_re == 0.0 && a.beta_im == 0.0);
  // one 16-row block row at a time; the C loads of block row i + 1 are issued
  // before block row i is stored, so only the first block's load latency is
  // exposed (short-K updates are bound by it); out-of-range elements read
  // zeros, so no load sits behind a branch
  const T* zero = reinterpret_cast<const T*>(g_zero_elem);
  double c_re[2][FJ][4], c_im[2][FJ][4];
  auto load_c = [&](int i, double (&cr)[FJ][4], double (&ci)[FJ][4]) {
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + lk + 4 * r;
        const int col = n0 + wn * WN + j * 16 + lr;
        ld((row < M && col < N) ? C + (long)row * a.ldc + col : zero, cr[j][r], ci[j][r]);
      }
  };
  // row scales of a block row (rows clamped into range: values of rows and
  // columns outside the problem go to the sink), loaded with its C values
  double rsv[2][4];
  auto load_rs = [&](int i, double (&v)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = rs ? rs[min(m0 + wm * WM + i * 16 + lk + 4 * r, M - 1)] : 1.0;
  };
  double csv[FJ];
#pragma unroll
  for (int j = 0; j < FJ; ++j) csv[j] = cs ? cs[min(n0 + wn * WN + j * 16 + lr, N - 1)] : 1.0;
  load_rs(0, rsv[0]);
  if (!beta0) load_c(0, c_re[0], c_im[0]);
#pragma unroll
  for (int i = 0; i < FI; ++i) {
    if (i + 1 < FI) {
      load_rs(i + 1, rsv[(i + 1) & 1]);
      if (!beta0) load_c(i + 1, c_re[(i + 1) & 1], c_im[(i + 1) & 1]);
    }
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + lk + 4 * r;
        const int col = n0 + wn * WN + j * 16 + lr;
        double vr = acc_re[i][j][r], vi = 0.0;
        if constexpr (CPLX) vi = acc_im[i][j][r];
        const double sc = rsv[i & 1][r] * csv[j];
        vr *= sc; vi *= sc;
        double outr = a.alpha_re * vr - a.alpha_im * vi;
        double outi = a.alpha_re * vi + a.alpha_im * vr;
        if (!beta0) {
          const double cr = c_re[i & 1][j][r], ci = c_im[i & 1][j][r];
          outr += a.beta_re * cr - a.beta_im * ci;
          outi += a.beta_re * ci + a.beta_im * cr;
        }
        st((row < M && col < N) ? C + (long)row * a.ldc + col : reinterpret_cast<T*>(g_sink_elem), outr, outi);
      }
  }
}

// ---------------------------------------------------------------------------
// FP32 matrix-core GEMM (float or complex-float storage), float accumulate.
// f32 16x16x4 output layout: lane l, register r holds row 4*(l/16) + r.
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs a) {
  constexpr bool CPLX = Elem<T>::cplx;
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FI = WM / 16, FJ = WN / 16;
  __shared__ float As_re[BK][BM + 2], As_im[BK][BM + 2];
  __shared__ float Bs_re[BK][BN + 2], Bs_im[BK][BN + 2];

  int tm, tn, b;
  tile_coords(tm, tn, b);
  int M, N, K;
  problem_dims(a, b, M, N, K);
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;
  if (a.lower_band > 0 && n0 - (m0 + BM - 1) >= a.lower_band) return;
  const T* A = reinterpret_cast<const T*>(a.A) + (long)b * a.sA;
  const T* B = reinterpret_cast<const T*>(a.B) + (long)b * a.sB;
  T* C = reinterpret_cast<T*>(a.C) + (long)b * a.sC;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;

  f4 acc_re[FI][FJ], acc_im[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) { acc_re[i][j] = f4{0, 0, 0, 0}; acc_im[i][j] = f4{0, 0, 0, 0}; }

  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    stage_rows_tile<T, float, BM, BK>(A, a.lda, a.opA, M, K, m0, k0, As_re, As_im);
    stage_cols_tile<T, float, BN, BK>(B, a.ldb, a.opB, N, K, n0, k0, Bs_re, Bs_im);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      float fa_re[FI], fa_im[FI], fb_re[FJ], fb_im[FJ];
#pragma unroll
      for (int i = 0; i < FI; ++i) {
        fa_re[i] = As_re[ks + lk][wm * WM + i * 16 + lr];
        fa_im[i] = As_im[ks + lk][wm * WM + i * 16 + lr];
      }
#pragma unroll
      for (int j = 0; j < FJ; ++j) {
        fb_re[j] = Bs_re[ks + lk][wn * WN + j * 16 + lr];
        fb_im[j] = Bs_im[ks + lk][wn * WN + j * 16 + lr];
      }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa_re[i], fb_re[j], acc_re[i][j], 0, 0, 0);
          if constexpr (CPLX) {
            acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-fa_im[i], fb_im[j], acc_re[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa_re[i], fb_im[j], acc_im[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa_im[i], fb_re[j], acc_im[i][j], 0, 0, 0);
          }
        }
    }
  }

  const double* rs = a.rs ? a.rs + (long)b * a.s_rs : nullptr;
  const double* cs = a.cs ? a.cs + (long)b * a.s_cs : nullptr;
  const bool beta0 = (a.beta_re == 0.0 && a.beta_im == 0.0);
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + 4 * lk + r;
        const int col = n0 + wn * WN + j * 16 + lr;
        if (row < M && col < N) {
          float vr = acc_re[i][j][r], vi = CPLX ? acc_im[i][j][r] : 0.f;
          float sc = 1.f;
          if (rs) sc *= (float)rs[row];
          if (cs) sc *= (float)cs[col];
          vr *= sc; vi *= sc;
          const float ar = (float)a.alpha_re, ai = (float)a.alpha_im;
          float outr = ar * vr - ai * vi, outi = ar * vi + ai * vr;
          T* p = C + (long)row * a.ldc + col;
          if (!beta0) {
            float cr, ci;
            ld(p, cr, ci);
            outr += (float)a.beta_re * cr - (float)a.beta_im * ci;
            outi += (float)a.beta_re * ci + (float)a.beta_im * cr;
          }
          st(p, outr, outi);
        }
      }
}

// ---------------------------------------------------------------------------
// Split-BF16 x3 GEMM (float or complex-float storage), float accumulate.
// LDS holds four bf16 planes per operand (re_hi, re_lo, im_hi, im_lo), k
// contiguous, so one lane fetches its 8 consecutive k values with one read.
// bf16 16x16x32 operand layout: lane l supplies row l%16, k 8*(l/16)..+7.
// ---------------------------------------------------------------------------
__device__ inline __bf16 rne_bf16(float x) { return (__bf16)x; }

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = rne_bf16(x);
  lo = rne_bf16(x - (float)hi);
}

template <typename T, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(GemmArgs a) {
  constexpr bool CPLX = Elem<T>::cplx;
  constexpr int BK = 32;
  constexpr int KP = BK + 8;  // padded k extent (bf16 elements)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FI = WM / 16, FJ = WN / 16;
  constexpr int NPL = CPLX ? 4 : 2;  // planes: re_hi, re_lo, (im_hi, im_lo)
  __shared__ __attribute__((aligned(16))) __bf16 As[NPL][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NPL][BN][KP];

  int tm, tn, b;
  tile_coords(tm, tn, b);
  int M, N, K;
  problem_dims(a, b, M, N, K);
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;
  if (a.lower_band > 0 && n0 - (m0 + BM - 1) >= a.lower_band) return;
  const T* A = reinterpret_cast<const T*>(a.A) + (long)b * a.sA;
  const T* B = reinterpret_cast<const T*>(a.B) + (long)b * a.sB;
  T* C = reinterpret_cast<T*>(a.C) + (long)b * a.sC;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int t = threadIdx.x;

  f4 acc_re[FI][FJ], acc_im[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) { acc_re[i][j] = f4{0, 0, 0, 0}; acc_im[i][j] = f4{0, 0, 0, 0}; }

  // the next k tile is loaded into registers while this one is multiplied;
  // the split into bf16 planes happens when it is written to LDS
  RowsStage<T, float, BM, BK> sa;
  ColsStage<T, float, BN, BK> sb;
  sa.load(A, a.lda, a.opA, M, K, m0, 0);
  sb.load(B, a.ldb, a.opB, N, K, n0, 0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    // op(A) tile (r, kk) -> As[plane][r][kk]
    {
      constexpr int PER = decltype(sa)::PER;
      const float sgn = (a.opA == OP_R || a.opA == OP_C) ? -1.f : 1.f;
      if (a.opA == OP_N || a.opA == OP_R) {
        constexpr int TPR = BK / PER;
        const int r = t / TPR, kk0 = (t % TPR) * PER;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          split_bf16(sa.re[e], As[0][r][kk0 + e], As[1][r][kk0 + e]);
          if constexpr (CPLX) split_bf16(sgn * sa.im[e], As[2][r][kk0 + e], As[3][r][kk0 + e]);
        }
      } else {
        constexpr int TPK = BM / PER;
        const int kk = t / TPK, r0 = (t % TPK) * PER;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          split_bf16(sa.re[e], As[0][r0 + e][kk], As[1][r0 + e][kk]);
          if constexpr (CPLX) split_bf16(sgn * sa.im[e], As[2][r0 + e][kk], As[3][r0 + e][kk]);
        }
      }
    }
    // op(B) tile (kk, c) -> Bs[plane][c][kk]
    {
      constexpr int PER = decltype(sb)::PER;
      const float sgn = (a.opB == OP_R || a.opB == OP_C) ? -1.f : 1.f;
      if (a.opB == OP_N || a.opB == OP_R) {
        constexpr int TPK = BN / PER;
        const int kk = t / TPK, c0 = (t % TPK) * PER;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          split_bf16(sb.re[e], Bs[0][c0 + e][kk], Bs[1][c0 + e][kk]);
          if constexpr (CPLX) split_bf16(sgn * sb.im[e], Bs[2][c0 + e][kk], Bs[3][c0 + e][kk]);
        }
      } else {
        constexpr int TPC = BK / PER;
        const int c = t / TPC, kk0 = (t % TPC) * PER;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          split_bf16(sb.re[e], Bs[0][c][kk0 + e], Bs[1][c][kk0 + e]);
          if constexpr (CPLX) split_bf16(sgn * sb.im[e], Bs[2][c][kk0 + e], Bs[3][c][kk0 + e]);
        }
      }
    }
    __syncthreads();
    if (k0 + BK < K) {
      sa.load(A, a.lda, a.opA, M, K, m0, k0 + BK);
      sb.load(B, a.ldb, a.opB, N, K, n0, k0 + BK);
    }

    bf8 fa[NPL][FI], fb[NPL][FJ];
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
#pragma unroll
      for (int i = 0; i < FI; ++i)
        fa[p][i] = *reinterpret_cast<const bf8*>(&As[p][wm * WM + i * 16 + lr][8 * lk]);
#pragma unroll
      for (int j = 0; j < FJ; ++j)
        fb[p][j] = *reinterpret_cast<const bf8*>(&Bs[p][wn * WN + j * 16 + lr][8 * lk]);
    }
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int j = 0; j < FJ; ++j) {
        // re += Are*Bre (3 terms)
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[0][j], acc_re[i][j], 0, 0, 0);
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[1][j], acc_re[i][j], 0, 0, 0);
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[0][j], acc_re[i][j], 0, 0, 0);
        if constexpr (CPLX) {
          // re -= Aim*Bim ; im += Are*Bim + Aim*Bre
          bf8 nh = -fa[2][i], nl = -fa[3][i];
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nh, fb[2][j], acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nh, fb[3][j], acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nl, fb[2][j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[2][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[3][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[2][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[0][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[1][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[3][i], fb[0][j], acc_im[i][j], 0, 0, 0);
        }
      }
  }

  const double* rs = a.rs ? a.rs + (long)b * a.s_rs : nullptr;
  const double* cs = a.cs ? a.cs + (long)b * a.s_cs : nullptr;
  const bool beta0 = (a.beta_re == 0.0 && a.beta_im == 0.0);
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + 4 * lk + r;
        const int col = n0 + wn * WN + j * 16 + lr;
        if (row < M && col < N) {
          float vr = acc_re[i][j][r], vi = CPLX ? acc_im[i][j][r] : 0.f;
          float sc = 1.f;
          if (rs) sc *= (float)rs[row];
          if (cs) sc *= (float)cs[col];
          vr *= sc; vi *= sc;
          const float ar = (float)a.alpha_re, ai = (float)a.alpha_im;
          float outr = ar * vr - ai * vi, outi = ar * vi + ai * vr;
          T* p = C + (long)row * a.ldc + col;
          if (!beta0) {
            float cr, ci;
            ld(p, cr, ci);
            outr += (float)a.beta_re * cr - (float)a.beta_im * ci;
            outi += (float)a.beta_re * ci + (float)a.beta_im * cr;
          }
          st(p, outr, outi);
        }
      }
}

// ---------------------------------------------------------------------------
// Second pass of a split-K launch: C = alpha * diag(rs) (sum of the chunks'
// partial products, in chunk order) diag(cs) + beta * C, the same epilogue
// as the single-pass kernel.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs a) {
  const int b = blockIdx.y, M = a.m, N = a.n;
  const long long mn = (long long)M * N;
  const T* P = reinterpret_cast<const T*>(a.kws);
  T* C = reinterpret_cast<T*>(a.C) + (long)b * a.sC;
  const double* rs = a.rs ? a.rs + (long)b * a.s_rs : nullptr;
  const double* cs = a.cs ? a.cs + (long)b * a.s_cs : nullptr;
  const bool beta0 = (a.beta_re == 0.0 && a.beta_im == 0.0);
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < mn; e += (long long)gridDim.x * 256) {
    const int row = (int)(e / N), col = (int)(e % N);
    double vr = 0.0, vi = 0.0;
    for (int sp = 0; sp < a.ksplit; ++sp) {
      double pr, pi;
      ld(P + ((long long)sp * a.batch + b) * mn + e, pr, pi);
      vr += pr;
      vi += pi;
    }
    double sc = 1.0;
    if (rs) sc *= rs[row];
    if (cs) sc *= cs[col];
    vr *= sc; vi *= sc;
    double outr = a.alpha_re * vr - a.alpha_im * vi;
    double outi = a.alpha_re * vi + a.alpha_im * vr;
    T* p = C + (long)row * a.ldc + col;
    if (!beta0) {
      double cr, ci;
      ld(p, cr, ci);
      outr += a.beta_re * cr - a.beta_im * ci;
      outi += a.beta_re * ci + a.beta_im * cr;
    }
    st(p, outr, outi);
  }
}

// ---------------------------------------------------------------------------
// Launcher
// ---------------------------------------------------------------------------
template <typename K>
static hipError_t launch(K kern, const GemmArgs& a, int BM, int BN, hipStream_t s) {
  dim3 grid((a.n + BN - 1) / BN, (a.m + BM - 1) / BM, a.batch);
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Number of K chunks for an FP64 launch (1 = no split).  Model: the chip runs
// 256 workgroups per round (one per compute unit), each at SPLITK_CU_RATE; a
// launch of W equal workgroups takes ceil(W / 256) rounds.  Cutting K into sp
// chunks multiplies W by sp and divides a round by sp, and adds a reduction
// pass that writes and reads sp partial slabs.  The cheapest sp wins (by 5%
// at least), with chunks of SPLITK_MIN_K or more and within the caller's
// scratch.
constexpr int SPLITK_MIN_K = 128;
constexpr int SPLITK_MAX = 32;
constexpr long long SPLITK_MAX_TILES = 1024;
constexpr double SPLITK_CU_RATE = 0.3e12;      // FP64 MFMA flop/s of one compute unit
constexpr double SPLITK_REDUCE_BW = 4.0e12;    // bytes/s of the reduction pass
constexpr double SPLITK_LAUNCH_S = 5e-6;

static int splitk_chunks(const GemmArgs& a, int BM, int BN, size_t es) {
  if (!a.kws || a.dims || a.lower_band > 0 || a.k < 2 * SPLITK_MIN_K) return 1;
  const long long tiles = (long long)((a.n + BN - 1) / BN) * ((a.m + BM - 1) / BM) * a.batch;
  if (tiles >= SPLITK_MAX_TILES) return 1;
  const double wg_s = (es == 16 ? 8.0 : 2.0) * BM * BN * (double)a.k / SPLITK_CU_RATE;   // one unsplit tile
  const double slab = (double)es * a.m * a.n * a.batch;
  auto rounds = [](long long w) { return (double)((w + 255) / 256); };
  int best = 1;
  double best_t = rounds(tiles) * wg_s;
  const int spmax = std::min<long long>(SPLITK_MAX, a.k / SPLITK_MIN_K);
  for (int sp = 2; sp <= spmax; ++sp) {
    if (sp * slab > (double)a.kws_bytes) break;
    const double t = rounds(tiles * sp) * wg_s / sp + 2.0 * sp * slab / SPLITK_REDUCE_BW + SPLITK_LAUNCH_S;
    if (t < 0.95 * best_t) {
      best = sp;
      best_t = t;
    }
  }
  return best;
}

template <typename T, int BM, int BN>
static hipError_t launch_f64(const GemmArgs& a0, hipStream_t s) {
  GemmArgs a = a0;
  a.ksplit = splitk_chunks(a, BM, BN, sizeof(T));
  if (a.ksplit <= 1) {
    a.ksplit = 0;
    return launch(gemm_f64_kernel<T, BM, BN>, a, BM, BN, s);
  }
  dim3 grid((a.n + BN - 1) / BN, (a.m + BM - 1) / BM, a.batch * a.ksplit);
  hipLaunchKernelGGL((gemm_f64_kernel<T, BM, BN>), grid, dim3(256), 0, s, a);
  const long long mn = (long long)a.m * a.n;
  const unsigned gx = (unsigned)std::min<long long>(1024, (mn + 255) / 256);
  hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3(gx, a.batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t gemm(int dtype, int prec, const GemmArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return hipSuccess;
  // algorithmic flops: 8 per complex multiply-add (four real products), 2 per
  // real one; split-BF16x3 executes three bf16 products per multiply-add
  const bool cplx = dtype == C64 || dtype == C128;
  double flops = (cplx ? 8.0 : 2.0) * a.m * (double)a.n * a.k * a.batch;
  if (a.lower_band > 0 && !a.dims) {
    // only the output tiles the kernel computes (FP64 tiles: 128 x 64 complex, 128 x 128 real)
    const int bm = 128, bn = cplx ? 64 : 128;
    double cells = 0.0;
    for (int m0 = 0; m0 < a.m; m0 += bm)
      for (int n0 = 0; n0 < a.n; n0 += bn)
        if (n0 - (m0 + bm - 1) < a.lower_band) cells += (double)std::min(bm, a.m - m0) * std::min(bn, a.n - n0);
    flops *= cells / ((double)a.m * a.n);
  }
  if ((dtype == C64 || dtype == F32) && prec == PREC_BF16X3) flops *= 3.0;
  const char* cls = dtype == C128 ? "c128_fp64" : dtype == F64 ? "f64_fp64"
                  : prec == PREC_BF16X3 ? (dtype == C64 ? "c64_bf16x3" : "f32_bf16x3")
                  : (dtype == C64 ? "c64_fp32" : "f32_fp32");
  ProfScope ps(s, flops, cls);
  if (a.k <= 0) {
    // empty sum: C = beta * C
    return gemm_scale_c(dtype, a, s);
  }
  switch (dtype) {
    case C128:
      return launch_f64<cd, 128, 64>(a, s);
    case F64:
      return launch_f64<double, 128, 128>(a, s);
    case C64:
      if (prec == PREC_BF16X3) return launch(gemm_bf16x3_kernel<cf, 64, 64>, a, 64, 64, s);
      return launch(gemm_f32_kernel<cf, 128, 64>, a, 128, 64, s);
    case F32:
      if (prec == PREC_BF16X3) return launch(gemm_bf16x3_kernel<float, 128, 64>, a, 128, 64, s);
      return launch(gemm_f32_kernel<float, 128, 128>, a, 128, 128, s);
  }
  return hipErrorInvalidValue;
}

// C = beta * C for an empty contraction dimension.
template <typename T> struct RealOf;
template <> struct RealOf<double> { typedef double type; };
template <> struct RealOf<cd> { typedef double type; };
template <> struct RealOf<float> { typedef float type; };
template <> struct RealOf<cf> { typedef float type; };

template <typename T>
__global__ void scale_c_kernel(GemmArgs a) {
  typedef typename RealOf<T>::type R;
  const int b = blockIdx.y;
  int M, N, K;
  problem_dims(a, b, M, N, K);
  T* C = reinterpret_cast<T*>(a.C) + (long)b * a.sC;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < (long)M * N;
       idx += (long)gridDim.x * blockDim.x) {
    const int row = (int)(idx / N), col = (int)(idx % N);
    T* p = C + (long)row * a.ldc + col;
    R cr = 0, ci = 0;
    if (a.beta_re != 0.0 || a.beta_im != 0.0) ld(p, cr, ci);
    st(p, (R)(a.beta_re * cr - a.beta_im * ci), (R)(a.beta_re * ci + a.beta_im * cr));
  }
}

hipError_t gemm_scale_c(int dtype, const GemmArgs& a, hipStream_t s) {
  dim3 grid(256, a.batch);
  switch (dtype) {
    case C128: hipLaunchKernelGGL(scale_c_kernel<cd>, grid, dim3(256), 0, s, a); break;
    case F64: hipLaunchKernelGGL(scale_c_kernel<double>, grid, dim3(256), 0, s, a); break;
    case C64: hipLaunchKernelGGL(scale_c_kernel<cf>, grid, dim3(256), 0, s, a); break;
    case F32: hipLaunchKernelGGL(scale_c_kernel<float>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tci
