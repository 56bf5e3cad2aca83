// Split-BF16x3 GEMM on pre-split operand planes.
//
// A float operand x is split once into x = hi + lo with hi = rne_bf16(x) and
// lo = rne_bf16(x - hi) (both round-to-nearest-even, lo from the exact FP32
// difference).  For complex operands the planes are (re_hi, re_lo, im_hi,
// im_lo).  The planes of op(A) are stored [plane][Mp][Kp] and those of op(B)
// as [plane][Np][Kp] (k contiguous, zero padded to the tile sizes), which is
// the order in which one lane of v_mfma_f32_16x16x32_bf16 consumes 8
// consecutive k values of one row (A) or one column (B).  The product keeps
// three terms, hi*hi + hi*lo + lo*hi, accumulated in FP32; the complex
// product uses four real products.
//
// Tiles: 128 x 128 outputs per workgroup (8 waves, 64 x 32 each), k tile 32,
// two LDS stages: the next k tile is fetched into registers while the
// current stage feeds the matrix cores, then stored to the other stage, so
// that one barrier per k tile suffices.  Each 64-byte LDS row holds four
// 16-byte k chunks, chunk c of row r at position c ^ f(r) with
// f(r) = ((r >> 1) ^ (r >> 2)) & 3: both every 8 and every 16 consecutive
// rows that a 16-byte operand load touches then fall into distinct banks
// (measured: no LDS bank conflicts, where f(r) = (r >> 2) & 3 left 0.6 per
// access).
#include <type_traits>

#include "common.hpp"
#include "gemm.hpp"
#include "bf16x3.hpp"
#include "prof.hpp"

namespace tci {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int XBM = 128, XBN = 128, XBK = 32;

// ---------------------------------------------------------------------------
// Splitting: X(r, k) = src[r*ld + k] (mode 0) or src[k*ld + r] (mode 1), with
// optional conjugation; writes planes[p][r][k] for r < Rp, k < Kp (zero pad).
// Mode 1 goes through a 64 x 64 LDS tile so that reads and writes coalesce.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void getf(const T* p, float& r, float& i);
template <> __device__ inline void getf(const float* p, float& r, float& i) { r = *p; i = 0.f; }
template <> __device__ inline void getf(const cf* p, float& r, float& i) { const cf v = *p; r = v.x; i = v.y; }

__device__ inline void split1(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <typename T>
__global__ __launch_bounds__(256) void split_planes_kernel(const T* src, long long ld, long long ssrc, int mode,
                                                           int conj, int R, int K, __bf16* dst, int Rp, int Kp,
                                                           long long sdst) {
  constexpr bool CPLX = sizeof(T) == 8;
  __shared__ float tre[64][65], tim[64][65];
  const int b = blockIdx.z;
  const T* s = src + b * ssrc;
  __bf16* d = dst + b * sdst;
  const long long plane = (long long)Rp * Kp;
  const int r0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
  const int t = threadIdx.x;
  const float sg = conj ? -1.f : 1.f;
  if (mode == 0) {
    for (int e = t; e < 64 * 64; e += 256) {
      const int rr = e / 64, kk = e % 64;
      const int r = r0 + rr, k = k0 + kk;
      float vr = 0.f, vi = 0.f;
      if (r < R && k < K) getf(s + (long long)r * ld + k, vr, vi);
      tre[rr][kk] = vr;
      tim[rr][kk] = sg * vi;
    }
  } else {
    for (int e = t; e < 64 * 64; e += 256) {
      const int kk = e / 64, rr = e % 64;
      const int r = r0 + rr, k = k0 + kk;
      float vr = 0.f, vi = 0.f;
      if (r < R && k < K) getf(s + (long long)k * ld + r, vr, vi);
      tre[rr][kk] = vr;
      tim[rr][kk] = sg * vi;
    }
  }
  __syncthreads();
  for (int e = t; e < 64 * 64; e += 256) {
    const int rr = e / 64, kk = e % 64;
    const int r = r0 + rr, k = k0 + kk;
    if (r >= Rp || k >= Kp) continue;
    const long long o = (long long)r * Kp + k;
    __bf16 h, l;
    split1(tre[rr][kk], h, l);
    d[o] = h;
    d[plane + o] = l;
    if constexpr (CPLX) {
      split1(tim[rr][kk], h, l);
      d[2 * plane + o] = h;
      d[3 * plane + o] = l;
    }
  }
}

hipError_t split_planes(int dtype, const void* src, long long ld, long long ssrc, int mode, int conj, int R, int K,
                        void* dst, int Rp, int Kp, long long sdst, int batch, hipStream_t s) {
  dim3 grid((Kp + 63) / 64, (Rp + 63) / 64, batch);
  if (dtype == C64)
    hipLaunchKernelGGL(split_planes_kernel<cf>, grid, dim3(256), 0, s, (const cf*)src, ld, ssrc, mode, conj, R, K,
                       (__bf16*)dst, Rp, Kp, sdst);
  else if (dtype == F32)
    hipLaunchKernelGGL(split_planes_kernel<float>, grid, dim3(256), 0, s, (const float*)src, ld, ssrc, mode, conj, R,
                       K, (__bf16*)dst, Rp, Kp, sdst);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GEMM on planes.  Workgroup tile 128 x 128 with 8 waves in a 2 x 4 grid,
// each wave 64 x 32 (4 x 2 MFMA blocks), so that a wave needs at most 256
// registers and two waves share each SIMD: one wave's LDS and global-load
// waits are covered by the other's matrix work.  Staging: each plane tile is
// 128 rows x 32 k = 8 KB = 512 chunks of 16 bytes; thread t moves chunk t of
// every plane of both operands, straight from global memory into LDS
// (global_load_lds, no staging registers), one k tile ahead.
// ---------------------------------------------------------------------------
constexpr int XWM = 64, XWN = 32;   // wave tile
template <bool CPLX>
__global__ __launch_bounds__(512) void gemm_planes_kernel(PlaneGemmArgs a) {
  constexpr int NP = CPLX ? 4 : 2;
  constexpr int IM = XWM / 16, JN = XWN / 16;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][NP][XBM][XBK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][NP][XBN][XBK];
  // tile coordinates, XCD-aware as in the plain GEMM
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const long total = (long)gx * gy * gz;
  long lin = blockIdx.x + (long)gx * (blockIdx.y + (long)gy * blockIdx.z);
  if ((total & 7) == 0) lin = (lin & 7) * (total >> 3) + (lin >> 3);
  // grouped order inside a problem: runs of 8 row tiles share each column
  // tile, so that the tiles an XCD runs at once re-use both operand panels
  const long per_b = (long)gx * gy;
  const int b = (int)(lin / per_b);
  const int tt = (int)(lin % per_b);
  constexpr int GM = 8;
  const int gsize = GM * gx;
  const int first = (tt / gsize) * GM;
  const int gm = min(GM, gy - first);
  const int rr = tt % gsize;
  const int tm = first + rr % gm, tn = rr / gm;
  const int m0 = tm * XBM, n0 = tn * XBN;
  const __bf16* A = a.Ap + b * a.sAp;
  const __bf16* B = a.Bp + b * a.sBp;
  const long long pa = (long long)a.Mp * a.Kp, pb = (long long)a.Np * a.Kp;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wm = wid >> 2, wn = wid & 3;
  const int lr = lane & 15, lk = lane >> 4;
  const int rd = 8 * (lk ^ (((lr >> 1) ^ (lr >> 2)) & 3));   // swizzled k offset of this lane's operand chunk

  // acc_ii collects the im x im products, subtracted from acc_re in the
  // epilogue (no negated operand copies in the inner loop)
  f4v acc_re[IM][JN], acc_im[IM][JN], acc_ii[IM][JN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      acc_re[i][j] = f4v{0, 0, 0, 0};
      acc_im[i][j] = f4v{0, 0, 0, 0};
      acc_ii[i][j] = f4v{0, 0, 0, 0};
    }

  // Global -> LDS without registers: each wave moves rows 16 wid .. 16 wid + 15
  // of every plane tile, lane l writing the 16 bytes at l * 16 of that
  // 1 KB block (row 16 wid + l / 4, chunk position l & 3), so it loads the
  // k chunk that the swizzle puts there, (l & 3) ^ swz(row).
  const int srow = t >> 2, skc = t & 3;
  const int gk = 8 * (skc ^ (((srow >> 1) ^ (srow >> 2)) & 3));
  typedef __attribute__((address_space(3))) void lds_void;
  typedef __attribute__((address_space(1))) void glb_void;
  const __bf16* ga = A + (long long)(m0 + srow) * a.Kp + gk;
  const __bf16* gb = B + (long long)(n0 + srow) * a.Kp + gk;
  auto issue = [&](int k0, int st) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      __builtin_amdgcn_global_load_lds((glb_void*)(ga + p * pa + k0), (lds_void*)&As[st][p][16 * wid][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds((glb_void*)(gb + p * pb + k0), (lds_void*)&Bs[st][p][16 * wid][0], 16, 0, 0);
    }
  };

  const int nk = a.Kp / XBK;
  issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    // tile kt has landed for every wave (the barrier waits for this wave's
    // loads), and every wave is done reading the other buffer
    __syncthreads();
    bf8v fa[NP][IM], fb[NP][JN];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int i = 0; i < IM; ++i)
        fa[p][i] = *reinterpret_cast<const bf8v*>(&As[cur][p][wm * XWM + i * 16 + lr][rd]);
#pragma unroll
      for (int j = 0; j < JN; ++j)
        fb[p][j] = *reinterpret_cast<const bf8v*>(&Bs[cur][p][wn * XWN + j * 16 + lr][rd]);
    }
    // the next tile's loads go out after this step's fragment reads (the
    // compiler waits for those reads before issuing them)
    if (more) issue((kt + 1) * XBK, cur ^ 1);
#pragma unroll
    for (int i = 0; i < IM; ++i) {
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[0][j], acc_re[i][j], 0, 0, 0);
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[1][j], acc_re[i][j], 0, 0, 0);
        acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[0][j], acc_re[i][j], 0, 0, 0);
        if constexpr (CPLX) {
          acc_ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[2][j], acc_ii[i][j], 0, 0, 0);
          acc_ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[3][j], acc_ii[i][j], 0, 0, 0);
          acc_ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[3][i], fb[2][j], acc_ii[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[2][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[3][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[2][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[0][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[1][j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[3][i], fb[0][j], acc_im[i][j], 0, 0, 0);
        }
      }
    }
  }

  // epilogue: C = alpha * acc + beta * C (rows 4*(l/16)+r, column l%16 of each block)
  const bool beta0 = (a.beta_re == 0.0 && a.beta_im == 0.0);
  const float ar = (float)a.alpha_re, ai = (float)a.alpha_im, br = (float)a.beta_re, bi = (float)a.beta_im;
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * XWM + i * 16 + 4 * lk + r;
        const int col = n0 + wn * XWN + j * 16 + lr;
        if (row < a.m && col < a.n) {
          const float vr = CPLX ? acc_re[i][j][r] - acc_ii[i][j][r] : acc_re[i][j][r];
          const float vi = CPLX ? acc_im[i][j][r] : 0.f;
          float orr = ar * vr - ai * vi, oi = ar * vi + ai * vr;
          if constexpr (CPLX) {
            cf* p = reinterpret_cast<cf*>(a.C) + b * a.sC + (long long)row * a.ldc + col;
            if (!beta0) {
              const cf c = *p;
              orr += br * c.x - bi * c.y;
              oi += br * c.y + bi * c.x;
            }
            *p = cf{orr, oi};
          } else {
            float* p = reinterpret_cast<float*>(a.C) + b * a.sC + (long long)row * a.ldc + col;
            if (!beta0) orr += br * *p;
            *p = orr;
          }
        }
      }
}

hipError_t gemm_planes(int dtype, const PlaneGemmArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return hipSuccess;
  if (a.Mp % XBM || a.Np % XBN || a.Kp % XBK || a.Mp < a.m || a.Np < a.n) return hipErrorInvalidValue;
  dim3 grid(a.Np / XBN, a.Mp / XBM, a.batch);
  const bool cplx = dtype == C64;
  const double flops = (cplx ? 8.0 : 2.0) * 3.0 * a.m * (double)a.n * a.k * a.batch;
  ProfScope ps(s, flops, cplx ? "c64_bf16x3_planes" : "f32_bf16x3_planes");
  if (cplx) hipLaunchKernelGGL(gemm_planes_kernel<true>, grid, dim3(512), 0, s, a);
  else hipLaunchKernelGGL(gemm_planes_kernel<false>, grid, dim3(512), 0, s, a);
  return hipGetLastError();
}

int planes_of(int dtype) { return dtype == C64 ? 4 : 2; }
int pad_rows(int r) { return (r + XBM - 1) / XBM * XBM; }
int pad_k(int k) { return (k + XBK - 1) / XBK * XBK; }

// op(A) (M x K) -> planes [P][Mp][Kp]
hipError_t split_a(int dtype, int opA, const void* A, long long lda, long long sA, int M, int K, void* dst, int batch,
                   hipStream_t s) {
  const int mode = (opA == OP_N || opA == OP_R) ? 0 : 1;
  const int conj = (opA == OP_C || opA == OP_R) ? 1 : 0;
  const int Mp = pad_rows(M), Kp = pad_k(K);
  return split_planes(dtype, A, lda, sA, mode, conj, M, K, dst, Mp, Kp, (long long)planes_of(dtype) * Mp * Kp, batch, s);
}

// op(B) (K x N) -> planes [P][Np][Kp] of op(B)^T
hipError_t split_b(int dtype, int opB, const void* B, long long ldb, long long sB, int K, int N, void* dst, int batch,
                   hipStream_t s) {
  const int mode = (opB == OP_N || opB == OP_R) ? 1 : 0;
  const int conj = (opB == OP_C || opB == OP_R) ? 1 : 0;
  const int Np = pad_rows(N), Kp = pad_k(K);
  return split_planes(dtype, B, ldb, sB, mode, conj, N, K, dst, Np, Kp, (long long)planes_of(dtype) * Np * Kp, batch, s);
}

size_t planes_bytes(int dtype, int rows, int k) {
  return sizeof(__bf16) * (size_t)planes_of(dtype) * pad_rows(rows) * pad_k(k);
}

}  // namespace tci

namespace tci {

// The middle step of the effective-Hamiltonian matvec fused with the split of
// its result:  X2[a][j][b] = sum_k W12[k][j] X1[a][k][b]  (k, j < KW), in FP32,
// written straight into the bf16 planes of the R-step operand, whose row is
// (a, j / w) and whose k index is (j % w) * chir + b.  One thread per (a, b);
// W12 sits in LDS.  The padding of the planes is never written (zeroed once).
template <bool CPLX, int KW>
__global__ __launch_bounds__(256) void w12_planes_kernel(const void* X1v, const void* W12v, int chil, int chir,
                                                         int w, __bf16* planes, int Mp, int Kp) {
  typedef typename std::conditional<CPLX, cf, float>::type T;
  __shared__ float Wr[KW * KW], Wi[KW * KW];
  const T* W12 = static_cast<const T*>(W12v);
  for (int e = threadIdx.x; e < KW * KW; e += 256) {
    float r, i;
    getf(W12 + e, r, i);
    Wr[e] = r;
    Wi[e] = i;
  }
  __syncthreads();
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= (long long)chil * chir) return;
  const int a = (int)(idx / chir), b = (int)(idx % chir);
  const T* x1 = static_cast<const T*>(X1v) + (long long)a * KW * chir + b;
  float xr[KW], xi[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k) getf(x1 + (long long)k * chir, xr[k], xi[k]);
  const long long plane = (long long)Mp * Kp;
  const int dd = KW / w;
#pragma unroll 4
  for (int j = 0; j < KW; ++j) {
    float yr = 0.f, yi = 0.f;
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const float wr = Wr[k * KW + j], wi = Wi[k * KW + j];
      yr += wr * xr[k];
      if constexpr (CPLX) {
        yr -= wi * xi[k];
        yi += wr * xi[k] + wi * xr[k];
      }
    }
    const long long o = (long long)(a * dd + j / w) * Kp + (long long)(j % w) * chir + b;
    __bf16 h, l;
    split1(yr, h, l);
    planes[o] = h;
    planes[plane + o] = l;
    if constexpr (CPLX) {
      split1(yi, h, l);
      planes[2 * plane + o] = h;
      planes[3 * plane + o] = l;
    }
  }
}

hipError_t w12_to_planes(int dtype, const void* X1, const void* W12, int chil, int kw, int chir, int w, void* planes,
                         int Mp, int Kp, hipStream_t s) {
  if (kw != 20) return hipErrorInvalidValue;
  const long long tot = (long long)chil * chir;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  const double flops = (dtype == C64 ? 8.0 : 2.0) * (double)kw * kw * tot;
  ProfScope ps(s, flops, dtype == C64 ? "c64_fp32_w12" : "f32_fp32_w12");
  if (dtype == C64)
    hipLaunchKernelGGL((w12_planes_kernel<true, 20>), dim3(grid), dim3(256), 0, s, X1, W12, chil, chir, w,
                       (__bf16*)planes, Mp, Kp);
  else if (dtype == F32)
    hipLaunchKernelGGL((w12_planes_kernel<false, 20>), dim3(grid), dim3(256), 0, s, X1, W12, chil, chir, w,
                       (__bf16*)planes, Mp, Kp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace tci
