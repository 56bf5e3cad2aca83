// U(1) block-sparse site tensors and the batched block-sparse two-site
// update (the block form of the dense update of Sec. II.B, one truncation
// across all charge sectors of a bond).
//
// Pipeline of tci_bs_two_site_update_batched for n updates:
//   1. host plan: the sector layout of every new bond, and one GEMM per
//      (output sub-block, contributing input pair) with the gate coefficient
//      as alpha;
//   2. the sector matrices of all updates are built by grouped FP32 GEMMs,
//      one launch per accumulation phase (a sub-block has at most two
//      contributions), tile shape autotuned;
//   3. sectors are padded into square FP64 batches by size class and split by
//      the plain truncated SVD's eigenvalue stage (Gram, tridiagonal
//      reduction, all eigenvalues);
//   4. per update the singular values of all sectors are merged and cut once
//      by the trunc_svd rule; the vector stage then runs with the per-sector
//      kept counts;
//   5. one scatter launch writes the kept factors into the output blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "../../include/tci_c.h"
#include "bsparse.hpp"
#include "common.hpp"
#include "grouped.hpp"
#include "prof.hpp"
#include "runtime.hpp"
#include "tsvd.hpp"
#include "vecops.hpp"

struct tci_bs_tensor_s {
  struct Blk {
    int a, s, b;
    int64_t off;
  };
  int dtype = TCI_F32;
  std::vector<int32_t> ql, qr;
  std::vector<int64_t> dl, dr;
  std::vector<Blk> blocks;
  int64_t nelem = 0;
  void* data = nullptr;
  size_t cap = 0;
  tci_allocator al{};  // allocator of data (the creating context's)
  uint32_t magic = 0xB5B5A11Cu;
};

namespace tci {
namespace {

constexpr int SPIN_CHARGE[2] = {1, -1};

tci_status bs_check(tci_bs_tensor t) {
  if (!t || t->magic != 0xB5B5A11Cu) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "invalid block-sparse tensor handle");
  return TCI_OK;
}

int find_charge(const std::vector<int32_t>& q, int c) {
  for (size_t i = 0; i < q.size(); ++i)
    if (q[i] == c) return (int)i;
  return -1;
}

// (Re)define the structure of t and make sure its buffer holds it.
tci_status bs_define(tci_context ctx, tci_bs_tensor t, int dtype, const std::vector<int32_t>& ql,
                     const std::vector<int64_t>& dl, const std::vector<int32_t>& qr, const std::vector<int64_t>& dr) {
  if (dtype != TCI_F32) TCI_RET(TCI_ERR_UNSUPPORTED, "block-sparse tensors are F32");
  if (ql.size() != dl.size() || qr.size() != dr.size()) TCI_RET(TCI_ERR_SHAPE, "bond arrays");
  for (auto x : dl)
    if (x < 0) TCI_RET(TCI_ERR_SHAPE, "negative sector dimension");
  for (auto x : dr)
    if (x < 0) TCI_RET(TCI_ERR_SHAPE, "negative sector dimension");
  for (size_t i = 0; i < ql.size(); ++i)
    for (size_t j = i + 1; j < ql.size(); ++j)
      if (ql[i] == ql[j]) TCI_RET(TCI_ERR_SHAPE, "repeated charge in the left bond");
  for (size_t i = 0; i < qr.size(); ++i)
    for (size_t j = i + 1; j < qr.size(); ++j)
      if (qr[i] == qr[j]) TCI_RET(TCI_ERR_SHAPE, "repeated charge in the right bond");
  t->dtype = dtype;
  t->ql = ql; t->dl = dl; t->qr = qr; t->dr = dr;
  t->blocks.clear();
  int64_t off = 0;
  for (size_t a = 0; a < ql.size(); ++a)
    for (int s = 0; s < 2; ++s) {
      const int b = find_charge(qr, ql[a] + SPIN_CHARGE[s]);
      if (b < 0) continue;
      t->blocks.push_back({(int)a, s, b, off});
      off += dl[a] * dr[b];
    }
  t->nelem = off;
  const size_t bytes = (size_t)std::max<int64_t>(off, 1) * elem_bytes(dtype);
  if (t->cap < bytes) {
    if (t->data) {
      TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
      dev_free(t->al, t->data, t->cap, ctx->stream);
    }
    t->data = nullptr;
    t->cap = 0;
    TCI_CHECK_HIP(hipSetDevice(ctx->device));
    t->data = dev_alloc(ctx->al, bytes, ctx->stream);
    if (!t->data) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "block-sparse storage");
    t->al = ctx->al;
    t->cap = bytes;
  }
  return TCI_OK;
}

const tci_bs_tensor_s::Blk* find_block(const tci_bs_tensor_s* t, int a, int s, int b) {
  for (const auto& k : t->blocks)
    if (k.a == a && k.s == s && k.b == b) return &k;
  return nullptr;
}

struct Sector {
  int u = 0, q = 0;
  std::vector<std::pair<int, int>> rows;   // (a, s1')
  std::vector<std::pair<int, int>> cols;   // (s2', b)
  std::vector<int> roff, coff;
  int r = 0, c = 0;
  float* buf = nullptr;
  int bucket = -1, slot = -1;
  int kept = 0;
};

// Recorded HIP graphs of the first half of the update (sector products,
// padding, Gram matrices, tridiagonal reductions, eigenvalues), keyed by the
// problem structure and the workspace addresses the recorded kernels use.
// A structure is recorded the second time it is seen and replayed from the
// third time on; the tables the kernels read (block pointers, gate
// coefficients, pad descriptors) are uploaded before every launch.
struct BsGraphEntry {
  int seen = 0;
  bool failed = false;
  hipGraphExec_t exec = nullptr;
  std::vector<size_t> arena_after;
  std::vector<TsvdStage> stages;
};
// Side streams on which the size classes' eigenvalue stages run side by
// side (each class is a batch of a few hundred small problems, too few
// workgroups to fill the GPU on its own), with the events that fork them
// from and join them back to the calling stream; inside a recording the
// fork and join become edges of the graph.
constexpr int BS_SIDE_STREAMS = 7;
struct BsGraphCache {
  hipStream_t cs = nullptr;
  hipStream_t side[BS_SIDE_STREAMS] = {};
  hipEvent_t fork = nullptr, join[BS_SIDE_STREAMS] = {};
  std::map<std::vector<long long>, BsGraphEntry> m;
  ~BsGraphCache() {
    for (auto& kv : m)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (cs) (void)hipStreamDestroy(cs);
    for (int k = 0; k < BS_SIDE_STREAMS; ++k) {
      if (side[k]) (void)hipStreamDestroy(side[k]);
      if (join[k]) (void)hipEventDestroy(join[k]);
    }
    if (fork) (void)hipEventDestroy(fork);
  }
};
constexpr size_t BS_GRAPH_MAX_ENTRIES = 16;

BsGraphCache* bs_cache(tci_context ctx) {
  if (!ctx->bs_graphs)
    ctx->bs_graphs = std::shared_ptr<void>(new BsGraphCache(), [](void* q) { delete static_cast<BsGraphCache*>(q); });
  return static_cast<BsGraphCache*>(ctx->bs_graphs.get());
}

// Creates the side streams (default priority) and events once per context.
tci_status bs_side_init(BsGraphCache* gc) {
  if (gc->fork) return TCI_OK;
  for (int k = 0; k < BS_SIDE_STREAMS; ++k) {   // a failed earlier attempt keeps what it made
    if (!gc->side[k]) TCI_CHECK_HIP(hipStreamCreateWithFlags(&gc->side[k], hipStreamNonBlocking));
    if (!gc->join[k]) TCI_CHECK_HIP(hipEventCreateWithFlags(&gc->join[k], hipEventDisableTiming));
  }
  TCI_CHECK_HIP(hipEventCreateWithFlags(&gc->fork, hipEventDisableTiming));
  return TCI_OK;
}

// Host form of the truncation rule (Spec, trunc_svd, rules a-c) on the
// merged descending values; W the total weight.
void trunc_rule_host(const std::vector<double>& s, double W, const TruncParams& tp, int& chi, double& eps) {
  const int L = (int)s.size();
  int n_a = 0;
  while (n_a < L && s[n_a] >= tp.s_min) ++n_a;
  auto eps_of = [&](double kept) { return W > 0.0 ? std::max(W - kept, 0.0) / W : 0.0; };
  double kept = 0.0;
  if (n_a <= tp.chi_min) {
    chi = n_a;
    for (int j = 0; j < chi; ++j) kept += s[j] * s[j];
  } else {
    const int lim = std::min(tp.chi_max, n_a);
    chi = tp.chi_min;
    for (int j = 0; j < chi; ++j) kept += s[j] * s[j];
    while (chi < lim && eps_of(kept) > tp.target) {
      kept += s[chi] * s[chi];
      ++chi;
    }
  }
  if (chi < 1 && L > 0) {
    chi = 1;
    kept = s[0] * s[0];
  }
  eps = eps_of(kept);
}

}  // namespace
}  // namespace tci

using namespace tci;

extern "C" {

tci_status tci_bs_create(tci_context ctx, tci_dtype dtype, int n_left, const int32_t* q_left, const int64_t* d_left,
                         int n_right, const int32_t* q_right, const int64_t* d_right, tci_bs_tensor* out) try {
  if (!ctx || !out || n_left < 0 || n_right < 0) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "bad arguments");
  if ((n_left > 0 && (!q_left || !d_left)) || (n_right > 0 && (!q_right || !d_right)))
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null bond arrays");
  tci_bs_tensor t = new tci_bs_tensor_s();
  tci_status st = bs_define(ctx, t, dtype, std::vector<int32_t>(q_left, q_left + n_left),
                            std::vector<int64_t>(d_left, d_left + n_left),
                            std::vector<int32_t>(q_right, q_right + n_right),
                            std::vector<int64_t>(d_right, d_right + n_right));
  if (st != TCI_OK) {
    if (t->data) dev_free(t->al, t->data, t->cap, ctx->stream);
    delete t;
    return st;
  }
  *out = t;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_destroy(tci_context ctx, tci_bs_tensor t) try {
  if (!t) return TCI_OK;
  TCI_TRY(bs_check(t));
  if (t->data) {
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    dev_free(t->al, t->data, t->cap, ctx ? ctx->stream : nullptr);
  }
  t->magic = 0;
  delete t;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_dims(tci_context ctx, tci_bs_tensor t, int* n_left, int* n_right, int* n_blocks, int64_t* n_elems) try {
  (void)ctx;
  TCI_TRY(bs_check(t));
  if (n_left) *n_left = (int)t->ql.size();
  if (n_right) *n_right = (int)t->qr.size();
  if (n_blocks) *n_blocks = (int)t->blocks.size();
  if (n_elems) *n_elems = t->nelem;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_bonds(tci_context ctx, tci_bs_tensor t, int32_t* q_left, int64_t* d_left, int32_t* q_right,
                        int64_t* d_right) try {
  (void)ctx;
  TCI_TRY(bs_check(t));
  for (size_t i = 0; i < t->ql.size(); ++i) {
    if (q_left) q_left[i] = t->ql[i];
    if (d_left) d_left[i] = t->dl[i];
  }
  for (size_t i = 0; i < t->qr.size(); ++i) {
    if (q_right) q_right[i] = t->qr[i];
    if (d_right) d_right[i] = t->dr[i];
  }
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_block_info(tci_context ctx, tci_bs_tensor t, int i, int* a, int* s, int* b, int64_t* offset) try {
  (void)ctx;
  TCI_TRY(bs_check(t));
  if (i < 0 || i >= (int)t->blocks.size()) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "block index");
  const auto& k = t->blocks[i];
  if (a) *a = k.a;
  if (s) *s = k.s;
  if (b) *b = k.b;
  if (offset) *offset = k.off;
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_from_host(tci_context ctx, tci_bs_tensor t, const void* host, size_t bytes) try {
  if (!ctx || !host) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_TRY(bs_check(t));
  if (bytes != (size_t)t->nelem * elem_bytes(t->dtype)) TCI_RET(TCI_ERR_SHAPE, "byte count");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  if (bytes) TCI_CHECK_HIP(hipMemcpyAsync(t->data, host, bytes, hipMemcpyHostToDevice, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_to_host(tci_context ctx, tci_bs_tensor t, void* host, size_t bytes) try {
  if (!ctx || !host) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  TCI_TRY(bs_check(t));
  if (bytes != (size_t)t->nelem * elem_bytes(t->dtype)) TCI_RET(TCI_ERR_SHAPE, "byte count");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  if (bytes) TCI_CHECK_HIP(hipMemcpyAsync(host, t->data, bytes, hipMemcpyDeviceToHost, ctx->stream));
  TCI_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return TCI_OK;
} TCI_API_CATCH

tci_status tci_bs_two_site_update_batched(tci_context ctx, int n, const tci_bs_tensor* A, const tci_bs_tensor* B,
                                          const tci_tensor* gates, const tci_update_params* params,
                                          const int64_t* chi_max_each, tci_bs_tensor* A_out, tci_tensor* s_out,
                                          tci_bs_tensor* B_out, tci_update_info* infos) try {
  if (!ctx || n < 1 || !A || !B || !A_out || !s_out || !B_out) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null argument");
  tci_update_params p;
  if (params) p = *params;
  else tci_update_params_default(&p);
  if (p.chi_min < 1 || p.chi_max < 1 || p.chi_min > p.chi_max)
    TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need 1 <= chi_min <= chi_max");
  if (chi_max_each)
    for (int u = 0; u < n; ++u)
      if (chi_max_each[u] < p.chi_min) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "need chi_min <= chi_max_each[i]");
  if (p.direction != TCI_DIR_LEFT && p.direction != TCI_DIR_RIGHT) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "direction");
  TCI_CHECK_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  for (int u = 0; u < n; ++u) {
    TCI_TRY(bs_check(A[u]));
    TCI_TRY(bs_check(B[u]));
    TCI_TRY(bs_check(A_out[u]));
    TCI_TRY(bs_check(B_out[u]));
    if (!s_out[u]) TCI_RET(TCI_ERR_INVALID_ARGUMENT, "null s_out");
    if (A[u]->dtype != TCI_F32 || B[u]->dtype != TCI_F32) TCI_RET(TCI_ERR_UNSUPPORTED, "block-sparse update is F32");
    if (A[u]->qr != B[u]->ql || A[u]->dr != B[u]->dl) TCI_RET(TCI_ERR_SHAPE, "A's right bond differs from B's left");
    if (A_out[u] == A[u] || A_out[u] == B[u] || B_out[u] == A[u] || B_out[u] == B[u] || A_out[u] == B_out[u])
      TCI_RET(TCI_ERR_INVALID_ARGUMENT, "outputs must be distinct from the inputs");
  }
  Trace tr(ctx, "bs_two_site_update_batched", std::to_string(n));
  ctx->arena.reset();

  // gates on the host (identity when absent)
  std::vector<std::array<double, 16>> G(n);
  for (int u = 0; u < n; ++u) {
    G[u].fill(0.0);
    for (int k = 0; k < 4; ++k) G[u][k * 5] = 1.0;
    if (gates && gates[u]) {
      const tci_tensor g = gates[u];
      if (tsize(g) != 16) TCI_RET(TCI_ERR_SHAPE, "gate must have 16 elements");
      if (g->dtype == TCI_F32) {
        float h[16];
        TCI_CHECK_HIP(hipMemcpyAsync(h, g->data, sizeof(h), hipMemcpyDeviceToHost, st));
        TCI_CHECK_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < 16; ++k) G[u][k] = h[k];
      } else if (g->dtype == TCI_F64) {
        TCI_CHECK_HIP(hipMemcpyAsync(G[u].data(), g->data, sizeof(double) * 16, hipMemcpyDeviceToHost, st));
        TCI_CHECK_HIP(hipStreamSynchronize(st));
      } else {
        TCI_RET(TCI_ERR_DTYPE, "gate must be real (F32 or F64)");
      }
    }
  }

  // 1. sector layout of every new bond
  std::vector<Sector> secs;
  std::vector<std::vector<int>> secs_of(n);
  size_t sec_elems = 0;
  for (int u = 0; u < n; ++u) {
    const auto* a = A[u];
    const auto* b = B[u];
    std::map<int, Sector> by_q;
    for (size_t ia = 0; ia < a->ql.size(); ++ia)
      for (int s1 = 0; s1 < 2; ++s1)
        if (a->dl[ia] > 0) by_q[a->ql[ia] + SPIN_CHARGE[s1]].rows.push_back({(int)ia, s1});
    for (int s2 = 0; s2 < 2; ++s2)
      for (size_t ib = 0; ib < b->qr.size(); ++ib)
        if (b->dr[ib] > 0) by_q[b->qr[ib] - SPIN_CHARGE[s2]].cols.push_back({s2, (int)ib});
    for (auto& kv : by_q) {
      Sector sc = kv.second;
      if (sc.rows.empty() || sc.cols.empty()) continue;
      sc.u = u;
      sc.q = kv.first;
      for (auto& rp : sc.rows) {
        sc.roff.push_back(sc.r);
        sc.r += (int)a->dl[rp.first];
      }
      for (auto& cp : sc.cols) {
        sc.coff.push_back(sc.c);
        sc.c += (int)b->dr[cp.second];
      }
      secs_of[u].push_back((int)secs.size());
      sec_elems += (size_t)sc.r * sc.c;
      secs.push_back(std::move(sc));
    }
  }
  float* sbuf = static_cast<float*>(ctx->arena.get(sizeof(float) * std::max<size_t>(sec_elems, 1)));
  float* scratch = static_cast<float*>(ctx->arena.get(sizeof(float) * std::max<size_t>(sec_elems, 1)));
  if (!sbuf || !scratch) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "sector buffers");
  {
    size_t off = 0;
    for (auto& sc : secs) {
      sc.buf = sbuf + off;
      off += (size_t)sc.r * sc.c;
    }
  }

  // 2. grouped products, at most two accumulation phases
  std::vector<GroupProb> phase[2];
  for (auto& sc : secs) {
    const auto* a = A[sc.u];
    const auto* b = B[sc.u];
    const auto& g = G[sc.u];
    for (size_t ri = 0; ri < sc.rows.size(); ++ri) {
      const int ia = sc.rows[ri].first, s1p = sc.rows[ri].second;
      for (size_t ci = 0; ci < sc.cols.size(); ++ci) {
        const int s2p = sc.cols[ci].first, ib = sc.cols[ci].second;
        int ph = 0;
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s2 = 0; s2 < 2; ++s2) {
            if (SPIN_CHARGE[s1] + SPIN_CHARGE[s2] != SPIN_CHARGE[s1p] + SPIN_CHARGE[s2p]) continue;
            const double coef = g[(s1p * 2 + s2p) * 4 + (s1 * 2 + s2)];
            if (coef == 0.0) continue;
            const int im = find_charge(a->qr, a->ql[ia] + SPIN_CHARGE[s1]);
            if (im < 0 || a->dr[im] == 0) continue;
            const auto* ba = find_block(a, ia, s1, im);
            const auto* bb = find_block(b, im, s2, ib);
            if (!ba || !bb) continue;
            GroupProb gp{};
            gp.a = static_cast<const float*>(a->data) + ba->off;
            gp.b = static_cast<const float*>(b->data) + bb->off;
            gp.c = sc.buf + (long long)sc.roff[ri] * sc.c + sc.coff[ci];
            gp.m = (int)a->dl[ia];
            gp.n = (int)b->dr[ib];
            gp.k = (int)a->dr[im];
            gp.lda = gp.k;
            gp.ldb = gp.n;
            gp.ldc = sc.c;
            gp.alpha = (float)coef;
            gp.beta = 1.f;
            if (ph > 1) TCI_RET(TCI_ERR_UNSUPPORTED, "gate is not charge conserving");
            phase[ph++].push_back(gp);
          }
      }
    }
  }
  // tables of the two accumulation phases (uploaded, tile shape tuned)
  GroupedPlan plan[2];
  {
    const long long shift = (long long)(scratch - sbuf);
    for (int ph = 0; ph < 2; ++ph) {
      const size_t np = std::max<size_t>(1, phase[ph].size());
      GroupProb* P_dev = static_cast<GroupProb*>(ctx->arena.get(sizeof(GroupProb) * np));
      int* t0_dev = static_cast<int*>(ctx->arena.get(sizeof(int) * np));
      if (!P_dev || !t0_dev) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "grouped GEMM tables");
      TCI_CHECK_HIP(grouped_prepare(ctx->device, phase[ph], P_dev, t0_dev, shift, st, plan[ph]));
    }
  }

  // 3. size classes (square padding to a multiple of 64) and their buffers
  std::map<int, std::vector<int>> classes;   // S -> sector ids
  for (size_t i = 0; i < secs.size(); ++i) {
    const int S = ((std::max(secs[i].r, secs[i].c) + 63) / 64) * 64;
    secs[i].bucket = S;
    secs[i].slot = (int)classes[S].size();
    classes[S].push_back((int)i);
  }
  struct Bucket {
    int S = 0;
    std::vector<int> ids;
    double* theta = nullptr;
    PadDesc* pd = nullptr;
    TsvdStage stage;
    std::vector<double> lam, total;
  };
  std::vector<Bucket> buckets;
  {
    std::vector<std::vector<PadDesc>> hps;
    for (auto& kv : classes) {
      Bucket bk;
      bk.S = kv.first;
      bk.ids = kv.second;
      const int nb = (int)bk.ids.size(), S = bk.S;
      bk.theta = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)nb * S * S));
      bk.pd = static_cast<PadDesc*>(ctx->arena.get(sizeof(PadDesc) * nb));
      if (!bk.theta || !bk.pd) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "sector batches");
      std::vector<PadDesc> hp(nb);
      for (int i = 0; i < nb; ++i) hp[i] = PadDesc{secs[bk.ids[i]].buf, secs[bk.ids[i]].r, secs[bk.ids[i]].c};
      TCI_CHECK_HIP(hipMemcpyAsync(bk.pd, hp.data(), sizeof(PadDesc) * nb, hipMemcpyHostToDevice, st));
      hps.push_back(std::move(hp));
      buckets.push_back(std::move(bk));
    }
    TCI_CHECK_HIP(hipStreamSynchronize(st));   // host tables leave scope
  }

  // the recordable first half: products, padding, eigenvalue stage
  // The size classes are independent after the products: class 0 stays on
  // the calling stream, the others run on side streams forked from it after
  // the products and joined back before the phase ends.
  BsGraphCache* sidec = bs_cache(ctx);
  TCI_TRY(bs_side_init(sidec));
  auto phase1 = [&](hipStream_t s1) -> tci_status {
    TCI_CHECK_HIP(zero_fill(sbuf, sizeof(float) * sec_elems, s1));
    for (int ph = 0; ph < 2; ++ph) TCI_CHECK_HIP(grouped_launch(plan[ph], s1));
    const int nside = std::min<int>(BS_SIDE_STREAMS, (int)buckets.size() - 1);
    if (nside > 0) {
      TCI_CHECK_HIP(hipEventRecord(sidec->fork, s1));
      for (int k = 0; k < nside; ++k) TCI_CHECK_HIP(hipStreamWaitEvent(sidec->side[k], sidec->fork, 0));
    }
    const hipStream_t saved = ctx->stream;
    for (size_t bi = 0; bi < buckets.size(); ++bi) {
      Bucket& bk = buckets[bi];
      const hipStream_t sb = bi == 0 ? s1 : sidec->side[(bi - 1) % nside];
      ctx->stream = sb;   // the eigenvalue stage launches on the context stream
      tci_status r = TCI_OK;
      const hipError_t he = pad_sectors(bk.pd, (int)bk.ids.size(), bk.theta, bk.S, sb);
      if (he == hipSuccess) r = tsvd_eigvals(ctx, TCI_F64, (int)bk.ids.size(), bk.S, bk.S, bk.theta, bk.S, bk.stage);
      ctx->stream = saved;
      TCI_CHECK_HIP(he);
      TCI_TRY(r);
    }
    for (int k = 0; k < nside; ++k) {
      TCI_CHECK_HIP(hipEventRecord(sidec->join[k], sidec->side[k]));
      TCI_CHECK_HIP(hipStreamWaitEvent(s1, sidec->join[k], 0));
    }
    return TCI_OK;
  };
  // key: structure, launch shapes and the workspace addresses
  std::vector<long long> key = ctx->arena.layout();
  key.push_back(n);
  key.push_back((long long)(uintptr_t)sbuf);
  key.push_back((long long)sec_elems);
  for (int ph = 0; ph < 2; ++ph) {
    key.push_back(plan[ph].np);
    key.push_back(plan[ph].ntiles);
    key.push_back(plan[ph].shape);
    key.push_back((long long)(uintptr_t)plan[ph].P_dev);
  }
  for (auto& bk : buckets) {
    key.push_back(bk.S);
    key.push_back((long long)bk.ids.size());
    key.push_back((long long)(uintptr_t)bk.theta);
    key.push_back((long long)(uintptr_t)bk.pd);
  }
  const bool use_graphs = !prof_on() && !std::getenv("TCI_NO_GRAPHS");
  BsGraphCache* gc = use_graphs ? bs_cache(ctx) : nullptr;
  BsGraphEntry* ent = nullptr;
  if (gc) {
    if (gc->m.size() >= BS_GRAPH_MAX_ENTRIES && !gc->m.count(key)) {
      for (auto& kv : gc->m)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      gc->m.clear();
    }
    ent = &gc->m[key];
  }
  if (ent && ent->exec) {
    // replay: the recorded allocations and stage descriptors are restored
    ctx->arena.restore(ent->arena_after);
    for (size_t bi = 0; bi < buckets.size(); ++bi) buckets[bi].stage = ent->stages[bi];
    TCI_CHECK_HIP(hipGraphLaunch(ent->exec, st));
  } else if (ent && ent->seen >= 1 && !ent->failed) {
    // record on a private stream, then launch on the context stream
    TCI_CHECK_HIP(hipStreamSynchronize(st));
    if (!gc->cs) TCI_CHECK_HIP(hipStreamCreateWithFlags(&gc->cs, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    ctx->stream = gc->cs;
    hipGraph_t graph = nullptr;
    tci_status rec = TCI_OK;
    hipError_t he = hipStreamBeginCapture(gc->cs, hipStreamCaptureModeRelaxed);
    if (he == hipSuccess) {
      rec = phase1(gc->cs);
      he = hipStreamEndCapture(gc->cs, &graph);
    }
    ctx->stream = saved;
    hipGraphExec_t exec = nullptr;
    if (rec == TCI_OK && he == hipSuccess && graph) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (rec != TCI_OK) return rec;
    if (he != hipSuccess || !exec) {
      (void)hipGetLastError();
      ent->failed = true;   // record once only; run the kernels directly
      TCI_TRY(phase1(st));
    } else {
      ent->exec = exec;
      ent->arena_after = ctx->arena.used_state();
      ent->stages.clear();
      for (auto& bk : buckets) ent->stages.push_back(bk.stage);
      TCI_CHECK_HIP(hipGraphLaunch(exec, st));
    }
  } else {
    TCI_TRY(phase1(st));
    if (ent) ent->seen++;
  }
  for (auto& bk : buckets) {
    const int nb = (int)bk.ids.size();
    bk.lam.resize((size_t)nb * bk.S);
    bk.total.resize(nb);
    TCI_CHECK_HIP(hipMemcpyAsync(bk.lam.data(), bk.stage.lam, sizeof(double) * bk.lam.size(), hipMemcpyDeviceToHost, st));
    TCI_CHECK_HIP(hipMemcpyAsync(bk.total.data(), bk.stage.total, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  }
  TCI_CHECK_HIP(hipStreamSynchronize(st));
  std::map<int, int> bucket_of_S;
  for (size_t i = 0; i < buckets.size(); ++i) bucket_of_S[buckets[i].S] = (int)i;

  // 4. merged truncation per update
  TruncParams tp{(int)std::min<int64_t>(p.chi_min, INT32_MAX), (int)std::min<int64_t>(p.chi_max, INT32_MAX),
                 p.target_trunc_err, p.s_min};
  std::vector<int> chi_u(n, 0);
  std::vector<double> eps_u(n, 0.0), W_u(n, 0.0), nrm_u(n, 0.0);
  for (int u = 0; u < n; ++u) {
    TruncParams tpu = tp;
    if (chi_max_each) tpu.chi_max = (int)std::min<int64_t>(chi_max_each[u], INT32_MAX);
    struct Ent {
      double s;
      int q, j, sec;
    };
    std::vector<Ent> ents;
    double W = 0.0;
    for (int id : secs_of[u]) {
      const Sector& sc = secs[id];
      const Bucket& bk = buckets[bucket_of_S[sc.bucket]];
      W += bk.total[sc.slot];
      const int rank = std::min(sc.r, sc.c);
      for (int j = 0; j < rank; ++j)
        ents.push_back({std::sqrt(std::max(bk.lam[(size_t)sc.slot * bk.S + j], 0.0)), sc.q, j, id});
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) {
      if (x.s != y.s) return x.s > y.s;
      if (x.q != y.q) return x.q < y.q;
      return x.j < y.j;
    });
    std::vector<double> sv(ents.size());
    for (size_t i = 0; i < ents.size(); ++i) sv[i] = ents[i].s;
    int chi = 0;
    double eps = 0.0;
    trunc_rule_host(sv, W, tpu, chi, eps);
    double kept = 0.0;
    for (int i = 0; i < chi; ++i) {
      secs[ents[i].sec].kept++;
      kept += sv[i] * sv[i];
    }
    chi_u[u] = chi;
    eps_u[u] = eps;
    W_u[u] = W;
    nrm_u[u] = std::sqrt(kept);
  }

  // vector stage per bucket with the kept counts
  std::vector<TsvdOut> outs(buckets.size());
  std::vector<int> kz_of(buckets.size(), 1);
  std::vector<double*> snorm_of(buckets.size(), nullptr);
  for (size_t bi = 0; bi < buckets.size(); ++bi) {
    Bucket& bk = buckets[bi];
    const int nb = (int)bk.ids.size(), S = bk.S;
    std::vector<int> chi_h(nb);
    std::vector<double> sinv_h((size_t)nb * S, 0.0), snorm_h((size_t)nb * S, 0.0);
    int kz = 1;
    for (int i = 0; i < nb; ++i) {
      const Sector& sc = secs[bk.ids[i]];
      chi_h[i] = sc.kept;
      kz = std::max(kz, sc.kept);
      for (int j = 0; j < sc.kept; ++j) {
        const double s = std::sqrt(std::max(bk.lam[(size_t)i * S + j], 0.0));
        sinv_h[(size_t)i * S + j] = s > 0.0 ? 1.0 / s : 0.0;
        snorm_h[(size_t)i * S + j] = nrm_u[sc.u] > 0.0 ? s / nrm_u[sc.u] : 0.0;
      }
    }
    int* chi_d = static_cast<int*>(ctx->arena.get(sizeof(int) * nb));
    double* sinv_d = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)nb * S));
    double* snorm_d = static_cast<double*>(ctx->arena.get(sizeof(double) * (size_t)nb * S));
    if (!chi_d || !sinv_d || !snorm_d) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "kept-value tables");
    TCI_CHECK_HIP(hipMemcpyAsync(chi_d, chi_h.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    TCI_CHECK_HIP(hipMemcpyAsync(sinv_d, sinv_h.data(), sizeof(double) * sinv_h.size(), hipMemcpyHostToDevice, st));
    TCI_CHECK_HIP(hipMemcpyAsync(snorm_d, snorm_h.data(), sizeof(double) * snorm_h.size(), hipMemcpyHostToDevice, st));
    TCI_CHECK_HIP(hipStreamSynchronize(st));
    outs[bi].kmax = S;
    TCI_TRY(tsvd_vectors(ctx, bk.stage, chi_d, kz, sinv_d, outs[bi]));
    kz_of[bi] = kz;
    snorm_of[bi] = snorm_d;
  }

  // 5. outputs
  std::vector<ScatDesc> sd;
  std::vector<std::vector<double>> s_host(n);
  for (int u = 0; u < n; ++u) {
    std::vector<int32_t> qn;
    std::vector<int64_t> dn;
    for (int id : secs_of[u])
      if (secs[id].kept > 0) {
        qn.push_back(secs[id].q);
        dn.push_back(secs[id].kept);
      }
    TCI_TRY(bs_define(ctx, A_out[u], TCI_F32, A[u]->ql, A[u]->dl, qn, dn));
    TCI_TRY(bs_define(ctx, B_out[u], TCI_F32, qn, dn, B[u]->qr, B[u]->dr));
    for (int id : secs_of[u]) {
      const Sector& sc = secs[id];
      if (sc.kept == 0) continue;
      const int bi = bucket_of_S[sc.bucket];
      const Bucket& bk = buckets[bi];
      const int S = bk.S, kz = kz_of[bi];
      const int iq = find_charge(qn, sc.q);
      const double* U = static_cast<const double*>(outs[bi].U) + (size_t)sc.slot * S * kz;
      const double* Vh = static_cast<const double*>(outs[bi].Vh) + (size_t)sc.slot * kz * S;
      const double* sn = snorm_of[bi] + (size_t)sc.slot * S;
      for (int j = 0; j < sc.kept; ++j) s_host[u].push_back(std::sqrt(std::max(bk.lam[(size_t)sc.slot * S + j], 0.0)) /
                                                            (nrm_u[u] > 0.0 ? nrm_u[u] : 1.0));
      for (size_t ri = 0; ri < sc.rows.size(); ++ri) {
        const auto* blk = find_block(A_out[u], sc.rows[ri].first, sc.rows[ri].second, iq);
        if (!blk) TCI_RET(TCI_ERR_UNSUPPORTED, "internal: missing output block");
        ScatDesc d{};
        d.src = U + (size_t)sc.roff[ri] * kz;
        d.lds = kz;
        d.rows = (int)A[u]->dl[sc.rows[ri].first];
        d.cols = sc.kept;
        d.dst = static_cast<float*>(A_out[u]->data) + blk->off;
        d.ldd = sc.kept;
        d.scale = sn;
        d.mode = p.direction == TCI_DIR_RIGHT ? 1 : 0;
        sd.push_back(d);
      }
      for (size_t ci = 0; ci < sc.cols.size(); ++ci) {
        const auto* blk = find_block(B_out[u], iq, sc.cols[ci].first, sc.cols[ci].second);
        if (!blk) TCI_RET(TCI_ERR_UNSUPPORTED, "internal: missing output block");
        ScatDesc d{};
        d.src = Vh + sc.coff[ci];
        d.lds = S;
        d.rows = sc.kept;
        d.cols = (int)B[u]->dr[sc.cols[ci].second];
        d.dst = static_cast<float*>(B_out[u]->data) + blk->off;
        d.ldd = d.cols;
        d.scale = sn;
        d.mode = p.direction == TCI_DIR_LEFT ? 2 : 0;
        sd.push_back(d);
      }
    }
  }
  if (!sd.empty()) {
    ScatDesc* sd_d = static_cast<ScatDesc*>(ctx->arena.get(sizeof(ScatDesc) * sd.size()));
    if (!sd_d) TCI_RET(TCI_ERR_OUT_OF_MEMORY, "scatter table");
    TCI_CHECK_HIP(hipMemcpyAsync(sd_d, sd.data(), sizeof(ScatDesc) * sd.size(), hipMemcpyHostToDevice, st));
    TCI_CHECK_HIP(scatter_blocks(sd_d, (int)sd.size(), st));
  }
  for (int u = 0; u < n; ++u) {
    const int64_t sh[1] = {(int64_t)s_host[u].size()};
    TCI_TRY(ensure_shape(ctx, s_out[u], TCI_F64, 1, sh));
    if (sh[0]) TCI_CHECK_HIP(hipMemcpyAsync(s_out[u]->data, s_host[u].data(), sizeof(double) * sh[0],
                                            hipMemcpyHostToDevice, st));
    if (infos) {
      infos[u].chi = chi_u[u];
      infos[u].trunc_err = eps_u[u];
      infos[u].discarded_abs = eps_u[u] * W_u[u];
      infos[u].norm2 = W_u[u];
      infos[u].used_fallback = 0;
      infos[u].sketch_rank = 0;
      infos[u].max_residual = 0.0;
    }
  }
  TCI_CHECK_HIP(hipStreamSynchronize(st));
  return TCI_OK;
} TCI_API_CATCH

}  // extern "C"
