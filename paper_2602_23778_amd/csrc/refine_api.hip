// Host runtime and C ABI of the refinement library (declared in refine.h).
//
// A context holds a "plan": the device table of problem descriptors, the
// work-item tables of every pass, and one contiguous workspace.  The step is
// enqueued as a fixed sequence of launches (product, Rayleigh quotients, Gram,
// Gram reduction, k-by-k solve, update, normalisation) and recorded once as a
// HIP graph; refine_step replays the graph, refine_run replays it in chunks
// and polls the device-side control word between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "refine.h"
#include "refine_debug.h"
#include "split.h"
#include "tune_cache.h"

namespace rfk {
hipError_t launch_gemm_f64(const Prob*, const GemmItem*, int, int, bool, int, hipStream_t);
int gemm_rows_per_block(int cfg);
int gemm_num_cfgs();
hipError_t launch_gram(const Prob*, const RowItem*, int, int, bool, hipStream_t);
struct GramRedItem {
  int32_t prob, s0;
};
hipError_t launch_gram_reduce(const Prob*, const GramRedItem*, int, hipStream_t);
hipError_t launch_kxk(const Prob*, int, int, bool, bool, hipStream_t);
hipError_t launch_update(const Prob*, const RowItem*, int, int, bool, hipStream_t);
hipError_t launch_fin_pre(const Prob*, int, hipStream_t);
hipError_t launch_fin_post(const Prob*, hipStream_t);
hipError_t launch_normalize(const Prob*, const RowItem*, int, hipStream_t);
hipError_t launch_wsum(const Prob*, int, int64_t, int, hipStream_t);
hipError_t launch_fin_d(const Prob*, int, hipStream_t);
hipError_t launch_fin_stats(const Prob*, int, hipStream_t);
hipError_t launch_ctrl_reset(const Prob*, int, int, double, hipStream_t);
hipError_t launch_set_x(Prob*, int, double*, int64_t, hipStream_t);
hipError_t launch_spmm(const Prob*, const RowItem*, int, int, int, int, hipStream_t);
int spmm_row_lanes(int k, int64_t n, int64_t nnz);
int gram_groups(int kmax);
hipError_t launch_rr_prep(const Prob*, int, hipStream_t);
hipError_t launch_rr_solve(const Prob*, int, hipStream_t);
hipError_t launch_rr_apply(const Prob*, const RowItem*, int, hipStream_t);
hipError_t launch_flip_sigma(const Prob*, int, hipStream_t);
hipError_t launch_flip_apply(const Prob*, const RowItem*, int, hipStream_t);
int spmm_chunk_rows(int lanes);
int spmm_grid(int nitems, int k, int lanes);
hipError_t launch_rowstats(int, int, const double*, int64_t, const int32_t*, const int32_t*,
                           const double*, double*, int, hipStream_t);
}  // namespace rfk

using namespace rfk;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
int iceil(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// One set of problems sharing launches.
struct Plan {
  std::vector<Prob> hprob;
  Prob* dprob = nullptr;
  GemmItem* gemm_items = nullptr;
  int n_gemm = 0;
  RowItem* row_items = nullptr;
  int n_row = 0;
  RowItem* gram_items = nullptr;
  int n_gram = 0;
  RowItem* spmm_items = nullptr;  // CSR product: chunks of spmm_chunk_rows(lanes) rows
  int n_spmm = 0;
  int spmm_lanes = 0;             // lanes per row of the row form (0: vector form)
  int spmm_grid = 0;              // blocks of the CSR product (one Rayleigh partial each)
  bool kxk_pipeline = false;      // one problem: k x k stage by the panel pipeline
  bool fused = false;             // k <= 32: statistics before the update, X written in place
  bool fused_pipe = false;        // one problem past k = 32 through the panel pipeline: the same
  GramRedItem* gred_items = nullptr;
  int n_gred = 0;
  int kmax = 0;
  int gemm_cfg = 1;
  int gemm_ks = 1;
  float gemm_ms = 0.f;
  bool vec2 = true;
  bool csr = false;
  bool split = false;
  bool square = false;            // B = A^2 - mu I: two products per step
  Prob* dprob1 = nullptr;         // descriptors of the first product (X -> W1)
  Prob* dprob2 = nullptr;         // and of the second (W1 -> W)
  SplitPlan sp;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Ctrl* ctrl = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_multi = nullptr;      // `multi` steps in one graph
  hipGraphExec_t exec_multi = nullptr;
  int multi = 0;
  hipStream_t cap_stream = nullptr;
};

struct Options {
  refine_options o;
};

// Per-problem sizes chosen by the planner.
struct Shape {
  int ksplit, kchunk, nrb, rbrows, ngb, gbrows;
};

Shape choose_shape(int64_t n, int k, bool single, bool csr) {
  Shape s{};
  s.ksplit = 1;
  s.kchunk = (int)n;
  // Row blocks of the streaming passes (split-K sum, update, normalisation):
  // at least 64 rows for one problem and about 1024 blocks for a long one
  // (four per CU to overlap their latencies; twice as many, smaller blocks
  // each pay the fixed latency of staging [M | N] and of the partial writes,
  // which measured slower at n = 150k and 2M).  From n = 2^20 on with
  // k <= 32, about 4096 blocks of 256 rows or more: the fused update writes
  // no partials and runs three blocks per CU (at n = 2M, k = 32: 1.001 ms
  // per step against 1.049 with 1024 blocks, which leave the third round of
  // blocks a third full; at n = 150k, 64-row blocks measured slower).  256
  // rows per block in a batch.
  if (single) {
    const int64_t target = (k <= 32 && n >= (int64_t)1 << 20) ? 4096 : 1024;
    s.rbrows = (int)std::max<int64_t>(64, (n + target - 1) / target + 63) / 64 * 64;
  } else {
    s.rbrows = 256;
  }
  // Gram blocks: at least k rows (the leading k rows must sit in block 0);
  // for one long problem about 512 blocks when k <= 32, and past k = 32,
  // where each block is one work item per 16-column tile, about 256 / tiles
  // blocks (one item per CU, and k-by-k partials of few blocks to reduce);
  // 512 rows in a batch (1.3 % faster steps than 256 or 1024 on 512 problems
  // of n <= 2048).
  {
    const int64_t kr = (k + 3) / 4 * 4;
    const int64_t nblk = k <= 32 ? 512 : std::max<int64_t>(1, 256 / ((k + 15) / 16));
    const int64_t per = single ? std::max<int64_t>(64, ((n + nblk - 1) / nblk + 3) / 4 * 4) : 512;
    s.gbrows = (int)std::max<int64_t>(std::max<int64_t>(kr, per), 16);
  }
  // tuning hooks: REFINE_RBROWS, REFINE_GBROWS (rows per streaming / Gram
  // block; a Gram block keeps at least k rows)
  if (const char* env = getenv("REFINE_RBROWS")) {
    const int v = atoi(env);
    if (v >= 16 && v % 16 == 0) s.rbrows = v;
  }
  if (const char* env = getenv("REFINE_GBROWS")) {
    const int v = atoi(env);
    if (v >= 16 && v % 4 == 0) s.gbrows = std::max(v, (k + 3) / 4 * 4);
  }
  s.nrb = iceil(n, s.rbrows);
  s.ngb = iceil(n, s.gbrows);
  return s;
}

constexpr int KSPLIT_MAX = 16;
// refine_run checks the control word once per RUN_CHUNK steps (one graph);
// batches replay BATCH_GRAPH_STEPS steps per graph.
constexpr int RUN_CHUNK = 8;
constexpr int BATCH_GRAPH_STEPS = 5;

// Upper bound of the Rayleigh partials: per row block of the smallest
// product tile (64 rows) and K split, or per streaming row block.
int64_t dpart_entries(int64_t n, const Shape& s, bool split) {
  const int ks = split ? SPLIT_KS_MAX : std::max(1, s.ksplit);
  return std::max<int64_t>((int64_t)iceil(n, 64) * ks, s.nrb);
}

// Largest k whose single-problem k x k stage runs in one workgroup rather
// than the panel pipeline (a tuning constant; REFINE_KXK_PIPE=0/1 forces
// either form).
constexpr int KXK_ONE_WG_MAX = 48;

// Rayleigh partial slots of one problem: the dense and split products' row
// blocks and K splits, or the CSR product's grid.
int64_t dpart_count(int64_t n, const Shape& s, const Plan& pl) {
  const int64_t d = dpart_entries(n, s, pl.split);
  return pl.csr ? std::max<int64_t>(d, pl.spmm_grid) : d;
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& v) {
  if (v.empty()) {
    *dst = nullptr;
    return hipSuccess;
  }
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

void free_plan(Plan& p) {
  if (p.exec) (void)hipGraphExecDestroy(p.exec);
  if (p.exec_multi) (void)hipGraphExecDestroy(p.exec_multi);
  if (p.graph_multi) (void)hipGraphDestroy(p.graph_multi);
  if (p.graph) (void)hipGraphDestroy(p.graph);
  if (p.cap_stream) (void)hipStreamDestroy(p.cap_stream);
  (void)hipFree(p.dprob);
  (void)hipFree(p.dprob1);
  (void)hipFree(p.dprob2);
  (void)hipFree(p.gemm_items);
  (void)hipFree(p.row_items);
  (void)hipFree(p.gram_items);
  (void)hipFree(p.spmm_items);
  (void)hipFree(p.gred_items);
  (void)hipFree(p.ws);
  split_free(p.sp);
  p = Plan();
}

#define RF_CHECK(expr)                         \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return REFINE_EHIP;  \
  } while (0)

// Work items of the dense product for launch configuration `cfg` with K
// split `ks` (single problem; batches use ks = 1).  Item it = rb * ks + sp, so
// blockIdx % 8 (the XCD running the block) fixes the K range when ks divides
// or is a multiple of 8.
std::vector<GemmItem> gemm_items(const std::vector<refine_matrix>& As, int cfg, int ks,
                                 std::vector<int>* kchunks) {
  std::vector<GemmItem> gi;
  const int bm = gemm_rows_per_block(cfg);
  kchunks->assign(As.size(), 0);
  for (size_t p = 0; p < As.size(); ++p) {
    const int64_t n = As[p].n;
    const int kchunk = (int)((iceil(n, ks) + 31) / 32 * 32);
    const int nks = iceil(n, kchunk);
    (*kchunks)[p] = nks;
    const int nrbg = iceil(n, bm);
    for (int rb = 0; rb < nrbg; ++rb)
      for (int sp = 0; sp < nks; ++sp) {
        GemmItem g{};
        g.prob = (int)p;
        g.row0 = rb * bm;
        g.k0 = sp * kchunk;
        g.k1 = (int)std::min<int64_t>(n, (int64_t)(sp + 1) * kchunk);
        g.split = sp;
        gi.push_back(g);
      }
  }
  if (As.size() > 1)  // larger problems first
    std::stable_sort(gi.begin(), gi.end(),
                     [&](const GemmItem& x, const GemmItem& y) { return As[x.prob].n > As[y.prob].n; });
  return gi;
}

// Squared variant: the descriptors of the two products, derived from the
// problem's own (first: X -> W1 with its Rayleigh partials in dpx; second:
// W1 -> W).  Rewritten whenever the problem descriptors are.
int upload_square_descs(Plan& pl) {
  if (!pl.square) return REFINE_OK;
  std::vector<Prob> d1(pl.hprob), d2(pl.hprob);
  for (size_t p = 0; p < pl.hprob.size(); ++p) {
    d1[p].square = 0;
    d1[p].w = pl.hprob[p].w1;
    d1[p].dpart = pl.hprob[p].dpx;
    d2[p].square = 0;
    d2[p].x = pl.hprob[p].w1;
    d2[p].ldx = pl.hprob[p].k;
  }
  const size_t bytes = sizeof(Prob) * pl.hprob.size();
  if (!pl.dprob1) RF_CHECK(hipMalloc((void**)&pl.dprob1, bytes));
  if (!pl.dprob2) RF_CHECK(hipMalloc((void**)&pl.dprob2, bytes));
  RF_CHECK(hipMemcpy(pl.dprob1, d1.data(), bytes, hipMemcpyHostToDevice));
  RF_CHECK(hipMemcpy(pl.dprob2, d2.data(), bytes, hipMemcpyHostToDevice));
  return REFINE_OK;
}

int install_gemm(Plan& pl, const std::vector<refine_matrix>& As, int cfg, int ks) {
  std::vector<int> nks;
  std::vector<GemmItem> gi = gemm_items(As, cfg, ks, &nks);
  (void)hipFree(pl.gemm_items);
  pl.gemm_items = nullptr;
  RF_CHECK(upload(&pl.gemm_items, gi));
  pl.n_gemm = (int)gi.size();
  pl.gemm_cfg = cfg;
  pl.gemm_ks = ks;
  for (size_t p = 0; p < As.size(); ++p) {
    pl.hprob[p].ksplit = nks[p];
    pl.hprob[p].ndp = iceil(As[p].n, gemm_rows_per_block(cfg)) * nks[p];
  }
  RF_CHECK(hipMemcpy(pl.dprob, pl.hprob.data(), sizeof(Prob) * pl.hprob.size(), hipMemcpyHostToDevice));
  return upload_square_descs(pl);
}


// Picks the product's launch configuration: REFINE_GEMM="cfg,ks" forces one;
// otherwise every configuration is timed (with each K split for a single
// problem, K split 1 for a batch) on the plan's own shapes, a few
// milliseconds once per shape and process, and the fastest is kept (and
// stored in the tuning cache when one is set).
int choose_gemm(Plan& pl, const std::vector<refine_matrix>& As, bool single,
                const std::vector<Shape>& shapes) {
  if (const char* env = getenv("REFINE_GEMM")) {
    int cfg = 0, ks = 1;
    if (sscanf(env, "%d,%d", &cfg, &ks) == 2 && cfg >= 0 && cfg < gemm_num_cfgs() && ks >= 1 &&
        ks <= shapes[0].ksplit)
      return install_gemm(pl, As, cfg, single ? ks : 1);
  }
  // tuning-cache key: (n, k, vector width) of one problem; a batch by its
  // total size, count and largest k
  int64_t nsum = 0;
  for (const auto& a : As) nsum += a.n;
  const std::vector<int64_t> key{single ? As[0].n : -nsum - (int64_t)As.size(),
                                 single ? pl.hprob[0].k : pl.kmax, pl.vec2 ? 1 : 0};
  std::vector<int> hit;
  if (tune_cache_get("gemm_f64", key, &hit) && hit.size() == 2 && hit[0] >= 0 &&
      hit[0] < gemm_num_cfgs() && hit[1] >= 1 && hit[1] <= (single ? shapes[0].ksplit : 1))
    return install_gemm(pl, As, hit[0], hit[1]);
  // time the candidates on a zero X (the workspace copy of the update)
  Prob& P = pl.hprob[0];
  std::vector<std::pair<double*, int64_t>> saved;
  for (Prob& q : pl.hprob) {
    saved.push_back({q.x, q.ldx});
    q.x = q.xn;
    q.ldx = q.k;
  }
  hipStream_t st = nullptr;
  RF_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  RF_CHECK(hipEventCreate(&e0));
  RF_CHECK(hipEventCreate(&e1));
  float best = 1e30f;
  int best_cfg = 1, best_ks = 1;
  const int ks_max = single ? shapes[0].ksplit : 1;
  for (int cfg = 0; cfg < gemm_num_cfgs(); ++cfg) {
    for (int ks = 1; ks <= ks_max; ks *= 2) {
      // at least one block per CU unless this is the largest split
      if (single && (int64_t)iceil(As[0].n, gemm_rows_per_block(cfg)) * ks < 256 && 2 * ks <= ks_max)
        continue;
      if (install_gemm(pl, As, cfg, ks) != REFINE_OK) return REFINE_EHIP;
      float t = 0.f, t1 = 0.f;
      hipError_t e = hipEventRecord(e0, st);
      if (e == hipSuccess)
        e = launch_gemm_f64(pl.dprob, pl.gemm_items, pl.n_gemm, pl.kmax, pl.vec2, cfg, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t1, e0, e1);
      if (e != hipSuccess) return REFINE_EHIP;
      if (t1 > 3.f * best / 3.f) continue;  // clearly slower than the best so far
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int r = 0; r < 3 && e == hipSuccess; ++r)
        e = launch_gemm_f64(pl.dprob, pl.gemm_items, pl.n_gemm, pl.kmax, pl.vec2, cfg, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) return REFINE_EHIP;
      if (getenv("REFINE_LOG") && atoi(getenv("REFINE_LOG")) >= 2)
        fprintf(stderr, "refine: tune n=%lld k=%d cfg %d ks %d: %.1f us\n", (long long)As[0].n,
                P.k, cfg, ks, t * 1000.f / 3.f);
      if (t < best) {
        best = t;
        best_cfg = cfg;
        best_ks = ks;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  for (size_t q = 0; q < pl.hprob.size(); ++q) {
    pl.hprob[q].x = saved[q].first;
    pl.hprob[q].ldx = saved[q].second;
  }
  tune_cache_put("gemm_f64", key, {best_cfg, best_ks});
  pl.gemm_ms = best / 3.f;
  if (getenv("REFINE_LOG"))
    fprintf(stderr, "refine: product n=%lld k=%d: cfg %d, K split %d, %.1f us\n", (long long)As[0].n,
            P.k, best_cfg, best_ks, best * 1000.f / 3.f);
  return install_gemm(pl, As, best_cfg, best_ks);
}

// Builds descriptors, work items and the workspace for a set of problems.
// mus/deltas/norms are per problem.
int build_plan(Plan& pl, const std::vector<refine_matrix>& As, const std::vector<int>& ks,
               const refine_options& opt, const std::vector<double>& mus,
               const std::vector<double>& deltas, const std::vector<double>& norms) {
  const int np = (int)As.size();
  const bool single = np == 1;
  pl.csr = As[0].kind == REFINE_CSR;
  pl.split = opt.precision == REFINE_SPLIT_INT8 || opt.precision == REFINE_SPLIT_CRT;
  pl.square = opt.target == REFINE_TARGET_SMALLEST_ABS;
  pl.spmm_lanes = pl.csr ? spmm_row_lanes(ks[0], As[0].n, As[0].nnz) : 0;
  if (pl.csr) {
    pl.spmm_grid = spmm_grid(iceil(As[0].n, spmm_chunk_rows(pl.spmm_lanes)), ks[0], pl.spmm_lanes);
    if (pl.spmm_grid <= 0) return REFINE_EINVAL;
  }
  pl.kxk_pipeline = single && ks[0] > KXK_ONE_WG_MAX;
  if (const char* env = getenv("REFINE_KXK_PIPE")) pl.kxk_pipeline = single && atoi(env) != 0;
  pl.hprob.resize(np);
  std::vector<Shape> shapes(np);
  size_t bytes = 0;
  std::vector<size_t> off(np);
  pl.kmax = 0;
  pl.vec2 = true;
  for (int p = 0; p < np; ++p) {
    const int64_t n = As[p].n;
    const int k = ks[p];
    pl.kmax = std::max(pl.kmax, k);
    Shape s = choose_shape(n, k, single, pl.csr);
    // single dense FP64 problems may split K (chosen by the tuner below)
    if (single && !pl.csr && !pl.split) s.ksplit = std::min<int64_t>(KSPLIT_MAX, std::max<int64_t>(1, n / 256));
    shapes[p] = s;
    off[p] = bytes;
    const size_t nk = (size_t)n * k * sizeof(double);
    size_t b = 0;
    if (s.ksplit > 1) b += align_up(nk * s.ksplit);
    b += align_up(nk);                                   // w
    if (pl.split) b += align_up(nk);                     // wlo
    b += align_up(nk);                                   // xn
    b += align_up((size_t)s.nrb * 5 * k * sizeof(double));
    b += align_up((size_t)dpart_count(n, s, pl) * 2 * k * sizeof(double));
    b += align_up((size_t)s.ngb * (2 * k * k + k) * sizeof(double));
    b += align_up((size_t)KK_COUNT * k * k * sizeof(double));
    b += align_up((size_t)(16 + 16 * k) * sizeof(double));  // kpp
    b += align_up((size_t)VEC_COUNT * k * sizeof(double));
    if (pl.square) {
      b += align_up(nk);                                                          // w1
      b += align_up((size_t)dpart_count(n, s, pl) * 2 * k * sizeof(double));  // dpx
    }
    bytes += b;
    if (As[p].kind == REFINE_DENSE) {
      // pairs of columns per lane: any n and leading dimension (an odd one
      // leaves every other row's pairs 8-byte aligned, which the loads
      // accept), A itself at least 8-byte aligned
      if ((uintptr_t)As[p].a & 7) pl.vec2 = false;
    }
  }
  const size_t ctrl_off = bytes;
  bytes += align_up(sizeof(Ctrl) * np);
  if (hipMalloc((void**)&pl.ws, bytes) != hipSuccess) return REFINE_ENOMEM;
  pl.ws_bytes = bytes;
  RF_CHECK(hipMemset(pl.ws, 0, bytes));
  pl.ctrl = (Ctrl*)(pl.ws + ctrl_off);

  std::vector<RowItem> ri, gri;
  pl.fused = pl.kmax <= 32;
  // one problem past k = 32 through the panel pipeline: the statistics before
  // the update as well (REFINE_FUSED_PIPE=0: update, statistics, normalisation)
  pl.fused_pipe = pl.kxk_pipeline && pl.kmax > 32;
  if (const char* env = getenv("REFINE_FUSED_PIPE")) pl.fused_pipe = pl.fused_pipe && atoi(env) != 0;
  std::vector<GramRedItem> rr;
  for (int p = 0; p < np; ++p) {
    const refine_matrix& A = As[p];
    const Shape& s = shapes[p];
    const int64_t n = A.n;
    const int k = ks[p];
    const size_t nk = (size_t)n * k * sizeof(double);
    Prob& P = pl.hprob[p];
    memset(&P, 0, sizeof(P));
    P.a = A.a;
    P.lda = A.lda;
    P.rp = A.row_ptr;
    P.ci = A.col_idx;
    P.av = A.val;
    P.x = nullptr;
    P.ldx = k;
    P.n = (int32_t)n;
    P.k = k;
    P.kind = A.kind;
    P.ksplit = s.ksplit;
    P.nrb = s.nrb;
    P.rbrows = s.rbrows;
    P.ngb = s.ngb;
    P.gbrows = s.gbrows;
    char* base = pl.ws + off[p];
    if (s.ksplit > 1) {
      P.wp = (double*)base;
      base += align_up(nk * s.ksplit);
    }
    P.w = (double*)base;
    base += align_up(nk);
    if (pl.split) {
      P.wlo = (double*)base;
      base += align_up(nk);
    }
    P.xn = (double*)base;
    base += align_up(nk);
    P.part = (double*)base;
    base += align_up((size_t)s.nrb * 5 * k * sizeof(double));
    P.dpart = (double*)base;
    // CSR: one partial per product block; dense: set with the product's items
    P.ndp = pl.csr ? pl.spmm_grid : s.nrb;
    base += align_up((size_t)dpart_count(n, s, pl) * 2 * k * sizeof(double));
    P.gpart = (double*)base;
    base += align_up((size_t)s.ngb * (2 * k * k + k) * sizeof(double));
    P.kk = (double*)base;
    base += align_up((size_t)KK_COUNT * k * k * sizeof(double));
    P.kpp = (double*)base;
    base += align_up((size_t)(16 + 16 * k) * sizeof(double));
    P.vec = (double*)base;
    base += align_up((size_t)VEC_COUNT * k * sizeof(double));
    if (pl.square) {
      P.square = 1;
      P.w1 = (double*)base;
      base += align_up((size_t)n * k * sizeof(double));
      P.dpx = (double*)base;
    }
    P.ctrl = pl.ctrl + p;
    P.mu = mus[p];
    P.delta = deltas[p];
    P.norm_a = norms[p];
    P.beta_zero = opt.beta == REFINE_BETA_ZERO;
    P.normalize = opt.normalize != 0;

    for (int b = 0; b < s.nrb; ++b) ri.push_back(RowItem{p, b});
    // Gram items: (row block, column tile) as blk = block * tiles + tile
    // past k = 32 (the kernel is chosen by the batch's largest k)
    const int gg = pl.kmax <= 32 ? 1 : (k + 15) / 16;
    if (single && gg > 1) {
      // the tiles of one row block on one XCD (workgroups go to the eight
      // XCDs in turn), so that its L2 holds the block's X rows for all of them
      std::vector<std::vector<int>> q(8);
      for (int rb = 0; rb < s.ngb; ++rb)
        for (int t = 0; t < gg; ++t) q[rb % 8].push_back(rb * gg + t);
      std::vector<size_t> pos(8, 0);
      for (int b = 0; b < s.ngb * gg; ++b) {
        int x = b % 8;
        while (pos[x] == q[x].size()) x = (x + 1) % 8;
        gri.push_back(RowItem{p, q[x][pos[x]++]});
      }
    } else {
      for (int b = 0; b < s.ngb * gg; ++b) gri.push_back(RowItem{p, b});
    }
    const int S = 2 * k * k + k;
    for (int s0 = 0; s0 < S; s0 += 64) rr.push_back(GramRedItem{p, s0});
  }
  if (!single) {
    // larger problems first: a rough longest-processing-time order
    auto bigger = [&](int a, int b) { return As[a].n > As[b].n; };
    auto sort_items = [&](auto& v) {
      std::stable_sort(v.begin(), v.end(), [&](const auto& x, const auto& y) { return bigger(x.prob, y.prob); });
    };
    sort_items(ri);
    sort_items(gri);
  }
  RF_CHECK(upload(&pl.dprob, pl.hprob));
  if (upload_square_descs(pl) != REFINE_OK) return REFINE_EHIP;
  RF_CHECK(upload(&pl.row_items, ri));
  RF_CHECK(upload(&pl.gram_items, gri));
  RF_CHECK(upload(&pl.gred_items, rr));
  if (pl.csr) {
    std::vector<RowItem> si;
    for (int b = 0; b < iceil(As[0].n, spmm_chunk_rows(pl.spmm_lanes)); ++b) si.push_back(RowItem{0, b});
    RF_CHECK(upload(&pl.spmm_items, si));
    pl.n_spmm = (int)si.size();
  }
  pl.n_row = (int)ri.size();
  pl.n_gram = (int)gri.size();
  pl.n_gred = (int)rr.size();
  if (!pl.csr && !pl.split) {
    int rc = choose_gemm(pl, As, single, shapes);
    if (rc != REFINE_OK) return rc;
  }
  return REFINE_OK;
}

// One product W = A X over the descriptors `probs` (and the K-split sum).
hipError_t enqueue_product_on(Plan& pl, const Prob* probs, hipStream_t st) {
  hipError_t e;
  const int np = (int)pl.hprob.size();
  if (pl.csr) {
    if ((e = launch_spmm(probs, pl.spmm_items, pl.n_spmm, pl.hprob[0].k, pl.spmm_lanes, pl.spmm_grid,
                         st)) != hipSuccess)
      return e;
  } else {
    if (pl.split) {
      if ((e = split_product(pl.sp, probs, st)) != hipSuccess) return e;
    } else {
      if ((e = launch_gemm_f64(probs, pl.gemm_items, pl.n_gemm, pl.kmax, pl.vec2, pl.gemm_cfg, st)) !=
          hipSuccess)
        return e;
    }
    for (int p = 0; p < np; ++p)
      if (!pl.split && pl.hprob[p].ksplit > 1 &&
          (e = launch_wsum(probs, p, pl.hprob[p].n, pl.hprob[p].k, st)) != hipSuccess)
        return e;
  }
  return hipSuccess;
}

// The product step of Algorithm 4 for every problem: W = A X, or for the squared
// variant (Sec. 5.2) W = A (A X) through W1 = A X, with no A^2 formed.
hipError_t enqueue_product(Plan& pl, hipStream_t st) {
  if (!pl.square) return enqueue_product_on(pl, pl.dprob, st);
  hipError_t e = enqueue_product_on(pl, pl.dprob1, st);
  if (e == hipSuccess) e = enqueue_product_on(pl, pl.dprob2, st);
  return e;
}

hipError_t enqueue_step(Plan& pl, hipStream_t st) {
  hipError_t e;
  const int np = (int)pl.hprob.size();
  if ((e = enqueue_product(pl, st)) != hipSuccess) return e;
  if ((e = launch_fin_d(pl.dprob, np, st)) != hipSuccess) return e;
  if ((e = launch_gram(pl.dprob, pl.gram_items, pl.n_gram, pl.kmax, pl.split, st)) != hipSuccess) return e;
  if ((e = launch_gram_reduce(pl.dprob, pl.gred_items, pl.n_gred, st)) != hipSuccess) return e;
  if ((e = launch_kxk(pl.dprob, np, pl.kmax, pl.kxk_pipeline, pl.fused_pipe, st)) != hipSuccess)
    return e;
  if (pl.fused_pipe) {
    // one problem through the panel pipeline: the statistics from k x k
    // quantities after it, then the update writes the normalised iterate in
    // place
    if ((e = launch_fin_post(pl.dprob, st)) != hipSuccess) return e;
    if ((e = launch_update(pl.dprob, pl.row_items, pl.n_row, pl.kmax, true, st)) != hipSuccess) return e;
    return hipSuccess;
  }
  if (pl.fused) {
    // k <= 32: statistics and scale factors from k x k quantities, then the
    // update writes the normalised iterate in place
    if ((e = launch_fin_pre(pl.dprob, np, st)) != hipSuccess) return e;
    if ((e = launch_update(pl.dprob, pl.row_items, pl.n_row, pl.kmax, true, st)) != hipSuccess) return e;
    return hipSuccess;
  }
  if ((e = launch_update(pl.dprob, pl.row_items, pl.n_row, pl.kmax, false, st)) != hipSuccess) return e;
  if ((e = launch_fin_stats(pl.dprob, np, st)) != hipSuccess) return e;
  if ((e = launch_normalize(pl.dprob, pl.row_items, pl.n_row, st)) != hipSuccess) return e;
  return hipSuccess;
}

// Records one step as a graph and, for the repeated-step loops, `multi`
// consecutive steps as a second graph (the kernels of later steps skip their
// work once the control word says stopped).
int capture_graph(Plan& pl, int multi) {
  RF_CHECK(hipStreamCreateWithFlags(&pl.cap_stream, hipStreamNonBlocking));
  for (int which = 0; which < 2; ++which) {
    const int steps = which == 0 ? 1 : multi;
    if (steps < 2 && which == 1) break;
    RF_CHECK(hipStreamBeginCapture(pl.cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < steps && e == hipSuccess; ++i) e = enqueue_step(pl, pl.cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(pl.cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return REFINE_EHIP;
    }
    if (which == 0) {
      pl.graph = g;
      RF_CHECK(hipGraphInstantiate(&pl.exec, g, nullptr, nullptr, 0));
    } else {
      pl.graph_multi = g;
      pl.multi = steps;
      RF_CHECK(hipGraphInstantiate(&pl.exec_multi, g, nullptr, nullptr, 0));
    }
  }
  return REFINE_OK;
}

// Enqueues `count` steps: whole multi-step graphs first, then single steps.
hipError_t launch_steps(Plan& pl, int count, hipStream_t st) {
  while (pl.exec_multi && count >= pl.multi) {
    hipError_t e = hipGraphLaunch(pl.exec_multi, st);
    if (e != hipSuccess) return e;
    count -= pl.multi;
  }
  for (int i = 0; i < count; ++i) {
    hipError_t e = hipGraphLaunch(pl.exec, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int status_from_ctrl(const Ctrl& c) { return c.status; }

}  // namespace

struct refine_ctx {
  hipStream_t stream = nullptr;
  refine_matrix A{};
  refine_options opt{};
  int k = 0;
  double mu = 0, norm_inf = 0, norm_used = 0, delta = 0, g_lo = 0, g_hi = 0;
  Plan plan;
  double* cur_x = nullptr;
  int64_t cur_ldx = -1;
  int stop_mode = 0;
  bool pending = false;     // steps enqueued without statistics since the last report
};

struct refine_batch {
  hipStream_t stream = nullptr;
  std::vector<refine_matrix> As;
  std::vector<int> ks;
  refine_options opt{};
  Plan plan;
  std::vector<double*> cur_x;
  std::vector<int64_t> cur_ldx;
  double* d_xs = nullptr;   // staging: (x, ldx) pairs
  bool pending = false;     // runs enqueued without statistics since the last report
};

namespace {

int validate_matrix(const refine_matrix* A, int32_t k, const refine_options& opt) {
  if (!A || A->n <= 0 || A->n >= (int64_t)1 << 31) return REFINE_EINVAL;
  if (k < 1 || k > KMAX || (int64_t)k >= A->n) return REFINE_EINVAL;
  if (A->kind == REFINE_DENSE) {
    if (!A->a || A->lda < A->n) return REFINE_EINVAL;
  } else if (A->kind == REFINE_CSR) {
    if (!A->row_ptr || !A->col_idx || !A->val || A->nnz < 0 || A->nnz >= (int64_t)1 << 31)
      return REFINE_EINVAL;
    if (opt.precision != REFINE_FP64) return REFINE_EINVAL;
  } else {
    return REFINE_EINVAL;
  }
  // REFINE_SPLIT_FP8 is declared but not offered (refine.h states why)
  if (opt.precision != REFINE_FP64 && opt.precision != REFINE_SPLIT_INT8 &&
      opt.precision != REFINE_SPLIT_CRT)
    return REFINE_EINVAL;
  if (opt.precision == REFINE_SPLIT_INT8 &&
      (A->n > SPLIT_NMAX || (opt.slices != 0 && (opt.slices < SPLIT_S_MIN || opt.slices > SPLIT_S_MAX))))
    return REFINE_EINVAL;
  if (opt.precision == REFINE_SPLIT_CRT &&
      (A->n > SPLIT_NMAX || (opt.slices != 0 && (opt.slices < CRT_N_MIN || opt.slices > CRT_N_MAX))))
    return REFINE_EINVAL;
  if (!(opt.delta_c >= 0.0)) return REFINE_EINVAL;
  if (opt.target < REFINE_TARGET_LARGEST_ABS || opt.target > REFINE_TARGET_SMALLEST_ABS)
    return REFINE_EINVAL;
  // the squared variant feeds W1 = A X into a second product: FP64 only
  if (opt.target == REFINE_TARGET_SMALLEST_ABS && opt.precision != REFINE_FP64) return REFINE_EINVAL;
  return REFINE_OK;
}

// ||A||_inf and Gershgorin bounds, synchronously on `st`.
int matrix_stats(const refine_matrix& A, hipStream_t st, double* ninf, double* lo, double* hi) {
  const int grid = std::min<int64_t>(1024, (A.n + 3) / 4);
  double* d = nullptr;
  RF_CHECK(hipMalloc((void**)&d, sizeof(double) * 3 * grid));
  hipError_t e = launch_rowstats(A.kind == REFINE_CSR ? 1 : 0, (int)A.n, A.a, A.lda, A.row_ptr,
                                 A.col_idx, A.val, d, grid, st);
  std::vector<double> h(3 * grid);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, sizeof(double) * 3 * grid, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d);
  if (e != hipSuccess) return REFINE_EHIP;
  double m = 0.0, gh = -INFINITY, gl = INFINITY;
  for (int b = 0; b < grid; ++b) {
    m = std::max(m, h[3 * b]);
    gh = std::max(gh, h[3 * b + 1]);
    gl = std::min(gl, h[3 * b + 2]);
  }
  *ninf = m;
  *lo = gl;
  *hi = gh;
  if (!std::isfinite(m) || !std::isfinite(gl) || !std::isfinite(gh)) return REFINE_ENONFINITE;
  return REFINE_OK;
}

double shift_for(const refine_options& opt, double lo, double hi) {
  switch (opt.target) {
    case REFINE_TARGET_SMALLEST:
      return hi;
    case REFINE_TARGET_LARGEST:
      return lo;
    case REFINE_TARGET_SHIFT:
      return opt.shift;
    default:
      return 0.0;
  }
}

// Squared variant (Sec. 5.2): B = A^2 - alpha I with alpha = (||A||^2 +
// lam^2) / 2, lam = opt.shift the caller's estimate of the (k+1)-th smallest
// |lambda|; without an estimate alpha = ||A||^2, which also separates the
// targets (more slowly).  Returns alpha; *norm_b receives ||A||^2, the bound
// of ||B|| used for delta and the residual statistic.
double square_alpha(const refine_options& opt, double norm, double* norm_b) {
  *norm_b = norm * norm;
  return opt.shift > 0.0 ? 0.5 * (norm * norm + opt.shift * opt.shift) : norm * norm;
}

int read_ctrl(Plan& pl, hipStream_t st, std::vector<Ctrl>& out) {
  out.resize(pl.hprob.size());
  RF_CHECK(hipMemcpyAsync(out.data(), pl.ctrl, sizeof(Ctrl) * out.size(), hipMemcpyDeviceToHost, st));
  RF_CHECK(hipStreamSynchronize(st));
  return REFINE_OK;
}

}  // namespace

extern "C" {

void refine_options_default(refine_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = REFINE_FP64;
  o->target = REFINE_TARGET_LARGEST_ABS;
  o->shift = 0.0;
  o->delta_c = 10.0;
  o->norm_a = 0.0;
  o->beta = REFINE_BETA_HALF_GRAM;
  o->normalize = 1;
  o->slices = 0;
}

const char* refine_status_string(int s) {
  switch (s) {
    case REFINE_OK:
      return "ok";
    case REFINE_NOT_CONVERGED:
      return "not converged within max_iters";
    case REFINE_EINVAL:
      return "invalid argument";
    case REFINE_ENOMEM:
      return "out of memory";
    case REFINE_EHIP:
      return "HIP runtime error";
    case REFINE_EWY_SINGULAR:
      return "Y1 = X(1:k,:) - I singular or ill-conditioned (compact WY needs it nonsingular; refine_sign_flip)";
    case REFINE_EDIVERGED:
      return "refinement diverged (||E_L||_F >= 1 or growing)";
    case REFINE_ENONFINITE:
      return "non-finite values";
    case REFINE_ERANK:
      return "X^T X is not positive definite (dependent columns)";
    default:
      return "unknown status";
  }
}

int refine_init(refine_ctx** out, const refine_matrix* A, int32_t k, const refine_options* optp,
                void* hip_stream) {
  if (!out) return REFINE_EINVAL;
  *out = nullptr;
  refine_options opt;
  if (optp)
    opt = *optp;
  else
    refine_options_default(&opt);
  if (opt.delta_c == 0.0 && !optp) opt.delta_c = 10.0;
  int rc = validate_matrix(A, k, opt);
  if (rc != REFINE_OK) return rc;
  refine_ctx* c = new (std::nothrow) refine_ctx();
  if (!c) return REFINE_ENOMEM;
  c->stream = (hipStream_t)hip_stream;
  c->A = *A;
  c->opt = opt;
  c->k = k;
  rc = matrix_stats(*A, c->stream, &c->norm_inf, &c->g_lo, &c->g_hi);
  if (rc != REFINE_OK) {
    delete c;
    return rc;
  }
  c->norm_used = opt.norm_a > 0.0 ? opt.norm_a : c->norm_inf;
  if (opt.target == REFINE_TARGET_SMALLEST_ABS)
    c->mu = square_alpha(opt, c->norm_used, &c->norm_used);
  else
    c->mu = shift_for(opt, c->g_lo, c->g_hi);
  c->delta = opt.delta_c * c->norm_used * UNIT_ROUNDOFF;
  std::vector<refine_matrix> As{*A};
  std::vector<int> ks{k};
  rc = build_plan(c->plan, As, ks, opt, {c->mu}, {c->delta}, {c->norm_used});
  if (rc == REFINE_OK && c->plan.split) {
    const bool crt = opt.precision == REFINE_SPLIT_CRT;
    rc = split_init(c->plan.sp, {*A}, {k}, crt ? 0 : (opt.slices > 0 ? opt.slices : SPLIT_S_DEFAULT),
                    crt ? (opt.slices > 0 ? opt.slices : CRT_N_DEFAULT) : 0, c->plan.hprob,
                    c->plan.dprob, c->stream);
  }
  if (rc == REFINE_OK) rc = capture_graph(c->plan, RUN_CHUNK);
  if (rc == REFINE_OK && launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess)
    rc = REFINE_EHIP;
  if (rc == REFINE_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = REFINE_EHIP;
  if (rc != REFINE_OK) {
    free_plan(c->plan);
    delete c;
    return rc;
  }
  *out = c;
  return REFINE_OK;
}

// Events of refine_time_product_parts: one before each timed launch of the
// product and one after each of its kernels (product_mark).
constexpr int PART_MAX = 8;        // kernels of one product launch, at most
constexpr int PART_REPS_MAX = 64;  // timed launches per call
struct PartTimer {
  hipEvent_t ev[(PART_MAX + 1) * PART_REPS_MAX] = {};
  int cap = 0, used = 0;
  bool overflow = false;
  void destroy() {
    for (hipEvent_t& v : ev)
      if (v) (void)hipEventDestroy(v), v = nullptr;
  }
};
static PartTimer* g_part_timer = nullptr;

// Steps enqueued without statistics leave an error status in the control
// word, where later steps see it and do nothing.  Every call that resets the
// control word first reports such a status (and clears it), so that an error
// surfaces at the next call that reports one instead of being reset away.
static int take_pending(refine_ctx* c, refine_stats* stats) {
  if (!c->pending) return REFINE_OK;
  c->pending = false;
  std::vector<Ctrl> cs;
  int rc = read_ctrl(c->plan, c->stream, cs);
  if (rc != REFINE_OK) return rc;
  const int st = cs[0].status;
  if (st == 0) return REFINE_OK;
  if (stats) {
    stats->corr_fro = cs[0].corr_fro;
    stats->resid_rel = cs[0].resid_rel;
    stats->iters = cs[0].iters;
    stats->status = st;
  }
  if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  return st;
}

static int set_x(refine_ctx* c, double* X, int64_t ldx, refine_stats* stats = nullptr) {
  if (!X || ldx < c->k) return REFINE_EINVAL;
  if (X != c->cur_x || ldx != c->cur_ldx) {
    int prc = take_pending(c, stats);
    if (prc != REFINE_OK) return prc;
    if (launch_set_x(c->plan.dprob, 0, X, ldx, c->stream) != hipSuccess) return REFINE_EHIP;
    if (c->plan.square && launch_set_x(c->plan.dprob1, 0, X, ldx, c->stream) != hipSuccess)
      return REFINE_EHIP;
    // a new iterate starts a new history for the divergence test
    if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
    c->cur_x = X;
    c->cur_ldx = ldx;
  }
  return REFINE_OK;
}

int refine_step(refine_ctx* c, double* X, int64_t ldx, refine_stats* stats) {
  if (!c) return REFINE_EINVAL;
  int rc = set_x(c, X, ldx);
  if (rc != REFINE_OK) return rc;
  if (hipGraphLaunch(c->plan.exec, c->stream) != hipSuccess) return REFINE_EHIP;
  if (!stats) {
    c->pending = true;
    return REFINE_OK;
  }
  c->pending = false;
  std::vector<Ctrl> cs;
  rc = read_ctrl(c->plan, c->stream, cs);
  if (rc != REFINE_OK) return rc;
  stats->corr_fro = cs[0].corr_fro;
  stats->resid_rel = cs[0].resid_rel;
  stats->iters = cs[0].iters;
  stats->status = cs[0].status;
  const int st = cs[0].status;
  if (st != 0) {
    // report once, then let the next step start afresh
    if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  }
  return st;
}

int refine_rayleigh_ritz(refine_ctx* c, double* X, int64_t ldx) {
  if (!c) return REFINE_EINVAL;
  int rc = set_x(c, X, ldx);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending(c, nullptr)) != REFINE_OK) return rc;
  Plan& pl = c->plan;
  hipStream_t st = c->stream;
  hipError_t e = launch_ctrl_reset(pl.dprob, 1, 0, 0.0, st);
  if (e == hipSuccess) e = enqueue_product(pl, st);
  if (e == hipSuccess) e = launch_rr_prep(pl.dprob, 1, st);
  if (e == hipSuccess) e = launch_gram(pl.dprob, pl.gram_items, pl.n_gram, pl.kmax, pl.split, st);
  if (e == hipSuccess) e = launch_gram_reduce(pl.dprob, pl.gred_items, pl.n_gred, st);
  if (e == hipSuccess) e = launch_rr_solve(pl.dprob, 1, st);
  if (e == hipSuccess) e = launch_rr_apply(pl.dprob, pl.row_items, pl.n_row, st);
  if (e != hipSuccess) return REFINE_EHIP;
  std::vector<Ctrl> cs;
  rc = read_ctrl(pl, st, cs);
  if (rc != REFINE_OK) return rc;
  const int status = cs[0].status;
  if (status != 0) {
    if (launch_ctrl_reset(pl.dprob, 1, 0, 0.0, st) != hipSuccess) return REFINE_EHIP;
    return status;
  }
  return REFINE_OK;
}

int refine_sign_flip(refine_ctx* c, double* X, int64_t ldx, int32_t* sigma) {
  if (!c) return REFINE_EINVAL;
  int rc = set_x(c, X, ldx);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending(c, nullptr)) != REFINE_OK) return rc;
  Plan& pl = c->plan;
  hipStream_t st = c->stream;
  hipError_t e = launch_ctrl_reset(pl.dprob, 1, 0, 0.0, st);
  if (e == hipSuccess) e = launch_flip_sigma(pl.dprob, 1, st);
  if (e == hipSuccess) e = launch_flip_apply(pl.dprob, pl.row_items, pl.n_row, st);
  if (e != hipSuccess) return REFINE_EHIP;
  std::vector<double> sg;
  if (sigma) {
    sg.resize(c->k);
    RF_CHECK(hipMemcpyAsync(sg.data(), pl.hprob[0].vec + VEC_SCALE * c->k, sizeof(double) * c->k,
                            hipMemcpyDeviceToHost, st));
  }
  std::vector<Ctrl> cs;
  rc = read_ctrl(pl, st, cs);
  if (rc != REFINE_OK) return rc;
  const int status = cs[0].status;
  if (status != 0) {
    if (launch_ctrl_reset(pl.dprob, 1, 0, 0.0, st) != hipSuccess) return REFINE_EHIP;
    return status;
  }
  for (int j = 0; sigma && j < c->k; ++j) sigma[j] = sg[j] < 0.0 ? -1 : 1;
  return REFINE_OK;
}

int refine_run(refine_ctx* c, double* X, int64_t ldx, int32_t max_iters, refine_stop stop,
               double tol, refine_stats* stats) {
  if (!c || max_iters < 0) return REFINE_EINVAL;
  if (stop != REFINE_STOP_ITERS && stop != REFINE_STOP_CORRECTION && stop != REFINE_STOP_RESIDUAL)
    return REFINE_EINVAL;
  int rc = set_x(c, X, ldx, stats);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending(c, stats)) != REFINE_OK) return rc;
  if (launch_ctrl_reset(c->plan.dprob, 1, (int)stop, tol, c->stream) != hipSuccess) return REFINE_EHIP;
  std::vector<Ctrl> cs(1);
  int done = 0;
  while (done < max_iters) {
    const int m = std::min(RUN_CHUNK, max_iters - done);
    if (launch_steps(c->plan, m, c->stream) != hipSuccess) return REFINE_EHIP;
    done += m;
    rc = read_ctrl(c->plan, c->stream, cs);
    if (rc != REFINE_OK) return rc;
    if (cs[0].stopped) break;
  }
  if (stats) {
    stats->corr_fro = cs[0].corr_fro;
    stats->resid_rel = cs[0].resid_rel;
    stats->iters = cs[0].iters;
    stats->status = cs[0].status;
  }
  int result;
  if (cs[0].status != 0)
    result = cs[0].status;
  else if (stop == REFINE_STOP_ITERS || cs[0].converged)
    result = REFINE_OK;
  else
    result = REFINE_NOT_CONVERGED;
  if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  return result;
}

int refine_time_product(refine_ctx* c, double* X, int64_t ldx, int32_t reps, float* ms) {
  if (!c || reps <= 0 || !ms) return REFINE_EINVAL;
  int rc = set_x(c, X, ldx);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending(c, nullptr)) != REFINE_OK) return rc;
  if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  hipEvent_t e0, e1;
  RF_CHECK(hipEventCreate(&e0));
  RF_CHECK(hipEventCreate(&e1));
  Plan& pl = c->plan;
  hipError_t e = hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    if (pl.csr)
      e = launch_spmm(pl.dprob, pl.spmm_items, pl.n_spmm, pl.hprob[0].k, pl.spmm_lanes, pl.spmm_grid,
                      c->stream);
    else if (pl.split)
      e = split_product(pl.sp, pl.dprob, c->stream);
    else
      e = launch_gemm_f64(pl.dprob, pl.gemm_items, pl.n_gemm, pl.kmax, pl.vec2, pl.gemm_cfg,
                          c->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return REFINE_EHIP;
  *ms = t / (float)reps;
  if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  return REFINE_OK;
}

int refine_time_product_parts(refine_ctx* c, double* X, int64_t ldx, int32_t reps, float* ms,
                              int32_t max_parts, int32_t* nparts) {
  if (!c || reps <= 0 || reps > PART_REPS_MAX || !ms || max_parts <= 0 || !nparts)
    return REFINE_EINVAL;
  int rc = set_x(c, X, ldx);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending(c, nullptr)) != REFINE_OK) return rc;
  if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  Plan& pl = c->plan;
  PartTimer tm;
  hipError_t e = hipSuccess;
  const int cap = (PART_MAX + 1) * reps;
  for (int i = 0; i < cap && e == hipSuccess; ++i) e = hipEventCreate(&tm.ev[i]);
  if (e != hipSuccess) {
    tm.destroy();
    return REFINE_EHIP;
  }
  tm.cap = cap;
  // a warm-up launch, then reps launches, each bracketed by its own events
  auto one = [&]() -> hipError_t {
    if (pl.csr) {
      hipError_t r = launch_spmm(pl.dprob, pl.spmm_items, pl.n_spmm, pl.hprob[0].k, pl.spmm_lanes,
                                 pl.spmm_grid, c->stream);
      product_mark(c->stream);
      return r;
    }
    if (pl.split) return split_product(pl.sp, pl.dprob, c->stream);
    hipError_t r = launch_gemm_f64(pl.dprob, pl.gemm_items, pl.n_gemm, pl.kmax, pl.vec2,
                                   pl.gemm_cfg, c->stream);
    product_mark(c->stream);
    return r;
  };
  e = one();
  int parts = 0;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    const int first = tm.used;
    e = hipEventRecord(tm.ev[tm.used++], c->stream);
    g_part_timer = &tm;
    if (e == hipSuccess) e = one();
    g_part_timer = nullptr;
    const int p = tm.used - first - 1;
    if (r == 0) parts = p;
    if (p != parts || tm.overflow) e = hipErrorInvalidValue;
  }
  if (e == hipSuccess) e = hipEventSynchronize(tm.ev[tm.used - 1]);
  std::vector<double> sum(parts, 0.0);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    for (int i = 0; i < parts && e == hipSuccess; ++i) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, tm.ev[r * (parts + 1) + i], tm.ev[r * (parts + 1) + i + 1]);
      sum[i] += t;
    }
  tm.destroy();
  if (e != hipSuccess) return REFINE_EHIP;
  *nparts = parts;
  for (int i = 0; i < parts && i < max_parts; ++i) ms[i] = (float)(sum[i] / reps);
  if (launch_ctrl_reset(c->plan.dprob, 1, 0, 0.0, c->stream) != hipSuccess) return REFINE_EHIP;
  return REFINE_OK;
}

int refine_get_info(const refine_ctx* c, double* mu, double* norm_inf, double* norm_used,
                    double* delta) {
  if (!c) return REFINE_EINVAL;
  if (mu) *mu = c->mu;
  if (norm_inf) *norm_inf = c->norm_inf;
  if (norm_used) *norm_used = c->norm_used;
  if (delta) *delta = c->delta;
  return REFINE_OK;
}

int refine_destroy(refine_ctx* c) {
  if (!c) return REFINE_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  free_plan(c->plan);
  delete c;
  return REFINE_OK;
}

int refine_batch_init(refine_batch** out, int32_t count, const refine_matrix* As,
                      const int32_t* ks, const refine_options* optp, void* hip_stream) {
  if (!out || count <= 0 || !As || !ks) return REFINE_EINVAL;
  *out = nullptr;
  refine_options opt;
  if (optp)
    opt = *optp;
  else
    refine_options_default(&opt);
  // the modular form serves one problem (its product is bound by the residue
  // planes' bytes, more than a batch's FP64 product reads)
  if (opt.precision == REFINE_SPLIT_CRT) return REFINE_EINVAL;
  for (int p = 0; p < count; ++p) {
    if (As[p].kind != REFINE_DENSE) return REFINE_EINVAL;
    int rc = validate_matrix(&As[p], ks[p], opt);
    if (rc != REFINE_OK) return rc;
  }
  refine_batch* b = new (std::nothrow) refine_batch();
  if (!b) return REFINE_ENOMEM;
  b->stream = (hipStream_t)hip_stream;
  b->opt = opt;
  b->As.assign(As, As + count);
  b->ks.assign(ks, ks + count);
  std::vector<double> mus(count), deltas(count), norms(count);
  for (int p = 0; p < count; ++p) {
    double ninf, lo, hi;
    int rc = matrix_stats(As[p], b->stream, &ninf, &lo, &hi);
    if (rc != REFINE_OK) {
      delete b;
      return rc;
    }
    norms[p] = opt.norm_a > 0.0 ? opt.norm_a : ninf;
    if (opt.target == REFINE_TARGET_SMALLEST_ABS)
      mus[p] = square_alpha(opt, norms[p], &norms[p]);
    else
      mus[p] = shift_for(opt, lo, hi);
    deltas[p] = opt.delta_c * norms[p] * UNIT_ROUNDOFF;
  }
  int rc = build_plan(b->plan, b->As, b->ks, opt, mus, deltas, norms);
  if (rc == REFINE_OK && b->plan.split)
    rc = split_init(b->plan.sp, b->As, b->ks, opt.slices > 0 ? opt.slices : SPLIT_S_DEFAULT, 0,
                    b->plan.hprob, b->plan.dprob, b->stream);
  if (rc == REFINE_OK) rc = capture_graph(b->plan, BATCH_GRAPH_STEPS);
  if (rc == REFINE_OK && hipMalloc((void**)&b->d_xs, sizeof(double*) * 2 * count) != hipSuccess)
    rc = REFINE_ENOMEM;
  if (rc == REFINE_OK && launch_ctrl_reset(b->plan.dprob, count, 0, 0.0, b->stream) != hipSuccess)
    rc = REFINE_EHIP;
  if (rc == REFINE_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = REFINE_EHIP;
  if (rc != REFINE_OK) {
    free_plan(b->plan);
    (void)hipFree(b->d_xs);
    delete b;
    return rc;
  }
  b->cur_x.assign(count, nullptr);
  b->cur_ldx.assign(count, -1);
  *out = b;
  return REFINE_OK;
}

// As take_pending, for the runs of a batch enqueued without statistics:
// returns the first failing problem's status (REFINE_OK if none) and fills
// per (count entries) when given.
static int take_pending_batch(refine_batch* b, refine_stats* per) {
  if (!b->pending) return REFINE_OK;
  b->pending = false;
  const int np = (int)b->As.size();
  std::vector<Ctrl> cs;
  int rc = read_ctrl(b->plan, b->stream, cs);
  if (rc != REFINE_OK) return rc;
  int worst = REFINE_OK;
  for (int p = 0; p < np; ++p)
    if (cs[p].status != 0 && worst == REFINE_OK) worst = cs[p].status;
  if (worst == REFINE_OK) return REFINE_OK;
  for (int p = 0; per && p < np; ++p) {
    per[p].corr_fro = cs[p].corr_fro;
    per[p].resid_rel = cs[p].resid_rel;
    per[p].iters = cs[p].iters;
    per[p].status = cs[p].status;
  }
  if (launch_ctrl_reset(b->plan.dprob, np, 0, 0.0, b->stream) != hipSuccess) return REFINE_EHIP;
  return worst;
}

// Binds the problems' iterates (device descriptors rewritten only on change).
static int bind_batch_x(refine_batch* b, double* const* Xs, const int64_t* ldxs) {
  const int np = (int)b->As.size();
  bool changed = false;
  for (int p = 0; p < np; ++p) {
    const int64_t ld = ldxs ? ldxs[p] : b->ks[p];
    if (!Xs[p] || ld < b->ks[p]) return REFINE_EINVAL;
    if (Xs[p] != b->cur_x[p] || ld != b->cur_ldx[p]) changed = true;
  }
  if (changed) {
    // an error of the old iterates is reported before their history is reset
    int prc = take_pending_batch(b, nullptr);
    if (prc != REFINE_OK) return prc;
    // descriptors are rewritten in place; wait for queued work first
    if (hipStreamSynchronize(b->stream) != hipSuccess) return REFINE_EHIP;
    for (int p = 0; p < np; ++p) {
      b->plan.hprob[p].x = Xs[p];
      b->plan.hprob[p].ldx = ldxs ? ldxs[p] : b->ks[p];
      b->cur_x[p] = Xs[p];
      b->cur_ldx[p] = b->plan.hprob[p].ldx;
    }
    if (hipMemcpy(b->plan.dprob, b->plan.hprob.data(), sizeof(Prob) * np, hipMemcpyHostToDevice) !=
        hipSuccess)
      return REFINE_EHIP;
    if (upload_square_descs(b->plan) != REFINE_OK) return REFINE_EHIP;
    // new iterates start a new history for the divergence test
    if (launch_ctrl_reset(b->plan.dprob, np, 0, 0.0, b->stream) != hipSuccess) return REFINE_EHIP;
  }
  return REFINE_OK;
}

int refine_batch_run(refine_batch* b, double* const* Xs, const int64_t* ldxs, int32_t iters,
                     refine_stats* per) {
  if (!b || !Xs || iters < 0) return REFINE_EINVAL;
  const int np = (int)b->As.size();
  int brc = bind_batch_x(b, Xs, ldxs);
  if (brc != REFINE_OK) return brc;
  if (launch_steps(b->plan, iters, b->stream) != hipSuccess) return REFINE_EHIP;
  if (!per) {
    b->pending = true;
    return REFINE_OK;
  }
  b->pending = false;
  std::vector<Ctrl> cs;
  int rc = read_ctrl(b->plan, b->stream, cs);
  if (rc != REFINE_OK) return rc;
  int worst = REFINE_OK;
  bool any_bad = false;
  for (int p = 0; p < np; ++p) {
    per[p].corr_fro = cs[p].corr_fro;
    per[p].resid_rel = cs[p].resid_rel;
    per[p].iters = cs[p].iters;
    per[p].status = cs[p].status;
    if (cs[p].status != 0) {
      any_bad = true;
      if (worst == REFINE_OK) worst = cs[p].status;
    }
  }
  if (any_bad && launch_ctrl_reset(b->plan.dprob, np, 0, 0.0, b->stream) != hipSuccess)
    return REFINE_EHIP;
  return worst;
}

int refine_batch_rayleigh_ritz(refine_batch* b, double* const* Xs, const int64_t* ldxs,
                               int32_t* status) {
  if (!b || !Xs) return REFINE_EINVAL;
  const int np = (int)b->As.size();
  int rc = bind_batch_x(b, Xs, ldxs);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending_batch(b, nullptr)) != REFINE_OK) return rc;
  Plan& pl = b->plan;
  hipStream_t st = b->stream;
  hipError_t e = launch_ctrl_reset(pl.dprob, np, 0, 0.0, st);
  if (e == hipSuccess) e = enqueue_product(pl, st);
  if (e == hipSuccess) e = launch_rr_prep(pl.dprob, np, st);
  if (e == hipSuccess) e = launch_gram(pl.dprob, pl.gram_items, pl.n_gram, pl.kmax, pl.split, st);
  if (e == hipSuccess) e = launch_gram_reduce(pl.dprob, pl.gred_items, pl.n_gred, st);
  if (e == hipSuccess) e = launch_rr_solve(pl.dprob, np, st);
  if (e == hipSuccess) e = launch_rr_apply(pl.dprob, pl.row_items, pl.n_row, st);
  if (e != hipSuccess) return REFINE_EHIP;
  std::vector<Ctrl> cs;
  rc = read_ctrl(pl, st, cs);
  if (rc != REFINE_OK) return rc;
  int worst = REFINE_OK;
  for (int p = 0; p < np; ++p) {
    if (status) status[p] = cs[p].status;
    if (cs[p].status != 0 && worst == REFINE_OK) worst = cs[p].status;
  }
  if (worst != REFINE_OK && launch_ctrl_reset(pl.dprob, np, 0, 0.0, st) != hipSuccess)
    return REFINE_EHIP;
  return worst;
}

int refine_batch_sign_flip(refine_batch* b, double* const* Xs, const int64_t* ldxs, int32_t* status) {
  if (!b || !Xs) return REFINE_EINVAL;
  const int np = (int)b->As.size();
  int rc = bind_batch_x(b, Xs, ldxs);
  if (rc != REFINE_OK) return rc;
  if ((rc = take_pending_batch(b, nullptr)) != REFINE_OK) return rc;
  Plan& pl = b->plan;
  hipStream_t st = b->stream;
  hipError_t e = launch_ctrl_reset(pl.dprob, np, 0, 0.0, st);
  if (e == hipSuccess) e = launch_flip_sigma(pl.dprob, np, st);
  if (e == hipSuccess) e = launch_flip_apply(pl.dprob, pl.row_items, pl.n_row, st);
  if (e != hipSuccess) return REFINE_EHIP;
  std::vector<Ctrl> cs;
  rc = read_ctrl(pl, st, cs);
  if (rc != REFINE_OK) return rc;
  int worst = REFINE_OK;
  for (int p = 0; p < np; ++p) {
    if (status) status[p] = cs[p].status;
    if (cs[p].status != 0 && worst == REFINE_OK) worst = cs[p].status;
  }
  if (worst != REFINE_OK && launch_ctrl_reset(pl.dprob, np, 0, 0.0, st) != hipSuccess)
    return REFINE_EHIP;
  return worst;
}

int refine_batch_time_product(refine_batch* b, int32_t reps, float* ms) {
  if (!b || reps <= 0 || !ms) return REFINE_EINVAL;
  for (double* x : b->cur_x)
    if (!x) return REFINE_EINVAL;  // no X bound yet
  int prc = take_pending_batch(b, nullptr);
  if (prc != REFINE_OK) return prc;
  Plan& pl = b->plan;
  const int np = (int)pl.hprob.size();
  hipEvent_t e0, e1;
  RF_CHECK(hipEventCreate(&e0));
  RF_CHECK(hipEventCreate(&e1));
  hipError_t e = hipSuccess;
  if (launch_ctrl_reset(pl.dprob, np, 0, 0.0, b->stream) != hipSuccess) e = hipErrorUnknown;
  if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = pl.split ? split_product(pl.sp, pl.dprob, b->stream)
                 : launch_gemm_f64(pl.dprob, pl.gemm_items, pl.n_gemm, pl.kmax, pl.vec2, pl.gemm_cfg,
                                   b->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return REFINE_EHIP;
  *ms = t / (float)reps;
  if (launch_ctrl_reset(pl.dprob, np, 0, 0.0, b->stream) != hipSuccess) return REFINE_EHIP;
  return REFINE_OK;
}

int refine_batch_destroy(refine_batch* b) {
  if (!b) return REFINE_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  free_plan(b->plan);
  (void)hipFree(b->d_xs);
  delete b;
  return REFINE_OK;
}

}  // extern "C"

// Diagnostic hook declared in refine_debug.h: device addresses of the
// workspace of a single-problem context, in the order w, wlo, xn, kk, vec,
// ctrl, wp, part, gpart.  Used by the tests to inspect intermediate quantities.
extern "C" int refine_debug_workspace(const refine_ctx* c, void** out, int32_t count) {
  if (!c || !out || count < 1) return REFINE_EINVAL;
  const Prob& P = c->plan.hprob[0];
  void* v[9] = {P.w, P.wlo, P.xn, P.kk, P.vec, P.ctrl, P.wp, P.part, P.gpart};
  for (int i = 0; i < 9 && i < count; ++i) out[i] = v[i];
  return REFINE_OK;
}

// ---------------------------------------------------------------------------
// One step without any allocation (refine_step_static).
//
// Every piece of device memory the step needs beyond A and X -- the problem
// descriptor, the work-item tables and the workspace (W, the update, the
// block partials, the k x k area and the control word) -- lives in the
// file-scope array below, carved up per call.  Host code never passes the
// array's name to a kernel: its device address on the current GPU comes from
// hipGetSymbolAddress on the first call made on that GPU and is kept per
// device.  A setup kernel writes the descriptor and the items and clears the
// workspace (a fill kernel, not a memset, so that a caller may capture the
// call in a graph), then the step's kernels run as in refine_step with a
// fixed launch configuration (no tuner, no K split).  Every call on a GPU
// uses that GPU's array: calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;  // 64 MiB per GPU
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int STATIC_GEMM_CFG = 3;   // 4 wavefronts, 64 rows per block, 32-row K chunks
constexpr int STATIC_MAX_GRAM_BLOCKS = 64;
constexpr int STATIC_MAX_DEVICES = 64;
char* g_scratch[STATIC_MAX_DEVICES] = {};

__global__ void static_setup_kernel(Prob p, Prob* dprob, GemmItem* gi, int n_gemm, int bm,
                                    RowItem* ri, int n_row, RowItem* gri, int n_gram,
                                    GramRedItem* rr, int n_gred, double* ws, int64_t ws_words) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) *dprob = p;
  for (int64_t i = tid; i < n_gemm; i += T) {
    GemmItem g{};
    g.row0 = (int)i * bm;
    g.k1 = p.n;
    gi[i] = g;
  }
  for (int64_t i = tid; i < n_row; i += T) ri[i] = RowItem{0, (int)i};
  for (int64_t i = tid; i < n_gram; i += T) gri[i] = RowItem{0, (int)i};
  for (int64_t i = tid; i < n_gred; i += T) rr[i] = GramRedItem{0, (int)i * 64};
  for (int64_t i = tid; i < ws_words; i += T) ws[i] = 0.0;
}

struct StaticLayout {
  Shape s;
  int n_gemm, n_row, n_gram, n_gred, gh;
  size_t o_prob, o_gemm, o_row, o_gram, o_gred, o_ws;
  size_t o_w, o_xn, o_part, o_dpart, o_gpart, o_kk, o_kpp, o_vec, o_ctrl, total;
};

StaticLayout static_layout(int64_t n, int k) {
  StaticLayout L{};
  L.s = choose_shape(n, k, true, false);
  // Gram blocks: at most STATIC_MAX_GRAM_BLOCKS, so that their k x k partials
  // stay a small part of the array
  const int64_t per = (n + STATIC_MAX_GRAM_BLOCKS - 1) / STATIC_MAX_GRAM_BLOCKS;
  L.s.gbrows = (int)std::max<int64_t>(L.s.gbrows, (per + 3) / 4 * 4);
  L.s.ngb = iceil(n, L.s.gbrows);
  L.s.ksplit = 1;
  L.gh = gram_groups(k);
  L.n_gemm = iceil(n, gemm_rows_per_block(STATIC_GEMM_CFG));
  L.n_row = L.s.nrb;
  L.n_gram = L.s.ngb * L.gh;
  L.n_gred = iceil(2 * (int64_t)k * k + k, 64);
  size_t o = 0;
  L.o_prob = o;  o += align_up(sizeof(Prob));
  L.o_gemm = o;  o += align_up(sizeof(GemmItem) * L.n_gemm);
  L.o_row = o;   o += align_up(sizeof(RowItem) * L.n_row);
  L.o_gram = o;  o += align_up(sizeof(RowItem) * L.n_gram);
  L.o_gred = o;  o += align_up(sizeof(GramRedItem) * L.n_gred);
  L.o_ws = o;
  const size_t nk = (size_t)n * k * sizeof(double);
  L.o_w = o;     o += align_up(nk);
  L.o_xn = o;    o += align_up(nk);
  L.o_part = o;  o += align_up((size_t)L.s.nrb * 5 * k * sizeof(double));
  L.o_dpart = o; o += align_up((size_t)std::max(L.n_gemm, L.s.nrb) * 2 * k * sizeof(double));
  L.o_gpart = o; o += align_up((size_t)L.s.ngb * (2 * k * k + k) * sizeof(double));
  L.o_kk = o;    o += align_up((size_t)KK_COUNT * k * k * sizeof(double));
  L.o_kpp = o;   o += align_up((size_t)(16 + 16 * k) * sizeof(double));
  L.o_vec = o;   o += align_up((size_t)VEC_COUNT * k * sizeof(double));
  L.o_ctrl = o;  o += align_up(sizeof(Ctrl));
  L.total = o;
  return L;
}

// The array's device address on the current GPU (hipGetSymbolAddress once
// per device, with that device current).
int static_scratch(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) return REFINE_EHIP;
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return REFINE_EHIP;
    g_scratch[dev] = (char*)p;
  }
  *out = g_scratch[dev];
  return REFINE_OK;
}

}  // namespace

extern "C" int refine_step_static(const refine_matrix* A, int32_t k, const refine_options* optp,
                                  double* X, int64_t ldx, void* hip_stream, refine_stats* stats) {
  refine_options opt;
  if (optp)
    opt = *optp;
  else
    refine_options_default(&opt);
  if (!A || A->kind != REFINE_DENSE || !A->a || A->n <= 0 || A->n >= (int64_t)1 << 31 ||
      A->lda < A->n || k < 1 || k > KMAX || (int64_t)k >= A->n || !X || ldx < k)
    return REFINE_EINVAL;
  if (opt.precision != REFINE_FP64 || !(opt.norm_a > 0.0) || !(opt.delta_c >= 0.0) ||
      (opt.target != REFINE_TARGET_LARGEST_ABS && opt.target != REFINE_TARGET_SHIFT))
    return REFINE_EINVAL;
  const int64_t n = A->n;
  const StaticLayout L = static_layout(n, k);
  if (L.total > STATIC_SCRATCH_BYTES) return REFINE_EINVAL;
  char* base = nullptr;
  int rc = static_scratch(&base);
  if (rc != REFINE_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;

  Prob P;
  memset(&P, 0, sizeof(P));
  P.a = A->a;
  P.lda = A->lda;
  P.x = X;
  P.ldx = ldx;
  P.n = (int32_t)n;
  P.k = k;
  P.kind = REFINE_DENSE;
  P.ksplit = 1;
  P.nrb = L.s.nrb;
  P.rbrows = L.s.rbrows;
  P.ngb = L.s.ngb;
  P.gbrows = L.s.gbrows;
  P.w = (double*)(base + L.o_w);
  P.xn = (double*)(base + L.o_xn);
  P.part = (double*)(base + L.o_part);
  P.dpart = (double*)(base + L.o_dpart);
  P.ndp = L.n_gemm;
  P.gpart = (double*)(base + L.o_gpart);
  P.kk = (double*)(base + L.o_kk);
  P.kpp = (double*)(base + L.o_kpp);
  P.vec = (double*)(base + L.o_vec);
  P.ctrl = (Ctrl*)(base + L.o_ctrl);
  P.mu = opt.target == REFINE_TARGET_SHIFT ? opt.shift : 0.0;
  P.delta = opt.delta_c * opt.norm_a * UNIT_ROUNDOFF;
  P.norm_a = opt.norm_a;
  P.beta_zero = opt.beta == REFINE_BETA_ZERO;
  P.normalize = opt.normalize != 0;
  Prob* dprob = (Prob*)(base + L.o_prob);
  GemmItem* gi = (GemmItem*)(base + L.o_gemm);
  RowItem* ri = (RowItem*)(base + L.o_row);
  RowItem* gri = (RowItem*)(base + L.o_gram);
  GramRedItem* rr = (GramRedItem*)(base + L.o_gred);
  const int64_t ws_words = (int64_t)((L.total - L.o_ws) / sizeof(double));
  const bool vec2 = ((uintptr_t)A->a & 7) == 0;
  const bool fused = k <= 32, pipeline = k > KXK_ONE_WG_MAX;

  hipLaunchKernelGGL(static_setup_kernel, dim3(1024), dim3(256), 0, st, P, dprob, gi, L.n_gemm,
                     gemm_rows_per_block(STATIC_GEMM_CFG), ri, L.n_row, gri, L.n_gram, rr, L.n_gred,
                     (double*)(base + L.o_ws), ws_words);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_ctrl_reset(dprob, 1, 0, 0.0, st);
  if (e == hipSuccess) e = launch_gemm_f64(dprob, gi, L.n_gemm, k, vec2, STATIC_GEMM_CFG, st);
  if (e == hipSuccess) e = launch_fin_d(dprob, 1, st);
  if (e == hipSuccess) e = launch_gram(dprob, gri, L.n_gram, k, false, st);
  if (e == hipSuccess) e = launch_gram_reduce(dprob, rr, L.n_gred, st);
  if (e == hipSuccess) e = launch_kxk(dprob, 1, k, pipeline, false, st);
  if (fused) {
    if (e == hipSuccess) e = launch_fin_pre(dprob, 1, st);
    if (e == hipSuccess) e = launch_update(dprob, ri, L.n_row, k, true, st);
  } else {
    if (e == hipSuccess) e = launch_update(dprob, ri, L.n_row, k, false, st);
    if (e == hipSuccess) e = launch_fin_stats(dprob, 1, st);
    if (e == hipSuccess) e = launch_normalize(dprob, ri, L.n_row, st);
  }
  if (e != hipSuccess) return REFINE_EHIP;
  if (!stats) return REFINE_OK;
  Ctrl c;
  e = hipMemcpyAsync(&c, base + L.o_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return REFINE_EHIP;
  stats->corr_fro = c.corr_fro;
  stats->resid_rel = c.resid_rel;
  stats->iters = c.iters;
  stats->status = c.status;
  return c.status;
}

namespace rfk {
void product_mark(hipStream_t st) {
  PartTimer* t = g_part_timer;
  if (!t) return;
  if (t->used >= t->cap) {
    t->overflow = true;
    return;
  }
  (void)hipEventRecord(t->ev[t->used++], st);
}
}  // namespace rfk
