// C-ABI of the MI355X CBS library: planner, launches, solver loops.
//
// A plan owns a copy of k^2 (in the operator precision and in FP64), the
// twiddle tables, the ragged work lists and every scratch buffer; calls after
// cbs_setup never allocate.  Operator applications are the three-launch
// pipeline of kernels.hpp.  The solvers keep the iterate in FP64 and run the
// bulk sweeps in the operator precision (FP32 for CBS_C64 plans).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/cbs.h"
#include "launch.hpp"
#include "params.hpp"

using namespace cbs;

namespace {

thread_local std::string g_err;

cbs_status fail(cbs_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(CBS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHK(expr)                    \
  do {                               \
    cbs_status s_ = (expr);          \
    if (s_ != CBS_OK) return s_;     \
  } while (0)

bool supported_n(int n) {
  switch (n) {
#define CBS_SUP(N) case N:
    CBS_FOR_EACH_N(CBS_SUP)
#undef CBS_SUP
    return true;
    default:
      return false;
  }
}

const int kSizes[] = {16, 32, 64, 128, 192, 256, 288, 384, 512, 1024};

}  // namespace

cbs_status cbs::report_error(cbs_status st, const std::string& msg) { return fail(st, msg); }

struct cbs_plan_s {
  int batch = 0;
  int dtype = CBS_C64;
  int max_restart = 0;
  int maxn = 0;
  std::map<int, int> ctile;  // column tile width per size class (FP32 kernels)
  int col_threads32 = kThreads;  // threads per FP32 column workgroup (kColThreadsWide: FP32 periodic Helmholtz)
  long long cells = 0;
  std::vector<int> n;
  std::vector<long long> off;
  std::vector<double> k0sq, eps;
  std::vector<InstDesc> inst;
  std::vector<int2> row_items;
  std::vector<int2> col_items32, col_items64;  // column work items per precision
  size_t col_lds32 = 0, col_lds64 = 0;          // dynamic LDS bytes of the column launches

  std::vector<void*> owned;
  InstDesc* d_inst = nullptr;
  int2* d_row_items = nullptr;
  int2* d_col_items32 = nullptr;
  int2* d_col_items64 = nullptr;
  cpx<float>* d_tw32 = nullptr;
  cpx<double>* d_tw64 = nullptr;
  void* d_k2 = nullptr;        // operator precision copy (== d_k2_64 for C128)
  cpx<double>* d_k2_64 = nullptr;
  void* d_inter = nullptr;     // spectral buffer, operator precision
  cpx<double>* d_inter64 = nullptr;
  double* d_partials = nullptr;
  // solver state
  cpx<double>* d_u64 = nullptr;  // FP64 iterate
  cpx<double>* d_s64 = nullptr;  // FP64 source copy (C64 plans) / scratch
  void* d_c = nullptr;           // right-hand side of the correction equation (op. precision)
  void* d_e = nullptr;           // correction iterate (op. precision)
  void* d_t = nullptr;           // scratch (op. precision)
  int* d_status = nullptr;
  int* d_iters = nullptr;
  int* d_chunk_active = nullptr;
  double* d_relres = nullptr;
  double* d_est = nullptr;
  double* d_bnorm = nullptr;
  double* d_bnorm_phys = nullptr;  // ||s|| per instance (physical stop rule)
  double* d_rtol = nullptr;
  double* d_rtol32 = nullptr;      // rtol of the FP32 per-sweep estimate
  double* d_tmp = nullptr;         // 2 x batch per-instance sums (cbs_relres)
  int* d_maxs = nullptr;
  // FGMRES
  cpx<double>* d_vbasis = nullptr;
  void* d_zbasis = nullptr;
  double* d_kry = nullptr;
  long long kry_stride = 0;
  double* d_dots = nullptr;
  double* d_scale = nullptr;
  int* d_kactive = nullptr;
  int* d_kjend = nullptr;

  // Work lists the launches use: the whole batch, or a compacted view holding
  // only the instances still iterating (cbs_iterate switches to it once the
  // running instances cover at most half of the current view's cells).
  // A work list: row items, column items per precision and (for a lane) the
  // instances it covers.
  struct Items {
    const int2* rows = nullptr;
    int nrows = 0;
    const int2* cols32 = nullptr;
    int ncols32 = 0;
    const int2* cols64 = nullptr;
    int ncols64 = 0;
    const int* ids = nullptr;
    int nids = 0;
  };
  struct View {
    int2* rows = nullptr;
    int nrows = 0;
    int2* cols32 = nullptr;
    int ncols32 = 0;
    int2* cols64 = nullptr;
    int ncols64 = 0;
    long long cells = 0;
    int gen = 0;
    // Two lanes of about equal cell count (nlanes == 0: no split).  Their
    // lists live back to back in lrows / lcols32 / lcols64 / lids; the host
    // copies stay alive while the uploads are in flight.
    int nlanes = 0;
    Items lane[2];
    int2* lrows = nullptr;
    int2* lcols32 = nullptr;
    int2* lcols64 = nullptr;
    int* lids = nullptr;
    std::vector<int2> h_rows, h_c32, h_c64;
    std::vector<int> h_ids;
    Items all() const { return Items{rows, nrows, cols32, ncols32, cols64, ncols64, nullptr, 0}; }
  };
  View full, compact;
  View* view = &full;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // (view generation, 2 chunk + stop rule)
  hipStream_t own_stream = nullptr;  // capture stream when the caller passes the null stream
  bool one_stream = false;           // CBS_FLAG_ONE_STREAM
  bool dirichlet = false;            // CBS_FLAG_DIRICHLET: DST-I instances
  bool undamped = false;             // CBS_FLAG_UNDAMPED: eps = 0, no gamma
  bool cdr = false;                  // convection-diffusion-reaction plan (cbs_setup_cdr)
  void* d_k2b = nullptr;             // CDR: (dvx, dvy) per cell, operator precision
  std::vector<double> vx0, vy0;      // CDR background velocity per instance
  double* d_mu = nullptr;            // Dirichlet eigenvalue table (all transform lengths)
  // FFT length that carries an instance of size n
  // length of the 1D transforms along a row or column: the FFT of the odd
  // extension for Dirichlet instances, n itself for the direct DST size
  int tlen(int n) const { return dirichlet ? (n == kDstDirectN ? n : dst_len(n)) : n; }
  hipStream_t lane_st[2] = {nullptr, nullptr};  // non-blocking lane streams
  hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
  int op_elem() const { return dtype == CBS_C64 ? 8 : 16; }
};

namespace {

void build_items(cbs_plan p) {
  p->row_items.clear();
  p->inst.clear();
  int part = 0;
  for (int i = 0; i < p->batch; ++i) {
    InstDesc d{};
    d.off = p->off[i];
    d.n = p->n[i];
    d.k0sq = p->k0sq.empty() ? 0.0 : p->k0sq[i];
    d.eps = p->eps.empty() ? 1.0 : p->eps[i];
    d.kind = p->dirichlet ? KIND_DIRICHLET : (p->cdr ? KIND_CDR : KIND_PERIODIC);
    d.vx0 = p->vx0.empty() ? 0.0 : p->vx0[i];
    d.vy0 = p->vy0.empty() ? 0.0 : p->vy0[i];
    const int m = p->tlen(d.n);
    const int rpw = (p->dirichlet && d.n == kDstDirectN) ? kDstDirectRPW : row_rpw(m);
    d.rpw = rpw;
    d.part_off = part;
    d.nparts = (d.n + rpw - 1) / rpw;
    part += d.nparts;
    auto it = p->ctile.find(d.n);
    d.ctile = it != p->ctile.end() ? it->second : col_tile_start_t(m, p->col_threads32);
    d.ctile64 = d.ctile;
    while (!col_tile_valid(m, d.ctile64, 16) && d.ctile64 > 2) d.ctile64 /= 2;
    p->inst.push_back(d);
  }
  // Largest instances first, so the short tail of the grid holds small items.
  std::vector<int> order(p->batch);
  for (int i = 0; i < p->batch; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->n[a] > p->n[b]; });
  for (int i : order) {
    const int rpw = p->inst[i].rpw;
    for (int r = 0; r < p->n[i]; r += rpw) p->row_items.push_back(int2{i, r});
  }
  // Column items, per instance with its own tile width.  Workgroups are
  // dispatched round-robin over the 8 XCDs (workgroup w runs on XCD w mod 8),
  // so the G = 128 B / (C * element) neighbouring tiles that share cache
  // lines are placed 8 positions apart: they run on the same XCD and hit one
  // L2.  Same-size instances are adjacent, so each size class is a contiguous
  // range of the list.
  p->col_items32.clear();
  p->col_items64.clear();
  p->col_lds32 = p->col_lds64 = 0;
  for (int prec = 0; prec < 2; ++prec) {
    std::vector<int2>& out = prec == 0 ? p->col_items32 : p->col_items64;
    const int elem = prec == 0 ? 8 : 16;
    for (int i : order) {
      const int c = prec == 0 ? p->inst[i].ctile : p->inst[i].ctile64;
      size_t& lds = prec == 0 ? p->col_lds32 : p->col_lds64;
      lds = std::max(lds, size_t(col_lds_elems(p->tlen(p->n[i]), c)) * elem);
      std::vector<int2> nat;
      for (int col = 0; col < p->n[i]; col += c) nat.push_back(int2{i, col});
      const size_t g = std::max(1, 128 / (c * elem)), blk = 8 * g;
      std::vector<int2> items(nat.size());
      size_t b = 0;
      for (; b + blk <= nat.size(); b += blk)
        for (size_t x = 0; x < 8; ++x)
          for (size_t q = 0; q < g; ++q) items[b + 8 * q + x] = nat[b + x * g + q];
      for (; b < nat.size(); ++b) items[b] = nat[b];
      out.insert(out.end(), items.begin(), items.end());
    }
  }
}

// Upper bound on column items (tile width 2 everywhere, the narrowest width
// compiled), for allocation.  An instance of n columns has ceil(n / c) tiles:
// Dirichlet sizes are odd and their last tile is partial.
size_t max_col_items(cbs_plan p) {
  size_t m = 0;
  for (int n : p->n) m += (n + 1) / 2;
  return m;
}

// Capacity of each work-list buffer, in items.
size_t item_capacity(cbs_plan p) { return std::max(max_col_items(p), p->row_items.size()); }

// Every column list a plan can form (any compiled width of any size) fits the
// work-list buffers; checked when the buffers are sized and before uploads.
cbs_status check_item_capacity(cbs_plan p) {
  const size_t cap = item_capacity(p);
  for (int elem : {8, 16}) {
    size_t worst = 0;
    for (int n : p->n) {
      const int m = p->tlen(n);
      size_t most = 0;
      for (int c = 2; c <= 32; c *= 2)
        if (col_tile_valid(m, c, elem)) most = std::max(most, size_t((n + c - 1) / c));
      worst += most;
    }
    if (worst > cap)
      return fail(CBS_ERR_WORKSPACE, "work-list capacity " + std::to_string(cap) + " below " +
                                         std::to_string(worst) + " column tiles");
  }
  if (p->row_items.size() > cap || p->col_items32.size() > cap || p->col_items64.size() > cap)
    return fail(CBS_ERR_WORKSPACE, "work list longer than its buffer");
  return CBS_OK;
}

void set_full_view(cbs_plan p) {
  cbs_plan_s::View& v = p->full;
  v.rows = p->d_row_items;
  v.nrows = int(p->row_items.size());
  v.cols32 = p->d_col_items32;
  v.ncols32 = int(p->col_items32.size());
  v.cols64 = p->d_col_items64;
  v.ncols64 = int(p->col_items64.size());
  v.cells = p->cells;
  v.gen = 0;
}

// Batches smaller than this (or of one instance) run on the caller's stream.
constexpr long long kLaneMinCells = 1LL << 21;

bool lanes_wanted(cbs_plan p, const std::vector<char>& keep) {
  if (p->one_stream) return false;
  int count = 0;
  long long cells = 0;
  for (int i = 0; i < p->batch; ++i)
    if (keep[i]) {
      ++count;
      cells += (long long)p->n[i] * p->n[i];
    }
  return count >= 2 && cells >= kLaneMinCells;
}

// Split the instances flagged in `keep` into two lanes (largest first, each
// to the lane with fewer cells so far) and upload the lanes' lists.  Each
// lane keeps the order of the full lists, so an instance's column tiles stay
// contiguous and tiles that share cache lines stay 8 launch positions apart.
cbs_status build_lanes(cbs_plan p, cbs_plan_s::View& v, const std::vector<char>& keep,
                       hipStream_t st) {
  v.nlanes = 0;
  if (!lanes_wanted(p, keep) || !p->lane_st[0]) return CBS_OK;
  std::vector<int> order;
  for (int i = 0; i < p->batch; ++i)
    if (keep[i]) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->n[a] > p->n[b]; });
  std::vector<int> lane_of(p->batch, -1);
  long long load[2] = {0, 0};
  for (int i : order) {
    const int l = load[1] < load[0] ? 1 : 0;
    lane_of[i] = l;
    load[l] += (long long)p->n[i] * p->n[i];
  }
  const std::vector<int2>& c32 = p->col_items32;
  const std::vector<int2>& c64 = p->col_items64;
  v.h_rows.clear();
  v.h_c32.clear();
  v.h_c64.clear();
  v.h_ids.clear();
  int cnt[2][4] = {};
  for (int l = 0; l < 2; ++l) {
    for (const int2& it : p->row_items)
      if (lane_of[it.x] == l) { v.h_rows.push_back(it); ++cnt[l][0]; }
    for (const int2& it : c32)
      if (lane_of[it.x] == l) { v.h_c32.push_back(it); ++cnt[l][1]; }
    for (const int2& it : c64)
      if (lane_of[it.x] == l) { v.h_c64.push_back(it); ++cnt[l][2]; }
    for (int i = 0; i < p->batch; ++i)
      if (lane_of[i] == l) { v.h_ids.push_back(i); ++cnt[l][3]; }
  }
  HIPCHK(hipMemcpyAsync(v.lrows, v.h_rows.data(), v.h_rows.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(v.lcols32, v.h_c32.data(), v.h_c32.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(v.lcols64, v.h_c64.data(), v.h_c64.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(v.lids, v.h_ids.data(), v.h_ids.size() * sizeof(int), hipMemcpyHostToDevice, st));
  for (int l = 0; l < 2; ++l) {
    const int o0 = l ? cnt[0][0] : 0, o1 = l ? cnt[0][1] : 0, o2 = l ? cnt[0][2] : 0,
              o3 = l ? cnt[0][3] : 0;
    v.lane[l] = cbs_plan_s::Items{v.lrows + o0, cnt[l][0], v.lcols32 + o1, cnt[l][1],
                                  v.lcols64 + o2, cnt[l][2], v.lids + o3, cnt[l][3]};
  }
  v.nlanes = 2;
  return CBS_OK;
}

// Compacted view over the instances flagged in `keep` (whole instances, so
// the per-instance XCD grouping of the column tiles is preserved).
cbs_status build_compact_view(cbs_plan p, const std::vector<char>& keep, hipStream_t st) {
  std::vector<int2> rows, c32, c64;
  for (const int2& it : p->row_items)
    if (keep[it.x]) rows.push_back(it);
  for (const int2& it : p->col_items32)
    if (keep[it.x]) c32.push_back(it);
  for (const int2& it : p->col_items64)
    if (keep[it.x]) c64.push_back(it);
  cbs_plan_s::View& v = p->compact;
  HIPCHK(hipMemcpyAsync(v.rows, rows.data(), rows.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(v.cols32, c32.data(), c32.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(v.cols64, c64.data(), c64.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  CHK(build_lanes(p, v, keep, st));
  HIPCHK(hipStreamSynchronize(st));
  v.nrows = int(rows.size());
  v.ncols32 = int(c32.size());
  v.ncols64 = int(c64.size());
  v.cells = 0;
  for (int i = 0; i < p->batch; ++i)
    if (keep[i]) v.cells += (long long)p->n[i] * p->n[i];
  // graphs captured on the previous compacted lists are stale
  for (auto it = p->graphs.begin(); it != p->graphs.end();) {
    if (it->first.first == v.gen) {
      hipGraphExecDestroy(it->second);
      it = p->graphs.erase(it);
    } else {
      ++it;
    }
  }
  v.gen += 1;
  p->view = &v;
  return CBS_OK;
}

cbs_status upload_items(cbs_plan p, hipStream_t st) {
  CHK(check_item_capacity(p));
  set_full_view(p);
  CHK(build_lanes(p, p->full, std::vector<char>(p->batch, 1), st));
  HIPCHK(hipMemcpyAsync(p->d_inst, p->inst.data(), p->inst.size() * sizeof(InstDesc),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->d_col_items32, p->col_items32.data(), p->col_items32.size() * sizeof(int2),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->d_col_items64, p->col_items64.data(), p->col_items64.size() * sizeof(int2),
                        hipMemcpyHostToDevice, st));
  return CBS_OK;
}

template <typename R>
const cpx<R>* k2_of(cbs_plan p) {
  return static_cast<const cpx<R>*>(sizeof(R) == 4 ? p->d_k2 : static_cast<void*>(p->d_k2_64));
}
template <typename R>
cpx<R>* inter_of(cbs_plan p) {
  return static_cast<cpx<R>*>(sizeof(R) == 4 ? p->d_inter : static_cast<void*>(p->d_inter64));
}

template <typename R>
Params<R> base_params(cbs_plan p) {
  Params<R> q{};
  q.inst = p->d_inst;
  q.k2 = k2_of<R>(p);
  q.inter = inter_of<R>(p);
  if constexpr (sizeof(R) == 4) q.tw = p->d_tw32;
  else q.tw = p->d_tw64;
  q.partials = p->d_partials;
  q.mask = nullptr;
  q.mask_mode = MASK_RUNNING;
  q.pro = PRO_VU_S;
  q.sym = SYM_GREEN;
  q.epi = EPI_STORE;
  q.dst = p->dirichlet ? 1 : 0;
  q.mu = p->d_mu;
  q.col_threads = sizeof(R) == 4 ? p->col_threads32 : kThreads;
  return q;
}

template <typename R>
void launch_cols(cbs_plan p, Params<R> q, hipStream_t st, const cbs_plan_s::Items& it) {
  if constexpr (sizeof(R) == 4) {
    q.items = it.cols32;
    launch_col(it.ncols32, p->col_lds32, st, q);
  } else {
    q.items = it.cols64;
    launch_col(it.ncols64, p->col_lds64, st, q);
  }
}
template <typename R>
void launch_cols(cbs_plan p, Params<R> q, hipStream_t st) {
  launch_cols(p, q, st, p->view->all());
}

// Fork the two lane streams off `st` / join them back into it (stream
// ordered, also under graph capture).
cbs_status lanes_fork(cbs_plan p, hipStream_t st) {
  HIPCHK(hipEventRecord(p->ev_fork, st));
  for (int l = 0; l < 2; ++l) HIPCHK(hipStreamWaitEvent(p->lane_st[l], p->ev_fork, 0));
  return CBS_OK;
}
cbs_status lanes_join(cbs_plan p, hipStream_t st) {
  for (int l = 0; l < 2; ++l) {
    HIPCHK(hipEventRecord(p->ev_join[l], p->lane_st[l]));
    HIPCHK(hipStreamWaitEvent(st, p->ev_join[l], 0));
  }
  return CBS_OK;
}

// Forward rows (prologue) -> columns (symbol) -> inverse rows (epilogue).
template <typename R>
cbs_status run_pipeline(cbs_plan p, Params<R> q, hipStream_t st) {
  const int nrow = p->view->nrows;
  q.items = p->view->rows;
  launch_row(0, nrow, st, q);
  launch_cols(p, q, st);
  launch_row(1, nrow, st, q);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// Issue a chain of `steps` launch groups, step(k, stream, items), on the
// view's lanes (between a fork and a join) or on `st` alone.  The lanes'
// launches alternate step by step: queued lane by lane, the second lane's
// first kernel would wait behind the host-side issue of the first lane's
// whole chain (also when a graph replays the chain in capture order).
template <typename F>
cbs_status issue_chain(cbs_plan p, hipStream_t st, int steps, F&& step) {
  const cbs_plan_s::View& v = *p->view;
  if (v.nlanes) {
    CHK(lanes_fork(p, st));
    for (int k = 0; k < steps; ++k)
      for (int l = 0; l < v.nlanes; ++l) step(k, p->lane_st[l], v.lane[l]);
    HIPCHK(hipGetLastError());
    return lanes_join(p, st);
  }
  const cbs_plan_s::Items all = v.all();
  for (int k = 0; k < steps; ++k) step(k, st, all);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// `count` CBS sweeps in place on q.u (= q.out), as count + 1 steps: forward
// rows, then (count - 1) times [columns, fused inverse/forward rows], then
// columns and inverse rows with the sweep epilogue.  The partial norms left
// behind are those of the last sweep.
template <typename R>
cbs_status run_sweeps(cbs_plan p, Params<R> q, int count, hipStream_t st) {
  // the fused sweep kernel reads rhs or s, not both
  if (q.rhs && q.s) return fail(CBS_ERR_ARG, "a fused sweep takes rhs or s, not both");
  return issue_chain(p, st, count + 1, [&](int k, hipStream_t ls, const cbs_plan_s::Items& it) {
    Params<R> f = q;
    f.items = it.rows;
    if (k == 0) {
      launch_row(0, it.nrows, ls, f);
      return;
    }
    launch_cols(p, q, ls, it);
    if (k < count) {
      launch_row(2, it.nrows, ls, f);
    } else {
      f.epi = EPI_SWEEP;
      launch_row(1, it.nrows, ls, f);
    }
  });
}

template <typename R>
cbs_status launch_pw(cbs_plan p, PwParams<R> w, hipStream_t st) {
  w.inst = p->d_inst;
  w.items = p->view->rows;
  w.k2 = k2_of<R>(p);
  launch_pointwise(p->view->nrows, st, w);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

IterState iter_state(cbs_plan p) {
  IterState s{};
  s.status = p->d_status;
  s.iters = p->d_iters;
  s.chunk_active = p->d_chunk_active;
  s.relres = p->d_relres;
  s.est = p->d_est;
  s.bnorm = p->d_bnorm;
  s.rtol = p->d_rtol;
  s.max_sweeps = p->d_maxs;
  return s;
}

cbs_status compute_stats(cbs_plan p, int phase, hipStream_t st, std::vector<double>& a,
                         std::vector<double>& b) {
  HIPCHK(hipMemcpyAsync(p->d_inst, p->inst.data(), p->inst.size() * sizeof(InstDesc),
                        hipMemcpyHostToDevice, st));
  launch_stats(int(p->row_items.size()), st, p->d_inst, p->d_row_items, p->d_k2_64, p->d_partials,
               phase);
  HIPCHK(hipGetLastError());
  std::vector<double> part(2 * p->row_items.size());
  HIPCHK(hipMemcpyAsync(part.data(), p->d_partials, part.size() * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  a.assign(p->batch, 0.0);
  b.assign(p->batch, 0.0);
  for (int i = 0; i < p->batch; ++i) {
    const InstDesc& d = p->inst[i];
    double va = part[2 * d.part_off], vb = part[2 * d.part_off + 1];
    for (int k = 1; k < d.nparts; ++k) {
      const double xa = part[2 * (d.part_off + k)], xb = part[2 * (d.part_off + k) + 1];
      va = (phase == 1) ? std::max(va, xa) : std::min(va, xa);
      vb = std::max(vb, xb);
    }
    a[i] = va;
    b[i] = vb;
  }
  return CBS_OK;
}

void drop_graphs(cbs_plan p) {
  for (auto& kv : p->graphs) hipGraphExecDestroy(kv.second);
  p->graphs.clear();
}

void free_plan(cbs_plan p) {
  drop_graphs(p);
  if (p->own_stream) {
    (void)hipStreamSynchronize(p->own_stream);
    (void)hipStreamDestroy(p->own_stream);
  }
  p->own_stream = nullptr;
  for (int l = 0; l < 2; ++l) {
    // the lanes may still run this plan's kernels: finish them before the
    // plan's memory (or the caller's workspace) can be reused
    if (p->lane_st[l]) {
      (void)hipStreamSynchronize(p->lane_st[l]);
      (void)hipStreamDestroy(p->lane_st[l]);
    }
    if (p->ev_join[l]) hipEventDestroy(p->ev_join[l]);
    p->lane_st[l] = nullptr;
    p->ev_join[l] = nullptr;
  }
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  p->ev_fork = nullptr;
  for (void* q : p->owned) hipFree(q);
  p->owned.clear();
}

// ---- generic entry helpers -------------------------------------------------------------

template <typename R>
cbs_status residual_impl(cbs_plan p, const void* u, const void* s, const void* rhs, void* r,
                         double* norm2, hipStream_t st) {
  Params<R> q = base_params<R>(p);
  q.u = static_cast<const cpx<R>*>(u);
  q.s = static_cast<const cpx<R>*>(s);
  q.rhs = static_cast<const cpx<R>*>(rhs);
  q.out = static_cast<cpx<R>*>(r);
  q.epi = EPI_RESID;
  CHK(run_pipeline(p, q, st));
  if (norm2) {
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, norm2);
    HIPCHK(hipGetLastError());
  }
  return CBS_OK;
}

template <typename R>
cbs_status sweep_impl(cbs_plan p, void* u, const void* s, int count, double* norm2, hipStream_t st) {
  Params<R> q = base_params<R>(p);
  q.u = static_cast<const cpx<R>*>(u);
  q.s = static_cast<const cpx<R>*>(s);
  q.out = static_cast<cpx<R>*>(u);
  q.epi = EPI_SWEEP;
  CHK(run_sweeps(p, q, count, st));
  if (norm2) {
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, norm2);
    HIPCHK(hipGetLastError());
  }
  return CBS_OK;
}

// `count` sweeps from field 0 of u_all, iterate k into field k: the chain of
// run_sweeps with the update of step k reading field k - 1 and writing field k.
template <typename R>
cbs_status sweep_ckpt_impl(cbs_plan p, void* u_all, const void* s, int count, hipStream_t st) {
  cpx<R>* f = static_cast<cpx<R>*>(u_all);
  const long long cells = p->cells;
  Params<R> q = base_params<R>(p);
  q.s = static_cast<const cpx<R>*>(s);
  q.epi = EPI_SWEEP;
  q.partials = nullptr;
  return issue_chain(p, st, count + 1, [&](int k, hipStream_t ls, const cbs_plan_s::Items& it) {
    Params<R> c = q;
    c.items = it.rows;
    if (k == 0) {
      c.u = f;
      launch_row(0, it.nrows, ls, c);
      return;
    }
    c.u = f + (long long)(k - 1) * cells;
    c.out = f + (long long)k * cells;
    launch_cols(p, c, ls, it);
    launch_row(k < count ? 2 : 1, it.nrows, ls, c);
  });
}

// The FP64 residual of the FP64 iterate (narrowed into c) and the status
// decision of every instance not yet final.
template <typename R>
cbs_status enqueue_check(cbs_plan p, int stop, hipStream_t st) {
  IterState is = iter_state(p);
  cpx<R>* c = static_cast<cpx<R>*>(p->d_c);
  {
    Params<double> q = base_params<double>(p);
    q.u = p->d_u64;
    q.s = p->d_s64;
    q.epi = EPI_RESID;
    if constexpr (sizeof(R) == 4) q.out_narrow = reinterpret_cast<cpx<float>*>(c);
    else q.out = reinterpret_cast<cpx<double>*>(c);
    q.mask = p->d_status;
    q.mask_mode = MASK_NOT_FINAL;
    CHK(run_pipeline(p, q, st));
    if (stop == CBS_STOP_PHYSICAL) {
      // the decision uses the physical residual s - A u64 instead
      Params<double> h = base_params<double>(p);
      h.u = p->d_u64;
      h.s = p->d_s64;
      h.pro = PRO_U;
      h.sym = SYM_LAP;
      h.epi = EPI_LAP;
      h.mask = p->d_status;
      h.mask_mode = MASK_NOT_FINAL;
      CHK(run_pipeline(p, h, st));
      IterState ip = is;
      ip.bnorm = p->d_bnorm_phys;
      launch_check64(p->batch, st, ip, p->d_inst, p->d_partials);
    } else {
      launch_check64(p->batch, st, is, p->d_inst, p->d_partials);
    }
  }
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// One refinement chunk of stationary CBS:
//   r64 = G(V u64 + s64) - u64 (FP64; narrowed into c), status check in FP64,
//   e = gamma c, (chunk - 1) sweeps e <- e + gamma (G(V e) + c - e) in the
//   operator precision with a per-sweep norm estimate, then u64 += e.
// In exact arithmetic this is exactly `chunk` CBS sweeps from u64.
template <typename R>
cbs_status enqueue_chunk(cbs_plan p, int chunk, int stop, hipStream_t st) {
  IterState is = iter_state(p);
  cpx<R>* c = static_cast<cpx<R>*>(p->d_c);
  cpx<R>* e = static_cast<cpx<R>*>(p->d_e);
  CHK(enqueue_check<R>(p, stop, st));
  // The FP32 estimate of each sweep stops an instance early only under the
  // Born rule (it estimates the Born residual); it always counts the sweep.
  is.rtol = p->d_rtol32;
  {
    PwParams<R> w{};
    w.op = PW_GAMMA;
    w.e_in = c;
    w.e_out = e;
    w.mask = p->d_status;
    w.mask_mode = MASK_RUNNING;
    CHK(launch_pw(p, w, st));
  }
  // (chunk - 1) sweeps e <- e + gamma (G(V e) + c - e); the status check after
  // each sweep runs between the fused kernels (a converged instance is masked
  // from the next launch on).
  if (chunk > 1) {
    Params<R> q = base_params<R>(p);
    q.u = e;
    q.rhs = c;  // and no s: the fused sweep kernel reads one of the two
    q.out = e;
    q.epi = EPI_SWEEP;
    q.mask = p->d_status;
    q.mask_mode = MASK_RUNNING;
    // The check of each sweep runs in the next column launch (its first
    // tiles' workgroups); the last sweep's check is a launch of its own.
    // Each lane checks only its own instances, so the lanes never wait on
    // each other inside the chunk.
    q.chk = is;
    const bool lanes = p->view->nlanes != 0;
    CHK(issue_chain(p, st, chunk + 1, [&](int k, hipStream_t ls, const cbs_plan_s::Items& it) {
      Params<R> c = q;
      c.items = it.rows;
      if (k == 0) {
        launch_row(0, it.nrows, ls, c);
      } else if (k < chunk) {
        c.check = k >= 2 ? 1 : 0;
        launch_cols(p, c, ls, it);
        c.check = 0;
        launch_row(k + 1 < chunk ? 2 : 1, it.nrows, ls, c);
      } else if (lanes) {
        launch_check32(it.nids, it.ids, ls, is, p->d_inst, p->d_partials);
      } else {
        launch_check32(p->batch, nullptr, ls, is, p->d_inst, p->d_partials);
      }
    }));
  }
  {
    PwParams<R> w{};
    w.op = PW_ADD_WIDE;
    w.e_in = e;
    w.x64 = p->d_u64;
    w.mask = p->d_chunk_active;
    w.mask_mode = MASK_NONZERO;
    CHK(launch_pw(p, w, st));
  }
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

template <typename R>
cbs_status relres_impl(cbs_plan p, const void* u, const void* s, int stop, double* relres, hipStream_t st);

// FP32 plans hand back the FP64 iterate rounded to FP32.  The relative
// residual reported is that of the returned field, evaluated in FP64 (the
// FP64 iterate's own residual decided the status): rounding can move it by
// about 1e-7 times the conditioning of the problem.
template <typename R>
cbs_status report_returned(cbs_plan p, const void* u, int stop, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    launch_widen_all(st, static_cast<const cpx<float>*>(u), p->d_u64, p->cells);
    HIPCHK(hipGetLastError());
    return relres_impl<double>(p, p->d_u64, p->d_s64, stop, p->d_relres, st);
  }
  return CBS_OK;
}

struct FullViewOnExit {
  cbs_plan p;
  ~FullViewOnExit() { p->view = &p->full; }
};

template <typename R>
cbs_status iterate_impl(cbs_plan p, void* u, const void* s, int max_sweeps, double rtol,
                        int chunk, int stop, int32_t* iters, double* relres, int32_t* status,
                        int use_graph, hipStream_t st) {
  const int B = p->batch;
  p->view = &p->full;
  FullViewOnExit restore{p};
  // u64 <- u ; s64 <- s
  if constexpr (sizeof(R) == 4) {
    launch_widen_all(st, static_cast<const cpx<float>*>(u), p->d_u64, p->cells);
    launch_widen_all(st, static_cast<const cpx<float>*>(s), p->d_s64, p->cells);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpyAsync(p->d_u64, u, p->cells * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_s64, s, p->cells * 16, hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipMemsetAsync(p->d_status, 0, B * sizeof(int), st));
  HIPCHK(hipMemsetAsync(p->d_iters, 0, B * sizeof(int), st));
  HIPCHK(hipMemcpyAsync(p->d_rtol, &rtol, sizeof(double), hipMemcpyHostToDevice, st));
  const double rtol32 = stop == CBS_STOP_PHYSICAL ? 0.0 : rtol;
  HIPCHK(hipMemcpyAsync(p->d_rtol32, &rtol32, sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->d_maxs, &max_sweeps, sizeof(int), hipMemcpyHostToDevice, st));
  // ||G s|| in FP64
  {
    Params<double> q = base_params<double>(p);
    q.s = p->d_s64;
    q.epi = EPI_RESID;
    CHK(run_pipeline(p, q, st));
    launch_set_bnorm(B, st, iter_state(p), p->d_inst, p->d_partials);
    HIPCHK(hipGetLastError());
  }
  // ||s|| in FP64 (s - A 0 through the physical-residual pipeline)
  if (stop == CBS_STOP_PHYSICAL) {
    Params<double> q = base_params<double>(p);
    q.s = p->d_s64;
    q.pro = PRO_U;
    q.sym = SYM_LAP;
    q.epi = EPI_LAP;
    CHK(run_pipeline(p, q, st));
    IterState ip = iter_state(p);
    ip.bnorm = p->d_bnorm_phys;
    launch_set_bnorm(B, st, ip, p->d_inst, p->d_partials);
    HIPCHK(hipGetLastError());
  }
  // Capture (once per view and chunk length) and replay.
  auto get_graph = [&](hipGraphExec_t* exec) -> cbs_status {
    *exec = nullptr;
    if (!use_graph) return CBS_OK;
    const auto key = std::make_pair(p->view->gen, 2 * chunk + stop);
    auto it = p->graphs.find(key);
    if (it != p->graphs.end()) {
      *exec = it->second;
      return CBS_OK;
    }
    HIPCHK(hipStreamSynchronize(st));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    cbs_status rc = enqueue_chunk<R>(p, chunk, stop, st);
    hipError_t ce = hipStreamEndCapture(st, &g);
    if (rc != CBS_OK) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (ce != hipSuccess) return fail(CBS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(CBS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    p->graphs[key] = *exec;
    return CBS_OK;
  };
  hipGraphExec_t exec = nullptr;
  CHK(get_graph(&exec));
  std::vector<int> hstat(B);
  std::vector<char> keep(B);
  const long long max_chunks = (long long)max_sweeps / std::max(1, chunk) + 3;
  for (long long ch = 0; ch <= max_chunks; ++ch) {
    if (exec) HIPCHK(hipGraphLaunch(exec, st));
    else CHK(enqueue_chunk<R>(p, chunk, stop, st));
    HIPCHK(hipMemcpyAsync(hstat.data(), p->d_status, B * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    long long active_cells = 0;
    for (int i = 0; i < B; ++i) {
      keep[i] = hstat[i] == ST_RUNNING || hstat[i] == ST_PENDING;
      if (keep[i]) active_cells += (long long)p->n[i] * p->n[i];
    }
    if (active_cells == 0) break;
    // Compact the work lists once the running instances cover at most half
    // of the current view: later launches then dispatch only their items.
    if (2 * active_cells <= p->view->cells) {
      CHK(build_compact_view(p, keep, st));
      CHK(get_graph(&exec));
    }
  }
  p->view = &p->full;
  // u <- u64
  if constexpr (sizeof(R) == 4) {
    PwParams<float> w{};
    w.op = PW_NARROW;
    w.x64 = p->d_u64;
    w.e_out = static_cast<cpx<float>*>(u);
    CHK(launch_pw(p, w, st));
  } else {
    HIPCHK(hipMemcpyAsync(u, p->d_u64, p->cells * 16, hipMemcpyDeviceToDevice, st));
  }
  CHK(report_returned<R>(p, u, stop, st));
  std::vector<int> hit(B);
  std::vector<double> hrel(B);
  HIPCHK(hipMemcpyAsync(hit.data(), p->d_iters, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hrel.data(), p->d_relres, B * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hstat.data(), p->d_status, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool all = true;
  for (int i = 0; i < B; ++i) {
    if (iters) iters[i] = hit[i];
    if (relres) relres[i] = hrel[i];
    if (status) status[i] = hstat[i];
    if (hstat[i] != ST_CONVERGED) all = false;
  }
  if (!all) {
    g_err = "at least one instance did not reach rtol";
    return CBS_NOT_CONVERGED;
  }
  return CBS_OK;
}

// ---- FGMRES ---------------------------------------------------------------------------------

KryParams kry_params(cbs_plan p, int m) {
  KryParams k{};
  k.inst = p->d_inst;
  k.items = p->d_row_items;
  k.vbasis = p->d_vbasis;
  k.cells = p->cells;
  k.kry = p->d_kry;
  k.kstride = p->kry_stride;
  k.m = m;
  k.dots = p->d_dots;
  k.dstride = 4LL * (m + 1) + 4;
  k.partials = p->d_partials;
  k.scale = p->d_scale;
  k.active = p->d_kactive;
  k.jend = p->d_kjend;
  k.iters = p->d_iters;
  k.status = p->d_status;
  k.relres = p->d_relres;
  k.rtol = p->d_rtol;
  k.max_iters = p->d_maxs;
  return k;
}

// True residual r = G(V x + s) - x in FP64 into v_0, then the restart decision.
cbs_status fg_restart(cbs_plan p, int m, int first, hipStream_t st) {
  Params<double> q = base_params<double>(p);
  if (!first) q.u = p->d_u64;
  q.s = p->d_s64;
  q.epi = EPI_RESID;
  q.out = first ? nullptr : p->d_vbasis;
  q.mask = p->d_status;
  q.mask_mode = MASK_RUNNING;
  CHK(run_pipeline(p, q, st));
  KryParams k = kry_params(p, m);
  launch_fg_restart(p->batch, st, k, first);
  HIPCHK(hipGetLastError());
  if (!first) {
    PwParams<double> w{};
    w.op = PW_SCALE64;
    w.x64 = p->d_vbasis;
    w.scale = p->d_scale;
    w.mask = p->d_kactive;
    w.mask_mode = MASK_NONZERO;
    CHK(launch_pw(p, w, st));
  }
  return CBS_OK;
}

// One Arnoldi step j for every active instance (Gram-Schmidt with delayed
// reorthogonalisation: slot j holds u_j, the next vector after one pass).
template <typename R>
cbs_status fg_step(cbs_plan p, int m, int j, int sweeps, hipStream_t st) {
  cpx<R>* z = static_cast<cpx<R>*>(p->d_zbasis) + (long long)j * p->cells;
  cpx<R>* c = static_cast<cpx<R>*>(p->d_c);
  cpx<double>* w = p->d_vbasis + (long long)(j + 1) * p->cells;
  // z_j = P_K(u_j / ||u_j||) (u_0 = v_0 is normalised): first sweep from zero
  // is z = gamma v, then K-1 full sweeps; K = 0 is no inner preconditioner
  {
    PwParams<R> pw{};
    if (sweeps == 0) {
      pw.op = PW_NARROW;
      pw.x64 = p->d_vbasis + (long long)j * p->cells;
    } else {
      pw.op = PW_FIRST64;
      pw.src64 = p->d_vbasis + (long long)j * p->cells;
      pw.c_out = c;
    }
    pw.scale = j > 0 ? p->d_scale : nullptr;
    pw.e_out = z;
    pw.mask = p->d_kactive;
    pw.mask_mode = MASK_NONZERO;
    CHK(launch_pw(p, pw, st));
  }
  if (sweeps > 1) {
    Params<R> q = base_params<R>(p);
    q.u = z;
    q.rhs = c;
    q.out = z;
    q.epi = EPI_SWEEP;
    q.partials = nullptr;
    q.mask = p->d_kactive;
    q.mask_mode = MASK_NONZERO;
    CHK(run_sweeps(p, q, sweeps - 1, st));
  }
  // w = B z_j = z_j - G(V z_j), widened to FP64
  {
    Params<R> q = base_params<R>(p);
    q.u = z;
    q.epi = EPI_BZ_WIDE;
    q.out_wide = w;
    q.partials = nullptr;
    q.mask = p->d_kactive;
    q.mask_mode = MASK_NONZERO;
    CHK(run_pipeline(p, q, st));
  }
  KryParams k = kry_params(p, m);
  k.j = j;
  const int nrow = int(p->row_items.size());
  launch_gs_dots(nrow, false, st, k);
  launch_gs_finish(p->batch, false, st, k);
  launch_gs_update(nrow, st, k);
  launch_gs_check(p->batch, st, k);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// End of a cycle: reorthogonalise u_jend of every instance that ran steps,
// finalise its last Hessenberg column, solve the small least-squares
// problem and add Z y to the FP64 iterate.
template <typename R>
cbs_status fg_cycle_end(cbs_plan p, int m, hipStream_t st) {
  KryParams k = kry_params(p, m);
  launch_gs_dots(int(p->row_items.size()), true, st, k);
  launch_gs_finish(p->batch, true, st, k);
  launch_backsolve(p->batch, st, k);
  launch_zupdate(int(p->row_items.size()), st, k, static_cast<const cpx<R>*>(p->d_zbasis), p->d_u64);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

template <typename R>
cbs_status fgmres_impl(cbs_plan p, void* u, const void* s, int m, int sweeps, int max_iters,
                       double rtol, int32_t* iters, double* relres, int32_t* status,
                       hipStream_t st) {
  const int B = p->batch;
  if constexpr (sizeof(R) == 4) {
    launch_widen_all(st, static_cast<const cpx<float>*>(u), p->d_u64, p->cells);
    launch_widen_all(st, static_cast<const cpx<float>*>(s), p->d_s64, p->cells);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpyAsync(p->d_u64, u, p->cells * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_s64, s, p->cells * 16, hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipMemsetAsync(p->d_status, 0, B * sizeof(int), st));
  HIPCHK(hipMemsetAsync(p->d_iters, 0, B * sizeof(int), st));
  HIPCHK(hipMemsetAsync(p->d_kjend, 0, B * sizeof(int), st));
  HIPCHK(hipMemcpyAsync(p->d_rtol, &rtol, sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->d_maxs, &max_iters, sizeof(int), hipMemcpyHostToDevice, st));
  CHK(fg_restart(p, m, 1, st));
  std::vector<int> hact(B), hstat(B);
  for (int cycle = 0; cycle < max_iters + 2; ++cycle) {
    CHK(fg_restart(p, m, 0, st));
    HIPCHK(hipMemcpyAsync(hstat.data(), p->d_status, B * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool any = false;
    for (int i = 0; i < B; ++i) any |= hstat[i] == ST_RUNNING;
    if (!any) break;
    for (int j = 0; j < m; ++j) {
      CHK(fg_step<R>(p, m, j, sweeps, st));
      HIPCHK(hipMemcpyAsync(hact.data(), p->d_kactive, B * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool act = false;
      for (int i = 0; i < B; ++i) act |= hact[i] != 0;
      if (!act) break;
    }
    CHK(fg_cycle_end<R>(p, m, st));
  }
  if constexpr (sizeof(R) == 4) {
    PwParams<float> w{};
    w.op = PW_NARROW;
    w.x64 = p->d_u64;
    w.e_out = static_cast<cpx<float>*>(u);
    CHK(launch_pw(p, w, st));
  } else {
    HIPCHK(hipMemcpyAsync(u, p->d_u64, p->cells * 16, hipMemcpyDeviceToDevice, st));
  }
  CHK(report_returned<R>(p, u, CBS_STOP_BORN, st));
  std::vector<int> hit(B);
  std::vector<double> hrel(B);
  HIPCHK(hipMemcpyAsync(hit.data(), p->d_iters, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hrel.data(), p->d_relres, B * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hstat.data(), p->d_status, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool all = true;
  for (int i = 0; i < B; ++i) {
    if (iters) iters[i] = hit[i];
    if (relres) relres[i] = hrel[i];
    if (status) status[i] = hstat[i] == ST_RUNNING ? ST_MAXIT : hstat[i];
    if (hstat[i] != ST_CONVERGED) all = false;
  }
  if (!all) {
    g_err = "at least one instance did not reach rtol";
    return CBS_NOT_CONVERGED;
  }
  return CBS_OK;
}

// ---- stream-ordered solvers ----------------------------------------------------------------
//
// The same chunks and Arnoldi steps as the host-driven loops above, enqueued
// for a fixed budget without any host synchronisation, so a caller can
// overlap a solve with other work or capture it into a graph.  Instances
// that finish early are masked out of every later launch (their workgroups
// return at once); there is no compaction of the work lists.

template <typename R>
cbs_status solver_load(cbs_plan p, const void* u, const void* s, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    launch_widen_all(st, static_cast<const cpx<float>*>(u), p->d_u64, p->cells);
    launch_widen_all(st, static_cast<const cpx<float>*>(s), p->d_s64, p->cells);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpyAsync(p->d_u64, u, p->cells * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p->d_s64, s, p->cells * 16, hipMemcpyDeviceToDevice, st));
  }
  return CBS_OK;
}

template <typename R>
cbs_status solver_store(cbs_plan p, void* u, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    PwParams<float> w{};
    w.op = PW_NARROW;
    w.x64 = p->d_u64;
    w.e_out = static_cast<cpx<float>*>(u);
    return launch_pw(p, w, st);
  } else {
    HIPCHK(hipMemcpyAsync(u, p->d_u64, p->cells * 16, hipMemcpyDeviceToDevice, st));
    return CBS_OK;
  }
}

template <typename R>
cbs_status iterate_async_impl(cbs_plan p, void* u, const void* s, int max_sweeps, double rtol, int chunk,
                              int stop, int32_t* iters, double* relres, int32_t* status, hipStream_t st) {
  const int B = p->batch;
  p->view = &p->full;
  FullViewOnExit restore{p};
  CHK(solver_load<R>(p, u, s, st));
  launch_solver_init(st, p->d_status, p->d_iters, p->d_relres, nullptr, p->d_rtol, p->d_rtol32, p->d_maxs, B,
                     rtol, stop == CBS_STOP_PHYSICAL ? 0.0 : rtol, max_sweeps);
  {
    Params<double> q = base_params<double>(p);
    q.s = p->d_s64;
    q.epi = EPI_RESID;
    CHK(run_pipeline(p, q, st));
    launch_set_bnorm(B, st, iter_state(p), p->d_inst, p->d_partials);
  }
  if (stop == CBS_STOP_PHYSICAL) {
    Params<double> q = base_params<double>(p);
    q.s = p->d_s64;
    q.pro = PRO_U;
    q.sym = SYM_LAP;
    q.epi = EPI_LAP;
    CHK(run_pipeline(p, q, st));
    IterState ip = iter_state(p);
    ip.bnorm = p->d_bnorm_phys;
    launch_set_bnorm(B, st, ip, p->d_inst, p->d_partials);
  }
  // ceil(max_sweeps / chunk) chunks bring every instance to a final status
  // or to its sweep cap; one more chunk start and a last check confirm them
  const long long nchunks = ((long long)max_sweeps + chunk - 1) / chunk + 1;
  for (long long c = 0; c < nchunks; ++c) CHK(enqueue_chunk<R>(p, chunk, stop, st));
  CHK(enqueue_check<R>(p, stop, st));
  CHK(solver_store<R>(p, u, st));
  CHK(report_returned<R>(p, u, stop, st));
  launch_solver_out(st, iter_state(p), B, iters, relres, status);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

template <typename R>
cbs_status fgmres_async_impl(cbs_plan p, void* u, const void* s, int m, int sweeps, int max_iters,
                             double rtol, int32_t* iters, double* relres, int32_t* status, hipStream_t st) {
  const int B = p->batch;
  p->view = &p->full;
  FullViewOnExit restore{p};
  CHK(solver_load<R>(p, u, s, st));
  launch_solver_init(st, p->d_status, p->d_iters, p->d_relres, p->d_kjend, p->d_rtol, nullptr, p->d_maxs, B,
                     rtol, 0.0, max_iters);
  CHK(fg_restart(p, m, 1, st));
  const long long ncycles = ((long long)max_iters + m - 1) / m + 1;
  for (long long cycle = 0; cycle < ncycles; ++cycle) {
    CHK(fg_restart(p, m, 0, st));
    for (int j = 0; j < m; ++j) CHK(fg_step<R>(p, m, j, sweeps, st));
    CHK(fg_cycle_end<R>(p, m, st));
  }
  CHK(fg_restart(p, m, 0, st));  // true residual of the last update decides the status
  CHK(solver_store<R>(p, u, st));
  CHK(report_returned<R>(p, u, CBS_STOP_BORN, st));
  launch_solver_out(st, iter_state(p), B, iters, relres, status);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// ---- NPBS step with a linear Fourier layer ------------------------------------------------

// count steps u <- u + F^-1(wf F r) + wloc r, r = G(V u + s) - u.  Periodic
// plans run them as one chain per lane: forward rows of V u + s, then per
// step [Green columns, rows r = z - u -> forward rows of r, layer columns
// (tabulated weights), rows u += z + wloc r -> forward rows of V u + s];
// the last step ends with inverse rows and the update.  Dirichlet plans run
// the residual pipeline and the layer's pipeline one after the other.
template <typename R>
void npbs_step(cbs_plan p, const Params<R>& base, int count, int k, hipStream_t st,
               const cbs_plan_s::Items& it) {
  Params<R> g = base;
  g.items = it.rows;
  if (k == 0) {
    launch_row(0, it.nrows, st, g);          // V u + s -> forward rows
    return;
  }
  Params<R> m = base;
  m.sym = SYM_TABLE;
  m.items = it.rows;
  launch_cols(p, base, st, it);              // Green
  launch_row(3, it.nrows, st, g);            // r = z - u -> forward rows of r
  launch_cols(p, m, st, it);                 // layer's spectral weights
  if (k < count) {
    launch_row(4, it.nrows, st, m);          // u += z + wloc r -> forward rows of V u + s
  } else {
    m.epi = EPI_NPBS;
    launch_row(1, it.nrows, st, m);          // u += z + wloc r
  }
}

template <typename R>
cbs_status npbs_impl(cbs_plan p, void* u, const void* s, const void* wf, const void* wloc,
                     int count, hipStream_t st) {
  cpx<R>* r = static_cast<cpx<R>*>(p->d_t);
  if (!p->dirichlet) {
    Params<R> q = base_params<R>(p);
    q.u = static_cast<const cpx<R>*>(u);
    q.s = static_cast<const cpx<R>*>(s);
    q.out = static_cast<cpx<R>*>(u);
    q.out2 = r;
    q.a = r;
    q.b = static_cast<const cpx<R>*>(wloc);
    q.table = static_cast<const cpx<R>*>(wf);
    q.partials = nullptr;
    return issue_chain(p, st, count + 1, [&](int k, hipStream_t ls, const cbs_plan_s::Items& it) {
      npbs_step(p, q, count, k, ls, it);
    });
  }
  for (int k = 0; k < count; ++k) {
    Params<R> q = base_params<R>(p);
    q.u = static_cast<const cpx<R>*>(u);
    q.s = static_cast<const cpx<R>*>(s);
    q.epi = EPI_RESID;
    q.out = r;
    q.partials = nullptr;
    CHK(run_pipeline(p, q, st));
    Params<R> m = base_params<R>(p);
    m.pro = PRO_A;
    m.a = r;
    m.sym = SYM_TABLE;
    m.table = static_cast<const cpx<R>*>(wf);
    m.epi = EPI_NPBS;
    m.u = static_cast<const cpx<R>*>(u);
    m.b = static_cast<const cpx<R>*>(wloc);
    m.out = static_cast<cpx<R>*>(u);
    m.partials = nullptr;
    CHK(run_pipeline(p, m, st));
  }
  return CBS_OK;
}

// ---- convection-diffusion-reaction plans ---------------------------------------------------

// Column pass of V: p_y = Dy(dkappa Dy u) - dvy Dy u (adj 0) or
// Dy(dkappa Dy g + dvy g) (adj 1), into d_e.
template <typename R>
cpx<R>* cdr_col_pass(cbs_plan p, const cpx<R>* u, int adj, hipStream_t st) {
  cpx<R>* py = static_cast<cpx<R>*>(p->d_e);
  Params<R> c = base_params<R>(p);
  c.k2b = static_cast<const cpx<R>*>(p->d_k2b);
  c.partials = nullptr;
  c.u = u;
  c.out = py;
  const cbs_plan_s::Items it = p->view->all();
  if constexpr (sizeof(R) == 4) {
    c.items = it.cols32;
    launch_cdr_col(adj, it.ncols32, p->col_lds32, st, c);
  } else {
    c.items = it.cols64;
    launch_cdr_col(adj, it.ncols64, p->col_lds64, st, c);
  }
  return py;
}

// Row pass of V (mode as in launch_cdr_row); py from cdr_col_pass.
template <typename R>
void cdr_row_pass(cbs_plan p, int mode, const cpx<R>* u, const cpx<R>* s, const cpx<R>* py, cpx<R>* out,
                  hipStream_t st) {
  Params<R> r = base_params<R>(p);
  r.k2b = static_cast<const cpx<R>*>(p->d_k2b);
  r.partials = nullptr;
  r.items = p->view->rows;
  r.u = u;
  r.s = s;
  r.b = py;
  r.out = out;
  launch_cdr_row(mode, p->view->nrows, st, r);
}

// y = G (V u + s) (epi EPI_STORE) or r = G (V u + s) - u + rhs (EPI_RESID):
// column pass of V, row pass of V fused with the forward rows of G, the
// Green column pass and the inverse rows with the epilogue.
template <typename R>
cbs_status cdr_green_impl(cbs_plan p, const void* u, const void* s, const void* rhs, void* out,
                          int epi, double* norm2, hipStream_t st) {
  Params<R> q = base_params<R>(p);
  q.sym = SYM_CDR;
  q.epi = epi;
  q.u = static_cast<const cpx<R>*>(u);
  q.rhs = static_cast<const cpx<R>*>(rhs);
  q.out = static_cast<cpx<R>*>(out);
  if (epi == EPI_STORE) q.partials = nullptr;
  if (u) {
    const cpx<R>* uu = static_cast<const cpx<R>*>(u);
    const cpx<R>* py = cdr_col_pass<R>(p, uu, 0, st);
    cdr_row_pass<R>(p, 0, uu, static_cast<const cpx<R>*>(s), py, nullptr, st);
    launch_cols(p, q, st);
    q.items = p->view->rows;
    launch_row(1, p->view->nrows, st, q);
    HIPCHK(hipGetLastError());
  } else {  // V 0 = 0: transform s itself (PRO_VU_S with u = NULL; s NULL reads as zero)
    q.s = static_cast<const cpx<R>*>(s);
    CHK(run_pipeline(p, q, st));
  }
  if (norm2) {
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, norm2);
    HIPCHK(hipGetLastError());
  }
  return CBS_OK;
}

// r = s - A u = (V u + s) - L0 u
template <typename R>
cbs_status cdr_physical_impl(cbs_plan p, const void* u, const void* s, void* r, double* norm2,
                             hipStream_t st) {
  const cpx<R>* uu = static_cast<const cpx<R>*>(u);
  cpx<R>* t = static_cast<cpx<R>*>(p->d_t);
  const cpx<R>* py = cdr_col_pass<R>(p, uu, 0, st);
  cdr_row_pass<R>(p, 1, uu, static_cast<const cpx<R>*>(s), py, t, st);
  Params<R> q = base_params<R>(p);
  q.pro = PRO_A;
  q.a = uu;
  q.sym = SYM_CDR_NEG_L0;
  q.epi = EPI_RESID;  // -L0 u - 0 + t
  q.u = nullptr;
  q.rhs = t;
  q.out = static_cast<cpx<R>*>(r);
  CHK(run_pipeline(p, q, st));
  if (norm2) {
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, norm2);
    HIPCHK(hipGetLastError());
  }
  return CBS_OK;
}

// out = R^H e for R = I - G V: e - V^H G^H e
template <typename R>
cbs_status born_adjoint_impl(cbs_plan p, const void* e, void* out, hipStream_t st) {
  Params<R> q = base_params<R>(p);
  q.pro = PRO_A;
  q.a = static_cast<const cpx<R>*>(e);
  q.partials = nullptr;
  if (!p->cdr) {  // V is pointwise: the epilogue applies e - conj(V) z
    q.sym = SYM_GREEN_CONJ;
    q.epi = EPI_BORN_ADJ;
    q.out = static_cast<cpx<R>*>(out);
    return run_pipeline(p, q, st);
  }
  cpx<R>* g = inter_of<R>(p);  // G^H e, written over the spectral buffer it came from
  q.sym = SYM_CDR_CONJ;
  q.epi = EPI_STORE;
  q.out = g;
  CHK(run_pipeline(p, q, st));
  const cpx<R>* py = cdr_col_pass<R>(p, g, 1, st);
  cdr_row_pass<R>(p, 2, g, static_cast<const cpx<R>*>(e), py, static_cast<cpx<R>*>(out), st);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// ---- residual norms and the metric-matched gradient ----------------------------------------

// r = s - A u with the plan's physical operator (A u = -Lap u - k^2 u, or
// the CDR operator), r nullable, and per-instance sums |r|^2.
template <typename R>
cbs_status physical_norm2(cbs_plan p, const void* u, const void* s, void* r, double* norm2, hipStream_t st) {
  if (p->cdr) return cdr_physical_impl<R>(p, u, s, r, norm2, st);
  Params<R> q = base_params<R>(p);
  q.u = static_cast<const cpx<R>*>(u);
  q.s = static_cast<const cpx<R>*>(s);
  q.out = static_cast<cpx<R>*>(r);
  q.pro = PRO_U;
  q.sym = SYM_LAP;
  q.epi = EPI_LAP;
  CHK(run_pipeline(p, q, st));
  if (norm2) {
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, norm2);
    HIPCHK(hipGetLastError());
  }
  return CBS_OK;
}

template <typename R>
cbs_status relres_impl(cbs_plan p, const void* u, const void* s, int stop, double* relres, hipStream_t st) {
  double* num = p->d_tmp;
  double* den = p->d_tmp + p->batch;
  if (stop == CBS_STOP_BORN) {
    // ||G(V u + s) - u||^2 and ||G s||^2
    if (p->cdr) {
      CHK(cdr_green_impl<R>(p, u, s, nullptr, nullptr, EPI_RESID, num, st));
      CHK(cdr_green_impl<R>(p, nullptr, s, nullptr, nullptr, EPI_RESID, den, st));
    } else {
      CHK(residual_impl<R>(p, u, s, nullptr, nullptr, num, st));
      CHK(residual_impl<R>(p, nullptr, s, nullptr, nullptr, den, st));
    }
  } else {
    // ||s - A u||^2 and ||s||^2
    CHK(physical_norm2<R>(p, u, s, nullptr, num, st));
    launch_norm2_rows(p->view->nrows, st, p->d_inst, p->view->rows, static_cast<const cpx<R>*>(s), p->d_partials);
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, den);
  }
  launch_ratio(p->batch, st, num, den, relres);
  HIPCHK(hipGetLastError());
  return CBS_OK;
}

// loss_i = ||G s - (I - G V) x||^2 (the Born residual r = G(V x + s) - x),
// grad = -2 scale_i R^H r with R = I - G V.
template <typename R>
cbs_status mm_grad_impl(cbs_plan p, const void* x, const void* s, const double* scale, double* loss,
                        void* grad, hipStream_t st) {
  cpx<R>* r = static_cast<cpx<R>*>(p->d_t);
  if (p->cdr) CHK(cdr_green_impl<R>(p, x, s, nullptr, r, EPI_RESID, loss, st));
  else CHK(residual_impl<R>(p, x, s, nullptr, r, loss, st));
  PwParams<R> w{};
  w.op = PW_SCALE;
  w.e_in = r;
  w.e_out = r;
  w.scale = scale;
  w.factor = -2.0;
  CHK(launch_pw(p, w, st));
  return born_adjoint_impl<R>(p, r, grad, st);
}

// ---- adjoint -------------------------------------------------------------------------------

template <typename R>
cbs_status adjoint_impl(cbs_plan p, const void* um, const void* s, const void* lam_in,
                        void* lam_out, void* grad, hipStream_t st) {
  cpx<R>* r = static_cast<cpx<R>*>(p->d_t);
  if (!p->dirichlet && !p->cdr) {
    // periodic plans: both transform pairs in three launches, each
    // workgroup transforming both fields; r never leaves the registers
    Params<R> q = base_params<R>(p);
    q.u = static_cast<const cpx<R>*>(um);
    q.s = static_cast<const cpx<R>*>(s);
    q.a = static_cast<const cpx<R>*>(lam_in);
    q.out = static_cast<cpx<R>*>(lam_out);
    q.out2 = static_cast<cpx<R>*>(grad);
    q.inter2 = r;  // the second spectral field
    q.dual = 1;
    q.sym = SYM_GREEN;
    q.partials = nullptr;
    q.items = p->view->rows;
    launch_row(5, p->view->nrows, st, q);
    launch_cols(p, q, st);
    launch_row(6, p->view->nrows, st, q);
    HIPCHK(hipGetLastError());
    return CBS_OK;
  }
  {
    Params<R> q = base_params<R>(p);
    q.u = static_cast<const cpx<R>*>(um);
    q.s = static_cast<const cpx<R>*>(s);
    q.epi = EPI_RESID;
    q.out = r;
    q.partials = nullptr;
    CHK(run_pipeline(p, q, st));
  }
  Params<R> q = base_params<R>(p);
  q.pro = PRO_CONJG_A;
  q.sym = SYM_GREEN_CONJ;
  q.epi = EPI_ADJ;
  q.a = static_cast<const cpx<R>*>(lam_in);
  q.b = r;
  q.u = static_cast<const cpx<R>*>(um);
  q.out = static_cast<cpx<R>*>(lam_out);
  q.out2 = static_cast<cpx<R>*>(grad);
  q.partials = nullptr;
  return run_pipeline(p, q, st);
}

template <typename R>
cbs_status seed_impl(cbs_plan p, const void* uk, const void* s, int wg, double* loss,
                     void* lam_out, void* grad, hipStream_t st) {
  cpx<R>* r = static_cast<cpx<R>*>(p->d_t);
  if (wg == 2) {
    // physical residual e = s - A u_K, then lam_K = -2 A^H e (symbol |xi|^2)
    Params<R> q = base_params<R>(p);
    q.u = static_cast<const cpx<R>*>(uk);
    q.s = static_cast<const cpx<R>*>(s);
    q.pro = PRO_U;
    q.sym = SYM_LAP;
    q.epi = EPI_LAP;
    q.out = r;
    q.partials = nullptr;
    CHK(run_pipeline(p, q, st));
    Params<R> a = base_params<R>(p);
    a.pro = PRO_A;
    a.sym = SYM_LAP;
    a.epi = EPI_PHYS_SEED;
    a.a = r;
    a.u = static_cast<const cpx<R>*>(uk);
    a.out = static_cast<cpx<R>*>(lam_out);
    a.out2 = static_cast<cpx<R>*>(grad);
    CHK(run_pipeline(p, a, st));
  } else {
    {
      Params<R> q = base_params<R>(p);
      q.u = static_cast<const cpx<R>*>(uk);
      q.s = static_cast<const cpx<R>*>(s);
      q.epi = EPI_RESID;
      q.out = r;
      q.partials = nullptr;
      CHK(run_pipeline(p, q, st));
    }
    Params<R> q = base_params<R>(p);
    q.pro = PRO_SEED;
    q.sym = SYM_GREEN_CONJ;
    q.epi = EPI_SEED;
    q.weight_gamma = wg ? 1 : 0;
    q.a = r;
    q.u = static_cast<const cpx<R>*>(uk);
    q.out = static_cast<cpx<R>*>(lam_out);
    q.out2 = static_cast<cpx<R>*>(grad);
    CHK(run_pipeline(p, q, st));
  }
  if (loss) {
    launch_instance_sums(p->batch, st, p->d_inst, p->d_partials, loss);
    HIPCHK(hipGetLastError());
  }
  return CBS_OK;
}

cbs_status check_setup_args(int batch, const int32_t* n, int dtype, int max_restart, uint32_t flags) {
  if (batch < 1 || !n) return fail(CBS_ERR_ARG, "batch < 1 or n NULL");
  if (dtype != CBS_C64 && dtype != CBS_C128) return fail(CBS_ERR_ARG, "dtype must be CBS_C64 or CBS_C128");
  if (max_restart < 0 || max_restart > kMaxRestart)
    return fail(CBS_ERR_ARG, "max_restart must be in [0, " + std::to_string(kMaxRestart) + "]");
  if (flags & ~uint32_t(CBS_FLAG_NO_GUARD | CBS_FLAG_ONE_STREAM | CBS_FLAG_DIRICHLET | CBS_FLAG_UNDAMPED))
    return fail(CBS_ERR_ARG, "unknown flag bits");
  const bool dir = (flags & CBS_FLAG_DIRICHLET) != 0;
  if ((flags & CBS_FLAG_UNDAMPED) && !dir)
    return fail(CBS_ERR_ARG, "CBS_FLAG_UNDAMPED needs CBS_FLAG_DIRICHLET (a periodic reference |xi|^2 - k0^2 "
                             "vanishes or nearly vanishes on the grid without damping)");
  for (int i = 0; i < batch; ++i)
    if (n[i] < 1 || !(dir ? (supported_n(dst_len(n[i])) || n[i] == kDstDirectN) : supported_n(n[i])))
      return fail(CBS_ERR_SIZE, std::string(dir ? "unsupported Dirichlet size " : "unsupported grid size ") +
                                    std::to_string(n[i]) + " (instance " + std::to_string(i) + ")");
  return CBS_OK;
}

// Host-side layout of a plan: sizes, packed offsets, work items.
void init_layout(cbs_plan p, int batch, const int32_t* n, int dtype, int max_restart, uint32_t flags) {
  p->batch = batch;
  p->dtype = dtype;
  p->max_restart = max_restart;
  p->one_stream = (flags & CBS_FLAG_ONE_STREAM) != 0;
  p->dirichlet = (flags & CBS_FLAG_DIRICHLET) != 0;
  p->undamped = (flags & CBS_FLAG_UNDAMPED) != 0;
  // FP32 periodic Helmholtz plans start with the wide column workgroups
  // (the faster ones on MI355X for the ragged and 1024^2 batches)
  p->col_threads32 = (dtype == CBS_C64 && !p->dirichlet && !p->cdr) ? kColThreadsWide : kThreads;
  p->n.assign(n, n + batch);
  long long off = 0;
  for (int i = 0; i < batch; ++i) {
    p->off.push_back(off);
    off += (long long)n[i] * n[i];
    p->maxn = std::max(p->maxn, n[i]);
  }
  p->cells = off;
  if (max_restart > 0) p->kry_stride = KryLayout{max_restart}.size();
  build_items(p);
}

// Every device buffer of a plan (pointer to set, bytes).
std::vector<std::pair<void**, size_t>> buffer_requests(cbs_plan p) {
  const long long cells = p->cells;
  const size_t oe = p->op_elem();
  const size_t batch = size_t(p->batch);
  const size_t nrow = p->row_items.size();
  std::vector<std::pair<void**, size_t>> req = {
      {reinterpret_cast<void**>(&p->d_inst), batch * sizeof(InstDesc)},
      {reinterpret_cast<void**>(&p->d_row_items), nrow * sizeof(int2)},
      {reinterpret_cast<void**>(&p->d_tw32), kTwTotal * sizeof(cpx<float>)},
      {reinterpret_cast<void**>(&p->d_tw64), kTwTotal * sizeof(cpx<double>)},
      {reinterpret_cast<void**>(&p->d_mu), kMuTotal * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_k2_64), cells * 16},
      {reinterpret_cast<void**>(&p->d_inter64), cells * 16},
      {reinterpret_cast<void**>(&p->d_u64), cells * 16},
      {reinterpret_cast<void**>(&p->d_s64), cells * 16},
      {&p->d_c, cells * oe},
      {&p->d_e, cells * oe},
      {&p->d_t, cells * oe},
      {reinterpret_cast<void**>(&p->d_partials), (2 * nrow + 64) * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_status), batch * sizeof(int)},
      {reinterpret_cast<void**>(&p->d_iters), batch * sizeof(int)},
      {reinterpret_cast<void**>(&p->d_chunk_active), batch * sizeof(int)},
      {reinterpret_cast<void**>(&p->d_relres), batch * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_est), batch * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_bnorm), batch * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_rtol), sizeof(double)},
      {reinterpret_cast<void**>(&p->d_rtol32), sizeof(double)},
      {reinterpret_cast<void**>(&p->d_tmp), 2 * batch * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_bnorm_phys), batch * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_maxs), sizeof(int)},
      {reinterpret_cast<void**>(&p->d_scale), batch * sizeof(double)},
      {reinterpret_cast<void**>(&p->d_kactive), batch * sizeof(int)},
      {reinterpret_cast<void**>(&p->d_kjend), batch * sizeof(int)},
      {reinterpret_cast<void**>(&p->full.lids), batch * sizeof(int)},
      {reinterpret_cast<void**>(&p->compact.lids), batch * sizeof(int)},
  };
  if (p->dtype == CBS_C64) {
    req.push_back({&p->d_k2, cells * 8});
    req.push_back({&p->d_inter, cells * 8});
  }
  if (p->cdr) req.push_back({&p->d_k2b, cells * oe});
  if (p->max_restart > 0) {
    const size_t m = size_t(p->max_restart);
    req.push_back({reinterpret_cast<void**>(&p->d_vbasis), cells * 16 * (m + 1)});
    req.push_back({&p->d_zbasis, cells * oe * m});
    req.push_back({reinterpret_cast<void**>(&p->d_kry), size_t(p->kry_stride) * batch * sizeof(double)});
    req.push_back({reinterpret_cast<void**>(&p->d_dots), (4 * (m + 1) + 4) * nrow * sizeof(double)});
  }
  // work lists (capacity: tile width 2 everywhere)
  const size_t cap = item_capacity(p) * sizeof(int2);
  for (int2** d : {&p->d_col_items32, &p->d_col_items64, &p->compact.rows, &p->compact.cols32,
                   &p->compact.cols64, &p->full.lrows, &p->full.lcols32, &p->full.lcols64,
                   &p->compact.lrows, &p->compact.lcols32, &p->compact.lcols64})
    req.push_back({reinterpret_cast<void**>(d), cap});
  return req;
}

size_t padded(size_t bytes) { return (std::max<size_t>(bytes, 16) + 255) / 256 * 256; }

size_t request_bytes(const std::vector<std::pair<void**, size_t>>& req) {
  size_t total = 0;
  for (const auto& r : req) total += padded(r.second);
  return total;
}

// Convection-diffusion-reaction setup data: the (vx, vy) field and the
// background constants (kappa0, vx0, vy0, sigma0) per instance.
struct CdrInit {
  const void* velocity;
  const double* background;
};

cbs_status setup_impl(cbs_plan* out, int batch, const int32_t* n, const void* k2,
                      const double* k0sq, const double* eps, int dtype, int max_restart,
                      uint32_t flags, void* ws, size_t ws_bytes, void* stream,
                      const CdrInit* cdr = nullptr);

}  // namespace

constexpr const char* kNoGamma =
    "an undamped plan (eps = 0) has no gamma = i V / eps: CBS sweeps, cbs_iterate, FGMRES inner sweeps, "
    "the sweep adjoint and the W = gamma seed are not available";

extern "C" {

const char* cbs_last_error(void) { return g_err.c_str(); }
const char* cbs_version(void) { return "cbs-mi355x 0.1 (gfx950)"; }

cbs_status cbs_setup(cbs_plan* out, int batch, const int32_t* n, const void* k2,
                     const double* k0sq, const double* eps, int dtype, int max_restart,
                     uint32_t flags, void* stream) {
  return setup_impl(out, batch, n, k2, k0sq, eps, dtype, max_restart, flags, nullptr, 0, stream);
}

cbs_status cbs_setup_ws(cbs_plan* out, int batch, const int32_t* n, const void* k2,
                        const double* k0sq, const double* eps, int dtype, int max_restart,
                        uint32_t flags, void* workspace, size_t workspace_bytes, void* stream) {
  if (!workspace) {
    if (out) *out = nullptr;
    return fail(CBS_ERR_ARG, "workspace is NULL");
  }
  return setup_impl(out, batch, n, k2, k0sq, eps, dtype, max_restart, flags, workspace,
                    workspace_bytes, stream);
}

}  // extern "C"

namespace {

// Arguments of a convection-diffusion-reaction plan: finite background
// constants whose symbol kappa0 |xi|^2 + sigma0 + i v0 . xi vanishes on no bin.
cbs_status check_cdr_args(int batch, const int32_t* n, const double* background, int dtype) {
  CHK(check_setup_args(batch, n, dtype, 0, 0));
  if (!background) return fail(CBS_ERR_ARG, "background is NULL");
  for (int i = 0; i < batch; ++i) {
    for (int k = 0; k < 4; ++k)
      if (!std::isfinite(background[4 * i + k]))
        return fail(CBS_ERR_ARG, "background constants must be finite (instance " + std::to_string(i) + ")");
    const double k0 = background[4 * i], vx = background[4 * i + 1], vy = background[4 * i + 2],
                 s0 = background[4 * i + 3];
    const int nn = n[i];
    const double h = 2.0 * M_PI / nn;
    double lo = INFINITY, hi = 0.0;
    for (int a = 0; a < nn; ++a) {
      const double xy = (a >= nn / 2 ? a - nn : a) * h;
      for (int b = 0; b < nn; ++b) {
        const double xx = (b >= nn / 2 ? b - nn : b) * h;
        const double re = k0 * (xx * xx + xy * xy) + s0, im = vx * xx + vy * xy;
        const double m = std::sqrt(re * re + im * im);
        lo = std::min(lo, m);
        hi = std::max(hi, m);
      }
    }
    if (!(lo > 1e-12 * hi))
      return fail(CBS_ERR_ILLCOND, "instance " + std::to_string(i) +
                                       ": the background symbol kappa0|xi|^2 + sigma0 + i v0.xi vanishes");
  }
  return CBS_OK;
}

cbs_status setup_cdr_common(cbs_plan* out, int batch, const int32_t* n, const void* kappa_sigma,
                            const void* velocity, const double* background, int dtype, void* ws,
                            size_t ws_bytes, void* stream) {
  if (!out) return fail(CBS_ERR_ARG, "plan pointer is NULL");
  *out = nullptr;
  if (!kappa_sigma || !velocity || !background)
    return fail(CBS_ERR_ARG, "kappa_sigma, velocity or background is NULL");
  CHK(check_cdr_args(batch, n, background, dtype));
  CdrInit c{velocity, background};
  return setup_impl(out, batch, n, kappa_sigma, nullptr, nullptr, dtype, 0, CBS_FLAG_ONE_STREAM, ws, ws_bytes,
                    stream, &c);
}

}  // namespace

extern "C" {

cbs_status cbs_setup_cdr(cbs_plan* out, int batch, const int32_t* n, const void* kappa_sigma,
                         const void* velocity, const double* background, int dtype, void* stream) {
  return setup_cdr_common(out, batch, n, kappa_sigma, velocity, background, dtype, nullptr, 0, stream);
}

cbs_status cbs_setup_cdr_ws(cbs_plan* out, int batch, const int32_t* n, const void* kappa_sigma,
                            const void* velocity, const double* background, int dtype, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!workspace) {
    if (out) *out = nullptr;
    return fail(CBS_ERR_ARG, "workspace is NULL");
  }
  return setup_cdr_common(out, batch, n, kappa_sigma, velocity, background, dtype, workspace, workspace_bytes,
                          stream);
}

cbs_status cbs_workspace_size_cdr(int batch, const int32_t* n, int dtype, size_t* bytes) {
  if (!bytes) return fail(CBS_ERR_ARG, "bytes is NULL");
  *bytes = 0;
  CHK(check_setup_args(batch, n, dtype, 0, 0));
  cbs_plan_s p;
  p.cdr = true;
  init_layout(&p, batch, n, dtype, 0, CBS_FLAG_ONE_STREAM);
  CHK(check_item_capacity(&p));
  *bytes = request_bytes(buffer_requests(&p));
  return CBS_OK;
}

cbs_status cbs_born_adjoint(cbs_plan p, const void* e, void* out, void* stream) {
  if (!p || !e || !out) return fail(CBS_ERR_ARG, "plan, e or out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return born_adjoint_impl<float>(p, e, out, st);
  return born_adjoint_impl<double>(p, e, out, st);
}

cbs_status cbs_workspace_size(int batch, const int32_t* n, int dtype, int max_restart,
                              uint32_t flags, size_t* bytes) {
  if (!bytes) return fail(CBS_ERR_ARG, "bytes is NULL");
  *bytes = 0;
  CHK(check_setup_args(batch, n, dtype, max_restart, flags));
  cbs_plan_s p;
  init_layout(&p, batch, n, dtype, max_restart, flags);
  CHK(check_item_capacity(&p));
  *bytes = request_bytes(buffer_requests(&p));
  return CBS_OK;
}

}  // extern "C"

namespace {

// An undamped Dirichlet reference L_D - k0^2 (App. B.2, Eq. newton_ref: J_0
// with no damping term) must be invertible: its eigenvalues mu_p + mu_q - k0^2,
// mu_p = 4/h^2 sin^2(p pi h/2), p = 1..n, stay away from zero.  Exactly
// singular is always rejected; closer than 1e-9 of the spectrum's scale
// unless the guard is off.
cbs_status check_undamped_reference(int n, double k0sq, int inst, bool no_guard) {
  const double h = 1.0 / (n + 1);
  std::vector<double> mu(n);
  for (int q = 0; q < n; ++q) {
    const double sn = std::sin((q + 1) * M_PI * h / 2);
    mu[q] = 4.0 / (h * h) * sn * sn;
  }
  double dmin = INFINITY;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) dmin = std::min(dmin, std::fabs(mu[a] + mu[b] - k0sq));
  const double scale = std::max(2.0 * mu[n - 1], std::fabs(k0sq));
  if (!(dmin > 0.0) || (!no_guard && dmin < 1e-9 * scale))
    return fail(CBS_ERR_ILLCOND, "instance " + std::to_string(inst) +
                                     ": undamped reference L_D - k0^2 is singular or nearly so "
                                     "(k0^2 at an eigenvalue of L_D)");
  return CBS_OK;
}

cbs_status setup_impl(cbs_plan* out, int batch, const int32_t* n, const void* k2,
                      const double* k0sq, const double* eps, int dtype, int max_restart,
                      uint32_t flags, void* ws, size_t ws_bytes, void* stream, const CdrInit* cdr) {
  if (!out) return fail(CBS_ERR_ARG, "plan pointer is NULL");
  *out = nullptr;
  if (!k2) return fail(CBS_ERR_ARG, "k2 is NULL");
  CHK(check_setup_args(batch, n, dtype, max_restart, flags));
  if (eps && (flags & CBS_FLAG_UNDAMPED)) return fail(CBS_ERR_ARG, "eps must be NULL on an undamped plan");
  if (eps)
    for (int i = 0; i < batch; ++i)
      if (std::isnan(eps[i]) || std::isinf(eps[i])) return fail(CBS_ERR_ARG, "eps must be finite");
  if (k0sq)
    for (int i = 0; i < batch; ++i)
      if (std::isinf(k0sq[i])) return fail(CBS_ERR_ARG, "k0sq must be finite or NaN (auto)");

  hipStream_t st = static_cast<hipStream_t>(stream);
  cbs_plan p = new cbs_plan_s();
  p->cdr = cdr != nullptr;
  init_layout(p, batch, n, dtype, max_restart, flags);

  auto bail = [&](cbs_status s, const std::string& m) {
    free_plan(p);
    delete p;
    return fail(s, m);
  };
  const long long cells = p->cells;
  const std::vector<std::pair<void**, size_t>> req = buffer_requests(p);
  if (ws) {
    // Every buffer is carved from the caller's workspace (256-byte aligned).
    const size_t need = request_bytes(req);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
      return bail(CBS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
      return bail(CBS_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                         std::to_string(need));
    char* cur = static_cast<char*>(ws);
    for (auto& r : req) {
      *r.first = cur;
      cur += padded(r.second);
    }
  } else {
    for (auto& r : req) {
      void* ptr = nullptr;
      hipError_t e = hipMalloc(&ptr, padded(r.second));
      if (e != hipSuccess) return bail(CBS_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
      p->owned.push_back(ptr);
      *r.first = ptr;
    }
  }
  if (dtype == CBS_C128) {
    p->d_k2 = p->d_k2_64;
    p->d_inter = p->d_inter64;
  }
  p->compact.gen = 1;
  {
    // capture stream for cbs_iterate's graphs when the caller passes the
    // null stream (the legacy null stream cannot be captured)
    hipError_t e = hipStreamCreate(&p->own_stream);
    if (e != hipSuccess) return bail(CBS_ERR_HIP, std::string("plan stream: ") + hipGetErrorString(e));
  }
  if (lanes_wanted(p, std::vector<char>(batch, 1))) {
    for (int l = 0; l < 2; ++l) {
      hipError_t e = hipStreamCreateWithFlags(&p->lane_st[l], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join[l], hipEventDisableTiming);
      if (e != hipSuccess) return bail(CBS_ERR_HIP, std::string("lane stream: ") + hipGetErrorString(e));
    }
    hipError_t e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    if (e != hipSuccess) return bail(CBS_ERR_HIP, std::string("lane event: ") + hipGetErrorString(e));
  }

  // Per-pass twiddle tables w^(q k), w = exp(-2 pi i / (Ns r)), evaluated in
  // FP64 on the host with the exponent reduced exactly, rounded once for FP32.
  std::vector<cpx<double>> t64(kTwTotal, cpx<double>{0.0, 0.0});
  std::vector<cpx<float>> t32(kTwTotal, cpx<float>{0.f, 0.f});
  for (int nn : kSizes) {
    for (int pass = 0; pass < plan_passes(nn); ++pass) {
      const int ns = plan_ns(nn, pass), rad = plan_radix(nn, pass), rp = radp(rad);
      if (ns == 1) continue;
      const int o = tw_pass_offset(nn, pass);
      for (int k = 0; k < ns; ++k)
        for (int q = 0; q < rad; ++q) {
          const long long m = ((long long)q * k) % ((long long)ns * rad);
          const double ang = -2.0 * M_PI * double(m) / double(ns * rad);
          t64[o + k * rp + q] = cpx<double>{std::cos(ang), std::sin(ang)};
          t32[o + k * rp + q] = cpx<float>{float(std::cos(ang)), float(std::sin(ang))};
        }
    }
  }
#define BAILCHK(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return bail(CBS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
  BAILCHK(hipMemcpyAsync(p->d_tw64, t64.data(), kTwTotal * sizeof(cpx<double>), hipMemcpyHostToDevice, st));
  // Dirichlet eigenvalue table mu_p = M^2 sin^2(pi p / M) (5-point FD Laplacian
  // on the unit square, h = 1/(n+1) = 2/M), FP64 on the host
  std::vector<double> mu(kMuTotal, 0.0);
  for (int mm : kSizes)
    for (int q = 0; q < mm; ++q) {
      const double sn = std::sin(M_PI * double(q) / double(mm));
      mu[mu_offset(mm) + q] = double(mm) * double(mm) * sn * sn;
    }
  for (int q = 0; q < kDstDirectM; ++q) {
    const double sn = std::sin(M_PI * double(q) / double(kDstDirectM));
    mu[kMuDirect + q] = double(kDstDirectM) * double(kDstDirectM) * sn * sn;
    mu[kSinDirect + q] = std::sin(M_PI * double(q) / double(kDstDirectN + 1));
  }
  BAILCHK(hipMemcpyAsync(p->d_mu, mu.data(), kMuTotal * sizeof(double), hipMemcpyHostToDevice, st));
  BAILCHK(hipMemcpyAsync(p->d_tw32, t32.data(), kTwTotal * sizeof(cpx<float>), hipMemcpyHostToDevice, st));
  BAILCHK(hipMemcpyAsync(p->d_row_items, p->row_items.data(), p->row_items.size() * sizeof(int2),
                         hipMemcpyHostToDevice, st));
  if (cdr) {
    // (kappa, sigma) and (vx, vy) -> deviations from the background, in the
    // operator precision only (no FP64 refinement runs on these plans)
    const size_t oe = p->op_elem();
    BAILCHK(hipMemcpyAsync(dtype == CBS_C64 ? p->d_k2 : static_cast<void*>(p->d_k2_64), k2, cells * oe,
                           hipMemcpyDeviceToDevice, st));
    BAILCHK(hipMemcpyAsync(p->d_k2b, cdr->velocity, cells * oe, hipMemcpyDeviceToDevice, st));
    p->k0sq.assign(batch, 0.0);
    p->eps.assign(batch, 0.0);
    p->vx0.assign(batch, 0.0);
    p->vy0.assign(batch, 0.0);
    for (int i = 0; i < batch; ++i) {
      p->k0sq[i] = cdr->background[4 * i];
      p->vx0[i] = cdr->background[4 * i + 1];
      p->vy0[i] = cdr->background[4 * i + 2];
      p->eps[i] = cdr->background[4 * i + 3];
    }
    build_items(p);
    cbs_status us = upload_items(p, st);
    if (us != CBS_OK) { std::string m = g_err; return bail(us, m); }
    const int nrow = int(p->row_items.size());
    if (dtype == CBS_C64)
      launch_cdr_split(nrow, st, p->d_inst, p->d_row_items, static_cast<cpx<float>*>(p->d_k2),
                       static_cast<cpx<float>*>(p->d_k2b));
    else
      launch_cdr_split(nrow, st, p->d_inst, p->d_row_items, p->d_k2_64, static_cast<cpx<double>*>(p->d_k2b));
    BAILCHK(hipGetLastError());
    BAILCHK(hipStreamSynchronize(st));
    *out = p;
    return CBS_OK;
  }
  if (dtype == CBS_C64) {
    BAILCHK(hipMemcpyAsync(p->d_k2, k2, cells * 8, hipMemcpyDeviceToDevice, st));
    launch_widen_all(st, static_cast<const cpx<float>*>(p->d_k2), p->d_k2_64, cells);
    BAILCHK(hipGetLastError());
  } else {
    BAILCHK(hipMemcpyAsync(p->d_k2_64, k2, cells * 16, hipMemcpyDeviceToDevice, st));
  }
#undef BAILCHK

  // Reference k0^2 and damping eps from FP64 statistics of k^2 on the GPU.
  p->k0sq.assign(batch, 0.0);
  p->eps.assign(batch, 1.0);
  build_items(p);
  std::vector<double> a, b;
  cbs_status s = compute_stats(p, 0, st, a, b);
  if (s != CBS_OK) { std::string m = g_err; return bail(s, m); }
  for (int i = 0; i < batch; ++i) {
    const bool autok = !k0sq || std::isnan(k0sq[i]);
    p->k0sq[i] = autok ? 0.5 * (a[i] + b[i]) : k0sq[i];
  }
  build_items(p);
  s = compute_stats(p, 1, st, a, b);
  if (s != CBS_OK) { std::string m = g_err; return bail(s, m); }
  for (int i = 0; i < batch && p->undamped; ++i) {
    p->eps[i] = 0.0;
    cbs_status us = check_undamped_reference(p->n[i], p->k0sq[i], i, (flags & CBS_FLAG_NO_GUARD) != 0);
    if (us != CBS_OK) { std::string m = g_err; return bail(us, m); }
  }
  for (int i = 0; i < batch && !p->undamped; ++i) {
    const bool autoe = !eps || !(eps[i] > 0.0);
    p->eps[i] = autoe ? a[i] : eps[i];
    if (!(p->eps[i] > 0.0))
      return bail(CBS_ERR_ILLCOND, "instance " + std::to_string(i) + ": k^2 == k0^2 everywhere, eps would be 0");
    if (!(flags & CBS_FLAG_NO_GUARD) && p->eps[i] < a[i] * (1.0 - 1e-12))
      return bail(CBS_ERR_ILLCOND, "instance " + std::to_string(i) + ": eps below max|k^2-k0^2|");
  }
  build_items(p);
  if (!p->undamped) {
    s = compute_stats(p, 2, st, a, b);
    if (s != CBS_OK) { std::string m = g_err; return bail(s, m); }
  }
  for (int i = 0; i < batch && !p->undamped; ++i)
    if (!(flags & CBS_FLAG_NO_GUARD) && !(a[i] >= 1e-3 * p->eps[i]))
      return bail(CBS_ERR_ILLCOND,
                  "instance " + std::to_string(i) + ": min|V|/eps below 1e-3 (gamma ~ 0 stalls CBS)");
  {
    cbs_status us = upload_items(p, st);
    if (us != CBS_OK) { std::string m = g_err; return bail(us, m); }
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return bail(CBS_ERR_HIP, std::string("setup sync: ") + hipGetErrorString(e));
  *out = p;
  return CBS_OK;
}

}  // namespace

namespace {

// ---- autotuning -----------------------------------------------------------------------------

// Sizes present in the plan, largest first.
std::vector<int> size_classes(cbs_plan p) {
  std::vector<int> classes;
  for (int n : p->n)
    if (std::find(classes.begin(), classes.end(), n) == classes.end()) classes.push_back(n);
  std::sort(classes.begin(), classes.end(), [](int a, int b) { return a > b; });
  return classes;
}

// Tune on what the plan runs: chains of fused CBS sweeps over all its
// instances, with its lanes, on scratch fields holding the plan's own k^2
// (realistic magnitudes: all-zero fields run several per cent faster, which
// would bias the comparison).  Configurations are timed in interleaved
// rounds and each keeps its fastest round, since single timings of the same
// configuration scatter by a few per cent.  First the thread count of the
// FP32 column launches (each at its start widths), then, size by size, each
// other compiled width against the current choice, kept only when more than
// 2 % faster.
template <typename R>
cbs_status tune_by_sweeps(cbs_plan p, hipStream_t st, std::ostringstream& rec) {
  const size_t bytes = size_t(p->cells) * p->op_elem();
  HIPCHK(hipMemcpyAsync(p->d_e, k2_of<R>(p), bytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(p->d_c, k2_of<R>(p), bytes, hipMemcpyDeviceToDevice, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int chain = 30;
  struct Cfg {
    int threads;
    std::map<int, int> tiles;
  };
  auto timed = [&](const Cfg& c, double* per_sweep) -> cbs_status {
    p->col_threads32 = c.threads;
    p->ctile = c.tiles;
    build_items(p);
    drop_graphs(p);
    CHK(upload_items(p, st));
    CHK(sweep_impl<R>(p, p->d_e, p->d_c, 2, nullptr, st));  // warm-up
    HIPCHK(hipEventRecord(e0, st));
    CHK(sweep_impl<R>(p, p->d_e, p->d_c, chain, nullptr, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    *per_sweep = double(ms) / chain;
    return CBS_OK;
  };
  // fastest of `rounds` interleaved timings of each configuration
  auto race = [&](const std::vector<Cfg>& cfgs, int rounds, std::vector<double>& best) -> cbs_status {
    best.assign(cfgs.size(), 1e300);
    for (int r = 0; r < rounds; ++r)
      for (size_t k = 0; k < cfgs.size(); ++k) {
        double ms = 0.0;
        CHK(timed(cfgs[k], &ms));
        best[k] = std::min(best[k], ms);
      }
    return CBS_OK;
  };
  // The races time the plan's own sweep kernels on scratch fields whose
  // values are discarded (on an undamped plan gamma = i V / 0 makes them
  // non-finite, which does not change the kernels' timing).
  const Cfg saved{p->col_threads32, p->ctile};
  std::vector<Cfg> cfgs = {Cfg{kThreads, {}}};
  if (sizeof(R) == 4 && !p->dirichlet) cfgs.push_back(Cfg{kColThreadsWide, {}});
  std::vector<double> t;
  cbs_status rc = race(cfgs, 4, t);
  rec << "{\"dtype\": \"" << (sizeof(R) == 4 ? "c64" : "c128") << "\", \"by\": \"sweep chains\", \"configs\": [";
  Cfg cur = cfgs[0];
  double cur_ms = 1e300;
  if (rc == CBS_OK) {
    for (size_t k = 0; k < cfgs.size(); ++k) {
      rec << (k ? ", " : "") << "{\"col_threads\": " << cfgs[k].threads << ", \"us_per_sweep\": " << t[k] * 1e3 << "}";
      if (t[k] < cur_ms) {
        cur_ms = t[k];
        cur = cfgs[k];
      }
    }
    const int thr_used = sizeof(R) == 4 ? cur.threads : kThreads;
    for (int n : size_classes(p)) {
      const int m = p->tlen(n);
      const int start = col_tile_start_t(m, thr_used);
      cur.tiles[n] = start;
      for (int c : {col_tile_default(m) / 2, col_tile_default(m), col_tile_default(m) * 2}) {
        if (c == cur.tiles[n] || c == start || !col_tile_valid_t(m, c, p->op_elem(), thr_used)) continue;
        Cfg cand = cur;
        cand.tiles[n] = c;
        rc = race({cur, cand}, 3, t);
        if (rc != CBS_OK) break;
        rec << ", {\"n\": " << n << ", \"tile\": " << c << ", \"us_per_sweep\": " << t[1] * 1e3
            << ", \"against\": " << t[0] * 1e3 << "}";
        if (t[1] < 0.98 * t[0]) cur = cand;
      }
      if (rc != CBS_OK) break;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != CBS_OK) {
    p->col_threads32 = saved.threads;
    p->ctile = saved.tiles;
    return rc;
  }
  p->col_threads32 = cur.threads;
  p->ctile = cur.tiles;
  rec << "], \"col_threads\": " << p->col_threads32 << ", \"tiles\": {";
  bool first = true;
  for (const auto& kv : p->ctile) {
    rec << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
    first = false;
  }
  rec << "}}";
  return CBS_OK;
}

// Convection-diffusion-reaction plans have no sweep: time the Green column
// pass of each size class alone at its compiled widths, three interleaved
// rounds, and keep each class's fastest.
cbs_status tune_by_columns(cbs_plan p, hipStream_t st, std::ostringstream& rec) {
  HIPCHK(hipMemsetAsync(p->d_inter, 0, p->cells * p->op_elem(), st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const std::vector<int> classes = size_classes(p);
  std::map<int, std::map<int, double>> best_of;
  cbs_status rc = CBS_OK;
  for (int round = 0; round < 3 && rc == CBS_OK; ++round) {
    for (int n : classes) {
      const int m = p->tlen(n);
      for (int c : {col_tile_default(m) / 2, col_tile_default(m), col_tile_default(m) * 2}) {
        if (!col_tile_valid(m, c, p->op_elem())) continue;
        p->ctile[n] = c;
        build_items(p);
        rc = upload_items(p, st);
        if (rc != CBS_OK) break;
        // the column items of size class n form one contiguous range
        const std::vector<int2>& items = p->dtype == CBS_C64 ? p->col_items32 : p->col_items64;
        size_t lo = items.size(), hi = 0;
        for (size_t k = 0; k < items.size(); ++k)
          if (p->n[items[k].x] == n) {
            lo = std::min(lo, k);
            hi = k + 1;
          }
        auto launch = [&]() {
          if (p->dtype == CBS_C64) {
            Params<float> q = base_params<float>(p);
            q.sym = SYM_CDR;
            q.items = p->d_col_items32 + lo;
            launch_col(int(hi - lo), size_t(col_lds_elems(m, c)) * 8, st, q);
          } else {
            Params<double> q = base_params<double>(p);
            q.sym = SYM_CDR;
            q.items = p->d_col_items64 + lo;
            launch_col(int(hi - lo), size_t(col_lds_elems(m, p->inst[items[lo].x].ctile64)) * 16, st, q);
          }
        };
        for (int rep = 0; rep < 2; ++rep) launch();
        HIPCHK(hipEventRecord(e0, st));
        const int reps = 10;
        for (int rep = 0; rep < reps; ++rep) launch();
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipGetLastError());
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const double per = double(ms) / reps;
        auto it = best_of[n].find(c);
        if (it == best_of[n].end() || per < it->second) best_of[n][c] = per;
      }
      if (rc != CBS_OK) break;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != CBS_OK) return rc;
  rec << "{\"dtype\": \"" << (p->dtype == CBS_C64 ? "c64" : "c128") << "\", \"by\": \"column pass\", \"tiles\": {";
  bool first = true;
  for (int n : classes) {
    int best = col_tile_start(p->tlen(n));
    double best_ms = 1e300;
    for (const auto& kv : best_of[n])
      if (kv.second < best_ms) {
        best_ms = kv.second;
        best = kv.first;
      }
    p->ctile[n] = best;
    rec << (first ? "" : ", ") << "\"" << n << "\": {\"tile\": " << best << ", \"col_ms\": " << best_ms << "}";
    first = false;
  }
  rec << "}}";
  return CBS_OK;
}

}  // namespace

extern "C" {

cbs_status cbs_plan_info(cbs_plan p, int64_t* cells, double* k0sq, double* eps) {
  if (!p) return fail(CBS_ERR_ARG, "plan is NULL");
  if (cells) *cells = p->cells;
  for (int i = 0; i < p->batch; ++i) {
    if (k0sq) k0sq[i] = p->k0sq[i];
    if (eps) eps[i] = p->eps[i];
  }
  return CBS_OK;
}

cbs_status cbs_plan_layout(cbs_plan p, int32_t* lanes, int32_t* tiles, int32_t* col_threads) {
  if (!p) return fail(CBS_ERR_ARG, "plan is NULL");
  if (lanes) *lanes = p->full.nlanes;
  if (col_threads) *col_threads = p->dtype == CBS_C64 ? p->col_threads32 : kThreads;
  if (tiles)
    for (int i = 0; i < p->batch; ++i) tiles[i] = p->dtype == CBS_C64 ? p->inst[i].ctile : p->inst[i].ctile64;
  return CBS_OK;
}

cbs_status cbs_set_tile(cbs_plan p, int n, int columns) {
  if (!p) return fail(CBS_ERR_ARG, "plan is NULL");
  bool any = false;
  for (int nn : p->n) {
    if (n != 0 && nn != n) continue;
    if (!col_tile_valid_t(p->tlen(nn), columns, p->op_elem(), p->dtype == CBS_C64 ? p->col_threads32 : kThreads))
      return fail(CBS_ERR_ARG, "tile width " + std::to_string(columns) + " not available for size " +
                                   std::to_string(nn));
    any = true;
  }
  if (!any) return fail(CBS_ERR_ARG, "no instance of size " + std::to_string(n) + " in the plan");
  for (int nn : p->n)
    if (n == 0 || nn == n) p->ctile[nn] = columns;
  build_items(p);
  drop_graphs(p);
  CHK(upload_items(p, nullptr));
  HIPCHK(hipDeviceSynchronize());
  return CBS_OK;
}

cbs_status cbs_set_col_threads(cbs_plan p, int threads) {
  if (!p) return fail(CBS_ERR_ARG, "plan is NULL");
  if (threads != kThreads && threads != kColThreadsWide)
    return fail(CBS_ERR_ARG, "threads must be " + std::to_string(kThreads) + " or " +
                                 std::to_string(kColThreadsWide));
  if (threads != kThreads && (p->dtype != CBS_C64 || p->dirichlet || p->cdr))
    return fail(CBS_ERR_ARG, "wide column workgroups exist for FP32 periodic Helmholtz plans only");
  if (threads != p->col_threads32) {
    p->col_threads32 = threads;
    p->ctile.clear();  // every size back to the start width of this thread count
  }
  build_items(p);
  drop_graphs(p);
  CHK(upload_items(p, nullptr));
  HIPCHK(hipDeviceSynchronize());
  return CBS_OK;
}

cbs_status cbs_apply(cbs_plan p, const void* u, const void* s, void* y, void* stream) {
  if (!p || !y) return fail(CBS_ERR_ARG, "plan or y is NULL");
  if (y == u || y == s) return fail(CBS_ERR_ARG, "y must not alias u or s");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->cdr) {
    if (p->dtype == CBS_C64) return cdr_green_impl<float>(p, u, s, nullptr, y, EPI_STORE, nullptr, st);
    return cdr_green_impl<double>(p, u, s, nullptr, y, EPI_STORE, nullptr, st);
  }
  if (p->dtype == CBS_C64) {
    Params<float> q = base_params<float>(p);
    q.u = static_cast<const cpx<float>*>(u);
    q.s = static_cast<const cpx<float>*>(s);
    q.out = static_cast<cpx<float>*>(y);
    q.partials = nullptr;
    return run_pipeline(p, q, st);
  }
  Params<double> q = base_params<double>(p);
  q.u = static_cast<const cpx<double>*>(u);
  q.s = static_cast<const cpx<double>*>(s);
  q.out = static_cast<cpx<double>*>(y);
  q.partials = nullptr;
  return run_pipeline(p, q, st);
}

cbs_status cbs_residual(cbs_plan p, const void* u, const void* s, const void* rhs, void* r,
                        double* norm2, void* stream) {
  if (!p) return fail(CBS_ERR_ARG, "plan is NULL");
  if (r && (r == u || r == s)) return fail(CBS_ERR_ARG, "r must not alias u or s");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->cdr) {
    if (p->dtype == CBS_C64) return cdr_green_impl<float>(p, u, s, rhs, r, EPI_RESID, norm2, st);
    return cdr_green_impl<double>(p, u, s, rhs, r, EPI_RESID, norm2, st);
  }
  if (p->dtype == CBS_C64) return residual_impl<float>(p, u, s, rhs, r, norm2, st);
  return residual_impl<double>(p, u, s, rhs, r, norm2, st);
}

cbs_status cbs_helmholtz_residual(cbs_plan p, const void* u, const void* s, void* r, double* norm2,
                                  void* stream) {
  if (!p || !u) return fail(CBS_ERR_ARG, "plan or u is NULL");
  if (r && (r == u || r == s)) return fail(CBS_ERR_ARG, "r must not alias u or s");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return physical_norm2<float>(p, u, s, r, norm2, st);
  return physical_norm2<double>(p, u, s, r, norm2, st);
}

cbs_status cbs_npbs_step(cbs_plan p, void* u, const void* s, const void* wf, const void* wloc,
                         int count, void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "cbs_npbs_step is not available for convection-diffusion-reaction plans");
  if (!p || !u || !wf) return fail(CBS_ERR_ARG, "plan, u or wf is NULL");
  if (u == s || u == wf || u == wloc) return fail(CBS_ERR_ARG, "u must not alias s, wf or wloc");
  if (count < 1 || count > 1000000) return fail(CBS_ERR_ARG, "count must be in [1, 1e6]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return npbs_impl<float>(p, u, s, wf, wloc, count, st);
  return npbs_impl<double>(p, u, s, wf, wloc, count, st);
}

cbs_status cbs_sweep_checkpoints(cbs_plan p, void* u_all, const void* s, int count, void* stream) {
  if (p && p->cdr)
    return fail(CBS_ERR_ARG, "cbs_sweep_checkpoints is not available for convection-diffusion-reaction plans");
  if (!p || !u_all) return fail(CBS_ERR_ARG, "plan or u_all is NULL");
  if (count < 1 || count > 1000000) return fail(CBS_ERR_ARG, "count must be in [1, 1e6]");
  if (p->undamped) return fail(CBS_ERR_ARG, kNoGamma);
  const size_t bytes = size_t(p->cells) * p->op_elem() * (size_t(count) + 1);
  const char* lo = static_cast<const char*>(u_all);
  const char* sp = static_cast<const char*>(s);
  if (sp && sp >= lo && sp < lo + bytes) return fail(CBS_ERR_ARG, "s must not lie inside u_all");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return sweep_ckpt_impl<float>(p, u_all, s, count, st);
  return sweep_ckpt_impl<double>(p, u_all, s, count, st);
}

cbs_status cbs_sweep(cbs_plan p, void* u, const void* s, int count, double* norm2, void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "cbs_sweep is not available for convection-diffusion-reaction plans");
  if (!p || !u) return fail(CBS_ERR_ARG, "plan or u is NULL");
  if (u == s) return fail(CBS_ERR_ARG, "u must not alias s");
  if (count < 1 || count > 1000000) return fail(CBS_ERR_ARG, "count must be in [1, 1e6]");
  if (p->undamped) return fail(CBS_ERR_ARG, kNoGamma);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return sweep_impl<float>(p, u, s, count, norm2, st);
  return sweep_impl<double>(p, u, s, count, norm2, st);
}

cbs_status cbs_iterate(cbs_plan p, void* u, const void* s, int max_sweeps, double rtol,
                       int check_every, int stop, int32_t* iters, double* relres, int32_t* status,
                       int use_graph, void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "cbs_iterate is not available for convection-diffusion-reaction plans");
  if (!p || !u || !s) return fail(CBS_ERR_ARG, "plan, u or s is NULL");
  if (stop != CBS_STOP_BORN && stop != CBS_STOP_PHYSICAL)
    return fail(CBS_ERR_ARG, "stop must be CBS_STOP_BORN or CBS_STOP_PHYSICAL");
  if (u == s) return fail(CBS_ERR_ARG, "u must not alias s");
  if (max_sweeps < 0 || check_every < 2 || check_every > 100000 || !(rtol >= 0.0))
    return fail(CBS_ERR_ARG, "need max_sweeps >= 0, 2 <= check_every <= 1e5, rtol >= 0");
  if (p->undamped) return fail(CBS_ERR_ARG, kNoGamma);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (use_graph && st == nullptr) {
    // The legacy null stream cannot be captured: run on a plan-owned stream
    // ordered after everything already queued on the null stream.
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e1 = hipEventRecord(ev, nullptr);
    hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(p->own_stream, ev, 0) : e1;
    hipEventDestroy(ev);
    if (e2 != hipSuccess) return fail(CBS_ERR_HIP, std::string("stream ordering: ") + hipGetErrorString(e2));
    st = p->own_stream;
  }
  if (p->dtype == CBS_C64)
    return iterate_impl<float>(p, u, s, max_sweeps, rtol, check_every, stop, iters, relres, status,
                               use_graph, st);
  return iterate_impl<double>(p, u, s, max_sweeps, rtol, check_every, stop, iters, relres, status,
                              use_graph, st);
}

cbs_status fgmres_solve(cbs_plan p, void* u, const void* s, int restart, int inner_sweeps,
                        int max_iters, double rtol, int32_t* iters, double* relres,
                        int32_t* status, void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "fgmres_solve is not available for convection-diffusion-reaction plans");
  if (!p || !u || !s) return fail(CBS_ERR_ARG, "plan, u or s is NULL");
  if (u == s) return fail(CBS_ERR_ARG, "u must not alias s");
  if (restart < 1 || inner_sweeps < 0 || inner_sweeps > 1000 || max_iters < 0 || !(rtol >= 0.0))
    return fail(CBS_ERR_ARG, "need restart >= 1, 0 <= inner_sweeps <= 1000, max_iters >= 0, rtol >= 0");
  if (p->undamped && inner_sweeps > 0) return fail(CBS_ERR_ARG, kNoGamma);
  if (restart > p->max_restart)
    return fail(CBS_ERR_WORKSPACE, "restart " + std::to_string(restart) + " exceeds the plan's max_restart " +
                                       std::to_string(p->max_restart));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64)
    return fgmres_impl<float>(p, u, s, restart, inner_sweeps, max_iters, rtol, iters, relres, status, st);
  return fgmres_impl<double>(p, u, s, restart, inner_sweeps, max_iters, rtol, iters, relres, status, st);
}

cbs_status cbs_iterate_async(cbs_plan p, void* u, const void* s, int max_sweeps, double rtol,
                             int check_every, int stop, int32_t* iters, double* relres, int32_t* status,
                             void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "cbs_iterate_async is not available for convection-diffusion-reaction plans");
  if (!p || !u || !s) return fail(CBS_ERR_ARG, "plan, u or s is NULL");
  if (stop != CBS_STOP_BORN && stop != CBS_STOP_PHYSICAL)
    return fail(CBS_ERR_ARG, "stop must be CBS_STOP_BORN or CBS_STOP_PHYSICAL");
  if (u == s) return fail(CBS_ERR_ARG, "u must not alias s");
  if (max_sweeps < 0 || check_every < 2 || check_every > 100000 || !(rtol >= 0.0))
    return fail(CBS_ERR_ARG, "need max_sweeps >= 0, 2 <= check_every <= 1e5, rtol >= 0");
  if ((long long)max_sweeps / check_every > 100000)
    return fail(CBS_ERR_ARG, "max_sweeps / check_every must not exceed 1e5 chunks");
  if (p->undamped) return fail(CBS_ERR_ARG, kNoGamma);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64)
    return iterate_async_impl<float>(p, u, s, max_sweeps, rtol, check_every, stop, iters, relres, status, st);
  return iterate_async_impl<double>(p, u, s, max_sweeps, rtol, check_every, stop, iters, relres, status, st);
}

cbs_status fgmres_solve_async(cbs_plan p, void* u, const void* s, int restart, int inner_sweeps,
                              int max_iters, double rtol, int32_t* iters, double* relres, int32_t* status,
                              void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "fgmres_solve_async is not available for convection-diffusion-reaction plans");
  if (!p || !u || !s) return fail(CBS_ERR_ARG, "plan, u or s is NULL");
  if (u == s) return fail(CBS_ERR_ARG, "u must not alias s");
  if (restart < 1 || inner_sweeps < 0 || inner_sweeps > 1000 || max_iters < 0 || !(rtol >= 0.0))
    return fail(CBS_ERR_ARG, "need restart >= 1, 0 <= inner_sweeps <= 1000, max_iters >= 0, rtol >= 0");
  if (p->undamped && inner_sweeps > 0) return fail(CBS_ERR_ARG, kNoGamma);
  if (max_iters > 100000) return fail(CBS_ERR_ARG, "max_iters must not exceed 1e5");
  if (restart > p->max_restart)
    return fail(CBS_ERR_WORKSPACE, "restart " + std::to_string(restart) + " exceeds the plan's max_restart " +
                                       std::to_string(p->max_restart));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64)
    return fgmres_async_impl<float>(p, u, s, restart, inner_sweeps, max_iters, rtol, iters, relres, status, st);
  return fgmres_async_impl<double>(p, u, s, restart, inner_sweeps, max_iters, rtol, iters, relres, status, st);
}

cbs_status cbs_relres(cbs_plan p, const void* u, const void* s, int stop, double* relres, void* stream) {
  if (!p || !u || !s || !relres) return fail(CBS_ERR_ARG, "plan, u, s or relres is NULL");
  if (stop != CBS_STOP_BORN && stop != CBS_STOP_PHYSICAL)
    return fail(CBS_ERR_ARG, "stop must be CBS_STOP_BORN or CBS_STOP_PHYSICAL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return relres_impl<float>(p, u, s, stop, relres, st);
  return relres_impl<double>(p, u, s, stop, relres, st);
}

cbs_status cbs_metric_matched_grad(cbs_plan p, const void* x, const void* s, const double* scale,
                                   double* loss, void* grad, void* stream) {
  if (!p || !x || !grad) return fail(CBS_ERR_ARG, "plan, x or grad is NULL");
  if (grad == s) return fail(CBS_ERR_ARG, "grad must not alias s");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return mm_grad_impl<float>(p, x, s, scale, loss, grad, st);
  return mm_grad_impl<double>(p, x, s, scale, loss, grad, st);
}

cbs_status cbs_adjoint_step(cbs_plan p, const void* u_m, const void* s, const void* lam_in,
                            void* lam_out, void* grad_k2, void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "cbs_adjoint_step is not available for convection-diffusion-reaction plans");
  if (!p || !u_m || !lam_in || !lam_out || !grad_k2) return fail(CBS_ERR_ARG, "NULL argument");
  if (p->undamped) return fail(CBS_ERR_ARG, kNoGamma);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return adjoint_impl<float>(p, u_m, s, lam_in, lam_out, grad_k2, st);
  return adjoint_impl<double>(p, u_m, s, lam_in, lam_out, grad_k2, st);
}

cbs_status cbs_loss_seed(cbs_plan p, const void* u_k, const void* s, int weight_gamma, double* loss,
                         void* lam_out, void* grad_k2, void* stream) {
  if (p && p->cdr) return fail(CBS_ERR_ARG, "cbs_loss_seed is not available for convection-diffusion-reaction plans");
  if (!p || !u_k || !lam_out || !grad_k2) return fail(CBS_ERR_ARG, "NULL argument");
  if (weight_gamma < 0 || weight_gamma > 2)
    return fail(CBS_ERR_ARG, "weight must be 0 (W = 1), 1 (W = gamma) or 2 (physical residual)");
  if (p->undamped && weight_gamma == 1) return fail(CBS_ERR_ARG, kNoGamma);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == CBS_C64) return seed_impl<float>(p, u_k, s, weight_gamma, loss, lam_out, grad_k2, st);
  return seed_impl<double>(p, u_k, s, weight_gamma, loss, lam_out, grad_k2, st);
}

cbs_status cbs_autotune(cbs_plan p, int32_t* tiles, void* stream) {
  if (!p) return fail(CBS_ERR_ARG, "plan is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::ostringstream rec;
  cbs_status rc = p->cdr ? tune_by_columns(p, st, rec)
                  : p->dtype == CBS_C64 ? tune_by_sweeps<float>(p, st, rec)
                                        : tune_by_sweeps<double>(p, st, rec);
  if (rc != CBS_OK) return rc;
  build_items(p);
  drop_graphs(p);
  CHK(upload_items(p, st));
  HIPCHK(hipStreamSynchronize(st));
  if (const char* path = std::getenv("CBS_AUTOTUNE_CACHE")) {
    std::ofstream f(path, std::ios::app);
    if (f) f << rec.str() << "\n";
  }
  if (tiles)
    for (int i = 0; i < p->batch; ++i) tiles[i] = p->dtype == CBS_C64 ? p->inst[i].ctile : p->inst[i].ctile64;
  return CBS_OK;
}

void cbs_destroy(cbs_plan p) {
  if (!p) return;
  free_plan(p);
  delete p;
}

}  // extern "C"
