// cbs_apply_static: y = G (V u + s) without a plan and without allocating.
//
// The operator is the one cbs_apply runs (Sec. 4.1, the Born fixed-point map;
// symbol and grid as in App. D), on the same row / column / row kernels.  What
// a plan keeps in its own memory -- the instance descriptors, the row and
// column work lists, the twiddle tables and the spectral buffer between the
// transform passes -- lives here in one file-scope device array, `scratch`,
// of fixed size.  Each call rewrites every part of it it reads (one setup
// kernel, then the three transform launches, all on the caller's stream), so
// nothing has to start at zero.  Calls that overlap on one GPU share the
// array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/cbs.h"
#include "launch.hpp"
#include "params.hpp"

namespace cbs {
namespace {

constexpr int kMaxBatch = CBS_STATIC_MAX_BATCH;
constexpr size_t kSpecBytes = size_t(CBS_STATIC_MAX_BYTES);
constexpr int kMaxItems = kMaxBatch * 1024;  // rows or column tiles of kMaxBatch instances of 1024

// Byte offsets of the parts of `scratch`, each on a 256-byte boundary.
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffTw32 = kSpecBytes;
constexpr size_t kOffTw64 = kOffTw32 + align256(size_t(kTwTotal) * sizeof(cpx<float>));
constexpr size_t kOffInst = kOffTw64 + align256(size_t(kTwTotal) * sizeof(cpx<double>));
constexpr size_t kOffRows = kOffInst + align256(kMaxBatch * sizeof(InstDesc));
constexpr size_t kOffCols = kOffRows + align256(kMaxItems * sizeof(int2));
constexpr size_t kScratchBytes = kOffCols + align256(kMaxItems * sizeof(int2));

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Everything the setup kernel needs, passed by value (no host-to-device copy).
struct StaticSetup {
  int batch;
  int elem;                  // bytes per complex element of the column kernels (8 or 16)
  int order[kMaxBatch];      // instances, largest first
  int n[kMaxBatch];
  int ctile[kMaxBatch];      // column tile width of the kernels that run (FP32 or FP64)
  int row_first[kMaxBatch];  // first row item of instance order[k]
  int col_first[kMaxBatch];  // first column item of instance order[k]
  long long off[kMaxBatch];
  double k0sq[kMaxBatch], eps[kMaxBatch];
  int nrows, ncols;
};

__device__ int size_index(int idx, int& o) {
  // segment of the concatenated twiddle tables that holds entry idx
  const int sizes[] = {16, 32, 64, 128, 192, 256, 288, 384, 512, 1024};
  for (int i = 9; i >= 0; --i)
    if (idx >= tw_offset(sizes[i])) {
      o = tw_offset(sizes[i]);
      return sizes[i];
    }
  o = 0;
  return sizes[0];
}

// Grid-stride over max(kTwTotal, items): the twiddle tables w^(q k) of every
// pass of every size (FP64, exponent reduced exactly, FP32 rounded from it),
// the instance descriptors and both work lists.
__global__ __launch_bounds__(256) void k_static_setup(StaticSetup a, unsigned char* base) {
  cpx<float>* tw32 = reinterpret_cast<cpx<float>*>(base + kOffTw32);
  cpx<double>* tw64 = reinterpret_cast<cpx<double>*>(base + kOffTw64);
  InstDesc* inst = reinterpret_cast<InstDesc*>(base + kOffInst);
  int2* rows = reinterpret_cast<int2*>(base + kOffRows);
  int2* cols = reinterpret_cast<int2*>(base + kOffCols);
  const int total = max(kTwTotal, max(a.nrows, a.ncols));
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    if (idx < kTwTotal) {
      int o = 0;
      const int nn = size_index(idx, o);
      int pass = 0;
      while (pass + 1 < plan_passes(nn) && idx >= tw_pass_offset(nn, pass + 1)) ++pass;
      o = tw_pass_offset(nn, pass);
      const int ns = plan_ns(nn, pass), rad = plan_radix(nn, pass), rp = radp(rad);
      const int k = (idx - o) / rp, q = (idx - o) % rp;
      cpx<double> w{0.0, 0.0};
      if (q < rad) {
        const long long m = ((long long)q * k) % ((long long)ns * rad);
        const double ang = -2.0 * M_PI * double(m) / double(ns * rad);
        w = cpx<double>{cos(ang), sin(ang)};
      }
      tw64[idx] = w;
      tw32[idx] = cpx<float>{float(w.x), float(w.y)};
    }
    if (idx < a.batch) {
      InstDesc d{};
      d.off = a.off[idx];
      d.n = a.n[idx];
      d.k0sq = a.k0sq[idx];
      d.eps = a.eps[idx];
      d.kind = KIND_PERIODIC;
      d.rpw = row_rpw(d.n);
      d.nparts = (d.n + d.rpw - 1) / d.rpw;
      d.part_off = 0;  // no partial sums: apply has no norm
      d.ctile = a.ctile[idx];
      d.ctile64 = a.ctile[idx];
      d.vx0 = d.vy0 = 0.0;
      inst[idx] = d;
    }
    // work lists in the order cbs_setup builds them: largest instances
    // first; the column tiles that share 128-byte lines placed 8 positions
    // apart (workgroups are dispatched round-robin over the 8 XCDs)
    for (int k = 0; k < a.batch; ++k) {
      const int i = a.order[k], n = a.n[i];
      const int rpw = row_rpw(n), nr = (n + rpw - 1) / rpw;
      if (idx >= a.row_first[k] && idx < a.row_first[k] + nr)
        rows[idx] = int2{i, (idx - a.row_first[k]) * rpw};
      const int c = a.ctile[i], nt = n / c;
      if (idx >= a.col_first[k] && idx < a.col_first[k] + nt) {
        const int p = idx - a.col_first[k];
        const int g = max(1, 128 / (c * a.elem)), blk = 8 * g;
        int t = p;
        if (p < nt / blk * blk) {
          const int b = p / blk * blk, r = p - b;
          t = b + (r % 8) * g + r / 8;
        }
        cols[idx] = int2{i, t * c};
      }
    }
  }
}

cbs_status sfail(cbs_status st, const std::string& m) { return report_error(st, m); }

// Device address of `scratch` per device (taken once per device).
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

cbs_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sfail(CBS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return sfail(CBS_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return sfail(CBS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return CBS_OK;
}

template <typename R>
cbs_status run_static(unsigned char* base, const StaticSetup& a, size_t col_lds, const void* k2,
                      const void* u, const void* s, void* y, hipStream_t st) {
  Params<R> q{};
  q.inst = reinterpret_cast<const InstDesc*>(base + kOffInst);
  q.k2 = static_cast<const cpx<R>*>(k2);
  q.inter = reinterpret_cast<cpx<R>*>(base);
  if constexpr (sizeof(R) == 4) q.tw = reinterpret_cast<const cpx<float>*>(base + kOffTw32);
  else q.tw = reinterpret_cast<const cpx<double>*>(base + kOffTw64);
  q.u = static_cast<const cpx<R>*>(u);
  q.s = static_cast<const cpx<R>*>(s);
  q.out = static_cast<cpx<R>*>(y);
  q.partials = nullptr;
  q.mask = nullptr;
  q.pro = PRO_VU_S;
  q.sym = SYM_GREEN;
  q.epi = EPI_STORE;
  q.items = reinterpret_cast<const int2*>(base + kOffRows);
  launch_row(0, a.nrows, st, q);
  Params<R> c = q;
  c.items = reinterpret_cast<const int2*>(base + kOffCols);
  launch_col(a.ncols, col_lds, st, c);
  launch_row(1, a.nrows, st, q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return sfail(CBS_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  return CBS_OK;
}

bool periodic_size(int n) {
  switch (n) {
#define CBS_SUP(N) case N:
    CBS_FOR_EACH_N(CBS_SUP)
#undef CBS_SUP
    return true;
    default:
      return false;
  }
}

}  // namespace
}  // namespace cbs

using namespace cbs;

extern "C" {

cbs_status cbs_apply_static(int batch, const int32_t* n, const void* k2, const double* k0sq,
                            const double* eps, int dtype, const void* u, const void* s, void* y,
                            void* stream) {
  if (batch < 1 || batch > kMaxBatch)
    return sfail(CBS_ERR_ARG, "batch must be in [1, " + std::to_string(kMaxBatch) + "]");
  if (!n || !k2 || !k0sq || !eps || !y) return sfail(CBS_ERR_ARG, "n, k2, k0sq, eps or y is NULL");
  if (dtype != CBS_C64 && dtype != CBS_C128) return sfail(CBS_ERR_ARG, "dtype must be CBS_C64 or CBS_C128");
  if (y == u || y == s) return sfail(CBS_ERR_ARG, "y must not alias u or s");
  const int elem = dtype == CBS_C64 ? 8 : 16;
  StaticSetup a{};
  a.batch = batch;
  a.elem = elem;
  long long cells = 0;
  for (int i = 0; i < batch; ++i) {
    if (!periodic_size(n[i]))
      return sfail(CBS_ERR_SIZE, "unsupported grid size " + std::to_string(n[i]) + " (instance " +
                                     std::to_string(i) + ")");
    if (!std::isfinite(k0sq[i]) || !std::isfinite(eps[i]) || !(eps[i] > 0.0))
      return sfail(CBS_ERR_ARG, "k0sq must be finite and eps finite and > 0 (instance " + std::to_string(i) + ")");
    a.n[i] = n[i];
    a.off[i] = cells;
    a.k0sq[i] = k0sq[i];
    a.eps[i] = eps[i];
    // the width a plan starts with, reduced as a plan reduces it for FP64
    int c = col_tile_start(n[i]);
    while (!col_tile_valid(n[i], c, 16) && elem == 16 && c > 2) c /= 2;
    a.ctile[i] = c;
    cells += (long long)n[i] * n[i];
  }
  if (size_t(cells) * size_t(elem) > kSpecBytes)
    return sfail(CBS_ERR_WORKSPACE, std::to_string(cells) + " cells exceed the fixed scratch of " +
                                        std::to_string(kSpecBytes) + " bytes (" +
                                        std::to_string(kSpecBytes / elem) + " cells at this dtype)");
  // largest first, stable, as the planner orders its work lists
  for (int i = 0; i < batch; ++i) a.order[i] = i;
  for (int i = 1; i < batch; ++i)
    for (int j = i; j > 0 && a.n[a.order[j]] > a.n[a.order[j - 1]]; --j) std::swap(a.order[j], a.order[j - 1]);
  size_t col_lds = 0;
  for (int k = 0; k < batch; ++k) {
    const int i = a.order[k];
    a.row_first[k] = a.nrows;
    a.col_first[k] = a.ncols;
    a.nrows += (a.n[i] + row_rpw(a.n[i]) - 1) / row_rpw(a.n[i]);
    a.ncols += a.n[i] / a.ctile[i];
    col_lds = std::max(col_lds, size_t(col_lds_elems(a.n[i], a.ctile[i])) * elem);
  }
  void* base = nullptr;
  cbs_status rc = scratch_address(&base);
  if (rc != CBS_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int total = std::max(kTwTotal, std::max(a.nrows, a.ncols));
  hipLaunchKernelGGL(k_static_setup, dim3((total + 255) / 256), dim3(256), 0, st, a,
                     static_cast<unsigned char*>(base));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return sfail(CBS_ERR_HIP, std::string("setup launch: ") + hipGetErrorString(e));
  unsigned char* b = static_cast<unsigned char*>(base);
  if (dtype == CBS_C64) return run_static<float>(b, a, col_lds, k2, u, s, y, st);
  return run_static<double>(b, a, col_lds, k2, u, s, y, st);
}

}  // extern "C"
