// Data structures shared by the host planner and the GPU kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace cbs {

#define CBS_FOR_EACH_N(X) X(16) X(32) X(64) X(128) X(192) X(256) X(288) X(384) X(512) X(1024)

constexpr int kThreads = 256;
constexpr int kRowLds = 2304;  // complex elements per row-kernel workgroup (2048 + skew)

// Threads per row transform and rows per row-kernel workgroup.
__host__ __device__ constexpr int row_tpf(int n) { return n / 8; }
__host__ __device__ constexpr int row_rpw(int n) {
  return (kThreads / row_tpf(n)) < n ? (kThreads / row_tpf(n)) : n;
}

// Instance kinds: periodic N x N grid (FFT, App. D) or the n x n interior of
// a unit square with homogeneous Dirichlet boundaries (five-point FD, DST-I,
// App. C "Newton linear systems").
enum InstKind { KIND_PERIODIC = 0, KIND_DIRICHLET = 1, KIND_CDR = 2 };

// Length of the FFT that carries a DST-I of length n (odd extension).
__host__ __device__ constexpr int dst_len(int n) { return 2 * (n + 1); }

struct InstDesc {
  long long off;  // element offset of the instance in packed fields
  int n;          // field size n x n
  int part_off;   // first partial-sum slot (one per row work item)
  int nparts;
  int ctile;      // column tile width: FP32 kernels (ctile) and FP64 kernels (ctile64)
  int ctile64;
  int kind;       // InstKind
  int rpw;        // rows per row work item
  double k0sq;    // Helmholtz: k0^2; CDR: kappa0
  double eps;     // Helmholtz: eta; CDR: sigma0
  double vx0, vy0;  // CDR: background velocity (x = fast axis), zero otherwise
};

enum Pro { PRO_VU_S = 0, PRO_CONJG_A = 1, PRO_SEED = 2, PRO_U = 3, PRO_A = 4 };
// SYM_CDR*: convection-diffusion-reaction plans, L0(xi) = kappa0 |xi|^2 +
// i v0 . xi + sigma0: 1/L0, 1/conj(L0) and -L0 (each with the 1/N^2 of the
// inverse transform)
enum Sym {
  SYM_GREEN = 0,
  SYM_GREEN_CONJ = 1,
  SYM_LAP = 2,
  SYM_TABLE = 3,
  SYM_CDR = 4,
  SYM_CDR_CONJ = 5,
  SYM_CDR_NEG_L0 = 6
};
enum Epi {
  EPI_STORE = 0,
  EPI_RESID = 1,
  EPI_SWEEP = 2,
  EPI_BZ_WIDE = 3,
  EPI_ADJ = 4,
  EPI_SEED = 5,
  EPI_LAP = 6,
  EPI_PHYS_SEED = 7,
  EPI_NPBS = 8,
  EPI_BORN_ADJ = 9  // out = a - conj(V) z: R^H a for R = I - G V, z = G^H a
};
// Instance masks: which status values let an instance run.
enum MaskMode { MASK_RUNNING = 0, MASK_NOT_FINAL = 1, MASK_NONZERO = 2 };
enum InstStatus { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXIT = 2, ST_DIVERGED = 3, ST_PENDING = 4 };

struct IterState {
  int* status;
  int* iters;
  int* chunk_active;
  double* relres;   // FP64-verified relative residual
  double* est;      // latest FP32 estimate
  double* bnorm;    // ||G s|| per instance
  const double* rtol;
  const int* max_sweeps;
};

template <typename R>
struct Params {
  const InstDesc* inst;
  const int2* items;
  const cpx<R>* k2;
  const cpx<R>* tw;
  const cpx<R>* u;
  const cpx<R>* s;
  const cpx<R>* rhs;
  const cpx<R>* a;
  const cpx<R>* b;
  const cpx<R>* table;  // SYM_TABLE: spectral weights on the DFT bins (packed like fields)
  const double* mu;     // Dirichlet plans: M^2 sin^2(pi p / M) per transform length M
  cpx<R>* inter;
  // dual != 0 (the adjoint step of periodic plans): each launch also
  // transforms a second field, spectral buffer inter2 (rows: MODE 5 / 6;
  // columns: the conjugate Green symbol)
  cpx<R>* inter2;
  int dual;
  cpx<R>* out;
  cpx<R>* out2;
  cpx<float>* out_narrow;
  cpx<double>* out_wide;
  double* partials;
  const int* mask;
  int mask_mode;
  int pro, sym, epi;
  int weight_gamma;
  // check != 0: the workgroup of each instance's first column tile also
  // runs the FP32 convergence check of the sweep that the previous row
  // launch finished (k_col only)
  IterState chk;
  int check;
  int dst;  // nonzero: Dirichlet plan (DST-I kernels)
  int col_threads;  // threads per column workgroup: kThreads or kColThreadsWide (FP32 periodic)
  // convection-diffusion-reaction passes: k2 holds (dkappa, dsigma), k2b
  // (dvx, dvy)
  const cpx<R>* k2b;
};


// ---- column tiles ------------------------------------------------------------------
//
// Column tile of c columns in LDS: element-interleaved, position x of column
// k at c * pos(x) + k.
__host__ __device__ constexpr int col_lds_elems(int n, int c) { return c * lds_len(n); }
constexpr int kColLdsBytes = 64 * 1024;
// Default tile: about 2048 elements per workgroup (C * n ~ 8 elements per thread).
__host__ __device__ constexpr int col_tile_default(int n) {
  int c = 2;
  while (c * 2 <= 32 && c * 2 * n <= 2048 && n % (c * 2) == 0) c *= 2;
  return c;
}
// Width a plan starts with before any cbs_autotune: the width the autotuner
// settles on for that size on MI355X (ragged 128..512 batch, 8 x 1024^2), the
// default elsewhere.  Always one of the compiled widths.
__host__ __device__ constexpr int col_tile_start(int n) {
  return (n == 128 || n == 192 || n == 256 || n == 512) ? 8
         : (n == 384 || n == 1024)                      ? 4
                                                         : col_tile_default(n);
}
// Tiles a kernel is compiled for at size n: the default, half and double.
__host__ __device__ constexpr bool col_tile_valid(int n, int c, int elem_bytes) {
  const int c0 = col_tile_default(n);
  return (c == c0 || c == c0 / 2 || c == c0 * 2) && c >= 2 && c <= 32 && n % c == 0 &&
         col_lds_elems(n, c) * elem_bytes <= kColLdsBytes;
}

// Column kernels of FP32 periodic Helmholtz plans also come with twice the
// threads per workgroup (kColThreadsWide): one radix-8 butterfly per thread
// and pass at the default-or-double width, fewer registers per thread and so
// more waves per SIMD.  A plan uses one thread count for all its column
// launches (every instance of a lane shares a launch).
constexpr int kColThreadsWide = 2 * kThreads;
__host__ __device__ constexpr bool col_tile_valid_t(int n, int c, int elem_bytes, int threads) {
  if (threads == kThreads) return col_tile_valid(n, c, elem_bytes);
  const int c0 = col_tile_default(n);
  return threads == kColThreadsWide && (c == c0 || c == c0 * 2) && c >= 2 && c <= 32 && n % c == 0 &&
         col_lds_elems(n, c) * elem_bytes <= kColLdsBytes;
}
// Width a plan starts with at a given thread count.
__host__ __device__ constexpr int col_tile_start_t(int n, int threads) {
  return threads == kThreads ? col_tile_start(n)
         : col_tile_valid_t(n, col_tile_default(n) * 2, 8, threads) ? col_tile_default(n) * 2
                                                                    : col_tile_default(n);
}

// Dirichlet eigenvalue table: for each supported transform length M the
// values M^2 sin^2(pi p / M), p = 0..M-1, back to back.
__host__ __device__ constexpr int mu_offset(int m) {
  int off = 0;
  const int sizes[] = {16, 32, 64, 128, 192, 256, 288, 384, 512, 1024};
  for (int i = 0; i < 10; ++i) {
    if (sizes[i] == m) return off;
    off += sizes[i];
  }
  return -1;
}
// The Dirichlet size without an FFT plan for its odd extension (2(n+1) =
// 130 = 2 5 13): n = 64, the grid of the paper's Newton experiments.  Its
// DST-I is formed directly; the eigenvalue table of length M = 130 and
// sin(pi m / (n+1)), m < M, follow the tables of the FFT lengths.
constexpr int kDstDirectN = 64;
constexpr int kDstDirectM = dst_len(kDstDirectN);
// Its row kernels give each row 32 threads (two outputs each), 8 rows per
// workgroup: the direct sums are serial in the row length, so short chains
// and more workgroups beat the FFT rows' 8 threads per row.
constexpr int kDstDirectTPF = 32;
constexpr int kDstDirectRPW = kThreads / kDstDirectTPF;
constexpr int kMuDirect = mu_offset(1024) + 1024;
constexpr int kSinDirect = kMuDirect + kDstDirectM;
constexpr int kMuTotal = kSinDirect + kDstDirectM;

enum PwOp {
  PW_GAMMA = 0,        // e_out = gamma * e_in
  PW_FIRST64 = 1,      // c_out = (R)(src64 * scale[instance]); e_out = gamma * c_out (scale NULL: 1)
  PW_ADD_WIDE = 2,     // x64 += e_in
  PW_WIDEN = 3,        // x64 = e_in
  PW_NARROW = 4,       // e_out = (R)(x64 * scale[instance]) (scale NULL: 1)
  PW_SCALE64 = 5,      // x64 *= scale[instance] (FP64)
  PW_SCALE = 6         // e_out = e_in * factor * scale[instance] (scale NULL: 1), operator precision
};

template <typename R>
struct PwParams {
  const InstDesc* inst;
  const int2* items;
  const cpx<R>* k2;
  const cpx<double>* src64;
  cpx<double>* x64;
  const cpx<R>* e_in;
  cpx<R>* e_out;
  cpx<R>* c_out;
  const double* scale;  // per-instance factor for PW_SCALE64 / PW_SCALE / PW_FIRST64 / PW_NARROW
  double factor;        // constant factor of PW_SCALE
  const int* mask;
  int mask_mode;
  int op;
};


// Largest FGMRES restart length a plan accepts.
constexpr int kMaxRestart = 200;

struct KryLayout {
  int m;
  __host__ __device__ long long h(int r, int c) const { return 2LL * (r * m + c); }
  __host__ __device__ long long cs() const { return 2LL * (m + 1) * m; }
  __host__ __device__ long long sn() const { return cs() + m; }
  __host__ __device__ long long g() const { return sn() + 2LL * m; }
  __host__ __device__ long long y() const { return g() + 2LL * (m + 1); }
  __host__ __device__ long long coef() const { return y() + 2LL * m; }
  __host__ __device__ long long coefs() const { return coef() + 2LL * (m + 1); }
  __host__ __device__ long long sc() const { return coefs() + 2LL * (m + 1); }
  __host__ __device__ long long size() const { return sc() + 8; }
};

struct KryParams {
  const InstDesc* inst;
  const int2* items;
  const cpx<double>* vbasis;  // (m+1) fields of `cells` elements
  long long cells;
  cpx<double>* w;             // vector being orthogonalised
  double* kry;                // per-instance state, stride kstride
  long long kstride;
  int m;
  int j;                      // current Arnoldi column
  double* dots;               // per partial slot: dstride doubles of partial dot products
  long long dstride;          // 4 (m + 1) + 4: t, s (m + 1 complex each), alpha and <u, w>
  double* partials;           // per partial slot: one double
  double* scale;              // per instance
  int* active;                // per instance: 1 while in the Arnoldi cycle
  int* jend;                  // per instance: Arnoldi steps done this cycle
  int* iters;                 // per instance: total Arnoldi steps
  int* status;                // per instance: solver status
  double* relres;             // per instance: last FP64 true relative residual
  const double* rtol;
  const int* max_iters;
};


}  // namespace cbs
