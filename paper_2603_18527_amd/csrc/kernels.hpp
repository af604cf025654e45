// HIP kernels of the CBS operator for gfx950.
//
// One application y = G(V u + s) is three launches over a ragged work list
// that covers every instance of the batch:
//   k_row_fwd : load a block of rows, form q (prologue), forward row FFTs in
//               LDS, write the half-transformed rows to the spectral buffer;
//   k_col     : load a tile of C full columns, forward column FFTs, multiply by
//               the Green symbol 1/(N^2 lambda) computed in FP64 from the
//               Fourier indices, inverse column FFTs, write back in place;
//   k_row_inv : load rows, inverse row FFTs, epilogue (store, Born residual,
//               CBS update, adjoint step ...) with per-block FP64 partial
//               sums of |r|^2.
// The prologue/epilogue/symbol variants are selected by uniform runtime modes.
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

struct InstDesc {
  long long off;  // element offset of the instance in packed fields
  int n;
  int part_off;  // first partial-sum slot (one per row work item)
  int nparts;
  int pad;
  double k0sq;
  double eps;
};

enum Pro { PRO_VU_S = 0, PRO_CONJG_A = 1, PRO_SEED = 2, PRO_U = 3 };
enum Sym { SYM_GREEN = 0, SYM_GREEN_CONJ = 1, SYM_LAP = 2 };
enum Epi {
  EPI_STORE = 0,
  EPI_RESID = 1,
  EPI_SWEEP = 2,
  EPI_BZ_WIDE = 3,
  EPI_ADJ = 4,
  EPI_SEED = 5,
  EPI_LAP = 6
};
// Instance masks: which status values let an instance run.
enum MaskMode { MASK_RUNNING = 0, MASK_NOT_FINAL = 1, MASK_NONZERO = 2 };
enum InstStatus { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXIT = 2, ST_DIVERGED = 3, ST_PENDING = 4 };

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
  cpx<R>* inter;
  cpx<R>* out;
  cpx<R>* out2;
  cpx<float>* out_narrow;
  cpx<double>* out_wide;
  double* partials;
  const int* mask;
  int mask_mode;
  int pro, sym, epi;
  int weight_gamma;
};

__device__ __forceinline__ bool inst_enabled(const int* mask, int mode, int i) {
  if (!mask) return true;
  const int m = mask[i];
  if (mode == MASK_RUNNING) return m == ST_RUNNING;
  if (mode == MASK_NOT_FINAL) return m == ST_RUNNING || m == ST_PENDING;
  return m != 0;
}

template <typename R>
__device__ __forceinline__ cpx<R> ld_or_zero(const cpx<R>* p, long long i) {
  return p ? p[i] : cpx<R>{R(0), R(0)};
}

template <typename R>
struct Coef {
  cpx<R> v;    // V = k^2 - k0^2 - i eps
  R inv_eps;
  __device__ __forceinline__ cpx<R> gamma() const { return {-v.y * inv_eps, v.x * inv_eps}; }
  __device__ __forceinline__ cpx<R> gamma_conj() const { return {-v.y * inv_eps, -v.x * inv_eps}; }
};

template <typename R>
__device__ __forceinline__ Coef<R> coef(const Params<R>& p, const InstDesc& d, long long i) {
  const cpx<R> k = p.k2[i];
  Coef<R> c;
  c.v = {k.x - R(d.k0sq), k.y - R(d.eps)};
  c.inv_eps = R(1.0 / d.eps);
  return c;
}

template <typename R>
__device__ __forceinline__ cpx<R> prologue(const Params<R>& p, const InstDesc& d, long long i) {
  switch (p.pro) {
    case PRO_VU_S: {
      cpx<R> q = ld_or_zero(p.s, i);
      if (p.u) {
        const Coef<R> c = coef(p, d, i);
        q = q + cmul(c.v, p.u[i]);
      }
      return q;
    }
    case PRO_CONJG_A: {
      const Coef<R> c = coef(p, d, i);
      return cmul(c.gamma_conj(), p.a[i]);
    }
    case PRO_SEED: {
      // conj(W) * 2 W r = 2 |W|^2 r
      R w2 = R(1);
      if (p.weight_gamma) {
        const Coef<R> c = coef(p, d, i);
        w2 = cabs2(c.v) * c.inv_eps * c.inv_eps;
      }
      return cscale(p.a[i], R(2) * w2);
    }
    default:  // PRO_U
      return p.u[i];
  }
}

// Epilogue for one cell; returns the value whose squared modulus enters the
// per-instance sum (zero when the mode has no norm).
template <typename R>
__device__ __forceinline__ double epilogue(const Params<R>& p, const InstDesc& d, long long i,
                                           cpx<R> z) {
  switch (p.epi) {
    case EPI_STORE:
      p.out[i] = z;
      return 0.0;
    case EPI_RESID: {
      const cpx<R> r = z - ld_or_zero(p.u, i) + ld_or_zero(p.rhs, i);
      if (p.out) p.out[i] = r;
      if (p.out_narrow) p.out_narrow[i] = cpx<float>{float(r.x), float(r.y)};
      return double(cabs2(r));
    }
    case EPI_SWEEP: {
      const cpx<R> u = p.u[i];
      const cpx<R> r = z - u + ld_or_zero(p.rhs, i);
      const Coef<R> c = coef(p, d, i);
      p.out[i] = u + cmul(c.gamma(), r);
      return double(cabs2(r));
    }
    case EPI_BZ_WIDE: {
      const cpx<R> w = p.u[i] - z;
      p.out_wide[i] = cpx<double>{double(w.x), double(w.y)};
      return 0.0;
    }
    case EPI_ADJ: {
      // t = z = G^H(conj(gamma) lam); lam_out = lam + conj(V) t - conj(gamma) lam
      // grad += (-i/eps) lam conj(r) + t conj(u)
      const Coef<R> c = coef(p, d, i);
      const cpx<R> lam = p.a[i];
      const cpx<R> r = p.b[i];
      const cpx<R> u = p.u[i];
      const cpx<R> gl = cmul(c.gamma_conj(), lam);
      p.out[i] = lam + cmulc(c.v, z) - gl;
      const cpx<R> lr = cmul(lam, cconj(r));
      const cpx<R> g0 = cpx<R>{lr.y * c.inv_eps, -lr.x * c.inv_eps};
      p.out2[i] = p.out2[i] + g0 + cmul(z, cconj(u));
      return 0.0;
    }
    case EPI_SEED: {
      // r = a (Born residual of u_K); gr = 2|W|^2 r; lam_K = conj(V) t - gr;
      // grad += t conj(u) [+ (2/eps^2) V |r|^2 when W = gamma]; loss term |W r|^2
      const Coef<R> c = coef(p, d, i);
      const cpx<R> r = p.a[i];
      const cpx<R> u = p.u[i];
      const R r2 = cabs2(r);
      R w2 = R(1);
      if (p.weight_gamma) w2 = cabs2(c.v) * c.inv_eps * c.inv_eps;
      const cpx<R> gr = cscale(r, R(2) * w2);
      p.out[i] = cmulc(c.v, z) - gr;
      cpx<R> g = cmul(z, cconj(u));
      if (p.weight_gamma) g = g + cscale(c.v, R(2) * c.inv_eps * c.inv_eps * r2);
      p.out2[i] = p.out2[i] + g;
      return double(w2) * double(r2);
    }
    default: {  // EPI_LAP: physical residual s - A u with A u = -Lap u - k^2 u
      const cpx<R> u = p.u[i];
      const cpx<R> au = z - cmul(p.k2[i], u);
      const cpx<R> r = ld_or_zero(p.s, i) - au;
      if (p.out) p.out[i] = r;
      return double(cabs2(r));
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup sum of one double per thread (all threads must call).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  }
  return s;
}

// ---- row kernels ---------------------------------------------------------------
//
// A row work item is (instance, first row); it covers row_rpw(N) rows (fewer at
// the bottom edge).  Thread tid works on row tid / TPF of the tile.  The first
// FFT pass reads straight from global memory (with the prologue) and the last
// pass writes straight to global memory (with the epilogue); both access
// patterns are contiguous across the threads of a row.  Only the exchanges
// between passes go through LDS (rows at stride lds_len(N), skewed).

template <int N>
struct RowTile {
  static constexpr int TPF = row_tpf(N);
  static constexpr int RPW = row_rpw(N);
  static constexpr int RS = lds_len(N);
  static_assert(RPW * RS <= kRowLds, "row tile does not fit");
};

// MODE 0: prologue + forward rows -> spectral buffer;
// MODE 1: spectral buffer -> inverse rows -> epilogue (with partial norms);
// MODE 2: spectral buffer -> inverse rows -> sweep epilogue u += gamma r
//         (written to global) -> next sweep's prologue V u + s formed from
//         the value just computed -> forward rows -> spectral buffer.
template <typename R, int N, int MODE>
__device__ __forceinline__ void row_body(const Params<R>& p, const InstDesc& d, int row0,
                                         cpx<R>* lds, double* red) {
  using T = RowTile<N>;
  const int tid = threadIdx.x;
  const int r = tid / T::TPF, t = tid - r * T::TPF;
  const int nrows = min(T::RPW, N - row0);
  const bool active = r < nrows;
  const long long rbase = d.off + (long long)(row0 + (active ? r : 0)) * N;
  cpx<R>* mine = lds + (active ? r : 0) * T::RS;
  if constexpr (MODE == 0) {
    auto ld = [&](int e) { return prologue(p, d, rbase + e); };
    auto st = [&](int e, cpx<R> v) { p.inter[rbase + e] = v; };
    fft_run<R, N, T::TPF, -1, false, false>(mine, t, active, p.tw, ld, st);
  } else if constexpr (MODE == 1) {
    double acc = 0.0;
    auto ld = [&](int e) { return p.inter[rbase + e]; };
    auto st = [&](int e, cpx<R> v) { acc += epilogue(p, d, rbase + e, v); };
    fft_run<R, N, T::TPF, 1, false, false>(mine, t, active, p.tw, ld, st);
    if (p.partials) {
      const double s = block_sum(acc, red);
      if (tid == 0) p.partials[d.part_off + row0 / T::RPW] = s;
    }
  } else {
    double acc = 0.0;
    auto ld = [&](int e) { return p.inter[rbase + e]; };
    auto st = [&](int e, cpx<R> z) {
      const long long g = rbase + e;
      const cpx<R> u = p.u[g];
      const cpx<R> rres = z - u + ld_or_zero(p.rhs, g);
      const Coef<R> c = coef(p, d, g);
      const cpx<R> un = u + cmul(c.gamma(), rres);
      p.out[g] = un;
      acc += double(cabs2(rres));
      mine[lds_pos(e)] = cmul(c.v, un) + ld_or_zero(p.s, g);
    };
    fft_run<R, N, T::TPF, 1, false, true>(mine, t, active, p.tw, ld, st);
    if (p.partials) {
      const double s = block_sum(acc, red);
      if (tid == 0) p.partials[d.part_off + row0 / T::RPW] = s;
    }
    auto ld2 = [&](int e) { return mine[lds_pos(e)]; };
    auto st2 = [&](int e, cpx<R> v) { p.inter[rbase + e] = v; };
    fft_run<R, N, T::TPF, -1, true, false>(mine, t, active, p.tw, ld2, st2);
  }
}

template <typename R, int MODE>
__device__ __forceinline__ void row_dispatch(const Params<R>& p) {
  __shared__ cpx<R> lds[kRowLds];
  __shared__ double red[kThreads / 64];
  const int2 w = p.items[blockIdx.x];
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  const InstDesc d = p.inst[w.x];
  switch (d.n) {
#define CBS_ROW_CASE(N) \
  case N:               \
    row_body<R, N, MODE>(p, d, w.y, lds, red); \
    break;
    CBS_FOR_EACH_N(CBS_ROW_CASE)
#undef CBS_ROW_CASE
    default:
      break;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_fwd(Params<R> p) {
  row_dispatch<R, 0>(p);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_inv(Params<R> p) {
  row_dispatch<R, 1>(p);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_sweep(Params<R> p) {
  row_dispatch<R, 2>(p);
}

// ---- column kernel ---------------------------------------------------------------

// Green-symbol factor for DFT bin (k1, k2), including the 1/N^2 of the inverse
// transform.  |xi|^2 - k0^2 is formed in FP64 (it cancels near the resonant
// shell |xi| = k0); the remaining arithmetic runs in the precision R.
template <typename R>
__device__ __forceinline__ cpx<R> symbol_factor(int n, int k1, int k2, double k0sq, double eps,
                                                int mode) {
  const int m1 = k1 >= n / 2 ? k1 - n : k1;
  const int m2 = k2 >= n / 2 ? k2 - n : k2;
  const double h = 6.283185307179586476925287 / double(n);
  const double xi2 = double(m1 * m1 + m2 * m2) * (h * h);
  const R inv_n2 = R(1.0 / (double(n) * double(n)));
  if (mode == SYM_LAP) return cpx<R>{R(xi2) * inv_n2, R(0)};
  const R a = R(xi2 - k0sq);  // lambda = a - i eps
  const R e = R(eps);
  const R sc = inv_n2 / (a * a + e * e);
  // 1/lambda = (a + i eps)/|lambda|^2 ; 1/conj(lambda) = (a - i eps)/|lambda|^2
  return cpx<R>{a * sc, (mode == SYM_GREEN ? e : -e) * sc};
}

// Column tile: C columns of one instance.  Thread tid works on column tid % C
// (so the C threads of a row segment read or write C neighbouring elements)
// and butterfly slot tid / C.  Between passes column c sits in LDS at
// c * col_stride(N, C) + pos(row); the stride is offset from a multiple of 32
// elements by 32/C, which spreads the C columns over the banks.
__host__ __device__ constexpr int col_stride(int n, int c) {
  return ((lds_len(n) + 31) / 32) * 32 + 32 / c;
}

template <typename R, int N, int C>
__device__ __forceinline__ void col_body(const Params<R>& p, const InstDesc& d, int col0,
                                         cpx<R>* lds) {
  constexpr int TPC = kThreads / C;
  constexpr int CS = col_stride(N, C);
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const long long cbase = d.off + col0 + c;
  const int kcol = col0 + c;
  cpx<R>* mine = lds + c * CS;
  auto ld = [&](int e) { return p.inter[cbase + (long long)e * N]; };
  // last forward pass: multiply by the Green symbol and keep the spectrum in LDS
  auto st = [&](int e, cpx<R> v) {
    mine[lds_pos(e)] = cmul(v, symbol_factor<R>(N, e, kcol, d.k0sq, d.eps, p.sym));
  };
  fft_run<R, N, TPC, -1, false, true>(mine, t, true, p.tw, ld, st);
  auto ld2 = [&](int e) { return mine[lds_pos(e)]; };
  auto st2 = [&](int e, cpx<R> v) { p.inter[cbase + (long long)e * N] = v; };
  fft_run<R, N, TPC, 1, true, false>(mine, t, true, p.tw, ld2, st2);
}

template <typename R, int C>
__global__ __launch_bounds__(kThreads) void k_col(Params<R> p) {
  extern __shared__ float4 smem_raw[];
  cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
  const int2 w = p.items[blockIdx.x];
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  const InstDesc d = p.inst[w.x];
  switch (d.n) {
#define CBS_COL_CASE(N) \
  case N:               \
    if constexpr (N % C == 0) col_body<R, N, C>(p, d, w.y, lds); \
    break;
    CBS_FOR_EACH_N(CBS_COL_CASE)
#undef CBS_COL_CASE
    default:
      break;
  }
}

// ---- pointwise kernels over row work items ------------------------------------------

enum PwOp {
  PW_GAMMA = 0,        // e_out = gamma * e_in
  PW_FIRST64 = 1,      // c_out = (R) src64; e_out = gamma * c_out
  PW_ADD_WIDE = 2,     // x64 += e_in
  PW_WIDEN = 3,        // x64 = e_in
  PW_NARROW = 4,       // e_out = (R) x64
  PW_SCALE64 = 5       // x64 *= scale[instance] (FP64)
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
  const double* scale;  // per-instance factor for PW_SCALE64
  const int* mask;
  int mask_mode;
  int op;
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_pointwise(PwParams<R> p) {
  const int2 w = p.items[blockIdx.x];
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  const InstDesc d = p.inst[w.x];
  const int n = d.n;
  const int rpw = row_rpw(n);
  const int nrows = min(rpw, n - w.y);
  const long long base = d.off + (long long)w.y * n;
  const int cnt = nrows * n;
  const R ie = R(1.0 / d.eps);
  const R k0 = R(d.k0sq), ep = R(d.eps);
  const double sc = (p.op == PW_SCALE64) ? p.scale[w.x] : 1.0;
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    const long long i = base + j;
    switch (p.op) {
      case PW_GAMMA:
      case PW_FIRST64: {
        cpx<R> v;
        if (p.op == PW_GAMMA) {
          v = p.e_in[i];
        } else {
          const cpx<double> x = p.src64[i];
          v = cpx<R>{R(x.x), R(x.y)};
          if (p.c_out) p.c_out[i] = v;
        }
        const cpx<R> k = p.k2[i];
        const cpx<R> g{-(k.y - ep) * ie, (k.x - k0) * ie};  // i V / eps
        p.e_out[i] = cmul(g, v);
        break;
      }
      case PW_ADD_WIDE: {
        const cpx<R> e = p.e_in[i];
        cpx<double> x = p.x64[i];
        x.x += double(e.x);
        x.y += double(e.y);
        p.x64[i] = x;
        break;
      }
      case PW_WIDEN: {
        const cpx<R> e = p.e_in[i];
        p.x64[i] = cpx<double>{double(e.x), double(e.y)};
        break;
      }
      case PW_NARROW: {
        const cpx<double> x = p.x64[i];
        p.e_out[i] = cpx<R>{R(x.x), R(x.y)};
        break;
      }
      default: {  // PW_SCALE64
        const cpx<double> x = p.x64[i];
        p.x64[i] = cpx<double>{x.x * sc, x.y * sc};
        break;
      }
    }
  }
}

// ---- per-instance reductions and solver bookkeeping -------------------------------

// norm2[i] = sum of the instance's partials (fixed order => deterministic).
__global__ void k_instance_sums(const InstDesc* inst, int batch, const double* partials,
                                double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const InstDesc d = inst[i];
  double s = 0.0;
  for (int k = 0; k < d.nparts; ++k) s += partials[d.part_off + k];
  out[i] = s;
}

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

// After the FP64 residual of the current iterate (start of a chunk).
__global__ void k_check64(IterState st, const InstDesc* inst, int batch,
                          const double* partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const int s0 = st.status[i];
  if (s0 == ST_CONVERGED || s0 == ST_MAXIT || s0 == ST_DIVERGED) {
    st.chunk_active[i] = 0;
    return;
  }
  const InstDesc d = inst[i];
  double sum = 0.0;
  for (int k = 0; k < d.nparts; ++k) sum += partials[d.part_off + k];
  const double bn = st.bnorm[i] > 0.0 ? st.bnorm[i] : 1.0;
  const double rel = sqrt(sum) / bn;
  st.relres[i] = rel;
  int s = ST_RUNNING;
  if (!isfinite(rel)) s = ST_DIVERGED;
  else if (rel <= st.rtol[0]) s = ST_CONVERGED;
  else if (st.iters[i] >= st.max_sweeps[0]) s = ST_MAXIT;
  st.status[i] = s;
  st.chunk_active[i] = (s == ST_RUNNING) ? 1 : 0;
  if (s == ST_RUNNING) st.iters[i] += 1;  // the pointwise first sweep that follows
}

// After an FP32 sweep of the correction: count it and test the estimate.
__global__ void k_check32(IterState st, const InstDesc* inst, int batch,
                          const double* partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  if (st.status[i] != ST_RUNNING) return;
  const InstDesc d = inst[i];
  double sum = 0.0;
  for (int k = 0; k < d.nparts; ++k) sum += partials[d.part_off + k];
  const double bn = st.bnorm[i] > 0.0 ? st.bnorm[i] : 1.0;
  const double rel = sqrt(sum) / bn;
  st.est[i] = rel;
  st.iters[i] += 1;
  if (!(rel > st.rtol[0]) || st.iters[i] >= st.max_sweeps[0]) st.status[i] = ST_PENDING;
}

// bnorm[i] = sqrt(sum of partials)
__global__ void k_set_bnorm(IterState st, const InstDesc* inst, int batch,
                            const double* partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const InstDesc d = inst[i];
  double sum = 0.0;
  for (int k = 0; k < d.nparts; ++k) sum += partials[d.part_off + k];
  st.bnorm[i] = sqrt(sum);
}

// ---- setup statistics ------------------------------------------------------------------
// phase 0: (min Re k2, max Re k2); phase 1: max |k2 - k0^2|; phase 2: min |k2 - k0^2 - i eps|
__global__ __launch_bounds__(kThreads) void k_stats(const InstDesc* inst, const int2* items,
                                                    const cpx<double>* k2, double* partials,
                                                    int phase) {
  __shared__ double red[kThreads / 64];
  const int2 w = items[blockIdx.x];
  const InstDesc d = inst[w.x];
  const int n = d.n;
  const int rpw = row_rpw(n);
  const int nrows = min(rpw, n - w.y);
  const long long base = d.off + (long long)w.y * n;
  const int cnt = nrows * n;
  double a = phase == 0 ? 1e300 : (phase == 1 ? 0.0 : 1e300);
  double b = -1e300;
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    const cpx<double> k = k2[base + j];
    if (phase == 0) {
      a = fmin(a, k.x);
      b = fmax(b, k.x);
    } else if (phase == 1) {
      a = fmax(a, hypot(k.x - d.k0sq, k.y));
    } else {
      a = fmin(a, hypot(k.x - d.k0sq, k.y - d.eps));
    }
  }
  // min/max reductions via the wave shuffles
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double oa = __shfl_xor(a, o, 64);
    const double ob = __shfl_xor(b, o, 64);
    a = (phase == 1) ? fmax(a, oa) : fmin(a, oa);
    b = fmax(b, ob);
  }
  __shared__ double redb[kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid] = a;
    redb[wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kThreads / 64; ++q) {
      a = (phase == 1) ? fmax(a, red[q]) : fmin(a, red[q]);
      b = fmax(b, redb[q]);
    }
    const int slot = d.part_off + w.y / rpw;
    partials[2 * slot] = a;
    partials[2 * slot + 1] = b;
  }
}

// ---- FGMRES: FP64 Arnoldi, CGS2, Givens least squares -------------------------------
//
// Per-instance small dense state (doubles), restart length m:
//   H  (m+1) x m complex, row-major        at 0
//   cs m real, sn m complex                 (Givens rotations)
//   g  m+1 complex                          (rotated beta e1)
//   y  m complex                            (least-squares solution)
//   coef m+1 complex                        (current Gram-Schmidt coefficients)
//   sc 8 scalars: [0] beta [1] bnorm [2] estimate
struct KryLayout {
  int m;
  __host__ __device__ long long h(int r, int c) const { return 2LL * (r * m + c); }
  __host__ __device__ long long cs() const { return 2LL * (m + 1) * m; }
  __host__ __device__ long long sn() const { return cs() + m; }
  __host__ __device__ long long g() const { return sn() + 2LL * m; }
  __host__ __device__ long long y() const { return g() + 2LL * (m + 1); }
  __host__ __device__ long long coef() const { return y() + 2LL * m; }
  __host__ __device__ long long sc() const { return coef() + 2LL * (m + 1); }
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
  double* dots;               // per partial slot: (m+1) complex partial dot products
  double* partials;           // per partial slot: one double
  double* scale;              // per instance
  int* active;                // per instance: 1 while in the Arnoldi cycle
  int* jend;                  // per instance: Arnoldi steps done this cycle
  int* iters;                 // per instance: total Arnoldi steps
  int* status;                // per instance: solver status
  double* relres;             // per instance: last FP64 true relative residual
  const double* rtol;
  const int* max_iters;
  int pass;                   // Gram-Schmidt pass 0 (sets H) or 1 (adds)
};

__device__ __forceinline__ void item_range(const InstDesc& d, int row0, long long& base, int& cnt,
                                           int& slot) {
  const int rpw = row_rpw(d.n);
  const int nrows = min(rpw, d.n - row0);
  base = d.off + (long long)row0 * d.n;
  cnt = nrows * d.n;
  slot = d.part_off + row0 / rpw;
}

// Partial dot products <v_q, w> for q = 0..j over one row item.
__global__ __launch_bounds__(kThreads) void k_dots(KryParams k) {
  __shared__ double red[kThreads / 64];
  const int2 it = k.items[blockIdx.x];
  if (!k.active[it.x]) return;
  const InstDesc d = k.inst[it.x];
  long long base;
  int cnt, slot;
  item_range(d, it.y, base, cnt, slot);
  constexpr int PER = 2048 / kThreads;  // row_rpw(N) * N <= 2048 for every N
  cpx<double> wv[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int j = threadIdx.x + e * kThreads;
    wv[e] = j < cnt ? k.w[base + j] : cpx<double>{0.0, 0.0};
  }
  for (int q = 0; q <= k.j; ++q) {
    const cpx<double>* v = k.vbasis + q * k.cells;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int j = threadIdx.x + e * kThreads;
      if (j < cnt) {
        const cpx<double> a = v[base + j];
        re += a.x * wv[e].x + a.y * wv[e].y;
        im += a.x * wv[e].y - a.y * wv[e].x;
      }
    }
    const double sre = block_sum(re, red);
    __syncthreads();
    const double sim = block_sum(im, red);
    __syncthreads();
    if (threadIdx.x == 0) {
      k.dots[2LL * ((long long)slot * (k.m + 1) + q)] = sre;
      k.dots[2LL * ((long long)slot * (k.m + 1) + q) + 1] = sim;
    }
  }
}

// coef_q = sum of partial dots; H[q][j] (+)= coef_q.
__global__ void k_dots_finish(KryParams k, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch || !k.active[i]) return;
  const InstDesc d = k.inst[i];
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  for (int q = 0; q <= k.j; ++q) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < d.nparts; ++t) {
      re += k.dots[2LL * ((long long)(d.part_off + t) * (k.m + 1) + q)];
      im += k.dots[2LL * ((long long)(d.part_off + t) * (k.m + 1) + q) + 1];
    }
    s[L.coef() + 2 * q] = re;
    s[L.coef() + 2 * q + 1] = im;
    if (k.pass == 0) {
      s[L.h(q, k.j)] = re;
      s[L.h(q, k.j) + 1] = im;
    } else {
      s[L.h(q, k.j)] += re;
      s[L.h(q, k.j) + 1] += im;
    }
  }
}

// w -= sum_q coef_q v_q ; also the partial |w|^2 for the norm that follows.
__global__ __launch_bounds__(kThreads) void k_cgs_update(KryParams k) {
  __shared__ double red[kThreads / 64];
  const int2 it = k.items[blockIdx.x];
  if (!k.active[it.x]) return;
  const InstDesc d = k.inst[it.x];
  long long base;
  int cnt, slot;
  item_range(d, it.y, base, cnt, slot);
  const KryLayout L{k.m};
  const double* s = k.kry + it.x * k.kstride + L.coef();
  double acc = 0.0;
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    cpx<double> wv = k.w[base + j];
    for (int q = 0; q <= k.j; ++q) {
      const cpx<double> v = k.vbasis[q * k.cells + base + j];
      const cpx<double> c{s[2 * q], s[2 * q + 1]};
      wv = wv - cmul(c, v);
    }
    k.w[base + j] = wv;
    acc += cabs2(wv);
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) k.partials[slot] = t;
}

// h_{j+1,j} = ||w||; scale = 1/h; Givens update and residual estimate.
__global__ void k_givens(KryParams k, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch || !k.active[i]) return;
  const InstDesc d = k.inst[i];
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  double sum = 0.0;
  for (int t = 0; t < d.nparts; ++t) sum += k.partials[d.part_off + t];
  const double hn = sqrt(sum);
  const int j = k.j;
  s[L.h(j + 1, j)] = hn;
  s[L.h(j + 1, j) + 1] = 0.0;
  k.scale[i] = hn > 0.0 ? 1.0 / hn : 0.0;
  // apply previous rotations to column j
  for (int q = 0; q < j; ++q) {
    const double c = s[L.cs() + q];
    const cpx<double> sn{s[L.sn() + 2 * q], s[L.sn() + 2 * q + 1]};
    const cpx<double> a{s[L.h(q, j)], s[L.h(q, j) + 1]};
    const cpx<double> b{s[L.h(q + 1, j)], s[L.h(q + 1, j) + 1]};
    const cpx<double> na = cscale(a, c) + cmul(sn, b);
    const cpx<double> nb = cscale(b, c) - cmul(cconj(sn), a);
    s[L.h(q, j)] = na.x;
    s[L.h(q, j) + 1] = na.y;
    s[L.h(q + 1, j)] = nb.x;
    s[L.h(q + 1, j) + 1] = nb.y;
  }
  // new rotation zeroing h_{j+1,j}
  const cpx<double> a{s[L.h(j, j)], s[L.h(j, j) + 1]};
  const cpx<double> b{s[L.h(j + 1, j)], s[L.h(j + 1, j) + 1]};
  const double aa = sqrt(cabs2(a));
  const double nu = sqrt(cabs2(a) + cabs2(b));
  double c;
  cpx<double> sn;
  if (aa == 0.0) {
    c = 0.0;
    sn = cpx<double>{1.0, 0.0};
  } else {
    c = aa / nu;
    sn = cscale(cmul(a, cconj(b)), 1.0 / (aa * nu));
  }
  s[L.cs() + j] = c;
  s[L.sn() + 2 * j] = sn.x;
  s[L.sn() + 2 * j + 1] = sn.y;
  const cpx<double> na = cscale(a, c) + cmul(sn, b);
  s[L.h(j, j)] = na.x;
  s[L.h(j, j) + 1] = na.y;
  s[L.h(j + 1, j)] = 0.0;
  s[L.h(j + 1, j) + 1] = 0.0;
  const cpx<double> gj{s[L.g() + 2 * j], s[L.g() + 2 * j + 1]};
  const cpx<double> g1 = cscale(cmul(cconj(sn), gj), -1.0);
  const cpx<double> g0 = cscale(gj, c);
  s[L.g() + 2 * j] = g0.x;
  s[L.g() + 2 * j + 1] = g0.y;
  s[L.g() + 2 * (j + 1)] = g1.x;
  s[L.g() + 2 * (j + 1) + 1] = g1.y;
  const double est = sqrt(cabs2(g1)) / (s[L.sc() + 1] > 0.0 ? s[L.sc() + 1] : 1.0);
  s[L.sc() + 2] = est;
  k.jend[i] = j + 1;
  k.iters[i] += 1;
  if (!(est > k.rtol[0]) || hn == 0.0 || k.iters[i] >= k.max_iters[0] || j + 1 >= k.m)
    k.active[i] = 0;
}

// Back substitution H[0:jend, 0:jend] y = g[0:jend] (H upper triangular after rotations).
__global__ void k_backsolve(KryParams k, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const int n = k.jend[i];
  if (n <= 0) return;
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  for (int r = n - 1; r >= 0; --r) {
    cpx<double> acc{s[L.g() + 2 * r], s[L.g() + 2 * r + 1]};
    for (int c = r + 1; c < n; ++c) {
      const cpx<double> h{s[L.h(r, c)], s[L.h(r, c) + 1]};
      const cpx<double> yc{s[L.y() + 2 * c], s[L.y() + 2 * c + 1]};
      acc = acc - cmul(h, yc);
    }
    const cpx<double> h{s[L.h(r, r)], s[L.h(r, r) + 1]};
    const double den = cabs2(h);
    const cpx<double> yr = den > 0.0 ? cscale(cmulc(h, acc), 1.0 / den) : cpx<double>{0.0, 0.0};
    s[L.y() + 2 * r] = yr.x;
    s[L.y() + 2 * r + 1] = yr.y;
  }
}

// x64 += sum_{q < jend} y_q z_q  (z in the operator precision)
template <typename R>
__global__ __launch_bounds__(kThreads) void k_zupdate(KryParams k, const cpx<R>* z,
                                                      cpx<double>* x) {
  const int2 it = k.items[blockIdx.x];
  const int n = k.jend[it.x];
  if (n <= 0) return;
  const InstDesc d = k.inst[it.x];
  long long base;
  int cnt, slot;
  item_range(d, it.y, base, cnt, slot);
  const KryLayout L{k.m};
  const double* s = k.kry + it.x * k.kstride + L.y();
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    cpx<double> acc = x[base + j];
    for (int q = 0; q < n; ++q) {
      const cpx<R> zv = z[q * k.cells + base + j];
      const cpx<double> yq{s[2 * q], s[2 * q + 1]};
      acc = acc + cmul(yq, cpx<double>{double(zv.x), double(zv.y)});
    }
    x[base + j] = acc;
  }
}

// After the FP64 true residual r = G(V x + s) - x was written to v_0 with its
// partial norms: decide convergence and start a new cycle.
__global__ void k_fg_restart(KryParams k, int batch, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  if (first) {  // partials hold |G s|^2: store ||G s||
    const InstDesc d0 = k.inst[i];
    double sum0 = 0.0;
    for (int t = 0; t < d0.nparts; ++t) sum0 += k.partials[d0.part_off + t];
    s[L.sc() + 1] = sqrt(sum0);
    return;
  }
  k.jend[i] = 0;
  const int st = k.status[i];
  if (st != ST_RUNNING) {
    k.active[i] = 0;
    return;
  }
  const InstDesc d = k.inst[i];
  double sum = 0.0;
  for (int t = 0; t < d.nparts; ++t) sum += k.partials[d.part_off + t];
  const double beta = sqrt(sum);
  const double rel = beta / (s[L.sc() + 1] > 0.0 ? s[L.sc() + 1] : 1.0);
  k.relres[i] = rel;
  s[L.sc() + 0] = beta;
  int ns = ST_RUNNING;
  if (!isfinite(rel)) ns = ST_DIVERGED;
  else if (rel <= k.rtol[0]) ns = ST_CONVERGED;
  else if (k.iters[i] >= k.max_iters[0]) ns = ST_MAXIT;
  k.status[i] = ns;
  k.active[i] = ns == ST_RUNNING ? 1 : 0;
  k.scale[i] = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int q = 0; q <= k.m; ++q) {
    s[L.g() + 2 * q] = q == 0 ? beta : 0.0;
    s[L.g() + 2 * q + 1] = 0.0;
  }
}

__global__ void k_widen_all(const cpx<float>* in, cpx<double>* out, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const cpx<float> v = in[i];
    out[i] = cpx<double>{double(v.x), double(v.y)};
  }
}

}  // namespace cbs
