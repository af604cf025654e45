// Row and column kernels for Dirichlet instances: the n x n interior of the
// unit square with homogeneous Dirichlet boundaries, five-point finite
// differences, h = 1/(n+1), whose reference operator the 2D DST-I
// diagonalises (App. B.2 and App. C, Newton linear systems).
//
// A DST-I of length n rides on the length M = 2(n+1) FFT of the odd
// extension x~ = (0, x_1..x_n, 0, -x_n..-x_1): its bins 1..n are
// -2i (S x)_k, (S x)_k = sum_j x_j sin(pi j k / (n+1)), and the inverse FFT's
// are +2i (S x)_k.  The transform of an odd sequence is odd again and the
// symbol is even in the bin (p and M - p carry the same eigenvalue), so the
// column pass runs forward transform, symbol and inverse transform exactly as
// in the periodic case.  The factors -2i, +2i and S^-1 = 2/(n+1) S of the four
// one-dimensional transforms combine to 1/M^2, the factor the symbol carries.
//
// Eigenvalues of the five-point negative Laplacian on bin (p, q):
// 4/h^2 (sin^2(p pi h / 2) + sin^2(q pi h / 2)) = mu_p + mu_q with
// mu_p = M^2 sin^2(pi p / M), tabulated in FP64 per transform length.
#pragma once
#include "kernels.hpp"

namespace cbs {

// DST bin (1..n) that FFT bin e of the odd extension carries; 0 for the bins
// 0 and n + 1, which are zero.
template <int M>
__device__ __forceinline__ int dst_bin(int e) {
  constexpr int n = M / 2 - 1;
  return e == 0 || e == n + 1 ? 0 : (e <= n ? e : M - e);
}

// Element e (0..M-1) of the odd extension of the length-n sequence g(0..n-1).
template <int M, typename R, class G>
__device__ __forceinline__ cpx<R> odd_ext(G g, int e) {
  constexpr int n = M / 2 - 1;
  if (e == 0 || e == n + 1) return cpx<R>{R(0), R(0)};
  if (e <= n) return g(e - 1);
  const cpx<R> v = g(M - 1 - e);
  return cpx<R>{-v.x, -v.y};
}

// Symbol factor on DST bins (p, q), both in 1..n: 1/(M^2 lambda) with
// lambda = mu_p + mu_q - k0^2 - i eps (conjugate for SYM_GREEN_CONJ), or
// (mu_p + mu_q) / M^2 for SYM_LAP.  mu_p + mu_q - k0^2 is formed in FP64.
template <typename R, int M>
__device__ __forceinline__ cpx<R> dst_symbol_factor(const double* mu, int mode, int pb, int qb,
                                                    double k0sq, double eps) {
  const double lap = mu[pb] + mu[qb];
  const R inv_m2 = R(1.0 / (double(M) * double(M)));
  if (mode == SYM_LAP) return cpx<R>{R(lap) * inv_m2, R(0)};
  const R a = R(lap - k0sq);
  const R e = R(eps);
  R sc;
  if constexpr (sizeof(R) == 4) sc = inv_m2 * __builtin_amdgcn_rcpf(a * a + e * e);
  else sc = inv_m2 / (a * a + e * e);
  return cpx<R>{a * sc, (mode == SYM_GREEN ? e : -e) * sc};
}

// MODE 0: prologue + forward rows -> spectral rows; MODE 1: inverse rows +
// epilogue (with partial norms); MODE 2: inverse rows -> CBS update (written)
// -> next prologue, staged in LDS -> forward rows.  Rows of n cells, FFTs of
// length M; only bins 1..n are stored.
template <typename R, int M, int MODE>
__device__ __forceinline__ void row_body_dst(const Params<R>& p, const InstDesc& d, int row0,
                                             cpx<R>* lds, double* red) {
  using T = RowTile<M>;
  constexpr int n = M / 2 - 1;
  const int tid = threadIdx.x;
  const int r = tid / T::TPF, t = tid - r * T::TPF;
  const int nrows = min(T::RPW, n - row0);
  const bool active = r < nrows;
  const long long rbase = d.off + (long long)(row0 + (active ? r : 0)) * n;
  cpx<R>* mine = lds + (active ? r : 0) * T::RS;
  auto keep = [](int e) { return e >= 1 && e <= n; };
  if constexpr (MODE == 0) {
    auto ld = [&](int e) {
      return odd_ext<M, R>([&](int j) { return prologue(p, d, rbase + j); }, e);
    };
    auto st = [&](int e, cpx<R> v) {
      if (keep(e)) p.inter[rbase + e - 1] = v;
    };
    fft_run<R, M, T::TPF, -1, false, false>(mine, t, active, p.tw, ld, st);
  } else if constexpr (MODE == 1) {
    double acc = 0.0;
    auto ld = [&](int e) { return odd_ext<M, R>([&](int j) { return p.inter[rbase + j]; }, e); };
    auto st = [&](int e, cpx<R> v) {
      if (keep(e)) acc += epilogue(p, d, rbase + e - 1, v);
    };
    fft_run<R, M, T::TPF, 1, false, false>(mine, t, active, p.tw, ld, st);
    if (p.partials) {
      const double s = block_sum(acc, red);
      if (tid == 0) p.partials[d.part_off + row0 / T::RPW] = s;
    }
  } else {
    double acc = 0.0;
    auto ld = [&](int e) { return odd_ext<M, R>([&](int j) { return p.inter[rbase + j]; }, e); };
    // u_new = u + gamma (z - u + rhs), written out; returns V u_new + s
    auto update = [&](int j, cpx<R> z) {
      const long long g = rbase + j;
      const cpx<R> u = p.u[g];
      const cpx<R> rres = z - u + ld_or_zero(p.rhs, g);
      const Coef<R> c = coef(p, d, g);
      const cpx<R> un = u + cmul(c.gamma(), rres);
      p.out[g] = un;
      acc += double(cabs2(rres));
      return cmul(c.v, un) + ld_or_zero(p.s, g);
    };
    auto st = [&](int e, cpx<R> z) {
      if (keep(e)) mine[lds_pos(e)] = update(e - 1, z);
    };
    fft_run<R, M, T::TPF, 1, false, true>(mine, t, active, p.tw, ld, st);
    auto ld2 = [&](int e) {
      return odd_ext<M, R>([&](int j) { return lds_ld(mine + lds_pos(j + 1)); }, e);
    };
    auto st2 = [&](int e, cpx<R> v) {
      if (keep(e)) p.inter[rbase + e - 1] = v;
    };
    fft_run<R, M, T::TPF, -1, true, false>(mine, t, active, p.tw, ld2, st2);
    if (p.partials) {
      const double s = block_sum(acc, red);
      if (tid == 0) p.partials[d.part_off + row0 / T::RPW] = s;
    }
  }
}

// ---- direct DST-I for n = 64 -------------------------------------------------------
//
// The odd extension of n = 64 has length 130 = 2 5 13, which has no FFT plan
// here, so its transforms are formed directly: (S x)_k = sum_j x_j
// sin(pi (j+1)(k+1)/(n+1)) from a row or column held in LDS, each of TPL
// threads forming n/TPL outputs, with sin(pi m/(n+1)), m < 2(n+1), tabulated
// (the index (j+1)(k+1) mod 2(n+1) advances by k+1 per j).  With the unscaled
// S both ways, S^-1 = (2/(n+1)) S = (4/M) S per dimension, so the symbol
// carries 16/M^2 where the FFT path's factors -2i, +2i leave 1/M^2.
template <typename R, int NN, int TPL, int ES>
__device__ __forceinline__ void dst_direct(const cpx<R>* buf, int t, bool active, const R* sn,
                                           cpx<R>* out) {
  constexpr int K = NN / TPL;
  constexpr int MM = 2 * (NN + 1);
  static_assert(NN % TPL == 0, "outputs per thread");
  int idx[K], inc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    out[q] = cpx<R>{R(0), R(0)};
    inc[q] = t + q * TPL + 1;
    idx[q] = inc[q];
  }
  if (!active) return;
  for (int j = 0; j < NN; ++j) {
    const cpx<R> x = lds_ld(buf + ES * lds_pos(j));
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const R w = sn[idx[q]];
      out[q].x += x.x * w;
      out[q].y += x.y * w;
      idx[q] += inc[q];
      if (idx[q] >= MM) idx[q] -= MM;
    }
  }
}

struct DirectRowTile {
  static constexpr int TPF = kDstDirectTPF;
  static constexpr int RPW = kDstDirectRPW;
  static constexpr int RS = lds_len(kDstDirectN);
  static_assert(RPW * RS <= kRowLds, "row tile does not fit");
};

// Rows of the direct size: MODE 0, 1, 2 as in row_body_dst.
template <typename R, int MODE>
__device__ __forceinline__ void row_body_dst_direct(const Params<R>& p, const InstDesc& d, int row0,
                                                    cpx<R>* lds, double* red, const R* sn) {
  constexpr int NN = kDstDirectN;
  using T = DirectRowTile;
  constexpr int K = NN / T::TPF;
  const int tid = threadIdx.x;
  const int r = tid / T::TPF, t = tid - r * T::TPF;
  const int nrows = min(T::RPW, NN - row0);
  const bool active = r < nrows;
  const long long rbase = d.off + (long long)(row0 + (active ? r : 0)) * NN;
  cpx<R>* mine = lds + (active ? r : 0) * T::RS;
  if (active)
    for (int j = t; j < NN; j += T::TPF) {
      if constexpr (MODE == 0) mine[lds_pos(j)] = prologue(p, d, rbase + j);
      else mine[lds_pos(j)] = p.inter[rbase + j];
    }
  __syncthreads();
  cpx<R> o[K];
  dst_direct<R, NN, T::TPF, 1>(mine, t, active, sn, o);
  double acc = 0.0;
  if constexpr (MODE == 0) {
    if (active)
#pragma unroll
      for (int q = 0; q < K; ++q) p.inter[rbase + t + q * T::TPF] = o[q];
  } else if constexpr (MODE == 1) {
    if (active)
#pragma unroll
      for (int q = 0; q < K; ++q) acc += epilogue(p, d, rbase + t + q * T::TPF, o[q]);
  } else {
    // u_new = u + gamma (z - u + rhs), written out; then V u_new + s forward
    cpx<R> v[K];
    if (active)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const long long g = rbase + t + q * T::TPF;
        const cpx<R> u = p.u[g];
        const cpx<R> rres = o[q] - u + ld_or_zero(p.rhs, g);
        const Coef<R> c = coef(p, d, g);
        const cpx<R> un = u + cmul(c.gamma(), rres);
        p.out[g] = un;
        acc += double(cabs2(rres));
        v[q] = cmul(c.v, un) + ld_or_zero(p.s, g);
      }
    __syncthreads();
    if (active)
#pragma unroll
      for (int q = 0; q < K; ++q) mine[lds_pos(t + q * T::TPF)] = v[q];
    __syncthreads();
    dst_direct<R, NN, T::TPF, 1>(mine, t, active, sn, o);
    if (active)
#pragma unroll
      for (int q = 0; q < K; ++q) p.inter[rbase + t + q * T::TPF] = o[q];
  }
  if (MODE != 0 && p.partials) {
    const double s = block_sum(acc, red);
    if (tid == 0) p.partials[d.part_off + row0 / T::RPW] = s;
  }
}

// Column tile of C columns of the direct size: forward DST, symbol (x 16),
// inverse DST, all in LDS.
template <typename R, int C>
__device__ __forceinline__ void col_body_dst_direct(const Params<R>& p, const InstDesc& d, int col0,
                                                    cpx<R>* lds, const R* sn) {
  constexpr int NN = kDstDirectN, M = kDstDirectM;
  constexpr int TPC = kThreads / C;
  constexpr int K = NN / TPC;
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const int kcol = col0 + c;
  const bool active = kcol < NN;
  const long long cbase = d.off + (active ? kcol : 0);
  cpx<R>* mine = lds + c;
  const double* mu = p.mu + kMuDirect;
  if (active)
    for (int j = t; j < NN; j += TPC) mine[C * lds_pos(j)] = p.inter[cbase + (long long)j * NN];
  __syncthreads();
  cpx<R> o[K];
  dst_direct<R, NN, TPC, C>(mine, t, active, sn, o);
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int k = t + q * TPC;
    if (p.sym == SYM_TABLE)
      o[q] = cscale(cmul(o[q], p.table[cbase + (long long)k * NN]), R(16.0 / (double(M) * double(M))));
    else
      o[q] = cscale(cmul(o[q], dst_symbol_factor<R, M>(mu, p.sym, k + 1, kcol + 1, d.k0sq, d.eps)), R(16));
  }
  __syncthreads();
  if (active)
#pragma unroll
    for (int q = 0; q < K; ++q) mine[C * lds_pos(t + q * TPC)] = o[q];
  __syncthreads();
  dst_direct<R, NN, TPC, C>(mine, t, active, sn, o);
  if (active)
#pragma unroll
    for (int q = 0; q < K; ++q) p.inter[cbase + (long long)(t + q * TPC) * NN] = o[q];
}

// sin(pi m / (n+1)), m < 2(n+1), of the direct size into LDS (every thread
// of the workgroup calls it).
template <typename R>
__device__ __forceinline__ void load_direct_sines(const Params<R>& p, R* sn) {
  for (int m = threadIdx.x; m < kDstDirectM; m += kThreads) sn[m] = R(p.mu[kSinDirect + m]);
  __syncthreads();
}

template <typename R, int MODE>
__device__ __forceinline__ void row_dispatch_dst(const Params<R>& p) {
  __shared__ cpx<R> lds[kRowLds];
  __shared__ double red[kThreads / 64];
  const int2 w = p.items[blockIdx.x];
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  const InstDesc d = p.inst[w.x];
  if (d.n == kDstDirectN) {
    __shared__ R sn[kDstDirectM];
    load_direct_sines(p, sn);
    row_body_dst_direct<R, MODE>(p, d, w.y, lds, red, sn);
    return;
  }
  switch (dst_len(d.n)) {
#define CBS_ROW_DST_CASE(M) \
  case M:                   \
    row_body_dst<R, M, MODE>(p, d, w.y, lds, red); \
    break;
    CBS_FOR_EACH_N(CBS_ROW_DST_CASE)
#undef CBS_ROW_DST_CASE
    default:
      break;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_fwd_dst(Params<R> p) {
  row_dispatch_dst<R, 0>(p);
}
template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_inv_dst(Params<R> p) {
  row_dispatch_dst<R, 1>(p);
}
template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_sweep_dst(Params<R> p) {
  row_dispatch_dst<R, 2>(p);
}

// Column tile of C columns (the last tile of an instance may be partial:
// columns >= n only join the barriers).  Layout in LDS as in col_body.
template <typename R, int M, int C>
__device__ __forceinline__ void col_body_dst(const Params<R>& p, const InstDesc& d, int col0,
                                             cpx<R>* lds) {
  constexpr int n = M / 2 - 1;
  constexpr int TPC = kThreads / C;
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const int kcol = col0 + c;
  const bool active = kcol < n;
  const long long cbase = d.off + (active ? kcol : 0);
  cpx<R>* mine = lds + c;
  const double* mu = p.mu + mu_offset(M);
  auto ld = [&](int e) {
    return odd_ext<M, R>([&](int j) { return p.inter[cbase + (long long)j * n]; }, e);
  };
  auto sym = [&](int e, cpx<R> v) {
    const int pb = dst_bin<M>(e);
    if (pb == 0) return cpx<R>{R(0), R(0)};
    if (p.sym == SYM_TABLE)  // tabulated weights on DST bins; 1/M^2 as in the symbol
      return cscale(cmul(v, p.table[cbase + (long long)(pb - 1) * n]),
                    R(1.0 / (double(M) * double(M))));
    return cmul(v, dst_symbol_factor<R, M>(mu, p.sym, pb, kcol + 1, d.k0sq, d.eps));
  };
  auto st2 = [&](int e, cpx<R> v) {
    if (e >= 1 && e <= n) p.inter[cbase + (long long)(e - 1) * n] = v;
  };
  if constexpr (plan_bridgeable(M)) {
    fft_run2<R, M, TPC, -1, 1, C>(mine, t, active, p.tw, ld, sym, st2);
  } else {
    auto st = [&](int e, cpx<R> v) { mine[C * lds_pos(e)] = sym(e, v); };
    fft_run<R, M, TPC, -1, false, true, C>(mine, t, active, p.tw, ld, st);
    auto ld2 = [&](int e) { return lds_ld(mine + C * lds_pos(e)); };
    fft_run<R, M, TPC, 1, true, false, C>(mine, t, active, p.tw, ld2, st2);
  }
}

template <typename R, int M>
__device__ __forceinline__ void col_dispatch_dst_n(const Params<R>& p, const InstDesc& d, int col0,
                                                   cpx<R>* lds) {
  constexpr int C0 = col_tile_default(M);
  constexpr int EB = int(sizeof(cpx<R>));
  const int c = sizeof(R) == 4 ? d.ctile : d.ctile64;
  if constexpr (col_tile_valid(M, C0, EB))
    if (c == C0) { col_body_dst<R, M, C0>(p, d, col0, lds); return; }
  if constexpr (col_tile_valid(M, C0 / 2, EB))
    if (c == C0 / 2) { col_body_dst<R, M, (C0 / 2 >= 2 ? C0 / 2 : 2)>(p, d, col0, lds); return; }
  if constexpr (col_tile_valid(M, C0 * 2, EB))
    if (c == C0 * 2) { col_body_dst<R, M, (C0 * 2 <= 32 ? C0 * 2 : 32)>(p, d, col0, lds); return; }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_col_dst(Params<R> p) {
  extern __shared__ float4 smem_raw[];
  cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
  const int2 w = p.items[blockIdx.x];
  if (p.check && w.y == 0 && threadIdx.x < 64) check32_instance(p.chk, p.inst, p.partials, w.x);
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  const InstDesc d = p.inst[w.x];
  if (d.n == kDstDirectN) {
    __shared__ R sn[kDstDirectM];
    load_direct_sines(p, sn);
    // compiled widths for the length-64 columns: the default 32 and half of it
    constexpr int C0 = col_tile_default(kDstDirectN);
    static_assert(C0 == 32, "direct DST column widths");
    if ((sizeof(R) == 4 ? d.ctile : d.ctile64) == C0 / 2)
      col_body_dst_direct<R, C0 / 2>(p, d, w.y, lds, sn);
    else
      col_body_dst_direct<R, C0>(p, d, w.y, lds, sn);
    return;
  }
  switch (dst_len(d.n)) {
#define CBS_COL_DST_CASE(M) \
  case M:                   \
    col_dispatch_dst_n<R, M>(p, d, w.y, lds); \
    break;
    CBS_FOR_EACH_N(CBS_COL_DST_CASE)
#undef CBS_COL_DST_CASE
    default:
      break;
  }
}

}  // namespace cbs
