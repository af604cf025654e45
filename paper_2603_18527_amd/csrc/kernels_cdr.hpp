// One-dimensional spectral-derivative passes for convection-diffusion-reaction
// plans (App. C, "Convection-diffusion-reaction").
//
// V_cdr u = d/dx(dkappa du/dx) + d/dy(dkappa du/dy) - dv . grad u - dsigma u
// needs derivatives of fields that are products with the coefficient fields,
// so it cannot be folded into the one Fourier multiplier that G_cdr is.  A
// derivative along x is diagonal after the row transform alone and one along
// y after the column transform alone, so each derivative here is a single
// pass: forward 1D transform, multiply by i xi / N (xi = 2 pi m / N on the
// signed index m, Nyquist bin -N/2), inverse 1D transform, with a pointwise
// prologue on the way in and a pointwise epilogue on the way out.
//
// V u + s (forward) and e - V^H g (adjoint, V^H = Dx(dkappa Dx + dvx) +
// Dy(dkappa Dy + dvy) - dsigma for real coefficients, since D^H = -D) both
// take four passes:
//   1. row pass   dx = Dx a
//   2. col pass   dy = Dy a
//   3. row pass   t  = Dx(dkappa dx [+ dvx g]) + q,
//                 q = -dvx dx - dvy dy - dsigma u + s   (forward)
//                 q = -dsigma g                        (adjoint)
//   4. col pass   w  = t + Dy(dkappa dy [+ dvy g]); out = w (forward) or
//                 e - w (adjoint)
// Field roles in Params: a = pass input / dx, b = dy, u = u (forward) or g
// (adjoint), s = s (forward) or e (adjoint, pass 4), rhs = t (pass 4).
#pragma once
#include "kernels.hpp"

namespace cbs {

// i xi(e) / N * v for bin e of a length-N transform
template <typename R, int N>
__device__ __forceinline__ cpx<R> deriv_factor(int e, cpx<R> v) {
  const int m = e >= N / 2 ? e - N : e;
  const R f = R(6.283185307179586476925287 * double(m) / (double(N) * double(N)));
  return cpx<R>{-v.y * f, v.x * f};
}

template <typename R>
__device__ __forceinline__ cpx<R> cdr_prologue(const Params<R>& p, long long i) {
  if (p.pro == CPRO_A) return p.a[i];
  const cpx<R> c1 = p.k2[i];  // (dkappa, dsigma)
  if (p.pro == CPRO_WX) {
    cpx<R> w = cscale(p.a[i], c1.x);
    if (p.cdr_adj) w = w + cscale(p.u[i], p.k2b[i].x);
    return w;
  }
  cpx<R> w = cscale(p.b[i], c1.x);  // CPRO_WY
  if (p.cdr_adj) w = w + cscale(p.u[i], p.k2b[i].y);
  return w;
}

template <typename R>
__device__ __forceinline__ void cdr_epilogue(const Params<R>& p, long long i, cpx<R> v) {
  if (p.epi == CEPI_STORE) {
    p.out[i] = v;
  } else if (p.epi == CEPI_Q) {
    const cpx<R> c1 = p.k2[i];
    const cpx<R> u = p.u[i];
    cpx<R> q = cscale(u, -c1.y);
    if (!p.cdr_adj) {
      const cpx<R> c2 = p.k2b[i];
      q = q - cscale(p.a[i], c2.x) - cscale(p.b[i], c2.y) + ld_or_zero(p.s, i);
    }
    p.out[i] = v + q;
  } else {  // CEPI_ACC
    const cpx<R> w = p.rhs[i] + v;
    p.out[i] = p.cdr_adj ? p.s[i] - w : w;
  }
}

// d/dx pass over a row tile (rows as in row_body)
template <typename R, int N>
__device__ __forceinline__ void cdr_row_body(const Params<R>& p, const InstDesc& d, int row0, cpx<R>* lds) {
  using T = RowTile<N>;
  const int tid = threadIdx.x;
  const int r = tid / T::TPF, t = tid - r * T::TPF;
  const int nrows = min(T::RPW, N - row0);
  const bool active = r < nrows;
  const long long rbase = d.off + (long long)(row0 + (active ? r : 0)) * N;
  cpx<R>* mine = lds + (active ? r : 0) * T::RS;
  auto ld = [&](int e) { return cdr_prologue(p, rbase + e); };
  auto mid = [&](int e, cpx<R> v) { return deriv_factor<R, N>(e, v); };
  auto st2 = [&](int e, cpx<R> v) { cdr_epilogue(p, rbase + e, v); };
  if constexpr (plan_bridgeable(N)) {
    fft_run2<R, N, T::TPF, -1, 1>(mine, t, active, p.tw, ld, mid, st2);
  } else {
    auto st = [&](int e, cpx<R> v) { mine[lds_pos(e)] = mid(e, v); };
    fft_run<R, N, T::TPF, -1, false, true>(mine, t, active, p.tw, ld, st);
    auto ld2 = [&](int e) { return lds_ld(mine + lds_pos(e)); };
    fft_run<R, N, T::TPF, 1, true, false>(mine, t, active, p.tw, ld2, st2);
  }
}

// d/dy pass over a column tile (C columns, layout as in col_body)
template <typename R, int N, int C>
__device__ __forceinline__ void cdr_col_body(const Params<R>& p, const InstDesc& d, int col0, cpx<R>* lds) {
  constexpr int TPC = kThreads / C;
  const int tid = threadIdx.x;
  const int c = tid % C, tt = tid / C;
  const long long cbase = d.off + col0 + c;
  cpx<R>* mine = lds + c;
  auto ld = [&](int e) { return cdr_prologue(p, cbase + (long long)e * N); };
  auto mid = [&](int e, cpx<R> v) { return deriv_factor<R, N>(e, v); };
  auto st2 = [&](int e, cpx<R> v) { cdr_epilogue(p, cbase + (long long)e * N, v); };
  if constexpr (plan_bridgeable(N)) {
    fft_run2<R, N, TPC, -1, 1, C>(mine, tt, true, p.tw, ld, mid, st2);
  } else {
    auto st = [&](int e, cpx<R> v) { mine[C * lds_pos(e)] = mid(e, v); };
    fft_run<R, N, TPC, -1, false, true, C>(mine, tt, true, p.tw, ld, st);
    auto ld2 = [&](int e) { return lds_ld(mine + C * lds_pos(e)); };
    fft_run<R, N, TPC, 1, true, false, C>(mine, tt, true, p.tw, ld2, st2);
  }
}

template <typename R, int N>
__device__ __forceinline__ void cdr_col_dispatch_n(const Params<R>& p, const InstDesc& d, int col0,
                                                   cpx<R>* lds) {
  constexpr int C0 = col_tile_default(N);
  constexpr int EB = int(sizeof(cpx<R>));
  const int c = sizeof(R) == 4 ? d.ctile : d.ctile64;
  if constexpr (col_tile_valid(N, C0, EB))
    if (c == C0) { cdr_col_body<R, N, C0>(p, d, col0, lds); return; }
  if constexpr (col_tile_valid(N, C0 / 2, EB))
    if (c == C0 / 2) { cdr_col_body<R, N, (C0 / 2 >= 2 ? C0 / 2 : 2)>(p, d, col0, lds); return; }
  if constexpr (col_tile_valid(N, C0 * 2, EB))
    if (c == C0 * 2) { cdr_col_body<R, N, (C0 * 2 <= 32 ? C0 * 2 : 32)>(p, d, col0, lds); return; }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_cdr_row(Params<R> p) {
  __shared__ cpx<R> lds[kRowLds];
  const int2 w = p.items[blockIdx.x];
  const InstDesc d = p.inst[w.x];
  switch (d.n) {
#define CBS_CDR_ROW_CASE(N) \
  case N:                   \
    cdr_row_body<R, N>(p, d, w.y, lds); \
    break;
    CBS_FOR_EACH_N(CBS_CDR_ROW_CASE)
#undef CBS_CDR_ROW_CASE
    default:
      break;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_cdr_col(Params<R> p) {
  extern __shared__ float4 smem_raw[];
  cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
  const int2 w = p.items[blockIdx.x];
  const InstDesc d = p.inst[w.x];
  switch (d.n) {
#define CBS_CDR_COL_CASE(N) \
  case N:                   \
    cdr_col_dispatch_n<R, N>(p, d, w.y, lds); \
    break;
    CBS_FOR_EACH_N(CBS_CDR_COL_CASE)
#undef CBS_CDR_COL_CASE
    default:
      break;
  }
}

// Coefficient fields (kappa, sigma) and (vx, vy) -> their deviations from the
// instance's background constants, in place (one row work item per block).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_cdr_split(const InstDesc* inst, const int2* items,
                                                        cpx<R>* c1, cpx<R>* c2) {
  const int2 w = items[blockIdx.x];
  const InstDesc d = inst[w.x];
  const long long base = d.off + (long long)w.y * d.n;
  const int cnt = min(d.rpw, d.n - w.y) * d.n;
  for (int j = threadIdx.x; j < cnt; j += kThreads) {
    const cpx<R> a = c1[base + j], b = c2[base + j];
    c1[base + j] = cpx<R>{a.x - R(d.k0sq), a.y - R(d.eps)};
    c2[base + j] = cpx<R>{b.x - R(d.vx0), b.y - R(d.vy0)};
  }
}

}  // namespace cbs
