// Spectral-derivative passes for convection-diffusion-reaction plans (App. B.1,
// Eqs. cdr_pde, cdr_L0 and cdr_V; the symbol of G_cdr is Eq. cdr_G_symbol,
// restated in App. C, "CDR case").
//
// V_cdr u = d/dx(dkappa du/dx) + d/dy(dkappa du/dy) - dv . grad u - dsigma u
// needs derivatives of products with the coefficient fields, so it is not
// one Fourier multiplier as G_cdr is.  A derivative along x is diagonal after
// the row transform alone and one along y after the column transform alone,
// so each axis takes one pass that keeps its rows (or columns) in LDS:
// forward 1D transform, times i xi / N (xi = 2 pi m / N on the signed index
// m, Nyquist bin -N/2), inverse, the pointwise product with the coefficients,
// forward, times i xi / N, inverse.
//
//   column pass   p_y = Dy(dkappa Dy u) - dvy Dy u                 (forward)
//                 p_y = Dy(dkappa Dy g + dvy g)                     (adjoint)
//   row pass      t = Dx(dkappa Dx u) - dvx Dx u - dsigma u + s + p_y = V u + s
//                 (MODE 0: then the forward row transform of t, i.e. the
//                 first pass of G t, into the spectral buffer; MODE 1: t
//                 itself into out)
//                 out = e - (Dx(dkappa Dx g + dvx g) + p_y - dsigma g)
//                 = e - V^H g   (MODE 2; V^H for real coefficients, D^H = -D)
//
// The term that is not differentiated a second time (-dvx Dx u ... on the
// forward side) is formed at the middle step and kept until the last
// transform adds it: in registers when the plan's first and last radix agree
// (each thread then holds the same elements at both stages), else parked in
// global memory (the pass's own output rows or columns), the workgroup's
// barriers ordering the two accesses.
// Field roles: u = u (forward) or g (adjoint); s = s (forward) or e
// (adjoint); b = p_y (row pass); k2 = (dkappa, dsigma); k2b = (dvx, dvy).
#pragma once
#include "kernels.hpp"

namespace cbs {

// Twiddles of one transform length, held in LDS by the FP32 passes: each pass
// of each of the chained transforms would otherwise fetch its twiddles from
// memory again, and these passes are bound by that latency.
__host__ __device__ constexpr int cdr_tw_max() {
  const int sizes[] = {16, 32, 64, 128, 192, 256, 288, 384, 512, 1024};
  int m = 0;
  for (int n : sizes) m = tw_size(n) > m ? tw_size(n) : m;
  return m;
}
constexpr int kCdrTwMax = cdr_tw_max();
static_assert(kCdrTwMax % 2 == 0, "the LDS table is declared as float4 (16-byte aligned)");

// FP32 passes copy the twiddles of length N into tws, q-major (conflict-free
// LDS reads by consecutive butterflies), and run every transform from there;
// FP64 passes keep the global table.
template <typename R, int N>
__device__ __forceinline__ auto cdr_twiddles(const cpx<R>* tw, float4* tws) {
  if constexpr (sizeof(R) == 4) {
    static_assert(twq_size(N) <= kCdrTwMax, "twiddle table");
    cpx<R>* dst = reinterpret_cast<cpx<R>*>(tws);
    twq_fill<R, N>(tw, dst, kThreads);
    __syncthreads();
    return TwQ<R>{dst};
  } else {
    return tw;
  }
}

// i xi(e) / N * v for bin e of a length-N transform
template <typename R, int N>
__device__ __forceinline__ cpx<R> deriv_factor(int e, cpx<R> v) {
  const int m = e >= N / 2 ? e - N : e;
  const R f = R(6.283185307179586476925287 * double(m) / (double(N) * double(N)));
  return cpx<R>{-v.y * f, v.x * f};
}

template <typename R, int N, int MODE>
__device__ __forceinline__ void cdr_row_body(const Params<R>& p, const InstDesc& d, int row0, cpx<R>* lds,
                                             float4* tws) {
  using T = RowTile<N>;
  const auto tw = cdr_twiddles<R, N>(p.tw, tws);
  const int tid = threadIdx.x;
  const int r = tid / T::TPF, t = tid - r * T::TPF;
  const int nrows = min(T::RPW, N - row0);
  const bool active = r < nrows;
  const long long rbase = d.off + (long long)(row0 + (active ? r : 0)) * N;
  cpx<R>* mine = lds + (active ? r : 0) * T::RS;
  cpx<R>* park = MODE == 0 ? p.inter : p.out;  // holds the undifferentiated part
  auto ld_u = [&](int e) { return p.u[rbase + e]; };
  auto ld_l = [&](int e) { return lds_ld(mine + lds_pos(e)); };
  auto st_d = [&](int e, cpx<R> v) { mine[lds_pos(e)] = deriv_factor<R, N>(e, v); };
  // middle step: dx -> dkappa dx (+ dvx g), and the rest of the row's terms
  auto st_m = [&](int e, cpx<R> dx) {
    const long long g = rbase + e;
    const cpx<R> c1 = p.k2[g];
    const cpx<R> c2 = p.k2b[g];
    const cpx<R> u = p.u[g];
    cpx<R> w = cscale(dx, c1.x);
    if constexpr (MODE == 2) {
      w = w + cscale(u, c2.x);
    } else {
      park[g] = p.b[g] - cscale(dx, c2.x) - cscale(u, c1.y) + ld_or_zero(p.s, g);
    }
    mine[lds_pos(e)] = w;
  };
  auto st_f = [&](int e, cpx<R> v) {
    const long long g = rbase + e;
    if constexpr (MODE == 2) {
      const cpx<R> vh = v + p.b[g] - cscale(p.u[g], p.k2[g].y);
      p.out[g] = p.s[g] - vh;
    } else {
      p.out[g] = v + p.out[g];
    }
  };
  auto st_s = [&](int e, cpx<R> v) { p.inter[rbase + e] = v; };
  if constexpr (plan_bridgeable(N)) {
    // The transforms chained through register bridges (fewer LDS round
    // trips).  The first pass, every bridge and the last pass give this
    // thread the same elements (slots p, q), so u and the part that is not
    // differentiated again stay in registers between the stages instead of
    // being parked in memory.
    constexpr int PL = plan_passes(N) - 1;
    constexpr int RAD = plan_radix(N, 0);
    constexpr int PER = (N / RAD + T::TPF - 1) / T::TPF;
    cpx<R> ureg[PER][RAD];  // u (or g) at the thread's elements
    cpx<R> preg[PER][RAD];  // the undifferentiated part
    auto none = [](int, cpx<R>) {};
    auto noload = [](int) { return cpx<R>{R(0), R(0)}; };
    auto ld_ur = [&](int e, int pp, int qq) {
      const cpx<R> x = p.u[rbase + e];
      ureg[pp][qq] = x;
      return x;
    };
    auto dmul = [&](int e, cpx<R> v) { return deriv_factor<R, N>(e, v); };
    auto mmid = [&](int e, cpx<R> dx, int pp, int qq) {
      const long long g = rbase + e;
      const cpx<R> c1 = p.k2[g];
      const cpx<R> c2 = p.k2b[g];
      const cpx<R> u = ureg[pp][qq];
      cpx<R> w = cscale(dx, c1.x);
      if constexpr (MODE == 2) w = w + cscale(u, c2.x);
      else preg[pp][qq] = p.b[g] - cscale(dx, c2.x) - cscale(u, c1.y) + ld_or_zero(p.s, g);
      return w;
    };
    fft_pass<R, N, 0, PL, T::TPF, -1, false, false, 1>(mine, t, active, tw, ld_ur, none);
    fft_bridge<R, N, T::TPF, -1, 1, 1>(mine, t, active, tw, dmul);
    fft_inner<R, N, T::TPF, 1, 1>(mine, t, active, tw);
    fft_bridge<R, N, T::TPF, 1, -1, 1>(mine, t, active, tw, mmid);
    fft_inner<R, N, T::TPF, -1, 1>(mine, t, active, tw);
    fft_bridge<R, N, T::TPF, -1, 1, 1>(mine, t, active, tw, dmul);
    if constexpr (MODE == 0) {
      auto tmid = [&](int e, cpx<R> v, int pp, int qq) { return v + preg[pp][qq]; };
      fft_inner<R, N, T::TPF, 1, 1>(mine, t, active, tw);
      fft_bridge<R, N, T::TPF, 1, -1, 1>(mine, t, active, tw, tmid);
      fft_pass<R, N, 1, PL + 1, T::TPF, -1, false, false, 1>(mine, t, active, tw, noload, st_s);
    } else if constexpr (MODE == 1) {
      auto st_p = [&](int e, cpx<R> v, int pp, int qq) { p.out[rbase + e] = v + preg[pp][qq]; };
      fft_pass<R, N, 1, PL + 1, T::TPF, 1, false, false, 1>(mine, t, active, tw, noload, st_p);
    } else {
      auto st_a = [&](int e, cpx<R> v, int pp, int qq) {
        const long long g = rbase + e;
        const cpx<R> vh = v + p.b[g] - cscale(ureg[pp][qq], p.k2[g].y);
        p.out[g] = p.s[g] - vh;
      };
      fft_pass<R, N, 1, PL + 1, T::TPF, 1, false, false, 1>(mine, t, active, tw, noload, st_a);
    }
  } else {
    fft_run<R, N, T::TPF, -1, false, true>(mine, t, active, tw, ld_u, st_d);
    fft_run<R, N, T::TPF, 1, true, true>(mine, t, active, tw, ld_l, st_m);
    fft_run<R, N, T::TPF, -1, true, true>(mine, t, active, tw, ld_l, st_d);
    if constexpr (MODE == 0) {
      auto st_t = [&](int e, cpx<R> v) { mine[lds_pos(e)] = v + p.inter[rbase + e]; };
      fft_run<R, N, T::TPF, 1, true, true>(mine, t, active, tw, ld_l, st_t);
      fft_run<R, N, T::TPF, -1, true, false>(mine, t, active, tw, ld_l, st_s);
    } else {
      fft_run<R, N, T::TPF, 1, true, false>(mine, t, active, tw, ld_l, st_f);
    }
  }
}

// Column tile of C columns, layout as in col_body (element-interleaved)
template <typename R, int N, int C, int ADJ>
__device__ __forceinline__ void cdr_col_body(const Params<R>& p, const InstDesc& d, int col0, cpx<R>* lds,
                                             float4* tws) {
  constexpr int TPC = kThreads / C;
  const auto tw = cdr_twiddles<R, N>(p.tw, tws);
  const int tid = threadIdx.x;
  const int c = tid % C, tt = tid / C;
  const long long cbase = d.off + col0 + c;
  cpx<R>* mine = lds + c;
  auto ld_u = [&](int e) { return p.u[cbase + (long long)e * N]; };
  auto ld_l = [&](int e) { return lds_ld(mine + C * lds_pos(e)); };
  auto st_d = [&](int e, cpx<R> v) { mine[C * lds_pos(e)] = deriv_factor<R, N>(e, v); };
  auto st_m = [&](int e, cpx<R> dy) {
    const long long g = cbase + (long long)e * N;
    const cpx<R> c1 = p.k2[g];
    const cpx<R> c2 = p.k2b[g];
    cpx<R> w = cscale(dy, c1.x);
    if constexpr (ADJ) w = w + cscale(p.u[g], c2.y);
    else p.out[g] = cscale(dy, -c2.y);
    mine[C * lds_pos(e)] = w;
  };
  auto st_f = [&](int e, cpx<R> v) {
    const long long g = cbase + (long long)e * N;
    if constexpr (ADJ) p.out[g] = v;
    else p.out[g] = v + p.out[g];
  };
  if constexpr (plan_bridgeable(N)) {
    // as in the row pass: u and the undifferentiated part in registers
    constexpr int PL = plan_passes(N) - 1;
    constexpr int RAD = plan_radix(N, 0);
    constexpr int PER = (N / RAD + TPC - 1) / TPC;
    cpx<R> ureg[PER][RAD];
    cpx<R> preg[PER][RAD];
    auto none = [](int, cpx<R>) {};
    auto noload = [](int) { return cpx<R>{R(0), R(0)}; };
    auto ld_ur = [&](int e, int pp, int qq) {
      const cpx<R> x = p.u[cbase + (long long)e * N];
      ureg[pp][qq] = x;
      return x;
    };
    auto dmul = [&](int e, cpx<R> v) { return deriv_factor<R, N>(e, v); };
    auto mmid = [&](int e, cpx<R> dy, int pp, int qq) {
      const long long g = cbase + (long long)e * N;
      const cpx<R> c1 = p.k2[g];
      const cpx<R> c2 = p.k2b[g];
      cpx<R> w = cscale(dy, c1.x);
      if constexpr (ADJ) w = w + cscale(ureg[pp][qq], c2.y);
      else preg[pp][qq] = cscale(dy, -c2.y);
      return w;
    };
    auto st_p = [&](int e, cpx<R> v, int pp, int qq) {
      const long long g = cbase + (long long)e * N;
      if constexpr (ADJ) p.out[g] = v;
      else p.out[g] = v + preg[pp][qq];
    };
    fft_pass<R, N, 0, PL, TPC, -1, false, false, C>(mine, tt, true, tw, ld_ur, none);
    fft_bridge<R, N, TPC, -1, 1, C>(mine, tt, true, tw, dmul);
    fft_inner<R, N, TPC, 1, C>(mine, tt, true, tw);
    fft_bridge<R, N, TPC, 1, -1, C>(mine, tt, true, tw, mmid);
    fft_inner<R, N, TPC, -1, C>(mine, tt, true, tw);
    fft_bridge<R, N, TPC, -1, 1, C>(mine, tt, true, tw, dmul);
    fft_pass<R, N, 1, PL + 1, TPC, 1, false, false, C>(mine, tt, true, tw, noload, st_p);
  } else {
    fft_run<R, N, TPC, -1, false, true, C>(mine, tt, true, tw, ld_u, st_d);
    fft_run<R, N, TPC, 1, true, true, C>(mine, tt, true, tw, ld_l, st_m);
    fft_run<R, N, TPC, -1, true, true, C>(mine, tt, true, tw, ld_l, st_d);
    fft_run<R, N, TPC, 1, true, false, C>(mine, tt, true, tw, ld_l, st_f);
  }
}

template <typename R, int N, int ADJ>
__device__ __forceinline__ void cdr_col_dispatch_n(const Params<R>& p, const InstDesc& d, int col0,
                                                   cpx<R>* lds, float4* tws) {
  constexpr int C0 = col_tile_default(N);
  constexpr int EB = int(sizeof(cpx<R>));
  const int c = sizeof(R) == 4 ? d.ctile : d.ctile64;
  if constexpr (col_tile_valid(N, C0, EB))
    if (c == C0) { cdr_col_body<R, N, C0, ADJ>(p, d, col0, lds, tws); return; }
  if constexpr (col_tile_valid(N, C0 / 2, EB))
    if (c == C0 / 2) { cdr_col_body<R, N, (C0 / 2 >= 2 ? C0 / 2 : 2), ADJ>(p, d, col0, lds, tws); return; }
  if constexpr (col_tile_valid(N, C0 * 2, EB))
    if (c == C0 * 2) { cdr_col_body<R, N, (C0 * 2 <= 32 ? C0 * 2 : 32), ADJ>(p, d, col0, lds, tws); return; }
}

template <typename R, int MODE>
__global__ __launch_bounds__(kThreads) void k_cdr_row(Params<R> p) {
  __shared__ cpx<R> lds[kRowLds];
  __shared__ float4 tws[sizeof(R) == 4 ? kCdrTwMax / 2 : 1];
  const int2 w = p.items[blockIdx.x];
  const InstDesc d = p.inst[w.x];
  switch (d.n) {
#define CBS_CDR_ROW_CASE(N) \
  case N:                   \
    cdr_row_body<R, N, MODE>(p, d, w.y, lds, tws); \
    break;
    CBS_FOR_EACH_N(CBS_CDR_ROW_CASE)
#undef CBS_CDR_ROW_CASE
    default:
      break;
  }
}

template <typename R, int ADJ>
__global__ __launch_bounds__(kThreads) void k_cdr_col(Params<R> p) {
  extern __shared__ float4 smem_raw[];
  __shared__ float4 tws[sizeof(R) == 4 ? kCdrTwMax / 2 : 1];
  cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
  const int2 w = p.items[blockIdx.x];
  const InstDesc d = p.inst[w.x];
  switch (d.n) {
#define CBS_CDR_COL_CASE(N) \
  case N:                   \
    cdr_col_dispatch_n<R, N, ADJ>(p, d, w.y, lds, tws); \
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
    c1[base + j] = cpx<R>{re_v(a.x, d.k0sq), a.y - R(d.eps)};
    c2[base + j] = cpx<R>{b.x - R(d.vx0), b.y - R(d.vy0)};
  }
}

}  // namespace cbs
