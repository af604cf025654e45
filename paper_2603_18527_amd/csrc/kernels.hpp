// HIP kernels of the CBS operator for gfx950 (device templates).
//
// One application y = G(V u + s) is three launches over a ragged work list
// that covers every instance of the batch:
//   k_row_fwd : prologue (V u + s) and forward row FFTs -> spectral buffer;
//   k_col     : a tile of C full columns: forward column FFTs, multiply by
//               the Green symbol 1/(N^2 lambda) (fused into the last forward
//               pass), inverse column FFTs, written back in place;
//   k_row_inv : inverse row FFTs and the epilogue (store, Born residual,
//               CBS update, adjoint step ...) with per-block FP64 partial
//               sums of |r|^2.
// k_row_sweep fuses the inverse rows and CBS update of one sweep with the
// prologue and forward rows of the next.  Prologue/epilogue/symbol variants
// are selected by uniform runtime modes.
#pragma once
#include <hip/hip_runtime.h>

#include "params.hpp"

namespace cbs {

__device__ __forceinline__ bool inst_enabled(const int* mask, int mode, int i) {
  if (!mask) return true;
  // atomic: a column launch may update an instance's status while other
  // workgroups of the same launch read it (k_col's folded check)
  const int m = __hip_atomic_load(mask + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (mode == MASK_RUNNING) return m == ST_RUNNING;
  if (mode == MASK_NOT_FINAL) return m == ST_RUNNING || m == ST_PENDING;
  return m != 0;
}

template <typename R>
__device__ __forceinline__ cpx<R> ld_or_zero(const cpx<R>* p, long long i) {
  return p ? p[i] : cpx<R>{R(0), R(0)};
}

// Re V = Re k^2 - k0^2.  In FP32, k0^2 enters as two parts (hi, its rounding;
// lo, the rest): Re k^2 - hi is exact while Re k^2 lies within a factor of two
// of hi, so Re V carries one rounding of its own size instead of one of the
// size of k0^2, which relative to |V| <= eps would be k0^2 / eps times larger.
template <typename R>
__device__ __forceinline__ R re_v(R kx, double k0sq) {
  const R hi = R(k0sq);
  if constexpr (sizeof(R) == 4) return (kx - hi) - R(k0sq - double(hi));
  return kx - hi;
}

template <typename R>
struct Coef {
  cpx<R> v;    // V = k^2 - k0^2 - i eps
  R inv_eps;
  __device__ __forceinline__ cpx<R> gamma() const { return {-v.y * inv_eps, v.x * inv_eps}; }
  __device__ __forceinline__ cpx<R> gamma_conj() const { return {-v.y * inv_eps, -v.x * inv_eps}; }
};

template <typename R>
__device__ __forceinline__ Coef<R> coef_of(const InstDesc& d, cpx<R> k) {
  Coef<R> c;
  c.v = {re_v(k.x, d.k0sq), k.y - R(d.eps)};
  c.inv_eps = R(1.0 / d.eps);
  return c;
}

template <typename R>
__device__ __forceinline__ Coef<R> coef(const Params<R>& p, const InstDesc& d, long long i) {
  const cpx<R> k = p.k2[i];
  Coef<R> c;
  c.v = {re_v(k.x, d.k0sq), k.y - R(d.eps)};
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
    case PRO_A:
      return p.a[i];
    default:  // PRO_U
      return ld_or_zero(p.u, i);
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
    case EPI_PHYS_SEED: {
      // e = a = s - A u_K, z = -Lap e; loss term |e|^2;
      // lam_K = -2 A^H e = -2 (z - conj(k^2) e); grad += 2 conj(u_K) e
      const cpx<R> e = p.a[i];
      const cpx<R> k = p.k2[i];
      p.out[i] = cscale(z - cmulc(k, e), R(-2));
      p.out2[i] = p.out2[i] + cscale(cmulc(p.u[i], e), R(2));
      return double(cabs2(e));
    }
    case EPI_NPBS: {
      // linear Fourier layer applied to r = a: u += F^-1(W^F F r) + W^loc r
      const cpx<R> r = p.a[i];
      p.out[i] = p.u[i] + z + cmul(ld_or_zero(p.b, i), r);
      return 0.0;
    }
    case EPI_BORN_ADJ: {
      const Coef<R> c = coef(p, d, i);
      p.out[i] = p.a[i] - cmulc(c.v, z);
      return 0.0;
    }
    default: {  // EPI_LAP: physical residual s - A u with A u = -Lap u - k^2 u
      const cpx<R> u = ld_or_zero(p.u, i);
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
// Sum of an instance's partial slots by one full wavefront: lane l adds
// slots l, l+64, ..., then a fixed shuffle tree (deterministic).
__device__ __forceinline__ double instance_sum(const double* partials, const InstDesc& d) {
  double s = 0.0;
  for (int k = threadIdx.x & 63; k < d.nparts; k += 64) s += partials[d.part_off + k];
  return wave_sum(s);
}

// FP32 convergence check of instance i after a correction sweep (one full
// wavefront): count the sweep, record the estimate ||r|| / ||G s|| and flag
// the instance ST_PENDING once it is at or below rtol or out of sweeps.
__device__ __forceinline__ void check32_instance(const IterState& st, const InstDesc* inst,
                                                 const double* partials, int i) {
  if (__hip_atomic_load(st.status + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ST_RUNNING)
    return;
  const InstDesc d = inst[i];
  const double sum = instance_sum(partials, d);
  if ((threadIdx.x & 63) != 0) return;
  const double bn = st.bnorm[i] > 0.0 ? st.bnorm[i] : 1.0;
  const double rel = sqrt(sum) / bn;
  st.est[i] = rel;
  st.iters[i] += 1;
  if (!(rel > st.rtol[0]) || st.iters[i] >= st.max_sweeps[0])
    __hip_atomic_store(st.status + i, int(ST_PENDING), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// The bridge step of a fused sweep (MODE 2 with a bridged plan): for each of
// the thread's elements, z from the inverse rows gives r = z - u + rhs and
// u_new = u + gamma r (written), and the value returned is the next sweep's
// V u_new + s.  A fused sweep takes rhs (correction sweeps) or s (plain
// sweeps) or neither, never both (the host checks).  pre() loads u, k^2 and
// that one field for all elements before the first store, without branches
// (a field that is absent is read from u and scaled by zero), so that the
// loads are in flight together.
template <typename R, int PER, int RAD>
struct SweepMid {
  const Params<R>& p;
  const InstDesc& d;
  long long rbase;
  double& acc;
  cpx<R> u[PER][RAD], k[PER][RAD], a[PER][RAD];
  // __host__ __device__, like the lambdas the bridge otherwise takes, so that
  // the bridge's compile-time checks for the call forms see them
  __host__ __device__ __forceinline__ void pre(int e, int pp, int qq) {
    const long long g = rbase + e;
    const cpx<R>* x = p.rhs ? p.rhs : p.s ? p.s : p.u;
    u[pp][qq] = p.u[g];
    k[pp][qq] = p.k2[g];
    a[pp][qq] = x[g];
  }
  __host__ __device__ __forceinline__ cpx<R> operator()(int e, cpx<R> z, int pp, int qq) {
    const R wr = p.rhs ? R(1) : R(0);
    const R ws = !p.rhs && p.s ? R(1) : R(0);
    const cpx<R> uu = u[pp][qq];
    const cpx<R> rres = z - uu + cscale(a[pp][qq], wr);
    const Coef<R> c = coef_of(d, k[pp][qq]);
    const cpx<R> un = uu + cmul(c.gamma(), rres);
    p.out[rbase + e] = un;
    acc += double(cabs2(rres));
    return cmul(c.v, un) + cscale(a[pp][qq], ws);
  }
};

// The bridge step of the two halves of a fused NPBS step (MODE 3: r = z - u,
// kept in out2; MODE 4: u_new = u + z + W^loc r, written, and the next step's
// V u_new + s returned).  The results are stored by post(), which the
// bridge calls after each group of kPostGroup elements, so a group's loads
// are issued ahead of its stores (all eight at once need more registers than
// the latency they hide is worth).
template <typename R, int PER, int RAD, int MODE>
struct NpbsMid {
  static constexpr int kPostGroup = RAD % 4 == 0 ? 4 : RAD;
  const Params<R>& p;
  const InstDesc& d;
  long long rbase;
  cpx<R> res[PER][RAD];  // r (MODE 3) or u_new (MODE 4), stored by post()
  // __host__ __device__, like the lambdas the bridge otherwise takes, so that
  // the bridge's compile-time checks for the call forms see them
  __host__ __device__ __forceinline__ cpx<R> operator()(int e, cpx<R> z, int pp, int qq) {
    const long long g = rbase + e;
    const cpx<R> u = p.u[g];
    if constexpr (MODE == 3) {
      const cpx<R> rr = z - u;
      res[pp][qq] = rr;
      return rr;
    } else {
      const cpx<R> un = u + z + cmul(ld_or_zero(p.b, g), p.a[g]);
      res[pp][qq] = un;
      const Coef<R> c = coef(p, d, g);
      return cmul(c.v, un) + ld_or_zero(p.s, g);
    }
  }
  __host__ __device__ __forceinline__ void post(int e, int pp, int qq) {
    if constexpr (MODE == 3) p.out2[rbase + e] = res[pp][qq];
    else p.out[rbase + e] = res[pp][qq];
  }
};

// MODE 0: prologue + forward rows -> spectral buffer;
// MODE 1: spectral buffer -> inverse rows -> epilogue (with partial norms);
// MODE 2: spectral buffer -> inverse rows -> sweep epilogue u += gamma r
//         (written to global) -> next sweep's prologue V u + s formed from
//         the value just computed -> forward rows -> spectral buffer.
// MODE 3 / 4: the two halves of a fused NPBS step with a linear Fourier
//         layer: after the Green pass r = z - u (kept in out2) -> forward rows
//         of r; after the layer's spectral pass u += z + W^loc r (written) ->
//         forward rows of the next step's V u + s.
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
  } else if constexpr (MODE == 5) {
    // the adjoint step's two forward row transforms (Sec. 4.2): V u + s, whose
    // Green transform gives the Born residual r, into inter, and
    // conj(gamma) lambda into inter2
    auto ld_a = [&](int e) {
      const long long g = rbase + e;
      const Coef<R> c = coef(p, d, g);
      return cmul(c.v, p.u[g]) + ld_or_zero(p.s, g);
    };
    auto st_a = [&](int e, cpx<R> v) { p.inter[rbase + e] = v; };
    fft_run<R, N, T::TPF, -1, false, false>(mine, t, active, p.tw, ld_a, st_a);
    __syncthreads();  // the second transform reuses the rows' LDS
    auto ld_b = [&](int e) {
      const long long g = rbase + e;
      const Coef<R> c = coef(p, d, g);
      return cmul(c.gamma_conj(), p.a[g]);
    };
    auto st_b = [&](int e, cpx<R> v) { p.inter2[rbase + e] = v; };
    fft_run<R, N, T::TPF, -1, false, false>(mine, t, active, p.tw, ld_b, st_b);
  } else if constexpr (MODE == 6) {
    // inverse rows of both: r = z_r - u stays in registers (the last pass of
    // both transforms gives each thread the same cells in the same slots),
    // then the adjoint epilogue of z = G^H(conj(gamma) lambda):
    // lambda_out = lambda + conj(V) z - conj(gamma) lambda,
    // grad += (-i/eps) lambda conj(r) + z conj(u)
    constexpr int RL = plan_radix(N, plan_passes(N) - 1);
    constexpr int PERL = (N / RL + T::TPF - 1) / T::TPF;
    cpx<R> rr[PERL][RL];
    auto ld_a = [&](int e) { return p.inter[rbase + e]; };
    auto st_a = [&](int e, cpx<R> z, int pp, int qq) { rr[pp][qq] = z - p.u[rbase + e]; };
    fft_run<R, N, T::TPF, 1, false, false>(mine, t, active, p.tw, ld_a, st_a);
    __syncthreads();  // the second transform reuses the rows' LDS
    auto ld_b = [&](int e) { return p.inter2[rbase + e]; };
    auto st_b = [&](int e, cpx<R> z, int pp, int qq) {
      const long long g = rbase + e;
      const Coef<R> c = coef(p, d, g);
      const cpx<R> lam = p.a[g];
      const cpx<R> r = rr[pp][qq];
      const cpx<R> u = p.u[g];
      p.out[g] = lam + cmulc(c.v, z) - cmul(c.gamma_conj(), lam);
      const cpx<R> lr = cmul(lam, cconj(r));
      const cpx<R> g0 = cpx<R>{lr.y * c.inv_eps, -lr.x * c.inv_eps};
      p.out2[g] = p.out2[g] + g0 + cmul(z, cconj(u));
    };
    fft_run<R, N, T::TPF, 1, false, false>(mine, t, active, p.tw, ld_b, st_b);
  } else if constexpr (MODE == 3 || MODE == 4) {
    auto ld = [&](int e) { return p.inter[rbase + e]; };
    auto mid = [&](int e, cpx<R> z) {
      const long long g = rbase + e;
      const cpx<R> u = p.u[g];
      if constexpr (MODE == 3) {
        const cpx<R> rr = z - u;
        p.out2[g] = rr;
        return rr;
      } else {
        const cpx<R> un = u + z + cmul(ld_or_zero(p.b, g), p.a[g]);
        p.out[g] = un;
        const Coef<R> c = coef(p, d, g);
        return cmul(c.v, un) + ld_or_zero(p.s, g);
      }
    };
    auto st2 = [&](int e, cpx<R> v) { p.inter[rbase + e] = v; };
    if constexpr (plan_bridgeable(N)) {
      constexpr int RAD = plan_radix(N, 0);
      constexpr int PER = (N / RAD + T::TPF - 1) / T::TPF;
      NpbsMid<R, PER, RAD, MODE> bm{p, d, rbase};
      fft_run2<R, N, T::TPF, 1, -1>(mine, t, active, p.tw, ld, bm, st2);
    } else {
      auto st = [&](int e, cpx<R> z) { mine[lds_pos(e)] = mid(e, z); };
      fft_run<R, N, T::TPF, 1, false, true>(mine, t, active, p.tw, ld, st);
      auto ld2 = [&](int e) { return lds_ld(mine + lds_pos(e)); };
      fft_run<R, N, T::TPF, -1, true, false>(mine, t, active, p.tw, ld2, st2);
    }
  } else {
    double acc = 0.0;
    auto ld = [&](int e) { return p.inter[rbase + e]; };
    // u_new = u + gamma (z - u + rhs), written out; returns V u_new + s
    auto update = [&](int e, cpx<R> z) {
      const long long g = rbase + e;
      const cpx<R> u = p.u[g];
      const cpx<R> rres = z - u + ld_or_zero(p.rhs, g);
      const Coef<R> c = coef(p, d, g);
      const cpx<R> un = u + cmul(c.gamma(), rres);
      p.out[g] = un;
      acc += double(cabs2(rres));
      return cmul(c.v, un) + ld_or_zero(p.s, g);
    };
    auto st2 = [&](int e, cpx<R> v) { p.inter[rbase + e] = v; };
    if constexpr (plan_bridgeable(N)) {
      constexpr int RAD = plan_radix(N, 0);
      constexpr int PER = (N / RAD + T::TPF - 1) / T::TPF;
      SweepMid<R, PER, RAD> mid{p, d, rbase, acc};
      fft_run2<R, N, T::TPF, 1, -1>(mine, t, active, p.tw, ld, mid, st2);
    } else {
      auto st = [&](int e, cpx<R> z) { mine[lds_pos(e)] = update(e, z); };
      fft_run<R, N, T::TPF, 1, false, true>(mine, t, active, p.tw, ld, st);
      auto ld2 = [&](int e) { return lds_ld(mine + lds_pos(e)); };
      fft_run<R, N, T::TPF, -1, true, false>(mine, t, active, p.tw, ld2, st2);
    }
    if (p.partials) {
      const double s = block_sum(acc, red);
      if (tid == 0) p.partials[d.part_off + row0 / T::RPW] = s;
    }
  }
}

template <typename R, int MODE>
__device__ __forceinline__ void row_dispatch(const Params<R>& p) {
  __shared__ cpx<R> lds[kRowLds];
  __shared__ double red[kThreads / 64];
  const int2 w = p.items[blockIdx.x];
  // the descriptor is loaded before the mask is tested, so the two loads are
  // in flight together
  const InstDesc d = p.inst[w.x];
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
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

// the adjoint step's forward / inverse rows over two fields (periodic plans)
template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_adj_fwd(Params<R> p) {
  row_dispatch<R, 5>(p);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_adj_inv(Params<R> p) {
  row_dispatch<R, 6>(p);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_npbs_a(Params<R> p) {
  row_dispatch<R, 3>(p);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_npbs_b(Params<R> p) {
  row_dispatch<R, 4>(p);
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
  R sc;
  if constexpr (sizeof(R) == 4) sc = inv_n2 * __builtin_amdgcn_rcpf(a * a + e * e);  // 1 ulp
  else sc = inv_n2 / (a * a + e * e);
  // 1/lambda = (a + i eps)/|lambda|^2 ; 1/conj(lambda) = (a - i eps)/|lambda|^2
  return cpx<R>{a * sc, (mode == SYM_GREEN ? e : -e) * sc};
}

// CDR symbol on DFT bin (k1 = row bin -> xi_y, k2 = column bin -> xi_x), with
// the 1/N^2 of the inverse transform.  L0 = a + i b, a = kappa0 |xi|^2 +
// sigma0 and b = v0 . xi formed in FP64.
template <typename R>
__device__ __forceinline__ cpx<R> cdr_symbol_factor(int n, int k1, int k2, const InstDesc& d, int mode) {
  const int my = k1 >= n / 2 ? k1 - n : k1;
  const int mx = k2 >= n / 2 ? k2 - n : k2;
  const double h = 6.283185307179586476925287 / double(n);
  const double xy = double(my) * h, xx = double(mx) * h;
  const R a = R(d.k0sq * (xx * xx + xy * xy) + d.eps);
  const R b = R(d.vx0 * xx + d.vy0 * xy);
  const R inv_n2 = R(1.0 / (double(n) * double(n)));
  if (mode == SYM_CDR_NEG_L0) return cpx<R>{-a * inv_n2, -b * inv_n2};
  R sc;
  if constexpr (sizeof(R) == 4) sc = inv_n2 * __builtin_amdgcn_rcpf(a * a + b * b);
  else sc = inv_n2 / (a * a + b * b);
  // 1/L0 = (a - i b)/|L0|^2 ; 1/conj(L0) = (a + i b)/|L0|^2
  return cpx<R>{a * sc, (mode == SYM_CDR ? -b : b) * sc};
}

// Column tile: C columns of one instance.  Thread tid works on column tid % C
// (so the C threads of a row segment read or write C neighbouring elements)
// and butterfly slot tid / C.  Between passes the tile sits in LDS
// element-interleaved (position x of column c at C * pos(x) + c), which keeps
// every pass's LDS reads and writes free of bank conflicts on gfx950.
template <typename R, int N, int C, int T = kThreads>
__device__ __forceinline__ void col_body(const Params<R>& p, const InstDesc& d, int col0,
                                         cpx<R>* lds) {
  constexpr int TPC = T / C;
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const long long cbase = d.off + col0 + c;
  const int kcol = col0 + c;
  cpx<R>* mine = lds + c;
  auto ld = [&](int e) { return p.inter[cbase + (long long)e * N]; };
  auto sym = [&](int e, cpx<R> v) {
    if (p.sym == SYM_TABLE)  // tabulated weights; 1/N^2 of the inverse transform
      return cscale(cmul(v, p.table[cbase + (long long)e * N]), R(1.0 / (double(N) * double(N))));
    if (p.sym >= SYM_CDR) return cmul(v, cdr_symbol_factor<R>(N, e, kcol, d, p.sym));
    return cmul(v, symbol_factor<R>(N, e, kcol, d.k0sq, d.eps, p.sym));
  };
  auto st2 = [&](int e, cpx<R> v) { p.inter[cbase + (long long)e * N] = v; };
  if constexpr (plan_bridgeable(N)) {
    // forward column transform, symbol, inverse transform; the last forward
    // and first inverse passes share registers
    fft_run2<R, N, TPC, -1, 1, C>(mine, t, true, p.tw, ld, sym, st2);
  } else {
    auto st = [&](int e, cpx<R> v) { mine[C * lds_pos(e)] = sym(e, v); };
    fft_run<R, N, TPC, -1, false, true, C>(mine, t, true, p.tw, ld, st);
    auto ld2 = [&](int e) { return lds_ld(mine + C * lds_pos(e)); };
    fft_run<R, N, TPC, 1, true, false, C>(mine, t, true, p.tw, ld2, st2);
  }
}

template <typename R, int N, int T = kThreads>
__device__ __forceinline__ void col_dispatch_n(const Params<R>& p, const InstDesc& d, int col0,
                                               cpx<R>* lds) {
  constexpr int C0 = col_tile_default(N);
  constexpr int EB = int(sizeof(cpx<R>));
  const int c = sizeof(R) == 4 ? d.ctile : d.ctile64;
  if constexpr (col_tile_valid_t(N, C0, EB, T))
    if (c == C0) { col_body<R, N, C0, T>(p, d, col0, lds); return; }
  if constexpr (T == kThreads && col_tile_valid(N, C0 / 2, EB))
    if (c == C0 / 2) { col_body<R, N, (C0 / 2 >= 2 ? C0 / 2 : 2), T>(p, d, col0, lds); return; }
  if constexpr (col_tile_valid_t(N, C0 * 2, EB, T))
    if (c == C0 * 2) { col_body<R, N, (C0 * 2 <= 32 ? C0 * 2 : 32), T>(p, d, col0, lds); return; }
}

template <typename R, int T>
__device__ __forceinline__ void col_kernel_body(const Params<R>& p) {
  extern __shared__ float4 smem_raw[];
  cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
  const int2 w = p.items[blockIdx.x];
  // the first tile's workgroup checks the sweep the previous launch finished
  // (the instance's next row launch sees the result; whether the other tiles
  // of this launch see it only decides whether they do work nobody reads)
  const InstDesc d = p.inst[w.x];
  if (p.check && w.y == 0 && threadIdx.x < 64) check32_instance(p.chk, p.inst, p.partials, w.x);
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  switch (d.n) {
#define CBS_COL_CASE(N) \
  case N:               \
    col_dispatch_n<R, N, T>(p, d, w.y, lds); \
    break;
    CBS_FOR_EACH_N(CBS_COL_CASE)
#undef CBS_COL_CASE
    default:
      break;
  }
  if (p.dual) {
    // the adjoint step's second field: the conjugate Green symbol on inter2
    __syncthreads();  // the second tile reuses the LDS
    Params<R> q = p;
    q.inter = p.inter2;
    q.sym = SYM_GREEN_CONJ;
    switch (d.n) {
#define CBS_COL_CASE2(N) \
  case N:                \
    col_dispatch_n<R, N, T>(q, d, w.y, lds); \
    break;
      CBS_FOR_EACH_N(CBS_COL_CASE2)
#undef CBS_COL_CASE2
      default:
        break;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_col(Params<R> p) {
  col_kernel_body<R, kThreads>(p);
}

// the same with kColThreadsWide threads per workgroup
template <typename R>
__global__ __launch_bounds__(kColThreadsWide) void k_col_wide(Params<R> p) {
  col_kernel_body<R, kColThreadsWide>(p);
}

// ---- pointwise kernels over row work items ------------------------------------------

template <typename R>
__global__ __launch_bounds__(kThreads) void k_pointwise(PwParams<R> p) {
  const int2 w = p.items[blockIdx.x];
  if (!inst_enabled(p.mask, p.mask_mode, w.x)) return;
  const InstDesc d = p.inst[w.x];
  const int n = d.n;
  const int rpw = d.rpw;
  const int nrows = min(rpw, n - w.y);
  const long long base = d.off + (long long)w.y * n;
  const int cnt = nrows * n;
  const R ie = R(1.0 / d.eps);
  const R ep = R(d.eps);
  const double sc = (p.op == PW_SCALE64) ? p.scale[w.x]
                    : (p.op == PW_SCALE)  ? p.factor * (p.scale ? p.scale[w.x] : 1.0)
                    : (p.op == PW_FIRST64 || p.op == PW_NARROW) ? (p.scale ? p.scale[w.x] : 1.0)
                                          : 1.0;
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
          v = cpx<R>{R(x.x * sc), R(x.y * sc)};
          if (p.c_out) p.c_out[i] = v;
        }
        const cpx<R> k = p.k2[i];
        const cpx<R> g{-(k.y - ep) * ie, re_v(k.x, d.k0sq) * ie};  // i V / eps
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
        p.e_out[i] = cpx<R>{R(x.x * sc), R(x.y * sc)};
        break;
      }
      case PW_SCALE:
        p.e_out[i] = cscale(p.e_in[i], R(sc));
        break;
      default: {  // PW_SCALE64
        const cpx<double> x = p.x64[i];
        p.x64[i] = cpx<double>{x.x * sc, x.y * sc};
        break;
      }
    }
  }
}

__device__ __forceinline__ void item_range(const InstDesc& d, int row0, long long& base, int& cnt,
                                           int& slot) {
  const int rpw = d.rpw;
  const int nrows = min(rpw, d.n - row0);
  base = d.off + (long long)row0 * d.n;
  cnt = nrows * d.n;
  slot = d.part_off + row0 / rpw;
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

}  // namespace cbs
