// Device FFT building blocks for gfx950: complex arithmetic, radix-2/3/4/8
// butterflies and a self-sorting (Stockham) mixed-radix pass over LDS.
//
// A length-N transform runs as a sequence of passes with radices r_0, r_1, ...
// (product N).  Before pass p the data holds DFTs of length Ns = r_0...r_{p-1}
// interleaved with stride N/Ns; butterfly j (0 <= j < N/r) reads elements
// j + q N/r (q < r), multiplies element q by w^(q k) with k = j mod Ns and
// w = exp(-+2 pi i / (Ns r)), applies an r-point DFT and writes element q to
// (j / Ns) Ns r + k + q Ns.  Output is in natural order; no bit reversal.
//
// Forward transforms use exp(-2 pi i j n / N), inverse ones exp(+...), both
// unnormalised; the 1/N^2 of the inverse 2D transform is folded into the
// Green-symbol multiply.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace cbs {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ R cabs2(cpx<R> a) { return a.x * a.x + a.y * a.y; }
// (DIR * i) * a with DIR = -1 (forward) or +1 (inverse)
template <int DIR, typename R>
__device__ __forceinline__ cpx<R> mul_dir_i(cpx<R> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// ---- butterflies (in registers) ------------------------------------------

template <int DIR, typename R>
__device__ __forceinline__ void bfly2(cpx<R>* v) {
  cpx<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <int DIR, typename R>
__device__ __forceinline__ void bfly4(cpx<R>* v) {
  cpx<R> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cpx<R> t2 = v[1] + v[3], t3 = mul_dir_i<DIR>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <int DIR, typename R>
__device__ __forceinline__ void bfly3(cpx<R>* v) {
  const R h = R(0.8660254037844386467637232);  // sin(pi/3)
  cpx<R> t1 = v[1] + v[2];
  cpx<R> t2 = v[0] - cscale(t1, R(0.5));
  cpx<R> t3 = mul_dir_i<DIR>(cscale(v[1] - v[2], h));
  v[0] = v[0] + t1;
  v[1] = t2 + t3;
  v[2] = t2 - t3;
}

template <int DIR, typename R>
__device__ __forceinline__ void bfly8(cpx<R>* v) {
  const R s = R(0.7071067811865475244008444);  // 1/sqrt(2)
  cpx<R> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<R> o[4] = {v[1], v[3], v[5], v[7]};
  bfly4<DIR>(e);
  bfly4<DIR>(o);
  // o[k] *= w8^k, w8 = exp(DIR i pi / 4)
  cpx<R> o1 = cscale(o[1] + mul_dir_i<DIR>(o[1]), s);     // (1 + DIR i)/sqrt2
  cpx<R> o2 = mul_dir_i<DIR>(o[2]);                        // DIR i
  cpx<R> o3 = cscale(mul_dir_i<DIR>(o[3]) - o[3], s);     // (-1 + DIR i)/sqrt2
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

template <int RAD, int DIR, typename R>
__device__ __forceinline__ void bfly(cpx<R>* v) {
  if constexpr (RAD == 2) bfly2<DIR>(v);
  else if constexpr (RAD == 3) bfly3<DIR>(v);
  else if constexpr (RAD == 4) bfly4<DIR>(v);
  else if constexpr (RAD == 8) bfly8<DIR>(v);
  else static_assert(RAD == 2, "unsupported radix");
}

// ---- size plans -------------------------------------------------------------

// Radix of pass p for length n (0 past the last pass).
__host__ __device__ constexpr int plan_radix(int n, int p) {
  switch (n) {
    case 16: return p < 2 ? 4 : 0;
    case 32: return p == 0 ? 8 : p == 1 ? 4 : 0;
    case 64: return p < 2 ? 8 : 0;
    case 128: return p == 0 ? 8 : p == 1 ? 2 : p == 2 ? 8 : 0;
    case 192: return p == 0 ? 8 : p == 1 ? 3 : p == 2 ? 8 : 0;
    case 256: return p == 0 ? 8 : p == 1 ? 4 : p == 2 ? 8 : 0;
    case 288: return p == 0 ? 8 : p == 1 ? 4 : p < 4 ? 3 : 0;
    case 384: return p == 0 ? 8 : p == 1 ? 2 : p == 2 ? 3 : p == 3 ? 8 : 0;
    case 512: return p < 3 ? 8 : 0;
    case 1024: return p == 0 ? 8 : p < 3 ? 4 : p == 3 ? 8 : 0;
    default: return 0;
  }
}

__host__ __device__ constexpr int plan_product(int n) {
  int prod = 1;
  for (int p = 0; plan_radix(n, p) > 0; ++p) prod *= plan_radix(n, p);
  return prod;
}

__host__ __device__ constexpr int plan_passes(int n) {
  int p = 0;
  while (plan_radix(n, p) > 0) ++p;
  return p;
}

// Length of the sub-transforms already formed before pass p.
__host__ __device__ constexpr int plan_ns(int n, int p) {
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= plan_radix(n, i);
  return ns;
}

// ---- twiddle tables ----------------------------------------------------------
//
// For pass p (Ns = plan_ns > 1, radix r) butterfly k (0 <= k < Ns) needs
// w^(q k), q = 1..r-1, w = exp(-2 pi i / (Ns r)).  They are stored
// contiguously per k, padded to radp(r) entries (entry 0 = 1), so one
// butterfly reads them with a few 16-byte loads.  Tables of all passes of all
// supported sizes are stored back to back.
__host__ __device__ constexpr int radp(int r) { return r == 3 ? 4 : r; }
__host__ __device__ constexpr int tw_pass_size(int n, int p) {
  return plan_ns(n, p) > 1 ? plan_ns(n, p) * radp(plan_radix(n, p)) : 0;
}
__host__ __device__ constexpr int tw_size(int n) {
  int s = 0;
  for (int p = 0; p < plan_passes(n); ++p) s += tw_pass_size(n, p);
  return s;
}
__host__ __device__ constexpr int tw_offset(int n) {
  int off = 0;
  const int sizes[] = {16, 32, 64, 128, 192, 256, 288, 384, 512, 1024};
  for (int i = 0; i < 10; ++i) {
    if (sizes[i] == n) return off;
    off += tw_size(sizes[i]);
  }
  return -1;
}
__host__ __device__ constexpr int tw_pass_offset(int n, int p) {
  int off = tw_offset(n);
  for (int i = 0; i < p; ++i) off += tw_pass_size(n, i);
  return off;
}
constexpr int kTwTotal = tw_offset(1024) + tw_size(1024);

// ---- LDS layout ------------------------------------------------------------------
//
// LDS positions are skewed by one element per eight, pos(e) = e + e/8, so the
// power-of-two strides of the Stockham writes (stride r in the first pass,
// blocks of Ns at stride Ns r later) spread over all banks.
__host__ __device__ constexpr int lds_pos(int e) { return e + (e >> 3); }
__host__ __device__ constexpr int lds_len(int n) { return lds_pos(n - 1) + 1; }

// pos(e + q * STEP) for q < RAD, given pos(e): a constant offset when STEP is a
// multiple of 8, or when e is a multiple of RAD, RAD divides 8 and STEP == 1
// (all RAD elements stay in one block of eight).
template <int STEP, int RAD>
__device__ __forceinline__ int lds_pos_step(int e, int pos_e, int q) {
  if constexpr (STEP % 8 == 0) return pos_e + q * (STEP + STEP / 8);
  else if constexpr (STEP == 1 && 8 % RAD == 0) return pos_e + q;
  else return lds_pos(e + q * STEP);
}

// One element from LDS.  FP32 elements are read by single 8-byte accesses
// (volatile, so the compiler does not pair neighbouring reads into
// ds_read2_b64: on gfx950 a paired read occupies the LDS for as many cycles
// as four single 8-byte reads of the same lanes).
template <typename R>
__device__ __forceinline__ cpx<R> lds_ld(const cpx<R>* p) {
  if constexpr (sizeof(R) == 4) {
    using lds_u64 = __attribute__((address_space(3))) const volatile unsigned long long;
    const unsigned long long b = *(lds_u64*)(p);
    return __builtin_bit_cast(cpx<R>, b);
  } else {
    return *p;
  }
}

template <typename R, int RADP>
__device__ __forceinline__ void load_tw(const cpx<R>* __restrict__ p, cpx<R>* w) {
  if constexpr (sizeof(R) == 4) {
    const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < RADP / 2; ++i) {
      const float4 v = p4[i];
      w[2 * i] = cpx<R>{v.x, v.y};
      w[2 * i + 1] = cpx<R>{v.z, v.w};
    }
  } else {
#pragma unroll
    for (int i = 0; i < RADP; ++i) w[i] = p[i];
  }
}

// Twiddles w^(q k) of butterfly k of pass P, fetched into w[0 .. radp(r)),
// and their multiply: v[q] *= w^(q k) (forward) or conj(w)^(q k) (inverse).
// The passes fetch a butterfly's twiddles before they read its inputs, so
// the fetch overlaps the LDS reads and the barrier that follows them.
template <typename R, int N, int P>
__device__ __forceinline__ void tw_fetch(cpx<R>* w, int k, const cpx<R>* __restrict__ tw) {
  constexpr int RP = radp(plan_radix(N, P));
  load_tw<R, RP>(tw + tw_pass_offset(N, P) + k * RP, w);
}
template <int RAD, int DIR, typename R>
__device__ __forceinline__ void tw_apply(cpx<R>* v, const cpx<R>* w) {
#pragma unroll
  for (int q = 1; q < RAD; ++q) v[q] = DIR < 0 ? cmul(w[q], v[q]) : cmulc(w[q], v[q]);
}

template <typename R, int N, int P, int DIR>
__device__ __forceinline__ void twiddle(cpx<R>* v, int k, const cpx<R>* __restrict__ tw) {
  constexpr int RAD = plan_radix(N, P);
  cpx<R> w[radp(RAD)];
  tw_fetch<R, N, P>(w, k, tw);
  tw_apply<RAD, DIR>(v, w);
}

// Twiddles of one transform length held q-major in LDS: for pass P (Ns > 1)
// entry (q, k), q = 1..r-1, sits at twq_pass_offset(N, P) + (q - 1) Ns + k, so
// the lanes of a wave, which work on consecutive butterflies k, read
// consecutive LDS words (the per-k layout of the global table puts them
// radp(r) entries apart, which serialises on the LDS banks).
__host__ __device__ constexpr int twq_pass_size(int n, int p) {
  return plan_ns(n, p) > 1 ? plan_ns(n, p) * (plan_radix(n, p) - 1) : 0;
}
__host__ __device__ constexpr int twq_pass_offset(int n, int p) {
  int off = 0;
  for (int i = 0; i < p; ++i) off += twq_pass_size(n, i);
  return off;
}
__host__ __device__ constexpr int twq_size(int n) { return twq_pass_offset(n, plan_passes(n)); }

template <typename R>
struct TwQ {
  const cpx<R>* base;  // LDS table of one transform length
};

template <typename R, int N, int P>
__device__ __forceinline__ void tw_fetch(cpx<R>* w, int k, TwQ<R> tw) {
  constexpr int RAD = plan_radix(N, P);
  constexpr int NS = plan_ns(N, P);
  const cpx<R>* b = tw.base + twq_pass_offset(N, P) + k;
#pragma unroll
  for (int q = 1; q < RAD; ++q) w[q] = lds_ld(b + (q - 1) * NS);
}

template <typename R, int N, int P, int DIR>
__device__ __forceinline__ void twiddle(cpx<R>* v, int k, TwQ<R> tw) {
  constexpr int RAD = plan_radix(N, P);
  cpx<R> w[radp(RAD)];
  tw_fetch<R, N, P>(w, k, tw);
  tw_apply<RAD, DIR>(v, w);
}

// Fills the q-major LDS table of length N from the global table (every
// thread of the workgroup calls it; `nthreads` = the workgroup size; the
// caller puts a barrier after it).
template <typename R, int N, int P = 0>
__device__ __forceinline__ void twq_fill(const cpx<R>* __restrict__ tw, cpx<R>* dst, int nthreads) {
  if constexpr (P < plan_passes(N)) {
    constexpr int NS = plan_ns(N, P);
    constexpr int RP = radp(plan_radix(N, P));
    if constexpr (NS > 1) {
      constexpr int CNT = twq_pass_size(N, P);
      for (int i = threadIdx.x; i < CNT; i += nthreads) {
        const int q = i / NS + 1, k = i - (q - 1) * NS;
        dst[twq_pass_offset(N, P) + i] = tw[tw_pass_offset(N, P) + k * RP + q];
      }
    }
    twq_fill<R, N, P + 1>(tw, dst, nthreads);
  }
}

// Functors of the first pass (ld), the last pass (st) and a bridge (mid) may
// also take the butterfly slot p and the element slot q of the thread's
// registers: in a plan whose first and last radix agree, every one of these
// stages gives thread t the same elements j + q N/r, j = t + p TPF, so a
// functor can keep per-element values in registers indexed by (p, q) from
// one stage to a later one.
template <class F, typename R>
__device__ __forceinline__ cpx<R> call_ld(F& f, int e, int p, int q) {
  if constexpr (std::is_invocable_v<F&, int, int, int>) return f(e, p, q);
  else return f(e);
}
template <class F, typename R>
__device__ __forceinline__ void call_st(F& f, int e, cpx<R> v, int p, int q) {
  if constexpr (std::is_invocable_v<F&, int, cpx<R>, int, int>) f(e, v, p, q);
  else f(e, v);
}
template <class F, typename R>
__device__ __forceinline__ cpx<R> call_mid(F& f, int e, cpx<R> v, int p, int q) {
  if constexpr (std::is_invocable_v<F&, int, cpx<R>, int, int>) return f(e, v, p, q);
  else return f(e, v);
}

// A bridge functor may also have pre(e, p, q): the bridge calls it for all of
// the thread's elements before it reads its inputs from LDS, so the functor
// can issue every global load it needs up front.  Without it a functor that
// loads and stores per element (an in-place update) gets its loads issued one
// element at a time: the compiler cannot move the next element's loads above
// a store that may alias them.
template <class F, class = void>
struct has_pre : std::false_type {};
template <class F>
struct has_pre<F, std::void_t<decltype(std::declval<F&>().pre(0, 0, 0))>> : std::true_type {};
// ... and post(e, p, q), which the bridge calls for all elements after the
// functor has run on every one of them: a functor can keep its stores there,
// so that no load of a later element waits behind a store of an earlier one.
// A functor may bound how many elements run before their post() calls with
// a constant kPostGroup (fewer loads in flight, fewer registers).
template <class F, class = void>
struct has_post : std::false_type {};
template <class F>
struct has_post<F, std::void_t<decltype(std::declval<F&>().post(0, 0, 0))>> : std::true_type {};
template <class F, int RAD, class = void>
struct post_group : std::integral_constant<int, RAD> {};
template <class F, int RAD>
struct post_group<F, RAD, std::void_t<decltype(F::kPostGroup)>> : std::integral_constant<int, F::kPostGroup> {};

// ---- one Stockham pass ----------------------------------------------------------
//
// TPF threads cooperate on one transform (t = 0..TPF-1); every thread of the
// workgroup calls this (barriers inside), `active` masks threads without a
// transform.  The first pass reads its inputs through `ld(e)` (element e of
// the transform, typically straight from global memory), the last pass hands
// its outputs to `st(e, v)`; the passes in between exchange data through LDS
// (`buf`, skewed positions, ES elements apart: position x of the transform is
// buf[ES * x], so ES transforms can share one buffer element-interleaved).
// LD_LDS / ST_LDS say that ld / st themselves touch this LDS buffer, which
// adds the barriers an in-place pass needs.
template <typename R, int N, int P, int PEND, int TPF, int DIR, bool LD_LDS, bool ST_LDS, int ES,
          class TW, class LD, class ST>
__device__ __forceinline__ void fft_pass_t(cpx<R>* buf, int t, bool active, TW tw, LD& ld, ST& st) {
  constexpr int RAD = plan_radix(N, P);
  constexpr int NS = plan_ns(N, P);
  constexpr int NB = N / RAD;
  constexpr bool FIRST = P == 0;
  constexpr bool LAST = P + 1 == plan_passes(N);
  constexpr int PER = (NB + TPF - 1) / TPF;
  constexpr bool EXACT = (NB % TPF) == 0;
  constexpr bool READS_LDS = !FIRST || LD_LDS;
  constexpr bool WRITES_LDS = !LAST || ST_LDS;
  cpx<R> v[PER][RAD];
  cpx<R> w[PER][radp(RAD)];
  if (active) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPF;
      if (EXACT || j < NB) {
        if constexpr (NS > 1) tw_fetch<R, N, P>(w[p], j % NS, tw);
        if constexpr (FIRST) {
#pragma unroll
          for (int q = 0; q < RAD; ++q) v[p][q] = call_ld<LD, R>(ld, j + q * NB, p, q);
        } else {
          const int pj = lds_pos(j);
#pragma unroll
          for (int q = 0; q < RAD; ++q) v[p][q] = lds_ld(buf + ES * lds_pos_step<NB, RAD>(j, pj, q));
        }
      }
    }
  }
  if constexpr (READS_LDS && WRITES_LDS) __syncthreads();
  if (active) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPF;
      if (EXACT || j < NB) {
        const int k = j % NS;
        if constexpr (NS > 1) tw_apply<RAD, DIR>(v[p], w[p]);
        bfly<RAD, DIR>(v[p]);
        const int o = (j / NS) * (NS * RAD) + k;
        if constexpr (LAST) {
#pragma unroll
          for (int q = 0; q < RAD; ++q) call_st<ST, R>(st, o + q * NS, v[p][q], p, q);
        } else {
          const int po = lds_pos(o);
#pragma unroll
          for (int q = 0; q < RAD; ++q) buf[ES * lds_pos_step<NS, RAD>(o, po, q)] = v[p][q];
        }
      }
    }
  }
  if constexpr (WRITES_LDS) __syncthreads();
  if constexpr (P + 1 < PEND)
    fft_pass_t<R, N, P + 1, PEND, TPF, DIR, LD_LDS, ST_LDS, ES>(buf, t, active, tw, ld, st);
}

// The passes above take the twiddle table as a restrict-qualified global
// pointer (the table is never written while a kernel runs) or as a q-major
// LDS table (TwQ).
template <typename R, int N, int P, int PEND, int TPF, int DIR, bool LD_LDS, bool ST_LDS, int ES,
          class LD, class ST>
__device__ __forceinline__ void fft_pass(cpx<R>* buf, int t, bool active, const cpx<R>* __restrict__ tw,
                                         LD& ld, ST& st) {
  fft_pass_t<R, N, P, PEND, TPF, DIR, LD_LDS, ST_LDS, ES>(buf, t, active, tw, ld, st);
}
template <typename R, int N, int P, int PEND, int TPF, int DIR, bool LD_LDS, bool ST_LDS, int ES,
          class LD, class ST>
__device__ __forceinline__ void fft_pass(cpx<R>* buf, int t, bool active, TwQ<R> tw, LD& ld, ST& st) {
  fft_pass_t<R, N, P, PEND, TPF, DIR, LD_LDS, ST_LDS, ES>(buf, t, active, tw, ld, st);
}

// Length-N transform (DIR = -1 forward, +1 inverse, unnormalised) from ld to st.
template <typename R, int N, int TPF, int DIR, bool LD_LDS, bool ST_LDS, int ES = 1, class LD, class ST>
__device__ __forceinline__ void fft_run(cpx<R>* buf, int t, bool active, const cpx<R>* __restrict__ tw,
                                        LD ld, ST st) {
  static_assert(plan_product(N) == N && plan_passes(N) >= 2, "no plan for this size");
  fft_pass_t<R, N, 0, plan_passes(N), TPF, DIR, LD_LDS, ST_LDS, ES>(buf, t, active, tw, ld, st);
}
template <typename R, int N, int TPF, int DIR, bool LD_LDS, bool ST_LDS, int ES = 1, class LD, class ST>
__device__ __forceinline__ void fft_run(cpx<R>* buf, int t, bool active, TwQ<R> tw, LD ld, ST st) {
  static_assert(plan_product(N) == N && plan_passes(N) >= 2, "no plan for this size");
  fft_pass_t<R, N, 0, plan_passes(N), TPF, DIR, LD_LDS, ST_LDS, ES>(buf, t, active, tw, ld, st);
}

// Two transforms back to back with an elementwise map between them, where the
// plan's first and last radix are equal: the last pass of the first transform
// and the first pass of the second act on the same elements in each thread,
// so they run in registers with `mid(e, v)` applied in between (no LDS round
// trip).  ld feeds the first pass of transform 1 (direction D1), st takes the
// last pass of transform 2 (direction D2).
__host__ __device__ constexpr bool plan_bridgeable(int n) {
  return plan_passes(n) >= 3 && plan_radix(n, 0) == plan_radix(n, plan_passes(n) - 1);
}

// The bridge between two transforms: the last pass of one in direction D1
// (reading LDS), `mid(e, v)` on each of its outputs, and the first pass of the
// next in direction D2 (writing LDS), in registers.  Needs plan_bridgeable(N):
// the last pass of transform 1 and the first pass of transform 2 then act on
// the same elements j + q N/RAD in each thread.
template <typename R, int N, int TPF, int D1, int D2, int ES, class TW, class MID>
__device__ __forceinline__ void fft_bridge_t(cpx<R>* buf, int t, bool active, TW tw, MID& mid) {
  static_assert(plan_bridgeable(N), "first and last radix differ");
  constexpr int PL = plan_passes(N) - 1;  // last pass index
  constexpr int RAD = plan_radix(N, PL);
  constexpr int NS = plan_ns(N, PL);      // = N / RAD
  constexpr int NB = N / RAD;
  constexpr int PER = (NB + TPF - 1) / TPF;
  constexpr bool EXACT = (NB % TPF) == 0;
  cpx<R> v[PER][RAD];
  cpx<R> w[PER][radp(RAD)];
  if (active) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPF;
      if (EXACT || j < NB) tw_fetch<R, N, PL>(w[p], j, tw);
    }
    if constexpr (has_pre<MID>::value) {
#pragma unroll
      for (int p = 0; p < PER; ++p) {
        const int j = t + p * TPF;
        if (EXACT || j < NB) {
#pragma unroll
          for (int q = 0; q < RAD; ++q) mid.pre(j + q * NS, p, q);
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPF;
      if (EXACT || j < NB) {
        const int pj = lds_pos(j);
#pragma unroll
        for (int q = 0; q < RAD; ++q) v[p][q] = lds_ld(buf + ES * lds_pos_step<NB, RAD>(j, pj, q));
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPF;
      if (EXACT || j < NB) {
        // last pass of transform 1: k = j (j < NS), outputs at j + q NS
        tw_apply<RAD, D1>(v[p], w[p]);
        bfly<RAD, D1>(v[p]);
        if constexpr (has_post<MID>::value) {
          constexpr int G = post_group<MID, RAD>::value;
          static_assert(RAD % G == 0, "post group");
#pragma unroll
          for (int q0 = 0; q0 < RAD; q0 += G) {
#pragma unroll
            for (int q = q0; q < q0 + G; ++q) v[p][q] = call_mid<MID, R>(mid, j + q * NS, v[p][q], p, q);
#pragma unroll
            for (int q = q0; q < q0 + G; ++q) mid.post(j + q * NS, p, q);
          }
        } else {
#pragma unroll
          for (int q = 0; q < RAD; ++q) v[p][q] = call_mid<MID, R>(mid, j + q * NS, v[p][q], p, q);
        }
        // first pass of transform 2 reads the same elements j + q N/RAD
        bfly<RAD, D2>(v[p]);
        const int o = j * RAD;
        const int po = lds_pos(o);
#pragma unroll
        for (int q = 0; q < RAD; ++q) buf[ES * lds_pos_step<1, RAD>(o, po, q)] = v[p][q];
      }
    }
  }
  __syncthreads();
}

template <typename R, int N, int TPF, int D1, int D2, int ES, class MID>
__device__ __forceinline__ void fft_bridge(cpx<R>* buf, int t, bool active, const cpx<R>* __restrict__ tw,
                                           MID& mid) {
  fft_bridge_t<R, N, TPF, D1, D2, ES>(buf, t, active, tw, mid);
}
template <typename R, int N, int TPF, int D1, int D2, int ES, class MID>
__device__ __forceinline__ void fft_bridge(cpx<R>* buf, int t, bool active, TwQ<R> tw, MID& mid) {
  fft_bridge_t<R, N, TPF, D1, D2, ES>(buf, t, active, tw, mid);
}

template <typename R, int N, int TPF, int D1, int D2, int ES, class TW, class LD, class MID, class ST>
__device__ __forceinline__ void fft_run2_t(cpx<R>* buf, int t, bool active, TW tw, LD ld, MID mid, ST st) {
  static_assert(plan_bridgeable(N), "first and last radix differ");
  constexpr int PL = plan_passes(N) - 1;  // last pass index
  auto none = [](int, cpx<R>) {};
  // transform 1, passes 0 .. PL-1 (the last of them writes LDS)
  fft_pass_t<R, N, 0, PL, TPF, D1, false, false, ES>(buf, t, active, tw, ld, none);
  fft_bridge_t<R, N, TPF, D1, D2, ES>(buf, t, active, tw, mid);
  // transform 2, passes 1 .. PL
  auto noload = [](int) { return cpx<R>{R(0), R(0)}; };
  fft_pass_t<R, N, 1, PL + 1, TPF, D2, false, false, ES>(buf, t, active, tw, noload, st);
}
template <typename R, int N, int TPF, int D1, int D2, int ES = 1, class LD, class MID, class ST>
__device__ __forceinline__ void fft_run2(cpx<R>* buf, int t, bool active, const cpx<R>* __restrict__ tw,
                                         LD ld, MID mid, ST st) {
  fft_run2_t<R, N, TPF, D1, D2, ES>(buf, t, active, tw, ld, mid, st);
}
template <typename R, int N, int TPF, int D1, int D2, int ES = 1, class LD, class MID, class ST>
__device__ __forceinline__ void fft_run2(cpx<R>* buf, int t, bool active, TwQ<R> tw, LD ld, MID mid, ST st) {
  fft_run2_t<R, N, TPF, D1, D2, ES>(buf, t, active, tw, ld, mid, st);
}

// Internal passes 1 .. PL-1 of a transform whose first and last passes are
// bridges (LDS in, LDS out).
template <typename R, int N, int TPF, int D, int ES, class TW>
__device__ __forceinline__ void fft_inner_t(cpx<R>* buf, int t, bool active, TW tw) {
  constexpr int PL = plan_passes(N) - 1;
  if constexpr (PL > 1) {
    auto noload = [](int) { return cpx<R>{R(0), R(0)}; };
    auto none = [](int, cpx<R>) {};
    fft_pass_t<R, N, 1, PL, TPF, D, false, false, ES>(buf, t, active, tw, noload, none);
  }
}
template <typename R, int N, int TPF, int D, int ES>
__device__ __forceinline__ void fft_inner(cpx<R>* buf, int t, bool active, const cpx<R>* __restrict__ tw) {
  fft_inner_t<R, N, TPF, D, ES>(buf, t, active, tw);
}
template <typename R, int N, int TPF, int D, int ES>
__device__ __forceinline__ void fft_inner(cpx<R>* buf, int t, bool active, TwQ<R> tw) {
  fft_inner_t<R, N, TPF, D, ES>(buf, t, active, tw);
}

}  // namespace cbs
