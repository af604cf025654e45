// Per-instance reductions, solver bookkeeping, setup statistics and the FP64
// Krylov kernels of FGMRES (Arnoldi with classical Gram-Schmidt applied twice,
// Givens rotations, back substitution).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"

namespace cbs {

// ---- per-instance reductions and solver bookkeeping -------------------------------
//
// One wavefront per instance: lane l sums partial slots l, l+64, ... and the
// wave is reduced by a fixed shuffle tree, so every sum is deterministic.
// Lane 0 then does the instance's bookkeeping.

__device__ __forceinline__ int wave_instance() {
  return int((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

// norm2[i] = sum of the instance's partials (fixed order => deterministic).
__global__ void k_instance_sums(const InstDesc* inst, int batch, const double* partials,
                                double* out) {
  const int i = wave_instance();
  if (i >= batch) return;
  const InstDesc d = inst[i];
  const double s = instance_sum(partials, d);
  if ((threadIdx.x & 63) == 0) out[i] = s;
}

// After the FP64 residual of the current iterate (start of a chunk).
__global__ void k_check64(IterState st, const InstDesc* inst, int batch,
                          const double* partials) {
  const int i = wave_instance();
  if (i >= batch) return;
  const int s0 = st.status[i];
  if (s0 == ST_CONVERGED || s0 == ST_MAXIT || s0 == ST_DIVERGED) {
    if ((threadIdx.x & 63) == 0) st.chunk_active[i] = 0;
    return;
  }
  const InstDesc d = inst[i];
  const double sum = instance_sum(partials, d);
  if ((threadIdx.x & 63) != 0) return;
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
// ids (nullable) lists the instances to check; count is its length (or the
// batch size when ids is NULL).
__global__ void k_check32(IterState st, const InstDesc* inst, const int* ids, int count,
                          const double* partials) {
  const int w = wave_instance();
  if (w >= count) return;
  check32_instance(st, inst, partials, ids ? ids[w] : w);
}

// bnorm[i] = sqrt(sum of partials)
__global__ void k_set_bnorm(IterState st, const InstDesc* inst, int batch,
                            const double* partials) {
  const int i = wave_instance();
  if (i >= batch) return;
  const InstDesc d = inst[i];
  const double sum = instance_sum(partials, d);
  if ((threadIdx.x & 63) == 0) st.bnorm[i] = sqrt(sum);
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
  const int rpw = d.rpw;
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

// ---- FGMRES: FP64 Arnoldi, Gram-Schmidt with delayed reorthogonalisation -------------
//
// Per-instance small dense state (doubles), restart length m:
//   H  (m+1) x m complex, row-major        at 0
//   cs m real, sn m complex                 (Givens rotations)
//   g  m+1 complex                          (rotated beta e1)
//   y  m complex                            (least-squares solution)
//   coef m+1 complex: t_q = <v_q, w>, and at q = j the coefficient of v_j
//   coefs m+1 complex: s_q = <v_q, u_j>
//   sc 8 scalars: [0] beta [1] bnorm [2] estimate [3] 1/r_jj [4] alpha
//                 [5..6] <u_j, w>
//
// Classical Gram-Schmidt applied twice, with the second pass of each vector
// carried out one step late so that a step reads the basis twice instead of
// four times (the DCGS2 scheme of Swirydowicz et al., "Low synchronization
// Gram-Schmidt and GMRES algorithms", 2020).  At the start of step j the
// basis slots 0..j-1 hold the final orthonormal v_q; slot j holds u_j, the
// next vector after one projection pass (slot 0 holds the final v_0).
//   z_j = P_K(u_j / ||u_j||),  w = B z_j                  (flexible: any z_j)
//   one pass over the basis: s = V^H u_j, t = V^H w, alpha = <u_j, u_j>,
//                            beta = <u_j, w>
//   r = sqrt(alpha - |s|^2), v_j = (u_j - V s) / r, <v_j, w> = (beta - s^H t) / r
//   H[:, j-1] += s, H[j, j-1] = r   (column j-1 is now final: rotate it)
//   H[:, j] = (t, <v_j, w>)         (first pass of column j)
//   one pass over the basis: v_j into slot j, u_{j+1} = w - V t - <v_j, w> v_j
//                            into slot j+1 with its partial |.|^2
// The stopping test of step j uses column j before its second pass (the
// correction is at rounding level); when an instance's cycle ends, a last
// pass reorthogonalises u_{jend} and finalises column jend-1.

// Partial dot products over one row item.  Step (FINAL false, step k.j of
// the active instances): <v_q, u_j> and <v_q, w> for q < j, <u_j, u_j> and
// <u_j, w>.  FINAL (cycle end, j = jend of each instance that ran steps):
// <v_q, u_j> for q < j and <u_j, u_j>.  Per partial slot, k.dstride doubles:
// t at 0, s at 2(m+1), the scalars at 4(m+1).
template <bool FINAL>
__global__ __launch_bounds__(kThreads) void k_gs_dots(KryParams k) {
  constexpr int QB = 4;
  __shared__ double red[4 * QB][kThreads / 64];
  const int2 it = k.items[blockIdx.x];
  int j;
  if constexpr (FINAL) {
    j = k.jend[it.x];
    if (j <= 0) return;
  } else {
    if (!k.active[it.x]) return;
    j = k.j;
  }
  const InstDesc d = k.inst[it.x];
  long long base;
  int cnt, slot;
  item_range(d, it.y, base, cnt, slot);
  constexpr int PER = 2048 / kThreads;  // row_rpw(N) * N <= 2048 for every N
  const cpx<double>* ub = k.vbasis + (long long)j * k.cells + base;
  const cpx<double>* wb = k.vbasis + (long long)(j + 1) * k.cells + base;
  cpx<double> uv[PER], wv[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int x = threadIdx.x + e * kThreads;
    uv[e] = x < cnt ? ub[x] : cpx<double>{0.0, 0.0};
    wv[e] = (!FINAL && x < cnt) ? wb[x] : cpx<double>{0.0, 0.0};
  }
  double* out = k.dots + (long long)slot * k.dstride;
  const int so = 2 * (k.m + 1), co = 4 * (k.m + 1);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  {
    double a = 0.0, br = 0.0, bi = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      a += cabs2(uv[e]);
      br += uv[e].x * wv[e].x + uv[e].y * wv[e].y;
      bi += uv[e].x * wv[e].y - uv[e].y * wv[e].x;
    }
    a = wave_sum(a);
    br = wave_sum(br);
    bi = wave_sum(bi);
    if (lane == 0) {
      red[0][wid] = a;
      red[1][wid] = br;
      red[2][wid] = bi;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) t += red[threadIdx.x][w];
      out[co + threadIdx.x] = t;
    }
    __syncthreads();
  }
  for (int q0 = 0; q0 < j; q0 += QB) {
    double acc[QB][4];
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) {
      acc[qq][0] = acc[qq][1] = acc[qq][2] = acc[qq][3] = 0.0;
      const int q = q0 + qq;
      if (q < j) {
        const cpx<double>* v = k.vbasis + (long long)q * k.cells + base;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int x = threadIdx.x + e * kThreads;
          if (x < cnt) {
            const cpx<double> a = v[x];
            acc[qq][0] += a.x * uv[e].x + a.y * uv[e].y;
            acc[qq][1] += a.x * uv[e].y - a.y * uv[e].x;
            if (!FINAL) {
              acc[qq][2] += a.x * wv[e].x + a.y * wv[e].y;
              acc[qq][3] += a.x * wv[e].y - a.y * wv[e].x;
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[qq][c] = wave_sum(acc[qq][c]);
    }
    if (lane == 0) {
#pragma unroll
      for (int qq = 0; qq < QB; ++qq)
#pragma unroll
        for (int c = 0; c < 4; ++c) red[4 * qq + c][wid] = acc[qq][c];
    }
    __syncthreads();
    if (threadIdx.x < 4 * QB) {
      const int qq = threadIdx.x >> 2, c = threadIdx.x & 3;
      const int q = q0 + qq;
      if (q < j && (!FINAL || c < 2)) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) t += red[threadIdx.x][w];
        // c 0, 1: s_q (with u); c 2, 3: t_q (with w)
        out[(c < 2 ? so : 0) + 2 * q + (c & 1)] = t;
      }
    }
    __syncthreads();
  }
}

// out[e] = sum over the instance's partial slots of dots[slot][first + e],
// e < count (every thread of the workgroup calls it; 16 values per round).
__device__ void sum_slots(const KryParams& k, const InstDesc& d, int first, int count, double* out) {
  constexpr int VB = 16;
  __shared__ double red[VB][kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int e0 = 0; e0 < count; e0 += VB) {
    double acc[VB];
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[v] = 0.0;
    for (int t = threadIdx.x; t < d.nparts; t += kThreads) {
      const double* row = k.dots + (long long)(d.part_off + t) * k.dstride + first + e0;
#pragma unroll
      for (int v = 0; v < VB; ++v)
        if (e0 + v < count) acc[v] += row[v];
    }
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[v] = wave_sum(acc[v]);
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < VB; ++v) red[v][wid] = acc[v];
    }
    __syncthreads();
    if (threadIdx.x < VB && e0 + threadIdx.x < count) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) t += red[threadIdx.x][w];
      out[e0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// Column c of H is final: apply rotations 0..c-1, form rotation c zeroing
// H[c+1][c], rotate g, and store |g_{c+1}| / ||G s|| as the estimate.  Every
// thread of the workgroup calls it: the column and the rotations are staged
// in LDS, so the sequential chain of rotations (one thread) runs at LDS
// latency instead of a dependent global access per rotation.
__device__ void givens_column(double* s, const KryLayout& L, int c) {
  __shared__ cpx<double> col[kMaxRestart + 1];
  __shared__ cpx<double> sns[kMaxRestart];
  __shared__ double css[kMaxRestart];
  for (int q = threadIdx.x; q <= c + 1; q += blockDim.x) col[q] = cpx<double>{s[L.h(q, c)], s[L.h(q, c) + 1]};
  for (int q = threadIdx.x; q < c; q += blockDim.x) {
    css[q] = s[L.cs() + q];
    sns[q] = cpx<double>{s[L.sn() + 2 * q], s[L.sn() + 2 * q + 1]};
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < c; ++q) {
      const cpx<double> a = col[q], b = col[q + 1];
      col[q] = cscale(a, css[q]) + cmul(sns[q], b);
      col[q + 1] = cscale(b, css[q]) - cmul(cconj(sns[q]), a);
    }
    const cpx<double> a = col[c], b = col[c + 1];
    const double aa = sqrt(cabs2(a));
    const double nu = sqrt(cabs2(a) + cabs2(b));
    double cs;
    cpx<double> sn;
    if (aa == 0.0) {
      cs = 0.0;
      sn = cpx<double>{1.0, 0.0};
    } else {
      cs = aa / nu;
      sn = cscale(cmul(a, cconj(b)), 1.0 / (aa * nu));
    }
    s[L.cs() + c] = cs;
    s[L.sn() + 2 * c] = sn.x;
    s[L.sn() + 2 * c + 1] = sn.y;
    col[c] = cscale(a, cs) + cmul(sn, b);
    col[c + 1] = cpx<double>{0.0, 0.0};
    const cpx<double> gc{s[L.g() + 2 * c], s[L.g() + 2 * c + 1]};
    const cpx<double> g1 = cscale(cmul(cconj(sn), gc), -1.0);
    const cpx<double> g0 = cscale(gc, cs);
    s[L.g() + 2 * c] = g0.x;
    s[L.g() + 2 * c + 1] = g0.y;
    s[L.g() + 2 * (c + 1)] = g1.x;
    s[L.g() + 2 * (c + 1) + 1] = g1.y;
    s[L.sc() + 2] = sqrt(cabs2(g1)) / (s[L.sc() + 1] > 0.0 ? s[L.sc() + 1] : 1.0);
  }
  __syncthreads();
  for (int q = threadIdx.x; q <= c + 1; q += blockDim.x) {
    s[L.h(q, c)] = col[q].x;
    s[L.h(q, c) + 1] = col[q].y;
  }
}

// One workgroup per instance: reduce the partial dot products, then (one
// thread) the norm r of the reorthogonalised u_j, the final column j-1 and
// its rotation, and (step) the first pass of column j with the update
// coefficients.
template <bool FINAL>
__global__ __launch_bounds__(kThreads) void k_gs_finish(KryParams k, int batch) {
  const int i = blockIdx.x;
  if (i >= batch) return;
  int j;
  if constexpr (FINAL) {
    j = k.jend[i];
    if (j <= 0) return;
  } else {
    if (!k.active[i]) return;
    j = k.j;
  }
  const InstDesc d = k.inst[i];
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  const int so = 2 * (k.m + 1), co = 4 * (k.m + 1);
  if (!FINAL) sum_slots(k, d, 0, 2 * j, s + L.coef());
  sum_slots(k, d, so, 2 * j, s + L.coefs());
  sum_slots(k, d, co, FINAL ? 1 : 3, s + L.sc() + 4);
  // |s|^2 and s^H t (workgroup sums; every thread gets them)
  __shared__ double red[3][kThreads / 64];
  __shared__ double tot[3];
  double ss = 0.0, hr = 0.0, hi = 0.0;
  for (int q = threadIdx.x; q < j; q += kThreads) {
    const cpx<double> sq{s[L.coefs() + 2 * q], s[L.coefs() + 2 * q + 1]};
    ss += cabs2(sq);
    if (!FINAL) {
      const cpx<double> p = cmulc(sq, cpx<double>{s[L.coef() + 2 * q], s[L.coef() + 2 * q + 1]});
      hr += p.x;
      hi += p.y;
    }
  }
  ss = wave_sum(ss);
  hr = wave_sum(hr);
  hi = wave_sum(hi);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = ss;
    red[1][wid] = hr;
    red[2][wid] = hi;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += red[threadIdx.x][w];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
  const double alpha = s[L.sc() + 4];
  const double r = j > 0 ? sqrt(fmax(alpha - tot[0], 0.0)) : 1.0;
  if (j > 0) {
    // column j-1 is final: add the second pass of u_j, then rotate it
    for (int q = threadIdx.x; q < j; q += kThreads) {
      s[L.h(q, j - 1)] += s[L.coefs() + 2 * q];
      s[L.h(q, j - 1) + 1] += s[L.coefs() + 2 * q + 1];
    }
    if (threadIdx.x == 0) {
      s[L.h(j, j - 1)] = r;
      s[L.h(j, j - 1) + 1] = 0.0;
    }
    __syncthreads();
    givens_column(s, L, j - 1);
  }
  if (FINAL) return;
  // <v_j, w> = (<u_j, w> - s^H t) / r; first pass of column j
  const double ir = r > 0.0 ? 1.0 / r : 0.0;
  const cpx<double> hj = cscale(cpx<double>{s[L.sc() + 5] - tot[1], s[L.sc() + 6] - tot[2]}, ir);
  for (int q = threadIdx.x; q < j; q += kThreads) {
    s[L.h(q, j)] = s[L.coef() + 2 * q];
    s[L.h(q, j) + 1] = s[L.coef() + 2 * q + 1];
  }
  if (threadIdx.x == 0) {
    s[L.coef() + 2 * j] = hj.x;
    s[L.coef() + 2 * j + 1] = hj.y;
    s[L.sc() + 3] = ir;
    s[L.h(j, j)] = hj.x;
    s[L.h(j, j) + 1] = hj.y;
  }
}

// v_j = (u_j - V s) / r into slot j (j > 0), u_{j+1} = w - V t - <v_j, w> v_j
// into slot j+1, and its partial |.|^2.  One read of the basis.
__global__ __launch_bounds__(kThreads) void k_gs_update(KryParams k) {
  __shared__ double red[kThreads / 64];
  const int2 it = k.items[blockIdx.x];
  if (!k.active[it.x]) return;
  const InstDesc d = k.inst[it.x];
  long long base;
  int cnt, slot;
  item_range(d, it.y, base, cnt, slot);
  const KryLayout L{k.m};
  const double* st = k.kry + it.x * k.kstride;
  const double* ct = st + L.coef();
  const double* cs = st + L.coefs();
  const int j = k.j;
  constexpr int PER = 2048 / kThreads;
  cpx<double>* ub = const_cast<cpx<double>*>(k.vbasis) + (long long)j * k.cells + base;
  cpx<double>* wb = const_cast<cpx<double>*>(k.vbasis) + (long long)(j + 1) * k.cells + base;
  cpx<double> uv[PER], wv[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int x = threadIdx.x + e * kThreads;
    uv[e] = x < cnt ? ub[x] : cpx<double>{0.0, 0.0};
    wv[e] = x < cnt ? wb[x] : cpx<double>{0.0, 0.0};
  }
  for (int q = 0; q < j; ++q) {
    const cpx<double> sq{cs[2 * q], cs[2 * q + 1]};
    const cpx<double> tq{ct[2 * q], ct[2 * q + 1]};
    const cpx<double>* v = k.vbasis + (long long)q * k.cells + base;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int x = threadIdx.x + e * kThreads;
      if (x < cnt) {
        const cpx<double> a = v[x];
        uv[e] = uv[e] - cmul(sq, a);
        wv[e] = wv[e] - cmul(tq, a);
      }
    }
  }
  const double ir = st[L.sc() + 3];
  const cpx<double> hj{ct[2 * j], ct[2 * j + 1]};
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int x = threadIdx.x + e * kThreads;
    if (x < cnt) {
      const cpx<double> vj = cscale(uv[e], ir);
      if (j > 0) ub[x] = vj;
      const cpx<double> nw = wv[e] - cmul(hj, vj);
      wb[x] = nw;
      acc += cabs2(nw);
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) k.partials[slot] = t;
}

// Stopping test of step j (one workgroup per instance): ||u_{j+1}|| (the
// scale of the next preconditioner input), the rotations applied to column j
// as it stands after its first pass (staged in LDS), and the residual
// estimate |g_j| |sin| / ||G s||.
__global__ __launch_bounds__(kThreads) void k_gs_check(KryParams k, int batch) {
  __shared__ cpx<double> col[kMaxRestart + 1];
  __shared__ cpx<double> sns[kMaxRestart];
  __shared__ double css[kMaxRestart];
  __shared__ double hsum;
  const int i = blockIdx.x;
  if (i >= batch || !k.active[i]) return;
  const InstDesc d = k.inst[i];
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  const int j = k.j;
  if (threadIdx.x < 64) {
    const double sum = instance_sum(k.partials, d);
    if (threadIdx.x == 0) hsum = sum;
  }
  for (int q = threadIdx.x; q <= j; q += kThreads) col[q] = cpx<double>{s[L.h(q, j)], s[L.h(q, j) + 1]};
  for (int q = threadIdx.x; q < j; q += kThreads) {
    css[q] = s[L.cs() + q];
    sns[q] = cpx<double>{s[L.sn() + 2 * q], s[L.sn() + 2 * q + 1]};
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double hn = sqrt(hsum);
  k.scale[i] = hn > 0.0 ? 1.0 / hn : 0.0;
  cpx<double> cur = col[0];
  for (int q = 0; q < j; ++q) cur = cscale(col[q + 1], css[q]) - cmul(cconj(sns[q]), cur);
  const double aa2 = cabs2(cur);
  const double nu = sqrt(aa2 + hn * hn);
  const double sabs = aa2 == 0.0 ? 1.0 : (nu > 0.0 ? hn / nu : 0.0);
  const cpx<double> gj{s[L.g() + 2 * j], s[L.g() + 2 * j + 1]};
  const double est = sqrt(cabs2(gj)) * sabs / (s[L.sc() + 1] > 0.0 ? s[L.sc() + 1] : 1.0);
  s[L.sc() + 2] = est;
  k.jend[i] = j + 1;
  k.iters[i] += 1;
  if (!(est > k.rtol[0]) || hn == 0.0 || k.iters[i] >= k.max_iters[0] || j + 1 >= k.m)
    k.active[i] = 0;
}

// Back substitution H[0:jend, 0:jend] y = g[0:jend] (H upper triangular after rotations).
__global__ void k_backsolve(KryParams k, int batch) {
  const int i = wave_instance();
  if (i >= batch || (threadIdx.x & 63) != 0) return;
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

// After the FP64 true residual r = G(V x + s) - x was written to v_0 with its
// partial norms: decide convergence and start a new cycle.
__global__ void k_fg_restart(KryParams k, int batch, int first) {
  const int i = wave_instance();
  if (i >= batch) return;
  const KryLayout L{k.m};
  double* s = k.kry + i * k.kstride;
  const InstDesc d = k.inst[i];
  const int lane = threadIdx.x & 63;
  if (first) {  // partials hold |G s|^2: store ||G s||
    const double sum0 = instance_sum(k.partials, d);
    if (lane == 0) s[L.sc() + 1] = sqrt(sum0);
    return;
  }
  const int st = k.status[i];
  if (st != ST_RUNNING) {
    if (lane == 0) {
      k.jend[i] = 0;
      k.active[i] = 0;
    }
    return;
  }
  const double sum = instance_sum(k.partials, d);
  if (lane != 0) return;
  k.jend[i] = 0;
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

// ---- stream-ordered solver bookkeeping and field norms --------------------------------

// Initial per-instance solver state (replaces host copies, so a solve can be
// enqueued without synchronising and captured into a graph).
__global__ void k_solver_init(int* status, int* iters, double* relres, int* kjend, double* rtol_d,
                              double* rtol32_d, int* max_d, int batch, double rtol, double rtol32,
                              int max_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *rtol_d = rtol;
    if (rtol32_d) *rtol32_d = rtol32;
    *max_d = max_count;
  }
  if (i < batch) {
    status[i] = ST_RUNNING;
    iters[i] = 0;
    relres[i] = 0.0;
    if (kjend) kjend[i] = 0;
  }
}

// Copy the per-instance results to the caller's device arrays; an instance
// still running (or pending confirmation) when the budget ran out reports
// ST_MAXIT.
__global__ void k_solver_out(const int* status, const int* iters, const double* relres, int batch,
                             int* o_iters, double* o_relres, int* o_status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const int s = status[i];
  if (o_iters) o_iters[i] = iters[i];
  if (o_relres) o_relres[i] = relres[i];
  if (o_status) o_status[i] = (s == ST_RUNNING || s == ST_PENDING) ? int(ST_MAXIT) : s;
}

// Partial sums of |x|^2 over one row work item (slot as for the row kernels).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_norm2_rows(const InstDesc* inst, const int2* items,
                                                         const cpx<R>* x, double* partials) {
  __shared__ double red[kThreads / 64];
  const int2 it = items[blockIdx.x];
  const InstDesc d = inst[it.x];
  long long base;
  int cnt, slot;
  item_range(d, it.y, base, cnt, slot);
  double acc = 0.0;
  for (int j = threadIdx.x; j < cnt; j += kThreads) acc += double(cabs2(x[base + j]));
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[slot] = t;
}

// out[i] = sqrt(num[i] / den[i]) (sqrt(num[i]) where den[i] is 0).
__global__ void k_ratio(const double* num, const double* den, double* out, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  out[i] = den[i] > 0.0 ? sqrt(num[i] / den[i]) : sqrt(num[i]);
}

__global__ void k_widen_all(const cpx<float>* in, cpx<double>* out, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const cpx<float> v = in[i];
    out[i] = cpx<double>{double(v.x), double(v.y)};
  }
}


// ---- launchers -----------------------------------------------------------------

// one wavefront per instance, four per 256-thread block
static int inst_blocks(int batch) { return (batch + 3) / 4; }

void launch_instance_sums(int batch, hipStream_t st, const InstDesc* inst, const double* partials,
                          double* out) {
  hipLaunchKernelGGL(k_instance_sums, dim3(inst_blocks(batch)), dim3(256), 0, st, inst, batch,
                     partials, out);
}
void launch_check64(int batch, hipStream_t st, const IterState& is, const InstDesc* inst,
                    const double* partials) {
  hipLaunchKernelGGL(k_check64, dim3(inst_blocks(batch)), dim3(256), 0, st, is, inst, batch, partials);
}
void launch_check32(int count, const int* ids, hipStream_t st, const IterState& is,
                    const InstDesc* inst, const double* partials) {
  hipLaunchKernelGGL(k_check32, dim3(inst_blocks(count)), dim3(256), 0, st, is, inst, ids, count,
                     partials);
}
void launch_set_bnorm(int batch, hipStream_t st, const IterState& is, const InstDesc* inst,
                      const double* partials) {
  hipLaunchKernelGGL(k_set_bnorm, dim3(inst_blocks(batch)), dim3(256), 0, st, is, inst, batch, partials);
}
void launch_stats(int grid, hipStream_t st, const InstDesc* inst, const int2* items,
                  const cpx<double>* k2, double* partials, int phase) {
  hipLaunchKernelGGL(k_stats, dim3(grid), dim3(kThreads), 0, st, inst, items, k2, partials, phase);
}
void launch_widen_all(hipStream_t st, const cpx<float>* in, cpx<double>* out, long long count) {
  hipLaunchKernelGGL(k_widen_all, dim3(1024), dim3(256), 0, st, in, out, count);
}
void launch_solver_init(hipStream_t st, int* status, int* iters, double* relres, int* kjend,
                        double* rtol_d, double* rtol32_d, int* max_d, int batch, double rtol,
                        double rtol32, int max_count) {
  hipLaunchKernelGGL(k_solver_init, dim3((batch + 255) / 256), dim3(256), 0, st, status, iters, relres, kjend,
                     rtol_d, rtol32_d, max_d, batch, rtol, rtol32, max_count);
}
void launch_solver_out(hipStream_t st, const IterState& is, int batch, int* o_iters, double* o_relres,
                       int* o_status) {
  hipLaunchKernelGGL(k_solver_out, dim3((batch + 255) / 256), dim3(256), 0, st, is.status, is.iters,
                     is.relres, batch, o_iters, o_relres, o_status);
}
void launch_norm2_rows(int grid, hipStream_t st, const InstDesc* inst, const int2* items,
                       const cpx<float>* x, double* partials) {
  hipLaunchKernelGGL(k_norm2_rows<float>, dim3(grid), dim3(kThreads), 0, st, inst, items, x, partials);
}
void launch_norm2_rows(int grid, hipStream_t st, const InstDesc* inst, const int2* items,
                       const cpx<double>* x, double* partials) {
  hipLaunchKernelGGL(k_norm2_rows<double>, dim3(grid), dim3(kThreads), 0, st, inst, items, x, partials);
}
void launch_ratio(int batch, hipStream_t st, const double* num, const double* den, double* out) {
  hipLaunchKernelGGL(k_ratio, dim3((batch + 255) / 256), dim3(256), 0, st, num, den, out, batch);
}
void launch_gs_dots(int grid, bool final_pass, hipStream_t st, const KryParams& k) {
  if (final_pass)
    hipLaunchKernelGGL(k_gs_dots<true>, dim3(grid), dim3(kThreads), 0, st, k);
  else
    hipLaunchKernelGGL(k_gs_dots<false>, dim3(grid), dim3(kThreads), 0, st, k);
}
void launch_gs_finish(int batch, bool final_pass, hipStream_t st, const KryParams& k) {
  if (final_pass)
    hipLaunchKernelGGL(k_gs_finish<true>, dim3(batch), dim3(kThreads), 0, st, k, batch);
  else
    hipLaunchKernelGGL(k_gs_finish<false>, dim3(batch), dim3(kThreads), 0, st, k, batch);
}
void launch_gs_update(int grid, hipStream_t st, const KryParams& k) {
  hipLaunchKernelGGL(k_gs_update, dim3(grid), dim3(kThreads), 0, st, k);
}
void launch_gs_check(int batch, hipStream_t st, const KryParams& k) {
  hipLaunchKernelGGL(k_gs_check, dim3(batch), dim3(kThreads), 0, st, k, batch);
}
void launch_backsolve(int batch, hipStream_t st, const KryParams& k) {
  hipLaunchKernelGGL(k_backsolve, dim3(inst_blocks(batch)), dim3(256), 0, st, k, batch);
}
void launch_fg_restart(int batch, hipStream_t st, const KryParams& k, int first) {
  hipLaunchKernelGGL(k_fg_restart, dim3(inst_blocks(batch)), dim3(256), 0, st, k, batch, first);
}

}  // namespace cbs
