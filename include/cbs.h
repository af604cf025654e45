/*
 * cbs.h -- C ABI of the MI355X (gfx950) Convergent-Born-Series library.
 *
 * The library applies, on one GPU, the Born-series operator of the heterogeneous
 * Helmholtz problem A u = s with A = -Laplacian - k(x)^2 on periodic N x N grids
 * (Sec. 3.1, Eq. helm and the discrete split A = L_eta - V_eta; App. D, Fourier
 * pseudospectral discretisation):
 *
 *   reference   L_eta = -Laplacian - (k0^2 + i eps),  eps > 0           (Sec. 3.1)
 *   symbol      lambda_n = |xi_n|^2 - k0^2 - i eps, xi = 2 pi n / N,
 *               n in {-N/2, ..., N/2-1}                                  (App. D)
 *   Green op.   G q = F^-1 (F q / lambda)                               (App. C, App. D)
 *   potential   V = k^2 - k0^2 - i eps  (pointwise)                      (Sec. 3.1)
 *   CBS step    u <- u + gamma (G (V u + s) - u),  gamma = i V / eps     (Sec. 3.1, Eq. CBS)
 *   Born resid. r = G (V u + s) - u = G (s - A u)                        (Sec. 4.1, Eq. npbs_iter)
 *
 * The paper's damping eta is called eps here.  Grid spacing is one cell.
 *
 * Layout and ownership
 * --------------------
 *  * A plan holds a batch of `batch` independent instances with sizes n[i]
 *    (square n x n, n in {16, 32, 64, 128, 192, 256, 288, 384, 512, 1024}).
 *  * Every field argument is a DEVICE pointer owned by the caller.  Fields are
 *    interleaved complex (re, im) numbers, complex64 for CBS_C64 plans and
 *    complex128 for CBS_C128 plans, row-major [y][x] per instance, and the
 *    instances are packed back to back in instance order: instance i starts at
 *    element sum_{j<i} n[j]^2.  Packed totals are returned by cbs_plan_cells.
 *  * The plan keeps a copy of k^2 and all scratch memory in device memory
 *    that cbs_setup allocates (freed by cbs_destroy), or that the caller
 *    provides to cbs_setup_ws (cbs_workspace_size bytes).  No other call
 *    allocates device memory.
 *  * `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Operator calls (cbs_apply, cbs_residual, cbs_sweep, cbs_relres, the
 *    adjoint and loss calls ...) and the solvers cbs_iterate_async and
 *    fgmres_solve_async are stream-ordered: they only enqueue work, return
 *    without synchronising, allocate nothing and can be captured into a
 *    HIP graph; their outputs are device arrays.  cbs_iterate and
 *    fgmres_solve run a host-driven loop instead (it reads each chunk's
 *    status to stop early and to shrink the work lists to the running
 *    instances) and synchronise the stream before returning host outputs.
 *    Setup-class calls (cbs_setup*, cbs_autotune, cbs_set_tile,
 *    cbs_destroy) synchronise.
 *  * Inputs are never modified, except the in/out solution u of the solvers.
 *
 * Errors
 * ------
 *  Every call returns a cbs_status.  Negative values are errors: nothing was
 *  launched for argument errors (detected before any launch); CBS_ERR_HIP
 *  reports a failing HIP call, including an asynchronous fault surfacing at a
 *  synchronisation point.  cbs_last_error() returns a thread-local message for
 *  the last non-OK status.  No call aborts or throws.
 */
#ifndef CBS_H_
#define CBS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cbs_plan_s* cbs_plan;

typedef enum {
  CBS_OK = 0,
  CBS_NOT_CONVERGED = 1,   /* solver finished; at least one instance did not reach rtol */
  CBS_ERR_ARG = -1,        /* null/invalid argument, bad batch or flag            */
  CBS_ERR_SIZE = -2,       /* unsupported grid size n                             */
  CBS_ERR_ILLCOND = -3,    /* eps < max|k^2-k0^2| or min|V|/eps below 1e-3        */
  CBS_ERR_WORKSPACE = -4,  /* plan was set up without room for this request       */
  CBS_ERR_HIP = -5         /* a HIP runtime call failed                           */
} cbs_status;

enum { CBS_C64 = 0, CBS_C128 = 1 };

/* Stopping rules of cbs_iterate. */
enum {
  CBS_STOP_BORN = 0,     /* ||G(V u + s) - u|| / ||G s|| (preconditioned residual) */
  CBS_STOP_PHYSICAL = 1  /* rTol = ||s - A u|| / ||s||, the paper's unified rule (Sec. 5) */
};

/* Per-instance solver status codes written by cbs_iterate / fgmres_solve. */
enum {
  CBS_INST_RUNNING = 0,
  CBS_INST_CONVERGED = 1,
  CBS_INST_MAX_ITERS = 2,
  CBS_INST_DIVERGED = 3
};

/* Setup flags. */
enum {
  CBS_FLAG_NO_GUARD = 1u,   /* skip the eps / min|V| conditioning guard */
  CBS_FLAG_ONE_STREAM = 2u, /* enqueue every kernel on the caller's stream (no lanes) */
  CBS_FLAG_DIRICHLET = 4u,  /* Dirichlet instances: DST-I reference (see cbs_setup) */
  CBS_FLAG_UNDAMPED = 8u    /* with CBS_FLAG_DIRICHLET: eps = 0, the reference L_D - k0^2 itself */
};

/*
 * cbs_setup -- build a plan for a batch of instances (step: setup; Sec. 3.1
 * defines V and gamma from k^2, k0 and eps; App. D the grid and symbol).
 *   plan       out: new plan handle (NULL on error)
 *   batch      number of instances, >= 1
 *   n          host[batch]: grid size of each instance
 *   k2         device: packed complex k^2 fields (dtype of the plan); copied
 *   k0sq       host[batch] or NULL: reference k0^2; a value that is NaN or
 *              NULL selects 0.5 (min Re k^2 + max Re k^2) over the instance
 *   eps        host[batch] or NULL: damping; a value <= 0 or NULL selects
 *              eps = max over cells |k^2 - k0^2|
 *   dtype      CBS_C64 (FP32 operator, FP64 norms/Krylov) or CBS_C128
 *   max_restart  largest FGMRES restart length later used (0: no FGMRES)
 *   flags      CBS_FLAG_* bits
 *   stream     hipStream_t as void*
 * Guard: unless CBS_FLAG_NO_GUARD, rejects eps < max|k^2 - k0^2| (1e-12
 * relative slack) and min|V|/eps < 1e-3 with CBS_ERR_ILLCOND (a cell with
 * V = 0 has gamma = 0 and never updates).  Synchronises `stream`.
 * Dirichlet plans (CBS_FLAG_DIRICHLET; App. C "Newton linear systems"): every
 * instance is the n x n interior of the unit square, h = 1/(n+1), with
 * homogeneous Dirichlet boundaries and the five-point negative Laplacian L_D;
 * the operator is A u = L_D u - k^2 u, the reference L_eta = L_D - (k0^2 +
 * i eps), and G = S^-1 diag(1/lambda) S with S the 2D DST-I and lambda_pq =
 * 4/h^2 (sin^2(p pi h/2) + sin^2(q pi h/2)) - k0^2 - i eps.  Every call then
 * uses that G and L_D in place of the periodic ones.  n must satisfy
 * 2(n+1) in {16, ..., 1024} above: n in {7, 15, 31, 63, 95, 127, 143, 191,
 * 255, 511}, the DST-I riding on the FFT of the odd extension; or n = 64,
 * the grid of the paper's Newton experiments (App. F), whose DST-I is formed
 * directly (2(n+1) = 130 has no FFT plan).  A Newton step J du = r with J = L_D - 2 diag(u) (App. B.2,
 * Eq. newton_linear_system) is the case k^2 = 2u.  Without further flags the
 * plan's reference is the damped L_D - (k0^2 + i eps), eps > 0.
 * Undamped Dirichlet plans (CBS_FLAG_DIRICHLET | CBS_FLAG_UNDAMPED): eps = 0
 * for every instance, so G = (L_D - k0^2)^-1 and V = k^2 - k0^2; with k0^2 =
 * 2 mean(u) - alpha that G is the paper's J_{0,m}^-1 (App. B.2, Eq.
 * newton_ref) and I - G V = G J (Eq. newton_born_identity).  eps must be
 * NULL.  Setup rejects (CBS_ERR_ILLCOND) a reference with an eigenvalue
 * mu_p + mu_q - k0^2 equal to zero, or, unless CBS_FLAG_NO_GUARD, within 1e-9
 * of max(2 mu_n, |k0^2|).  Without damping there is no gamma = i V / eps:
 * cbs_sweep, cbs_iterate(_async), FGMRES with inner sweeps, cbs_adjoint_step
 * and the W = gamma seed return CBS_ERR_ARG; the apply, residuals, relres,
 * NPBS steps, the metric-matched gradient, the Born adjoint and FGMRES with
 * inner_sweeps = 0 (GMRES on I - G V) are available.
 * Lanes: a batch of at least two instances and 2^21 cells is split into two
 * lanes of about equal cell count.  Sweep chains (cbs_sweep, the sweeps of
 * cbs_iterate and of the FGMRES preconditioner) run each lane on a
 * plan-owned non-blocking stream, forked from and joined back into the
 * caller's stream with events, so one lane's memory-bound row transforms
 * overlap the other lane's compute-bound column transforms.  Results are
 * bitwise the same as with CBS_FLAG_ONE_STREAM; calls stay ordered on the
 * caller's stream.
 */
cbs_status cbs_setup(cbs_plan* plan, int batch, const int32_t* n, const void* k2,
                     const double* k0sq, const double* eps, int dtype, int max_restart,
                     uint32_t flags, void* stream);

/*
 * cbs_workspace_size -- device bytes a plan of these sizes needs when the
 * caller provides its memory (cbs_setup_ws).  Host-only; touches no device.
 *   batch, n, dtype, max_restart, flags as in cbs_setup; bytes out.
 * The plan's buffers: FP64 copies of k^2, the spectral buffer, the FP64
 * iterate and source, three operator-precision fields, per-row partial sums,
 * per-instance solver state, twiddle tables, work lists, and for
 * max_restart m > 0 the FGMRES bases (m + 1 FP64 fields and m
 * operator-precision fields) with the Hessenberg/Givens storage.
 */
cbs_status cbs_workspace_size(int batch, const int32_t* n, int dtype, int max_restart,
                              uint32_t flags, size_t* bytes);

/*
 * cbs_setup_ws -- cbs_setup with caller-owned device memory: every device
 * buffer of the plan is carved from `workspace` (device pointer, 256-byte
 * aligned, at least cbs_workspace_size bytes; owned by the caller and kept
 * alive, unused by anything else, until cbs_destroy).  The plan then
 * allocates no device memory of its own.  CBS_ERR_WORKSPACE if the
 * workspace is too small or misaligned, CBS_ERR_ARG if it is NULL.
 */
cbs_status cbs_setup_ws(cbs_plan* plan, int batch, const int32_t* n, const void* k2,
                        const double* k0sq, const double* eps, int dtype, int max_restart,
                        uint32_t flags, void* workspace, size_t workspace_bytes, void* stream);

/*
 * cbs_setup_cdr -- plan for the periodic convection-diffusion-reaction
 *   problem -div(kappa grad u) + v . grad u + sigma u = s (App. B.1,
 *   Eqs. cdr_pde to cdr_G_symbol; App. C "CDR case" restates the symbol) with the
 *   constant background L0 = -kappa0 Lap + v0 . grad + sigma0, G = L0^-1
 *   (Fourier symbol 1/(kappa0 |xi|^2 + i v0 . xi + sigma0)) and
 *   V = L0 - L = div(dkappa grad) - dv . grad - dsigma.  Derivatives are
 *   spectral: d/dx = F^-1 diag(i xi_x) F, xi = 2 pi m / N on the signed mode
 *   index m (Nyquist bin -N/2), x the fast (column) axis, h = 1.
 *   kappa_sigma  device, packed complex fields in the plan's precision:
 *                real part kappa, imaginary part sigma (copied)
 *   velocity     device, packed complex fields: real part vx, imaginary vy
 *   background   host double[4 * batch]: kappa0, vx0, vy0, sigma0 per
 *                instance (finite; the symbol must not vanish on any bin,
 *                else CBS_ERR_ILLCOND)
 *   n            host int32[batch], grid sizes as for cbs_setup (periodic)
 *   The coefficients are meant real; their imaginary parts are not used.
 *   The plan allocates its memory (cbs_setup_cdr_ws: the caller provides
 *   it) and synchronises `stream`.
 *   On such a plan cbs_apply, cbs_residual, cbs_helmholtz_residual (which
 *   then returns s - A u with A the CDR operator above), cbs_born_adjoint,
 *   cbs_plan_info (k0sq = kappa0, eps = sigma0), cbs_autotune, cbs_set_tile
 *   and cbs_destroy apply; the CBS-step entry points (cbs_sweep,
 *   cbs_iterate, fgmres_solve, cbs_npbs_step, cbs_adjoint_step,
 *   cbs_loss_seed) return CBS_ERR_ARG.  Each apply or residual runs one
 *   column pass (d/dy of dkappa d/dy, in LDS), one row pass (d/dx of dkappa
 *   d/dx, fused with the forward row transform of G) and G's column and
 *   inverse row passes.
 */
cbs_status cbs_setup_cdr(cbs_plan* plan, int batch, const int32_t* n, const void* kappa_sigma,
                         const void* velocity, const double* background, int dtype, void* stream);

/* cbs_setup_cdr with caller-owned device memory (the plan then allocates
 * nothing): workspace as for cbs_setup_ws, of at least
 * cbs_workspace_size_cdr bytes (host-only query; touches no device). */
cbs_status cbs_setup_cdr_ws(cbs_plan* plan, int batch, const int32_t* n, const void* kappa_sigma,
                            const void* velocity, const double* background, int dtype, void* workspace,
                            size_t workspace_bytes, void* stream);
cbs_status cbs_workspace_size_cdr(int batch, const int32_t* n, int dtype, size_t* bytes);

/* Total packed cells (sum n[i]^2) and the per-instance k0^2 and eps in use
 * (host arrays of length batch, may be NULL). */
cbs_status cbs_plan_info(cbs_plan plan, int64_t* cells, double* k0sq, double* eps);

/* Execution layout of a plan (host outputs, nullable): the number of lane
 * streams its sweep chains fork into (0 = the caller's stream only, else 2),
 * the column tile width each instance's column launches use (FP32 kernels
 * for CBS_C64 plans, FP64 kernels for CBS_C128 plans) and the threads per
 * column workgroup of those launches (256 or 512). */
cbs_status cbs_plan_layout(cbs_plan plan, int32_t* lanes, int32_t* tiles, int32_t* col_threads);

/*
 * cbs_apply -- y = G (V u + s)   (Sec. 4.1, the Born fixed-point map).
 *   u, s nullable (treated as zero).  y must not alias u or s.
 */
cbs_status cbs_apply(cbs_plan plan, const void* u, const void* s, void* y, void* stream);

/*
 * cbs_residual -- r = G (V u + s) - u + rhs   (Sec. 4.1, Born residual; the
 * optional rhs is already in preconditioned coordinates).
 *   u, s, rhs nullable (zero); r nullable (not stored);
 *   norm2 nullable DEVICE double[batch]: per-instance sum |r|^2 accumulated
 *   in FP64.  r may alias rhs but not u or s.
 */
cbs_status cbs_residual(cbs_plan plan, const void* u, const void* s, const void* rhs,
                        void* r, double* norm2, void* stream);

/*
 * cbs_sweep -- `count` CBS steps in place: u <- u + gamma (G (V u + s) - u)
 *   (Sec. 3.1, Eq. CBS).  Consecutive sweeps are fused (the update of one
 *   sweep and the potential multiply and forward row transforms of the next
 *   share a pass over memory).  s nullable.  norm2 as in cbs_residual: the
 *   residual of the input to the last sweep.  count in [1, 1e6].
 */
cbs_status cbs_sweep(cbs_plan plan, void* u, const void* s, int count, double* norm2, void* stream);

/*
 * cbs_sweep_checkpoints -- `count` CBS steps u_k = u_{k-1} + gamma (G (V
 *   u_{k-1} + s) - u_{k-1}) (Sec. 3.1, Eq. CBS) keeping every iterate: the
 *   checkpoints of the unrolled loss (Sec. 4.2) that cbs_adjoint_step reads
 *   back.  The sweeps are fused as in cbs_sweep (two launches per sweep).
 *   u_all  DEVICE, count + 1 packed fields back to back, field k at element
 *          k * cbs_plan_cells: field 0 holds u_0 (read), fields 1..count
 *          receive u_1..u_count.  Owned by the caller.
 *   s      nullable (zero); must not lie inside u_all.
 *   count in [1, 1e6].  Not for convection-diffusion-reaction or undamped
 *   plans (CBS_ERR_ARG).  Stream-ordered.
 */
cbs_status cbs_sweep_checkpoints(cbs_plan plan, void* u_all, const void* s, int count, void* stream);

/*
 * cbs_npbs_step -- `count` NPBS steps in place (Sec. 4.1, Eq. npbs_integral)
 *   with the linear Fourier layer of App. E (Eq. lfl) as the preconditioner:
 *     r = G(V u + s) - u,   u <- u + F^-1(wf * F r) + wloc * r
 *   (F the unnormalised forward DFT, F^-1 its inverse with the 1/N^2).
 *   wf    device, packed like the fields: per instance the N x N spectral
 *         weights on the DFT bins in FFT order (bin (k1, k2), k = 0..N-1 with
 *         k >= N/2 standing for k - N, at offset_i + k1 N + k2); required
 *   wloc  device, packed field of per-cell local weights (the 1 x 1 channel
 *         weight, or any fixed per-cell factor); NULL = 0
 *   s nullable; u must not alias s, wf or wloc.  count in [1, 1e6].
 *   wf = 0, wloc = gamma gives cbs_sweep's step.  Two transform pairs per
 *   step; uses the plan's scratch field, so calls on one plan serialise.
 */
cbs_status cbs_npbs_step(cbs_plan plan, void* u, const void* s, const void* wf, const void* wloc,
                         int count, void* stream);

/*
 * cbs_helmholtz_residual -- physical residual r = s - A u with the Fourier
 *   pseudospectral A u = F^-1(|xi|^2 F u) - k^2 u (App. D, relation to A;
 *   Sec. 5 stops on ||s - A u|| / ||s||).  One transform pair per call.
 *   u required; s nullable (zero); r nullable (not stored); norm2 nullable
 *   DEVICE double[batch]: per-instance sum |r|^2 in FP64.  r must not alias
 *   u or s.
 */
cbs_status cbs_helmholtz_residual(cbs_plan plan, const void* u, const void* s, void* r,
                                  double* norm2, void* stream);

/*
 * cbs_relres -- per-instance relative residual of a field u (FP64 sums):
 *   stop CBS_STOP_BORN: ||G(V u + s) - u|| / ||G s|| (the preconditioned
 *   residual, Sec. 4.1); CBS_STOP_PHYSICAL: the paper's unified rule
 *   rTol = ||s - A u|| / ||s|| (Sec. 5; A as in cbs_helmholtz_residual, the
 *   CDR operator on CDR plans).  u, s required; relres DEVICE double[batch].
 *   Two transform pairs (Born) or one and a norm pass (physical).  Uses the
 *   plan's scratch, so calls on one plan serialise.
 */
cbs_status cbs_relres(cbs_plan plan, const void* u, const void* s, int stop, double* relres, void* stream);

/*
 * cbs_iterate -- stationary CBS (Sec. 3.1, Eq. CBS) per instance until its
 *   relative residual is at most rtol.
 *   u          device, in/out: initial guess and result
 *   s          device: source
 *   max_sweeps per-instance cap on applied sweeps
 *   check_every  sweeps per refinement chunk (>= 2): the iterate is kept in
 *              FP64 and its residual recomputed in FP64 every check_every
 *              sweeps; sweeps in the plan's dtype advance the correction
 *   stop       CBS_STOP_BORN: ||G(V u + s) - u|| / ||G s||, tested in FP64
 *              at each chunk start and estimated after every sweep (an
 *              instance stops at the first sweep whose estimate is <= rtol
 *              and is confirmed at the next chunk start);
 *              CBS_STOP_PHYSICAL: the paper's rTol = ||s - A u|| / ||s||
 *              (Sec. 5; A u = -Lap u - k^2 u, App. D), tested in FP64 at each
 *              chunk start only (one more transform pair per chunk), so the
 *              sweep count is a multiple of check_every
 *   iters, relres, status  host[batch] outputs (sweeps applied; relative
 *              residual of the returned u under the chosen rule, evaluated
 *              in FP64 -- for CBS_C64 plans that is the FP64 iterate rounded
 *              to FP32, whose residual can exceed the iterate's by about
 *              1e-7 times the conditioning; CBS_INST_* code, decided by the
 *              FP64 iterate's residual); nullable
 *   use_graph  nonzero: replay each chunk from a captured hipGraph
 * Returns CBS_NOT_CONVERGED if any instance stopped without reaching rtol.
 */
cbs_status cbs_iterate(cbs_plan plan, void* u, const void* s, int max_sweeps, double rtol,
                       int check_every, int stop, int32_t* iters, double* relres,
                       int32_t* status, int use_graph, void* stream);

/*
 * fgmres_solve -- flexible GMRES(restart) on B u = G s with B = I - G V = G A
 *   (Prop. 3.1), right-preconditioned by K = inner_sweeps CBS sweeps from zero
 *   (Sec. 4.1: CBS is the diagonal gamma in these coordinates; Sec. 5.1.3 uses
 *   FGMRES with CBS as preconditioner).  The Arnoldi basis, classical
 *   Gram-Schmidt (applied twice), Hessenberg/Givens least squares and the true
 *   residual at each restart are FP64 on the GPU; operator applications run in
 *   the plan's dtype.  iters counts Arnoldi steps.  Outputs as in cbs_iterate.
 *   inner_sweeps in [0, 1000]; 0 is no inner preconditioner (z_j = v_j: GMRES
 *   on B itself), the only choice on undamped plans.
 *   restart must not exceed the plan's max_restart (else CBS_ERR_WORKSPACE).
 */
cbs_status fgmres_solve(cbs_plan plan, void* u, const void* s, int restart, int inner_sweeps,
                        int max_iters, double rtol, int32_t* iters, double* relres,
                        int32_t* status, void* stream);

/*
 * cbs_iterate_async, fgmres_solve_async -- the solvers above as stream-
 *   ordered calls: no host synchronisation, nothing allocated, capturable
 *   into a HIP graph.  iters, relres, status are DEVICE arrays [batch]
 *   (nullable), valid once the stream reaches the end of the call; an
 *   instance that did not finish within the budget reports
 *   CBS_INST_MAX_ITERS.  Instead of stopping when every instance is done,
 *   they enqueue a fixed budget -- ceil(max_sweeps / check_every) + 1 chunks
 *   of cbs_iterate, ceil(max_iters / restart) + 1 restart cycles of
 *   fgmres_solve -- in which finished instances are masked out of every
 *   launch (their workgroups return at once), and the work lists are never
 *   shrunk.  Results are the same as the host-driven calls' (graph replay
 *   off) when the budget is not the binding limit.  Bounds: at most 1e5
 *   chunks / 1e5 Arnoldi steps.
 */
cbs_status cbs_iterate_async(cbs_plan plan, void* u, const void* s, int max_sweeps, double rtol,
                             int check_every, int stop, int32_t* iters, double* relres,
                             int32_t* status, void* stream);
cbs_status fgmres_solve_async(cbs_plan plan, void* u, const void* s, int restart, int inner_sweeps,
                              int max_iters, double rtol, int32_t* iters, double* relres,
                              int32_t* status, void* stream);

/*
 * cbs_adjoint_step -- reverse step of u_{m+1} = u_m + gamma r(u_m) for the
 *   metric-matched loss (Sec. 4.2) and medium gradients.  With
 *   t = G^H(conj(gamma) lam_in), G^H = F^-1 diag(1/conj(lambda)) F:
 *     lam_out = lam_in + conj(V) t - conj(gamma) lam_in
 *     grad_k2 += (-i/eps) lam_in conj(r_m) + t conj(u_m)
 *   where r_m = G(V u_m + s) - u_m is recomputed from the checkpoint u_m.
 *   Gradients follow d/dRe + i d/dIm; eps and k0 are held fixed.
 *   grad_k2 is accumulated (caller zeroes it).  lam_out may alias lam_in.
 */
cbs_status cbs_adjoint_step(cbs_plan plan, const void* u_m, const void* s, const void* lam_in,
                            void* lam_out, void* grad_k2, void* stream);

/*
 * cbs_born_adjoint -- out = R^H e with R = I - G V, the operator of the
 *   metric-matched objective (Sec. 4.2; Prop. 3.1 for Helmholtz, Eq.
 *   cdr_identity for convection-diffusion-reaction plans).  For the loss
 *   l = || G s - R x ||^2 of a network output x its gradient is
 *   dl/dx = -2 R^H (G s - R x), i.e. -2 cbs_born_adjoint of cbs_residual(x, s)
 *   (PyTorch's convention d/dRe + i d/dIm).  Helmholtz and Dirichlet plans:
 *   e - conj(V) G^H e (one transform pair); CDR plans: e - V^H G^H e with
 *   V^H = Dx(dkappa Dx + dvx) + Dy(dkappa Dy + dvy) - dsigma (one transform
 *   pair, then one column and one row derivative pass).  e, out: device packed fields; out may
 *   alias e.  Uses the plan's scratch fields, so calls on one plan serialise.
 */
cbs_status cbs_born_adjoint(cbs_plan plan, const void* e, void* out, void* stream);

/*
 * cbs_metric_matched_grad -- the residual of the metric-matched objective
 *   for a network output x and the residual s it preconditions (Sec. 4.2,
 *   Eq. L_bs^{R_eta}; Eq. cdr_bs_loss on CDR plans), with its gradient:
 *     loss_i = || G s - (I - G V) x ||^2   (FP64 sums, DEVICE double[batch],
 *              nullable)
 *     grad   = -2 scale_i R^H (G s - R x),  R = I - G V
 *   (PyTorch's convention d/dRe + i d/dIm).  scale: DEVICE double[batch] or
 *   NULL (= 1), e.g. the upstream gradient of each instance's loss.  x, grad
 *   required; s nullable (zero); grad may alias x, not s.  Uses the plan's
 *   scratch fields, so calls on one plan serialise.
 */
cbs_status cbs_metric_matched_grad(cbs_plan plan, const void* x, const void* s, const double* scale,
                                   double* loss, void* grad, void* stream);

/*
 * cbs_loss_seed -- a residual loss of the iterate u_K, its adjoint seed
 *   lam_K = dl/du_K and its direct k^2 term (Sec. 4 and 4.2).
 *   weight 0 or 1: l = sum |W r_K|^2 with the Born residual
 *     r_K = G(V u_K + s) - u_K and W = 1 (weight 0; the residual of the
 *     metric-matched loss L_bs^{R_eta}) or W = gamma (weight 1):
 *     lam_K = conj(V) G^H(conj(W) mu) - conj(W) mu,  mu = 2 W r_K,
 *     grad_k2 += G^H(conj(W) mu) conj(u_K)  (+ (-i/eps) mu conj(r_K) for W = gamma).
 *   weight 2: l = sum |e|^2 with the physical residual e = s - A u_K,
 *     A u = -Lap u - k^2 u (App. D; the residual of L_dir and L_bs^{l2}):
 *     lam_K = -2 A^H e = -2 (-Lap e - conj(k^2) e),  grad_k2 += 2 conj(u_K) e.
 *   Other weights: CBS_ERR_ARG.  loss: DEVICE double[batch] (per-instance
 *   FP64 sums), nullable.  grad_k2 is accumulated.  Two transform pairs.
 */
cbs_status cbs_loss_seed(cbs_plan plan, const void* u_k, const void* s, int weight,
                         double* loss, void* lam_out, void* grad_k2, void* stream);

/*
 * cbs_autotune -- for every grid size in the batch, time the column pass at
 *   the tile widths compiled for that size (about 2048 / N columns rounded
 *   down to a power of two, and half and twice that; with 512 threads per
 *   workgroup the default and twice it) on this plan's own instances, in
 *   three interleaved rounds, and keep the fastest; the thread count is one
 *   for the whole plan (the one whose per-size best widths sum to the least
 *   time).  The choice is appended as one JSON line
 *   to the file named by the CBS_AUTOTUNE_CACHE environment variable when it
 *   is set.  tiles: host[batch], nullable: chosen width per instance.
 *   Synchronises `stream`.
 */
cbs_status cbs_autotune(cbs_plan plan, int32_t* tiles, void* stream);

/* Force the column tile width for grid size n (n = 0: every size in the
 * plan).  CBS_ERR_ARG if the width is not one of the widths compiled for a
 * size it applies to at the plan's column thread count.  Synchronises the
 * device. */
cbs_status cbs_set_tile(cbs_plan plan, int n, int columns);

/* Threads per column workgroup of the plan's FP32 column launches: 256, or
 * 512 (one radix-8 butterfly per thread and pass at the default or double
 * width; CBS_C64 periodic Helmholtz plans only, else CBS_ERR_ARG).  Changing
 * it puts every size back to the start width of that thread count.
 * cbs_autotune chooses it too.  Synchronises the device. */
cbs_status cbs_set_col_threads(cbs_plan plan, int threads);

/*
 * cbs_apply_static -- y = G (V u + s), the operator of cbs_apply, for callers
 *   that cannot allocate device memory (code under HIP graph capture, tight
 *   serving loops, harnesses that forbid hipMalloc): no plan, no device
 *   allocation, no host-to-device copy and no synchronisation.  Its scratch
 *   memory -- the spectral buffer between the transform passes, the twiddle
 *   tables, instance descriptors and work lists -- is a fixed device array
 *   inside the library (CBS_STATIC_MAX_BYTES for the spectral buffer plus
 *   0.34 MiB of tables), one per GPU, held from the first call on that
 *   GPU until the process ends.  Every call rewrites all of it that it reads
 *   (one setup kernel before the three transform launches, all on `stream`).
 *   Calls that overlap on one GPU (other streams, other threads) share that
 *   array and race: the caller must order them.
 *   batch      1 .. CBS_STATIC_MAX_BATCH periodic instances, sizes n[i] as for
 *              cbs_setup (host array)
 *   k2         device, packed complex k^2 in the dtype (read by every call)
 *   k0sq, eps  host[batch]: reference k0^2 (finite) and damping eps (finite,
 *              > 0), given explicitly (no automatic choice, no guard)
 *   dtype      CBS_C64 or CBS_C128; u, s nullable (zero); y must not alias
 *              u or s.  Packed cells times the element size (8 or 16 bytes)
 *              must not exceed CBS_STATIC_MAX_BYTES (else CBS_ERR_WORKSPACE).
 *   Column tiles are the widths a plan starts with, so the result is that of
 *   cbs_apply on a plan of the same instances, k0sq and eps.
 */
#define CBS_STATIC_MAX_BATCH 16
#define CBS_STATIC_MAX_BYTES (16u << 20)
cbs_status cbs_apply_static(int batch, const int32_t* n, const void* k2, const double* k0sq,
                            const double* eps, int dtype, const void* u, const void* s, void* y,
                            void* stream);

/* Release a plan: waits for the plan's own streams (the lanes), then frees
 * what cbs_setup allocated.  Work the caller queued on its own streams is
 * the caller's to finish first; a caller-owned workspace may be reused once
 * this returns.  A null plan is ignored. */
void cbs_destroy(cbs_plan plan);
const char* cbs_last_error(void);
const char* cbs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CBS_H_ */
