// Host-side launchers of the CBS kernels.  The kernels live in separate
// translation units (ops_f32.hip, ops_f64.hip, misc.hip) that are compiled in
// parallel; the host planner only sees these declarations.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/cbs.h"
#include "params.hpp"

namespace cbs {

// Record the message cbs_last_error() returns for this thread and pass the
// status through (defined with the C ABI in cbs.hip).
cbs_status report_error(cbs_status st, const std::string& msg);

// mode 0: prologue + forward rows, 1: inverse rows + epilogue,
// 2: fused inverse rows + CBS update + next prologue + forward rows,
// 3 / 4: the two fused halves of an NPBS step (periodic plans only)
void launch_row(int mode, int grid, hipStream_t st, const Params<float>& p);
void launch_row(int mode, int grid, hipStream_t st, const Params<double>& p);
void launch_col(int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p);
void launch_col(int grid, size_t lds_bytes, hipStream_t st, const Params<double>& p);
// the same for Dirichlet plans (DST-I kernels; called by launch_row / launch_col)
void launch_row_dst(int mode, int grid, hipStream_t st, const Params<float>& p);
void launch_row_dst(int mode, int grid, hipStream_t st, const Params<double>& p);
void launch_col_dst(int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p);
void launch_col_dst(int grid, size_t lds_bytes, hipStream_t st, const Params<double>& p);
// convection-diffusion-reaction plans: the row pass (mode 0: V u + s -> forward
// rows; 1: V u + s; 2: e - V^H g), the column pass (adj 0 / 1) and the
// coefficient split at setup
void launch_cdr_row(int mode, int grid, hipStream_t st, const Params<float>& p);
void launch_cdr_row(int mode, int grid, hipStream_t st, const Params<double>& p);
void launch_cdr_col(int adj, int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p);
void launch_cdr_col(int adj, int grid, size_t lds_bytes, hipStream_t st, const Params<double>& p);
void launch_cdr_split(int grid, hipStream_t st, const InstDesc* inst, const int2* items, cpx<float>* c1,
                      cpx<float>* c2);
void launch_cdr_split(int grid, hipStream_t st, const InstDesc* inst, const int2* items, cpx<double>* c1,
                      cpx<double>* c2);
void launch_pointwise(int grid, hipStream_t st, const PwParams<float>& p);
void launch_pointwise(int grid, hipStream_t st, const PwParams<double>& p);
void launch_zupdate(int grid, hipStream_t st, const KryParams& k, const cpx<float>* z, cpx<double>* x);
void launch_zupdate(int grid, hipStream_t st, const KryParams& k, const cpx<double>* z, cpx<double>* x);

void launch_instance_sums(int batch, hipStream_t st, const InstDesc* inst, const double* partials,
                          double* out);
void launch_check64(int batch, hipStream_t st, const IterState& is, const InstDesc* inst,
                    const double* partials);
void launch_check32(int count, const int* ids, hipStream_t st, const IterState& is,
                    const InstDesc* inst, const double* partials);
void launch_set_bnorm(int batch, hipStream_t st, const IterState& is, const InstDesc* inst,
                      const double* partials);
void launch_stats(int grid, hipStream_t st, const InstDesc* inst, const int2* items,
                  const cpx<double>* k2, double* partials, int phase);
void launch_widen_all(hipStream_t st, const cpx<float>* in, cpx<double>* out, long long count);
// stream-ordered solver state: initial values, and the per-instance results
// copied to the caller's device arrays (running / pending -> ST_MAXIT)
void launch_solver_init(hipStream_t st, int* status, int* iters, double* relres, int* kjend,
                        double* rtol_d, double* rtol32_d, int* max_d, int batch, double rtol,
                        double rtol32, int max_count);
void launch_solver_out(hipStream_t st, const IterState& is, int batch, int* o_iters, double* o_relres,
                       int* o_status);
// per-row-item partial sums of |x|^2 (then launch_instance_sums), and
// out = sqrt(num / den) per instance
void launch_norm2_rows(int grid, hipStream_t st, const InstDesc* inst, const int2* items,
                       const cpx<float>* x, double* partials);
void launch_norm2_rows(int grid, hipStream_t st, const InstDesc* inst, const int2* items,
                       const cpx<double>* x, double* partials);
void launch_ratio(int batch, hipStream_t st, const double* num, const double* den, double* out);
void launch_gs_dots(int grid, bool final_pass, hipStream_t st, const KryParams& k);
void launch_gs_finish(int batch, bool final_pass, hipStream_t st, const KryParams& k);
void launch_gs_update(int grid, hipStream_t st, const KryParams& k);
void launch_gs_check(int batch, hipStream_t st, const KryParams& k);
void launch_backsolve(int batch, hipStream_t st, const KryParams& k);
void launch_fg_restart(int batch, hipStream_t st, const KryParams& k, int first);

}  // namespace cbs
