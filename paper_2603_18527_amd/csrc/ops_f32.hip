// FP32 instantiations of the row, column, pointwise and
// FGMRES-update kernels.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"

namespace cbs {

void launch_row(int mode, int grid, hipStream_t st, const Params<float>& p) {
  if (p.dst) {
    launch_row_dst(mode, grid, st, p);
    return;
  }
  if (mode == 0)
    hipLaunchKernelGGL(k_row_fwd<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 1)
    hipLaunchKernelGGL(k_row_inv<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 2)
    hipLaunchKernelGGL(k_row_sweep<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 3)
    hipLaunchKernelGGL(k_row_npbs_a<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 4)
    hipLaunchKernelGGL(k_row_npbs_b<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 5)
    hipLaunchKernelGGL(k_row_adj_fwd<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else
    hipLaunchKernelGGL(k_row_adj_inv<float>, dim3(grid), dim3(kThreads), 0, st, p);
}

void launch_col(int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p) {
  if (p.dst) {
    launch_col_dst(grid, lds_bytes, st, p);
    return;
  }
  if (p.col_threads == kColThreadsWide)
    hipLaunchKernelGGL(k_col_wide<float>, dim3(grid), dim3(kColThreadsWide), lds_bytes, st, p);
  else
    hipLaunchKernelGGL(k_col<float>, dim3(grid), dim3(kThreads), lds_bytes, st, p);
}

void launch_pointwise(int grid, hipStream_t st, const PwParams<float>& p) {
  hipLaunchKernelGGL(k_pointwise<float>, dim3(grid), dim3(kThreads), 0, st, p);
}

void launch_zupdate(int grid, hipStream_t st, const KryParams& k, const cpx<float>* z, cpx<double>* x) {
  hipLaunchKernelGGL(k_zupdate<float>, dim3(grid), dim3(kThreads), 0, st, k, z, x);
}

}  // namespace cbs
