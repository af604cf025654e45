// F64 instantiations of the Dirichlet (DST-I) row and column kernels.
#include <hip/hip_runtime.h>

#include "kernels_dst.hpp"
#include "launch.hpp"

namespace cbs {

void launch_row_dst(int mode, int grid, hipStream_t st, const Params<double>& p) {
  if (mode == 0)
    hipLaunchKernelGGL(k_row_fwd_dst<double>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 1)
    hipLaunchKernelGGL(k_row_inv_dst<double>, dim3(grid), dim3(kThreads), 0, st, p);
  else
    hipLaunchKernelGGL(k_row_sweep_dst<double>, dim3(grid), dim3(kThreads), 0, st, p);
}

void launch_col_dst(int grid, size_t lds_bytes, hipStream_t st, const Params<double>& p) {
  hipLaunchKernelGGL(k_col_dst<double>, dim3(grid), dim3(kThreads), lds_bytes, st, p);
}

}  // namespace cbs
