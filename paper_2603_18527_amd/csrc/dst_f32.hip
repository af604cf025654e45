// F32 instantiations of the Dirichlet (DST-I) row and column kernels.
#include <hip/hip_runtime.h>

#include "kernels_dst.hpp"
#include "launch.hpp"

namespace cbs {

void launch_row_dst(int mode, int grid, hipStream_t st, const Params<float>& p) {
  if (mode == 0)
    hipLaunchKernelGGL(k_row_fwd_dst<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 1)
    hipLaunchKernelGGL(k_row_inv_dst<float>, dim3(grid), dim3(kThreads), 0, st, p);
  else
    hipLaunchKernelGGL(k_row_sweep_dst<float>, dim3(grid), dim3(kThreads), 0, st, p);
}

void launch_col_dst(int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p) {
  hipLaunchKernelGGL(k_col_dst<float>, dim3(grid), dim3(kThreads), lds_bytes, st, p);
}

}  // namespace cbs
