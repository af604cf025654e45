// FP32 instantiations of the convection-diffusion-reaction derivative passes.
#include <hip/hip_runtime.h>

#include "kernels_cdr.hpp"
#include "launch.hpp"

namespace cbs {

void launch_cdr_row(int mode, int grid, hipStream_t st, const Params<float>& p) {
  if (mode == 0)
    hipLaunchKernelGGL((k_cdr_row<float, 0>), dim3(grid), dim3(kThreads), 0, st, p);
  else if (mode == 1)
    hipLaunchKernelGGL((k_cdr_row<float, 1>), dim3(grid), dim3(kThreads), 0, st, p);
  else
    hipLaunchKernelGGL((k_cdr_row<float, 2>), dim3(grid), dim3(kThreads), 0, st, p);
}

void launch_cdr_col(int adj, int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p) {
  if (adj)
    hipLaunchKernelGGL((k_cdr_col<float, 1>), dim3(grid), dim3(kThreads), lds_bytes, st, p);
  else
    hipLaunchKernelGGL((k_cdr_col<float, 0>), dim3(grid), dim3(kThreads), lds_bytes, st, p);
}

void launch_cdr_split(int grid, hipStream_t st, const InstDesc* inst, const int2* items, cpx<float>* c1,
                      cpx<float>* c2) {
  hipLaunchKernelGGL(k_cdr_split<float>, dim3(grid), dim3(kThreads), 0, st, inst, items, c1, c2);
}

}  // namespace cbs
