// FP32 instantiations of the convection-diffusion-reaction derivative passes.
#include <hip/hip_runtime.h>

#include "kernels_cdr.hpp"
#include "launch.hpp"

namespace cbs {

void launch_row_cdr(int grid, hipStream_t st, const Params<float>& p) {
  hipLaunchKernelGGL(k_cdr_row<float>, dim3(grid), dim3(kThreads), 0, st, p);
}

void launch_col_cdr(int grid, size_t lds_bytes, hipStream_t st, const Params<float>& p) {
  hipLaunchKernelGGL(k_cdr_col<float>, dim3(grid), dim3(kThreads), lds_bytes, st, p);
}

void launch_cdr_split(int grid, hipStream_t st, const InstDesc* inst, const int2* items, cpx<float>* c1,
                      cpx<float>* c2) {
  hipLaunchKernelGGL(k_cdr_split<float>, dim3(grid), dim3(kThreads), 0, st, inst, items, c1, c2);
}

}  // namespace cbs
