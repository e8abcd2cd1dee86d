// lbm_step3d.hip -- the D3Q19 instances of the fused step kernel.
//
// A translation unit of its own so that the build can compile these kernels
// with the machine scheduler's ILP strategy (-mllvm
// --amdgpu-sched-strategy=max-ilp) and the rest of the library with the
// default one: on D3Q19 256^3 the ILP schedule takes 2.7 % off the FP32
// forcing step, 2 % off FP32 storage with FP64 arithmetic and 2.8 % off the
// FP64 equilibrium step, but it slows the batched D2Q9 FP32 kernel by 5 %.
// lbm_capi.hip declares these instances extern and launches them.
#include <hip/hip_runtime.h>

#include "lbm.h"
#include "lbm_step.h"

namespace lbm {
#define LBM_STEP3D_DEFINE(SCH, S, R, TX, TY) \
    template __global__ void step_kernel<D3Q19, SCH, S, R, TX, TY>(StepArgs<R>);
LBM_STEP3D_INSTANCES(LBM_STEP3D_DEFINE)
#undef LBM_STEP3D_DEFINE
} // namespace lbm
