// ppt_kernels_ext.hip -- the kernel variants for scenes with the light-stage features (normal maps,
// specular maps, circularly polarized emitters), compiled in a unit of their own so that their FP32
// division and square root stay correctly rounded (the main unit uses the faster hardware
// sequences): these variants differentiate the shading normal through the smooth dielectric's s/p
// rotators, whose derivative amplifies rounding.  The definitions are those of ppt_kernels.hip.
#define PPT_EXT_TU 1
#include "ppt_kernels.hip"

namespace ppt {
template __global__ void k_shade<0, true>(WArgs);
template __global__ void k_shade<1, true>(WArgs);
template __global__ void k_shade<2, true>(WArgs);
template __global__ void k_fold<true, true, false, false>(WArgs);
template __global__ void k_replay<false, true, false, false>(WArgs);
template __global__ void k_replay<true, true, false, false>(WArgs);
template __global__ void k_replay<true, true, true, false>(WArgs);
template __global__ void k_replay<false, true, false, true>(WArgs);
}  // namespace ppt
