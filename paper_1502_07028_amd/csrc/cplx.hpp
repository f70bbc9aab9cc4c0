// Complex scalar and wavefront lane helpers shared by the reduction kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace tca {

template <typename R>
struct cx {
  R re, im;
};

// Value of v in lane l (l must be wavefront-uniform).
__device__ __forceinline__ double readlane_t(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float readlane_t(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

}  // namespace tca
