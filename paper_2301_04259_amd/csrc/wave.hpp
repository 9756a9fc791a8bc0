// Wave64 reductions shared by the device kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace soap {

// Sum v[0..15] over the 64 lanes of a wave; lane l ends with the total of
// slot (l >> 2) & 15.  Each butterfly step sends half of the remaining slots
// to the partner lane and keeps the other half, so the 16 sums cost 17
// shuffles instead of 96.  The order of additions is fixed.
__device__ __forceinline__ double butterfly16(double (&v)[16], int lane) {
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double send = b5 ? v[i] : v[i + 8];
    double keep = b5 ? v[i + 8] : v[i];
    v[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double send = b4 ? v[i] : v[i + 4];
    double keep = b4 ? v[i + 4] : v[i];
    v[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    double send = b3 ? v[i] : v[i + 2];
    double keep = b3 ? v[i + 2] : v[i];
    v[i] = keep + __shfl_xor(send, 8, 64);
  }
  {
    double send = b2 ? v[0] : v[1];
    double keep = b2 ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 4, 64);
  }
  double s = v[0];
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 1, 64);
  return s;
}

// value of a double held by one lane, in every lane (scalar registers)
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

}  // namespace soap
