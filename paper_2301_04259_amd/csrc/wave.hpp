// Wave64 reductions shared by the device kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace soap {

// value of a double held by one lane, in every lane (scalar registers)
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// DPP row permutations used by the in-row reductions below
constexpr int DPP_PAIR = 0xB1;         // quad_perm 1,0,3,2
constexpr int DPP_QUAD = 0x4E;         // quad_perm 2,3,0,1
constexpr int DPP_HALF_MIRROR = 0x141; // row_half_mirror
constexpr int DPP_MIRROR = 0x140;      // row_mirror

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave (all lanes active), the same in every
// lane: each 16-lane row is summed by DPP exchanges with the partner in the
// other pair, quad, half row and row half, then the four row sums are added
// in row order.  The order of additions is fixed.
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<DPP_PAIR>(v);
  v += dpp_f64<DPP_QUAD>(v);
  v += dpp_f64<DPP_HALF_MIRROR>(v);
  v += dpp_f64<DPP_MIRROR>(v);
  return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

// Sum v[0..15] over the 64 lanes of a wave (all lanes active); lane l ends
// with the total of slot l & 15.  The four in-row levels are transposed
// butterflies on DPP exchanges, partner lanes differing in one lane-index
// bit within the row (row mirror: bit 3, half-row mirror: bit 2, quad swaps:
// bits 1 and 0); each level sends half of the remaining slots to the
// partner and keeps the other half.  The last value is then added over the
// four rows with two shuffles.  The order of additions is fixed.
__device__ __forceinline__ double butterfly16_rows(double (&v)[16], int lane) {
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double send = b3 ? v[i] : v[i + 8];
    const double keep = b3 ? v[i + 8] : v[i];
    v[i] = keep + dpp_f64<DPP_MIRROR>(send);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b2 ? v[i] : v[i + 4];
    const double keep = b2 ? v[i + 4] : v[i];
    v[i] = keep + dpp_f64<DPP_HALF_MIRROR>(send);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b1 ? v[i] : v[i + 2];
    const double keep = b1 ? v[i + 2] : v[i];
    v[i] = keep + dpp_f64<DPP_QUAD>(send);
  }
  {
    const double send = b0 ? v[0] : v[1];
    const double keep = b0 ? v[1] : v[0];
    v[0] = keep + dpp_f64<DPP_PAIR>(send);
  }
  double s = v[0];
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

// OR over the 64 lanes of a wave (all lanes active): in-row swaps by DPP
// (pairs, quads, half rows, rows), then the four row results by readlane.
__device__ __forceinline__ unsigned wave_or32(unsigned v) {
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  return (unsigned)(__builtin_amdgcn_readlane((int)v, 0) | __builtin_amdgcn_readlane((int)v, 16) |
                    __builtin_amdgcn_readlane((int)v, 32) | __builtin_amdgcn_readlane((int)v, 48));
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long v) {
  const unsigned lo = wave_or32((unsigned)v);
  const unsigned hi = wave_or32((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

}  // namespace soap
