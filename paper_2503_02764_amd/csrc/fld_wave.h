// Wave-level reduction on gfx950 through DPP lane moves (no LDS round trip).
#pragma once
#include <hip/hip_runtime.h>

namespace fld {

// Move a double across lanes with one DPP control; lanes whose source is out
// of range, or whose row is masked off, receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi =
      __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum of v over the 64 lanes of the wave, returned to every lane; all lanes
// must be active.  Within each row of 16 lanes, shifts by 1, 2, 4 and 8 leave
// the row's sum in its last lane; broadcasting lane 15 into row 1 and lane 47
// into row 3, then lane 31 into rows 2 and 3, leaves the wave's sum in lane
// 63.  The order of the additions is fixed, so every call site that sums the
// same values gets the same bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111, 0xf>(v);  // row_shr:1
  v += dpp_move<0x112, 0xf>(v);  // row_shr:2
  v += dpp_move<0x114, 0xf>(v);  // row_shr:4
  v += dpp_move<0x118, 0xf>(v);  // row_shr:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

}  // namespace fld
