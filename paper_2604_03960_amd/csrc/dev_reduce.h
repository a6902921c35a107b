// Cross-lane FP64 sums on gfx950 wavefronts (64 lanes, four DPP rows of 16) built from DPP
// moves: quad swaps, half-row and row mirrors, and the row-15 / row-31 broadcasts.  Each step is a
// VALU move with no LDS traffic; the grouping of the additions is fixed, so every lane that
// receives a sum receives the same bits.
#pragma once
#include <hip/hip_runtime.h>

namespace tna {

template <int CTRL, int ROWS>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of each DPP row, returned to all 16 lanes
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_d<0x140, 0xf>(v);  // row_mirror
  return v;
}

// sum over the whole wavefront; the total lands in lane 63
__device__ inline double wave_total(double v) {
  v = row16_sum(v);
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

}  // namespace tna
