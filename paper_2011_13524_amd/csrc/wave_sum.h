// Wavefront reductions on the vector ALU (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace qsv {

// Sum over the 64 lanes of a wavefront, complete in lane 63 (the other lanes
// hold partial sums), by DPP row operations inside the vector ALU -- quad
// permutes, the row half-mirror and mirror, then the broadcasts of lanes 15
// and 31 into the rows above -- instead of LDS permutes; the order of the
// additions is fixed. Lanes a DPP step does not write read 0 (the old value
// passed in).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_to_last(double v) {
  v += dpp_f64<0xb1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e, 0xf>(v);   // quad_perm [2, 3, 0, 1]: every lane holds its quad's sum
  v += dpp_f64<0x141, 0xf>(v);  // row_half_mirror: its 8 lanes' sum
  v += dpp_f64<0x140, 0xf>(v);  // row_mirror: its row's (16 lanes') sum
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3: rows 0 + 1, rows 2 + 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3: row 3 holds all 64 lanes
  return v;
}

}  // namespace qsv
