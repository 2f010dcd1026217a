// Tile and split-K plan of a partial-MTTKRP launch, and dispatch by tensor dtype.
#include "pm_common.hpp"

namespace nncpk {

// Heuristic: aim for >= ~4 work-groups per CU over the chip, keep each split at
// least two LDS tiles deep, and use the narrow M tile (one wave along M, four
// along K) when the output has few rows, so split-K partial traffic stays small.
PmLaunch pm_plan(int side, int dtype, int64_t IL, int64_t IR, int R) {
  PmLaunch L{};
  L.side = side;
  L.dtype = dtype;
  const int Rc = R < kPmMaxCols ? R : kPmMaxCols;
  L.nb = Rc <= 16 ? 1 : (Rc <= 32 ? 2 : 4);
  const int64_t Mtot = side == 0 ? IL : IR;
  const int64_t Ktot = side == 0 ? IR : IL;
  const int wave_rows = dtype == NNCP_F32 ? pm_f32_wave_rows(side, L.nb) : pm_16_wave_rows(side, L.nb);
  const int64_t target = 1024;
  int wm = 4;
  if ((Mtot + 4 * wave_rows - 1) / (4 * wave_rows) < 64) wm = 1;
  L.mtile = wm * wave_rows;
  L.mtiles = (int)((Mtot + L.mtile - 1) / L.mtile);
  const int64_t ktiles = (Ktot + BK - 1) / BK;
  int64_t ns = (target + L.mtiles - 1) / L.mtiles;
  const int64_t maxs = ktiles / 2 > 0 ? ktiles / 2 : 1;
  if (ns > maxs) ns = maxs;
  if (ns > 256) ns = 256;
  if (ns < 1) ns = 1;
  const int64_t tiles_per = (ktiles + ns - 1) / ns;
  L.kchunk = tiles_per * BK;
  L.nsplit = (int)((Ktot + L.kchunk - 1) / L.kchunk);
  if (L.nsplit < 1) L.nsplit = 1;
  L.partial_doubles = L.nsplit > 1 ? (size_t)L.nsplit * L.nb * 16 * (size_t)L.mtiles * L.mtile : 0;
  L.ncounters = L.mtiles;
  return L;
}

hipError_t pm_launch(const PmLaunch& L, const PmArgs& a, hipStream_t st) {
  if (L.dtype == NNCP_F32) return pm_launch_f32(L, a, st);
  return pm_launch_16(L, a, st);
}

}  // namespace nncpk
