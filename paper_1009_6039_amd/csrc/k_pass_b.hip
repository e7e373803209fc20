// Pass B of Strain's operator: instantiations for every grid size and launch-geometry
// variant, the launcher and the geometry query used by the autotuner.
#include "strain.h"

#define MA_VARIANT_CASES(NV) X(NV, 0) X(NV, 1) X(NV, 2) X(NV, 3)

int passB_geometry(int n, int v, int* units, int* threads) {
  switch (n * 4 + v) {
#define X(NV, VV)                                           \
  case NV * 4 + VV:                                         \
    *units = Cfg<NV, VV>::B_CPB;                    \
    *threads = Cfg<NV, VV>::B_BLOCK;                  \
    return Canon<NV, VV>::B;
#define Y(NV) MA_VARIANT_CASES(NV)
    MA_FOR_EACH_N(Y)
#undef Y
#undef X
    default:
      return -1;
  }
}

int passB_blocks(int n, int v) {
  int units = 0, threads = 0;
  if (passB_geometry(n, v, &units, &threads) < 0 || units == 0) return 0;
  return n / 2 / units;
}

void launch_passB(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw,
                 hipStream_t st, const TimedLaunch& ev) {
  switch (n * 4 + c.var[1]) {
#define X(NV, VV)                                                                                        \
  case NV * 4 + VV:                                                                                      \
    MA_LAUNCH(ev, (k_passB<NV, Canon<NV, VV>::B>), dim3(NV / 2 / Cfg<NV, VV>::B_CPB, npairs),            \
              dim3(Cfg<NV, VV>::B_BLOCK), st, c, mode, j, tw);                                    \
    break;
#define Y(NV) MA_VARIANT_CASES(NV)
    MA_FOR_EACH_N(Y)
#undef Y
#undef X
    default:
      break;
  }
}
