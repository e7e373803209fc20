// Pass C of Strain's operator: instantiations for every grid size and launch-geometry
// variant, the launcher and the geometry query used by the autotuner.  Variants 0..3
// are the block-shared kernels (Cfg), 4 and 5 the wave-owned kernels with one and two
// row pairs per block (n >= 128), 6 and 7 the block-shared kernels of variants 0 and 3
// that load the combination's coefficients before the transforms, 8..11 the radix
// plans.
#include "strain.h"

#define MA_VARIANT_CASES(NV) X(NV, 0) X(NV, 1) X(NV, 2) X(NV, 3)

namespace {
// LDS of the wave-owned kernel: five padded transforms per row pair
constexpr bool wave_fits(int n, int ppb) { return 5L * ppb * (n + n / 8) * 8 <= 65536; }

// row pairs per block of wave-owned variant v (4, 5), 0 where it is not offered
int wave_ppb(int n, int v) {
  if (n < 128 || v < 4 || v > 5) return 0;
  const int ppb = v == 5 ? 2 : 1;
  return wave_fits(n, ppb) ? ppb : 0;
}

template <int N, int PPB>
void launch_wave(const LaunchCtx& c, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                 const TimedLaunch& ev) {
  if constexpr (wave_fits(N, PPB))
    MA_LAUNCH(ev, (k_passC_w<N, PPB>), dim3(N / 2 / PPB, npairs), dim3(320 * PPB), st, c, mode, j, tw);
}

// variants 6 and 7: block-shared geometry 0 or 3, coefficients loaded first
int prefetch_base(int v) { return v == 6 ? 0 : 3; }

// block-shared kernel of geometry VV with radix plan P
template <int N, int VV, int P>
void launch_planC(const LaunchCtx& c, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  constexpr int G = Canon<N, VV>::C;
  constexpr int PL = plan_differs(N, P) ? P : 0;
  MA_LAUNCH(ev, (k_passC<N, G, false, PL>), dim3(N / 2 / Cfg<N, VV>::C_PPB, npairs), dim3(Cfg<N, VV>::C_BLOCK),
            st, c, mode, j, tw);
}
}  // namespace

int passC_geometry(int n, int v, int* units, int* threads) {
  if (is_plan_variant(v)) {
    const int g = passC_geometry(n, plan_geometry(v, 3), units, threads);
    if (g < 0 || !plan_differs(n, plan_of_variant(v))) return g;
    return g == 0 ? (v < 10 ? v : v - 2) : v;
  }
  if (v == 6 || v == 7) {
    const int c = passC_geometry(n, prefetch_base(v), units, threads);
    if (c < 0) return -1;
    return c == 0 ? 6 : v;  // variant 3 with the geometry of 0: a duplicate of 6
  }
  if (v >= 4 && v < MA_NVARIANTS) {
    if (!fft_size_supported(n)) return -1;
    const int ppb = wave_ppb(n, v);
    if (ppb == 0) return passC_geometry(n, 0, units, threads) < 0 ? -1 : 0;
    *units = ppb;
    *threads = 320 * ppb;
    return v;
  }
  switch (n * 4 + v) {
#define X(NV, VV)                                           \
  case NV * 4 + VV:                                         \
    *units = Cfg<NV, VV>::C_PPB;                    \
    *threads = Cfg<NV, VV>::C_BLOCK;                  \
    return Canon<NV, VV>::C;
#define Y(NV) MA_VARIANT_CASES(NV)
    MA_FOR_EACH_N(Y)
#undef Y
#undef X
    default:
      return -1;
  }
}

int passC_blocks(int n, int v) {
  int units = 0, threads = 0;
  if (passC_geometry(n, v, &units, &threads) < 0 || units == 0) return 0;
  return n / 2 / units;
}

void launch_passC_only(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw,
                 hipStream_t st, const TimedLaunch& ev) {
  if (is_plan_variant(c.var[2])) {
    const bool p1 = plan_of_variant(c.var[2]) == 1;
    switch (n * 4 + plan_geometry(c.var[2], 3)) {
#define X(NV, VV)                                                       \
  case NV * 4 + VV:                                                     \
    if (p1) launch_planC<NV, VV, 1>(c, npairs, mode, j, tw, st, ev);    \
    else launch_planC<NV, VV, 2>(c, npairs, mode, j, tw, st, ev);       \
    break;
#define Y(NV) X(NV, 0) X(NV, 3)
      MA_FOR_EACH_N(Y)
#undef Y
#undef X
      default:
        break;
    }
    return;
  }
  const int ppb = wave_ppb(n, c.var[2]);
  if (ppb > 0) {
    switch (n * 2 + ppb) {
#define X(NV)                                                   \
  case NV * 2 + 1:                                              \
    launch_wave<NV, 1>(c, npairs, mode, j, tw, st, ev);         \
    break;                                                      \
  case NV * 2 + 2:                                              \
    launch_wave<NV, 2>(c, npairs, mode, j, tw, st, ev);         \
    break;
      MA_FOR_EACH_N_WAVE(X)
#undef X
      default:
        break;
    }
    return;
  }
  const bool pf = c.var[2] == 6 || c.var[2] == 7;
  const int v = pf ? prefetch_base(c.var[2]) : (c.var[2] >= 4 ? 0 : c.var[2]);
  switch (n * 4 + v) {
#define X(NV, VV)                                                                                        \
  case NV * 4 + VV:                                                                                      \
    if (pf) {                                                                                            \
      if constexpr (VV == 0 || VV == 3)                                                                  \
        MA_LAUNCH(ev, (k_passC<NV, Canon<NV, VV>::C, true>), dim3(NV / 2 / Cfg<NV, VV>::C_PPB, npairs),  \
                  dim3(Cfg<NV, VV>::C_BLOCK), st, c, mode, j, tw);                                \
    } else                                                                                               \
      MA_LAUNCH(ev, (k_passC<NV, Canon<NV, VV>::C>), dim3(NV / 2 / Cfg<NV, VV>::C_PPB, npairs),          \
                dim3(Cfg<NV, VV>::C_BLOCK), st, c, mode, j, tw);                                  \
    break;
#define Y(NV) MA_VARIANT_CASES(NV)
    MA_FOR_EACH_N(Y)
#undef Y
#undef X
    default:
      break;
  }
}
