// Pass B of Strain's operator: instantiations for every grid size and launch-geometry
// variant, the launcher and the geometry query used by the autotuner.  Variants 0..3
// are the block-shared kernels (Cfg), 4..6 the wave-owned ones, 8..11 the radix plans.
#include "strain.h"

#define MA_VARIANT_CASES(NV) X(NV, 0) X(NV, 1) X(NV, 2) X(NV, 3)

namespace {
// wave-owned column pass B: one column per wave, W waves per block
constexpr int waveB_region(int n) {  // WaveRegion<n>::size
  return (n + n / 8) + ((8 - (n + n / 8) % 32) + 32) % 32;
}
constexpr bool waveB_fits(int n, int w) { return (long)w * waveB_region(n) * 8 <= 65536; }
static_assert(waveB_region(512) == WaveRegion<512>::size, "region stride");
int waveB_w(int n, int v) {
  if (n < 128 || n % 64 != 0 || v < 4 || v > 7) return 0;
  const int w = v == 5 ? 4 : (v == 6 ? 2 : 8);
  return ((n / 2) % w == 0 && waveB_fits(n, w)) ? w : 0;
}
template <int N, int W>
void launch_waveB(const LaunchCtx& c, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  if constexpr (waveB_fits(N, W) && (N / 2) % W == 0 && N % 64 == 0)
    MA_LAUNCH(ev, (k_passB_w<N, W>), dim3(N / 2 / W, npairs), dim3(64 * W), st, c, mode, j, tw);
}

// block-shared kernel of geometry VV with radix plan P
template <int N, int VV, int P>
void launch_planB(const LaunchCtx& c, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  constexpr int G = Canon<N, VV>::B;
  constexpr int PL = plan_differs(N, P) ? P : 0;
  MA_LAUNCH(ev, (k_passB<N, G, PL>), dim3(N / 2 / Cfg<N, VV>::B_CPB, npairs), dim3(Cfg<N, VV>::B_BLOCK), st, c,
            mode, j, tw);
}
}  // namespace

int passB_geometry(int n, int v, int* units, int* threads) {
  if (is_plan_variant(v)) {
    const int g = passB_geometry(n, plan_geometry(v, 2), units, threads);
    if (g < 0 || !plan_differs(n, plan_of_variant(v))) return g;
    return g == 0 ? (v < 10 ? v : v - 2) : v;
  }
  if (v >= 4 && v < MA_NVARIANTS) {
    if (!fft_size_supported(n)) return -1;
    const int w = waveB_w(n, v);
    if (w == 0) return passB_geometry(n, 0, units, threads) < 0 ? -1 : 0;
    *units = w;
    *threads = 64 * w;
    return v == 7 ? 4 : v;
  }
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
  if (is_plan_variant(c.var[1])) {
    const bool p1 = plan_of_variant(c.var[1]) == 1;
    switch (n * 4 + plan_geometry(c.var[1], 2)) {
#define X(NV, VV)                                                       \
  case NV * 4 + VV:                                                     \
    if (p1) launch_planB<NV, VV, 1>(c, npairs, mode, j, tw, st, ev);    \
    else launch_planB<NV, VV, 2>(c, npairs, mode, j, tw, st, ev);       \
    break;
#define Y(NV) X(NV, 0) X(NV, 2)
      MA_FOR_EACH_N(Y)
#undef Y
#undef X
      default:
        break;
    }
    return;
  }
  const int w = waveB_w(n, c.var[1]);
  if (w > 0) {
    switch (n * 16 + w) {
#define X(NV)                                                           \
  case NV * 16 + 2: launch_waveB<NV, 2>(c, npairs, mode, j, tw, st, ev); break; \
  case NV * 16 + 4: launch_waveB<NV, 4>(c, npairs, mode, j, tw, st, ev); break; \
  case NV * 16 + 8: launch_waveB<NV, 8>(c, npairs, mode, j, tw, st, ev); break;
      MA_FOR_EACH_N_WAVE(X)
#undef X
      default:
        break;
    }
    return;
  }
  switch (n * 4 + (c.var[1] >= 4 ? 0 : c.var[1])) {
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
