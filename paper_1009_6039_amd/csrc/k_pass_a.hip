// Pass A of Strain's operator: instantiations for every grid size and launch-geometry
// variant, the launcher and the geometry query used by the autotuner.  Variants 0..3
// are the block-shared kernels (Cfg), 4..6 the wave-owned ones, 8..11 the radix plans.
#include "strain.h"

#define MA_VARIANT_CASES(NV) X(NV, 0) X(NV, 1) X(NV, 2) X(NV, 3)

namespace {
// wave-owned row pass A: one row pair per wave, W waves per block
constexpr bool waveA_fits(int n, int w) { return (long)w * (n + n / 8) * 8 + 512 <= 65536; }
int waveA_w(int n, int v) {
  if (n < 128 || v < 4 || v > 7) return 0;
  const int w = v == 5 ? 2 : (v == 6 ? 8 : 4);
  return ((n / 2) % w == 0 && waveA_fits(n, w)) ? w : 0;
}
template <int N, int W>
void launch_waveA(const LaunchCtx& c, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  if constexpr (waveA_fits(N, W) && (N / 2) % W == 0)
    MA_LAUNCH(ev, (k_passA_w<N, W>), dim3(N / 2 / W, npairs), dim3(64 * W), st, c, mode, jn, tw);
}

// block-shared kernel of geometry VV with radix plan P
template <int N, int VV, int P>
void launch_planA(const LaunchCtx& c, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  constexpr int G = Canon<N, VV>::A;
  constexpr int PL = plan_differs(N, P) ? P : 0;
  MA_LAUNCH(ev, (k_passA<N, G, PL>), dim3(N / 2 / Cfg<N, VV>::A_PPB, npairs), dim3(Cfg<N, VV>::A_BLOCK), st, c,
            mode, jn, tw);
}
}  // namespace

int passA_geometry(int n, int v, int* units, int* threads) {
  if (is_plan_variant(v)) {
    const int g = passA_geometry(n, plan_geometry(v, 2), units, threads);
    if (g < 0 || !plan_differs(n, plan_of_variant(v))) return g;
    return g == 0 ? (v < 10 ? v : v - 2) : v;
  }
  if (v >= 4 && v < MA_NVARIANTS) {
    if (!fft_size_supported(n)) return -1;
    const int w = waveA_w(n, v);
    if (w == 0) return passA_geometry(n, 0, units, threads) < 0 ? -1 : 0;
    *units = w;
    *threads = 64 * w;
    return v == 7 ? 4 : v;
  }
  switch (n * 4 + v) {
#define X(NV, VV)                                           \
  case NV * 4 + VV:                                         \
    *units = Cfg<NV, VV>::A_PPB;                    \
    *threads = Cfg<NV, VV>::A_BLOCK;                  \
    return Canon<NV, VV>::A;
#define Y(NV) MA_VARIANT_CASES(NV)
    MA_FOR_EACH_N(Y)
#undef Y
#undef X
    default:
      return -1;
  }
}

int passA_blocks(int n, int v) {
  int units = 0, threads = 0;
  if (passA_geometry(n, v, &units, &threads) < 0 || units == 0) return 0;
  return n / 2 / units;
}

void launch_passA_only(const LaunchCtx& c, int n, int npairs, int mode, int jn, const float2* tw,
                 hipStream_t st, const TimedLaunch& ev) {
  if (is_plan_variant(c.var[0])) {
    const bool p1 = plan_of_variant(c.var[0]) == 1;
    switch (n * 4 + plan_geometry(c.var[0], 2)) {
#define X(NV, VV)                                                        \
  case NV * 4 + VV:                                                      \
    if (p1) launch_planA<NV, VV, 1>(c, npairs, mode, jn, tw, st, ev);    \
    else launch_planA<NV, VV, 2>(c, npairs, mode, jn, tw, st, ev);       \
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
  const int w = waveA_w(n, c.var[0]);
  if (w > 0) {
    switch (n * 16 + w) {
#define X(NV)                                                            \
  case NV * 16 + 2: launch_waveA<NV, 2>(c, npairs, mode, jn, tw, st, ev); break; \
  case NV * 16 + 4: launch_waveA<NV, 4>(c, npairs, mode, jn, tw, st, ev); break; \
  case NV * 16 + 8: launch_waveA<NV, 8>(c, npairs, mode, jn, tw, st, ev); break;
      MA_FOR_EACH_N_WAVE(X)
#undef X
      default:
        break;
    }
    return;
  }
  switch (n * 4 + (c.var[0] >= 4 ? 0 : c.var[0])) {
#define X(NV, VV)                                                                                        \
  case NV * 4 + VV:                                                                                      \
    MA_LAUNCH(ev, (k_passA<NV, Canon<NV, VV>::A>), dim3(NV / 2 / Cfg<NV, VV>::A_PPB, npairs),            \
              dim3(Cfg<NV, VV>::A_BLOCK), st, c, mode, jn, tw);                                    \
    break;
#define Y(NV) MA_VARIANT_CASES(NV)
    MA_FOR_EACH_N(Y)
#undef Y
#undef X
    default:
      break;
  }
}
