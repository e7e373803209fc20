// Autotuner of the launch geometry: for one grid size it times every distinct
// variant of each pass (row pass A, column pass B, row pass C, residual stencil) on
// synthetic fields, rejects a variant whose output differs from the default's
// beyond FP32 reordering, keeps the fastest, and caches the choice in a JSON file
// keyed by device, library sources, grid size, batch and restart length.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "ma_ot.h"
#include "plan_internal.h"

#ifndef MA_SOURCE_HASH
#define MA_SOURCE_HASH "unknown"
#endif

namespace {

#define TRY_HIP(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return MA_EHIP;  \
  } while (0)

int geometry(int pass, int n, int v, int* units, int* threads) {
  switch (pass) {
    case 0: return passA_geometry(n, v, units, threads);
    case 1: return passB_geometry(n, v, units, threads);
    case 2: return passC_geometry(n, v, units, threads);
    case 3: return residual_geometry(n, v, units, threads);
    default: return -1;
  }
}

// pair 0's outputs of one pass, for the comparison with the default geometry
struct Snapshot {
  std::vector<float> a;    // FP32 field outputs
  std::vector<double> s;   // folded partial sums (sum, min or max per slot)
};

int run_pass(const TunerView& t, int pass, int jn, hipStream_t st) {
  switch (pass) {
    case 0: launch_passA_only(t.ctx, t.n, t.npairs, PA_ARNOLDI, jn, t.tw, st); break;
    case 1: launch_passB(t.ctx, t.n, t.npairs, PB_MATVEC, jn, t.tw, st); break;
    case 2: launch_passC_only(t.ctx, t.n, t.npairs, PC_MATVEC, jn, t.tw, st); break;
    default: launch_residual_only(t.ctx, t.n, t.npairs, st); break;
  }
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int snapshot(const TunerView& t, int pass, int v, int jn, hipStream_t st, Snapshot& out) {
  const PairDesc& d = t.desc0;
  const size_t nn = (size_t)t.n * t.n;
  const float* src = nullptr;
  size_t count = 0;
  int nblk = 0, slots = 0;
  std::vector<int> kinds;
  switch (pass) {
    case 0: src = (const float*)d.H; count = 2 * (nn / 2); nblk = passA_blocks(t.n, v); slots = 1; break;
    case 1: src = (const float*)d.T; count = 3 * nn; break;
    case 2: src = d.V + (size_t)(jn + 1) * nn; count = nn; nblk = passC_blocks(t.n, v); slots = MA_MMAX + 1; break;
    default: src = d.coef; count = 5 * nn; nblk = residual_blocks(t.n, v); slots = MA_NPART_RES; break;
  }
  out.a.resize(count);
  TRY_HIP(hipMemcpyAsync(out.a.data(), src, count * 4, hipMemcpyDeviceToHost, st));
  std::vector<double> part((size_t)nblk * std::max(slots, 1));
  if (nblk) TRY_HIP(hipMemcpyAsync(part.data(), d.part, part.size() * 8, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  out.s.clear();
  if (pass == 0) {
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += part[b];
    out.s.push_back(a);
  } else if (pass == 2) {
    for (int l = 0; l <= jn; ++l) {
      double a = 0.0;
      for (int b = 0; b < nblk; ++b) a += part[(size_t)b * slots + l];
      out.s.push_back(a);
    }
  } else if (pass == 3) {
    // slots 10, 11, 13 hold minima, 12 a maximum, the rest sums (the residual kernel's layout)
    for (int k = 0; k < slots; ++k) {
      const int kind = (k == 10 || k == 11 || k == 13) ? 1 : (k == 12 ? 2 : 0);
      double a = kind == 0 ? 0.0 : part[k];
      for (int b = 0; b < nblk; ++b) {
        const double x = part[(size_t)b * slots + k];
        a = kind == 0 ? a + x : (kind == 1 ? std::min(a, x) : std::max(a, x));
      }
      out.s.push_back(a);
    }
  }
  return MA_OK;
}

// fields: identical up to FP32 reordering (the transforms themselves do not depend on
// the geometry); folded sums: within 1e-5 of their magnitude
bool same_output(const Snapshot& ref, const Snapshot& x) {
  if (ref.a.size() != x.a.size() || ref.s.size() != x.s.size()) return false;
  double amax = 0.0, dmax = 0.0;
  for (size_t i = 0; i < ref.a.size(); ++i) {
    if (!std::isfinite(x.a[i])) return false;
    amax = std::max(amax, (double)std::fabs(ref.a[i]));
    dmax = std::max(dmax, (double)std::fabs(ref.a[i] - x.a[i]));
  }
  if (dmax > 1e-6 * amax) return false;
  double smax = 0.0;
  for (double v : ref.s) smax = std::max(smax, std::fabs(v));
  for (size_t i = 0; i < ref.s.size(); ++i)
    if (!(std::fabs(ref.s[i] - x.s[i]) <= 1e-5 * smax + 1e-300)) return false;
  return true;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  return a.substr(0, a.find(':'));
}

// one entry per line: {"arch": "...", "source": "...", "n": N, "pairs": P, "m": M, "v": [a, b, c, r], ...}
bool field_ints(const std::string& line, const char* key, int* out, int count) {
  const std::string k = std::string("\"") + key + "\": ";
  size_t i = line.find(k);
  if (i == std::string::npos) return false;
  i += k.size();
  if (count > 1) {
    if (line[i] != '[') return false;
    ++i;
  }
  for (int c = 0; c < count; ++c) {
    char* end = nullptr;
    const long v = std::strtol(line.c_str() + i, &end, 10);
    if (end == line.c_str() + i) return false;
    out[c] = (int)v;
    i = end - line.c_str();
    while (i < line.size() && (line[i] == ',' || line[i] == ' ')) ++i;
  }
  return true;
}

bool field_doubles(const std::string& line, const char* key, double* out, int count) {
  const std::string k = std::string("\"") + key + "\": [";
  size_t i = line.find(k);
  if (i == std::string::npos) return false;
  i += k.size();
  for (int c = 0; c < count; ++c) {
    char* end = nullptr;
    out[c] = std::strtod(line.c_str() + i, &end);
    if (end == line.c_str() + i) return false;
    i = end - line.c_str();
    while (i < line.size() && (line[i] == ',' || line[i] == ' ')) ++i;
  }
  return true;
}

std::string entry_key(const std::string& arch, int n, int npairs, int m) {
  std::ostringstream k;
  k << "{\"arch\": \"" << arch << "\", \"source\": \"" << MA_SOURCE_HASH << "\", \"n\": " << n
    << ", \"pairs\": " << npairs << ", \"m\": " << m << ",";
  return k.str();
}

bool cache_lookup(const char* path, const std::string& key, ma_tuning* t) {
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t i = line.find(key);
    if (i == std::string::npos) continue;
    int v[4];
    if (!field_ints(line, "v", v, 4)) continue;
    for (int k = 0; k < 4; ++k) t->variant[k] = v[k];
    field_doubles(line, "us", t->us, 4);
    field_doubles(line, "us_default", t->us_default, 4);
    field_ints(line, "rejected", &t->rejected, 1);
    return true;
  }
  return false;
}

void cache_store(const char* path, const std::string& key, const ma_tuning& t) {
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line))
      if (line.find("{\"arch\"") != std::string::npos && line.find(key) == std::string::npos) {
        while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
        keep.push_back(line);
      }
  }
  std::ostringstream e;
  e << key << " \"v\": [" << t.variant[0] << ", " << t.variant[1] << ", " << t.variant[2] << ", " << t.variant[3]
    << "], \"us\": [";
  for (int k = 0; k < 4; ++k) e << (k ? ", " : "") << t.us[k];
  e << "], \"us_default\": [";
  for (int k = 0; k < 4; ++k) e << (k ? ", " : "") << t.us_default[k];
  e << "], \"rejected\": " << t.rejected << "}";
  keep.push_back(e.str());
  std::ofstream out(path);
  out << "{\"entries\": [\n";
  for (size_t i = 0; i < keep.size(); ++i) out << "  " << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
  out << "]}\n";
}

}  // namespace

int tune_passes(const TunerView& view, ma_tuning* t, hipStream_t st) {
  TunerView tv = view;
  const int jn = std::max(0, std::min(tv.ctx.m - 1, 5));  // an Arnoldi step inside the restart length
  hipEvent_t e0, e1;
  TRY_HIP(hipEventCreate(&e0));
  TRY_HIP(hipEventCreate(&e1));
  int err = MA_OK;
  const int npart = std::max(1, tv.npairs / 16);
  t->npairs_part = npart;
  for (int k = 0; k < 4; ++k)
    for (int v = 0; v < MA_TUNE_SLOTS; ++v) t->us_variant[k][v] = t->us_part_variant[k][v] = -1.0;
  // the residual first: it writes the coefficients that pass C reads
  const int order[4] = {3, 0, 1, 2};
  for (int oi = 0; oi < 4 && !err; ++oi) {
    const int pass = order[oi];
    Snapshot ref;
    double best = 0.0;
    int best_v = 0;
    for (int v = 0; v < MA_NVARIANTS && !err; ++v) {
      int units = 0, threads = 0;
      if (geometry(pass, tv.n, v, &units, &threads) != v) continue;  // a duplicate of a smaller index
      tv.ctx.var[pass] = v;
      if ((err = run_pass(tv, pass, jn, st))) break;
      Snapshot snap;
      if ((err = snapshot(tv, pass, v, jn, st, snap))) break;
      if (v == 0) {
        ref = snap;
      } else if (!same_output(ref, snap)) {
        t->rejected++;
        continue;
      }
      // microseconds per launch of this pass over the view's pairs (2 untimed launches,
      // then 20 timed)
      auto time_pass = [&](const TunerView& view, double& us_out) {
        const int reps = 20;
        for (int w = 0; w < 2 && !err; ++w) err = run_pass(view, pass, jn, st);
        if (err || hipEventRecord(e0, st) != hipSuccess) {
          err = err ? err : MA_EHIP;
          return;
        }
        for (int r = 0; r < reps && !err; ++r) err = run_pass(view, pass, jn, st);
        float ms = 0.f;
        if (err || hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          err = err ? err : MA_EHIP;
          return;
        }
        us_out = 1e3 * ms / reps;
      };
      // A solve's launches shrink as pairs finish their GMRES cycles and their Newton
      // steps, so each variant is timed on the whole batch and on a sixteenth of it; the
      // score adds the two per full batch of work.
      double us = 0.0, us_part = 0.0;
      time_pass(tv, us);
      TunerView part = tv;
      part.npairs = npart;
      if (!err && part.npairs < tv.npairs) time_pass(part, us_part);
      if (err) break;
      const double score = us + us_part * ((double)tv.npairs / part.npairs);
      t->us_variant[pass][v] = us;
      t->us_part_variant[pass][v] = us_part;
      if (v == 0) t->us_default[pass] = us;
      if (v == 0 || score < 0.98 * best) {  // a variant must win by 2% to displace an earlier one
        best = score;
        best_v = v;
        t->us[pass] = us;
      }
    }
    tv.ctx.var[pass] = best_v;  // later passes run on the chosen geometry of this one
    t->variant[pass] = best_v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return err;
}

int tune_cache_lookup(const char* path, int n, int npairs, int m, ma_tuning* t) {
  if (!path) return 0;
  return cache_lookup(path, entry_key(arch_name(), n, npairs, m), t) ? 1 : 0;
}

void tune_cache_store(const char* path, int n, int npairs, int m, const ma_tuning& t) {
  if (path) cache_store(path, entry_key(arch_name(), n, npairs, m), t);
}

extern "C" int ma_tune_geometry(int pass, int n, int variant, int* per_block, int* threads) {
  if (!per_block || !threads || variant < 0 || variant >= MA_NVARIANTS) return -1;
  return geometry(pass, n, variant, per_block, threads);
}
