// Autotuner: the pass kernels exist in several tile shapes ("variants").  For a plan it times
// each variant of each launch group on scratch buffers and keeps the fastest:
//   * five-pass kernels: per (pass, transform length, padding), variants 0 and 1;
//   * fused passes A and C: per (pass, Ny, Nx), every variant that exists for the box
//     (fused_variant_ok), pass A and pass C chosen independently.
// Results are cached in a text file keyed by GPU architecture and precision (SBP_TUNE_CACHE,
// default $HOME/.cache/sbp_tune.txt) so later plans skip the measurement.  Each box records
// where each of its variants came from (default, cache or measurement); the plan's describe()
// reports it per launch group.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <tuple>

#include "tune.hpp"
#include "wide.hpp"

namespace sbp {

const char* const kVarSrcName[3] = {"default", "cache", "measured"};

void default_variants(int prec, const BoxGeom& g, int var[kKinds]) {
  for (int k = 0; k < 5; ++k) var[k] = 1;
  for (int k = 5; k < kKinds; ++k) var[k] = 0;
  // float passes A and C keep 32-byte rows (variant 0; pass C then transforms eight planes at a
  // time, one wavefront each, where Ny <= 256); double passes A and C split the z columns of a
  // position over a lane pair
  if (!prec && g.ny <= 256) var[kFA] = var[kFC] = 3;
  // with A = Nx/16 <= 8 planes a thread holds half the spectra of A = 16 or less, which leaves room
  // for 64-byte rows (variant 1): twice the z cells per block, half the blocks
  if (prec && g.nx <= 128 && g.ny <= 256) var[kFA] = var[kFC] = 1;
  // five-pass float y transforms longer than 512: half-width rows (1024 x 1024 x 256: 809 -> 552 us
  // forward, 1235 -> 696 us inverse, the autotuner's choice too)
  if (prec && g.ny > 512) var[kYFwd] = var[kYInv] = 0;
  // fused float boxes wider than 256 cells take the wide schedule (B = 64), one kernel per pass
  if (prec && g.nx > 256) var[kFA] = var[kFB] = var[kFC] = kWideVariant;
}

// The fused pass-A/C kernels that exist: variant 0 (32-byte rows) always; variant 1 (64-byte
// rows) for float with A <= 8 and Ny <= 256; variant 2 (16-byte rows, 256 threads) for pass C
// with Ny <= 256; variant 3 (the split kernels, one z column per lane) with Ny <= 256.
bool fused_variant_ok(int prec, int kind, const BoxGeom& g, int v) {
  if (g.nx > 256) return v == kWideVariant;
  if (kind != kFA && kind != kFC) return v == 0;
  const int a = g.nx / 16;
  switch (v) {
    case 0: return true;
    case 1: return prec == 1 && a >= 1 && a <= 8 && g.ny <= 256;
    case 2: return kind == kFC && g.ny <= 256;
    case 3: return g.ny <= 256;
    default: return false;
  }
}

namespace {

// arch, prec, kind, len, aux: aux is the padding for the z pass, Nx for fused passes A and C
// (len = Ny), 0 otherwise.  Kind kPlanChoice records, for one set of fused box shapes (len = a
// hash of them, aux = the box count), whether the per-key choices beat the defaults (1) or not.
using Key = std::tuple<std::string, int, int, int, int>;
constexpr int kPlanChoice = 100;

std::string cache_path() {
  const char* p = getenv("SBP_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/sbp_tune.txt";
}

std::map<Key, int> load_cache(const std::string& path) {
  std::map<Key, int> m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string arch;
    int prec, kind, len, q, v;
    if (ss >> arch >> prec >> kind >> len >> q >> v) m[Key(arch, prec, kind, len, q)] = v;
  }
  return m;
}

void save_cache(const std::string& path, const std::map<Key, int>& m) {
  std::ofstream f(path, std::ios::trunc);
  if (!f) return;  // a cache that cannot be written only costs a re-measurement
  for (auto& kv : m)
    f << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' ' << std::get<2>(kv.first) << ' '
      << std::get<3>(kv.first) << ' ' << std::get<4>(kv.first) << ' ' << kv.second << '\n';
}

int launch_len(const BoxInfo& b, int kind) {
  if (kind == kFA || kind == kFC) return b.g.ny;
  return (kind == kYFwd || kind == kYInv) ? b.g.ny : (kind == kZ ? b.g.m : b.g.nx);
}
int launch_aux(const BoxInfo& b, int kind) {
  if (kind == kZ) return b.pad;
  if (kind == kFA || kind == kFC) return b.g.nx;
  return 0;
}
Key key_of(const std::string& arch, int prec, const BoxInfo& b, int kind) {
  return Key(arch, prec, kind, launch_len(b, kind), launch_aux(b, kind));
}

// kinds a box's schedule uses that have a choice of variants
bool tunable(const BoxInfo& b, int kind) {
  if (b.fused) return (kind == kFA || kind == kFC) && b.g.nx <= 256;  // the wide schedule has one variant
  return kind < 5;
}

}  // namespace

sbp_status autotune(sbp_plan p) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, plan_device(p)) != hipSuccess) return fail(SBP_E_HIP, "device properties");
  const std::string arch = prop.gcnArchName;
  const int prec = plan_prec(p);
  std::vector<BoxInfo>& boxes = plan_boxes(p);
  const std::string path = cache_path();
  std::map<Key, int> cache = load_cache(path);
  constexpr int kReps = 10;

  // keys missing from the cache, per schedule
  std::set<Key> missing;
  for (auto& b : boxes)
    for (int k = 0; k < kKinds; ++k)
      if (tunable(b, k) && !cache.count(key_of(arch, prec, b, k))) missing.insert(key_of(arch, prec, b, k));

  if (!missing.empty()) {
    std::map<Key, std::vector<double>> best;  // key -> summed group time per variant (< 0: not run)
    plan_set_nomix(p, true);
    sbp_status st = SBP_OK;
    for (int v = 0; v < kFusedVariants && st == SBP_OK; ++v) {
      bool any = false;
      for (auto& b : boxes) {
        int dv[kKinds];
        default_variants(prec, b.g, dv);
        for (int k = 0; k < kKinds; ++k) {
          if (!tunable(b, k)) continue;
          const bool ok = b.fused ? fused_variant_ok(prec, k, b.g, v) : v < kVariants;
          b.var[k] = ok ? v : dv[k];
          any = any || (ok && missing.count(key_of(arch, prec, b, k)));
        }
      }
      if (!any) continue;
      std::vector<Launch> ls;
      std::vector<double> ms;
      st = plan_time_groups(p, kReps, ls, ms);
      if (st != SBP_OK) break;
      for (size_t i = 0; i < ls.size(); ++i) {
        const Launch& l = ls[i];
        if (l.variant != v || l.kind == kFB) continue;
        // every box of a group shares its key: the group's time goes to that key
        const BoxInfo& b0 = boxes[plan_group_box(p, l)];
        if (!tunable(b0, l.kind)) continue;
        auto& slot = best[key_of(arch, prec, b0, l.kind)];
        slot.resize(kFusedVariants, -1.0);
        slot[v] = (slot[v] < 0.0 ? 0.0 : slot[v]) + ms[i];
      }
    }
    plan_set_nomix(p, false);
    if (st != SBP_OK) return st;
    for (auto& kv : best) {
      if (!missing.count(kv.first)) continue;
      int arg = -1;
      for (int v = 0; v < kFusedVariants; ++v)
        if (kv.second[v] >= 0.0 && (arg < 0 || kv.second[v] < kv.second[arg])) arg = v;
      if (arg >= 0) cache[kv.first] = arg;
    }
    save_cache(path, cache);
  }
  bool any_measured = !missing.empty(), any_cached = false;
  for (auto& b : boxes) {
    default_variants(prec, b.g, b.var);
    for (int k = 0; k < kKinds; ++k) {
      b.var_src[k] = kVarDefault;
      if (!tunable(b, k)) continue;
      const Key key = key_of(arch, prec, b, k);
      auto it = cache.find(key);
      if (it == cache.end()) continue;
      // a cache entry for a variant that does not exist for this box (a stale or edited file)
      // is ignored
      const bool ok = b.fused ? fused_variant_ok(prec, k, b.g, it->second) : (it->second >= 0 && it->second < kVariants);
      if (!ok) continue;
      b.var[k] = it->second;
      b.var_src[k] = missing.count(key) ? kVarMeasured : kVarCache;
      any_cached = any_cached || !missing.count(key);
    }
  }

  // The per-key choices were timed group by group with every (Ny, A) in a launch of its own, but
  // float plans merge the boxes with A <= 8 and 64-byte rows (the default), of any Ny <= 256 and
  // across Ny <= 128, into few launches.  Where that merging happens, whether the per-key choices beat the defaults is a
  // property of the whole plan: time both once (per set of fused box shapes, cached) and keep
  // the faster.
  bool differs = false;
  std::map<int, std::set<int>> mixed;  // remap -> (Ny, A) of the boxes merged by default
  uint32_t sig = 2166136261u;  // FNV-1a over the fused boxes' kernel shapes
  auto mix = [&](uint32_t v) {
    for (int i = 0; i < 4; ++i) {
      sig ^= (v >> (8 * i)) & 0xffu;
      sig *= 16777619u;
    }
  };
  for (auto& b : boxes) {
    if (!b.fused) continue;
    int dv[kKinds];
    default_variants(prec, b.g, dv);
    differs = differs || b.var[kFA] != dv[kFA] || b.var[kFC] != dv[kFC];
    if (dv[kFA] == 1) mixed[b.g.remap].insert(1000 * b.g.ny + b.g.nx / 16);
    mix((uint32_t)b.g.nx);
    mix((uint32_t)b.g.ny);
    mix((uint32_t)b.g.nz);
    mix((uint32_t)b.pad);
    mix((uint32_t)b.g.remap);
  }
  bool merges = false;  // a default launch would serve boxes of several (Ny, A)
  for (auto& kv : mixed) merges = merges || kv.second.size() > 1;
  if (differs && merges) {
    const Key pk(arch, prec, kPlanChoice, (int)(sig & 0x7fffffffu), (int)boxes.size());
    int use_tuned = 1;
    auto it = cache.find(pk);
    if (it != cache.end()) {
      use_tuned = it->second;
    } else {
      std::vector<int> tuned(2 * boxes.size());
      for (size_t i = 0; i < boxes.size(); ++i) {
        tuned[2 * i] = boxes[i].var[kFA];
        tuned[2 * i + 1] = boxes[i].var[kFC];
      }
      double total[2] = {0.0, 0.0};  // defaults, per-key choices
      for (int c = 0; c < 2; ++c) {
        for (size_t i = 0; i < boxes.size(); ++i) {
          if (!boxes[i].fused) continue;
          int dv[kKinds];
          default_variants(prec, boxes[i].g, dv);
          boxes[i].var[kFA] = c ? tuned[2 * i] : dv[kFA];
          boxes[i].var[kFC] = c ? tuned[2 * i + 1] : dv[kFC];
        }
        std::vector<Launch> ls;
        std::vector<double> ms;
        sbp_status st = plan_time_groups(p, kReps, ls, ms);
        if (st != SBP_OK) return st;
        for (double m : ms) total[c] += m;
      }
      use_tuned = total[1] < total[0] ? 1 : 0;
      cache[pk] = use_tuned;
      save_cache(path, cache);
      any_measured = true;
    }
    if (!use_tuned) {
      for (auto& b : boxes) {
        if (!b.fused) continue;
        int dv[kKinds];
        default_variants(prec, b.g, dv);
        b.var[kFA] = dv[kFA];
        b.var[kFC] = dv[kFC];
      }
    }
  }
  plan_set_tune_source(p, any_measured ? "measured" : any_cached ? "cache" : "defaults");
  return SBP_OK;
}

}  // namespace sbp
