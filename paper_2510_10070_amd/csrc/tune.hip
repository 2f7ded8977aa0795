// Autotuner: every pass kernel exists in kVariants tile shapes.  For a plan it times each
// variant of each launch group on scratch buffers and keeps the fastest per (pass, transform
// length, padding); results are cached in a text file keyed by GPU architecture and precision
// (SBP_TUNE_CACHE, default $HOME/.cache/sbp_tune.txt) so later plans skip the measurement.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <tuple>

#include "tune.hpp"

namespace sbp {

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
}

namespace {

using Key = std::tuple<std::string, int, int, int, int>;  // arch, prec, kind, len, q

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
  return (kind == kYFwd || kind == kYInv) ? b.g.ny : (kind == kZ ? b.g.m : b.g.nx);
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

  // which (pass, length, padding) keys are missing from the cache
  bool missing = false;
  for (auto& b : boxes)
    for (int k = 0; k < 5; ++k)
      if (!b.fused && !cache.count(Key(arch, prec, k, launch_len(b, k), k == kZ ? b.pad : 0))) missing = true;

  if (missing) {
    // time every variant for all boxes at once, then pick per key
    std::map<Key, std::vector<double>> best;  // key -> time per variant
    for (int v = 0; v < kVariants; ++v) {
      for (auto& b : boxes)
        for (int k = 0; k < 5; ++k) b.var[k] = v;
      std::vector<Launch> ls;
      std::vector<double> ms;
      sbp_status st = plan_time_groups(p, 5, ls, ms);
      if (st != SBP_OK) return st;
      for (size_t i = 0; i < ls.size(); ++i) {
        if (ls[i].kind >= 5) continue;
        auto& slot = best[Key(arch, prec, ls[i].kind, ls[i].len, ls[i].q)];
        slot.resize(kVariants, 0.0);
        slot[v] += ms[i];
      }
    }
    for (auto& kv : best) {
      int arg = 0;
      for (int v = 1; v < kVariants; ++v)
        if (kv.second[v] < kv.second[arg]) arg = v;
      cache[kv.first] = arg;
    }
    save_cache(path, cache);
    plan_set_tune_source(p, "measured");
  } else {
    plan_set_tune_source(p, "cache");
  }
  for (auto& b : boxes) {
    if (b.fused) continue;
    for (int k = 0; k < 5; ++k) b.var[k] = cache[Key(arch, prec, k, launch_len(b, k), k == kZ ? b.pad : 0)];
  }
  return SBP_OK;
}

}  // namespace sbp
