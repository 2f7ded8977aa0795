// Host side of the C ABI: descriptor validation, plan tables, workspace, launch groups, the
// per-solve record copy, HIP-graph capture, kernel timing and the autotuner hooks.  Every entry
// point catches all C++ exceptions and reports through sbp_status plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/sbp.h"
#include "fft_device.hpp"
#include "sbp_internal.hpp"
#include "tune.hpp"
#include "wide.hpp"

namespace {

thread_local std::string g_last_error;

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return sbp::fail(SBP_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

const char* kPassName[8] = {"y_forward", "x_forward", "z_green", "x_inverse", "y_inverse",
                            "fused_a", "fused_b", "fused_c"};

}  // namespace

// Fixed workspace of sbp_solve_static: one array per device, held until the process ends.  In
// host code this name is only a stand-in for the symbol; the device address comes from
// hipGetSymbolAddress (static_scratch_setup) and only that address is ever used.
static __device__ __align__(256) unsigned char scratch[SBP_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};        // device address of `scratch`, per device
bool g_scratch_tried[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Resolve the device address of `scratch` on `device`, once per device; the device must be
// current.  A failure is kept and reported by sbp_solve_static (other entry points still work).
void static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
}

}  // namespace

namespace sbp {

sbp_status fail(sbp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

}  // namespace sbp

using sbp::BoxInfo;
using sbp::fail;
using sbp::Launch;

struct sbp_plan_s {
  int device = 0;
  int prec = 0;  // 0 double, 1 float
  uint32_t flags = 0;
  std::vector<BoxInfo> boxes;
  std::vector<Launch> launches;
  std::vector<int> ints;  // host copy of the group int block
  char* d_tables = nullptr;
  char* d_aux = nullptr;  // records, coefficients, partial sums, group ints
  sbp::BoxRec* d_recs = nullptr;
  sbp::SashaCoef* d_coef = nullptr;
  double* d_partials = nullptr;
  int* d_ints = nullptr;
  size_t nints_cap = 0;
  std::vector<int> blk;     // per-block (box id, tile) pairs of the multi-box launch groups
  int2* d_blk = nullptr;    // device copy (own allocation)
  size_t nblk_cap = 0;      // capacity of d_blk in pairs
  std::vector<sbp::BoxRec> master;  // record templates (plan constants filled in)
  size_t ws_need = 0;
  char* ws = nullptr;
  bool ws_owned = false;
  // pinned staging ring for the per-solve records (h_stage: host view, d_stage: device view)
  sbp::BoxRec* h_stage = nullptr;
  const sbp::BoxRec* d_stage = nullptr;
  int* d_ctl = nullptr;  // graph mode: {next ring slot, finished fetch blocks}
  int nslots = 0, slot = 0;
  size_t nrec = 0;  // records per solve
  std::vector<hipEvent_t> slot_ev;
  std::vector<bool> slot_used;
  // graph mode
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;  // capture happens here; replays go to the caller's stream
  // profiling
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> free_events;
  std::map<std::string, std::pair<long long, double>> totals;
  std::vector<std::string> names;  // stable storage for sbp_profile_read
  std::string describe;
  std::string tune_source = "defaults";
  bool nomix = false;  // autotuning: no merged mixed-Nx groups
};

namespace {

size_t elem_size(int prec) { return prec ? sizeof(float) : sizeof(double); }

sbp_status validate_box(const sbp_box& b, int i, int prec) {
  if (!(b.nx > 0 && b.ny > 0 && b.nz > 0)) return fail(SBP_E_ARG, "box %d: non-positive cell count", i);
  if (!sbp::supported_len(b.nx)) return fail(SBP_E_SIZE, "box %d: nx=%d not a supported length", i, b.nx);
  if (!sbp::supported_len(b.ny)) return fail(SBP_E_SIZE, "box %d: ny=%d not a supported length", i, b.ny);
  if (b.nz < 4 || (b.nz & 1)) return fail(SBP_E_SIZE, "box %d: nz=%d must be even and >= 4", i, b.nz);
  const int pad = b.pad == 0 ? 2 : b.pad;
  if (pad != 2 && pad != 4) return fail(SBP_E_ARG, "box %d: pad=%d not in {2,4}", i, b.pad);
  if (!sbp::supported_len(pad * b.nz))
    return fail(SBP_E_SIZE, "box %d: padded nz=%d not a supported length", i, pad * b.nz);
  if (!(std::isfinite(b.lx) && std::isfinite(b.ly) && std::isfinite(b.lz) && b.lx > 0 && b.ly > 0 && b.lz > 0))
    return fail(SBP_E_ARG, "box %d: box lengths must be finite and > 0", i);
  if (!(std::isfinite(b.alpha)) || b.alpha < 0) return fail(SBP_E_ARG, "box %d: alpha must be >= 0", i);
  if (b.alpha != 0.0 && (b.alpha < 1.0 || b.alpha > 0.5 * pad))
    return fail(SBP_E_ARG,
                "box %d: alpha=%g outside [1, pad/2]: periodic images of the truncated kernel would reach the box",
                i, b.alpha);
  if (b.method != SBP_VGF && b.method != SBP_SASHA) return fail(SBP_E_ARG, "box %d: unknown method %d", i, b.method);
  if (b.remap != SBP_REMAP_SPECTRAL && b.remap != SBP_REMAP_LINEAR)
    return fail(SBP_E_ARG, "box %d: unknown remap %d", i, b.remap);
  const double n = (double)b.nx * b.ny * b.nz;
  if (n * elem_size(prec) > 64.0 * (1ull << 30)) return fail(SBP_E_SIZE, "box %d: grid too large", i);
  return SBP_OK;
}

// exp(-2 pi i m/n) for m < n, from 64-bit-mantissa sin/cos (the angle itself carries a relative
// error near 1e-19), rounded once to the table precision; quarter-turn points are exact
void twiddles(int n, std::vector<long double>& re, std::vector<long double>& im) {
  re.resize(n);
  im.resize(n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int m = 0; m < n; ++m) {
    const long double a = two_pi * (long double)m / (long double)n;
    re[m] = cosl(a);
    im[m] = -sinl(a);
    if (4 * m == n) { re[m] = 0.0L; im[m] = -1.0L; }
    if (2 * m == n) { re[m] = -1.0L; im[m] = 0.0L; }
    if (4 * m == 3 * n) { re[m] = 0.0L; im[m] = 1.0L; }
    if (m == 0) { re[m] = 1.0L; im[m] = 0.0L; }
  }
}

// stage-major table of schedule RL (the layout the transform kernels read, see TwS): stage s
// (ns = product of the earlier radices, radix R) holds exp(-2 pi i k r/(ns R)) at
// ns - 1 + (r - 1) ns + k; n slots, the last one unused
template <class RL>
void stage_major(int n, const std::vector<long double>& re, const std::vector<long double>& im,
                 std::vector<long double>& ore, std::vector<long double>& oim) {
  ore.assign(n, 0.0L);
  oim.assign(n, 0.0L);
  int ns = 1;
  for (int s = 0; s < RL::n; ++s) {
    const int R = RL::r[s];
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < ns; ++k) {
        const int m = k * r * (n / (ns * R));
        ore[ns - 1 + (r - 1) * ns + k] = re[m];
        oim[ns - 1 + (r - 1) * ns + k] = im[m];
      }
    ns *= R;
  }
}

// the forward schedule's table of length n, then the inverse schedule's (z: the schedules of the
// padded z transforms, ZSched)
bool stage_major_pair(int n, bool z, const std::vector<long double>& re, const std::vector<long double>& im,
                      std::vector<long double>& ore, std::vector<long double>& oim) {
  std::vector<long double> fr, fi, ir, ii;
  bool ok = false;
#define SBP_CASE(N_)                                                 \
  if (n == N_) {                                                     \
    if (z) {                                                         \
      stage_major<typename sbp::ZSched<N_>::F>(n, re, im, fr, fi);   \
      stage_major<typename sbp::ZSched<N_>::I>(n, re, im, ir, ii);   \
    } else {                                                         \
      stage_major<typename sbp::Fwd<N_>::L>(n, re, im, fr, fi);      \
      stage_major<typename sbp::Inv<N_>::L>(n, re, im, ir, ii);      \
    }                                                                \
    ok = true;                                                       \
  }
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  if (!ok) return false;
  ore = fr;
  oim = fi;
  ore.insert(ore.end(), ir.begin(), ir.end());
  oim.insert(oim.end(), ii.begin(), ii.end());
  return true;
}

struct TableBuilder {
  std::vector<char> host;
  std::map<std::pair<int, int>, size_t> tw;  // (n, prec) -> offset
  std::map<std::tuple<int, int, bool>, size_t> tws;  // (n, prec, z) -> offset of the stage-major pair
  size_t put(const void* p, size_t bytes) {
    size_t off = align_up(host.size());
    host.resize(off + bytes);
    memcpy(host.data() + off, p, bytes);
    return off;
  }
  size_t twiddle(int n, int prec) {
    auto key = std::make_pair(n, prec);
    auto it = tw.find(key);
    if (it != tw.end()) return it->second;
    std::vector<long double> re, im;
    twiddles(n, re, im);
    size_t off;
    if (prec) {
      std::vector<float> v(2 * n);
      for (int m = 0; m < n; ++m) { v[2 * m] = (float)re[m]; v[2 * m + 1] = (float)im[m]; }
      off = put(v.data(), v.size() * sizeof(float));
    } else {
      std::vector<double> v(2 * n);
      for (int m = 0; m < n; ++m) { v[2 * m] = (double)re[m]; v[2 * m + 1] = (double)im[m]; }
      off = put(v.data(), v.size() * sizeof(double));
    }
    tw[key] = off;
    return off;
  }
  template <typename T> size_t put_cplx(const std::vector<long double>& re, const std::vector<long double>& im) {
    std::vector<T> v(2 * re.size());
    for (size_t m = 0; m < re.size(); ++m) {
      v[2 * m] = (T)re[m];
      v[2 * m + 1] = (T)im[m];
    }
    return put(v.data(), v.size() * sizeof(T));
  }
  // stage-major twiddles of length n: 2n entries, forward schedule then inverse schedule (z: the
  // schedules of the padded z transforms)
  size_t stage_twiddles(int n, int prec, bool z = false) {
    auto key = std::make_tuple(n, prec, z);
    auto it = tws.find(key);
    if (it != tws.end()) return it->second;
    std::vector<long double> re, im, sre, sim;
    twiddles(n, re, im);
    stage_major_pair(n, z, re, im, sre, sim);  // n is a validated length
    const size_t off = prec ? put_cplx<float>(sre, sim) : put_cplx<double>(sre, sim);
    tws[key] = off;
    return off;
  }
};

// per-kz tables: 1 - cos(kz L), kz sin(kz L), kz^2, for kz = 2 pi ms/(P Lz)
void ztables(const sbp::BoxGeom& g, int pad, std::vector<long double>& s2, std::vector<long double>& ks,
             std::vector<long double>& kz2) {
  const int M = g.m;
  s2.resize(M);
  ks.resize(M);
  kz2.resize(M);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int mz = 0; mz < M; ++mz) {
    const int ms = mz < M / 2 ? mz : mz - M;
    const long double kz = two_pi * (long double)ms / ((long double)pad * (long double)g.lz);
    const long double th = kz * (long double)g.L;
    const long double h = sinl(0.5L * th);
    s2[mz] = 2.0L * h * h;
    ks[mz] = kz * sinl(th);
    kz2[mz] = kz * kz;
  }
}

template <typename T>
size_t put_vec(TableBuilder& tb, const std::vector<long double>& v) {
  std::vector<T> t(v.size());
  for (size_t i = 0; i < v.size(); ++i) t[i] = (T)v[i];
  return tb.put(t.data(), t.size() * sizeof(T));
}

void ev_get(sbp_plan p, hipEvent_t* e) {
  if (!p->free_events.empty()) {
    *e = p->free_events.back();
    p->free_events.pop_back();
  } else {
    hipEventCreate(e);
  }
}

struct Marker {
  sbp_plan p;
  hipStream_t st;
  hipEvent_t last = nullptr;
  const char* name = nullptr;
  void mark(const char* next) {
    if (!p->prof) return;
    hipEvent_t e;
    ev_get(p, &e);
    hipEventRecord(e, st);
    if (last) p->pending.push_back({name, last, e});
    if (next) {
      last = e;
      name = next;
    } else {
      last = nullptr;
    }
  }
};

void mark_cb(void* ctx, const char* name) { static_cast<Marker*>(ctx)->mark(name); }

int tiles_of(int prec, int kind, const sbp::BoxGeom& g, int variant) {
  switch (kind) {
    case sbp::kYFwd:
    case sbp::kYInv: return sbp::y_tiles(prec, g, variant);
    case sbp::kXFwd:
    case sbp::kXInv: return sbp::x_tiles(prec, g, variant);
    case sbp::kZ: return sbp::z_tiles(prec, g, variant);
    case sbp::kFA:
    case sbp::kFC: return sbp::fused_ac_tiles(prec, g, variant);
    default: return sbp::fused_b_tiles(g);
  }
}

// transform length a launch of this kind is specialised on
int kind_len(const BoxInfo& bi, int kind) {
  switch (kind) {
    case sbp::kYFwd:
    case sbp::kYInv:
    case sbp::kFA:
    case sbp::kFC: return bi.g.ny;
    case sbp::kZ:
    case sbp::kFB: return bi.g.m;
    default: return bi.g.nx;
  }
}

bool kind_applies(const BoxInfo& bi, int kind) { return bi.fused ? kind >= sbp::kFA : kind < sbp::kFA; }

// group boxes by kernel shape for each pass, in pass order
void build_launches(sbp_plan p) {
  p->launches.clear();
  p->ints.clear();
  p->blk.clear();
  const int nb = (int)p->boxes.size();
  for (int phase = 0; phase < 5; ++phase)
  for (int kind = 0; kind < sbp::kKinds; ++kind) {
    if (sbp::kPhase[kind] != phase) continue;
    // group key: transform length, tile variant, padding (z kinds), A (fused kinds), linear
    // remap (fused passes A and C)
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> groups;
    for (int b = 0; b < nb; ++b) {
      const BoxInfo& bi = p->boxes[b];
      if (!kind_applies(bi, kind)) continue;
      const int q = (kind == sbp::kZ || kind == sbp::kFB) ? bi.pad : 0;
      // pass B reads A = Nx/16 from each box's record, so its groups mix A
      const int a = (kind == sbp::kFA || kind == sbp::kFC) ? sbp::fused_a(bi.g) : 0;
      const int lin = (kind == sbp::kFA || kind == sbp::kFC) && bi.g.remap == SBP_REMAP_LINEAR;
      groups[std::make_tuple(kind_len(bi, kind), bi.var[kind], q, a, lin)].push_back(b);
    }
    if ((kind == sbp::kFA || kind == sbp::kFC) && p->prec == SBP_FP32 && !p->nomix) {
      // float passes A and C in 64-byte rows (A <= 8): groups that differ only in A share one
      // launch (k_fa_mix / k_fc_mix, a = 0), rather than one small launch each
      std::map<std::tuple<int, int, int, int>, std::vector<std::tuple<int, int, int, int, int>>> same;
      for (auto& kv : groups) {
        const auto& [len, var, q, a, lin] = kv.first;
        if (var == 1 && a >= 1 && a <= 8) same[std::make_tuple(len, var, q, lin)].push_back(kv.first);
      }
      for (auto& sv : same) {
        if (sv.second.size() < 2) continue;
        const auto& [len, var, q, lin] = sv.first;
        std::vector<int>& merged = groups[std::make_tuple(len, var, q, 0, lin)];
        for (const auto& key : sv.second) {
          merged.insert(merged.end(), groups[key].begin(), groups[key].end());
          groups.erase(key);
        }
        std::sort(merged.begin(), merged.end());
      }
      // and groups of 64-byte rows that differ in Ny <= 128 as well: one launch (len = 0) for all
      std::map<int, std::vector<std::tuple<int, int, int, int, int>>> multi;  // lin -> group keys
      for (auto& kv : groups) {
        const auto& [len, var, q, a, lin] = kv.first;
        if (var == 1 && len > 0 && len <= 128 && a <= 8) multi[lin].push_back(kv.first);
      }
      for (auto& mv : multi) {
        if (mv.second.size() < 2) continue;
        std::vector<int>& merged = groups[std::make_tuple(0, 1, 0, 0, mv.first)];
        for (const auto& key : mv.second) {
          merged.insert(merged.end(), groups[key].begin(), groups[key].end());
          groups.erase(key);
        }
        std::sort(merged.begin(), merged.end());
      }
    }
    if (kind == sbp::kFB && p->prec == SBP_FP32 && !p->nomix) {
      // float pass B with padding 2 and M <= 256: groups of different M share one launch
      // (k_fb_multi, len = 0), rather than one launch each whose blocks all start together
      std::vector<std::tuple<int, int, int, int, int>> keys;
      for (auto& kv : groups) {
        const auto& [len, var, q, a, lin] = kv.first;
        bool ok = len > 0;
        for (int b : kv.second) ok = ok && sbp::fused_b_items_per_block(p->boxes[b].g, p->boxes[b].pad) > 0;
        if (ok) keys.push_back(kv.first);
      }
      if (keys.size() >= 2) {
        std::vector<int>& merged = groups[std::make_tuple(0, 0, 2, 0, 0)];
        for (const auto& key : keys) {
          merged.insert(merged.end(), groups[key].begin(), groups[key].end());
          groups.erase(key);
        }
        std::sort(merged.begin(), merged.end());
      }
    }
    for (auto& kv : groups) {
      Launch l;
      l.kind = kind;
      int lin = 0;
      std::tie(l.len, l.variant, l.q, l.a, lin) = kv.first;
      l.lin = lin != 0;
      l.n = (int)kv.second.size();
      l.ints_off = p->ints.size();
      for (int b : kv.second) p->ints.push_back(b);
      int acc = 0;
      p->ints.push_back(0);
      for (int b : kv.second) {
        const sbp::BoxGeom& g = p->boxes[b].g;
        int nt;
        if (kind == sbp::kFB && l.len == 0)  // a block takes items_per_block items of its box
          nt = sbp::fused_b_tiles(g) / sbp::fused_b_items_per_block(g, p->boxes[b].pad);
        else if ((kind == sbp::kFA || kind == sbp::kFC) && l.len == 0)  // rows by Ny
          nt = sbp::fused_ac_multi_tiles(g);
        else
          nt = tiles_of(p->prec, kind, g, l.variant);
        // each tile of the first pass writes one SASHA partial-sum pair
        if (kind == sbp::kFA || kind == sbp::kYFwd) p->boxes[b].first_tiles = nt;
        acc += nt;
        p->ints.push_back(acc);
      }
      l.blocks = acc;
      if (l.n > 1) {
        // (box id, tile) of every block, so that a block finds its box with one load.  Pass B
        // lists tile 0 of every box first: in float that block also convolves the k = 0 pencil
        // in double, the longest block of the launch, so it should not start last.
        l.blk_off = p->blk.size() / 2;
        const int first = kind == sbp::kFB ? 1 : 0;
        for (int i = 0; i < l.n && first; ++i) {
          p->blk.push_back(kv.second[i]);
          p->blk.push_back(0);
        }
        for (int i = 0; i < l.n; ++i) {
          const int nt = p->ints[l.ints_off + l.n + i + 1] - p->ints[l.ints_off + l.n + i];
          for (int t = first; t < nt; ++t) {
            p->blk.push_back(kv.second[i]);
            p->blk.push_back(t);
          }
        }
      }
      const BoxInfo& b0 = p->boxes[kv.second[0]];
      switch (kind) {
        case sbp::kYFwd:
        case sbp::kYInv: l.tw = b0.tws_y; break;
        case sbp::kZ: l.tw = b0.tws_m; l.tw64 = b0.tw_m64; break;
        case sbp::kFA:
        case sbp::kFC: l.tw = b0.tws_y; l.tw64 = b0.tw_x; break;
        case sbp::kFB: l.tw = b0.tws_m; l.tw64 = b0.tw_m64; break;
        default: l.tw = b0.tws_x;
      }
      p->launches.push_back(l);
    }
  }
}

// arg: the solve's record for a one-box group that is the solve's first launch (direct launches),
// handed to the kernel with the launch
hipError_t launch_one(sbp_plan p, const Launch& l, hipStream_t st, const sbp::BoxRec* arg = nullptr) {
  const char* T = p->d_tables;
  sbp::GroupArgs ga{p->d_ints + l.ints_off, p->d_ints + l.ints_off + l.n, l.n, l.blocks, p->ints[l.ints_off],
                    l.n > 1 ? p->d_blk + l.blk_off : nullptr};
  if (arg) {
    ga.use_arg = 1;
    ga.pub = p->d_recs + ga.box0;
    ga.arg = *arg;
  }
  switch (l.kind) {
    case sbp::kYFwd:
      return sbp::launch_y(p->prec, true, true, l.len, l.variant, ga, l.blocks, p->d_recs, T + l.tw, st);
    case sbp::kYInv:
      return sbp::launch_y(p->prec, false, true, l.len, l.variant, ga, l.blocks, p->d_recs, T + l.tw, st);
    case sbp::kXFwd:
    case sbp::kXInv:
      return sbp::launch_x(p->prec, l.kind == sbp::kXFwd ? -1 : +1, l.len, l.variant, ga, l.blocks, p->d_recs,
                           T + l.tw, st);
    case sbp::kZ:
      return sbp::launch_z(p->prec, l.len, l.variant, l.q, ga, l.blocks, p->d_recs, T + l.tw, T + l.tw64, st);
    default:
      return sbp::launch_fused(p->prec, l.kind - sbp::kFA, l.len, l.a, l.variant, l.q, l.lin, ga, l.blocks, p->d_recs,
                               T + l.tw, T + l.tw64, st);
  }
}

// launch one solve: the record fetch, then the passes.  Records come from `arg_recs` (host
// memory, passed as kernel arguments) when given, else from ring slot fetch_slot, or, when
// fetch_slot < 0, from the slot named by the device-side ring counter (graph capture).
sbp_status enqueue(sbp_plan p, hipStream_t st, Marker* mk, int fetch_slot, const sbp::BoxRec* arg_recs = nullptr) {
  const char* T = p->d_tables;
  // a one-box plan whose first launch is its box's first pass (fused pass A or the forward y
  // pass) hands the record to that launch
  const bool inline_rec = arg_recs && !(p->flags & SBP_FLAG_PLAIN) && p->nrec == 1 && !p->launches.empty() &&
                          (p->launches[0].kind == sbp::kFA || p->launches[0].kind == sbp::kYFwd) &&
                          p->launches[0].n == 1;
  if (!inline_rec) {
    if (mk) mk->mark("records");
    if (arg_recs)
      HIP_TRY(sbp::launch_fetch_args(arg_recs, p->d_recs, (int)p->nrec, st));
    else
      HIP_TRY(sbp::launch_fetch(p->d_stage, p->d_recs, (int)p->nrec, p->nslots, fetch_slot, p->d_ctl, st));
  }
  if (p->flags & SBP_FLAG_PLAIN) {
    const BoxInfo& bi = p->boxes[0];
    sbp::GroupArgs one{p->d_ints, p->d_ints + 1, 1, 0, 0, nullptr};
    HIP_TRY(sbp::launch_plain(&p->master[0], p->d_recs, p->d_recs + 1, one, bi.var[sbp::kYFwd], bi.var[sbp::kXFwd],
                              T + bi.tws_x, T + bi.tws_y, T + bi.tw_m, st, mk ? mark_cb : nullptr, mk));
    return SBP_OK;
  }
  for (size_t i = 0; i < p->launches.size(); ++i) {
    const Launch& l = p->launches[i];
    if (mk) mk->mark(kPassName[l.kind]);  // kinds stay distinct in the timing records
    HIP_TRY(launch_one(p, l, st, (i == 0 && inline_rec) ? arg_recs : nullptr));
  }
  if (mk) mk->mark(nullptr);
  return SBP_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

void destroy_graph(sbp_plan p) {
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
}

// workspace pointers in the record templates, for the workspace at `ws`
void bind_workspace(sbp_plan p, char* ws) {
  if (p->flags & SBP_FLAG_PLAIN) {
    p->master[0].W = ws + p->boxes[0].ws2_off;
    p->master[1].W = ws + p->boxes[0].ws_off;
    return;
  }
  for (size_t b = 0; b < p->boxes.size(); ++b) p->master[b].W = ws + p->boxes[b].ws_off;
}
void bind_workspace(sbp_plan p) { bind_workspace(p, p->ws); }

// the records of one solve: the plan's templates with the per-solve fields filled in
void fill_records(sbp_plan p, const void* const* rho, void* const* phi, const sbp_shear* params, sbp::BoxRec* hs) {
  for (size_t r = 0; r < p->nrec; ++r) {
    const size_t b = (p->flags & SBP_FLAG_PLAIN) ? 0 : r;
    hs[r] = p->master[r];
    const sbp::BoxGeom& g = p->boxes[b].g;
    const sbp_shear& s = params[b];
    double d = std::fmod(s.q * s.omega * g.lx * s.t, g.ly);
    if (d < 0.0) d += g.ly;
    if (d >= g.ly) d = 0.0;
    hs[r].rho = rho[b];
    hs[r].phi = phi[b];
    hs[r].s = d / g.lx;
    hs[r].fy = g.remap == SBP_REMAP_LINEAR ? 0.0 : (d / g.ly) / (2.0 * g.nx);
    hs[r].shy = (d / g.lx) * (g.lx / g.nx) / (g.ly / g.ny);
    hs[r].fourpiG = 4.0 * M_PI * s.G;
    hs[r].scale = hs[r].fourpiG / ((double)g.nx * g.ny * g.m);
  }
}

// fill the next ring slot with the records of one solve (the fetch kernel copies it to the
// device); waits only if that slot's previous solve has not yet been fetched
sbp_status stage_records(sbp_plan p, const void* const* rho, void* const* phi, const sbp_shear* params, int* slot_out) {
  const int slot = p->slot;
  if (p->slot_used[slot]) HIP_TRY(hipEventSynchronize(p->slot_ev[slot]));
  fill_records(p, rho, phi, params, p->h_stage + (size_t)slot * p->nrec);
  *slot_out = slot;
  return SBP_OK;
}

// after the solve using `slot` is enqueued: advance the ring and mark the slot in flight
sbp_status commit_slot(sbp_plan p, int slot, hipStream_t st) {
  p->slot = (slot + 1) % p->nslots;
  HIP_TRY(hipEventRecord(p->slot_ev[slot], st));
  p->slot_used[slot] = true;
  return SBP_OK;
}

std::string describe_plan(sbp_plan p) {
  std::string s = "{\"path\":\"";
  bool any_fused = false, any_five = false;
  for (const BoxInfo& b : p->boxes) (b.fused ? any_fused : any_five) = true;
  s += (p->flags & SBP_FLAG_PLAIN) ? "plain" : (any_fused ? (any_five ? "mixed" : "fused-3pass") : "streaming-5pass");
  s += "\",\"precision\":\"";
  s += p->prec ? "fp32" : "fp64";
  // modelled HBM bytes of one solve (data arrays only): each pass reads and writes N w bytes, three
  // passes fused, five streaming; the plain path's eleven steps touch the padded spectrum (P N w)
  // in six of them: 12 + 10 P
  double model = 0.0;
  for (const BoxInfo& b : p->boxes) {
    const double nw = (double)b.g.nx * b.g.ny * b.g.nz * elem_size(p->prec);
    model += nw * ((p->flags & SBP_FLAG_PLAIN) ? 12.0 + 10.0 * b.pad : b.fused ? 6.0 : 10.0);
  }
  char buf[400];
  snprintf(buf, sizeof buf,
           "\",\"nbox\":%zu,\"launches\":%zu,\"graph\":%s,\"workspace_bytes\":%zu,\"tuning\":\"%s\","
           "\"bytes_model\":%.0f",
           p->boxes.size(), (p->flags & SBP_FLAG_PLAIN) ? (size_t)13 : p->launches.size(),
           (p->flags & SBP_FLAG_GRAPH) ? "true" : "false", p->ws_need, p->tune_source.c_str(), model);
  s += buf;
  s += ",\"groups\":[";
  for (size_t i = 0; i < p->launches.size(); ++i) {
    const Launch& l = p->launches[i];
    const BoxInfo& b0 = p->boxes[p->ints[l.ints_off]];
    snprintf(buf, sizeof buf,
             "%s{\"pass\":\"%s\",\"len\":%d,\"variant\":%d,\"tuned\":\"%s\",\"boxes\":%d,\"blocks\":%d}",
             i ? "," : "", kPassName[l.kind], l.len, l.variant, sbp::kVarSrcName[b0.var_src[l.kind]], l.n, l.blocks);
    s += buf;
  }
  s += "]}";
  return s;
}

sbp_status upload_groups(sbp_plan p) {
  build_launches(p);
  if (p->ints.size() > p->nints_cap) return fail(SBP_E_STATE, "group table overflow");
  HIP_TRY(hipMemcpy(p->d_ints, p->ints.data(), p->ints.size() * sizeof(int), hipMemcpyHostToDevice));
  // the per-block table (multi-box groups) grows with the tile variants the autotuner tries;
  // it is only rebuilt while the plan is being created, before any solve uses it
  if (p->blk.size() / 2 > p->nblk_cap) {
    if (p->d_blk) HIP_TRY(hipFree(p->d_blk));
    p->d_blk = nullptr;
    p->nblk_cap = 0;
    if (hipMalloc(&p->d_blk, p->blk.size() * sizeof(int)) != hipSuccess)
      return fail(SBP_E_NOMEM, "block table allocation (%zu bytes)", p->blk.size() * sizeof(int));
    p->nblk_cap = p->blk.size() / 2;
  }
  if (!p->blk.empty())
    HIP_TRY(hipMemcpy(p->d_blk, p->blk.data(), p->blk.size() * sizeof(int), hipMemcpyHostToDevice));
  p->describe = describe_plan(p);
  return SBP_OK;
}

}  // namespace

// --- plan access for the autotuner -------------------------------------------------------
namespace sbp {

int plan_prec(sbp_plan p) { return p->prec; }
int plan_device(sbp_plan p) { return p->device; }
std::vector<BoxInfo>& plan_boxes(sbp_plan p) { return p->boxes; }
void plan_set_tune_source(sbp_plan p, const std::string& s) { p->tune_source = s; }
void plan_set_nomix(sbp_plan p, bool on) { p->nomix = on; }
int plan_group_box(sbp_plan p, const Launch& l) { return p->ints[l.ints_off]; }

// Time every launch group of the current variant assignment (reps solves after one warm-up) on
// scratch buffers.  ms[i] is the mean time of launches()[i].
sbp_status plan_time_groups(sbp_plan p, int reps, std::vector<Launch>& launches, std::vector<double>& ms) {
  sbp_status us = upload_groups(p);
  if (us != SBP_OK) return us;
  std::vector<void*> bufs;
  std::vector<const void*> rho;
  std::vector<void*> phi;
  std::vector<sbp_shear> sh;
  auto release = [&]() {
    for (void* b : bufs) hipFree(b);
    bufs.clear();
  };
  for (const BoxInfo& bi : p->boxes) {
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bi.data_bytes) != hipSuccess) {
      release();
      return fail(SBP_E_NOMEM, "autotune scratch allocation");
    }
    bufs.push_back(a);
    if (hipMalloc(&b, bi.data_bytes) != hipSuccess) {
      release();
      return fail(SBP_E_NOMEM, "autotune scratch allocation");
    }
    bufs.push_back(b);
    hipMemset(a, 0, bi.data_bytes);
    rho.push_back(a);
    phi.push_back(b);
    sh.push_back(sbp_shear{1.5, 1.0, 0.3, 1.0});
  }
  void* tws = nullptr;
  if (hipMalloc(&tws, std::max<size_t>(p->ws_need, 256)) != hipSuccess) {
    release();
    return fail(SBP_E_NOMEM, "autotune workspace allocation");
  }
  bufs.push_back(tws);
  char* saved_ws = p->ws;
  p->ws = (char*)tws;
  bind_workspace(p);
  hipStream_t st = nullptr;
  sbp_status res = SBP_OK;
  std::vector<double> acc(p->launches.size(), 0.0);
  std::vector<hipEvent_t> ev(p->launches.size() + 1);
  for (auto& e : ev) hipEventCreate(&e);
  for (int r = 0; r <= reps && res == SBP_OK; ++r) {
    int slot = 0;
    res = stage_records(p, rho.data(), phi.data(), sh.data(), &slot);
    if (res != SBP_OK) break;
    if (hipError_t e = sbp::launch_fetch(p->d_stage, p->d_recs, (int)p->nrec, p->nslots, slot, p->d_ctl, st);
        e != hipSuccess) {
      res = fail(SBP_E_HIP, "autotune record fetch: %s", hipGetErrorString(e));
      break;
    }
    res = commit_slot(p, slot, st);
    if (res != SBP_OK) break;
    hipEventRecord(ev[0], st);
    for (size_t i = 0; i < p->launches.size(); ++i) {
      hipError_t e = launch_one(p, p->launches[i], st);
      if (e != hipSuccess) {
        res = fail(SBP_E_HIP, "autotune launch: %s", hipGetErrorString(e));
        break;
      }
      hipEventRecord(ev[i + 1], st);
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
      res = fail(SBP_E_HIP, "autotune synchronise");
      break;
    }
    for (size_t i = 0; r > 0 && i < p->launches.size(); ++i) {
      float t = 0.f;
      hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      acc[i] += t;
    }
  }
  for (auto& e : ev) hipEventDestroy(e);
  p->ws = saved_ws;
  if (p->ws) bind_workspace(p);
  release();
  if (res != SBP_OK) return res;
  launches = p->launches;
  ms.assign(acc.size(), 0.0);
  for (size_t i = 0; i < acc.size(); ++i) ms[i] = acc[i] / reps;
  return SBP_OK;
}

}  // namespace sbp

extern "C" {

const char* sbp_status_str(sbp_status s) {
  switch (s) {
    case SBP_OK: return "ok";
    case SBP_E_ARG: return "invalid argument";
    case SBP_E_SIZE: return "unsupported grid size";
    case SBP_E_NOMEM: return "out of memory";
    case SBP_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case SBP_E_HIP: return "HIP runtime error";
    case SBP_E_STATE: return "invalid plan state";
  }
  return "unknown status";
}

const char* sbp_last_error(void) { return g_last_error.c_str(); }

sbp_status sbp_plan_create(const sbp_box* boxes, int32_t nbox, int32_t precision, int32_t device, uint32_t flags,
                           sbp_plan* out) {
  try {
    if (!out) return fail(SBP_E_ARG, "out is NULL");
    *out = nullptr;
    g_last_error.clear();
    if (!boxes) return fail(SBP_E_ARG, "boxes is NULL");
    if (nbox < 1 || nbox > 4096) return fail(SBP_E_ARG, "nbox=%d outside [1, 4096]", nbox);
    if (precision != SBP_FP64 && precision != SBP_FP32) return fail(SBP_E_ARG, "unknown precision %d", precision);
    if (flags & ~(SBP_FLAG_GRAPH | SBP_FLAG_AUTOTUNE | SBP_FLAG_PLAIN | SBP_FLAG_FIVE_PASS | SBP_FLAG_FUSED))
      return fail(SBP_E_ARG, "unknown flags 0x%x", flags);
    if ((flags & SBP_FLAG_FIVE_PASS) && (flags & SBP_FLAG_FUSED))
      return fail(SBP_E_ARG, "SBP_FLAG_FIVE_PASS and SBP_FLAG_FUSED are exclusive");
    if ((flags & SBP_FLAG_PLAIN) && (precision != SBP_FP64 || nbox != 1 || (flags & (SBP_FLAG_FIVE_PASS | SBP_FLAG_FUSED))))
      return fail(SBP_E_ARG, "the plain path is FP64, single-box and takes no schedule flag");
    if ((flags & SBP_FLAG_PLAIN) && boxes[0].remap != SBP_REMAP_SPECTRAL)
      return fail(SBP_E_ARG, "the plain path implements the spectral remap only");
    if (device < 0) return fail(SBP_E_ARG, "device=%d", device);
    const int prec = precision == SBP_FP32 ? 1 : 0;
    for (int i = 0; i < nbox; ++i) {
      sbp_status st = validate_box(boxes[i], i, prec);
      if (st != SBP_OK) return st;
    }
    // --- descriptors valid: from here on HIP is used
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev)
      return fail(SBP_E_HIP, "device %d not available (%d visible)", device, ndev);
    std::unique_ptr<sbp_plan_s> p(new sbp_plan_s);
    p->device = device;
    p->prec = prec;
    p->flags = flags;
    HIP_TRY(hipSetDevice(device));
    static_scratch_setup(device);

    TableBuilder tb;
    size_t ws = 0, npart = 0;
    const size_t w = elem_size(prec);
    for (int i = 0; i < nbox; ++i) {
      const sbp_box& b = boxes[i];
      BoxInfo bi;
      const int pad = b.pad == 0 ? 2 : b.pad;
      const double alpha = b.alpha == 0.0 ? 0.5 * pad : b.alpha;
      bi.pad = pad;
      bi.g = sbp::BoxGeom{b.nx, b.ny, b.nz, pad * b.nz, b.method, b.remap, b.lx, b.ly, b.lz, alpha * b.lz};
      bi.tw_x = tb.twiddle(b.nx, prec);
      bi.tw_m = tb.twiddle(pad * b.nz, prec);
      bi.tw_m64 = tb.twiddle(pad * b.nz, 0);
      bi.tws_x = tb.stage_twiddles(b.nx, prec);
      bi.tws_y = tb.stage_twiddles(b.ny, prec);
      bi.tws_m = tb.stage_twiddles(pad * b.nz, prec, true);
      std::vector<long double> s2, ks, kz2;
      ztables(bi.g, pad, s2, ks, kz2);
      bi.zt64[0] = put_vec<double>(tb, s2);
      bi.zt64[1] = put_vec<double>(tb, ks);
      bi.zt64[2] = put_vec<double>(tb, kz2);
      std::vector<long double> rows(4 * s2.size(), 0.0L);
      for (size_t i = 0; i < s2.size(); ++i) {
        rows[4 * i] = s2[i];
        rows[4 * i + 1] = ks[i];
        rows[4 * i + 2] = kz2[i];
      }
      bi.zt = prec ? put_vec<float>(tb, rows) : put_vec<double>(tb, rows);
      {
        // the k = 0 Green's function does not depend on t: its real-space form on the padded
        // grid, h[n] = sum_m G(0, kz_m) cos(2 pi m n / M), turns the k = 0 pencil into a short
        // convolution (float plans evaluate it in double)
        const int M = bi.g.m;
        const long double L = (long double)bi.g.L;
        std::vector<long double> gk(M), h(M, 0.0L);
        for (int m = 0; m < M; ++m) {
          if (b.method == SBP_SASHA)
            gk[m] = m == 0 ? 0.0L : -1.0L / kz2[m];
          else
            gk[m] = m == 0 ? 0.5L * L * L : (L * ks[m] - s2[m]) / kz2[m];
        }
        const long double two_pi = 6.283185307179586476925286766559005768L;
        for (int n = 0; n < M; ++n) {
          long double acc = 0.0L;
          for (int m = 0; m < M; ++m) acc += gk[m] * cosl(two_pi * (long double)(((long long)m * n) % M) / M);
          h[n] = acc;
        }
        bi.k0h = put_vec<double>(tb, h);
      }
      sbp::default_variants(prec, bi.g, bi.var);
      const bool want_fused = (flags & SBP_FLAG_FUSED) || !(flags & (SBP_FLAG_PLAIN | SBP_FLAG_FIVE_PASS));
      // the wide float boxes run fused on request only: five-pass is faster there (the wide passes
      // A and C stream 8- or 16-byte z rows with one block per CU)
      bi.fused = want_fused && (sbp::fused_ok(bi.g) || ((flags & SBP_FLAG_FUSED) && sbp::fused_wide_ok(prec, bi.g)));
      const size_t n = (size_t)b.nx * b.ny * b.nz;
      bi.data_bytes = n * w;
      if (flags & SBP_FLAG_PLAIN) {
        bi.ws_off = ws;
        ws = align_up(ws + (size_t)b.nx * (b.ny / 2) * bi.g.m * 2 * sizeof(double));
        bi.ws2_off = ws;
        ws = align_up(ws + n * sizeof(double));
        bi.npartials = sbp::kPlainPartials;
      } else {
        bi.ws_off = ws;
        ws = align_up(ws + n * w);  // nx * (ny/2) * nz complex
        // one partial-sum pair per tile of the first pass, for every tile variant the plan or
        // the autotuner may pick (each pass-A/y tile writes its own slot)
        int most = 0;
        for (int v = 0; v < sbp::kVariants; ++v) {
          most = std::max(most, sbp::y_tiles(prec, bi.g, v));
          most = std::max(most, sbp::fused_ac_tiles(prec, bi.g, v));
        }
        most = std::max(most, sbp::fused_ac_tiles(prec, bi.g, 2));
        most = std::max(most, sbp::fused_ac_tiles(prec, bi.g, 3));
        bi.npartials = most;
      }
      bi.part_off = npart;
      npart += 2 * (size_t)bi.npartials;
      p->boxes.push_back(bi);
    }
    p->ws_need = ws;
    p->nrec = (flags & SBP_FLAG_PLAIN) ? 2 : (size_t)nbox;

    void* d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(tb.host.size(), 256)) != hipSuccess)
      return fail(SBP_E_NOMEM, "table allocation (%zu bytes)", tb.host.size());
    p->d_tables = (char*)d;
    HIP_TRY(hipMemcpy(p->d_tables, tb.host.data(), tb.host.size(), hipMemcpyHostToDevice));

    // group ints: per pass at most nbox groups; each box appears once per pass with 2 ints,
    // plus one leading start per group
    p->nints_cap = 8 * (3 * (size_t)nbox) + 8;
    const size_t aux = align_up(2 * sizeof(int)) + align_up(p->nrec * sizeof(sbp::BoxRec)) +
                       align_up(nbox * sizeof(sbp::SashaCoef)) +
                       align_up(std::max<size_t>(npart, 2) * sizeof(double)) + align_up(p->nints_cap * sizeof(int));
    if (hipMalloc(&d, aux) != hipSuccess) return fail(SBP_E_NOMEM, "aux allocation (%zu bytes)", aux);
    p->d_aux = (char*)d;
    char* cur = p->d_aux;
    p->d_ctl = (int*)cur;
    cur += align_up(2 * sizeof(int));
    {
      const int zero[2] = {0, 0};
      HIP_TRY(hipMemcpy(p->d_ctl, zero, sizeof zero, hipMemcpyHostToDevice));
    }
    p->d_recs = (sbp::BoxRec*)cur;
    cur += align_up(p->nrec * sizeof(sbp::BoxRec));
    p->d_coef = (sbp::SashaCoef*)cur;
    cur += align_up(nbox * sizeof(sbp::SashaCoef));
    p->d_partials = (double*)cur;
    cur += align_up(std::max<size_t>(npart, 2) * sizeof(double));
    p->d_ints = (int*)cur;

    // record templates
    p->master.resize(p->nrec);
    for (size_t r = 0; r < p->nrec; ++r) {
      const size_t b = (flags & SBP_FLAG_PLAIN) ? 0 : r;
      const BoxInfo& bi = p->boxes[b];
      sbp::BoxRec& rec = p->master[r];
      memset(&rec, 0, sizeof rec);
      rec.g = bi.g;
      rec.partials = p->d_partials + bi.part_off;
      rec.npartials = 0;
      rec.coef = p->d_coef + b;
      rec.zt = p->d_tables + bi.zt;
      rec.k0h = (const double*)(p->d_tables + bi.k0h);
      rec.twx = p->d_tables + bi.tw_x;
      rec.twy = p->d_tables + bi.tws_y;
      rec.twz = p->d_tables + bi.tws_m;
      for (int k = 0; k < 3; ++k) rec.zt64[k] = (const double*)(p->d_tables + bi.zt64[k]);
    }

    p->nslots = 64;
    void* h = nullptr;
    if (hipHostMalloc(&h, (size_t)p->nslots * p->nrec * sizeof(sbp::BoxRec), hipHostMallocDefault) != hipSuccess)
      return fail(SBP_E_NOMEM, "pinned staging allocation");
    p->h_stage = (sbp::BoxRec*)h;
    void* dv = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&dv, h, 0));
    p->d_stage = (const sbp::BoxRec*)dv;
    p->slot_ev.resize(p->nslots);
    p->slot_used.assign(p->nslots, false);
    for (auto& e : p->slot_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));

    if (flags & SBP_FLAG_PLAIN) {
      p->master[1].g.nz = p->master[1].g.m;  // the padded spectrum seen as a box with nz = M
      const BoxInfo& bi = p->boxes[0];
      sbp::BoxGeom gp = bi.g;
      gp.nz = gp.m;
      // layout read by launch_plain: box_ids {0}, starts {0, y blocks}, then {0, x blocks}
      const int lay[5] = {0, 0, sbp::y_tiles(0, bi.g, bi.var[sbp::kYFwd]), 0, sbp::x_tiles(0, gp, bi.var[sbp::kXFwd])};
      HIP_TRY(hipMemcpy(p->d_ints, lay, sizeof lay, hipMemcpyHostToDevice));
      p->describe = describe_plan(p.get());
    } else {
      if (flags & SBP_FLAG_AUTOTUNE) {
        sbp_status ts = sbp::autotune(p.get());
        if (ts != SBP_OK) return ts;
      }
      sbp_status us = upload_groups(p.get());
      if (us != SBP_OK) return us;
    }
    // partial-sum slots written by the first pass as launched (its tiles)
    for (size_t r = 0; r < p->nrec; ++r) {
      const BoxInfo& bi = p->boxes[(flags & SBP_FLAG_PLAIN) ? 0 : r];
      if (!(flags & SBP_FLAG_PLAIN) && (bi.first_tiles <= 0 || bi.first_tiles > bi.npartials))
        return fail(SBP_E_STATE, "box %zu: %d first-pass tiles for %d partial-sum slots", r, bi.first_tiles,
                    bi.npartials);
      p->master[r].npartials = (flags & SBP_FLAG_PLAIN) ? sbp::kPlainPartials : bi.first_tiles;
    }
    *out = p.release();
    return SBP_OK;
  } catch (const std::bad_alloc&) {
    return fail(SBP_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SBP_E_STATE, "internal error");
  }
}

sbp_status sbp_workspace_size(sbp_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(SBP_E_ARG, "NULL argument");
  *bytes = p->ws_need;
  return SBP_OK;
}

sbp_status sbp_set_workspace(sbp_plan p, void* ptr, size_t bytes) {
  if (!p) return fail(SBP_E_ARG, "NULL plan");
  if (ptr == nullptr) {
    if (!p->ws_owned) p->ws = nullptr;
    return SBP_OK;
  }
  if (((uintptr_t)ptr) % kAlign) return fail(SBP_E_WORKSPACE, "workspace not %zu-byte aligned", kAlign);
  if (bytes < p->ws_need) return fail(SBP_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, p->ws_need);
  if (p->ws_owned && p->ws) {
    hipSetDevice(p->device);
    hipDeviceSynchronize();
    hipFree(p->ws);
  }
  p->ws = (char*)ptr;
  p->ws_owned = false;
  return SBP_OK;
}

}  // extern "C"

namespace {

// One solve of every box.  fixed_ws: take the workspace from the device's static array (the
// allocation-free entry point) rather than the plan's own or the caller's; that path also makes
// no event or stream of its own (no profiling records), so it allocates nothing.
sbp_status solve_common(sbp_plan p, const void* const* rho, void* const* phi, const sbp_shear* params, void* stream,
                        bool fixed_ws) {
  try {
    if (!p) return fail(SBP_E_ARG, "NULL plan");
    if (!rho || !phi || !params) return fail(SBP_E_ARG, "NULL rho/phi/params array");
    const size_t nb = p->boxes.size();
    for (size_t b = 0; b < nb; ++b) {
      if (!rho[b] || !phi[b]) return fail(SBP_E_ARG, "box %zu: NULL rho or phi", b);
      const size_t n = p->boxes[b].data_bytes;
      if (((uintptr_t)rho[b]) % 16 || ((uintptr_t)phi[b]) % 16)
        return fail(SBP_E_ARG, "box %zu: rho/phi must be 16-byte aligned", b);
      for (size_t c = 0; c < nb; ++c) {
        if (overlap(phi[b], n, rho[c], p->boxes[c].data_bytes))
          return fail(SBP_E_ARG, "phi of box %zu overlaps rho of box %zu", b, c);
        if (c != b && overlap(phi[b], n, phi[c], p->boxes[c].data_bytes))
          return fail(SBP_E_ARG, "phi of boxes %zu and %zu overlap", b, c);
      }
      const sbp_shear& s = params[b];
      const double a = s.q * s.omega * p->boxes[b].g.lx * s.t;
      if (!std::isfinite(a) || !std::isfinite(s.G)) return fail(SBP_E_ARG, "box %zu: non-finite shear parameters", b);
    }
    char* ws = nullptr;
    if (fixed_ws) {
      if (p->ws_need > (size_t)SBP_STATIC_WORKSPACE_BYTES)
        return fail(SBP_E_SIZE, "the plan needs %zu bytes of workspace; the static workspace holds %zu",
                    p->ws_need, (size_t)SBP_STATIC_WORKSPACE_BYTES);
      if ((p->flags & SBP_FLAG_GRAPH) && !p->gexec)
        return fail(SBP_E_STATE, "the graph of this plan is captured by its first sbp_solve; call that first");
      if (p->device >= kMaxDevices) return fail(SBP_E_ARG, "device %d has no static workspace", p->device);
      {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ws = (char*)g_scratch_ptr[p->device];
        if (!ws)
          return fail(SBP_E_HIP, "static workspace unavailable on device %d: %s", p->device,
                      g_scratch_tried[p->device] ? hipGetErrorString(g_scratch_err[p->device]) : "not set up");
      }
      HIP_TRY(hipSetDevice(p->device));
    } else {
      HIP_TRY(hipSetDevice(p->device));
      if (!p->ws) {
        void* d = nullptr;
        if (hipMalloc(&d, std::max<size_t>(p->ws_need, 256)) != hipSuccess)
          return fail(SBP_E_NOMEM, "workspace allocation (%zu bytes)", p->ws_need);
        p->ws = (char*)d;
        p->ws_owned = true;
      }
      ws = p->ws;
    }
    for (size_t b = 0; b < nb; ++b)
      if (overlap(phi[b], p->boxes[b].data_bytes, ws, p->ws_need) ||
          overlap(rho[b], p->boxes[b].data_bytes, ws, p->ws_need))
        return fail(SBP_E_ARG, "rho or phi of box %zu overlaps the workspace", b);
    bind_workspace(p, ws);
    hipStream_t st = (hipStream_t)stream;
    const bool prof = p->prof && !fixed_ws;
    if ((p->flags & SBP_FLAG_GRAPH) && !p->gexec) {
      // the replayed fetch kernel follows the device-side ring counter: start it and the host
      // ring at slot 0, once every earlier (direct, e.g. autotuning) use of the ring is done
      for (int i = 0; i < p->nslots; ++i)
        if (p->slot_used[i]) HIP_TRY(hipEventSynchronize(p->slot_ev[i]));
      const int zero[2] = {0, 0};
      HIP_TRY(hipMemcpy(p->d_ctl, zero, sizeof zero, hipMemcpyHostToDevice));
      p->slot = 0;
    }
    if (!(p->flags & SBP_FLAG_GRAPH) && p->nrec <= (size_t)sbp::kArgRecs) {
      // direct launches of a small plan: the records travel as kernel arguments, no ring slot
      sbp::BoxRec recs[sbp::kArgRecs];
      fill_records(p, rho, phi, params, recs);
      Marker mk{p, st};
      return enqueue(p, st, prof ? &mk : nullptr, 0, recs);
    }
    int slot = 0;
    sbp_status ss = stage_records(p, rho, phi, params, &slot);
    if (ss != SBP_OK) return ss;

    if (p->flags & SBP_FLAG_GRAPH) {
      if (!p->gexec) {
        // the launches read everything per-solve from the device records: capture once
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        sbp_status es = enqueue(p, p->cap_stream, nullptr, -1);
        hipGraph_t gr = nullptr;
        hipError_t ce = hipStreamEndCapture(p->cap_stream, &gr);
        if (es != SBP_OK) {
          if (gr) hipGraphDestroy(gr);
          return es;
        }
        if (ce != hipSuccess) return fail(SBP_E_HIP, "graph capture: %s", hipGetErrorString(ce));
        p->graph = gr;
        HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
      }
      // the replay fetches ring slot ctl[0], which advances in step with p->slot
      Marker mk{p, st};
      if (prof) mk.mark("graph");
      HIP_TRY(hipGraphLaunch(p->gexec, st));
      if (prof) mk.mark(nullptr);
      return commit_slot(p, slot, st);
    }
    Marker mk{p, st};
    sbp_status es = enqueue(p, st, prof ? &mk : nullptr, slot);
    if (es != SBP_OK) return es;
    return commit_slot(p, slot, st);
  } catch (const std::bad_alloc&) {
    return fail(SBP_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SBP_E_STATE, "internal error");
  }
}

}  // namespace

extern "C" {

sbp_status sbp_solve(sbp_plan p, const void* const* rho, void* const* phi, const sbp_shear* params, void* stream) {
  return solve_common(p, rho, phi, params, stream, false);
}

sbp_status sbp_solve_static(sbp_plan p, const void* const* rho, void* const* phi, const sbp_shear* params,
                            void* stream) {
  return solve_common(p, rho, phi, params, stream, true);
}

sbp_status sbp_ghosts(sbp_plan p, const void* const* phi, void* const* out, int32_t ng, void* stream) {
  try {
    if (!p) return fail(SBP_E_ARG, "NULL plan");
    if (!phi || !out) return fail(SBP_E_ARG, "NULL phi/out array");
    if (ng < 1 || ng > 16) return fail(SBP_E_ARG, "ng=%d outside [1, 16]", ng);
    const size_t w = elem_size(p->prec);
    for (size_t b = 0; b < p->boxes.size(); ++b) {
      const sbp::BoxGeom& g = p->boxes[b].g;
      if (!phi[b] || !out[b]) return fail(SBP_E_ARG, "box %zu: NULL phi or out", b);
      const size_t rows = (size_t)g.nx * g.ny;
      if (overlap(phi[b], rows * g.nz * w, out[b], rows * (g.nz + 2 * ng) * w))
        return fail(SBP_E_ARG, "box %zu: out overlaps phi", b);
    }
    HIP_TRY(hipSetDevice(p->device));
    for (size_t b = 0; b < p->boxes.size(); ++b)
      HIP_TRY(sbp::launch_ghosts(p->prec, p->boxes[b].g, phi[b], out[b], ng, (hipStream_t)stream));
    return SBP_OK;
  } catch (...) {
    return fail(SBP_E_STATE, "internal error");
  }
}

sbp_status sbp_gravity(sbp_plan p, const void* const* phi, void* const* gx, void* const* gy, void* const* gz,
                       const sbp_shear* params, void* stream) {
  try {
    if (!p) return fail(SBP_E_ARG, "NULL plan");
    if (!phi || !gx || !gy || !gz || !params) return fail(SBP_E_ARG, "NULL argument array");
    const size_t w = elem_size(p->prec);
    for (size_t b = 0; b < p->boxes.size(); ++b) {
      const sbp::BoxGeom& g = p->boxes[b].g;
      const size_t n = (size_t)g.nx * g.ny * g.nz * w;
      const void* ptr[4] = {phi[b], gx[b], gy[b], gz[b]};
      for (int i = 0; i < 4; ++i) {
        if (!ptr[i]) return fail(SBP_E_ARG, "box %zu: NULL pointer", b);
        for (int k = 0; k < i; ++k)
          if (overlap(ptr[i], n, ptr[k], n)) return fail(SBP_E_ARG, "box %zu: overlapping phi/gx/gy/gz", b);
      }
      const sbp_shear& s = params[b];
      if (!std::isfinite(s.q * s.omega * g.lx * s.t)) return fail(SBP_E_ARG, "box %zu: non-finite shear", b);
    }
    HIP_TRY(hipSetDevice(p->device));
    for (size_t b = 0; b < p->boxes.size(); ++b) {
      const sbp::BoxGeom& g = p->boxes[b].g;
      const sbp_shear& s = params[b];
      double d = std::fmod(s.q * s.omega * g.lx * s.t, g.ly);
      if (d < 0.0) d += g.ly;
      if (d >= g.ly) d = 0.0;
      HIP_TRY(sbp::launch_gravity(p->prec, g, d, phi[b], gx[b], gy[b], gz[b], (hipStream_t)stream));
    }
    return SBP_OK;
  } catch (...) {
    return fail(SBP_E_STATE, "internal error");
  }
}

sbp_status sbp_plan_destroy(sbp_plan p) {
  if (!p) return SBP_OK;
  hipSetDevice(p->device);
  // work enqueued by this plan may still read its tables, records, ring and workspace: wait for
  // the device before freeing them (a plan is destroyed rarely; the streams it was used on are
  // not tracked, and may already be gone)
  hipDeviceSynchronize();
  destroy_graph(p);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  for (auto& r : p->pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : p->free_events) hipEventDestroy(e);
  for (auto e : p->slot_ev) hipEventDestroy(e);
  if (p->h_stage) hipHostFree(p->h_stage);
  if (p->ws_owned && p->ws) hipFree(p->ws);
  if (p->d_aux) hipFree(p->d_aux);
  if (p->d_blk) hipFree(p->d_blk);
  if (p->d_tables) hipFree(p->d_tables);
  delete p;
  return SBP_OK;
}

sbp_status sbp_profile_enable(sbp_plan p, int32_t enable) {
  if (!p) return fail(SBP_E_ARG, "NULL plan");
  p->prof = enable != 0;
  return SBP_OK;
}

sbp_status sbp_profile_read(sbp_plan p, const char** names, int64_t* launches, double* total_ms, int32_t cap,
                            int32_t* count) {
  if (!p || !count) return fail(SBP_E_ARG, "NULL argument");
  hipSetDevice(p->device);
  // events are shared between consecutive records; recycle each once
  std::vector<hipEvent_t> seen;
  for (auto& r : p->pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    auto& t = p->totals[r.name];
    t.first += 1;
    t.second += ms;
    seen.push_back(r.a);
    seen.push_back(r.b);
  }
  std::sort(seen.begin(), seen.end());
  seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
  for (auto e : seen) p->free_events.push_back(e);
  p->pending.clear();
  p->names.clear();
  for (auto& kv : p->totals) p->names.push_back(kv.first);
  int i = 0;
  for (auto& kv : p->totals) {
    if (i < cap) {
      if (names) names[i] = p->names[i].c_str();
      if (launches) launches[i] = kv.second.first;
      if (total_ms) total_ms[i] = kv.second.second;
    }
    ++i;
  }
  *count = i;
  p->totals.clear();
  return SBP_OK;
}

sbp_status sbp_plan_describe(sbp_plan p, char* buf, size_t len) {
  if (!p || !buf || len == 0) return fail(SBP_E_ARG, "NULL argument");
  snprintf(buf, len, "%s", p->describe.c_str());
  return SBP_OK;
}

}  // extern "C"
