// Host side of the C ABI: descriptor validation, plan tables, workspace, launch sequence,
// HIP-graph capture and kernel timing.  Every entry point catches all C++ exceptions and
// reports through sbp_status plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sbp.h"
#include "sbp_internal.hpp"

namespace {

thread_local std::string g_last_error;

sbp_status fail(sbp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(SBP_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

struct BoxPlan {
  sbp::BoxGeom g;
  size_t tw_x = 0, tw_y = 0, tw_m = 0, tw_m64 = 0;  // offsets into the table block
  size_t zt[3] = {0, 0, 0}, zt64[3] = {0, 0, 0};
  size_t ws_off = 0;     // complex half spectrum (fused) or padded spectrum (plain)
  size_t ws2_off = 0;    // plain: unpadded half spectrum
  size_t part_off = 0;   // SASHA partial sums (doubles) in the aux block
  int npartials = 0;
  size_t data_bytes = 0; // bytes of rho (= bytes of phi)
};

}  // namespace

struct sbp_plan_s {
  int device = 0;
  int prec = 0;  // 0 double, 1 float
  uint32_t flags = 0;
  std::vector<BoxPlan> boxes;
  char* d_tables = nullptr;
  char* d_aux = nullptr;
  sbp::SolveScalars* d_sp = nullptr;
  sbp::SashaCoef* d_coef = nullptr;
  double* d_partials = nullptr;
  size_t ws_need = 0;
  char* ws = nullptr;
  bool ws_owned = false;
  // pinned staging ring for per-solve scalars
  sbp::SolveScalars* h_stage = nullptr;
  int nslots = 0, slot = 0;
  std::vector<hipEvent_t> slot_ev;
  std::vector<bool> slot_used;
  // graph mode
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> g_rho;
  std::vector<void*> g_phi;
  char* g_ws = nullptr;
  hipStream_t cap_stream = nullptr;  // capture happens here; replays go to the caller's stream
  // profiling
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> free_events;
  std::map<std::string, std::pair<long long, double>> totals;
  std::vector<std::string> names;  // stable storage for sbp_profile_read
  std::string describe;
};

namespace {

size_t elem_size(int prec) { return prec ? sizeof(float) : sizeof(double); }

sbp_status validate_box(const sbp_box& b, int i, int prec, uint32_t flags) {
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
    return fail(SBP_E_ARG, "box %d: alpha=%g outside [1, pad/2]: periodic images of the truncated kernel "
                           "would reach the box", i, b.alpha);
  if (b.method != SBP_VGF && b.method != SBP_SASHA) return fail(SBP_E_ARG, "box %d: unknown method %d", i, b.method);
  const double n = (double)b.nx * b.ny * b.nz;
  if (n * elem_size(prec) > 64.0 * (1ull << 30)) return fail(SBP_E_SIZE, "box %d: grid too large", i);
  (void)flags;
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

struct TableBuilder {
  std::vector<char> host;
  std::map<std::pair<int, int>, size_t> tw;  // (n, prec) -> offset
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

// launch one solve of every box; pointers already validated
sbp_status enqueue(sbp_plan p, const void* const* rho, void* const* phi, hipStream_t st, Marker* mk) {
  for (size_t b = 0; b < p->boxes.size(); ++b) {
    const BoxPlan& bp = p->boxes[b];
    const sbp::BoxGeom& g = bp.g;
    const char* T = p->d_tables;
    const sbp::SolveScalars* sp = p->d_sp + b;
    sbp::SashaCoef* coef = p->d_coef + b;
    double* part = g.method == SBP_SASHA ? p->d_partials + bp.part_off : nullptr;
    if (p->flags & SBP_FLAG_PLAIN) {
      HIP_TRY(sbp::launch_plain(g, (const double*)rho[b], (double*)phi[b], (double*)(p->ws + bp.ws_off),
                                (double*)(p->ws + bp.ws2_off), T + bp.tw_x, T + bp.tw_y, T + bp.tw_m, (const double*)(T + bp.zt64[0]),
                                (const double*)(T + bp.zt64[1]), (const double*)(T + bp.zt64[2]), sp,
                                p->d_partials + bp.part_off, coef, st, mk ? mark_cb : nullptr, mk));
      continue;
    }
    void* W = p->ws + bp.ws_off;
    if (mk) mk->mark("y_forward");
    HIP_TRY(sbp::launch_yfwd(p->prec, g, rho[b], W, T + bp.tw_y, sp, part, st));
    if (mk) mk->mark("x_forward");
    HIP_TRY(sbp::launch_x(p->prec, -1, g, W, T + bp.tw_x, st));
    if (mk) mk->mark("z_green");
    HIP_TRY(sbp::launch_z(p->prec, g, W, T + bp.tw_m, T + bp.tw_m64, T + bp.zt[0], T + bp.zt[1], T + bp.zt[2],
                          (const double*)(T + bp.zt64[0]), (const double*)(T + bp.zt64[1]),
                          (const double*)(T + bp.zt64[2]), sp, part, bp.npartials,
                          g.method == SBP_SASHA ? coef : nullptr, st));
    if (mk) mk->mark("x_inverse");
    HIP_TRY(sbp::launch_x(p->prec, +1, g, W, T + bp.tw_x, st));
    if (mk) mk->mark("y_inverse");
    HIP_TRY(sbp::launch_yinv(p->prec, g, W, phi[b], T + bp.tw_y, sp, g.method == SBP_SASHA ? coef : nullptr, st));
    if (mk) mk->mark(nullptr);
  }
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

}  // namespace

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
    if (flags & ~(SBP_FLAG_GRAPH | SBP_FLAG_AUTOTUNE | SBP_FLAG_PLAIN)) return fail(SBP_E_ARG, "unknown flags 0x%x", flags);
    if ((flags & SBP_FLAG_PLAIN) && (precision != SBP_FP64 || nbox != 1))
      return fail(SBP_E_ARG, "the plain path is FP64 and single-box");
    if (device < 0) return fail(SBP_E_ARG, "device=%d", device);
    const int prec = precision == SBP_FP32 ? 1 : 0;
    for (int i = 0; i < nbox; ++i) {
      sbp_status st = validate_box(boxes[i], i, prec, flags);
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

    TableBuilder tb;
    size_t ws = 0, npart = 0;
    const size_t w = elem_size(prec);
    for (int i = 0; i < nbox; ++i) {
      const sbp_box& b = boxes[i];
      BoxPlan bp;
      const int pad = b.pad == 0 ? 2 : b.pad;
      const double alpha = b.alpha == 0.0 ? 0.5 * pad : b.alpha;
      bp.g = sbp::BoxGeom{b.nx, b.ny, b.nz, pad * b.nz, b.method, b.lx, b.ly, b.lz, alpha * b.lz};
      bp.tw_x = tb.twiddle(b.nx, prec);
      bp.tw_y = tb.twiddle(b.ny, prec);
      bp.tw_m = tb.twiddle(pad * b.nz, prec);
      bp.tw_m64 = tb.twiddle(pad * b.nz, 0);
      std::vector<long double> s2, ks, kz2;
      ztables(bp.g, pad, s2, ks, kz2);
      bp.zt64[0] = put_vec<double>(tb, s2);
      bp.zt64[1] = put_vec<double>(tb, ks);
      bp.zt64[2] = put_vec<double>(tb, kz2);
      if (prec) {
        bp.zt[0] = put_vec<float>(tb, s2);
        bp.zt[1] = put_vec<float>(tb, ks);
        bp.zt[2] = put_vec<float>(tb, kz2);
      } else {
        for (int k = 0; k < 3; ++k) bp.zt[k] = bp.zt64[k];
      }
      const size_t n = (size_t)b.nx * b.ny * b.nz;
      bp.data_bytes = n * w;
      if (flags & SBP_FLAG_PLAIN) {
        bp.ws_off = ws;
        ws = align_up(ws + (size_t)b.nx * (b.ny / 2) * bp.g.m * 2 * sizeof(double));
        bp.ws2_off = ws;
        ws = align_up(ws + n * sizeof(double));
        bp.npartials = sbp::kPlainPartials;
      } else {
        bp.ws_off = ws;
        ws = align_up(ws + n * w);  // nx * (ny/2) * nz complex
        bp.npartials = sbp::yfwd_partials(prec, bp.g);
      }
      bp.part_off = npart;
      npart += 2 * (size_t)bp.npartials;
      p->boxes.push_back(bp);
    }
    p->ws_need = ws;

    void* d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(tb.host.size(), 256)) != hipSuccess)
      return fail(SBP_E_NOMEM, "table allocation (%zu bytes)", tb.host.size());
    p->d_tables = (char*)d;
    HIP_TRY(hipMemcpy(p->d_tables, tb.host.data(), tb.host.size(), hipMemcpyHostToDevice));
    const size_t aux = align_up(nbox * sizeof(sbp::SolveScalars)) + align_up(nbox * sizeof(sbp::SashaCoef)) +
                       align_up(std::max<size_t>(npart, 2) * sizeof(double));
    if (hipMalloc(&d, aux) != hipSuccess) return fail(SBP_E_NOMEM, "aux allocation (%zu bytes)", aux);
    p->d_aux = (char*)d;
    p->d_sp = (sbp::SolveScalars*)p->d_aux;
    p->d_coef = (sbp::SashaCoef*)(p->d_aux + align_up(nbox * sizeof(sbp::SolveScalars)));
    p->d_partials = (double*)((char*)p->d_coef + align_up(nbox * sizeof(sbp::SashaCoef)));

    p->nslots = 64;
    void* h = nullptr;
    if (hipHostMalloc(&h, (size_t)p->nslots * nbox * sizeof(sbp::SolveScalars), hipHostMallocDefault) != hipSuccess)
      return fail(SBP_E_NOMEM, "pinned staging allocation");
    p->h_stage = (sbp::SolveScalars*)h;
    p->slot_ev.resize(p->nslots);
    p->slot_used.assign(p->nslots, false);
    for (auto& e : p->slot_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));

    char buf[512];
    const BoxPlan& b0 = p->boxes[0];
    snprintf(buf, sizeof buf,
             "{\"path\":\"%s\",\"precision\":\"%s\",\"nbox\":%d,\"passes\":%d,\"graph\":%s,"
             "\"box0\":[%d,%d,%d],\"pad_len\":%d,\"workspace_bytes\":%zu}",
             (flags & SBP_FLAG_PLAIN) ? "plain" : "streaming-5pass", prec ? "fp32" : "fp64", nbox,
             (flags & SBP_FLAG_PLAIN) ? 13 : 5, (flags & SBP_FLAG_GRAPH) ? "true" : "false", b0.g.nx, b0.g.ny,
             b0.g.nz, b0.g.m, p->ws_need);
    p->describe = buf;
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
    destroy_graph(p);
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
  destroy_graph(p);
  return SBP_OK;
}

sbp_status sbp_solve(sbp_plan p, const void* const* rho, void* const* phi, const sbp_shear* params, void* stream) {
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
    HIP_TRY(hipSetDevice(p->device));
    if (!p->ws) {
      void* d = nullptr;
      if (hipMalloc(&d, std::max<size_t>(p->ws_need, 256)) != hipSuccess)
        return fail(SBP_E_NOMEM, "workspace allocation (%zu bytes)", p->ws_need);
      p->ws = (char*)d;
      p->ws_owned = true;
    }
    for (size_t b = 0; b < nb; ++b)
      if (overlap(phi[b], p->boxes[b].data_bytes, p->ws, p->ws_need))
        return fail(SBP_E_ARG, "phi of box %zu overlaps the workspace", b);
    hipStream_t st = (hipStream_t)stream;

    // per-solve scalars -> pinned slot -> device
    const int slot = p->slot;
    p->slot = (p->slot + 1) % p->nslots;
    if (p->slot_used[slot]) HIP_TRY(hipEventSynchronize(p->slot_ev[slot]));
    sbp::SolveScalars* hs = p->h_stage + (size_t)slot * nb;
    for (size_t b = 0; b < nb; ++b) {
      const sbp::BoxGeom& g = p->boxes[b].g;
      const sbp_shear& s = params[b];
      double d = std::fmod(s.q * s.omega * g.lx * s.t, g.ly);
      if (d < 0.0) d += g.ly;
      if (d >= g.ly) d = 0.0;
      hs[b].s = d / g.lx;
      hs[b].fy = (d / g.ly) / (2.0 * g.nx);
      hs[b].fourpiG = 4.0 * M_PI * s.G;
      hs[b].scale = hs[b].fourpiG / ((double)g.nx * g.ny * g.m);
    }
    HIP_TRY(hipMemcpyAsync(p->d_sp, hs, nb * sizeof(sbp::SolveScalars), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(p->slot_ev[slot], st));
    p->slot_used[slot] = true;

    if (p->flags & SBP_FLAG_GRAPH) {
      bool same = p->gexec && p->g_ws == p->ws;
      for (size_t b = 0; same && b < nb; ++b) same = p->g_rho[b] == rho[b] && p->g_phi[b] == phi[b];
      if (!same) {
        destroy_graph(p);
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        sbp_status es = enqueue(p, rho, phi, p->cap_stream, nullptr);
        hipGraph_t gr = nullptr;
        hipError_t ce = hipStreamEndCapture(p->cap_stream, &gr);
        if (es != SBP_OK) {
          if (gr) hipGraphDestroy(gr);
          return es;
        }
        if (ce != hipSuccess) return fail(SBP_E_HIP, "graph capture: %s", hipGetErrorString(ce));
        p->graph = gr;
        HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
        p->g_rho.assign(rho, rho + nb);
        p->g_phi.assign(phi, phi + nb);
        p->g_ws = p->ws;
      }
      Marker mk{p, st};
      if (p->prof) mk.mark("graph");
      HIP_TRY(hipGraphLaunch(p->gexec, st));
      if (p->prof) mk.mark(nullptr);
      return SBP_OK;
    }
    Marker mk{p, st};
    return enqueue(p, rho, phi, st, p->prof ? &mk : nullptr);
  } catch (const std::bad_alloc&) {
    return fail(SBP_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(SBP_E_STATE, "internal error");
  }
}

sbp_status sbp_plan_destroy(sbp_plan p) {
  if (!p) return SBP_OK;
  hipSetDevice(p->device);
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
  // events are shared between consecutive records; destroy each once
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
