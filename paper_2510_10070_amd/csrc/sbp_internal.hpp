// Internal types shared by the host plan and the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sbp {

// Static geometry of one box.
struct BoxGeom {
  int nx, ny, nz;  // physical cells; ny/2 stored y modes (Nyquist dropped)
  int m;           // padded z length P*nz
  int method;      // 0 = VGF-HybridBC, 1 = SASHA
  int remap;       // 0 = spectral phase, 1 = linear interpolation in y
  double lx, ly, lz;
  double L;        // truncation length alpha*lz of the VGF kernel
};

// SASHA analytic part Phi_0(z) = c2 z^2 + c1 z, produced on the device from the reductions.
struct SashaCoef {
  double c2, c1;
};

// Everything a kernel needs about one box, in device memory.  The per-solve fields are
// rewritten by the first kernel of every solve (also under graph replay), from the solve's
// kernel arguments or from a pinned ring slot.
struct BoxRec {
  BoxGeom g;
  // per solve
  const void* rho;
  void* phi;
  double s;        // Delta_y0/Lx: kx = Kx + s Ky
  double fy;       // Delta_y0/(2 Ly Nx): remap phase in cycles per unit of my*(2i+1) (0: linear remap)
  double shy;      // linear remap: row x_i is shifted by shy (i + 1/2) y cells (s dx/dy)
  double scale;    // 4 pi G/(Nx Ny M)
  double fourpiG;
  // plan constants
  void* W;         // half spectrum [nx][ny/2][nz] complex (plain path: padded [..][m])
  double* partials;
  int npartials;
  SashaCoef* coef;
  const void* zt;        // rows {1 - cos(kz L), kz sin(kz L), kz^2, 0} per kz, plan precision
  const double* zt64[3]; // the three columns separately in double
  const double* k0h;     // k = 0 pencil in real space: h[n] = sum_m G(0, kz_m) cos(2 pi m n/M)
  const void* twx;       // x twiddles w_Nx^m, m < Nx, plan precision (fused passes A and C)
  const void* twy;       // stage-major y twiddles of Ny (fused passes A and C of groups mixing Ny)
  const void* twz;       // stage-major z twiddles of M (fused pass B of groups mixing M)
};

// Pointers held in the records and launch arguments address device global memory.  Kernels
// access that memory through gmem<T>* (from hbm()) so that the accesses compile to global
// rather than flat instructions: a flat access also counts against the LDS counter, so every
// LDS wait behind an outstanding flat load or store would wait for HBM as well.
// (The host pass of the same source, which only checks kernel bodies, sees plain types.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using gmem = __attribute__((address_space(1))) T;
#else
template <class T> using gmem = T;
#endif
template <class T> __device__ __forceinline__ gmem<T>* hbm(T* p) { return (gmem<T>*)p; }

// A launch serves a group of boxes with the same kernel shape.
struct GroupArgs {
  const int* box_ids;  // boxes of the group (indices into the BoxRec array)
  const int* starts;   // first block of each box; starts[n] = total blocks
  int n;
  int total;           // = starts[n], the launch's block count
  int box0;            // = box_ids[0]: a one-box group needs no table lookup
  const int2* blk;     // n > 1: (box id, tile) of every block b < total, so one load finds both
  // Direct launches of a one-box plan: the solve's first pass receives the record with its own
  // launch (use_arg = 1) rather than from the device array, and its block 0 stores it to `pub`
  // for the later passes, so no separate record copy runs before it.
  int use_arg = 0;
  BoxRec* pub = nullptr;
  BoxRec arg{};
};

// Supported transform lengths (x, y and padded z).
#define SBP_FOR_EACH_LEN(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

inline bool supported_len(int n) {
#define SBP_CASE(N_) if (n == N_) return true;
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return false;
}

constexpr int kVariants = 2;  // tile variants per pass kernel

// Tiles (= blocks) one box needs in each pass for a variant.  prec: 0 double, 1 float.
int y_tiles(int prec, const BoxGeom& g, int variant);
int x_tiles(int prec, const BoxGeom& g, int variant);
int z_tiles(int prec, const BoxGeom& g, int variant);

// Launchers; `blocks` is the total block count of the group (ga.starts[ga.n] on the host).
hipError_t launch_y(int prec, bool forward, bool remap, int ny, int variant, GroupArgs ga, int blocks,
                    const BoxRec* recs, const void* tw, hipStream_t st);
hipError_t launch_x(int prec, int dir, int nx, int variant, GroupArgs ga, int blocks, const BoxRec* recs,
                    const void* tw, hipStream_t st);
hipError_t launch_z(int prec, int m, int variant, int q, GroupArgs ga, int blocks, const BoxRec* recs,
                    const void* tw, const void* tw64, hipStream_t st);

// Fused three-pass schedule (four-step x split Nx = A * 16).  kind: 0 pass A, 1 pass B, 2 pass C.
bool fused_ok(const BoxGeom& g);
int fused_ac_tiles(int prec, const BoxGeom& g, int variant);
int fused_b_tiles(const BoxGeom& g);
int fused_a(const BoxGeom& g);
// float pass B groups that mix M (padding 2, M <= 256): items of one box per block, 0 if the box
// cannot join such a group
int fused_b_items_per_block(const BoxGeom& g, int pad);
// float pass A/C groups that mix Ny: tiles of one box (rows of 64 or 128 bytes by Ny)
int fused_ac_multi_tiles(const BoxGeom& g);
hipError_t launch_fused(int prec, int kind, int len, int a, int variant, int q, bool lin, GroupArgs ga, int blocks,
                        const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st);

// Copy the records of one solve from pinned ring slot `slot` (or, with slot < 0, from the slot
// named by ctl[0], which the kernel then advances) into the device record array.
hipError_t launch_fetch(const BoxRec* ring, BoxRec* recs, int nrec, int nslots, int slot, int* ctl, hipStream_t st);
// records of at most kArgRecs boxes passed as kernel arguments (direct launches)
constexpr int kArgRecs = 8;
hipError_t launch_fetch_args(const BoxRec* host, BoxRec* recs, int nrec, hipStream_t st);

// Output for the hydrodynamics: vertical ghost layers and the acceleration (gravity.hip).
hipError_t launch_ghosts(int prec, const BoxGeom& g, const void* phi, void* out, int ng, hipStream_t st);
hipError_t launch_gravity(int prec, const BoxGeom& g, double dy0, const void* phi, void* gx, void* gy, void* gz,
                          hipStream_t st);

// Plain (unfused) FP64 path for one box: rec0 views the half spectrum, rec_pad the padded one.
constexpr int kPlainPartials = 1024;
hipError_t launch_plain(const BoxRec* h_rec, const BoxRec* d_rec0, const BoxRec* d_rec_pad, GroupArgs one,
                        int y_var, int x_var, const void* tws_x, const void* tws_y, const void* tw_m,
                        hipStream_t st, void (*mark)(void*, const char*), void* mark_ctx);

}  // namespace sbp
