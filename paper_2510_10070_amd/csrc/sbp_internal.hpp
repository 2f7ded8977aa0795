// Internal types shared by the host plan and the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sbp {

// Static geometry of one box, passed to kernels by value.
struct BoxGeom {
  int nx, ny, nz;  // physical cells; ny/2 stored y modes (Nyquist dropped)
  int m;           // padded z length P*nz
  int method;      // 0 = VGF-HybridBC, 1 = SASHA
  double lx, ly, lz;
  double L;        // truncation length alpha*lz of the VGF kernel
};

// Per-solve scalars of one box, written to device memory before each solve.
struct SolveScalars {
  double s;      // Delta_y0/Lx: shear of the wave vector, kx = Kx + s Ky
  double fy;     // Delta_y0/(2 Ly Nx): remap phase in cycles per unit of my*(2i+1)
  double scale;  // 4 pi G/(Nx Ny M): Green's-function factor including DFT normalisation
  double fourpiG;
};

// SASHA analytic part Phi_0(z) = c2 z^2 + c1 z, produced on the device from the reductions.
struct SashaCoef {
  double c2, c1;
};

// Per-kz tables of the padded z grid (plan constants), in precision T:
//   s2 = 1 - cos(kz L) = 2 sin^2(kz L/2),  ks = kz sin(kz L),  kz2 = kz^2.
template <typename T> struct ZTables {
  const T* s2;
  const T* ks;
  const T* kz2;
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

// Launchers (defined in the pass translation units).  prec: 0 = double, 1 = float.
hipError_t launch_yfwd(int prec, const BoxGeom& g, const void* rho, void* W, const void* tw_y,
                       const SolveScalars* sp, double* partials, hipStream_t st);
hipError_t launch_x(int prec, int dir, const BoxGeom& g, void* W, const void* tw_x, hipStream_t st);
hipError_t launch_z(int prec, const BoxGeom& g, void* W, const void* tw_m, const void* tw_m64,
                    const void* zt_s2, const void* zt_ks, const void* zt_kz2, const double* zt64_s2,
                    const double* zt64_ks, const double* zt64_kz2, const SolveScalars* sp,
                    const double* partials, int npartials, SashaCoef* coef, hipStream_t st);
hipError_t launch_yinv(int prec, const BoxGeom& g, const void* W, void* phi, const void* tw_y,
                       const SolveScalars* sp, const SashaCoef* coef, hipStream_t st);

// Number of SASHA partial-sum slots written by launch_yfwd for this box and precision.
int yfwd_partials(int prec, const BoxGeom& g);

// Plain (unfused) FP64 path.
hipError_t launch_y_plain(int dir, const BoxGeom& g, const double* in, double* out, const void* tw_y,
                          hipStream_t st);
hipError_t launch_zfft_plain(int dir, const BoxGeom& g, double* P, const void* tw_m, hipStream_t st);
constexpr int kPlainPartials = 1024;
hipError_t launch_plain(const BoxGeom& g, const double* rho, double* phi, double* work_pad, double* work_half,
                        const void* tw_x, const void* tw_y, const void* tw_m, const double* zt_s2,
                        const double* zt_ks, const double* zt_kz2, const SolveScalars* sp,
                        double* partials, SashaCoef* coef, hipStream_t st,
                        void (*mark)(void*, const char*), void* mark_ctx);

}  // namespace sbp
