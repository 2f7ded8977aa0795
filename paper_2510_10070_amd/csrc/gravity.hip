// Output for the hydrodynamics (Sect. 2.4): the potential with vertical ghost layers, and the
// gravitational acceleration -grad Phi by second-order centred differences.
//
// Ghost layers continue Phi with the vertical gradient of the last active cell.  The
// acceleration uses periodic y, that ghost rule in z, and shear-periodic x: the lab field
// satisfies f(x + Lx, y) = f(x, y + Dy0), so the neighbour beyond the last x row is the first
// row sampled at y + Dy0 and the one before the first row is the last row sampled at y - Dy0,
// both by linear interpolation between neighbouring y cells.
//
// One block per (x, y) row, threads along z (coalesced); neighbours come from L1/L2.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sbp_internal.hpp"

namespace sbp {

namespace {

constexpr int kRowThreads = 256;

template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_ghosts(const T* __restrict__ phi, T* __restrict__ out, int nx, int ny,
                                                        int nz, int ng) {
  const int row = blockIdx.x;  // x * ny + y
  const T* src = phi + (size_t)row * nz;
  T* dst = out + (size_t)row * (nz + 2 * ng);
  const T lo = src[1] - src[0];
  const T hi = src[nz - 1] - src[nz - 2];
  for (int k = threadIdx.x; k < nz + 2 * ng; k += blockDim.x) {
    T v;
    if (k < ng)
      v = src[0] - (T)(ng - k) * lo;
    else if (k >= ng + nz)
      v = src[nz - 1] + (T)(k - ng - nz + 1) * hi;
    else
      v = src[k - ng];
    dst[k] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_gravity(const T* __restrict__ phi, T* __restrict__ gx,
                                                         T* __restrict__ gy, T* __restrict__ gz, int nx, int ny,
                                                         int nz, T idx2, T idy2, T idz2, int m_lo, T w_lo, int m_hi,
                                                         T w_hi) {
  const int row = blockIdx.x;
  const int x = row / ny, y = row - x * ny;
  const size_t plane = (size_t)ny * nz;
  const T* c = phi + (size_t)row * nz;
  const T* yp = phi + (size_t)x * plane + (size_t)(y + 1 == ny ? 0 : y + 1) * nz;
  const T* ym = phi + (size_t)x * plane + (size_t)(y == 0 ? ny - 1 : y - 1) * nz;
  // x neighbours; at the edges, the opposite edge row sampled at y -/+ Dy0 (two rows, weights)
  const T *xp0, *xp1, *xm0, *xm1;
  T wp = T(0), wm = T(0);
  if (x + 1 < nx) {
    xp0 = xp1 = c + plane;
  } else {  // row 0 at y + Dy0: cells y + m_hi and y + m_hi + 1
    const int a = (y + m_hi) % ny, b = (a + 1) % ny;
    xp0 = phi + (size_t)a * nz;
    xp1 = phi + (size_t)b * nz;
    wp = w_hi;
  }
  if (x > 0) {
    xm0 = xm1 = c - plane;
  } else {  // row nx-1 at y - Dy0: cells y + m_lo and y + m_lo + 1
    const int a = (y + m_lo) % ny, b = (a + 1) % ny;
    xm0 = phi + (size_t)(nx - 1) * plane + (size_t)a * nz;
    xm1 = phi + (size_t)(nx - 1) * plane + (size_t)b * nz;
    wm = w_lo;
  }
  for (int k = threadIdx.x; k < nz; k += blockDim.x) {
    const T f = c[k];
    const T fxp = (T(1) - wp) * xp0[k] + wp * xp1[k];
    const T fxm = (T(1) - wm) * xm0[k] + wm * xm1[k];
    // z: the ghost value beyond an edge continues the last active gradient
    const T fzp = k + 1 < nz ? c[k + 1] : T(2) * f - c[k - 1];
    const T fzm = k > 0 ? c[k - 1] : T(2) * f - c[k + 1];
    const size_t o = (size_t)row * nz + k;
    gx[o] = -(fxp - fxm) * idx2;
    gy[o] = -(yp[k] - ym[k]) * idy2;
    gz[o] = -(fzp - fzm) * idz2;
  }
}

// floor and weight of a sample at fractional y index j + d (periodic in n)
void split(double d, int n, int& m, double& w) {
  const double fl = std::floor(d);
  w = d - fl;
  long long mm = static_cast<long long>(fl) % n;
  if (mm < 0) mm += n;
  m = static_cast<int>(mm);
}

}  // namespace

hipError_t launch_ghosts(int prec, const BoxGeom& g, const void* phi, void* out, int ng, hipStream_t st) {
  const dim3 grid(g.nx * g.ny), block(kRowThreads);
  if (prec)
    hipLaunchKernelGGL(k_ghosts<float>, grid, block, 0, st, static_cast<const float*>(phi), static_cast<float*>(out),
                       g.nx, g.ny, g.nz, ng);
  else
    hipLaunchKernelGGL(k_ghosts<double>, grid, block, 0, st, static_cast<const double*>(phi),
                       static_cast<double*>(out), g.nx, g.ny, g.nz, ng);
  return hipGetLastError();
}

hipError_t launch_gravity(int prec, const BoxGeom& g, double dy0, const void* phi, void* gx, void* gy, void* gz,
                          hipStream_t st) {
  const double dx = g.lx / g.nx, dy = g.ly / g.ny, dz = g.lz / g.nz;
  const double cells = dy0 / dy;
  int m_lo, m_hi;
  double w_lo, w_hi;
  split(-cells, g.ny, m_lo, w_lo);
  split(cells, g.ny, m_hi, w_hi);
  const dim3 grid(g.nx * g.ny), block(kRowThreads);
  if (prec)
    hipLaunchKernelGGL(k_gravity<float>, grid, block, 0, st, static_cast<const float*>(phi), static_cast<float*>(gx),
                       static_cast<float*>(gy), static_cast<float*>(gz), g.nx, g.ny, g.nz, (float)(0.5 / dx),
                       (float)(0.5 / dy), (float)(0.5 / dz), m_lo, (float)w_lo, m_hi, (float)w_hi);
  else
    hipLaunchKernelGGL(k_gravity<double>, grid, block, 0, st, static_cast<const double*>(phi),
                       static_cast<double*>(gx), static_cast<double*>(gy), static_cast<double*>(gz), g.nx, g.ny,
                       g.nz, 0.5 / dx, 0.5 / dy, 0.5 / dz, m_lo, w_lo, m_hi, w_hi);
  return hipGetLastError();
}

}  // namespace sbp
