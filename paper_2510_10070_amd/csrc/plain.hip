// Plain FP64 path: the same discrete operator with one kernel per step and the zero-padded
// spectrum materialised in HBM.  It is the unfused reference the streaming passes are measured
// against: y transform, remap, zero padding, x transform, z transform, Green multiply, z and x
// inverse transforms, extraction, reverse remap, inverse y transform, SASHA Phi_0.
#include "fft_device.hpp"
#include "sbp_internal.hpp"

namespace sbp {

constexpr int kEw = 256;  // elementwise block size

__device__ __forceinline__ double2 remap_factor(int my, int x, double fy, int sign) {
  const double c = static_cast<double>(my * (2 * x + 1)) * fy;
  const double r = c - floor(c);
  double sv, cv;
  sincospi(2.0 * r, &sv, &cv);
  return make_double2(cv, sign * sv);
}

// W[x][my][z] *= exp(sign * i Ky s x)  (sign -1: map to the shearing frame, +1: back)
__global__ void k_plain_remap(double2* __restrict__ W, BoxGeom g, const SolveScalars* __restrict__ sp, int sign) {
  const int hy = g.ny / 2;
  const size_t n = (size_t)g.nx * hy * g.nz;
  const double fy = sp->fy;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t r = i / g.nz;
    const int my = (int)(r % hy), x = (int)(r / hy);
    const double2 f = remap_factor(my, x, fy, sign);
    const double2 v = W[i];
    W[i] = make_double2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
  }
}

// P[x][my][0..M) = [W[x][my][0..nz), 0...]
__global__ void k_plain_pad(const double2* __restrict__ W, double2* __restrict__ P, BoxGeom g) {
  const size_t n = (size_t)g.nx * (g.ny / 2) * g.m;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t pencil = i / g.m;
    const int z = (int)(i - pencil * g.m);
    P[i] = z < g.nz ? W[pencil * g.nz + z] : make_double2(0.0, 0.0);
  }
}

// W[x][my][z] = P[x][my][z], z < nz
__global__ void k_plain_extract(const double2* __restrict__ P, double2* __restrict__ W, BoxGeom g) {
  const size_t n = (size_t)g.nx * (g.ny / 2) * g.nz;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t pencil = i / g.nz;
    const int z = (int)(i - pencil * g.nz);
    W[i] = P[pencil * g.m + z];
  }
}

// P *= 4 pi G/(Nx Ny M) * G(k, kz), k from the sheared wave vector (Sect. 2.1, 2.3, Eq. 2)
__global__ void k_plain_green(double2* __restrict__ P, BoxGeom g, const SolveScalars* __restrict__ sp,
                              const double* __restrict__ s2t, const double* __restrict__ kst,
                              const double* __restrict__ kz2t) {
  const int hy = g.ny / 2;
  const size_t n = (size_t)g.nx * hy * g.m;
  const double two_pi = 6.283185307179586476925286766559;
  const double s = sp->s, scale = sp->scale, L = g.L;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t pencil = i / g.m;
    const int mz = (int)(i - pencil * g.m);
    const int my = (int)(pencil % hy), mx = (int)(pencil / hy);
    const int sx = mx < g.nx / 2 ? mx : mx - g.nx;
    const double Ky = (two_pi / g.ly) * my;
    const double kx = (two_pi / g.lx) * sx + s * Ky;
    const double k2 = kx * kx + Ky * Ky;
    const bool zero = (mx == 0 && my == 0);
    double gk;
    if (g.method == 1) {
      gk = (zero && mz == 0) ? 0.0 : -1.0 / (k2 + kz2t[mz]);
    } else if (!zero) {
      const double k = sqrt(k2);
      const double e = exp(-k * L);
      gk = -(-expm1(-k * L) + e * (s2t[mz] + kst[mz] / k)) / (k2 + kz2t[mz]);
    } else {
      gk = mz == 0 ? 0.5 * L * L : (L * kst[mz] - s2t[mz]) / kz2t[mz];
    }
    gk *= scale;
    const double2 v = P[i];
    P[i] = make_double2(v.x * gk, v.y * gk);
  }
}

// SASHA reductions: per-block sums of rho and z*rho (block b covers a strided subset)
__global__ void k_plain_reduce(const double* __restrict__ rho, BoxGeom g, double* __restrict__ partials) {
  __shared__ double red[2][kEw];
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const double dz = g.lz / g.nz;
  double a = 0.0, b = 0.0;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const int z = (int)(i % g.nz);
    const double v = rho[i];
    a += v;
    b += (-0.5 * g.lz + (z + 0.5) * dz) * v;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = kEw / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = red[0][0];
    partials[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_plain_coef(const double* __restrict__ partials, int np, BoxGeom g,
                             const SolveScalars* __restrict__ sp, SashaCoef* __restrict__ coef) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < np; ++i) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  SashaCoef c;
  c.c2 = 0.0;
  c.c1 = 0.0;
  if (a != 0.0) {
    const double mean = a / ((double)g.nx * g.ny * g.m);
    c.c2 = 0.5 * sp->fourpiG * mean;
    c.c1 = -sp->fourpiG * mean * (b / a);
  }
  *coef = c;
}

__global__ void k_plain_phi0(double* __restrict__ phi, BoxGeom g, const SashaCoef* __restrict__ coef) {
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const double dz = g.lz / g.nz;
  const double c2 = coef->c2, c1 = coef->c1;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const int z = (int)(i % g.nz);
    const double zc = -0.5 * g.lz + (z + 0.5) * dz;
    phi[i] += (c2 * zc + c1) * zc;
  }
}

// contiguous length-M pencils, PP per workgroup
template <int M> constexpr int zplain_pp() {
  constexpr int pp = 16384 / (M * 16);
  return pp < 1 ? 1 : pp;
}

template <int M, int D>
__global__ __launch_bounds__(256) void k_plain_zfft(double2* __restrict__ P, const double2* __restrict__ tw, int npencils) {
  constexpr int PP = zplain_pp<M>();
  using L = Tile<PP, 1, M, false>;
  __shared__ double2 tile[lds_slots(PP * M)];
  const int p0 = blockIdx.x * PP;
  const int nvalid = min(PP, npencils - p0);
  double2* base = P + (size_t)p0 * M;
  for (int w = threadIdx.x; w < PP * M; w += 256)
    tile[L::at(w % M, w / M)] = w < nvalid * M ? base[w] : make_double2(0.0, 0.0);
  __syncthreads();
  lds_fft<double, M, L, 256, D>(tile, tw, threadIdx.x);
  for (int w = threadIdx.x; w < nvalid * M; w += 256) base[w] = tile[L::at(w % M, w / M)];
}

hipError_t launch_zfft_plain(int dir, const BoxGeom& g, double* P, const void* tw_m, hipStream_t st) {
  const int np = g.nx * (g.ny / 2);
#define SBP_CASE(N_)                                                                                    \
  if (g.m == N_) {                                                                                      \
    constexpr int PP = zplain_pp<N_>();                                                                 \
    dim3 grid((np + PP - 1) / PP);                                                                      \
    if (dir < 0)                                                                                        \
      hipLaunchKernelGGL((k_plain_zfft<N_, -1>), grid, dim3(256), 0, st, (double2*)P, (const double2*)tw_m, np); \
    else                                                                                                \
      hipLaunchKernelGGL((k_plain_zfft<N_, +1>), grid, dim3(256), 0, st, (double2*)P, (const double2*)tw_m, np); \
    return hipGetLastError();                                                                           \
  }
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

static int ew_blocks(size_t n) {
  size_t b = (n + kEw - 1) / kEw;
  return (int)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

#define PLAIN_STEP(name, call)             \
  do {                                     \
    if (mark) mark(mark_ctx, name);        \
    call;                                  \
    hipError_t e_ = hipGetLastError();     \
    if (e_ != hipSuccess) return e_;       \
  } while (0)

hipError_t launch_plain(const BoxGeom& g, const double* rho, double* phi, double* work_pad, double* work_half,
                        const void* tw_x, const void* tw_y, const void* tw_m, const double* zt_s2,
                        const double* zt_ks, const double* zt_kz2, const SolveScalars* sp, double* partials,
                        SashaCoef* coef, hipStream_t st, void (*mark)(void*, const char*), void* mark_ctx) {
  const size_t nhalf = (size_t)g.nx * (g.ny / 2) * g.nz;
  const size_t npad = (size_t)g.nx * (g.ny / 2) * g.m;
  double2* W = (double2*)work_half;
  double2* P = (double2*)work_pad;
  BoxGeom gp = g;  // the padded spectrum seen as a box with nz = M
  gp.nz = g.m;
  if (g.method == 1) {
    PLAIN_STEP("plain_reduce",
               hipLaunchKernelGGL(k_plain_reduce, dim3(kPlainPartials), dim3(kEw), 0, st, rho, g, partials));
    PLAIN_STEP("plain_coef", hipLaunchKernelGGL(k_plain_coef, dim3(1), dim3(64), 0, st, (const double*)partials,
                                                kPlainPartials, g, sp, coef));
  }
  PLAIN_STEP("plain_y_forward", { hipError_t e = launch_y_plain(-1, g, rho, work_half, tw_y, st); if (e) return e; });
  PLAIN_STEP("plain_remap", hipLaunchKernelGGL(k_plain_remap, dim3(ew_blocks(nhalf)), dim3(kEw), 0, st, W, g, sp, -1));
  PLAIN_STEP("plain_pad", hipLaunchKernelGGL(k_plain_pad, dim3(ew_blocks(npad)), dim3(kEw), 0, st, (const double2*)W, P, g));
  PLAIN_STEP("plain_x_forward", { hipError_t e = launch_x(0, -1, gp, P, tw_x, st); if (e) return e; });
  PLAIN_STEP("plain_z_forward", { hipError_t e = launch_zfft_plain(-1, g, work_pad, tw_m, st); if (e) return e; });
  PLAIN_STEP("plain_green", hipLaunchKernelGGL(k_plain_green, dim3(ew_blocks(npad)), dim3(kEw), 0, st, P, g, sp,
                                               zt_s2, zt_ks, zt_kz2));
  PLAIN_STEP("plain_z_inverse", { hipError_t e = launch_zfft_plain(+1, g, work_pad, tw_m, st); if (e) return e; });
  PLAIN_STEP("plain_x_inverse", { hipError_t e = launch_x(0, +1, gp, P, tw_x, st); if (e) return e; });
  PLAIN_STEP("plain_extract", hipLaunchKernelGGL(k_plain_extract, dim3(ew_blocks(nhalf)), dim3(kEw), 0, st,
                                                 (const double2*)P, W, g));
  PLAIN_STEP("plain_unremap", hipLaunchKernelGGL(k_plain_remap, dim3(ew_blocks(nhalf)), dim3(kEw), 0, st, W, g, sp, +1));
  PLAIN_STEP("plain_y_inverse", { hipError_t e = launch_y_plain(+1, g, work_half, phi, tw_y, st); if (e) return e; });
  if (g.method == 1)
    PLAIN_STEP("plain_phi0", hipLaunchKernelGGL(k_plain_phi0, dim3(ew_blocks(nhalf * 2)), dim3(kEw), 0, st, phi, g,
                                                (const SashaCoef*)coef));
  if (mark) mark(mark_ctx, nullptr);
  return hipSuccess;
}

}  // namespace sbp
