// Plain FP64 path: the same discrete operator with one kernel per step and the zero-padded
// spectrum materialised in HBM.  It is the unfused reference the streaming passes are measured
// against: y transform, remap, zero padding, x transform, z transform, Green multiply, z and x
// inverse transforms, extraction, reverse remap, inverse y transform, SASHA Phi_0.
// Per-solve values are read from the device box record, so graph replay stays valid.
#include "passes.hpp"

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
__global__ void k_plain_remap(const BoxRec* __restrict__ rec, int sign) {
  const BoxGeom g = rec->g;
  double2* W = static_cast<double2*>(rec->W);
  const int hy = g.ny / 2;
  const size_t n = (size_t)g.nx * hy * g.nz;
  const double fy = rec->fy;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t r = i / g.nz;
    const int my = (int)(r % hy), x = (int)(r / hy);
    const double2 f = remap_factor(my, x, fy, sign);
    const double2 v = W[i];
    W[i] = make_double2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
  }
}

// P[x][my][0..M) = [W[x][my][0..nz), 0...]
__global__ void k_plain_pad(const BoxRec* __restrict__ rec, const BoxRec* __restrict__ pad) {
  const BoxGeom g = rec->g;
  const double2* W = static_cast<const double2*>(rec->W);
  double2* P = static_cast<double2*>(pad->W);
  const size_t n = (size_t)g.nx * (g.ny / 2) * g.m;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t pencil = i / g.m;
    const int z = (int)(i - pencil * g.m);
    P[i] = z < g.nz ? W[pencil * g.nz + z] : make_double2(0.0, 0.0);
  }
}

// W[x][my][z] = P[x][my][z], z < nz
__global__ void k_plain_extract(const BoxRec* __restrict__ rec, const BoxRec* __restrict__ pad) {
  const BoxGeom g = rec->g;
  double2* W = static_cast<double2*>(rec->W);
  const double2* P = static_cast<const double2*>(pad->W);
  const size_t n = (size_t)g.nx * (g.ny / 2) * g.nz;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const size_t pencil = i / g.nz;
    const int z = (int)(i - pencil * g.nz);
    W[i] = P[pencil * g.m + z];
  }
}

// P *= 4 pi G/(Nx Ny M) * G(k, kz), k from the sheared wave vector (Sect. 2.1, 2.3, Eq. 2)
__global__ void k_plain_green(const BoxRec* __restrict__ rec, const BoxRec* __restrict__ pad) {
  const BoxGeom g = rec->g;
  double2* P = static_cast<double2*>(pad->W);
  const double* s2t = rec->zt64[0];
  const double* kst = rec->zt64[1];
  const double* kz2t = rec->zt64[2];
  const int hy = g.ny / 2;
  const size_t n = (size_t)g.nx * hy * g.m;
  const double two_pi = 6.283185307179586476925286766559;
  const double s = rec->s, scale = rec->scale, L = g.L;
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
__global__ void k_plain_reduce(const BoxRec* __restrict__ rec) {
  __shared__ double red[2][kEw];
  lds_poison(red);
  const BoxGeom g = rec->g;
  const double* rho = static_cast<const double*>(rec->rho);
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
    rec->partials[2 * blockIdx.x] = red[0][0];
    rec->partials[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_plain_coef(const BoxRec* __restrict__ rec) {
  if (threadIdx.x != 0) return;
  const BoxGeom g = rec->g;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < kPlainPartials; ++i) {
    a += rec->partials[2 * i];
    b += rec->partials[2 * i + 1];
  }
  SashaCoef c;
  c.c2 = 0.0;
  c.c1 = 0.0;
  if (a != 0.0) {
    const double mean = a / ((double)g.nx * g.ny * g.m);
    c.c2 = 0.5 * rec->fourpiG * mean;
    c.c1 = -rec->fourpiG * mean * (b / a);
  }
  *rec->coef = c;
}

__global__ void k_plain_phi0(const BoxRec* __restrict__ rec) {
  const BoxGeom g = rec->g;
  double* phi = static_cast<double*>(rec->phi);
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const double dz = g.lz / g.nz;
  const double c2 = rec->coef->c2, c1 = rec->coef->c1;
  for (size_t i = blockIdx.x * (size_t)kEw + threadIdx.x; i < n; i += (size_t)gridDim.x * kEw) {
    const int z = (int)(i % g.nz);
    const double zc = -0.5 * g.lz + (z + 0.5) * dz;
    phi[i] += (c2 * zc + c1) * zc;
  }
}

// contiguous length-M pencils of the padded spectrum, PP per workgroup
template <int M> constexpr int zplain_pp() {
  constexpr int pp = 16384 / (M * 16);
  return pp < 1 ? 1 : pp;
}

template <int M, int D>
__global__ __launch_bounds__(256) void k_plain_zfft(const BoxRec* __restrict__ pad, const double2* __restrict__ tw) {
  constexpr int PP = zplain_pp<M>();
  using L = Tile<PP, 1, M, false>;
  __shared__ double2 buf[lds_slots(PP * M)];
  lds_poison(buf);
  const BoxGeom g = pad->g;
  const int npencils = g.nx * (g.ny / 2);
  const int p0 = blockIdx.x * PP;
  const int nvalid = min(PP, npencils - p0);
  double2* base = static_cast<double2*>(pad->W) + (size_t)p0 * M;
  fft_run<double, M, typename Fwd<M>::L, L, 256, D, false, false>(
      buf, tw, threadIdx.x,
      [&](int e, int p) { return p < nvalid ? base[(size_t)p * M + e] : make_double2(0.0, 0.0); },
      [&](int e, int p, double2 v) {
        if (p < nvalid) base[(size_t)p * M + e] = v;
      });
}

static hipError_t zfft_plain(int dir, const BoxGeom& g, const BoxRec* pad, const void* tw_m, hipStream_t st) {
  const int np = g.nx * (g.ny / 2);
#define SBP_CASE(N_)                                                                                 \
  if (g.m == N_) {                                                                                   \
    constexpr int PP = zplain_pp<N_>();                                                              \
    const dim3 grid((np + PP - 1) / PP);                                                             \
    if (dir < 0)                                                                                     \
      hipLaunchKernelGGL((k_plain_zfft<N_, -1>), grid, dim3(256), 0, st, pad, (const double2*)tw_m); \
    else                                                                                             \
      hipLaunchKernelGGL((k_plain_zfft<N_, +1>), grid, dim3(256), 0, st, pad, (const double2*)tw_m); \
    return hipGetLastError();                                                                        \
  }
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

static int ew_blocks(size_t n) {
  size_t b = (n + kEw - 1) / kEw;
  return (int)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

#define PLAIN_STEP(name, call)         \
  do {                                 \
    if (mark) mark(mark_ctx, name);    \
    call;                              \
    hipError_t e_ = hipGetLastError(); \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

hipError_t launch_plain(const BoxRec* h_rec, const BoxRec* rec, const BoxRec* pad, GroupArgs one, int y_var, int x_var,
                        const void* tws_x, const void* tws_y, const void* tw_m, hipStream_t st,
                        void (*mark)(void*, const char*), void* mark_ctx) {
  const BoxGeom& g = h_rec->g;
  const size_t nhalf = (size_t)g.nx * (g.ny / 2) * g.nz;
  const size_t npad = (size_t)g.nx * (g.ny / 2) * g.m;
  BoxGeom gp = g;  // the padded spectrum seen as a box with nz = M
  gp.nz = g.m;
  const int yb = y_tiles(0, g, y_var), xb = x_tiles(0, gp, x_var);
  // `one`: box ids {0}; starts {0, y blocks} at [0..1] and {0, x blocks} at [2..3]
  GroupArgs gy = one, gx = one;
  gx.starts = one.starts + 2;
  gy.total = yb;
  gx.total = xb;
  if (g.method == 1) {
    PLAIN_STEP("plain_reduce", hipLaunchKernelGGL(k_plain_reduce, dim3(kPlainPartials), dim3(kEw), 0, st, rec));
    PLAIN_STEP("plain_coef", hipLaunchKernelGGL(k_plain_coef, dim3(1), dim3(64), 0, st, rec));
  }
  PLAIN_STEP("plain_y_forward", {
    hipError_t e = launch_y(0, true, false, g.ny, y_var, gy, yb, rec, tws_y, st);
    if (e) return e;
  });
  PLAIN_STEP("plain_remap", hipLaunchKernelGGL(k_plain_remap, dim3(ew_blocks(nhalf)), dim3(kEw), 0, st, rec, -1));
  PLAIN_STEP("plain_pad", hipLaunchKernelGGL(k_plain_pad, dim3(ew_blocks(npad)), dim3(kEw), 0, st, rec, pad));
  PLAIN_STEP("plain_x_forward", {
    hipError_t e = launch_x(0, -1, g.nx, x_var, gx, xb, pad, tws_x, st);
    if (e) return e;
  });
  PLAIN_STEP("plain_z_forward", {
    hipError_t e = zfft_plain(-1, g, pad, tw_m, st);
    if (e) return e;
  });
  PLAIN_STEP("plain_green", hipLaunchKernelGGL(k_plain_green, dim3(ew_blocks(npad)), dim3(kEw), 0, st, rec, pad));
  PLAIN_STEP("plain_z_inverse", {
    hipError_t e = zfft_plain(+1, g, pad, tw_m, st);
    if (e) return e;
  });
  PLAIN_STEP("plain_x_inverse", {
    hipError_t e = launch_x(0, +1, g.nx, x_var, gx, xb, pad, tws_x, st);
    if (e) return e;
  });
  PLAIN_STEP("plain_extract", hipLaunchKernelGGL(k_plain_extract, dim3(ew_blocks(nhalf)), dim3(kEw), 0, st, rec, pad));
  PLAIN_STEP("plain_unremap", hipLaunchKernelGGL(k_plain_remap, dim3(ew_blocks(nhalf)), dim3(kEw), 0, st, rec, +1));
  PLAIN_STEP("plain_y_inverse", {
    hipError_t e = launch_y(0, false, false, g.ny, y_var, gy, yb, rec, tws_y, st);
    if (e) return e;
  });
  if (g.method == 1)
    PLAIN_STEP("plain_phi0", hipLaunchKernelGGL(k_plain_phi0, dim3(ew_blocks(nhalf * 2)), dim3(kEw), 0, st, rec));
  if (mark) mark(mark_ctx, nullptr);
  return hipSuccess;
}

}  // namespace sbp
