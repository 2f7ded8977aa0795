// y passes of the streaming solve.
//
// Forward (steps a1 + a7): one workgroup per (x plane, chunk of ZC consecutive z cells).  The
// real tile rho[x][0..Ny)[z0..z0+ZC) is read with z fastest (ZC*w = 128 bytes per row where
// the tile fits); consecutive z pairs (z, z+1) are packed as one complex column, so one
// complex length-Ny FFT transforms two real columns.  The two half spectra are separated,
// multiplied by the remap phase exp(-i Ky s x_i) that maps the density to the shearing frame
// (Sect. 2.1), and stored for my < Ny/2 (the Nyquist row is dropped).  For SASHA the
// workgroup also accumulates sum(rho) and sum(z rho) in double.
//
// Inverse (step a6, last part): the same tile shape in reverse: half spectra for my < Ny/2
// times the reverse-mapping phase exp(+i Ky s x_i), rebuilt into two Hermitian columns packed
// as one complex signal, one complex inverse FFT, real/imaginary parts written as z and z+1,
// plus Phi_0(z) for SASHA.
#include "fft_device.hpp"
#include "sbp_internal.hpp"

namespace sbp {

// real z cells per tile: 128-byte rows while the tile stays within 64 KiB
template <typename T, int N> constexpr int y_zc() {
  return sizeof(T) == 4 ? (N <= 512 ? 32 : 16) : (N <= 512 ? 16 : 8);
}
constexpr int kYThreads = 256;

// remap phase exp(-i 2 pi c) for c = my*(2x+1)*fy cycles, evaluated in double
__device__ __forceinline__ void remap_phase(int my, int x, double fy, double& cs, double& sn) {
  const double c = static_cast<double>(my * (2 * x + 1)) * fy;
  const double r = c - floor(c);
  double sv, cv;
  sincospi(2.0 * r, &sv, &cv);
  cs = cv;
  sn = -sv;
}

// load 2 consecutive complex pairs (4 reals) or 1 pair; v[0..n) valid
template <typename T> struct Vec2c;
template <> struct Vec2c<float> {
  static constexpr int K = 2;  // complex values per 16-byte access
  static __device__ __forceinline__ void ld(const float* p, float2* v) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = make_float2(q.x, q.y);
    v[1] = make_float2(q.z, q.w);
  }
  static __device__ __forceinline__ void st(float* p, const float2* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
  }
};
template <> struct Vec2c<double> {
  static constexpr int K = 1;
  static __device__ __forceinline__ void ld(const double* p, double2* v) { v[0] = *reinterpret_cast<const double2*>(p); }
  static __device__ __forceinline__ void st(double* p, const double2* v) { *reinterpret_cast<double2*>(p) = v[0]; }
};

template <typename T, int NY, bool REMAP = true>
__global__ __launch_bounds__(kYThreads) void k_yfwd(const T* __restrict__ rho, cplx<T>* __restrict__ W,
                                                    const cplx<T>* __restrict__ twg, const SolveScalars* __restrict__ sp,
                                                    BoxGeom g, double* __restrict__ partials) {
  constexpr int ZC = y_zc<T, NY>();
  constexpr int NB = ZC / 2;  // complex columns
  constexpr int NT = kYThreads;
  using L = Tile<NB, NB, 1, true>;
  __shared__ cplx<T> tile[lds_slots(NY * NB)];
  __shared__ cplx<T> tw[NY];
  __shared__ cplx<T> ph[NY / 2];
  __shared__ double red[2][NT / 64];

  const int tid = threadIdx.x;
  const int nzc = (g.nz + ZC - 1) / ZC;
  const int tile_id = xcd_tile(blockIdx.x, g.nx * nzc);
  const int x = tile_id / nzc;
  const int z0 = (tile_id - x * nzc) * ZC;
  const int nz = g.nz;
  const int hy = NY / 2;

  load_twiddles<T, NY, NT>(tw, twg, tid);
  double s0 = 0.0, s1 = 0.0;
  const double dz = g.lz / nz;
  // load: NY rows of ZC reals, z fastest, 16-byte accesses where aligned
  constexpr int K = Vec2c<T>::K;
  const bool vec = (nz % (2 * K)) == 0;
  const int kk = vec ? K : 1;
  for (int w = tid; w < NY * NB / kk; w += NT) {
    const int c = (w % (NB / kk)) * kk, y = w / (NB / kk);
    const int z = z0 + 2 * c;
    cplx<T> v[K];
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = mk<T>(T(0), T(0));
    if (z < nz) {
      const T* src = rho + ((size_t)x * NY + y) * nz + z;
      if (vec)
        Vec2c<T>::ld(src, v);
      else
        v[0] = *reinterpret_cast<const cplx<T>*>(src);
      if (partials) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          if (i >= kk) break;
          const double za = -0.5 * g.lz + (z + 2 * i + 0.5) * dz;
          const double a = (double)v[i].x, b = (double)v[i].y;
          s0 += a + b;
          s1 += za * a + (za + dz) * b;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i < kk) tile[L::at(y, c + i)] = v[i];
  }
  if (REMAP) {
    const double fy = sp->fy;
    for (int my = tid; my < hy; my += NT) {
      double cs, sn;
      remap_phase(my, x, fy, cs, sn);
      ph[my] = mk<T>((T)cs, (T)sn);
    }
  }
  if (partials) {
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_down(s0, o);
      s1 += __shfl_down(s1, o);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = s0;
      red[1][tid >> 6] = s1;
    }
  }
  __syncthreads();
  if (partials && tid == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < NT / 64; ++i) {
      a += red[0][i];
      b += red[1][i];
    }
    const size_t slot = (size_t)(z0 / ZC) * g.nx + x;
    partials[2 * slot] = a;
    partials[2 * slot + 1] = b;
  }

  lds_fft<T, NY, L, NT, -1>(tile, tw, tid);

  // separate the two real columns, remap, store my < NY/2 (16-byte stores: A and B adjacent)
  for (int w = tid; w < hy * NB; w += NT) {
    const int c = w % NB, ky = w / NB;
    const int z = z0 + 2 * c;
    if (z >= nz) continue;
    const cplx<T> c1 = tile[L::at(ky, c)];
    const cplx<T> c2 = tile[L::at((NY - ky) % NY, c)];
    cplx<T> ab[2];
    ab[0] = mk<T>(T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y));
    ab[1] = mk<T>(T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x));
    if (REMAP) {
      const cplx<T> p = ph[ky];
      ab[0] = cmul<T>(ab[0], p);
      ab[1] = cmul<T>(ab[1], p);
    }
    T* dst = reinterpret_cast<T*>(W + ((size_t)x * hy + ky) * nz + z);
    if constexpr (sizeof(T) == 4) {
      Vec2c<float>::st(reinterpret_cast<float*>(dst), reinterpret_cast<const float2*>(ab));
    } else {
      reinterpret_cast<cplx<T>*>(dst)[0] = ab[0];
      reinterpret_cast<cplx<T>*>(dst)[1] = ab[1];
    }
  }
}

template <typename T, int NY, bool REMAP = true>
__global__ __launch_bounds__(kYThreads) void k_yinv(const cplx<T>* __restrict__ W, T* __restrict__ phi,
                                                    const cplx<T>* __restrict__ twg, const SolveScalars* __restrict__ sp,
                                                    BoxGeom g, const SashaCoef* __restrict__ coef) {
  constexpr int ZC = y_zc<T, NY>();
  constexpr int NB = ZC / 2;
  constexpr int NT = kYThreads;
  using L = Tile<NB, NB, 1, true>;
  __shared__ cplx<T> tile[lds_slots(NY * NB)];
  __shared__ cplx<T> tw[NY];
  __shared__ cplx<T> ph[NY / 2];

  const int tid = threadIdx.x;
  const int nzc = (g.nz + ZC - 1) / ZC;
  const int tile_id = xcd_tile(blockIdx.x, g.nx * nzc);
  const int x = tile_id / nzc;
  const int z0 = (tile_id - x * nzc) * ZC;
  const int nz = g.nz;
  const int hy = NY / 2;

  load_twiddles<T, NY, NT>(tw, twg, tid);
  if (REMAP) {
    const double fy = sp->fy;
    for (int my = tid; my < hy; my += NT) {
      double cs, sn;
      remap_phase(my, x, fy, cs, sn);
      ph[my] = mk<T>((T)cs, (T)sn);  // exp(-i theta); used conjugated below
    }
  }
  for (int c = tid; c < NB; c += NT) tile[L::at(hy, c)] = mk<T>(T(0), T(0));  // y Nyquist
  __syncthreads();

  for (int w = tid; w < hy * NB; w += NT) {
    const int c = w % NB, ky = w / NB;
    const int z = z0 + 2 * c;
    cplx<T> a = mk<T>(T(0), T(0)), b = a;
    if (z < nz) {
      const cplx<T>* src = W + ((size_t)x * hy + ky) * nz + z;
      if constexpr (sizeof(T) == 4) {
        cplx<T> ab[2];
        Vec2c<float>::ld(reinterpret_cast<const float*>(src), reinterpret_cast<float2*>(ab));
        a = ab[0];
        b = ab[1];
      } else {
        a = src[0];
        b = src[1];
      }
      if (REMAP) {
        a = cmulc<T>(a, ph[ky]);
        b = cmulc<T>(b, ph[ky]);
      }
    }
    if (ky == 0) {
      tile[L::at(0, c)] = mk<T>(a.x, b.x);  // the DC terms of real columns are real
    } else {
      tile[L::at(ky, c)] = mk<T>(a.x - b.y, a.y + b.x);         // A + iB
      tile[L::at(NY - ky, c)] = mk<T>(a.x + b.y, b.x - a.y);    // conj(A) + i conj(B)
    }
  }
  __syncthreads();

  lds_fft<T, NY, L, NT, +1>(tile, tw, tid);

  const bool sasha = coef != nullptr;
  double c2 = 0.0, c1 = 0.0;
  if (sasha) {
    c2 = coef->c2;
    c1 = coef->c1;
  }
  const double dz = g.lz / nz;
  constexpr int K = Vec2c<T>::K;
  const bool vec = (nz % (2 * K)) == 0;
  const int kk = vec ? K : 1;
  auto finish = [&](cplx<T> v, int z) {
    if (sasha) {
      const double za = -0.5 * g.lz + (z + 0.5) * dz;
      const double zb = za + dz;
      v.x = (T)((double)v.x + (c2 * za + c1) * za);
      v.y = (T)((double)v.y + (c2 * zb + c1) * zb);
    }
    return v;
  };
  for (int w = tid; w < NY * NB / kk; w += NT) {
    const int c = (w % (NB / kk)) * kk, y = w / (NB / kk);
    const int z = z0 + 2 * c;
    if (z >= nz) continue;
    T* dst = phi + ((size_t)x * NY + y) * nz + z;
    if (K == 2 && vec) {
      cplx<T> v[K];
      v[0] = finish(tile[L::at(y, c)], z);
      v[K - 1] = finish(tile[L::at(y, c + 1)], z + 2);
      Vec2c<T>::st(dst, v);
    } else {
      *reinterpret_cast<cplx<T>*>(dst) = finish(tile[L::at(y, c)], z);
    }
  }
}

template <typename T, int NY, bool REMAP>
static dim3 y_grid(const BoxGeom& g) {
  constexpr int ZC = y_zc<T, NY>();
  return dim3(g.nx * ((g.nz + ZC - 1) / ZC));
}

template <typename T, int NY>
static hipError_t yfwd_t(const BoxGeom& g, const void* rho, void* W, const void* tw, const SolveScalars* sp,
                         double* partials, hipStream_t st) {
  const dim3 grid = y_grid<T, NY, true>(g);
  hipLaunchKernelGGL((k_yfwd<T, NY>), grid, dim3(kYThreads), 0, st, (const T*)rho, (cplx<T>*)W,
                     (const cplx<T>*)tw, sp, g, partials);
  return hipGetLastError();
}

template <typename T, int NY>
static hipError_t yinv_t(const BoxGeom& g, const void* W, void* phi, const void* tw, const SolveScalars* sp,
                         const SashaCoef* coef, hipStream_t st) {
  const dim3 grid = y_grid<T, NY, true>(g);
  hipLaunchKernelGGL((k_yinv<T, NY>), grid, dim3(kYThreads), 0, st, (const cplx<T>*)W, (T*)phi,
                     (const cplx<T>*)tw, sp, g, coef);
  return hipGetLastError();
}

// plain path: y transforms without the remap (it runs as a separate kernel there)
hipError_t launch_y_plain(int dir, const BoxGeom& g, const double* in, double* out, const void* tw_y, hipStream_t st) {
#define SBP_CASE(N_)                                                                                      \
  if (g.ny == N_) {                                                                                       \
    const dim3 grid = y_grid<double, N_, false>(g);                                                       \
    if (dir < 0)                                                                                          \
      hipLaunchKernelGGL((k_yfwd<double, N_, false>), grid, dim3(kYThreads), 0, st, in, (double2*)out,    \
                         (const double2*)tw_y, (const SolveScalars*)nullptr, g, (double*)nullptr);        \
    else                                                                                                  \
      hipLaunchKernelGGL((k_yinv<double, N_, false>), grid, dim3(kYThreads), 0, st, (const double2*)in,   \
                         out, (const double2*)tw_y, (const SolveScalars*)nullptr, g, (const SashaCoef*)nullptr); \
    return hipGetLastError();                                                                             \
  }
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

int yfwd_partials(int prec, const BoxGeom& g) {
  int zc = 0;
#define SBP_CASE(N_) \
  if (g.ny == N_) zc = prec ? y_zc<float, N_>() : y_zc<double, N_>();
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  if (zc == 0) return 0;
  return g.nx * ((g.nz + zc - 1) / zc);
}

hipError_t launch_yfwd(int prec, const BoxGeom& g, const void* rho, void* W, const void* tw_y,
                       const SolveScalars* sp, double* partials, hipStream_t st) {
#define SBP_CASE(N_)                                                                  \
  if (g.ny == N_) return prec ? yfwd_t<float, N_>(g, rho, W, tw_y, sp, partials, st) \
                              : yfwd_t<double, N_>(g, rho, W, tw_y, sp, partials, st);
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_yinv(int prec, const BoxGeom& g, const void* W, void* phi, const void* tw_y,
                       const SolveScalars* sp, const SashaCoef* coef, hipStream_t st) {
#define SBP_CASE(N_)                                                             \
  if (g.ny == N_) return prec ? yinv_t<float, N_>(g, W, phi, tw_y, sp, coef, st) \
                              : yinv_t<double, N_>(g, W, phi, tw_y, sp, coef, st);
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

}  // namespace sbp
