// z pass of the streaming solve (steps a2-a5, and the SASHA coefficients of a7).
//
// One workgroup per PP consecutive (Kx, Ky) pencils.  Each pencil's Nz spectrum values are
// contiguous in W, so the tile load is one contiguous run of PP*Nz values.  In LDS the pencil
// is zero-padded to M = P*Nz (Hockney padding; the padded spectrum never reaches HBM),
// transformed forward, multiplied by the Green's function at the sheared wave vector
// k = |(Kx + s Ky, Ky)| (Sect. 2.1) times 4 pi G/(Nx Ny M), transformed back, and its first
// Nz values are stored in place.
//
// Green's function (Sect. 2.3, App. A), L = alpha Lz, with E = exp(-kL):
//   VGF, k > 0:  -(1 - E cos(kz L) + E (kz/k) sin(kz L)) / (k^2 + kz^2)
//                written as -((1 - E) + E (1 - cos(kz L)) + E (kz/k) sin(kz L)) / (k^2 + kz^2),
//                with 1 - E = -expm1(-kL) and 1 - cos(kz L) = 2 sin^2(kz L/2) taken from
//                accurate tables, so no term cancels;
//   VGF, k = 0:  (kz L sin(kz L) + cos(kz L) - 1) / kz^2, and L^2/2 at kz = 0;
//   SASHA:       -1/(k^2 + kz^2), and 0 for the zero mode (mean subtraction, Sect. 2.2).
// The per-pencil scalars (1 - E, E, 1/k, k^2, with the 4 pi G/(Nx Ny M) factor folded in) are
// evaluated in double and rounded once.  Float plans transform, multiply and transform back
// the k = 0 pencil (the horizontally averaged density, which carries most of the potential)
// entirely in double.
#include <type_traits>

#include "fft_device.hpp"
#include "sbp_internal.hpp"

namespace sbp {

template <typename T, int M> constexpr int z_pp() {
  constexpr int pp = 32768 / (M * 2 * (int)sizeof(T));
  return pp < 1 ? 1 : (pp > 32 ? 32 : pp);
}
constexpr int kZThreads = 256;

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

template <typename T, int M>
__global__ __launch_bounds__(kZThreads) void k_z(cplx<T>* __restrict__ W, const cplx<T>* __restrict__ twg,
                                                 const double2* __restrict__ tw64, ZTables<T> zt, ZTables<double> zt64,
                                                 const SolveScalars* __restrict__ sp, BoxGeom g,
                                                 const double* __restrict__ partials, int npartials,
                                                 SashaCoef* __restrict__ coef) {
  constexpr int PP = z_pp<T, M>();
  constexpr int NT = kZThreads;
  constexpr bool kF32 = std::is_same<T, float>::value;
  using L = Tile<PP, 1, M, false>;
  using L1 = Tile<1, 1, M, false>;
  __shared__ cplx<T> tile[lds_slots(PP * M)];
  __shared__ cplx<T> tw[M];
  __shared__ T pa0[PP], pe[PP], pik[PP], pk2[PP];
  __shared__ int pzero[PP];
  __shared__ double2 dbuf[kF32 ? lds_slots(M) : 1];  // float plans: the k = 0 pencil in double

  const int tid = threadIdx.x;
  const int hy = g.ny / 2;
  const int np = g.nx * hy;
  const int p0 = blockIdx.x * PP;
  const int nz = g.nz;
  const int nvalid = min(PP, np - p0);
  const bool sasha = g.method == 1;
  const double scale = sp->scale;

  load_twiddles<T, M, NT>(tw, twg, tid);
  // contiguous load of nvalid pencils (pairs of complex values: nz is even), then the padding
  const cplx<T>* src = W + (size_t)p0 * nz;
  for (int w = tid; w < nvalid * nz / 2; w += NT) {
    const int e = 2 * w;
    const int p = e / nz, z = e - p * nz;
    cplx<T> v0, v1;
    if constexpr (kF32) {
      const float4 q = *reinterpret_cast<const float4*>(src + e);
      v0 = mk<T>(q.x, q.y);
      v1 = mk<T>(q.z, q.w);
    } else {
      v0 = src[e];
      v1 = src[e + 1];
    }
    tile[L::at(z, p)] = v0;
    tile[L::at(z + 1, p)] = v1;
  }
  for (int w = tid; w < PP * (M - nz); w += NT) {
    const int p = w / (M - nz), z = nz + (w - p * (M - nz));
    tile[L::at(z, p)] = mk<T>(T(0), T(0));
  }
  for (int w = tid; w < (PP - nvalid) * nz; w += NT) {
    const int p = nvalid + w / nz, z = w % nz;
    tile[L::at(z, p)] = mk<T>(T(0), T(0));
  }
  if (tid < PP) {
    const int q = p0 + tid;
    const int mx = q / hy, my = q - mx * hy;
    const int sx = mx < g.nx / 2 ? mx : mx - g.nx;
    const double two_pi = 6.283185307179586476925286766559;
    const double Ky = (two_pi / g.ly) * my;
    const double kx = (two_pi / g.lx) * sx + sp->s * Ky;
    const double k2 = kx * kx + Ky * Ky;
    const double k = sqrt(k2);
    const int zero = (mx == 0 && my == 0);
    pzero[tid] = zero;
    pk2[tid] = (T)k2;
    if (!zero && !sasha) {
      pa0[tid] = (T)(-expm1(-k * g.L) * scale);
      pe[tid] = (T)(exp(-k * g.L) * scale);
      pik[tid] = (T)(1.0 / k);
    } else {
      pa0[tid] = T(0);
      pe[tid] = T(0);
      pik[tid] = T(0);
    }
  }

  // float plans: the k = 0 pencil in double (only block 0 holds it)
  if constexpr (kF32) {
    if (blockIdx.x == 0) {
      const float2* s0 = reinterpret_cast<const float2*>(W);
      for (int z = tid; z < M; z += NT) {
        double2 v;
        v.x = 0.0;
        v.y = 0.0;
        if (z < nz) {
          v.x = (double)s0[z].x;
          v.y = (double)s0[z].y;
        }
        dbuf[L1::at(z, 0)] = v;
      }
      __syncthreads();
      lds_fft<double, M, L1, NT, -1>(dbuf, tw64, tid);
      for (int mz = tid; mz < M; mz += NT) {
        double gk;
        if (sasha)
          gk = mz == 0 ? 0.0 : -1.0 / zt64.kz2[mz];
        else
          gk = mz == 0 ? 0.5 * g.L * g.L : (g.L * zt64.ks[mz] - zt64.s2[mz]) / zt64.kz2[mz];
        gk *= scale;
        dbuf[L1::at(mz, 0)].x *= gk;
        dbuf[L1::at(mz, 0)].y *= gk;
      }
      __syncthreads();
      lds_fft<double, M, L1, NT, +1>(dbuf, tw64, tid);
    }
  }

  // SASHA: <rho> and the centre of mass from the per-tile partial sums (fixed order)
  if (sasha && blockIdx.x == 0) {
    __shared__ double red[2][NT];
    double a = 0.0, b = 0.0;
    for (int i = tid; i < npartials; i += NT) {
      a += partials[2 * i];
      b += partials[2 * i + 1];
    }
    red[0][tid] = a;
    red[1][tid] = b;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (tid < o) {
        red[0][tid] += red[0][tid + o];
        red[1][tid] += red[1][tid + o];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double s0 = red[0][0], s1 = red[1][0];
      SashaCoef c;
      c.c2 = 0.0;
      c.c1 = 0.0;
      if (s0 != 0.0) {
        const double mean = s0 / ((double)g.nx * g.ny * g.m);
        const double zc = s1 / s0;
        c.c2 = 0.5 * sp->fourpiG * mean;
        c.c1 = -sp->fourpiG * mean * zc;
      }
      *coef = c;
    }
  }
  __syncthreads();

  lds_fft<T, M, L, NT, -1>(tile, tw, tid);

  // Green multiply: each thread owns kz values and walks the pencils of the tile
  const T L_ = (T)g.L;
  const T sc = (T)scale;
  for (int mz = tid; mz < M; mz += NT) {
    const T s2 = zt.s2[mz], ks = zt.ks[mz], kz2 = zt.kz2[mz];
#pragma unroll 4
    for (int p = 0; p < PP; ++p) {
      T gk;
      if (sasha) {
        gk = (pzero[p] && mz == 0) ? T(0) : -sc * fast_rcp(pk2[p] + kz2);
      } else if (!pzero[p]) {
        gk = -(pa0[p] + pe[p] * (s2 + pik[p] * ks)) * fast_rcp(pk2[p] + kz2);
      } else {
        gk = sc * (mz == 0 ? T(0.5) * L_ * L_ : (L_ * ks - s2) / kz2);
      }
      cplx<T>& v = tile[L::at(mz, p)];
      v.x *= gk;
      v.y *= gk;
    }
  }
  __syncthreads();

  lds_fft<T, M, L, NT, +1>(tile, tw, tid);

  cplx<T>* dst = W + (size_t)p0 * nz;
  for (int w = tid; w < nvalid * nz / 2; w += NT) {
    const int e = 2 * w;
    const int p = e / nz, z = e - p * nz;
    cplx<T> v0 = tile[L::at(z, p)], v1 = tile[L::at(z + 1, p)];
    if constexpr (kF32) {
      if (blockIdx.x == 0 && p == 0) {
        v0 = mk<T>((T)dbuf[L1::at(z, 0)].x, (T)dbuf[L1::at(z, 0)].y);
        v1 = mk<T>((T)dbuf[L1::at(z + 1, 0)].x, (T)dbuf[L1::at(z + 1, 0)].y);
      }
      *reinterpret_cast<float4*>(dst + e) = make_float4(v0.x, v0.y, v1.x, v1.y);
    } else {
      dst[e] = v0;
      dst[e + 1] = v1;
    }
  }
}

template <typename T, int M>
static hipError_t z_t(const BoxGeom& g, void* W, const void* tw, const void* tw64, ZTables<T> zt,
                      ZTables<double> zt64, const SolveScalars* sp, const double* partials, int npartials,
                      SashaCoef* coef, hipStream_t st) {
  constexpr int PP = z_pp<T, M>();
  const int np = g.nx * (g.ny / 2);
  dim3 grid((np + PP - 1) / PP);
  hipLaunchKernelGGL((k_z<T, M>), grid, dim3(kZThreads), 0, st, (cplx<T>*)W, (const cplx<T>*)tw,
                     (const double2*)tw64, zt, zt64, sp, g, partials, npartials, coef);
  return hipGetLastError();
}

hipError_t launch_z(int prec, const BoxGeom& g, void* W, const void* tw_m, const void* tw_m64, const void* zt_s2,
                    const void* zt_ks, const void* zt_kz2, const double* zt64_s2, const double* zt64_ks,
                    const double* zt64_kz2, const SolveScalars* sp, const double* partials, int npartials,
                    SashaCoef* coef, hipStream_t st) {
  ZTables<double> z64{zt64_s2, zt64_ks, zt64_kz2};
  if (prec) {
    ZTables<float> zf{(const float*)zt_s2, (const float*)zt_ks, (const float*)zt_kz2};
#define SBP_CASE(N_) \
  if (g.m == N_) return z_t<float, N_>(g, W, tw_m, tw_m64, zf, z64, sp, partials, npartials, coef, st);
    SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  } else {
#define SBP_CASE(N_) \
  if (g.m == N_) return z_t<double, N_>(g, W, tw_m, tw_m64, z64, z64, sp, partials, npartials, coef, st);
    SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace sbp
