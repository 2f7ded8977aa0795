// Streaming passes of the solve, written once for float and double and for several tile
// shapes ("variants", chosen per plan, optionally by the autotuner).  Each launch serves a
// group of boxes that share a kernel shape: block b of the launch finds its box by a search
// over the group's block offsets, so many boxes of uneven size run in a few launches.
//
//   y forward  (a1 + a7): rho -> half spectrum W[x][my][z] (my < Ny/2), remap phase applied
//   x          (a1 / a6): complex length-Nx transforms of W in place
//   z          (a2 - a5): zero padding, z transform, Green multiply, inverse, extraction
//   y inverse  (a6):      W -> phi, reverse remap, SASHA Phi_0
#pragma once

#include <type_traits>

#include "fft_device.hpp"
#include "sbp_internal.hpp"

namespace sbp {

// one row {1 - cos(kz L), kz sin(kz L), kz^2} of the z table: one 16-byte load in float, two in
// double
template <typename T> struct ZRow {
  T s2, ks, kz2;
};
__device__ __forceinline__ ZRow<float> zrow(gmem<const float>* t, int mz) {
  const float4 v = reinterpret_cast<gmem<const float4>*>(t)[mz];
  return {v.x, v.y, v.z};
}
__device__ __forceinline__ ZRow<double> zrow(gmem<const double>* t, int mz) {
  const double2 a = reinterpret_cast<gmem<const double2>*>(t)[2 * mz];
  const double b = t[4 * mz + 2];
  return {a.x, a.y, b};
}

// reciprocal: the hardware estimate in float (about 1 ulp), exact division in double
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// Green's-function coefficients of one horizontal mode (Sect. 2.3, App. A; SASHA Sect. 2.2),
// scaled by 4 pi G/(Nx Ny M): the multiplier at the z-table row {s2, ks, kz^2} is
//   G = -(a0 + e (s2 + ik ks)) / (k^2 + kz^2),
// and the one element whose denominator vanishes (k = 0, kz = 0) takes `zero` instead.
//   VGF, k > 0:  a0 = 1 - exp(-kL), e = exp(-kL), ik = 1/k      (the stable form of G^L)
//   VGF, k = 0:  a0 = 0, e = 1, ik = -L, zero = L^2/2           ((kz L sin kz L + cos kz L - 1)/kz^2)
//   SASHA:       a0 = 1, e = ik = 0, zero = 0                    (-1/|k|^2, the mean mode dropped)
template <typename T> struct ModeGreen {
  T a0, e, ik, k2, zero;
};
template <typename T>
__device__ __forceinline__ ModeGreen<T> mode_green(double kk2, bool k_zero, bool sasha, double L, double scale) {
  ModeGreen<T> c;
  c.k2 = (T)kk2;
  c.zero = T(0);
  if (sasha) {
    c.a0 = (T)scale;
    c.e = T(0);
    c.ik = T(0);
  } else if (!k_zero) {
    const double k = sqrt(kk2);
    c.a0 = (T)(-expm1(-k * L) * scale);
    c.e = (T)(exp(-k * L) * scale);
    c.ik = (T)(1.0 / k);
  } else {
    c.a0 = T(0);
    c.e = (T)scale;
    c.ik = (T)(-L);
    c.zero = (T)(0.5 * L * L * scale);
  }
  return c;
}
template <typename T>
__device__ __forceinline__ T green_at(T a0, T e, T ik, T k2, T zero, const ZRow<T>& zr) {
  const T den = k2 + zr.kz2;
  const T gk = -(a0 + e * (zr.s2 + ik * zr.ks)) * fast_rcp(den);
  return den == T(0) ? zero : gk;
}
// The same where the element with a zero denominator (Kx = Ky = kz = 0) is never used: float
// plans take the whole k = 0 pencil in double apart from the transforms.
template <typename T>
__device__ __forceinline__ T green_at_nonzero(T a0, T e, T ik, T k2, const ZRow<T>& zr) {
  return -(a0 + e * (zr.s2 + ik * zr.ks)) * fast_rcp(k2 + zr.kz2);
}

constexpr int kPassThreads = 256;
// threads of an x or y pass block: transforms of 512 points or more take 512 threads, so that the
// two or three blocks that fit a CU in LDS bring twice the wavefronts to its FFT stages
template <int N> constexpr int xy_threads() { return N >= 512 ? 512 : kPassThreads; }

// ------------------------------------------------------------------------------------------
// tile shapes per (precision, transform length, variant)

// y: real z cells per tile (even); variant 1 = 128-byte rows, variant 0 = half of that
template <typename T, int N, int V> constexpr int y_zc() {
  constexpr int big = sizeof(T) == 4 ? (N <= 512 ? 32 : 16) : (N <= 512 ? 16 : 8);
  return V ? big : big / 2;
}
// x: complex z cells per tile; float transforms of 1024 points take 128-byte rows in variant 1,
// whose 128 KB tile leaves room for one block per CU, made of 1024 threads
template <typename T, int N, int V> constexpr int x_zc() {
  constexpr int big = sizeof(T) == 4 ? (N <= 512 || (N == 1024 && V) ? 16 : 8) : (N <= 512 ? 8 : 4);
  return V ? big : big / 2;
}
template <typename T, int N, int V> constexpr int x_threads() {
  return (sizeof(T) == 4 && N == 1024 && V == 1) ? 1024 : xy_threads<N>();
}
// z: pencils one wavefront transforms side by side (about eight points per lane), pencils per
// wavefront (variant 1: four such groups, variant 0: two; at most 64), pencils per block
template <int M> constexpr int z_pw() { return M >= 512 ? 1 : 512 / M; }
template <int M, int V> constexpr int z_ppw() {
  constexpr int k = V ? 4 : 2;
  constexpr int cap = 64 / z_pw<M>() < 1 ? 1 : 64 / z_pw<M>();
  return z_pw<M>() * (k < cap ? k : cap);
}
template <typename T, int M, int V> constexpr int z_pp() { return (kPassThreads / 64) * z_ppw<M, V>(); }

// ------------------------------------------------------------------------------------------
// launch groups

// locate this block's box and its tile index within the box (XCD-aware order over the launch)
__device__ __forceinline__ const BoxRec* group_box(const GroupArgs& ga, const BoxRec* __restrict__ recs, int& tile) {
  const int b = xcd_tile(blockIdx.x, ga.total);
  if (ga.n == 1) {
    tile = b;
    return recs + ga.box0;
  }
  const int2 e = hbm(ga.blk)[b];
  tile = e.y;
  return recs + e.x;
}

// The record of this block's box for the first pass of a solve, as a value: from the launch
// arguments (block 0 publishing it to the device array for the later passes) or from that array.
__device__ __forceinline__ BoxRec first_pass_rec(const GroupArgs& ga, const BoxRec* __restrict__ recs, int& tile) {
  if (ga.use_arg) {
    tile = xcd_tile(blockIdx.x, ga.total);
    if (blockIdx.x == 0 && threadIdx.x == 0) *hbm(ga.pub) = ga.arg;
    return ga.arg;
  }
  return *hbm(group_box(ga, recs, tile));
}

// remap phase exp(-i 2 pi c) for c = my*(2x+1)*fy cycles, evaluated in double
__device__ __forceinline__ void remap_phase(int my, int x, double fy, double& cs, double& sn) {
  const double c = static_cast<double>(my * (2 * x + 1)) * fy;
  const double r = c - floor(c);
  double sv, cv;
  sincospi(2.0 * r, &sv, &cv);
  cs = cv;
  sn = -sv;
}

// Linear remap (Sect. 2.1, interpolation variant): row values sampled at the fractional y index
// j + d, periodic in n, as (1 - w) f[(j + m) mod n] + w f[(j + m + 1) mod n], m = floor(d).
struct YInterp {
  int m = 0;
  double w = 0.0;
  __device__ __forceinline__ void init(double d, int n) {
    const double fl = floor(d);
    w = d - fl;
    long long mm = static_cast<long long>(fl) % n;
    if (mm < 0) mm += n;
    m = static_cast<int>(mm);
  }
  __device__ __forceinline__ int at(int j, int n) const {
    const int a = j + m;
    return a >= n ? a - n : a;
  }
  template <typename T, class F> __device__ __forceinline__ cplx<T> sample(int j, int n, F&& f) const {
    const int j0 = at(j, n);
    const int j1 = j0 + 1 == n ? 0 : j0 + 1;
    const cplx<T> a = f(j0), b = f(j1);
    const T wb = static_cast<T>(w), wa = T(1) - wb;
    return mk<T>(wa * a.x + wb * b.x, wa * a.y + wb * b.y);
  }
};

// ------------------------------------------------------------------------------------------
// y forward: one block per (x plane, chunk of ZC consecutive z cells).  Consecutive z pairs
// (z, z+1) are packed as one complex column, so one complex length-Ny FFT transforms two real
// columns; the halves are separated, multiplied by exp(-i Ky s x_i) (shearing frame, Sect. 2.1)
// and stored for my < Ny/2 (the Nyquist row is dropped).  SASHA: double partial sums.

template <typename T, int NY, int V, bool REMAP>
__global__ __launch_bounds__(xy_threads<NY>()) void k_yfwd(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                       const cplx<T>* __restrict__ twg) {
  constexpr int ZC = y_zc<T, NY, V>();
  constexpr int NB = ZC / 2;
  constexpr int NT = xy_threads<NY>();
  constexpr int PAD = sizeof(T) == 4 ? 1 : 0;  // float: three spare slots per 32 (bank conflicts)
  using L = Tile<NB, NB, 1, true, PAD>;
  __shared__ cplx<T> tile[pad_slots<PAD>(NY * NB)];
  __shared__ cplx<T> tw[NY];
  __shared__ cplx<T> ph[NY / 2];
  __shared__ double red[2][NT / 64];
  lds_poison(tile, tw, ph, red);

  int t;
  const BoxRec rec = first_pass_rec(ga, recs, t);
  const BoxRec* br = &rec;
  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int x = t / nzc;
  const int z0 = (t - x * nzc) * ZC;
  const int hy = NY / 2;
  gmem<const T>* rho = hbm(static_cast<const T*>(br->rho));
  gmem<cplx<T>>* W = hbm(static_cast<cplx<T>*>(br->W));
  gmem<double>* partials = (REMAP && g.method == 1) ? hbm(br->partials) : nullptr;  // SASHA sums only

  load_twiddles<T, NY, NT>(tw, twg, tid);
  if (REMAP) {
    const double fy = br->fy;
    for (int my = tid; my < hy; my += NT) {
      double cs, sn;
      remap_phase(my, x, fy, cs, sn);
      ph[my] = mk<T>((T)cs, (T)sn);
    }
  }
  if (partials) {
    double s0 = 0.0, s1 = 0.0;
    const double dz = g.lz / nz;
    for (int w = tid; w < NY * NB; w += NT) {
      const int c = w % NB, y = w / NB;
      const int z = z0 + 2 * c;
      if (z < nz) {
        const cplx<T> v = *reinterpret_cast<gmem<const cplx<T>>*>(rho + ((size_t)x * NY + y) * nz + z);
        const double za = -0.5 * g.lz + (z + 0.5) * dz;
        s0 += (double)v.x + (double)v.y;
        s1 += za * (double)v.x + (za + dz) * (double)v.y;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_down(s0, o);
      s1 += __shfl_down(s1, o);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = s0;
      red[1][tid >> 6] = s1;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int i = 0; i < NT / 64; ++i) {
        a += red[0][i];
        b += red[1][i];
      }
      partials[2 * t] = a;
      partials[2 * t + 1] = b;
    }
  }

  gmem<const T>* src = rho + (size_t)x * NY * nz + z0;
  const int zn = min(ZC, nz - z0);
  // linear remap: the periodic field at y_j is the lab field at y_j - shy (x + 1/2) cells
  const bool lin = REMAP && g.remap == 1;
  YInterp yi;
  if (lin) yi.init(-br->shy * (x + 0.5), NY);
  fft_run<T, NY, typename Fwd<NY>::L, L, NT, -1, false, true>(
      tile, TwS<T>{tw}, tid,
      [&](int e, int c) {
        if (2 * c >= zn) return mk<T>(T(0), T(0));
        auto ld = [&](int y) { return *reinterpret_cast<gmem<const cplx<T>>*>(src + (size_t)y * nz + 2 * c); };
        return lin ? yi.sample<T>(e, NY, ld) : ld(e);
      },
      [&](int e, int c, cplx<T> v) { tile[L::at(e, c)] = v; });
  __syncthreads();

  for (int w = tid; w < hy * NB; w += NT) {
    const int c = w % NB, ky = w / NB;
    if (2 * c >= zn) continue;
    const cplx<T> c1 = tile[L::at(ky, c)];
    const cplx<T> c2 = tile[L::at((NY - ky) % NY, c)];
    cplx<T> a = mk<T>(T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y));
    cplx<T> b = mk<T>(T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x));
    if (REMAP) {
      const cplx<T> p = ph[ky];
      a = cmul<T>(a, p);
      b = cmul<T>(b, p);
    }
    gmem<cplx<T>>* dst = W + ((size_t)x * hy + ky) * nz + z0 + 2 * c;
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<gmem<float4>*>(dst) = make_float4(a.x, a.y, b.x, b.y);
    } else {
      dst[0] = a;
      dst[1] = b;
    }
  }
}

// y inverse: half spectra times exp(+i Ky s x_i), rebuilt into two Hermitian columns packed
// as one complex signal, one inverse FFT, real/imaginary parts written as z and z+1, plus
// Phi_0(z) for SASHA.
template <typename T, int NY, int V, bool REMAP>
__global__ __launch_bounds__(xy_threads<NY>()) void k_yinv(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                       const cplx<T>* __restrict__ twg) {
  constexpr int ZC = y_zc<T, NY, V>();
  constexpr int NB = ZC / 2;
  constexpr int NT = xy_threads<NY>();
  constexpr int PAD = sizeof(T) == 4 ? 1 : 0;  // float: three spare slots per 32 (bank conflicts)
  using L = Tile<NB, NB, 1, true, PAD>;
  __shared__ cplx<T> tile[pad_slots<PAD>(NY * NB)];
  __shared__ cplx<T> tw[NY];
  __shared__ cplx<T> ph[NY / 2];
  lds_poison(tile, tw, ph);

  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int x = t / nzc;
  const int z0 = (t - x * nzc) * ZC;
  const int hy = NY / 2;
  gmem<const cplx<T>>* W = hbm(static_cast<const cplx<T>*>(br->W));
  gmem<T>* phi = hbm(static_cast<T*>(br->phi));
  const int zn = min(ZC, nz - z0);

  load_twiddles<T, NY, NT>(tw, twg, tid);
  if (REMAP) {
    const double fy = br->fy;
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
    cplx<T> a = mk<T>(T(0), T(0)), b = a;
    if (2 * c < zn) {
      gmem<const cplx<T>>* src = W + ((size_t)x * hy + ky) * nz + z0 + 2 * c;
      if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<gmem<const float4>*>(src);
        a = mk<T>(q.x, q.y);
        b = mk<T>(q.z, q.w);
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
      tile[L::at(ky, c)] = mk<T>(a.x - b.y, a.y + b.x);       // A + iB
      tile[L::at(NY - ky, c)] = mk<T>(a.x + b.y, b.x - a.y);  // conj(A) + i conj(B)
    }
  }
  __syncthreads();

  const bool sasha = REMAP && g.method == 1;
  double c2 = 0.0, c1 = 0.0;
  if (sasha) {
    c2 = hbm(br->coef)->c2;
    c1 = hbm(br->coef)->c1;
  }
  const double dz = g.lz / nz;
  gmem<T>* dst = phi + (size_t)x * NY * nz + z0;
  auto store = [&](int e, int c, cplx<T> v) {
    if (2 * c < zn) {
      if (sasha) {
        const double za = -0.5 * g.lz + (z0 + 2 * c + 0.5) * dz;
        const double zb = za + dz;
        v.x = (T)((double)v.x + (c2 * za + c1) * za);
        v.y = (T)((double)v.y + (c2 * zb + c1) * zb);
      }
      *reinterpret_cast<gmem<cplx<T>>*>(dst + (size_t)e * nz + 2 * c) = v;
    }
  };
  if (REMAP && g.remap == 1) {
    // linear remap: the lab potential at y_j is the periodic one at y_j + shy (x + 1/2) cells,
    // so the transformed columns stay in LDS for the interpolation
    YInterp yi;
    yi.init(br->shy * (x + 0.5), NY);
    fft_run<T, NY, typename Fwd<NY>::L, L, NT, +1, true, true>(
        tile, TwS<T>{tw}, tid, [&](int e, int c) { return tile[L::at(e, c)]; },
        [&](int e, int c, cplx<T> v) { tile[L::at(e, c)] = v; });
    __syncthreads();
    for (int w = tid; w < NY * NB; w += NT) {
      const int c = w % NB, e = w / NB;
      store(e, c, yi.sample<T>(e, NY, [&](int y) { return tile[L::at(y, c)]; }));
    }
  } else {
    fft_run<T, NY, typename Fwd<NY>::L, L, NT, +1, true, false>(
        tile, TwS<T>{tw}, tid, [&](int e, int c) { return tile[L::at(e, c)]; }, store);
  }
}

// ------------------------------------------------------------------------------------------
// x: one block per (my, chunk of ZC consecutive z cells); rows of ZC contiguous complex values.

template <typename T, int NX, int V, int D>
__global__ __launch_bounds__((x_threads<T, NX, V>())) void k_x(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                            const cplx<T>* __restrict__ twg) {
  constexpr int ZC = x_zc<T, NX, V>();
  constexpr int NT = x_threads<T, NX, V>();
  constexpr int PAD = sizeof(T) == 4 ? 1 : 0;  // float: three spare slots per 32 (bank conflicts)
  using L = Tile<ZC, ZC, 1, true, PAD>;
  __shared__ cplx<T> buf[pad_slots<PAD>(NX * ZC)];
  __shared__ cplx<T> tw[NX];
  lds_poison(buf, tw);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int hy = g.ny / 2;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int my = t / nzc;
  const int z0 = (t - my * nzc) * ZC;
  const int zn = min(ZC, nz - z0);
  const size_t row = (size_t)hy * nz;
  gmem<cplx<T>>* base = hbm(static_cast<cplx<T>*>(br->W)) + (size_t)my * nz + z0;
  load_twiddles<T, NX, NT>(tw, twg, tid);
  fft_run<T, NX, typename Fwd<NX>::L, L, NT, D, false, false>(
      buf, TwS<T>{tw}, tid, [&](int e, int c) { return c < zn ? base[e * row + c] : mk<T>(T(0), T(0)); },
      [&](int e, int c, cplx<T> v) {
        if (c < zn) base[e * row + c] = v;
      });
}

// ------------------------------------------------------------------------------------------
// z: one block per 4 * PPW consecutive (Kx, Ky) pencils (contiguous in W); each wavefront owns
// PPW of them and runs them PW at a time (eight points per lane) through its private LDS
// exchange tile, with no workgroup barrier.  Each pencil is padded to M = Q*Nz (Hockney; never
// stored), transformed, multiplied by the Green's function at k = |(Kx + s Ky, Ky)| (Sect. 2.1)
// times 4 pi G/(Nx Ny M), transformed back; its first Nz values are stored in place.  The
// forward output feeds the inverse in registers; the zero half of the input and the discarded
// half of the output are dropped at compile time.
//
// Green's function (Sect. 2.3, App. A), L = alpha Lz, E = exp(-kL):
//   VGF, k > 0:  -((1 - E) + E (1 - cos(kz L)) + E (kz/k) sin(kz L)) / (k^2 + kz^2)
//                (the printed form regrouped; 1 - E = -expm1(-kL) and 1 - cos = 2 sin^2(kz L/2)
//                come from accurate tables, so nothing cancels);
//   VGF, k = 0:  (kz L sin(kz L) + cos(kz L) - 1) / kz^2, L^2/2 at kz = 0;
//   SASHA:       -1/(k^2 + kz^2), 0 for the zero mode (mean subtraction, Sect. 2.2).
// Per-pencil scalars are evaluated in double and rounded once; float plans run the k = 0
// pencil (the horizontal mean, which carries most of the potential) entirely in double.

template <typename T, int M, int V, int Q>
__global__ __launch_bounds__(kPassThreads) void k_z(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                    const cplx<T>* __restrict__ twg, const double2* __restrict__ tw64) {
  constexpr int PW = z_pw<M>();
  constexpr int PPW = z_ppw<M, V>();
  constexpr int WV = kPassThreads / 64;
  constexpr int NT = kPassThreads;
  constexpr bool kF32 = std::is_same<T, float>::value;
  // float 512-point pencils, one per transform: three spare slots per 32 (bank conflicts)
  constexpr int PAD = (kF32 && PW == 1 && M == 512) ? 1 : 0;
  using LW = Tile<PW, 1, M, false, PAD>;
  constexpr int XS = pad_slots<PAD>(PW * M);
  __shared__ cplx<T> xbuf[WV * XS];
  lds_poison(xbuf);
  // stage-major twiddles of the forward schedule of M, then of the inverse one if it differs; in
  // float, where one table serves both and a lane runs at most two butterflies per stage, each
  // lane keeps its own twiddles in registers (read once from HBM) instead
  constexpr bool kOneTw = same_schedule<typename ZSched<M>::F, typename ZSched<M>::I>();
  constexpr bool kTwReg = kF32 && kOneTw && max_per<typename ZSched<M>::F, M, PW>() <= 2;
  __shared__ cplx<T> tw[kTwReg ? 1 : kOneTw ? M : 2 * M];
  __shared__ T pa0[WV][PPW], pe[WV][PPW], pik[WV][PPW], pk2[WV][PPW], psp[WV][PPW];
  lds_poison(tw, pa0, pe, pik, pk2, psp);
  // block-0 work before the wavefront transforms borrows xbuf (SASHA reduction, then the double
  // k = 0 exchange tile of float plans)
  static_assert(lds_slots(M) * 16 <= WV * XS * (int)sizeof(cplx<T>), "k = 0 tile must fit");
  static_assert(2 * NT * 8 <= WV * XS * (int)sizeof(cplx<T>), "reduction scratch must fit");

  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int hy = g.ny / 2;
  const int np = g.nx * hy;
  const int nz = g.nz;
  const bool sasha = g.method == 1;
  const double scale = br->scale;
  gmem<cplx<T>>* W = hbm(static_cast<cplx<T>*>(br->W));
  gmem<const T>* zt = hbm(static_cast<const T*>(br->zt));
  const int pw0 = (t * WV + wave) * PPW;  // first pencil of this wavefront

  if constexpr (!kTwReg) load_twiddles<T, kOneTw ? M : 2 * M, NT>(tw, twg, tid);
  TwReg<T, M, typename ZSched<M>::F, LW, 64, TwS<T>> twr{TwS<T>{twg}};
  if constexpr (kTwReg) twr.load(lane);
  if (lane < PPW) {
    const int q = min(pw0 + lane, np - 1);
    const int mx = q / hy, my = q - mx * hy;
    const int sx = mx < g.nx / 2 ? mx : mx - g.nx;
    const double two_pi = 6.283185307179586476925286766559;
    const double Ky = (two_pi / g.ly) * my;
    const double kx = (two_pi / g.lx) * sx + br->s * Ky;
    const ModeGreen<T> c = mode_green<T>(kx * kx + Ky * Ky, mx == 0 && my == 0, sasha, g.L, scale);
    pa0[wave][lane] = c.a0;
    pe[wave][lane] = c.e;
    pik[wave][lane] = c.ik;
    pk2[wave][lane] = c.k2;
    psp[wave][lane] = c.zero;
  }

  // SASHA: <rho> and the centre of mass from the y-pass partial sums (fixed order)
  if (sasha && t == 0) {
    double* red = reinterpret_cast<double*>(xbuf);
    double a = 0.0, b = 0.0;
    for (int i = tid; i < br->npartials; i += NT) {
      a += hbm(br->partials)[2 * i];
      b += hbm(br->partials)[2 * i + 1];
    }
    red[tid] = a;
    red[NT + tid] = b;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (tid < o) {
        red[tid] += red[tid + o];
        red[NT + tid] += red[NT + tid + o];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double s0 = red[0], s1 = red[NT];
      SashaCoef c;
      c.c2 = 0.0;
      c.c1 = 0.0;
      if (s0 != 0.0) {
        const double mean = s0 / ((double)g.nx * g.ny * g.m);
        c.c2 = 0.5 * br->fourpiG * mean;
        c.c1 = -br->fourpiG * mean * (s1 / s0);
      }
      *hbm(br->coef) = c;
    }
  }
  __syncthreads();  // twiddles loaded; reduction scratch free

  // float plans: the k = 0 pencil (pencil 0 of tile 0) in double, block-wide
  const bool own0 = kF32 && t == 0;
  if constexpr (kF32) {
    if (t == 0) {
      using L1 = Tile<1, 1, M, false>;
      double2* dbuf = reinterpret_cast<double2*>(xbuf);
      gmem<float2>* w0 = reinterpret_cast<gmem<float2>*>(W);
      gmem<const double>* z64s2 = hbm(br->zt64[0]);
      gmem<const double>* z64ks = hbm(br->zt64[1]);
      gmem<const double>* z64kz2 = hbm(br->zt64[2]);
      fft_fwd_op_inv<double, M, L1, NT, 0, Q>(
          dbuf, tw64, tw64, tid,
          [&](int e, int) { return e < nz ? make_double2((double)w0[e].x, (double)w0[e].y) : make_double2(0.0, 0.0); },
          [&](int mz, int, double2& v) {
            double gk;
            if (sasha)
              gk = mz == 0 ? 0.0 : -1.0 / z64kz2[mz];
            else
              gk = mz == 0 ? 0.5 * g.L * g.L : (g.L * z64ks[mz] - z64s2[mz]) / z64kz2[mz];
            gk *= scale;
            v.x *= gk;
            v.y *= gk;
          },
          [&](int e, int, double2 v) {
            if (e < nz) w0[e] = make_float2((float)v.x, (float)v.y);
          });
      __syncthreads();  // xbuf is handed to the wavefronts
    }
  }

  cplx<T>* xw = xbuf + wave * XS;
  // the z-table rows of this lane's spectrum elements: the same for every pencil it transforms
  constexpr int NSL = spectrum_slots<T, M, LW, 64>();
  ZRow<T> zr[NSL];
#pragma unroll
  for (int i = 0; i < NSL; ++i) {
    const int mz = spectrum_slot<T, M, LW, 64>(lane, i);
    zr[i] = zrow(zt, mz < 0 ? 0 : mz);
  }
#pragma unroll 1
  for (int g0 = 0; g0 < PPW; g0 += PW) {
    if (pw0 + g0 >= np) break;  // uniform across the wavefront
    fft_fwd_op_inv<T, M, LW, 64, 0, Q, WaveSync>(
        xw, [&] { if constexpr (kTwReg) return twr; else return TwS<T>{tw}; }(),
        [&] { if constexpr (kTwReg) return twr; else return TwS<T>{tw + (kOneTw ? 0 : M)}; }(), lane,
        [&](int e, int p) {
          const int q = pw0 + g0 + p;
          return (e < nz && q < np && !(own0 && q == 0)) ? W[(size_t)q * nz + e] : mk<T>(T(0), T(0));
        },
        [&](int, int p, cplx<T>& v, int sl) {
          const int i = g0 + p;
          const T gk = green_at(pa0[wave][i], pe[wave][i], pik[wave][i], pk2[wave][i], psp[wave][i], zr[sl]);
          v.x *= gk;
          v.y *= gk;
        },
        [&](int e, int p, cplx<T> v) {
          const int q = pw0 + g0 + p;
          if (e < nz && q < np && !(own0 && q == 0)) W[(size_t)q * nz + e] = v;
        });
    WaveSync::sync();  // the exchange tile is rewritten by the next pencils of this wavefront
  }
}

// ------------------------------------------------------------------------------------------
// host-side dispatch helpers (instantiated per precision in the pass translation units)

template <typename T> int y_tiles_t(const BoxGeom& g, int variant) {
  int zc = 0;
#define SBP_CASE(N_) \
  if (g.ny == N_) zc = variant ? y_zc<T, N_, 1>() : y_zc<T, N_, 0>();
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return zc ? g.nx * ((g.nz + zc - 1) / zc) : 0;
}
template <typename T> int x_tiles_t(const BoxGeom& g, int variant) {
  int zc = 0;
#define SBP_CASE(N_) \
  if (g.nx == N_) zc = variant ? x_zc<T, N_, 1>() : x_zc<T, N_, 0>();
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return zc ? (g.ny / 2) * ((g.nz + zc - 1) / zc) : 0;
}
template <typename T> int z_tiles_t(const BoxGeom& g, int variant) {
  int pp = 0;
#define SBP_CASE(N_) \
  if (g.m == N_) pp = variant ? z_pp<T, N_, 1>() : z_pp<T, N_, 0>();
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  const int np = g.nx * (g.ny / 2);
  return pp ? (np + pp - 1) / pp : 0;
}

// per-precision launchers, specialised in the pass translation units
template <typename T>
hipError_t launch_y_impl(bool forward, bool remap, int ny, int variant, GroupArgs ga, int blocks, const BoxRec* recs,
                         const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_x_impl(int dir, int nx, int variant, GroupArgs ga, int blocks, const BoxRec* recs, const void* tw,
                         hipStream_t st);
template <typename T>
hipError_t launch_z_impl(int m, int variant, int q, GroupArgs ga, int blocks, const BoxRec* recs, const void* tw,
                         const void* tw64, hipStream_t st);
template <> hipError_t launch_y_impl<float>(bool, bool, int, int, GroupArgs, int, const BoxRec*, const void*, hipStream_t);
template <> hipError_t launch_y_impl<double>(bool, bool, int, int, GroupArgs, int, const BoxRec*, const void*, hipStream_t);
template <> hipError_t launch_x_impl<float>(int, int, int, GroupArgs, int, const BoxRec*, const void*, hipStream_t);
template <> hipError_t launch_x_impl<double>(int, int, int, GroupArgs, int, const BoxRec*, const void*, hipStream_t);
template <> hipError_t launch_z_impl<float>(int, int, int, GroupArgs, int, const BoxRec*, const void*, const void*,
                                            hipStream_t);
template <> hipError_t launch_z_impl<double>(int, int, int, GroupArgs, int, const BoxRec*, const void*, const void*,
                                             hipStream_t);

}  // namespace sbp
