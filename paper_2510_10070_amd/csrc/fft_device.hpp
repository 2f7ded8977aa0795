// Device-side FFT building blocks for gfx950: complex helpers, radix-2/3/4/8 butterflies and
// a Stockham auto-sort stage that transforms a batch of pencils held in LDS.
//
// A tile in LDS holds NB independent length-N transforms; element j of transform b has the
// logical index j*LD + b*BS.  The physical LDS slot is pad8(logical) = i + i/8: one spare
// slot every eight elements breaks the power-of-two strides of the Stockham write pattern
// that would otherwise hit the same LDS banks.  Each Stockham stage with radix R reads R
// elements per butterfly at stride N/R, applies twiddles exp(-+2 pi i k r/(Ns R)), runs the
// radix-R DFT and writes the results at stride Ns, so the output is in natural order after
// the last stage.  Every stage is read-all / barrier / write-all / barrier, so it works in
// place.
#pragma once

#include <hip/hip_runtime.h>

namespace sbp {

template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) {
  cplx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by i*D (D = -1 forward, +1 inverse): i*(a+ib) = -b + ia
template <int D, typename T> __device__ __forceinline__ cplx<T> rot(cplx<T> a) {
  return D < 0 ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
}

__host__ __device__ constexpr int pad8(int i) { return i + (i >> 3); }

// ------------------------------------------------------------------------------------------
// Radix-R DFTs in registers.  D = -1: X_k = sum x_n exp(-2 pi i nk/R); D = +1: conjugate kernel.

template <int R, int D, typename T> struct Dft;

template <int D, typename T> struct Dft<2, D, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  }
};

template <int D, typename T> struct Dft<3, D, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    cplx<T> s = cadd<T>(v[1], v[2]);
    cplx<T> d = csub<T>(v[1], v[2]);
    cplx<T> a = v[0];
    v[0] = cadd<T>(a, s);
    cplx<T> m = mk<T>(a.x - T(0.5) * s.x, a.y - T(0.5) * s.y);
    cplx<T> r = rot<D, T>(d);  // i*D*(b - c)
    v[1] = mk<T>(m.x + h * r.x, m.y + h * r.y);
    v[2] = mk<T>(m.x - h * r.x, m.y - h * r.y);
  }
};

template <int D, typename T> struct Dft<4, D, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> y0 = cadd<T>(v[0], v[2]);
    cplx<T> y1 = csub<T>(v[0], v[2]);
    cplx<T> y2 = cadd<T>(v[1], v[3]);
    cplx<T> y3 = rot<D, T>(csub<T>(v[1], v[3]));
    v[0] = cadd<T>(y0, y2);
    v[2] = csub<T>(y0, y2);
    v[1] = cadd<T>(y1, y3);
    v[3] = csub<T>(y1, y3);
  }
};

template <int D, typename T> struct Dft<8, D, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T c = T(0.70710678118654752440084436210485);  // sqrt(2)/2
    // first level: pairs (n, n+4)
    cplx<T> a0 = cadd<T>(v[0], v[4]), b0 = csub<T>(v[0], v[4]);
    cplx<T> a1 = cadd<T>(v[1], v[5]), b1 = csub<T>(v[1], v[5]);
    cplx<T> a2 = cadd<T>(v[2], v[6]), b2 = csub<T>(v[2], v[6]);
    cplx<T> a3 = cadd<T>(v[3], v[7]), b3 = csub<T>(v[3], v[7]);
    // twiddles w8^n on the odd half: w8 = exp(i D pi/4)
    b1 = mk<T>(c * (b1.x - D * b1.y), c * (b1.y + D * b1.x));
    b2 = rot<D, T>(b2);
    b3 = mk<T>(c * (-b3.x - D * b3.y), c * (-b3.y + D * b3.x));
    cplx<T> e[4] = {a0, a1, a2, a3};
    cplx<T> o[4] = {b0, b1, b2, b3};
    Dft<4, D, T>::run(e);
    Dft<4, D, T>::run(o);
    v[0] = e[0]; v[2] = e[1]; v[4] = e[2]; v[6] = e[3];
    v[1] = o[0]; v[3] = o[1]; v[5] = o[2]; v[7] = o[3];
  }
};

// ------------------------------------------------------------------------------------------
// Radix schedules per transform length (product of the radices = N).

template <int N> struct Sched;
#define SBP_SCHED(N_, ...)                                   \
  template <> struct Sched<N_> {                             \
    static constexpr int r[] = {__VA_ARGS__};                \
    static constexpr int n = sizeof(r) / sizeof(int);        \
  };
SBP_SCHED(8, 8)
SBP_SCHED(12, 4, 3)
SBP_SCHED(16, 4, 4)
SBP_SCHED(24, 8, 3)
SBP_SCHED(32, 8, 4)
SBP_SCHED(48, 4, 4, 3)
SBP_SCHED(64, 8, 8)
SBP_SCHED(96, 8, 4, 3)
SBP_SCHED(128, 8, 4, 4)
SBP_SCHED(192, 8, 8, 3)
SBP_SCHED(256, 8, 8, 4)
SBP_SCHED(384, 8, 4, 4, 3)
SBP_SCHED(512, 8, 8, 8)
SBP_SCHED(768, 8, 8, 4, 3)
SBP_SCHED(1024, 8, 8, 4, 4)
#undef SBP_SCHED

// Tile layout: NB transforms, element (j, b) at logical index j*LD + b*BS, LDS slot pad8(.).
// BFAST selects which index consecutive threads walk (batch index for z-fastest tiles,
// element index otherwise), so that neighbouring lanes touch neighbouring LDS words.
template <int NB_, int LD_, int BS_, bool BFAST_> struct Tile {
  static constexpr int NB = NB_, LD = LD_, BS = BS_;
  static constexpr bool BFAST = BFAST_;
  static __device__ __forceinline__ int at(int j, int b) { return pad8(j * LD + b * BS); }
};

// LDS slots needed for a tile of n logical elements
__host__ __device__ constexpr int lds_slots(int n) { return pad8(n - 1) + 1; }

template <typename T, int N, int R, int NS, class L, int NT, int D>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, const cplx<T>* tw, int tid) {
  constexpr int NBF = N / R;
  constexpr int ITEMS = NBF * L::NB;
  constexpr int PER = (ITEMS + NT - 1) / NT;
  cplx<T> v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int w = tid + p * NT;
    if (ITEMS % NT == 0 || w < ITEMS) {
      const int b = L::BFAST ? w % L::NB : w / NBF;
      const int j = L::BFAST ? w / L::NB : w % NBF;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = buf[L::at(j + r * NBF, b)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int w = tid + p * NT;
    if (ITEMS % NT == 0 || w < ITEMS) {
      const int b = L::BFAST ? w % L::NB : w / NBF;
      const int j = L::BFAST ? w / L::NB : w % NBF;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cplx<T> t = tw[k * r * (N / (NS * R))];
          v[p][r] = D < 0 ? cmul<T>(v[p][r], t) : cmulc<T>(v[p][r], t);
        }
      }
      Dft<R, D, T>::run(v[p]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[L::at(base + r * NS, b)] = v[p][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int S, int NS, class L, int NT, int D>
__device__ __forceinline__ void fft_stages(cplx<T>* buf, const cplx<T>* tw, int tid) {
  if constexpr (S < Sched<N>::n) {
    constexpr int R = Sched<N>::r[S];
    stockham_stage<T, N, R, NS, L, NT, D>(buf, tw, tid);
    fft_stages<T, N, S + 1, NS * R, L, NT, D>(buf, tw, tid);
  }
}

// Transform all NB pencils of the tile in place.  tw[m] = exp(-2 pi i m/N), m < N (in LDS or
// global memory).  D = -1 forward, +1 inverse (unnormalised).  Called by all NT threads;
// the tile must be complete (a barrier separates its producers from this call).
template <typename T, int N, class L, int NT, int D>
__device__ __forceinline__ void lds_fft(cplx<T>* buf, const cplx<T>* tw, int tid) {
  fft_stages<T, N, 0, 1, L, NT, D>(buf, tw, tid);
}

// copy the N-entry twiddle table into LDS
template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* __restrict__ src, int tid) {
  for (int i = tid; i < N; i += NT) dst[i] = src[i];
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Give each XCD
// a contiguous range of the T tiles so that tiles sharing cache lines run on the same L2 at
// about the same time.
__device__ __forceinline__ int xcd_tile(int b, int T) {
  const int q = T >> 3, r = T & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

}  // namespace sbp
