// Device-side FFT engine for gfx950: complex helpers, radix-2/3/4/8 butterflies and a
// register-resident Stockham auto-sort schedule whose stages exchange data through LDS.
//
// A tile holds NB independent length-N transforms; element j of transform b has the logical
// index j*LD + b*BS and, by default, the LDS slot pad8(logical) = i + i/8 (one spare slot every
// eight elements breaks the power-of-two strides of the Stockham write pattern, which would
// otherwise land on the same LDS banks); a tile may choose three spare slots per 32 instead.
//
// Stage s of radix R (Ns = product of the earlier radices) takes, for butterfly j of
// transform b, the R inputs j + r N/R, applies the twiddles exp(-+2 pi i k r/(Ns R)),
// k = j mod Ns, runs the radix-R DFT and produces the outputs base + r Ns,
// base = (j - k) R + k; after the last stage the transform is in natural order.
//
// Each thread keeps its butterflies in registers.  The first stage reads its inputs through
// a caller functor (straight from HBM, from LDS or from registers) and the last stage hands
// its outputs to a caller functor (straight to HBM, or to LDS), so a transform costs only
// (stages - 1) LDS exchanges.  A forward transform whose last radix equals the first radix
// of the inverse schedule can hand its outputs to the inverse in registers: the outputs
// j + r Ns of the last forward stage are exactly the inputs j + r N/R of the first inverse
// stage, held by the same thread.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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
// LDS slots needed for a tile of n logical elements
__host__ __device__ constexpr int lds_slots(int n) { return pad8(n - 1) + 1; }
// Paddings with E spare slots after every P logical elements: PAD 0 = pad8, PAD 1 = three per 32
// (with 8-byte elements it leaves a third of pad8's LDS bank conflicts in the 8.8.8 exchanges:
// stride-8 writes, stride-1 reads, 64-blocked stride-8 writes, and in 256-point four-column
// transforms).
template <int PAD> constexpr int kPadShift = PAD == 0 ? 3 : 5;
template <int PAD> constexpr int kPadPeriod = 1 << kPadShift<PAD>;
template <int PAD> constexpr int kPadSpare = PAD == 1 ? 3 : 1;
template <int PAD> __host__ __device__ constexpr int pad_map(int i) {
  return i + kPadSpare<PAD> * (i >> kPadShift<PAD>);
}
template <int PAD> __host__ __device__ constexpr int pad_slots(int n) { return pad_map<PAD>(n - 1) + 1; }

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

// 6 = 3 x 2: DFT3 over the even and the odd inputs, then radix-2 with the twiddles w6^k
template <int D, typename T> struct Dft<6, D, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    cplx<T> e[3] = {v[0], v[2], v[4]};
    cplx<T> o[3] = {v[1], v[3], v[5]};
    Dft<3, D, T>::run(e);
    Dft<3, D, T>::run(o);
    // w6^1 = 1/2 + i D sqrt(3)/2, w6^2 = -1/2 + i D sqrt(3)/2
    const cplx<T> o1 = mk<T>(T(0.5) * o[1].x - D * h * o[1].y, T(0.5) * o[1].y + D * h * o[1].x);
    const cplx<T> o2 = mk<T>(-T(0.5) * o[2].x - D * h * o[2].y, -T(0.5) * o[2].y + D * h * o[2].x);
    v[0] = cadd<T>(e[0], o[0]);
    v[3] = csub<T>(e[0], o[0]);
    v[1] = cadd<T>(e[1], o1);
    v[4] = csub<T>(e[1], o1);
    v[2] = cadd<T>(e[2], o2);
    v[5] = csub<T>(e[2], o2);
  }
};

template <int D, typename T> struct Dft<1, D, T> {
  static __device__ __forceinline__ void run(cplx<T>*) {}
};

// 16 = 4 x 4: inner DFT4 over n1 (stride 4), twiddles w16^(n2 k1), outer DFT4 over n2
template <int D, typename T> struct Dft<16, D, T> {
  static __device__ __forceinline__ cplx<T> twc(cplx<T> a, T c, T s) {  // a * (c + i D s)
    return mk<T>(a.x * c - D * a.y * s, a.y * c + D * a.x * s);
  }
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
    const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
    const T c2 = T(0.70710678118654752440084436210485);  // cos(pi/4)
    cplx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cplx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<4, D, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
    }
    // w^(n2 k1): (1,1)->w1 (1,2)->w2 (1,3)->w3 (2,1)->w2 (2,2)->w4 (2,3)->w6 (3,1)->w3 (3,2)->w6 (3,3)->w9
    y[1][1] = twc(y[1][1], c1, s1);
    y[1][2] = twc(y[1][2], c2, c2);
    y[1][3] = twc(y[1][3], s1, c1);
    y[2][1] = twc(y[2][1], c2, c2);
    y[2][2] = rot<D, T>(y[2][2]);
    y[2][3] = twc(y[2][3], -c2, c2);
    y[3][1] = twc(y[3][1], s1, c1);
    y[3][2] = twc(y[3][2], -c2, c2);
    y[3][3] = twc(y[3][3], -c1, -s1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cplx<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<4, D, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// ------------------------------------------------------------------------------------------
// Radix schedules.  Fwd<N> is the forward schedule; Inv<N> is its reverse, so the first
// inverse radix equals the last forward radix (register hand-off).

template <int... Rs> struct RList {
  static constexpr int n = sizeof...(Rs);
  static constexpr int r[] = {Rs...};
  static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= r[i];
    return v;
  }
};
template <int N> struct Fwd;
template <int N> struct Inv;
// the inverse schedule is the forward one reversed: one stage-major table serves both when the
// radix list reads the same both ways
template <class A, class B> constexpr bool same_schedule() {
  if (A::n != B::n) return false;
  for (int i = 0; i < A::n; ++i)
    if (A::r[i] != B::r[i]) return false;
  return true;
}
template <> struct Fwd<8> { using L = RList<8>; };
template <> struct Inv<8> { using L = RList<8>; };
template <> struct Fwd<12> { using L = RList<4, 3>; };
template <> struct Inv<12> { using L = RList<3, 4>; };
template <> struct Fwd<16> { using L = RList<4, 4>; };
template <> struct Inv<16> { using L = RList<4, 4>; };
template <> struct Fwd<24> { using L = RList<8, 3>; };
template <> struct Inv<24> { using L = RList<3, 8>; };
template <> struct Fwd<32> { using L = RList<8, 4>; };
template <> struct Inv<32> { using L = RList<4, 8>; };
template <> struct Fwd<48> { using L = RList<4, 4, 3>; };
template <> struct Inv<48> { using L = RList<3, 4, 4>; };
template <> struct Fwd<64> { using L = RList<8, 8>; };
template <> struct Inv<64> { using L = RList<8, 8>; };
template <> struct Fwd<96> { using L = RList<8, 4, 3>; };
template <> struct Inv<96> { using L = RList<3, 4, 8>; };
template <> struct Fwd<128> { using L = RList<8, 4, 4>; };
template <> struct Inv<128> { using L = RList<4, 4, 8>; };
template <> struct Fwd<192> { using L = RList<8, 8, 3>; };
template <> struct Inv<192> { using L = RList<3, 8, 8>; };
template <> struct Fwd<256> { using L = RList<8, 8, 4>; };
template <> struct Inv<256> { using L = RList<4, 8, 8>; };
template <> struct Fwd<384> { using L = RList<8, 4, 4, 3>; };
template <> struct Inv<384> { using L = RList<3, 4, 4, 8>; };
template <> struct Fwd<512> { using L = RList<8, 8, 8>; };
template <> struct Inv<512> { using L = RList<8, 8, 8>; };
template <> struct Fwd<768> { using L = RList<8, 8, 4, 3>; };
template <> struct Inv<768> { using L = RList<3, 4, 8, 8>; };
template <> struct Fwd<1024> { using L = RList<8, 8, 4, 4>; };
template <> struct Inv<1024> { using L = RList<4, 4, 8, 8>; };

// Radix schedules of the padded z transforms (forward F, inverse I), which run forward and back
// with the hand-off in registers (fft_fwd_op_inv): those of Fwd and Inv, except where a palindrome
// lets one stage-major table serve both directions, so that a lane can keep its twiddles in
// registers for every pencil it transforms (TwReg).
template <int N> struct ZSched {
  using F = typename Fwd<N>::L;
  using I = typename Inv<N>::L;
};
template <> struct ZSched<128> {
  using F = RList<4, 8, 4>;
  using I = RList<4, 8, 4>;
};
template <> struct ZSched<192> {
  using F = RList<8, 3, 8>;
  using I = RList<8, 3, 8>;
};
template <> struct ZSched<256> {
  using F = RList<8, 4, 8>;
  using I = RList<8, 4, 8>;
};

// Tile layout: NB transforms, element (j, b) at logical index j*LD + b*BS, LDS slot
// pad_map<PAD>(.) (PAD 0: pad8).  BFAST selects which index consecutive threads walk (batch index
// for z-fastest tiles, element index otherwise), so that neighbouring lanes touch neighbouring
// words.
template <int NB_, int LD_, int BS_, bool BFAST_, int PAD_ = 0> struct Tile {
  static constexpr int NB = NB_, LD = LD_, BS = BS_;
  static constexpr bool BFAST = BFAST_;
  static constexpr int PAD = PAD_;
  static __device__ __forceinline__ int logical(int j, int b) { return j * LD + b * BS; }
  static __device__ __forceinline__ int map(int i) { return pad_map<PAD>(i); }
  static __device__ __forceinline__ int at(int j, int b) { return map(j * LD + b * BS); }
};

// Stage-major twiddle table of a schedule: stage S (Ns = product of the earlier radices, radix
// R) keeps exp(-2 pi i k r/(Ns R)), r = 1 .. R-1, k < Ns, at slot Ns - 1 + (r - 1) Ns + k, so
// N - 1 slots in all.  The lanes of a stage then read consecutive slots (no LDS bank
// conflicts, where the strided plain table has up to 8-way conflicts), and the r offsets are
// compile-time constants.
template <typename T> struct TwS {
  static constexpr bool kInRegisters = false;
  const cplx<T>* p;
  __device__ __forceinline__ cplx<T> at(int i) const { return p[i]; }
};
// The same table kept in the spare slots of a pad8 tile (slot 9 i + 8 holds entry i): a tile of
// 8 (N - 1) + 8 logical elements or more has room for it, and its stride-9 reads are
// conflict-free as well.
template <typename T> struct TwH {
  static constexpr bool kInRegisters = false;
  const cplx<T>* tile;
  __device__ __forceinline__ cplx<T> at(int i) const { return tile[9 * i + 8]; }
};

// One Stockham stage of schedule RL for a tile L processed by NT threads.
template <typename T, int N, class RL, int S, class L, int NT, int D> struct Stage {
  static constexpr int R = RL::r[S];
  static constexpr int NS = RL::ns(S);
  static constexpr int NBF = N / R;
  static constexpr int ITEMS = NBF * L::NB;
  static constexpr int PER = (ITEMS + NT - 1) / NT;
  static constexpr bool FULL = ITEMS % NT == 0;

  static __device__ __forceinline__ bool item(int tid, int p, int& j, int& b) {
    const int w = tid + p * NT;
    if constexpr (L::BFAST) {
      b = w % L::NB;
      j = w / L::NB;
    } else {
      j = w % NBF;
      b = w / NBF;
    }
    return FULL || w < ITEMS;
  }
  // inputs j + r NBF from a functor f(elem, b); inputs r >= RIN are known zeros
  template <int RIN = R, class F>
  static __device__ __forceinline__ void read_fn(cplx<T> (&v)[PER][R], int tid, F&& f) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int j, b;
      if (item(tid, p, j, b)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // a functor taking a third argument also gets the register slot p R + r
          if constexpr (std::is_invocable_v<F&, int, int, int>)
            v[p][r] = r < RIN ? f(j + r * NBF, b, p * R + r) : mk<T>(T(0), T(0));
          else
            v[p][r] = r < RIN ? f(j + r * NBF, b) : mk<T>(T(0), T(0));
        }
      }
    }
  }
  static __device__ __forceinline__ void read_lds(cplx<T> (&v)[PER][R], const cplx<T>* buf, int tid) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int j, b;
      if (item(tid, p, j, b)) {
        const int a = L::logical(j, b);
        const int pa = L::map(a);
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = buf[pad_off<NBF * L::LD>(pa, a, r)];
      }
    }
  }
  // stride-C offset r*C from the padded base
  template <int C> static __device__ __forceinline__ int pad_off(int pa, int a, int r) {
    constexpr int P = kPadPeriod<L::PAD>, E = kPadSpare<L::PAD>;
    if constexpr (C % P == 0)
      return pa + r * (C + E * (C / P));
    else
      return L::map(a + r * C);
  }
  // tw: the plain table exp(-2 pi i m/N), m < N (a pointer), or the stage-major table of this
  // schedule (TwS)
  template <class TW>
  static __device__ __forceinline__ void twiddle_dft(cplx<T> (&v)[PER][R], TW tw, int tid) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int j, b;
      if (item(tid, p, j, b)) {
        if constexpr (NS > 1) {
          const int k = j % NS;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cplx<T> t;
            if constexpr (std::is_pointer_v<TW>)
              t = tw[k * r * (N / (NS * R))];
            else if constexpr (TW::kInRegisters)
              t = tw.template stage<S, NS>(p, r, k);
            else
              t = tw.at(NS - 1 + (r - 1) * NS + k);
            v[p][r] = D < 0 ? cmul<T>(v[p][r], t) : cmulc<T>(v[p][r], t);
          }
        }
        Dft<R, D, T>::run(v[p]);
      }
    }
  }
  // outputs base + r NS to a functor f(elem, b, value); outputs r >= ROUT are not needed
  template <int ROUT = R, class F>
  static __device__ __forceinline__ void write_fn(cplx<T> (&v)[PER][R], int tid, F&& f) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int j, b;
      if (item(tid, p, j, b)) {
        const int k = j % NS;
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < ROUT; ++r) {
          if constexpr (std::is_invocable_v<F&, int, int, cplx<T>, int>)
            f(base + r * NS, b, v[p][r], p * R + r);
          else
            f(base + r * NS, b, v[p][r]);
        }
      }
    }
  }
  static __device__ __forceinline__ void write_lds(cplx<T> (&v)[PER][R], cplx<T>* buf, int tid) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      int j, b;
      if (item(tid, p, j, b)) {
        const int k = j % NS;
        const int base = (j - k) * R + k;
        const int a = L::logical(base, b);
        if constexpr (L::PAD == 0 && (NS * L::LD) % 8 == 0) {
          const int pa = pad8(a);
#pragma unroll
          for (int r = 0; r < R; ++r) buf[pa + r * (NS * L::LD + (NS * L::LD) / 8)] = v[p][r];
        } else if constexpr (L::PAD != 0 && (NS * L::LD) % kPadPeriod<L::PAD> == 0) {
          constexpr int P = kPadPeriod<L::PAD>, E = kPadSpare<L::PAD>;
          const int pa = L::map(a);
#pragma unroll
          for (int r = 0; r < R; ++r) buf[pa + r * (NS * L::LD + E * ((NS * L::LD) / P))] = v[p][r];
        } else if constexpr (L::PAD != 0 && kPadPeriod<L::PAD> % (NS * L::LD) == 0 &&
                             (NS * R * L::LD) % kPadPeriod<L::PAD> == 0 &&
                             (L::BS % kPadPeriod<L::PAD> == 0 || L::NB == 1 || L::NB * L::BS <= NS * L::LD)) {
          // a mod P = k LD + b BS < NS LD, which divides P: output r crosses the same periods for
          // every lane, so its offset from the padded base is a constant
          constexpr int P = kPadPeriod<L::PAD>, E = kPadSpare<L::PAD>, C = NS * L::LD;
          const int pa = L::map(a);
#pragma unroll
          for (int r = 0; r < R; ++r) buf[pa + r * C + E * ((r * C) / P)] = v[p][r];
        } else if constexpr (NS == 1 && R == 8 && L::LD == 1 && (L::BS % 8 == 0 || L::NB == 1)) {
          // base = 8j: a multiple of 8, so the eight outputs share one pad shift (both paddings)
          const int pa = L::map(a);
#pragma unroll
          for (int r = 0; r < R; ++r) buf[pa + r] = v[p][r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) buf[L::map(a + r * NS * L::LD)] = v[p][r];
        }
      }
    }
  }
};

// The twiddles one thread needs, held in registers: the butterflies a thread runs in each stage
// (PER of them) are the same for every transform of schedule RL it runs, so their twiddle
// indices k are fixed, and the R - 1 twiddles of each butterfly of stages FIRST.. can be fetched
// once from the stage-major table `src` and reused; earlier stages still read `src`.  (Where two
// butterflies of a thread share k, the two fetches read one address.)  An inverse transform may
// use the same object when its schedule equals RL (the stages conjugate).
template <typename T, int N, class RL, class L, int NT, class SRC, int FIRST = 1> struct TwReg {
  static constexpr bool kInRegisters = true;
  static constexpr int kPerMax = 2;
  SRC src;
  cplx<T> w[RL::n][kPerMax][8];
  __device__ __forceinline__ void load(int tid) { load_stage<FIRST>(tid); }
  template <int S> __device__ __forceinline__ void load_stage(int tid) {
    if constexpr (S < RL::n) {
      using St = Stage<T, N, RL, S, L, NT, -1>;
      static_assert(St::PER <= kPerMax, "butterflies per thread and stage above the register table");
      static_assert(St::R <= 8, "radix above the register table");
#pragma unroll
      for (int p = 0; p < St::PER; ++p) {
        int j, b;
        St::item(tid, p, j, b);
        const int k = j % St::NS;
#pragma unroll
        for (int r = 1; r < St::R; ++r) w[S][p][r] = src.at(St::NS - 1 + (r - 1) * St::NS + k);
      }
      load_stage<S + 1>(tid);
    }
  }
  template <int S, int NS> __device__ __forceinline__ cplx<T> stage(int p, int r, int k) const {
    if constexpr (S >= FIRST)
      return w[S][p][r];
    else
      return src.at(NS - 1 + (r - 1) * NS + k);
  }
};

// the most butterflies a lane runs in one stage of schedule RL, for PW transforms of length N over
// 64 lanes (TwReg holds up to two per stage)
template <class RL, int N, int PW> constexpr int max_per() {
  int m = 0;
  for (int s = 0; s < RL::n; ++s) {
    const int per = ((N / RL::r[s]) * PW + 63) / 64;
    m = per > m ? per : m;
  }
  return m;
}

// Barrier policies of the engine.  BlockSync: the tile is shared by the whole workgroup.
// WaveSync: the tile belongs to one wavefront; its LDS operations complete in issue order, so
// only the compiler must be kept from moving accesses across the exchange point.
struct BlockSync {
  static __device__ __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
  static __device__ __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// Full transform of every pencil in the tile.
//   src(elem, b) -> cplx: input element of transform b (read by stage 0 only);
//   dst(elem, b, v): output element of transform b (written by the last stage only).
// `buf` is the LDS exchange tile (lds_slots(N*LD*NB) slots for the layout L).  SRC_LDS: src
// reads `buf`; DST_LDS: dst writes `buf`.  Barriers separate every read of `buf` from the
// next write to it.  On return without DST_LDS the last stage has read `buf`: the caller must
// barrier before writing it again; with DST_LDS the caller must barrier before reading it.
// Sy0 is the barrier after stage 0's exchange write.  Stage 0 uses no twiddles, so where the
// twiddle table in LDS was written by other wavefronts of the block and nothing has synchronised
// the block since, a wavefront-owned transform (Sy = WaveSync) passes Sy0 = BlockSync: the first
// twiddle read then follows every wavefront's table writes.
template <typename T, int N, class RL, class L, int NT, int D, bool SRC_LDS, bool DST_LDS, int S = 0, int Q = 1,
          class Sy = BlockSync, class Sy0 = Sy, class TW, class Src, class Dst>
__device__ __forceinline__ void fft_run(cplx<T>* buf, TW tw, int tid, Src&& src, Dst&& dst) {
  using St = Stage<T, N, RL, S, L, NT, D>;
  constexpr bool LAST = S == RL::n - 1;
  cplx<T> v[St::PER][St::R];
  if constexpr (S == 0) {
    St::read_fn(v, tid, src);
    if constexpr (SRC_LDS && (!LAST || DST_LDS)) Sy::sync();
  } else {
    St::read_lds(v, buf, tid);
    if constexpr (!LAST || DST_LDS) Sy::sync();
  }
  St::twiddle_dft(v, tw, tid);
  if constexpr (LAST) {
    // with Q > 1 only the outputs below N/Q are wanted: r < R/Q when the radix divides
    St::template write_fn<(St::R % Q == 0) ? St::R / Q : St::R>(v, tid, dst);
  } else {
    St::write_lds(v, buf, tid);
    if constexpr (S == 0)
      Sy0::sync();
    else
      Sy::sync();
    fft_run<T, N, RL, L, NT, D, SRC_LDS, DST_LDS, S + 1, Q, Sy>(buf, tw, tid, src, dst);
  }
}

// Forward transform, pointwise op, inverse transform, with the hand-off between the last
// forward stage and the first inverse stage kept in registers (the z schedules ZSched<N>).
//   src(elem, b) -> cplx (forward inputs), op(elem, b, cplx&) on spectrum values (op(elem, b,
//   cplx&, slot) also gets the register slot, which is fixed per thread and element, see
//   spectrum_slot), dst(elem, b, v) (inverse outputs); twf, twi: twiddles of the forward and of the inverse
//   schedule (the same plain table, or each schedule's stage-major table).
// Q > 1 (zero padding by Q): forward inputs at or above N/Q are zero and inverse outputs at or
// above N/Q are discarded; both are dropped at compile time where the radix allows.
// The spectrum element that thread tid holds at register slot i of the forward-inverse
// hand-off in fft_fwd_op_inv (-1 where the slot is unused): the op's arguments per slot are the
// same on every call, so per-element constants can be fetched once per thread.
template <typename T, int N, class L, int NT>
__device__ __forceinline__ int spectrum_slot(int tid, int i) {
  using RF = typename ZSched<N>::F;
  using Sf = Stage<T, N, RF, RF::n - 1, L, NT, -1>;
  int j, b;
  if (!Sf::item(tid, i / Sf::R, j, b)) return -1;
  return j + (i % Sf::R) * Sf::NBF;
}
template <typename T, int N, class L, int NT> constexpr int spectrum_slots() {
  using RF = typename ZSched<N>::F;
  using Sf = Stage<T, N, RF, RF::n - 1, L, NT, -1>;
  return Sf::PER * Sf::R;
}

template <typename T, int N, class L, int NT, int S, int Q = 1, class Sy = BlockSync, class TWF, class TWI,
          class Src, class Op, class Dst>
__device__ __forceinline__ void fft_fwd_op_inv(cplx<T>* buf, TWF twf, TWI twi, int tid, Src&& src, Op&& op,
                                               Dst&& dst) {
  using RF = typename ZSched<N>::F;
  using RI = typename ZSched<N>::I;
  static_assert(RF::r[RF::n - 1] == RI::r[0], "hand-off needs matching radices");
  if constexpr (S < RF::n - 1) {
    // forward stages before the last one
    using St = Stage<T, N, RF, S, L, NT, -1>;
    cplx<T> v[St::PER][St::R];
    if constexpr (S == 0) {
      St::template read_fn<(St::R % Q == 0) ? St::R / Q : St::R>(v, tid, src);
    } else {
      St::read_lds(v, buf, tid);
      Sy::sync();
    }
    St::twiddle_dft(v, twf, tid);
    St::write_lds(v, buf, tid);
    Sy::sync();
    fft_fwd_op_inv<T, N, L, NT, S + 1, Q, Sy>(buf, twf, twi, tid, src, op, dst);
  } else {
    using Sf = Stage<T, N, RF, RF::n - 1, L, NT, -1>;
    using Si = Stage<T, N, RI, 0, L, NT, +1>;
    static_assert(Sf::PER == Si::PER && Sf::R == Si::R, "stage shapes must agree");
    cplx<T> v[Sf::PER][Sf::R];
    if constexpr (RF::n == 1) {
      Sf::template read_fn<(Sf::R % Q == 0) ? Sf::R / Q : Sf::R>(v, tid, src);
    } else {
      Sf::read_lds(v, buf, tid);
      Sy::sync();
    }
    Sf::twiddle_dft(v, twf, tid);
    // last forward stage: outputs j + r*NBF (base = j since j < NS = NBF)
#pragma unroll
    for (int p = 0; p < Sf::PER; ++p) {
      int j, b;
      if (Sf::item(tid, p, j, b)) {
#pragma unroll
        for (int r = 0; r < Sf::R; ++r) {
          // an op taking a fourth argument also gets the register slot p R + r
          if constexpr (std::is_invocable_v<Op&, int, int, cplx<T>&, int>)
            op(j + r * Sf::NBF, b, v[p][r], p * Sf::R + r);
          else
            op(j + r * Sf::NBF, b, v[p][r]);
        }
      }
    }
    // first inverse stage on the same registers (Ns = 1: no twiddles)
    Si::twiddle_dft(v, twi, tid);
    if constexpr (RI::n == 1) {
      Si::template write_fn<(Si::R % Q == 0) ? Si::R / Q : Si::R>(v, tid, dst);
    } else {
      Si::write_lds(v, buf, tid);
      Sy::sync();
      fft_run<T, N, RI, L, NT, +1, false, false, 1, Q, Sy>(buf, twi, tid, src, dst);
    }
  }
}

// copy COUNT entries of a stage-major table (built on the host, see TwS) into LDS; entry i goes
// to dst[STRIDE i + OFF] (STRIDE 9, OFF 8: the spare slots of a pad8 tile)
template <typename T, int COUNT, int NT, int STRIDE = 1, int OFF = 0>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* __restrict__ src, int tid) {
  for (int i = tid; i < COUNT; i += NT) dst[STRIDE * i + OFF] = src[i];
}

// Debug builds (SBP_POISON_LDS defined) fill a kernel's shared arrays with a quiet NaN before any
// thread uses them, so that a read of an element that no thread wrote turns the result into NaN,
// which the parity tests catch.  The barrier makes the fill complete before first use.  In
// other builds this is empty.
template <class... A> __device__ __forceinline__ void lds_poison(A&... arrays) {
#ifdef SBP_POISON_LDS
  auto fill = [](auto& a) {
    unsigned* w = reinterpret_cast<unsigned*>(&a);
    for (unsigned i = threadIdx.x; i < sizeof(a) / 4; i += blockDim.x) w[i] = 0x7fc00000u;
  };
  (fill(arrays), ...);
  __syncthreads();
#else
  ((void)arrays, ...);
#endif
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
