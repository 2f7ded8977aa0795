// Fused three-pass schedule: the half spectrum crosses HBM three times (rho -> W, W -> W,
// W -> phi) instead of five.  The x transform of length Nx = A*B is split four-step:
//   X[k1 + A k2] = sum_j w_B^(j k2) [ w_Nx^(j k1) sum_a x[j + B a] w_A^(a k1) ]
// Pass A does, for B-strided x planes {j + B a}, the y transform and remap of every plane and
// the A-point DFT across the planes in registers (plus the w_Nx^(j k1) twiddle).  Pass B does,
// for each (k1, my), the B-point DFT across j in registers, the padded z transform with the
// Green multiply for every Kx = k1 + A k2, and the inverse B-point DFT.  Pass C inverts pass A.
//
// Intermediate layout: W[k1][my][j][z] (complex, k1 < A, my < Ny/2, j < B, z < Nz), so the B
// pencils that pass B needs for one (k1, my) are one contiguous run of B*Nz values.
#pragma once

#include "passes.hpp"

namespace sbp {

constexpr int kFusedAC = 512;  // threads of passes A and C

// real z cells per pass-A/C tile: variant 0 = 32-byte rows, 1 = 64-byte rows, 2 = 16-byte rows;
// kWideRows = 128-byte rows, taken only by the launches that mix Ny (for Ny <= 64 or A <= 4)
constexpr int kWideRows = 4;
template <typename T, int V> constexpr int fa_zc() {
  return (V == kWideRows ? 128 : V == 1 ? 64 : V == 2 ? 16 : 32) / (int)sizeof(T);
}
// threads per pass-A/C block: variant 2 tiles are half as wide and take half the threads, so
// that two blocks fit on a CU at the register count of pass C
template <int V> constexpr int fa_threads() { return V == 2 ? kFusedAC / 2 : kFusedAC; }
// variant 3 (split passes A and C, k_fas / k_fcs): four z cells per tile in either precision
constexpr int kSplitZC = 4;

// four-step split used by the fused schedule: B = 16 pencils per pass-B block, A = Nx/16
constexpr int kFusedB16 = 16;
// instantiated lengths: Nx = 16 A with A in {1, 2, 4, 6, 8, 16}; Ny a power of two in
// [16, 512] or 96; M = pad Nz a power of two in [32, 512] or 192
inline bool fused_supported(int nx, int ny, int m) {
  auto pow2 = [](int n) { return n > 0 && (n & (n - 1)) == 0; };
  return ((pow2(nx) && nx >= 16 && nx <= 256) || nx == 96) && ((pow2(ny) && ny >= 16 && ny <= 512) || ny == 96) &&
         ((pow2(m) && m >= 32 && m <= 512) || m == 192);
}
// planes transformed side by side in passes A and C: the largest power of two that divides A,
// capped (the plane groups must tile the A planes and the threads)
template <int A, int CAP> constexpr int fa_pg() {
  int p = 1;
  while (2 * p <= CAP && A % (2 * p) == 0) p *= 2;
  return p;
}

// LDS of a pass-A (C = false) or pass-C (C = true) block for tile variant V in {0, 1, 2}
template <typename T, int NY, int A, int V, bool C> struct AcShape {
  // float tiles pad three slots per 32 (fewer bank conflicts in the y exchanges), double pad8
  static constexpr int PAD = sizeof(T) == 4 ? 1 : 0;
  static constexpr int NB = fa_zc<T, V>() / 2;
  static constexpr int NT = fa_threads<V>();
  // pass C with 32-byte rows and Ny <= 256: eight planes at a time, one wavefront per plane
  static constexpr int PG = C ? fa_pg<A, ((V == 0 || V == 1 || V == kWideRows) && NY <= 256) ? 8 : 4>()
                               : fa_pg<A, (V == 1 || V == kWideRows) ? 8 : 4>();
  static constexpr int TILE = PG * pad_slots<PAD>(NY * NB);  // PG plane tiles
};
// the largest tile over A in {1, 2, 4, 6, 8} (launch groups that mix Nx)
template <typename T, int NY, int V, bool C> constexpr int ac_mix_tile() {
  constexpr int t[5] = {AcShape<T, NY, 1, V, C>::TILE, AcShape<T, NY, 2, V, C>::TILE, AcShape<T, NY, 4, V, C>::TILE,
                        AcShape<T, NY, 6, V, C>::TILE, AcShape<T, NY, 8, V, C>::TILE};
  int m = 0;
  for (int v : t) m = v > m ? v : m;
  return m;
}

// remap phase of plane x = j + B a as P_j Q^a in double: exp(-i 2 pi my (2x+1) fy)
struct PlanePhase {
  double pr, pi, qr, qi;  // current phase and the per-plane step
  __device__ __forceinline__ void init(int my, int j, int B, double fy) {
    double s, c;
    const double c0 = static_cast<double>(my * (2 * j + 1)) * fy;
    sincospi(2.0 * (c0 - floor(c0)), &s, &c);
    pr = c;
    pi = -s;
    const double c1 = static_cast<double>(my) * (2.0 * B) * fy;
    sincospi(2.0 * (c1 - floor(c1)), &s, &c);
    qr = c;
    qi = -s;
  }
  __device__ __forceinline__ void step() {
    const double r = pr * qr - pi * qi;
    pi = pr * qi + pi * qr;
    pr = r;
  }
};

// ------------------------------------------------------------------------------------------
// Pass A: one block per (j, z chunk).  The A planes x = j + B a go through the y transform in
// groups of PG, each plane handled by NT/PG threads with its own LDS tile; every thread then
// keeps the remapped half spectra of its positions for all A planes in registers.  Finally the
// A-point DFT across planes, the w_Nx^(j k1) twiddle and the store to W[k1][my][j][z].

template <typename T, int NY, int A, int B, int V, bool LIN>
__device__ __forceinline__ void fa_body(const BoxRec* br, int t, const cplx<T>* __restrict__ twy,
                                        const cplx<T>* __restrict__ twx, cplx<T>* tile, cplx<T>* tw, double* red) {
  constexpr int ZC = fa_zc<T, V>();
  constexpr int NB = ZC / 2;
  constexpr int NT = fa_threads<V>();
  constexpr int PG = AcShape<T, NY, A, V, false>::PG;  // planes transformed side by side
  constexpr int TNT = NT / PG;       // threads per plane transform
  // a transform owned by one wavefront needs no workgroup barrier between its stages
  using Sy = std::conditional_t<TNT == 64, WaveSync, BlockSync>;
  constexpr int HY = NY / 2;
  constexpr int QN = HY * NB;        // output positions (ky, c) of one plane
  constexpr int POS = (QN + NT - 1) / NT;
  constexpr int PAD = AcShape<T, NY, A, V, false>::PAD;
  constexpr int SLOTS = pad_slots<PAD>(NY * NB);
  using L = Tile<NB, NB, 1, true, PAD>;

  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int sub = tid / TNT, stid = tid - sub * TNT;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int j = t / nzc;
  const int z0 = (t - j * nzc) * ZC;
  const int zn = min(ZC, nz - z0);
  gmem<const T>* rho = hbm(static_cast<const T*>(br->rho));
  gmem<cplx<T>>* W = hbm(static_cast<cplx<T>*>(br->W));
  const bool sasha = g.method == 1;
  const double dz = g.lz / nz;
  cplx<T>* mytile = tile + sub * SLOTS;
  load_twiddles<T, NY, NT>(tw, twy, tid);

  PlanePhase pp[POS];
#pragma unroll
  for (int i = 0; i < POS; ++i) {
    const int q = tid + i * NT;
    pp[i].init(q < QN ? q / NB : 0, j, B, br->fy);
  }

  cplx<T> acc[A][POS][2];
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int a0 = 0; a0 < A; a0 += PG) {
    // PG thread groups transform planes a0 .. a0+PG-1 (x = j + B a) into their LDS tiles
    const int x = j + B * (a0 + sub);
    gmem<const T>* src = rho + (size_t)x * NY * nz + z0;
    // linear remap: the periodic field at y_j is the lab field at y_j - shy (x + 1/2) cells
    constexpr bool lin = LIN;  // linear remap (one instantiation each: the spectral path keeps its registers)
    YInterp yi;
    if (lin) yi.init(-br->shy * (x + 0.5), NY);
    auto ld_plane = [&](int e, int c) {
      cplx<T> v = mk<T>(T(0), T(0));
      if (2 * c < zn) {
        auto ld = [&](int y) { return *reinterpret_cast<gmem<const cplx<T>>*>(src + (size_t)y * nz + 2 * c); };
        v = lin ? yi.sample<T>(e, NY, ld) : ld(e);
        if (sasha) {
          const double za = -0.5 * g.lz + (z0 + 2 * c + 0.5) * dz;
          s0 += (double)v.x + (double)v.y;
          s1 += za * (double)v.x + (za + dz) * (double)v.y;
        }
      }
      return v;
    };
    auto st_tile = [&](int e, int c, cplx<T> v) { mytile[L::at(e, c)] = v; };
    // the twiddle table was written by every wavefront of the block: the first planes' transforms
    // pass a workgroup barrier before their first twiddle read
    if (a0 == 0)
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, -1, false, true, 0, 1, Sy, BlockSync>(mytile, TwS<T>{tw}, stid,
                                                                                          ld_plane, st_tile);
    else
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, -1, false, true, 0, 1, Sy>(mytile, TwS<T>{tw}, stid, ld_plane,
                                                                             st_tile);
    __syncthreads();
    // every thread collects its positions of all PG planes: separate, remap, keep in registers
#pragma unroll
    for (int sp = 0; sp < PG; ++sp) {
      const cplx<T>* tl = tile + sp * SLOTS;
#pragma unroll
      for (int i = 0; i < POS; ++i) {
        const int q = tid + i * NT;
        acc[a0 + sp][i][0] = acc[a0 + sp][i][1] = mk<T>(T(0), T(0));
        if (q < QN) {
          const int ky = q / NB, c = q - ky * NB;
          const cplx<T> c1 = tl[L::at(ky, c)];
          const cplx<T> c2 = tl[L::at((NY - ky) % NY, c)];
          const cplx<T> p = mk<T>((T)pp[i].pr, (T)pp[i].pi);
          acc[a0 + sp][i][0] = cmul<T>(mk<T>(T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y)), p);
          acc[a0 + sp][i][1] = cmul<T>(mk<T>(T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x)), p);
        }
        pp[i].step();
      }
    }
    __syncthreads();  // the tiles are reused by the next planes
  }

  if (sasha) {
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_down(s0, o);
      s1 += __shfl_down(s1, o);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = s0;
      red[NT / 64 + (tid >> 6)] = s1;
    }
    __syncthreads();
    if (tid == 0) {
      double sa = 0.0, sb = 0.0;
      for (int i = 0; i < NT / 64; ++i) {
        sa += red[i];
        sb += red[NT / 64 + i];
      }
      hbm(br->partials)[2 * t] = sa;
      hbm(br->partials)[2 * t + 1] = sb;
    }
  }

  // A-point DFT across planes, twiddle w_Nx^(j k1), store
#pragma unroll
  for (int i = 0; i < POS; ++i) {
    const int q = tid + i * NT;
    if (q >= QN) continue;
    const int ky = q / NB, c = q - ky * NB;
    if (2 * c >= zn) continue;
    cplx<T> va[A], vb[A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      va[a] = acc[a][i][0];
      vb[a] = acc[a][i][1];
    }
    Dft<A, -1, T>::run(va);
    Dft<A, -1, T>::run(vb);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      const cplx<T> w = twx[j * k1];  // j k1 < B A = Nx
      const cplx<T> ra = cmul<T>(va[k1], w), rb = cmul<T>(vb[k1], w);
      gmem<cplx<T>>* dst = W + (((size_t)k1 * HY + ky) * B + j) * nz + z0 + 2 * c;
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<gmem<float4>*>(dst) = make_float4(ra.x, ra.y, rb.x, rb.y);
      } else {
        dst[0] = ra;
        dst[1] = rb;
      }
    }
  }
}

template <typename T, int NY, int A, int B, int V, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fa(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                 const cplx<T>* __restrict__ twy, const cplx<T>* __restrict__ twx) {
  using S = AcShape<T, NY, A, V, false>;
  __shared__ cplx<T> tile[S::TILE];
  __shared__ cplx<T> tw[NY];
  __shared__ double red[2 * (S::NT / 64)];
  lds_poison(tile, tw, red);
  int t;
  const BoxRec rec = first_pass_rec(ga, recs, t);
  const BoxRec* br = &rec;
  fa_body<T, NY, A, B, V, LIN>(br, t, twy, twx, tile, tw, red);
}

// Pass A for a launch group whose boxes differ in Nx = B A (A <= 8): every block runs the body
// of its own box's A with that box's x twiddles, so one launch covers what would otherwise be
// one small launch per A.  Registers and LDS are those of the largest body.
template <typename T, int NY, int B, int V, bool LIN>
__device__ __forceinline__ void fa_mix_body(const BoxRec* br, int t, const cplx<T>* __restrict__ twy, cplx<T>* tile,
                                            cplx<T>* tw, double* red) {
  const cplx<T>* twx = static_cast<const cplx<T>*>(br->twx);
  switch (br->g.nx / B) {
    case 1: fa_body<T, NY, 1, B, V, LIN>(br, t, twy, twx, tile, tw, red); break;
    case 2: fa_body<T, NY, 2, B, V, LIN>(br, t, twy, twx, tile, tw, red); break;
    case 4: fa_body<T, NY, 4, B, V, LIN>(br, t, twy, twx, tile, tw, red); break;
    case 6: fa_body<T, NY, 6, B, V, LIN>(br, t, twy, twx, tile, tw, red); break;
    default: fa_body<T, NY, 8, B, V, LIN>(br, t, twy, twx, tile, tw, red); break;
  }
}

template <typename T, int NY, int B, int V, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fa_mix(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                     const cplx<T>* __restrict__ twy, const cplx<T>* __restrict__) {
  constexpr int NT = fa_threads<V>();
  __shared__ cplx<T> tile[ac_mix_tile<T, NY, V, false>()];
  __shared__ cplx<T> tw[NY];
  __shared__ double red[2 * (NT / 64)];
  lds_poison(tile, tw, red);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  fa_mix_body<T, NY, B, V, LIN>(br, t, twy, tile, tw, red);
}

// ------------------------------------------------------------------------------------------
// Pass C: inverse of pass A.  Load W[k1][my][j][z chunk] for all k1, conjugate twiddle,
// A-point inverse DFT across k1 in registers, then per plane: reverse remap, Hermitian columns
// in LDS, inverse y transform straight to phi (+ Phi_0 for SASHA).

template <typename T, int NY, int A, int B, int V, bool LIN>
__device__ __forceinline__ void fc_body(const BoxRec* br, int t, const cplx<T>* __restrict__ twy,
                                        const cplx<T>* __restrict__ twx, cplx<T>* tile, cplx<T>* tw) {
  constexpr int ZC = fa_zc<T, V>();
  constexpr int NB = ZC / 2;
  constexpr int NT = fa_threads<V>();
  constexpr int PG = AcShape<T, NY, A, V, true>::PG;
  constexpr int TNT = NT / PG;
  // a transform owned by one wavefront needs no workgroup barrier between its stages
  using Sy = std::conditional_t<TNT == 64, WaveSync, BlockSync>;
  constexpr int HY = NY / 2;
  constexpr int QN = HY * NB;
  constexpr int POS = (QN + NT - 1) / NT;
  constexpr int PAD = AcShape<T, NY, A, V, true>::PAD;
  constexpr int SLOTS = pad_slots<PAD>(NY * NB);
  using L = Tile<NB, NB, 1, true, PAD>;

  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int sub = tid / TNT, stid = tid - sub * TNT;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int j = t / nzc;
  const int z0 = (t - j * nzc) * ZC;
  const int zn = min(ZC, nz - z0);
  gmem<const cplx<T>>* W = hbm(static_cast<const cplx<T>*>(br->W));
  gmem<T>* phi = hbm(static_cast<T*>(br->phi));
  cplx<T>* mytile = tile + sub * SLOTS;
  load_twiddles<T, NY, NT>(tw, twy, tid);

  cplx<T> acc[A][POS][2];
  PlanePhase pp[POS];
#pragma unroll
  for (int i = 0; i < POS; ++i) {
    const int q = tid + i * NT;
    const int ky = q < QN ? q / NB : 0, c = q < QN ? q - ky * NB : 0;
    pp[i].init(ky, j, B, br->fy);
    cplx<T> va[A], vb[A];
    // one branch around all A loads, so that they issue back to back
    if (q < QN && 2 * c < zn) {
      gmem<const cplx<T>>* src = W + ((size_t)ky * B + j) * nz + z0 + 2 * c;
      const size_t plane = (size_t)HY * B * nz;  // W stride between consecutive k1
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        cplx<T> a0, b0;
        if constexpr (sizeof(T) == 4) {
          const float4 v4 = *reinterpret_cast<gmem<const float4>*>(src + k1 * plane);
          a0 = mk<T>(v4.x, v4.y);
          b0 = mk<T>(v4.z, v4.w);
        } else {
          a0 = src[k1 * plane];
          b0 = src[k1 * plane + 1];
        }
        const cplx<T> w = twx[j * k1];  // j k1 < B A = Nx
        va[k1] = cmulc<T>(a0, w);
        vb[k1] = cmulc<T>(b0, w);
      }
    } else {
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) va[k1] = vb[k1] = mk<T>(T(0), T(0));
    }
    Dft<A, +1, T>::run(va);
    Dft<A, +1, T>::run(vb);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      acc[a][i][0] = va[a];
      acc[a][i][1] = vb[a];
    }
  }

  const bool sasha = g.method == 1;
  double c2 = 0.0, c1 = 0.0;
  if (sasha) {
    c2 = hbm(br->coef)->c2;
    c1 = hbm(br->coef)->c1;
  }
  const double dz = g.lz / nz;
#pragma unroll
  for (int a0 = 0; a0 < A; a0 += PG) {
    // every thread writes its positions of planes a0 .. a0+PG-1 as Hermitian columns
#pragma unroll
    for (int sp = 0; sp < PG; ++sp) {
      cplx<T>* tl = tile + sp * SLOTS;
      const auto& cur = acc[a0 + sp];
      for (int c = tid; c < NB; c += NT) tl[L::at(HY, c)] = mk<T>(T(0), T(0));  // y Nyquist
#pragma unroll
      for (int i = 0; i < POS; ++i) {
        const int q = tid + i * NT;
        if (q < QN) {
          const int ky = q / NB, c = q - ky * NB;
          const cplx<T> p = mk<T>((T)pp[i].pr, (T)pp[i].pi);  // exp(-i theta); conjugated here
          const cplx<T> av = cmulc<T>(cur[i][0], p), bv = cmulc<T>(cur[i][1], p);
          if (ky == 0) {
            tl[L::at(0, c)] = mk<T>(av.x, bv.x);
          } else {
            tl[L::at(ky, c)] = mk<T>(av.x - bv.y, av.y + bv.x);
            tl[L::at(NY - ky, c)] = mk<T>(av.x + bv.y, bv.x - av.y);
          }
        }
        pp[i].step();
      }
    }
    __syncthreads();
    // PG thread groups run the inverse y transforms of their planes straight to phi
    const int x = j + B * (a0 + sub);
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
    if constexpr (LIN) {
      // linear remap: the lab potential at y_j is the periodic one at y_j + shy (x + 1/2)
      // cells, so the transformed columns stay in LDS for the interpolation
      YInterp yi;
      yi.init(br->shy * (x + 0.5), NY);
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, +1, true, true, 0, 1, Sy>(
          mytile, TwS<T>{tw}, stid, [&](int e, int c) { return mytile[L::at(e, c)]; },
          [&](int e, int c, cplx<T> v) { mytile[L::at(e, c)] = v; });
      Sy::sync();  // the interpolation reads this wavefront's own plane only when TNT = 64
      for (int w = stid; w < NY * NB; w += TNT) {
        const int c = w % NB, e = w / NB;
        store(e, c, yi.sample<T>(e, NY, [&](int y) { return mytile[L::at(y, c)]; }));
      }
    } else {
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, +1, true, false, 0, 1, Sy>(
          mytile, TwS<T>{tw}, stid, [&](int e, int c) { return mytile[L::at(e, c)]; }, store);
    }
    __syncthreads();  // the tiles are rebuilt for the next planes
  }
}

template <typename T, int NY, int A, int B, int V, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fc(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                 const cplx<T>* __restrict__ twy, const cplx<T>* __restrict__ twx) {
  __shared__ cplx<T> tile[AcShape<T, NY, A, V, true>::TILE];
  __shared__ cplx<T> tw[NY];
  lds_poison(tile, tw);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  fc_body<T, NY, A, B, V, LIN>(br, t, twy, twx, tile, tw);
}

// Pass C for a launch group whose boxes differ in Nx (A <= 8), as k_fa_mix
template <typename T, int NY, int B, int V, bool LIN>
__device__ __forceinline__ void fc_mix_body(const BoxRec* br, int t, const cplx<T>* __restrict__ twy, cplx<T>* tile,
                                            cplx<T>* tw) {
  const cplx<T>* twx = static_cast<const cplx<T>*>(br->twx);
  switch (br->g.nx / B) {
    case 1: fc_body<T, NY, 1, B, V, LIN>(br, t, twy, twx, tile, tw); break;
    case 2: fc_body<T, NY, 2, B, V, LIN>(br, t, twy, twx, tile, tw); break;
    case 4: fc_body<T, NY, 4, B, V, LIN>(br, t, twy, twx, tile, tw); break;
    case 6: fc_body<T, NY, 6, B, V, LIN>(br, t, twy, twx, tile, tw); break;
    default: fc_body<T, NY, 8, B, V, LIN>(br, t, twy, twx, tile, tw); break;
  }
}

template <typename T, int NY, int B, int V, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fc_mix(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                     const cplx<T>* __restrict__ twy, const cplx<T>* __restrict__) {
  __shared__ cplx<T> tile[ac_mix_tile<T, NY, V, true>()];
  __shared__ cplx<T> tw[NY];
  lds_poison(tile, tw);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  fc_mix_body<T, NY, B, V, LIN>(br, t, twy, tile, tw);
}

// Passes A and C for a launch group whose boxes differ in Ny <= 128 as well as in A <= 8 (float):
// every block runs the body of its own box's Ny and A with that box's y and x twiddles, so the
// groups of a batch that would each be one launch per Ny share one, and their blocks fill the chip
// together.  Boxes of Ny <= 64, and boxes of A <= 4, take 128-byte rows, the others 64-byte rows,
// so that a block holds about as many (y, z) positions times planes as one of Ny = 128 and A = 8
// (the same LDS tile and registers, twice the loads in flight per lane and half the blocks of
// 64-byte rows).  Registers and LDS are those of the largest body.
constexpr int kMultiNyMax = 128;
// row width in such a launch: 128-byte rows where Ny <= 64 or A <= 4, which keeps a thread's
// positions times planes (and the plane tiles of a block) within those of Ny = 128 and A = 8 in
// 64-byte rows
constexpr int multi_rows(int ny, int a) { return (ny <= 64 || a <= 4) ? kWideRows : 1; }
template <typename T, int NY, bool C> constexpr int ac_multi_ny_tile() {
  constexpr int t[5] = {AcShape<T, NY, 1, multi_rows(NY, 1), C>::TILE, AcShape<T, NY, 2, multi_rows(NY, 2), C>::TILE,
                        AcShape<T, NY, 4, multi_rows(NY, 4), C>::TILE, AcShape<T, NY, 6, multi_rows(NY, 6), C>::TILE,
                        AcShape<T, NY, 8, multi_rows(NY, 8), C>::TILE};
  int m = 0;
  for (int v : t) m = v > m ? v : m;
  return m;
}
template <typename T, bool C> constexpr int ac_multi_tile() {
  constexpr int t[5] = {ac_multi_ny_tile<T, 16, C>(), ac_multi_ny_tile<T, 32, C>(), ac_multi_ny_tile<T, 64, C>(),
                        ac_multi_ny_tile<T, 96, C>(), ac_multi_ny_tile<T, 128, C>()};
  int m = 0;
  for (int v : t) m = v > m ? v : m;
  return m;
}
// tiles of one box in such a launch (host side)
template <typename T> int fused_ac_multi_tiles_t(const BoxGeom& g) {
  const int zc = multi_rows(g.ny, g.nx / kFusedB16) == kWideRows ? fa_zc<T, kWideRows>() : fa_zc<T, 1>();
  return kFusedB16 * ((g.nz + zc - 1) / zc);
}
// the bodies of a block's box: its Ny (template) and A, with that box's x twiddles
template <typename T, int NY, int B, bool LIN>
__device__ __forceinline__ void fa_multi_body(const BoxRec* br, int t, const cplx<T>* __restrict__ twy, cplx<T>* tile,
                                              cplx<T>* tw, double* red) {
  const cplx<T>* twx = static_cast<const cplx<T>*>(br->twx);
  switch (br->g.nx / B) {
    case 1: fa_body<T, NY, 1, B, multi_rows(NY, 1), LIN>(br, t, twy, twx, tile, tw, red); break;
    case 2: fa_body<T, NY, 2, B, multi_rows(NY, 2), LIN>(br, t, twy, twx, tile, tw, red); break;
    case 4: fa_body<T, NY, 4, B, multi_rows(NY, 4), LIN>(br, t, twy, twx, tile, tw, red); break;
    case 6: fa_body<T, NY, 6, B, multi_rows(NY, 6), LIN>(br, t, twy, twx, tile, tw, red); break;
    default: fa_body<T, NY, 8, B, multi_rows(NY, 8), LIN>(br, t, twy, twx, tile, tw, red); break;
  }
}
template <typename T, int NY, int B, bool LIN>
__device__ __forceinline__ void fc_multi_body(const BoxRec* br, int t, const cplx<T>* __restrict__ twy, cplx<T>* tile,
                                              cplx<T>* tw) {
  const cplx<T>* twx = static_cast<const cplx<T>*>(br->twx);
  switch (br->g.nx / B) {
    case 1: fc_body<T, NY, 1, B, multi_rows(NY, 1), LIN>(br, t, twy, twx, tile, tw); break;
    case 2: fc_body<T, NY, 2, B, multi_rows(NY, 2), LIN>(br, t, twy, twx, tile, tw); break;
    case 4: fc_body<T, NY, 4, B, multi_rows(NY, 4), LIN>(br, t, twy, twx, tile, tw); break;
    case 6: fc_body<T, NY, 6, B, multi_rows(NY, 6), LIN>(br, t, twy, twx, tile, tw); break;
    default: fc_body<T, NY, 8, B, multi_rows(NY, 8), LIN>(br, t, twy, twx, tile, tw); break;
  }
}

template <typename T, int B, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fa_multi(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                       const cplx<T>* __restrict__, const cplx<T>* __restrict__) {
  static_assert(fa_threads<1>() == kFusedAC && fa_threads<kWideRows>() == kFusedAC, "one block size");
  __shared__ cplx<T> tile[ac_multi_tile<T, false>()];
  __shared__ cplx<T> tw[kMultiNyMax];
  __shared__ double red[2 * (kFusedAC / 64)];
  lds_poison(tile, tw, red);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const cplx<T>* twy = static_cast<const cplx<T>*>(br->twy);
  switch (br->g.ny) {
    case 16: fa_multi_body<T, 16, B, LIN>(br, t, twy, tile, tw, red); break;
    case 32: fa_multi_body<T, 32, B, LIN>(br, t, twy, tile, tw, red); break;
    case 64: fa_multi_body<T, 64, B, LIN>(br, t, twy, tile, tw, red); break;
    case 96: fa_multi_body<T, 96, B, LIN>(br, t, twy, tile, tw, red); break;
    default: fa_multi_body<T, 128, B, LIN>(br, t, twy, tile, tw, red); break;
  }
}

template <typename T, int B, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fc_multi(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                       const cplx<T>* __restrict__, const cplx<T>* __restrict__) {
  __shared__ cplx<T> tile[ac_multi_tile<T, true>()];
  __shared__ cplx<T> tw[kMultiNyMax];
  lds_poison(tile, tw);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const cplx<T>* twy = static_cast<const cplx<T>*>(br->twy);
  switch (br->g.ny) {
    case 16: fc_multi_body<T, 16, B, LIN>(br, t, twy, tile, tw); break;
    case 32: fc_multi_body<T, 32, B, LIN>(br, t, twy, tile, tw); break;
    case 64: fc_multi_body<T, 64, B, LIN>(br, t, twy, tile, tw); break;
    case 96: fc_multi_body<T, 96, B, LIN>(br, t, twy, tile, tw); break;
    default: fc_multi_body<T, 128, B, LIN>(br, t, twy, tile, tw); break;
  }
}

// ------------------------------------------------------------------------------------------
// Split passes A and C (tile variant 3: four z cells per tile, Ny <= 256).  The two real z
// columns of a position (ky, c), which share one complex y transform, are held by a lane pair,
// one column per lane, so that each thread keeps one complex value per plane instead of two:
// half the registers, all 512 threads busy (with four z cells and Ny = 256 a tile has 256
// positions), eight planes transformed side by side.

template <typename T, int NY, int A, int B, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fas(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                  const cplx<T>* __restrict__ twy, const cplx<T>* __restrict__ twx) {
  constexpr int ZC = kSplitZC;
  constexpr int NB = ZC / 2;
  constexpr int NT = kFusedAC;
  constexpr int HY = NY / 2;
  constexpr int QN = HY * NB;  // positions (ky, c)
  static_assert(2 * QN <= NT, "one position per lane pair");
  constexpr int PG = fa_pg<A, 8>();
  constexpr int TNT = NT / PG;
  // a transform owned by one wavefront needs no workgroup barrier between its stages
  using Sy = std::conditional_t<TNT == 64, WaveSync, BlockSync>;
  constexpr int SLOTS = lds_slots(NY * NB);
  using L = Tile<NB, NB, 1, true>;
  __shared__ cplx<T> tile[PG * SLOTS];
  __shared__ cplx<T> tw[NY];
  __shared__ double red[2][NT / 64];
  lds_poison(tile, tw, red);

  int t;
  const BoxRec rec = first_pass_rec(ga, recs, t);
  const BoxRec* br = &rec;
  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int sub = tid / TNT, stid = tid - sub * TNT;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int j = t / nzc;
  const int z0 = (t - j * nzc) * ZC;
  const int zn = min(ZC, nz - z0);
  gmem<const T>* rho = hbm(static_cast<const T*>(br->rho));
  gmem<cplx<T>>* W = hbm(static_cast<cplx<T>*>(br->W));
  const bool sasha = g.method == 1;
  const double dz = g.lz / nz;
  cplx<T>* mytile = tile + sub * SLOTS;
  load_twiddles<T, NY, NT>(tw, twy, tid);

  const int q = tid >> 1, h = tid & 1;  // position and column of this lane
  const bool qv = q < QN;
  const int ky = qv ? q / NB : 0, c = qv ? q - ky * NB : 0;
  PlanePhase pp;
  pp.init(ky, j, B, br->fy);
  cplx<T> acc[A];
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int a0 = 0; a0 < A; a0 += PG) {
    // PG thread groups transform planes a0 .. a0+PG-1 (x = j + B a) into their LDS tiles
    const int x = j + B * (a0 + sub);
    gmem<const T>* src = rho + (size_t)x * NY * nz + z0;
    YInterp yi;
    if (LIN) yi.init(-br->shy * (x + 0.5), NY);
    auto ld_plane = [&](int e, int cc) {
      cplx<T> v = mk<T>(T(0), T(0));
      if (2 * cc < zn) {
        auto ld = [&](int y) { return *reinterpret_cast<gmem<const cplx<T>>*>(src + (size_t)y * nz + 2 * cc); };
        v = LIN ? yi.sample<T>(e, NY, ld) : ld(e);
        if (sasha) {
          const double za = -0.5 * g.lz + (z0 + 2 * cc + 0.5) * dz;
          s0 += (double)v.x + (double)v.y;
          s1 += za * (double)v.x + (za + dz) * (double)v.y;
        }
      }
      return v;
    };
    auto st_tile = [&](int e, int cc, cplx<T> v) { mytile[L::at(e, cc)] = v; };
    // the twiddle table was written by every wavefront of the block: the first planes' transforms
    // pass a workgroup barrier before their first twiddle read
    if (a0 == 0)
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, -1, false, true, 0, 1, Sy, BlockSync>(mytile, TwS<T>{tw}, stid,
                                                                                          ld_plane, st_tile);
    else
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, -1, false, true, 0, 1, Sy>(mytile, TwS<T>{tw}, stid, ld_plane,
                                                                             st_tile);
    __syncthreads();
    // each lane separates its column of its position from the Hermitian pair and remaps it
#pragma unroll
    for (int sp = 0; sp < PG; ++sp) {
      const cplx<T>* tl = tile + sp * SLOTS;
      acc[a0 + sp] = mk<T>(T(0), T(0));
      if (qv) {
        const cplx<T> c1 = tl[L::at(ky, c)];
        const cplx<T> c2 = tl[L::at((NY - ky) % NY, c)];
        const cplx<T> v = h == 0 ? mk<T>(T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y))
                                 : mk<T>(T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x));
        acc[a0 + sp] = cmul<T>(v, mk<T>((T)pp.pr, (T)pp.pi));
      }
      pp.step();
    }
    __syncthreads();  // the tiles are reused by the next planes
  }

  if (sasha) {
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
      double sa = 0.0, sb = 0.0;
      for (int i = 0; i < NT / 64; ++i) {
        sa += red[0][i];
        sb += red[1][i];
      }
      hbm(br->partials)[2 * t] = sa;
      hbm(br->partials)[2 * t + 1] = sb;
    }
  }

  // A-point DFT across planes, twiddle w_Nx^(j k1), store this lane's column
  Dft<A, -1, T>::run(acc);
  if (qv && 2 * c + h < zn) {
    gmem<cplx<T>>* dst = W + ((size_t)ky * B + j) * nz + z0 + 2 * c + h;
    const size_t plane = (size_t)HY * B * nz;  // W stride between consecutive k1
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) dst[k1 * plane] = cmul<T>(acc[k1], twx[j * k1]);  // j k1 < Nx
  }
}

// Inverse of k_fas.  After the inverse A-point DFT and the remap phase the lane pair swaps its
// values, and each lane writes one of the two Hermitian slots of the position.
template <typename T, int NY, int A, int B, bool LIN>
__global__ __launch_bounds__(kFusedAC) void k_fcs(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                  const cplx<T>* __restrict__ twy, const cplx<T>* __restrict__ twx) {
  constexpr int ZC = kSplitZC;
  constexpr int NB = ZC / 2;
  constexpr int NT = kFusedAC;
  constexpr int HY = NY / 2;
  constexpr int QN = HY * NB;  // positions (ky, c)
  static_assert(2 * QN <= NT, "one position per lane pair");
  constexpr int PG = fa_pg<A, 8>();
  constexpr int TNT = NT / PG;
  // a transform owned by one wavefront needs no workgroup barrier between its stages
  using Sy = std::conditional_t<TNT == 64, WaveSync, BlockSync>;
  constexpr int SLOTS = lds_slots(NY * NB);
  using L = Tile<NB, NB, 1, true>;
  __shared__ cplx<T> tile[PG * SLOTS];
  __shared__ cplx<T> tw[NY];
  lds_poison(tile, tw);

  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const BoxGeom g = br->g;
  const int tid = threadIdx.x;
  const int sub = tid / TNT, stid = tid - sub * TNT;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int j = t / nzc;
  const int z0 = (t - j * nzc) * ZC;
  const int zn = min(ZC, nz - z0);
  gmem<const cplx<T>>* W = hbm(static_cast<const cplx<T>*>(br->W));
  gmem<T>* phi = hbm(static_cast<T*>(br->phi));
  cplx<T>* mytile = tile + sub * SLOTS;
  load_twiddles<T, NY, NT>(tw, twy, tid);

  const int q = tid >> 1, h = tid & 1;  // position and column of this lane
  const bool qv = q < QN;
  const int ky = qv ? q / NB : 0, c = qv ? q - ky * NB : 0;
  PlanePhase pp;
  pp.init(ky, j, B, br->fy);
  cplx<T> acc[A];
  if (qv && 2 * c + h < zn) {
    gmem<const cplx<T>>* src = W + ((size_t)ky * B + j) * nz + z0 + 2 * c + h;
    const size_t plane = (size_t)HY * B * nz;  // W stride between consecutive k1
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) acc[k1] = cmulc<T>(src[k1 * plane], twx[j * k1]);  // j k1 < Nx
  } else {
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) acc[k1] = mk<T>(T(0), T(0));
  }
  Dft<A, +1, T>::run(acc);

  const bool sasha = g.method == 1;
  double c2 = 0.0, c1 = 0.0;
  if (sasha) {
    c2 = hbm(br->coef)->c2;
    c1 = hbm(br->coef)->c1;
  }
  const double dz = g.lz / nz;
#pragma unroll
  for (int a0 = 0; a0 < A; a0 += PG) {
    // the lane pairs write their positions of planes a0 .. a0+PG-1 as Hermitian columns
#pragma unroll
    for (int sp = 0; sp < PG; ++sp) {
      cplx<T>* tl = tile + sp * SLOTS;
      if (tid < NB) tl[L::at(HY, tid)] = mk<T>(T(0), T(0));  // y Nyquist
      const cplx<T> mine = cmulc<T>(acc[a0 + sp], mk<T>((T)pp.pr, (T)pp.pi));  // exp(-i theta), conjugated
      const cplx<T> other = mk<T>(__shfl_xor(mine.x, 1), __shfl_xor(mine.y, 1));
      const cplx<T> av = h ? other : mine, bv = h ? mine : other;
      if (qv) {
        if (ky == 0) {
          if (h == 0) tl[L::at(0, c)] = mk<T>(av.x, bv.x);
        } else if (h == 0) {
          tl[L::at(ky, c)] = mk<T>(av.x - bv.y, av.y + bv.x);
        } else {
          tl[L::at(NY - ky, c)] = mk<T>(av.x + bv.y, bv.x - av.y);
        }
      }
      pp.step();
    }
    __syncthreads();
    // PG thread groups run the inverse y transforms of their planes straight to phi
    const int x = j + B * (a0 + sub);
    gmem<T>* dst = phi + (size_t)x * NY * nz + z0;
    auto store = [&](int e, int cc, cplx<T> v) {
      if (2 * cc < zn) {
        if (sasha) {
          const double za = -0.5 * g.lz + (z0 + 2 * cc + 0.5) * dz;
          const double zb = za + dz;
          v.x = (T)((double)v.x + (c2 * za + c1) * za);
          v.y = (T)((double)v.y + (c2 * zb + c1) * zb);
        }
        *reinterpret_cast<gmem<cplx<T>>*>(dst + (size_t)e * nz + 2 * cc) = v;
      }
    };
    if constexpr (LIN) {
      YInterp yi;
      yi.init(br->shy * (x + 0.5), NY);
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, +1, true, true, 0, 1, Sy>(
          mytile, TwS<T>{tw}, stid, [&](int e, int cc) { return mytile[L::at(e, cc)]; },
          [&](int e, int cc, cplx<T> v) { mytile[L::at(e, cc)] = v; });
      Sy::sync();
      for (int w = stid; w < NY * NB; w += TNT) {
        const int cc = w % NB, e = w / NB;
        store(e, cc, yi.sample<T>(e, NY, [&](int y) { return mytile[L::at(y, cc)]; }));
      }
    } else {
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, +1, true, false, 0, 1, Sy>(
          mytile, TwS<T>{tw}, stid, [&](int e, int cc) { return mytile[L::at(e, cc)]; }, store);
    }
    __syncthreads();  // the tiles are rebuilt for the next planes
  }
}

// ------------------------------------------------------------------------------------------
// Pass B: one block per (k1, my) item.
// The B-point DFT across the j pencils runs in registers (one thread per z) and parks the B
// pencils in the LDS tile.  Every wavefront then takes tuples of Q pencil groups (PW pencils
// each): it lifts the inputs of the tuple into registers, uses the tuple's tile area as its
// exchange buffer for the padded z transform, the Green multiply for Kx = k1 + A k2 and the
// inverse of each group in turn, and writes the results back; no workgroup barrier and no LDS
// beyond the tile.  A barrier, and the inverse B-point DFT goes back to HBM.  Float plans take
// the k = 0 pencil (tile 0, pencil 0) in double as a direct convolution with the
// time-independent real-space kernel h.

// pencils per transform (about eight points per lane; Q such groups share one tile area, whose
// Q * PW * Nz slots are exactly one group's padded exchange buffer) and wavefronts per block
template <int M, int B, int Q> constexpr int fb_pw() {
  constexpr int a = M >= 512 ? 1 : 512 / M;
  return a < B / Q ? a : B / Q;
}
template <int M, int B, int Q> constexpr int fb_tuples() { return B / (Q * fb_pw<M, B, Q>()); }
template <int M, int B, int Q> constexpr int fb_waves() { return fb_tuples<M, B, Q>() < 4 ? fb_tuples<M, B, Q>() : 4; }
template <int M, int B, int Q> constexpr int fb_threads() { return 64 * fb_waves<M, B, Q>(); }

// Twiddles: the stage-major table of the forward schedule of M, then that of the inverse one if
// it differs.  When one table serves both and the tile's spare pad8 slots can hold it, it lives
// there (TwH), which keeps pass B's LDS small enough for four blocks per CU in float (M = 512 in
// float needs neither: its twiddles live in registers, below).
template <int M, int B, int Q> constexpr bool fb_tw_in_holes() {
  return same_schedule<typename ZSched<M>::F, typename ZSched<M>::I>() && B * (M / Q) >= 8 * (M - 1) + 8;
}
// Float plans whose z schedule gives each lane at most two butterflies per stage keep the lane's
// twiddles in registers, read once per block from the table in HBM: pass B is bound by LDS
// issue, and those reads would be the same for every pencil.  The hint asks for at least three
// waves per SIMD (the M = 512 kernel fits four).
template <typename T, int M, int B, int Q> constexpr bool fb_tw_in_registers() {
  using RL = typename ZSched<M>::F;
  return std::is_same<T, float>::value && fb_tw_in_holes<M, B, Q>() && max_per<RL, M, fb_pw<M, B, Q>()>() <= 2;
}
template <typename T, int M, int B, int Q> constexpr int fb_waves_per_eu() {
  if constexpr (fb_tw_in_registers<T, M, B, Q>())
    return 3;
  else
    return (sizeof(T) == 4 && fb_tw_in_holes<M, B, Q>()) ? 4 : 1;
}

template <typename T, int M, int B, int Q> struct FbShared {
  static constexpr int PW = fb_pw<M, B, Q>();
  static constexpr int NZ = M / Q;
  static constexpr bool kF32 = std::is_same<T, float>::value;
  static constexpr bool kOneTw = same_schedule<typename ZSched<M>::F, typename ZSched<M>::I>();
  // register twiddles (read once from HBM): the tile needs no twiddle slots, and at M = 512 it
  // takes the padding with fewer bank conflicts in the 8.8.8 exchanges
  static constexpr bool kTwReg = fb_tw_in_registers<T, M, B, Q>();
  // the float 8.8.8 one-pencil exchange: three spare slots per 32 (double tiles keep pad8, whose
  // spare slots hold the twiddle table; one spare slot per 16 measured slower there)
  static constexpr int PAD = (kTwReg && PW == 1 && M == 512) ? 1 : 0;
  static constexpr bool kHoles = !kTwReg && PAD == 0 && fb_tw_in_holes<M, B, Q>();
  cplx<T> tile[pad_slots<PAD>(B * NZ)];
  cplx<T> tw[(kHoles || kTwReg) ? 1 : kOneTw ? M : 2 * M];
  T pa0[B], pe[B], pik[B], pk2[B], psp[B];  // Green's-function coefficients of the B modes
};

template <typename T, int M, int B, int Q> __device__ __forceinline__ auto fb_twf(const FbShared<T, M, B, Q>& sh) {
  if constexpr (FbShared<T, M, B, Q>::kHoles)
    return TwH<T>{sh.tile};
  else
    return TwS<T>{sh.tw};
}
template <typename T, int M, int B, int Q> __device__ __forceinline__ auto fb_twi(const FbShared<T, M, B, Q>& sh) {
  if constexpr (FbShared<T, M, B, Q>::kHoles)
    return TwH<T>{sh.tile};
  else
    return TwS<T>{sh.tw + (FbShared<T, M, B, Q>::kOneTw ? 0 : M)};
}

// one (k1, my) item of a box
template <typename T> struct FbItem {
  const BoxRec* br;
  int t, k1, my;
  gmem<cplx<T>>* base;  // the item's B pencils, B*Nz contiguous values
  bool own0;      // float plans: this item holds Kx = Ky = 0 (pencil k2 = 0)
};

template <typename T, int M, int B, int Q>
__device__ __forceinline__ FbItem<T> fb_item(const BoxRec* br, int t) {
  FbItem<T> it;
  it.br = br;
  it.t = t;
  const int hy = br->g.ny / 2;
  it.k1 = t / hy;
  it.my = t - it.k1 * hy;
  it.base = hbm(static_cast<cplx<T>*>(br->W)) + (size_t)t * B * (M / Q);
  it.own0 = std::is_same<T, float>::value && t == 0;
  return it;
}

// Green's-function scalars of the B pencils (double, rounded once), and for SASHA the mean and
// centre of mass from the pass-A partial sums (first wavefront of the box's first item)
template <typename T, int M, int B, int Q>
__device__ __forceinline__ void fb_scalars(FbShared<T, M, B, Q>& sh, const FbItem<T>& it, int A, int tid) {
  const BoxRec* br = it.br;
  const BoxGeom& g = br->g;
  const bool sasha = g.method == 1;
  if (tid < B) {
    const double two_pi = 6.283185307179586476925286766559;
    const double Ky = (two_pi / g.ly) * it.my;
    const int mx = it.k1 + A * tid;
    const int sx = mx < g.nx / 2 ? mx : mx - g.nx;
    const double kx = (two_pi / g.lx) * sx + br->s * Ky;
    const ModeGreen<T> c = mode_green<T>(kx * kx + Ky * Ky, mx == 0 && it.my == 0, sasha, g.L, br->scale);
    sh.pa0[tid] = c.a0;
    sh.pe[tid] = c.e;
    sh.pik[tid] = c.ik;
    sh.pk2[tid] = c.k2;
    sh.psp[tid] = c.zero;
  }
  if (sasha && it.t == 0 && tid < 64) {
    double a = 0.0, b = 0.0;
    for (int i = tid; i < br->npartials; i += 64) {
      a += hbm(br->partials)[2 * i];
      b += hbm(br->partials)[2 * i + 1];
    }
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      b += __shfl_xor(b, o);
    }
    if (tid == 0) {
      SashaCoef c;
      c.c2 = 0.0;
      c.c1 = 0.0;
      if (a != 0.0) {
        const double mean = a / ((double)g.nx * g.ny * g.m);
        c.c2 = 0.5 * br->fourpiG * mean;
        c.c1 = -br->fourpiG * mean * (b / a);
      }
      *hbm(br->coef) = c;
    }
  }
}

// B-point DFT across j for each z; src(jj, z) is element z of pencil jj
template <typename T, int M, int B, int Q, int NT, class Src>
__device__ __forceinline__ void fb_dft_in(FbShared<T, M, B, Q>& sh, int tid, Src&& src) {
  constexpr int NZ = M / Q;
  constexpr int ZPT = (NZ + NT - 1) / NT;
  using LT = Tile<B, 1, NZ, false, FbShared<T, M, B, Q>::PAD>;  // parked pencils: element z of pencil k2
#pragma unroll
  for (int zi = 0; zi < ZPT; ++zi) {
    const int z = tid + zi * NT;
    if (NZ % NT == 0 || z < NZ) {
      cplx<T> v[B];
#pragma unroll
      for (int jj = 0; jj < B; ++jj) v[jj] = src(jj, z);
      Dft<B, -1, T>::run(v);
      // NZ is a multiple of the padding period: pencil k2 starts k2 * map(NZ) slots further on
      const int mz = LT::map(z);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) sh.tile[mz + k2 * LT::map(NZ)] = v[k2];
    }
  }
}

// wavefront-private padded z transforms, Green multiply and inverse: Q groups per tile area
template <typename T, int M, int B, int Q, int WV>
__device__ __forceinline__ void fb_pencils(FbShared<T, M, B, Q>& sh, const FbItem<T>& it, int tid,
                                           const cplx<T>* __restrict__ twm) {
  constexpr int PW = fb_pw<M, B, Q>();
  constexpr int NTUP = fb_tuples<M, B, Q>();
  constexpr int NZ = M / Q;
  static_assert(Q * PW * NTUP == B, "groups must tile the B pencils");
  constexpr int PAD = FbShared<T, M, B, Q>::PAD;
  using LT = Tile<B, 1, NZ, false, PAD>;
  using LW = Tile<PW, 1, M, false, PAD>;  // one group's exchange layout inside its tuple's tile area
  using RF = typename ZSched<M>::F;
  using RI = typename ZSched<M>::I;
  using S0 = Stage<T, M, RF, 0, LW, 64, -1>;
  using SL = Stage<T, M, RI, RI::n - 1, LW, 64, +1>;
  constexpr int RIN = (S0::R % Q == 0) ? S0::R / Q : S0::R;
  constexpr int ROUT = (SL::R % Q == 0) ? SL::R / Q : SL::R;
  const bool own0 = it.own0;
  const int wave = tid >> 6, lane = tid & 63;
  cplx<T>* tile = sh.tile;
  // the lane's twiddles, the same for every pencil, read once from HBM when registers allow (the
  // inverse schedule equals the forward one wherever this applies: fb_tw_in_holes)
  constexpr bool kTwReg = fb_tw_in_registers<T, M, B, Q>();
  TwReg<T, M, RF, LW, 64, TwS<T>> twr{TwS<T>{twm}};  // from the stage-major table in HBM
  if constexpr (kTwReg) twr.load(lane);
  // the z-table rows of this lane's spectrum elements: the same for every pencil it transforms
  constexpr int NSL = spectrum_slots<T, M, LW, 64>();
  ZRow<T> zr[NSL];
  {
    gmem<const T>* zt = hbm(static_cast<const T*>(it.br->zt));
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
      const int mz = spectrum_slot<T, M, LW, 64>(lane, i);
      zr[i] = zrow(zt, mz < 0 ? 0 : mz);
    }
  }
  const int mlane = LT::map(lane);
#pragma unroll 1
  for (int tu = wave; tu < NTUP; tu += WV) {
    const int k0 = Q * PW * tu;  // first pencil of the tuple
    cplx<T>* area = tile + pad_map<PAD>(k0 * NZ);  // Q * PW * NZ = PW * M logical slots
    auto skip = [&](int k2) { return own0 && k2 == 0; };
    cplx<T> in[Q][S0::PER][S0::R];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if constexpr (PAD != 0) {
        // one pencil per transform and e = lane + 64 r: slot map(lane) + r map(64) in its pencil
        static_assert(PW == 1 && S0::NBF == 64 && S0::PER == 1, "the 512-point layout");
        S0::template read_fn<RIN>(in[q], lane, [&](int e, int, int i) {
          const int k2 = k0 + q;
          return (e < NZ && !skip(k2)) ? area[q * LT::map(NZ) + mlane + (i % S0::R) * LT::map(64)]
                                       : mk<T>(T(0), T(0));
        });
      } else {
        S0::template read_fn<RIN>(in[q], lane, [&](int e, int p) {
          const int k2 = k0 + q * PW + p;
          return (e < NZ && !skip(k2)) ? tile[LT::at(e, k2)] : mk<T>(T(0), T(0));
        });
      }
    }
    WaveSync::sync();  // the area is free once every lane holds its inputs
    cplx<T> out[Q][SL::PER][SL::R];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      __builtin_amdgcn_sched_barrier(0);  // one transform at a time (register pressure)
      const int kq = k0 + q * PW;
      fft_fwd_op_inv<T, M, LW, 64, 0, Q, WaveSync>(
          area, [&] { if constexpr (kTwReg) return twr; else return fb_twf(sh); }(),
          [&] { if constexpr (kTwReg) return twr; else return fb_twi(sh); }(), lane,
          [&](int, int, int i) { return in[q][i / S0::R][i % S0::R]; },
          [&](int, int p, cplx<T>& v, int i) {
            const int k2 = kq + p;
            // float: the k = 0 pencil (own0) is neither read nor written back here
            const T gk = FbShared<T, M, B, Q>::kF32
                             ? green_at_nonzero(sh.pa0[k2], sh.pe[k2], sh.pik[k2], sh.pk2[k2], zr[i])
                             : green_at(sh.pa0[k2], sh.pe[k2], sh.pik[k2], sh.pk2[k2], sh.psp[k2], zr[i]);
            v.x *= gk;
            v.y *= gk;
          },
          [&](int, int, cplx<T> v, int i) { out[q][i / SL::R][i % SL::R] = v; });
      WaveSync::sync();
    }
    // the exchange reads are done: the results go back into the area
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if constexpr (PAD != 0) {
        static_assert(SL::NS == 64 && SL::PER == 1, "the 512-point layout");
        SL::template write_fn<ROUT>(out[q], lane, [&](int e, int, cplx<T> v, int i) {
          const int k2 = k0 + q;
          if (e < NZ && !skip(k2)) area[q * LT::map(NZ) + mlane + (i % SL::R) * LT::map(64)] = v;
        });
      } else {
        SL::template write_fn<ROUT>(out[q], lane, [&](int e, int p, cplx<T> v) {
          const int k2 = k0 + q * PW + p;
          if (e < NZ && !skip(k2)) tile[LT::at(e, k2)] = v;
        });
      }
    }
    WaveSync::sync();  // this wavefront's next tuple starts from fresh reads
  }
}

// inverse B-point DFT across k2, store to the item's pencils in HBM
template <typename T, int M, int B, int Q, int NT>
__device__ __forceinline__ void fb_dft_out(FbShared<T, M, B, Q>& sh, const FbItem<T>& it, int tid) {
  constexpr int NZ = M / Q;
  constexpr int ZPT = (NZ + NT - 1) / NT;
  using LT = Tile<B, 1, NZ, false, FbShared<T, M, B, Q>::PAD>;
  const double scale = it.br->scale;
  if (FbShared<T, M, B, Q>::kF32 && it.own0) {
    // the real k = 0 pencil input in double, from the item's pencils (still in HBM), parked as a
    // float pair (hi, lo) in the tile slots of pencil 0, whose transformed values are not used
#pragma unroll
    for (int zi = 0; zi < ZPT; ++zi) {
      const int z = tid + zi * NT;
      if (NZ % NT == 0 || z < NZ) {
        double sx = 0.0;
#pragma unroll
        for (int jj = 0; jj < B; ++jj) sx += (double)it.base[(size_t)jj * NZ + z].x;
        const T hi = (T)sx;
        sh.tile[LT::at(z, 0)] = mk<T>(hi, (T)(sx - (double)hi));
      }
    }
    __syncthreads();
    // every thread takes its pencil values into registers; then the slots after pencil 0 hold
    // the convolution kernel h (M doubles), so that the convolution reads it from LDS
    cplx<T> vk[ZPT][B];
#pragma unroll
    for (int zi = 0; zi < ZPT; ++zi) {
      const int z = tid + zi * NT;
      if (NZ % NT == 0 || z < NZ) {
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) vk[zi][k2] = sh.tile[LT::map(z) + k2 * LT::map(NZ)];
      }
    }
    static_assert(pad_map<LT::PAD>(NZ) + M <= pad_slots<LT::PAD>(B * NZ), "h fits after pencil 0");
    double* hl = reinterpret_cast<double*>(sh.tile + LT::map(NZ));
    __syncthreads();  // every pencil value has been read
    {
      gmem<const double>* h = hbm(it.br->k0h);
      for (int i = tid; i < M; i += NT) hl[i] = h[i];
    }
    __syncthreads();
#pragma unroll
    for (int zi = 0; zi < ZPT; ++zi) {
      const int z = tid + zi * NT;
      if (NZ % NT == 0 || z < NZ) {
        // the k = 0 pencil in double: the padded circular convolution
        // phi_0[z] = scale sum_z' h[(z - z') mod M] d0[z'], four partial sums over z' = 4i + u
        static_assert(NZ % 4 == 0, "z cells in groups of four");
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
        for (int zp = 0; zp < NZ; zp += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int d = z - zp - u;
            const cplx<T> d0 = sh.tile[LT::at(zp + u, 0)];
            acc[u] += hl[d < 0 ? d + M : d] * ((double)d0.x + (double)d0.y);
          }
        }
        auto& v = vk[zi];
        v[0] = mk<T>((T)(((acc[0] + acc[1]) + (acc[2] + acc[3])) * scale), T(0));
        Dft<B, +1, T>::run(v);
#pragma unroll
        for (int jj = 0; jj < B; ++jj) it.base[(size_t)jj * NZ + z] = v[jj];
      }
    }
    return;
  }
#pragma unroll
  for (int zi = 0; zi < ZPT; ++zi) {
    const int z = tid + zi * NT;
    if (NZ % NT == 0 || z < NZ) {
      cplx<T> v[B];
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k2] = sh.tile[LT::map(z) + k2 * LT::map(NZ)];
      Dft<B, +1, T>::run(v);
#pragma unroll
      for (int jj = 0; jj < B; ++jj) it.base[(size_t)jj * NZ + z] = v[jj];
    }
  }
}

template <typename T, int M, int B, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fb_waves_per_eu<T, M, B, Q>()))) void k_fb(GroupArgs ga, const BoxRec* __restrict__ recs,
                                            const cplx<T>* __restrict__ twm) {
  constexpr int WV = fb_waves<M, B, Q>();
  constexpr int NT = 64 * WV;
  __shared__ FbShared<T, M, B, Q> sh;
  lds_poison(sh);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const int tid = threadIdx.x;
  const FbItem<T> it = fb_item<T, M, B, Q>(br, t);
  if constexpr (FbShared<T, M, B, Q>::kTwReg) {
    // each lane reads its own twiddles from HBM in fb_pencils
  } else if constexpr (FbShared<T, M, B, Q>::kHoles) {
    load_twiddles<T, M - 1, NT, 9, 8>(sh.tile, twm, tid);
  } else {
    load_twiddles<T, FbShared<T, M, B, Q>::kOneTw ? M : 2 * M, NT>(sh.tw, twm, tid);
  }
  fb_scalars(sh, it, it.br->g.nx / B, tid);  // A = Nx/B of this block's box
  fb_dft_in<T, M, B, Q, NT>(sh, tid,
                                   [&](int jj, int z) { return it.base[(size_t)jj * (M / Q) + z]; });
  __syncthreads();
  fb_pencils<T, M, B, Q, WV>(sh, it, tid, twm);
  __syncthreads();
  fb_dft_out<T, M, B, Q, NT>(sh, it, tid);
}

// Pass B for a launch group whose boxes differ in M <= 256 (float, padding 2): every block runs
// the body of its own box's M with that box's z twiddles, so the groups of a batch that would
// each be one launch per M share one, and their blocks overlap instead of each launch waiting
// for its slowest block.  An item of M <= 128 needs fewer than four wavefronts: a block then
// takes IPB consecutive items of its box, one per wavefront group, each with its own LDS part.
constexpr int kMultiMMax = 256;
template <int M, int B, int Q> constexpr int fb_multi_ipb() { return 4 / fb_waves<M, B, Q>(); }
template <typename T, int M, int B, int Q> constexpr size_t fb_multi_bytes() {
  return fb_multi_ipb<M, B, Q>() * sizeof(FbShared<T, M, B, Q>);
}
template <typename T, int B, int Q> constexpr size_t fb_multi_lds() {
  constexpr size_t s[5] = {fb_multi_bytes<T, 32, B, Q>(), fb_multi_bytes<T, 64, B, Q>(), fb_multi_bytes<T, 128, B, Q>(),
                           fb_multi_bytes<T, 192, B, Q>(), fb_multi_bytes<T, 256, B, Q>()};
  size_t m = 0;
  for (size_t v : s) m = v > m ? v : m;
  return m;
}
// items per block of a box in such a group (host side: the box's block count is items / IPB)
inline int fb_multi_items_per_block(int m) {
  switch (m) {
    case 32: return fb_multi_ipb<32, kFusedB16, 2>();
    case 64: return fb_multi_ipb<64, kFusedB16, 2>();
    case 128: return fb_multi_ipb<128, kFusedB16, 2>();
    case 192: return fb_multi_ipb<192, kFusedB16, 2>();
    case 256: return fb_multi_ipb<256, kFusedB16, 2>();
    default: return 0;
  }
}

template <typename T, int M, int B, int Q>
__device__ __forceinline__ void fb_multi_body(const BoxRec* br, int t, cplx<T>* lds) {
  constexpr int WV = fb_waves<M, B, Q>();
  constexpr int NT = 64 * WV;
  constexpr int IPB = fb_multi_ipb<M, B, Q>();
  using Sh = FbShared<T, M, B, Q>;
  static_assert(sizeof(Sh) % sizeof(cplx<T>) == 0, "item parts stay aligned");
  const int sub = (int)threadIdx.x / NT, tid = (int)threadIdx.x - sub * NT;
  Sh& sh = *reinterpret_cast<Sh*>(lds + sub * (sizeof(Sh) / sizeof(cplx<T>)));
  const cplx<T>* twm = static_cast<const cplx<T>*>(br->twz);
  const FbItem<T> it = fb_item<T, M, B, Q>(br, t * IPB + sub);
  if constexpr (Sh::kTwReg) {
    // each lane reads its own twiddles from HBM in fb_pencils
  } else if constexpr (Sh::kHoles) {
    load_twiddles<T, M - 1, NT, 9, 8>(sh.tile, twm, tid);
  } else {
    load_twiddles<T, Sh::kOneTw ? M : 2 * M, NT>(sh.tw, twm, tid);
  }
  fb_scalars(sh, it, br->g.nx / B, tid);
  fb_dft_in<T, M, B, Q, NT>(sh, tid, [&](int jj, int z) { return it.base[(size_t)jj * (M / Q) + z]; });
  __syncthreads();
  fb_pencils<T, M, B, Q, WV>(sh, it, tid, twm);
  __syncthreads();
  fb_dft_out<T, M, B, Q, NT>(sh, it, tid);
  // in float the k = 0 item passes three more workgroup barriers in fb_dft_out than the others:
  // the other items of its block (t = 0) pass as many, so that every wavefront meets the same count
  if constexpr (IPB > 1 && Sh::kF32) {
    if (t == 0 && !it.own0) {
      __syncthreads();
      __syncthreads();
      __syncthreads();
    }
  }
}

template <typename T, int B, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_fb_multi(GroupArgs ga,
                                                                                           const BoxRec* __restrict__ recs) {
  __shared__ cplx<T> lds[fb_multi_lds<T, B, Q>() / sizeof(cplx<T>)];
  lds_poison(lds);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  switch (br->g.m) {
    case 32: fb_multi_body<T, 32, B, Q>(br, t, lds); break;
    case 64: fb_multi_body<T, 64, B, Q>(br, t, lds); break;
    case 128: fb_multi_body<T, 128, B, Q>(br, t, lds); break;
    case 192: fb_multi_body<T, 192, B, Q>(br, t, lds); break;
    default: fb_multi_body<T, 256, B, Q>(br, t, lds); break;
  }
}

template <typename T>
hipError_t launch_fused_impl(int kind, int len, int a, int variant, int q, bool lin, GroupArgs ga, int blocks,
                             const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st);
template <> hipError_t launch_fused_impl<float>(int, int, int, int, int, bool, GroupArgs, int, const BoxRec*, const void*,
                                                const void*, hipStream_t);
template <> hipError_t launch_fused_impl<double>(int, int, int, int, int, bool, GroupArgs, int, const BoxRec*, const void*,
                                                 const void*, hipStream_t);

template <typename T> int fused_ac_tiles_t(const BoxGeom& g, int variant) {
  const int zc = variant == 1 ? fa_zc<T, 1>() : variant == 2 ? fa_zc<T, 2>() : variant == 3 ? kSplitZC : fa_zc<T, 0>();
  return kFusedB16 * ((g.nz + zc - 1) / zc);
}

}  // namespace sbp
