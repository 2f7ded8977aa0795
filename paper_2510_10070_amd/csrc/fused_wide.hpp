// Fused three-pass schedule for wide float boxes, Nx in {512, 1024} and Ny in {512, 1024}, with
// padding 2 and M <= 512.  Same four-step split as the narrow schedule,
//   X[k1 + A k2] = sum_j w_B^(j k2) [ w_Nx^(j k1) sum_a x[j + B a] w_A^(a k1) ],
// but with B = 64 pencils per pass-B item and A = Nx/64 in {8, 16}, so that pass A holds 8 or 16
// planes of a y spectrum rather than 32 or 64, which do not fit a CU.  The price is in pass B: a
// 64-pencil tile (144 KB of LDS at M = 512, one 1024-thread block per CU) and a 64-point DFT
// across the pencils, taken as 8 x 8 through LDS.  The intermediate layout is the narrow one,
// W[k1][my][j][z] with j < 64.
#pragma once

#include "fused.hpp"
#include "wide.hpp"

namespace sbp {

constexpr int kWideB = 64;          // pencils per pass-B item
constexpr int kWideThreads = 1024;  // threads of every wide kernel (one block per CU)

// real z cells per pass-A/C tile: 16-byte rows, or 8-byte rows at Ny = 1024 with A = 16, where a
// lane would otherwise hold 32 complex values (the register file has room for 16 beside the y
// transform)
__host__ __device__ constexpr int wide_zc(int ny, int a) { return ny * a >= 16384 ? 2 : 4; }

inline bool fused_wide_supported(int nx, int ny, int nz, int m) {
  return (nx == 512 || nx == 1024) && (ny == 512 || ny == 1024) && m == 2 * nz &&
         (m == 64 || m == 128 || m == 256 || m == 512);
}
inline int fused_wide_ac_tiles(const BoxGeom& g) {
  const int zc = wide_zc(g.ny, g.nx / kWideB);
  return kWideB * ((g.nz + zc - 1) / zc);
}

// ------------------------------------------------------------------------------------------
// Pass A: one block per (j, chunk of ZC z cells).  The two real z columns of a position
// (ky, c) are held by a lane pair, one column per lane, and each lane pair owns POS positions,
// so that every lane keeps POS x A complex values (at most 16).  PG planes are transformed side
// by side (four of 256 threads over 16-byte rows; over 8-byte rows all sixteen, one wavefront
// each).

template <int NY, int A> struct WideAc {
  static constexpr int ZC = wide_zc(NY, A);
  static constexpr int NB = ZC / 2;       // complex columns per y row
  static constexpr int NT = kWideThreads;
  static constexpr int HY = NY / 2;
  static constexpr int QN = HY * NB;      // positions (ky, c)
  static constexpr int LP = NT / 2;       // lane pairs
  static_assert(QN % LP == 0, "positions tile the lane pairs");
  static constexpr int POS = QN / LP;
  // planes transformed side by side: over 8-byte rows all A = 16 at once, one wavefront each
  // (no workgroup barrier between the stages of a transform); over 16-byte rows four of 256
  // threads
  static constexpr int PG = NB == 1 ? A : 4;
  static_assert(A % PG == 0, "plane groups tile the planes");
  static constexpr int TNT = NT / PG;
  using Sy = std::conditional_t<TNT == 64, WaveSync, BlockSync>;
  static constexpr int PAD = 1;           // three spare slots per 32
  static constexpr int SLOTS = pad_slots<PAD>(NY * NB);
  using L = Tile<NB, NB, 1, true, PAD>;
};

template <int NY, int A, bool LIN>
__global__ __launch_bounds__(kWideThreads) void k_faw(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                      const cplx<float>* __restrict__ twy,
                                                      const cplx<float>* __restrict__ twx) {
  using T = float;
  using S = WideAc<NY, A>;
  using L = typename S::L;
  constexpr int B = kWideB, ZC = S::ZC, NB = S::NB, NT = S::NT, HY = S::HY, POS = S::POS, PG = S::PG;
  constexpr int TNT = S::TNT, SLOTS = S::SLOTS;
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

  const int lp = tid >> 1, h = tid & 1;  // lane pair and column of this lane
  PlanePhase pp[POS];
#pragma unroll
  for (int i = 0; i < POS; ++i) pp[i].init((lp + i * S::LP) / NB, j, B, br->fy);
  cplx<T> acc[POS][A];
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
    // the first planes' transforms pass a workgroup barrier after their first exchange write, so
    // that the twiddle table written by every wavefront is complete before its first read
    using Sy = typename S::Sy;
    if (a0 == 0)
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, -1, false, true, 0, 1, Sy, BlockSync>(mytile, TwS<T>{tw}, stid,
                                                                                          ld_plane, st_tile);
    else
      fft_run<T, NY, typename Fwd<NY>::L, L, TNT, -1, false, true, 0, 1, Sy>(mytile, TwS<T>{tw}, stid, ld_plane,
                                                                             st_tile);
    __syncthreads();
    // each lane separates its column of its positions from the Hermitian pairs and remaps them
#pragma unroll
    for (int sp = 0; sp < PG; ++sp) {
      const cplx<T>* tl = tile + sp * SLOTS;
#pragma unroll
      for (int i = 0; i < POS; ++i) {
        const int q = lp + i * S::LP;
        const int ky = q / NB, c = q - ky * NB;
        const cplx<T> c1 = tl[L::at(ky, c)];
        const cplx<T> c2 = tl[L::at((NY - ky) % NY, c)];
        const cplx<T> v = h == 0 ? mk<T>(T(0.5) * (c1.x + c2.x), T(0.5) * (c1.y - c2.y))
                                 : mk<T>(T(0.5) * (c1.y + c2.y), T(-0.5) * (c1.x - c2.x));
        acc[i][a0 + sp] = cmul<T>(v, mk<T>((T)pp[i].pr, (T)pp[i].pi));
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

  // A-point DFT across planes, twiddle w_Nx^(j k1), store this lane's column of each position
  const size_t plane = (size_t)HY * B * nz;  // W stride between consecutive k1
#pragma unroll
  for (int i = 0; i < POS; ++i) {
    const int q = lp + i * S::LP;
    const int ky = q / NB, c = q - ky * NB;
    Dft<A, -1, T>::run(acc[i]);
    if (2 * c + h < zn) {
      gmem<cplx<T>>* dst = W + ((size_t)ky * B + j) * nz + z0 + 2 * c + h;
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) dst[k1 * plane] = cmul<T>(acc[i][k1], twx[j * k1]);  // j k1 < Nx
    }
  }
}

// Pass C: the inverse of k_faw.  After the inverse A-point DFT and the remap phase the lane pair
// swaps its values, and each lane writes one of the two Hermitian slots of the position.
template <int NY, int A, bool LIN>
__global__ __launch_bounds__(kWideThreads) void k_fcw(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                      const cplx<float>* __restrict__ twy,
                                                      const cplx<float>* __restrict__ twx) {
  using T = float;
  using S = WideAc<NY, A>;
  using L = typename S::L;
  constexpr int B = kWideB, ZC = S::ZC, NB = S::NB, NT = S::NT, HY = S::HY, POS = S::POS, PG = S::PG;
  constexpr int TNT = S::TNT, SLOTS = S::SLOTS;
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

  const int lp = tid >> 1, h = tid & 1;
  PlanePhase pp[POS];
  cplx<T> acc[POS][A];
  const size_t plane = (size_t)HY * B * nz;
#pragma unroll
  for (int i = 0; i < POS; ++i) {
    const int q = lp + i * S::LP;
    const int ky = q / NB, c = q - ky * NB;
    pp[i].init(ky, j, B, br->fy);
    if (2 * c + h < zn) {
      gmem<const cplx<T>>* src = W + ((size_t)ky * B + j) * nz + z0 + 2 * c + h;
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) acc[i][k1] = cmulc<T>(src[k1 * plane], twx[j * k1]);  // j k1 < Nx
    } else {
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) acc[i][k1] = mk<T>(T(0), T(0));
    }
    Dft<A, +1, T>::run(acc[i]);
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
    // the lane pairs write their positions of planes a0 .. a0+PG-1 as Hermitian columns
#pragma unroll
    for (int sp = 0; sp < PG; ++sp) {
      cplx<T>* tl = tile + sp * SLOTS;
      if (tid < NB) tl[L::at(HY, tid)] = mk<T>(T(0), T(0));  // y Nyquist
#pragma unroll
      for (int i = 0; i < POS; ++i) {
        const int q = lp + i * S::LP;
        const int ky = q / NB, c = q - ky * NB;
        const cplx<T> mine = cmulc<T>(acc[i][a0 + sp], mk<T>((T)pp[i].pr, (T)pp[i].pi));  // exp(-i theta), conjugated
        const cplx<T> other = mk<T>(__shfl_xor(mine.x, 1), __shfl_xor(mine.y, 1));
        const cplx<T> av = h ? other : mine, bv = h ? mine : other;
        if (ky == 0) {
          if (h == 0) tl[L::at(0, c)] = mk<T>(av.x, bv.x);
        } else if (h == 0) {
          tl[L::at(ky, c)] = mk<T>(av.x - bv.y, av.y + bv.x);
        } else {
          tl[L::at(NY - ky, c)] = mk<T>(av.x + bv.y, bv.x - av.y);
        }
        pp[i].step();
      }
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
    using Sy = typename S::Sy;
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
// Pass B: one 1024-thread block per (k1, my) item of 64 pencils.  The 64-point DFT across the
// pencils j = r + 8 s, k2 = u + 8 v is split 8 x 8:
//   X[u + 8 v] = sum_r w_8^(r v) [ w_64^(r u) sum_s x[r + 8 s] w_8^(s u) ],
// the inner transform per (z, r) from HBM, the outer one per (z, u) in LDS.  Between the inner
// and the outer step the value (r, u) sits in the slots of pencil u + 8 r, so that the outer
// step of (z, u) reads and writes the same eight slots.  The padded z transforms, the Green
// multiply and their inverse are those of the narrow pass B (fb_pencils, sixteen wavefronts).
// The inverse runs the two steps in the opposite order.  w_64^m is the x twiddle w_Nx^(m A).

template <int M> using WideB = FbShared<float, M, kWideB, 2>;

template <int M>
__device__ __forceinline__ void fbw_dft_in(WideB<M>& sh, const FbItem<float>& it, int tid) {
  using T = float;
  constexpr int NZ = M / 2, NT = kWideThreads;
  using LT = Tile<kWideB, 1, NZ, false, WideB<M>::PAD>;  // element z of pencil k2
  const int A = it.br->g.nx / kWideB;
  gmem<const cplx<T>>* twx = hbm(static_cast<const cplx<T>*>(it.br->twx));
  for (int w = tid; w < 8 * NZ; w += NT) {
    const int z = w % NZ, r = w / NZ;
    cplx<T> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = it.base[(size_t)(r + 8 * s) * NZ + z];
    Dft<8, -1, T>::run(v);
#pragma unroll
    for (int u = 0; u < 8; ++u) sh.tile[LT::at(z, u + 8 * r)] = u == 0 ? v[0] : cmul<T>(v[u], twx[r * u * A]);
  }
  __syncthreads();
  for (int w = tid; w < 8 * NZ; w += NT) {
    const int z = w % NZ, u = w / NZ;
    cplx<T> v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = sh.tile[LT::at(z, u + 8 * r)];
    Dft<8, -1, T>::run(v);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh.tile[LT::at(z, u + 8 * k)] = v[k];
  }
}

// inverse 64-point DFT across k2 and store to the item's pencils in HBM.  The k = 0 pencil of
// item 0 is first replaced by its double convolution with h (as in the narrow pass B).
template <int M>
__device__ __forceinline__ void fbw_dft_out(WideB<M>& sh, double* hk, const FbItem<float>& it, int tid) {
  using T = float;
  constexpr int NZ = M / 2, NT = kWideThreads;
  static_assert(NZ <= NT && NZ % 4 == 0, "one z cell per thread in the k = 0 convolution");
  using LT = Tile<kWideB, 1, NZ, false, WideB<M>::PAD>;
  if (it.own0) {
    // the real k = 0 pencil input in double, from the item's pencils (still in HBM), parked as a
    // float pair (hi, lo) in the slots of pencil 0, whose transformed values are not used
    for (int z = tid; z < NZ; z += NT) {
      double sx = 0.0;
#pragma unroll 8
      for (int jj = 0; jj < kWideB; ++jj) sx += (double)it.base[(size_t)jj * NZ + z].x;
      const T hi = (T)sx;
      sh.tile[LT::at(z, 0)] = mk<T>(hi, (T)(sx - (double)hi));
    }
    {
      gmem<const double>* h = hbm(it.br->k0h);
      for (int i = tid; i < M; i += NT) hk[i] = h[i];
    }
    __syncthreads();
    // phi_0[z] = scale sum_z' h[(z - z') mod M] d0[z'], four partial sums over z' = 4i + u
    double r = 0.0;
    if (tid < NZ) {
      const int z = tid;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
      for (int zp = 0; zp < NZ; zp += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int d = z - zp - u;
          const cplx<T> d0 = sh.tile[LT::at(zp + u, 0)];
          acc[u] += hk[d < 0 ? d + M : d] * ((double)d0.x + (double)d0.y);
        }
      }
      r = ((acc[0] + acc[1]) + (acc[2] + acc[3])) * it.br->scale;
    }
    __syncthreads();  // every d0 has been read
    if (tid < NZ) sh.tile[LT::at(tid, 0)] = mk<T>((T)r, T(0));
    __syncthreads();
  }
  const int A = it.br->g.nx / kWideB;
  gmem<const cplx<T>>* twx = hbm(static_cast<const cplx<T>*>(it.br->twx));
  for (int w = tid; w < 8 * NZ; w += NT) {
    const int z = w % NZ, u = w / NZ;
    cplx<T> v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = sh.tile[LT::at(z, u + 8 * k)];
    Dft<8, +1, T>::run(v);
#pragma unroll
    for (int r = 0; r < 8; ++r) sh.tile[LT::at(z, u + 8 * r)] = r == 0 ? v[0] : cmulc<T>(v[r], twx[r * u * A]);
  }
  __syncthreads();
  for (int w = tid; w < 8 * NZ; w += NT) {
    const int z = w % NZ, r = w / NZ;
    cplx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = sh.tile[LT::at(z, u + 8 * r)];
    Dft<8, +1, T>::run(v);
#pragma unroll
    for (int s = 0; s < 8; ++s) it.base[(size_t)(r + 8 * s) * NZ + z] = v[s];
  }
}

template <int M>
__global__ __launch_bounds__(kWideThreads) void k_fbw(GroupArgs ga, const BoxRec* __restrict__ recs,
                                                      const cplx<float>* __restrict__ twm) {
  using T = float;
  constexpr int NT = kWideThreads;
  using Sh = WideB<M>;
  __shared__ Sh sh;
  __shared__ double hk[M];  // the k = 0 kernel h, read by item 0 only
  lds_poison(sh, hk);
  int t;
  const BoxRec* br = group_box(ga, recs, t);
  const int tid = threadIdx.x;
  const FbItem<T> it = fb_item<T, M, kWideB, 2>(br, t);
  if constexpr (Sh::kTwReg) {
    // each lane reads its own twiddles from HBM in fb_pencils
  } else if constexpr (Sh::kHoles) {
    load_twiddles<T, M - 1, NT, 9, 8>(sh.tile, twm, tid);
  } else {
    load_twiddles<T, Sh::kOneTw ? M : 2 * M, NT>(sh.tw, twm, tid);
  }
  fb_scalars(sh, it, br->g.nx / kWideB, tid);
  fbw_dft_in<M>(sh, it, tid);
  __syncthreads();
  fb_pencils<T, M, kWideB, 2, NT / 64>(sh, it, tid, twm);
  __syncthreads();
  fbw_dft_out<M>(sh, hk, it, tid);
}

}  // namespace sbp
