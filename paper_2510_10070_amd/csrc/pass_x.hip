// x pass of the streaming solve (steps a1 forward, a6 inverse): complex length-Nx transforms of
// the half spectrum W[x][my][z].  One workgroup per (my, chunk of ZC consecutive z cells);
// each of the Nx rows of the tile is ZC contiguous complex values (128 bytes where the tile
// fits in 64 KiB).
#include "fft_device.hpp"
#include "sbp_internal.hpp"

namespace sbp {

template <typename T, int N> constexpr int x_zc() {
  return sizeof(T) == 4 ? (N <= 512 ? 16 : 8) : (N <= 512 ? 8 : 4);
}
constexpr int kXThreads = 256;

template <typename T> __device__ __forceinline__ void ld2(const cplx<T>* p, cplx<T>* v);
template <> __device__ __forceinline__ void ld2<float>(const float2* p, float2* v) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = make_float2(q.x, q.y);
  v[1] = make_float2(q.z, q.w);
}
template <> __device__ __forceinline__ void ld2<double>(const double2* p, double2* v) {
  v[0] = p[0];
  v[1] = p[1];
}
template <typename T> __device__ __forceinline__ void st2(cplx<T>* p, const cplx<T>* v);
template <> __device__ __forceinline__ void st2<float>(float2* p, const float2* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
}
template <> __device__ __forceinline__ void st2<double>(double2* p, const double2* v) {
  p[0] = v[0];
  p[1] = v[1];
}

template <typename T, int NX, int D>
__global__ __launch_bounds__(kXThreads) void k_x(cplx<T>* __restrict__ W, const cplx<T>* __restrict__ twg, BoxGeom g) {
  constexpr int ZC = x_zc<T, NX>();
  constexpr int NT = kXThreads;
  using L = Tile<ZC, ZC, 1, true>;
  __shared__ cplx<T> tile[lds_slots(NX * ZC)];
  __shared__ cplx<T> tw[NX];
  const int tid = threadIdx.x;
  const int hy = g.ny / 2;
  const int nz = g.nz;
  const int nzc = (nz + ZC - 1) / ZC;
  const int tile_id = xcd_tile(blockIdx.x, hy * nzc);
  const int my = tile_id / nzc;
  const int z0 = (tile_id - my * nzc) * ZC;
  const size_t row = (size_t)hy * nz;  // stride between x rows
  cplx<T>* base = W + (size_t)my * nz + z0;
  load_twiddles<T, NX, NT>(tw, twg, tid);
  // pairs of complex values per access (nz and z0 are even)
  for (int w = tid; w < NX * ZC / 2; w += NT) {
    const int c = (w % (ZC / 2)) * 2, x = w / (ZC / 2);
    cplx<T> v[2] = {mk<T>(T(0), T(0)), mk<T>(T(0), T(0))};
    if (z0 + c < nz) ld2<T>(base + x * row + c, v);
    tile[L::at(x, c)] = v[0];
    tile[L::at(x, c + 1)] = v[1];
  }
  __syncthreads();
  lds_fft<T, NX, L, NT, D>(tile, tw, tid);
  for (int w = tid; w < NX * ZC / 2; w += NT) {
    const int c = (w % (ZC / 2)) * 2, x = w / (ZC / 2);
    if (z0 + c < nz) {
      cplx<T> v[2] = {tile[L::at(x, c)], tile[L::at(x, c + 1)]};
      st2<T>(base + x * row + c, v);
    }
  }
}

template <typename T, int NX>
static hipError_t x_t(int dir, const BoxGeom& g, void* W, const void* tw, hipStream_t st) {
  constexpr int ZC = x_zc<T, NX>();
  dim3 grid((g.ny / 2) * ((g.nz + ZC - 1) / ZC));
  if (dir < 0)
    hipLaunchKernelGGL((k_x<T, NX, -1>), grid, dim3(kXThreads), 0, st, (cplx<T>*)W, (const cplx<T>*)tw, g);
  else
    hipLaunchKernelGGL((k_x<T, NX, +1>), grid, dim3(kXThreads), 0, st, (cplx<T>*)W, (const cplx<T>*)tw, g);
  return hipGetLastError();
}

hipError_t launch_x(int prec, int dir, const BoxGeom& g, void* W, const void* tw_x, hipStream_t st) {
#define SBP_CASE(N_) \
  if (g.nx == N_) return prec ? x_t<float, N_>(dir, g, W, tw_x, st) : x_t<double, N_>(dir, g, W, tw_x, st);
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

}  // namespace sbp
