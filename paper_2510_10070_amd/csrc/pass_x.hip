// x pass of the streaming solve (steps a1 forward, a6 inverse): complex length-Nx transforms of
// the half spectrum W[x][my][z].  One workgroup per (my, chunk of ZC consecutive z cells);
// each of the Nx rows of the tile is ZC contiguous complex values.
#include "fft_device.hpp"
#include "sbp_internal.hpp"

namespace sbp {

template <typename T, int N> constexpr int x_zc() {
  return sizeof(T) == 4 ? (N <= 512 ? 8 : 4) : (N <= 512 ? 4 : 2);
}
constexpr int kXThreads = 256;

template <typename T, int NX, int D>
__global__ __launch_bounds__(kXThreads) void k_x(cplx<T>* __restrict__ W, const cplx<T>* __restrict__ tw, BoxGeom g) {
  constexpr int ZC = x_zc<T, NX>();
  constexpr int NT = kXThreads;
  __shared__ cplx<T> tile[NX * ZC];
  const int tid = threadIdx.x;
  const int my = blockIdx.x;
  const int z0 = blockIdx.y * ZC;
  const int nz = g.nz;
  const size_t row = (size_t)(g.ny / 2) * nz;  // stride between x rows
  cplx<T>* base = W + (size_t)my * nz + z0;
  for (int w = tid; w < NX * ZC; w += NT) {
    const int c = w % ZC, x = w / ZC;
    tile[w] = (z0 + c < nz) ? base[x * row + c] : mk<T>(T(0), T(0));
  }
  __syncthreads();
  lds_fft<T, NX, Tile<ZC, ZC, 1, true>, NT, D>(tile, tw, tid);
  for (int w = tid; w < NX * ZC; w += NT) {
    const int c = w % ZC, x = w / ZC;
    if (z0 + c < nz) base[x * row + c] = tile[w];
  }
}

template <typename T, int NX>
static hipError_t x_t(int dir, const BoxGeom& g, void* W, const void* tw, hipStream_t st) {
  constexpr int ZC = x_zc<T, NX>();
  dim3 grid(g.ny / 2, (g.nz + ZC - 1) / ZC);
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
