// Precision dispatch of the pass launchers (no kernels are instantiated here).
#include <cstring>

#include "fused_wide.hpp"

namespace sbp {

int y_tiles(int prec, const BoxGeom& g, int variant) {
  return prec ? y_tiles_t<float>(g, variant) : y_tiles_t<double>(g, variant);
}
int x_tiles(int prec, const BoxGeom& g, int variant) {
  return prec ? x_tiles_t<float>(g, variant) : x_tiles_t<double>(g, variant);
}
int z_tiles(int prec, const BoxGeom& g, int variant) {
  return prec ? z_tiles_t<float>(g, variant) : z_tiles_t<double>(g, variant);
}

hipError_t launch_y(int prec, bool forward, bool remap, int ny, int variant, GroupArgs ga, int blocks,
                    const BoxRec* recs, const void* tw, hipStream_t st) {
  return prec ? launch_y_impl<float>(forward, remap, ny, variant, ga, blocks, recs, tw, st)
              : launch_y_impl<double>(forward, remap, ny, variant, ga, blocks, recs, tw, st);
}
hipError_t launch_x(int prec, int dir, int nx, int variant, GroupArgs ga, int blocks, const BoxRec* recs,
                    const void* tw, hipStream_t st) {
  return prec ? launch_x_impl<float>(dir, nx, variant, ga, blocks, recs, tw, st)
              : launch_x_impl<double>(dir, nx, variant, ga, blocks, recs, tw, st);
}
hipError_t launch_z(int prec, int m, int variant, int q, GroupArgs ga, int blocks, const BoxRec* recs, const void* tw,
                    const void* tw64, hipStream_t st) {
  return prec ? launch_z_impl<float>(m, variant, q, ga, blocks, recs, tw, tw64, st)
              : launch_z_impl<double>(m, variant, q, ga, blocks, recs, tw, tw64, st);
}

}  // namespace sbp

namespace sbp {

// fused boxes with Nx > 256 are the wide float boxes (B = 64)
static int fused_bsize(const BoxGeom& g) { return g.nx > 256 ? kWideB : kFusedB16; }
bool fused_ok(const BoxGeom& g) { return fused_supported(g.nx, g.ny, g.m); }
bool fused_wide_ok(int prec, const BoxGeom& g) { return prec == 1 && fused_wide_supported(g.nx, g.ny, g.nz, g.m); }
int fused_ac_tiles(int prec, const BoxGeom& g, int variant) {
  if (g.nx > 256) return fused_wide_ac_tiles(g);
  return prec ? fused_ac_tiles_t<float>(g, variant) : fused_ac_tiles_t<double>(g, variant);
}
int fused_b_tiles(const BoxGeom& g) { return (g.nx / fused_bsize(g)) * (g.ny / 2); }
int fused_a(const BoxGeom& g) { return g.nx / fused_bsize(g); }
int fused_ac_multi_tiles(const BoxGeom& g) { return fused_ac_multi_tiles_t<float>(g); }
int fused_b_items_per_block(const BoxGeom& g, int pad) {
  if (pad != 2 || g.m > kMultiMMax || g.nx > 256) return 0;
  const int ipb = fb_multi_items_per_block(g.m);
  return ipb > 0 && fused_b_tiles(g) % ipb == 0 ? ipb : 0;
}
hipError_t launch_fused(int prec, int kind, int len, int a, int variant, int q, bool lin, GroupArgs ga, int blocks,
                        const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st) {
  if (variant == kWideVariant) {
    if (prec != 1) return hipErrorInvalidValue;
    return kind == 1 ? launch_fused_wide_b(len, q, ga, blocks, recs, tw, st)
                     : launch_fused_wide_ac(kind, len, a, lin, ga, blocks, recs, tw, tw2, st);
  }
  return prec ? launch_fused_impl<float>(kind, len, a, variant, q, lin, ga, blocks, recs, tw, tw2, st)
              : launch_fused_impl<double>(kind, len, a, variant, q, lin, ga, blocks, recs, tw, tw2, st);
}

}  // namespace sbp

namespace sbp {

// Per-solve records: the host writes them into a pinned ring slot and this kernel, the first of
// every solve, copies the slot into the device record array.  Direct launches pass the slot;
// a captured graph passes -1 and the kernel takes the slot from ctl[0], which the last block to
// finish advances (ctl[1] counts finished blocks), so the replayed graph never changes.
__global__ __launch_bounds__(256) void k_fetch(const BoxRec* __restrict__ ring, BoxRec* __restrict__ recs, int nrec,
                                               int nslots, int slot_arg, int* ctl) {
  const int slot = slot_arg >= 0 ? slot_arg : ctl[0];
  constexpr int W = sizeof(BoxRec) / sizeof(uint2);
  const size_t words = (size_t)nrec * W;
  const uint2* src = reinterpret_cast<const uint2*>(ring + (size_t)slot * nrec);
  uint2* dst = reinterpret_cast<uint2*>(recs);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
  if (slot_arg < 0) {
    __syncthreads();  // every thread of this block has read the slot number
    if (threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(&ctl[1], 1) == (int)gridDim.x - 1) {
        atomicExch(&ctl[1], 0);
        atomicExch(&ctl[0], slot + 1 == nslots ? 0 : slot + 1);
      }
    }
  }
}
static_assert(sizeof(BoxRec) % sizeof(uint2) == 0, "records are copied as 8-byte words");

// Direct launches of plans with few boxes pass the records by value: the kernel arguments reach
// device memory with the launch, so the copy needs no read of host memory across PCIe.
template <int N> struct RecArgs {
  BoxRec r[N];
};
template <int N>
__global__ __launch_bounds__(256) void k_fetch_args(RecArgs<N> in, BoxRec* __restrict__ recs, int nrec) {
  constexpr int W = sizeof(BoxRec) / sizeof(uint2);
  const uint2* src = reinterpret_cast<const uint2*>(in.r);
  uint2* dst = reinterpret_cast<uint2*>(recs);
  for (int i = threadIdx.x; i < nrec * W; i += blockDim.x) dst[i] = src[i];
}
template <int N> hipError_t fetch_args_n(const BoxRec* host, BoxRec* recs, int nrec, hipStream_t st) {
  RecArgs<N> in;
  std::memcpy(in.r, host, sizeof(BoxRec) * nrec);
  std::memset(in.r + nrec, 0, sizeof(BoxRec) * (N - nrec));
  hipLaunchKernelGGL(k_fetch_args<N>, dim3(1), dim3(256), 0, st, in, recs, nrec);
  return hipGetLastError();
}

hipError_t launch_fetch_args(const BoxRec* host, BoxRec* recs, int nrec, hipStream_t st) {
  if (nrec <= 1) return fetch_args_n<1>(host, recs, nrec, st);
  if (nrec <= 2) return fetch_args_n<2>(host, recs, nrec, st);
  if (nrec <= 4) return fetch_args_n<4>(host, recs, nrec, st);
  if (nrec <= kArgRecs) return fetch_args_n<kArgRecs>(host, recs, nrec, st);
  return hipErrorInvalidValue;
}

hipError_t launch_fetch(const BoxRec* ring, BoxRec* recs, int nrec, int nslots, int slot, int* ctl, hipStream_t st) {
  const size_t words = (size_t)nrec * (sizeof(BoxRec) / sizeof(uint2));
  const int blocks = (int)std::min<size_t>((words + 255) / 256, 256);
  hipLaunchKernelGGL(k_fetch, dim3(blocks), dim3(256), 0, st, ring, recs, nrec, nslots, slot, ctl);
  return hipGetLastError();
}

}  // namespace sbp
