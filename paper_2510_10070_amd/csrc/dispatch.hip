// Precision dispatch of the pass launchers (no kernels are instantiated here).
#include "fused.hpp"

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

bool fused_ok(const BoxGeom& g) { return fused_supported(g.nx, g.ny, g.m); }
int fused_ac_tiles(int prec, const BoxGeom& g, int variant) {
  return prec ? fused_ac_tiles_t<float>(g, variant) : fused_ac_tiles_t<double>(g, variant);
}
int fused_b_tiles(const BoxGeom& g) { return (g.nx / kFusedB16) * (g.ny / 2); }
int fused_a(const BoxGeom& g) { return g.nx / kFusedB16; }
hipError_t launch_fused(int prec, int kind, int len, int a, int variant, int q, GroupArgs ga, int blocks,
                        const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st) {
  return prec ? launch_fused_impl<float>(kind, len, a, variant, q, ga, blocks, recs, tw, tw2, st)
              : launch_fused_impl<double>(kind, len, a, variant, q, ga, blocks, recs, tw, tw2, st);
}

}  // namespace sbp
