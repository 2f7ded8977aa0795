// Fused three-pass schedule for double: pass B and the launch dispatch.
#include "fused_launch.hpp"

namespace sbp {

// kind: 0 = pass A (len = Ny), 1 = pass B (len = M, q = padding), 2 = pass C (len = Ny);
// a = A = Nx/16 (passes A and C; pass B reads it from each box).  tw: y twiddles (A, C) or z
// twiddles (B); tw2: x twiddles (A, C).
template <>
hipError_t launch_fused_impl<double>(int kind, int len, int a, int variant, int q, bool lin, GroupArgs ga, int blocks,
                                 const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st) {
  return launch_fused_dispatch<double>(kind, len, a, q, variant, lin, ga, blocks, recs, tw, tw2, st);
}

}  // namespace sbp
