// Fused pass B of the wide float schedule (Nx in {512, 1024}: 64 pencils per item).
#include "fused_wide.hpp"

namespace sbp {

// len = M (padding 2); tw: the stage-major z twiddles of M
hipError_t launch_fused_wide_b(int len, int q, GroupArgs ga, int blocks, const BoxRec* recs, const void* tw,
                               hipStream_t st) {
  const dim3 grid(blocks), block(kWideThreads);
  const cplx<float>* t1 = static_cast<const cplx<float>*>(tw);
  if (q != 2) return hipErrorInvalidValue;
  switch (len) {
    case 64: hipLaunchKernelGGL(k_fbw<64>, grid, block, 0, st, ga, recs, t1); break;
    case 128: hipLaunchKernelGGL(k_fbw<128>, grid, block, 0, st, ga, recs, t1); break;
    case 256: hipLaunchKernelGGL(k_fbw<256>, grid, block, 0, st, ga, recs, t1); break;
    case 512: hipLaunchKernelGGL(k_fbw<512>, grid, block, 0, st, ga, recs, t1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sbp
