// Fused passes A (kind 0) and C (kind 2) of the wide float schedule: Ny in {512, 1024}, A = Nx/64
// in {8, 16}.
#include "fused_wide.hpp"

namespace sbp {

namespace {
template <int NY, int A>
hipError_t launch_ac(int kind, bool lin, GroupArgs ga, int blocks, const BoxRec* recs, const cplx<float>* t1,
                     const cplx<float>* t2, hipStream_t st) {
  const dim3 grid(blocks), block(kWideThreads);
  if (kind == 0) {
    if (lin) hipLaunchKernelGGL((k_faw<NY, A, true>), grid, block, 0, st, ga, recs, t1, t2);
    else hipLaunchKernelGGL((k_faw<NY, A, false>), grid, block, 0, st, ga, recs, t1, t2);
  } else {
    if (lin) hipLaunchKernelGGL((k_fcw<NY, A, true>), grid, block, 0, st, ga, recs, t1, t2);
    else hipLaunchKernelGGL((k_fcw<NY, A, false>), grid, block, 0, st, ga, recs, t1, t2);
  }
  return hipGetLastError();
}
}  // namespace

// len = Ny; tw: the stage-major y twiddles, tw2: the x twiddles w_Nx^m
hipError_t launch_fused_wide_ac(int kind, int len, int a, bool lin, GroupArgs ga, int blocks, const BoxRec* recs,
                                const void* tw, const void* tw2, hipStream_t st) {
  const cplx<float>* t1 = static_cast<const cplx<float>*>(tw);
  const cplx<float>* t2 = static_cast<const cplx<float>*>(tw2);
  if (kind != 0 && kind != 2) return hipErrorInvalidValue;
  if (len == 512 && a == 8) return launch_ac<512, 8>(kind, lin, ga, blocks, recs, t1, t2, st);
  if (len == 512 && a == 16) return launch_ac<512, 16>(kind, lin, ga, blocks, recs, t1, t2, st);
  if (len == 1024 && a == 8) return launch_ac<1024, 8>(kind, lin, ga, blocks, recs, t1, t2, st);
  if (len == 1024 && a == 16) return launch_ac<1024, 16>(kind, lin, ga, blocks, recs, t1, t2, st);
  return hipErrorInvalidValue;
}

}  // namespace sbp
