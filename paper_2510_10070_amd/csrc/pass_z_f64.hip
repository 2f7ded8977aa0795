// z passes (pad, transform, Green multiply, inverse, extract) instantiated for double.
#include "passes.hpp"

namespace sbp {

template <>
hipError_t launch_z_impl<double>(int m, int variant, int q, GroupArgs ga, int blocks, const BoxRec* recs,
                             const void* tw, const void* tw64, hipStream_t st) {
  using T = double;
  const dim3 grid(blocks), block(kPassThreads);
  const cplx<T>* t = static_cast<const cplx<T>*>(tw);
  const double2* t64 = static_cast<const double2*>(tw64);
#define SBP_LAUNCH(N_, V_)                                                                        \
  if (q == 4) hipLaunchKernelGGL((k_z<T, N_, V_, 4>), grid, block, 0, st, ga, recs, t, t64);      \
  else hipLaunchKernelGGL((k_z<T, N_, V_, 2>), grid, block, 0, st, ga, recs, t, t64);
#define SBP_CASE(N_)                  \
  if (m == N_) {                      \
    if (variant) { SBP_LAUNCH(N_, 1) } \
    else { SBP_LAUNCH(N_, 0) }        \
    return hipGetLastError();         \
  }
  SBP_FOR_EACH_LEN(SBP_CASE)
#undef SBP_CASE
#undef SBP_LAUNCH
  return hipErrorInvalidValue;
}


}  // namespace sbp
