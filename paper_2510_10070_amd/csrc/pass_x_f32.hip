// x passes (forward and inverse) instantiated for float.
#include "passes.hpp"

namespace sbp {

template <>
hipError_t launch_x_impl<float>(int dir, int nx, int variant, GroupArgs ga, int blocks, const BoxRec* recs,
                             const void* tw, hipStream_t st) {
  using T = float;
  const dim3 grid(blocks);
  const cplx<T>* t = static_cast<const cplx<T>*>(tw);
#define SBP_LAUNCH(N_, V_)                                                                     \
  if (dir < 0) hipLaunchKernelGGL((k_x<T, N_, V_, -1>), grid, dim3(x_threads<T, N_, V_>()), 0, st, ga, recs, t);      \
  else hipLaunchKernelGGL((k_x<T, N_, V_, +1>), grid, dim3(x_threads<T, N_, V_>()), 0, st, ga, recs, t);
#define SBP_CASE(N_)                  \
  if (nx == N_) {                     \
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
