// y passes (forward and inverse) instantiated for float.
#include "passes.hpp"

namespace sbp {

template <>
hipError_t launch_y_impl<float>(bool forward, bool remap, int ny, int variant, GroupArgs ga, int blocks,
                             const BoxRec* recs, const void* tw, hipStream_t st) {
  using T = float;
  const dim3 grid(blocks);
  const cplx<T>* t = static_cast<const cplx<T>*>(tw);
#define SBP_LAUNCH(N_, V_)                                                                           \
  if (forward && remap) hipLaunchKernelGGL((k_yfwd<T, N_, V_, true>), grid, dim3(xy_threads<N_>()), 0, st, ga, recs, t);  \
  else if (forward) hipLaunchKernelGGL((k_yfwd<T, N_, V_, false>), grid, dim3(xy_threads<N_>()), 0, st, ga, recs, t);     \
  else if (remap) hipLaunchKernelGGL((k_yinv<T, N_, V_, true>), grid, dim3(xy_threads<N_>()), 0, st, ga, recs, t);        \
  else hipLaunchKernelGGL((k_yinv<T, N_, V_, false>), grid, dim3(xy_threads<N_>()), 0, st, ga, recs, t);
#define SBP_CASE(N_)                  \
  if (ny == N_) {                     \
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
