// Fused passes A and C for float, Ny in {96, 128}.
#include "fused_launch.hpp"

namespace sbp {
template hipError_t launch_ac_ny<float, 96>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<float>*,
                                              const cplx<float>*, hipStream_t);
template hipError_t launch_ac_ny<float, 128>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<float>*,
                                              const cplx<float>*, hipStream_t);
}  // namespace sbp
