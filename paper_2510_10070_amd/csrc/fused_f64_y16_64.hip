// Fused passes A and C for double, Ny in {16, 32, 64}.
#include "fused_launch.hpp"

namespace sbp {
template hipError_t launch_ac_ny<double, 16>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<double>*,
                                              const cplx<double>*, hipStream_t);
template hipError_t launch_ac_ny<double, 32>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<double>*,
                                              const cplx<double>*, hipStream_t);
template hipError_t launch_ac_ny<double, 64>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<double>*,
                                              const cplx<double>*, hipStream_t);
}  // namespace sbp
