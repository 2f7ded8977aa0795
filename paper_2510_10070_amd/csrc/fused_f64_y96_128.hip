// Fused passes A and C for double, Ny in {96, 128}.
#include "fused_launch.hpp"

namespace sbp {
template hipError_t launch_ac_ny<double, 96>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<double>*,
                                              const cplx<double>*, hipStream_t);
template hipError_t launch_ac_ny<double, 128>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<double>*,
                                              const cplx<double>*, hipStream_t);
}  // namespace sbp
