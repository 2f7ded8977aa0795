// Fused passes A and C for float, Ny in {16, 32, 64}.
#include "fused_launch.hpp"

namespace sbp {
template hipError_t launch_ac_ny<float, 16>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<float>*,
                                              const cplx<float>*, hipStream_t);
template hipError_t launch_ac_ny<float, 32>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<float>*,
                                              const cplx<float>*, hipStream_t);
template hipError_t launch_ac_ny<float, 64>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<float>*,
                                              const cplx<float>*, hipStream_t);
}  // namespace sbp
