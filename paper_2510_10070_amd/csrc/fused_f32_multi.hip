// Fused passes A and C for float launch groups that mix Ny <= 128 (and A <= 8).
#include "fused_launch.hpp"

namespace sbp {
template hipError_t launch_ac_multi<float>(int, bool, GroupArgs, int, const BoxRec*, hipStream_t);
}  // namespace sbp
