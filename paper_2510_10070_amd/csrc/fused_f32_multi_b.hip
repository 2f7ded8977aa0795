// Fused pass B for float launch groups that mix M <= 256 (padding 2).
#include "fused_launch.hpp"

namespace sbp {
template hipError_t launch_fb_multi<float>(GroupArgs, int, const BoxRec*, hipStream_t);
}  // namespace sbp
