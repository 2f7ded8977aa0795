// Fused three-pass schedule instantiated for double.
#include "fused.hpp"

namespace sbp {

// variants for Ny <= 256 only: 2 (pass C in 256-thread blocks over 16-byte rows) and 3 (split
// passes A and C, k_fas / k_fcs); anything else is rejected, never replaced, since the plan
// sized the grid for the variant
template <typename T, int NY, int A, int B>
static hipError_t launch_ac_narrow(int kind, int variant, bool lin, int blocks, GroupArgs ga, const BoxRec* recs,
                                   const cplx<T>* t1, const cplx<T>* t2, hipStream_t st) {
  if constexpr (NY <= 256) {
    const dim3 grid(blocks);
    if (variant == 2 && kind == 2) {
      if (lin) hipLaunchKernelGGL((k_fc<T, NY, A, B, 2, true>), grid, dim3(fa_threads<2>()), 0, st, ga, recs, t1, t2);
      else hipLaunchKernelGGL((k_fc<T, NY, A, B, 2, false>), grid, dim3(fa_threads<2>()), 0, st, ga, recs, t1, t2);
    } else if (variant == 3 && kind == 0) {
      if (lin) hipLaunchKernelGGL((k_fas<T, NY, A, B, true>), grid, dim3(kFusedAC), 0, st, ga, recs, t1, t2);
      else hipLaunchKernelGGL((k_fas<T, NY, A, B, false>), grid, dim3(kFusedAC), 0, st, ga, recs, t1, t2);
    } else if (variant == 3 && kind == 2) {
      if (lin) hipLaunchKernelGGL((k_fcs<T, NY, A, B, true>), grid, dim3(kFusedAC), 0, st, ga, recs, t1, t2);
      else hipLaunchKernelGGL((k_fcs<T, NY, A, B, false>), grid, dim3(kFusedAC), 0, st, ga, recs, t1, t2);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  } else {
    (void)kind; (void)variant; (void)lin; (void)blocks; (void)ga; (void)recs; (void)t1; (void)t2; (void)st;
    return hipErrorInvalidValue;
  }
}

// kind: 0 = pass A (len = Ny), 1 = pass B (len = M, q = padding), 2 = pass C (len = Ny);
// a = A = Nx/16.  tw: y twiddles (A, C) or z twiddles (B); tw2: x twiddles (A, C) or the
// double z twiddles (B).
template <>
hipError_t launch_fused_impl<double>(int kind, int len, int a, int variant, int q, bool lin, GroupArgs ga, int blocks,
                                 const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st) {
  using T = double;
  constexpr int B = kFusedB16;
  const dim3 grid(blocks);
  const cplx<T>* t1 = static_cast<const cplx<T>*>(tw);
  if (kind == 1) {
    (void)tw2;
#define SBP_CASE(M_)                \
    if (len == M_) {                \
      if (q == 4) hipLaunchKernelGGL((k_fb<T, M_, B, 4>), grid, dim3(fb_threads<M_, B, 4>()), 0, st, ga, recs, t1, a); \
      else hipLaunchKernelGGL((k_fb<T, M_, B, 2>), grid, dim3(fb_threads<M_, B, 2>()), 0, st, ga, recs, t1, a);       \
      return hipGetLastError();     \
    }
    SBP_CASE(32) SBP_CASE(64) SBP_CASE(128) SBP_CASE(256) SBP_CASE(512)
#undef SBP_CASE
    return hipErrorInvalidValue;
  }
  const cplx<T>* t2 = static_cast<const cplx<T>*>(tw2);
#define SBP_AC(NY_, A_)                                                      \
  if (len == NY_ && a == A_) {                                              \
    if (variant >= 2) return launch_ac_narrow<T, NY_, A_, B>(kind, variant, lin, blocks, ga, recs, t1, t2, st); \
    if (kind == 0) {                                                        \
      if (lin) hipLaunchKernelGGL((k_fa<T, NY_, A_, B, 0, true>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2); \
      else hipLaunchKernelGGL((k_fa<T, NY_, A_, B, 0, false>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2);   \
    } else {                                                                \
      if (lin) hipLaunchKernelGGL((k_fc<T, NY_, A_, B, 0, true>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2); \
      else hipLaunchKernelGGL((k_fc<T, NY_, A_, B, 0, false>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2);   \
    }                                                                       \
    return hipGetLastError();                                               \
  }
#define SBP_NY(NY_) SBP_AC(NY_, 1) SBP_AC(NY_, 2) SBP_AC(NY_, 4) SBP_AC(NY_, 8) SBP_AC(NY_, 16)
  SBP_NY(16) SBP_NY(32) SBP_NY(64) SBP_NY(128) SBP_NY(256) SBP_NY(512)
#undef SBP_NY
#undef SBP_AC
  return hipErrorInvalidValue;
}

}  // namespace sbp
