// Launch helpers of the fused schedule, shared by the translation units that instantiate it:
// fused_{f32,f64}.hip hold pass B and the dispatch; fused_{f32,f64}_y*.hip instantiate passes A
// and C for subsets of Ny (so that the build compiles them in parallel).
#pragma once

#include "fused.hpp"

namespace sbp {

// variants for Ny <= 256 only: 2 (pass C in 256-thread blocks over 16-byte rows) and 3 (split
// passes A and C, k_fas / k_fcs); anything else is rejected, never replaced, since the plan
// sized the grid for the variant
template <typename T, int NY, int A, int B>
hipError_t launch_ac_narrow(int kind, int variant, bool lin, int blocks, GroupArgs ga, const BoxRec* recs,
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

// passes A (kind 0) and C (kind 2) for one Ny, A = Nx/16 in {1, 2, 4, 6, 8, 16}, or a = 0 for a
// group whose boxes have different A <= 8; tile variant 1 (64-byte rows) only for float, A <= 8
// and Ny <= 256
template <typename T, int NY>
hipError_t launch_ac_ny(int kind, int a, int variant, bool lin, GroupArgs ga, int blocks, const BoxRec* recs,
                        const cplx<T>* t1, const cplx<T>* t2, hipStream_t st) {
  constexpr int B = kFusedB16;
  const dim3 grid(blocks);
  if (a == 0) {
    // a group that mixes Nx (A <= 8): each block takes its box's A and x twiddles from the record
    if (variant != 1 || sizeof(T) != 4 || NY > 256) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4 && NY <= 256) {
    if (kind == 0) {
      if (lin) hipLaunchKernelGGL((k_fa_mix<T, NY, B, 1, true>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2);
      else hipLaunchKernelGGL((k_fa_mix<T, NY, B, 1, false>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2);
    } else {
      if (lin) hipLaunchKernelGGL((k_fc_mix<T, NY, B, 1, true>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2);
      else hipLaunchKernelGGL((k_fc_mix<T, NY, B, 1, false>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2);
    }
    }
    return hipGetLastError();
  }
#define SBP_AC(A_)                                                                                                \
  if (a == A_) {                                                                                                  \
    if (variant >= 2) return launch_ac_narrow<T, NY, A_, B>(kind, variant, lin, blocks, ga, recs, t1, t2, st);  \
    if (variant == 1) {                                                                                           \
      if constexpr (sizeof(T) == 4 && A_ <= 8 && NY <= 256) {                                                     \
        if (kind == 0) {                                                                                          \
          if (lin) hipLaunchKernelGGL((k_fa<T, NY, A_, B, 1, true>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2); \
          else hipLaunchKernelGGL((k_fa<T, NY, A_, B, 1, false>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2);   \
        } else {                                                                                                  \
          if (lin) hipLaunchKernelGGL((k_fc<T, NY, A_, B, 1, true>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2); \
          else hipLaunchKernelGGL((k_fc<T, NY, A_, B, 1, false>), grid, dim3(fa_threads<1>()), 0, st, ga, recs, t1, t2);   \
        }                                                                                                         \
        return hipGetLastError();                                                                                 \
      }                                                                                                           \
      return hipErrorInvalidValue; /* the grid was sized for that variant's tiles */                              \
    }                                                                                                             \
    if (kind == 0) {                                                                                              \
      if (lin) hipLaunchKernelGGL((k_fa<T, NY, A_, B, 0, true>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2); \
      else hipLaunchKernelGGL((k_fa<T, NY, A_, B, 0, false>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2);   \
    } else {                                                                                                      \
      if (lin) hipLaunchKernelGGL((k_fc<T, NY, A_, B, 0, true>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2); \
      else hipLaunchKernelGGL((k_fc<T, NY, A_, B, 0, false>), grid, dim3(fa_threads<0>()), 0, st, ga, recs, t1, t2);   \
    }                                                                                                             \
    return hipGetLastError();                                                                                     \
  }
  SBP_AC(1) SBP_AC(2) SBP_AC(4) SBP_AC(6) SBP_AC(8) SBP_AC(16)
#undef SBP_AC
  return hipErrorInvalidValue;
}

#define SBP_FUSED_NY(X) X(16) X(32) X(64) X(96) X(128) X(256) X(512)
#define SBP_EXTERN_AC(T_, NY_)                                                                                      \
  extern template hipError_t launch_ac_ny<T_, NY_>(int, int, int, bool, GroupArgs, int, const BoxRec*, const cplx<T_>*, \
                                                   const cplx<T_>*, hipStream_t);
#define SBP_EXTERN_AC_F(NY_) SBP_EXTERN_AC(float, NY_)
#define SBP_EXTERN_AC_D(NY_) SBP_EXTERN_AC(double, NY_)
SBP_FUSED_NY(SBP_EXTERN_AC_F)
SBP_FUSED_NY(SBP_EXTERN_AC_D)
#undef SBP_EXTERN_AC_F
#undef SBP_EXTERN_AC_D

// passes A (kind 0) and C (kind 2) for a group that mixes Ny <= 128 and A <= 8 (float, variant 1
// boxes, run in 64- or 128-byte rows by Ny; instantiated in fused_f32_multi.hip)
template <typename T>
hipError_t launch_ac_multi(int kind, bool lin, GroupArgs ga, int blocks, const BoxRec* recs, hipStream_t st);
extern template hipError_t launch_ac_multi<float>(int, bool, GroupArgs, int, const BoxRec*, hipStream_t);

template <typename T>
hipError_t launch_ac_multi(int kind, bool lin, GroupArgs ga, int blocks, const BoxRec* recs, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    constexpr int B = kFusedB16;
    const dim3 grid(blocks), block(fa_threads<1>());
    const cplx<T>* none = nullptr;
    if (kind == 0) {
      if (lin) hipLaunchKernelGGL((k_fa_multi<T, B, true>), grid, block, 0, st, ga, recs, none, none);
      else hipLaunchKernelGGL((k_fa_multi<T, B, false>), grid, block, 0, st, ga, recs, none, none);
    } else {
      if (lin) hipLaunchKernelGGL((k_fc_multi<T, B, true>), grid, block, 0, st, ga, recs, none, none);
      else hipLaunchKernelGGL((k_fc_multi<T, B, false>), grid, block, 0, st, ga, recs, none, none);
    }
    return hipGetLastError();
  } else {
    (void)kind; (void)lin; (void)ga; (void)blocks; (void)recs; (void)st;
    return hipErrorInvalidValue;
  }
}

// pass B for a group that mixes M <= 256 (float, padding 2; instantiated in fused_f32_multi.hip)
template <typename T> hipError_t launch_fb_multi(GroupArgs ga, int blocks, const BoxRec* recs, hipStream_t st);
extern template hipError_t launch_fb_multi<float>(GroupArgs, int, const BoxRec*, hipStream_t);

template <typename T> hipError_t launch_fb_multi(GroupArgs ga, int blocks, const BoxRec* recs, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    hipLaunchKernelGGL((k_fb_multi<T, kFusedB16, 2>), dim3(blocks), dim3(256), 0, st, ga, recs);
    return hipGetLastError();
  } else {
    (void)ga; (void)blocks; (void)recs; (void)st;
    return hipErrorInvalidValue;
  }
}

// the launcher of one precision: pass B here, passes A and C in their own translation units
template <typename T>
hipError_t launch_fused_dispatch(int kind, int len, int a, int q, int variant, bool lin, GroupArgs ga, int blocks,
                                 const BoxRec* recs, const void* tw, const void* tw2, hipStream_t st) {
  constexpr int B = kFusedB16;
  const dim3 grid(blocks);
  const cplx<T>* t1 = static_cast<const cplx<T>*>(tw);
  if (kind == 1) {
    if (len == 0) return launch_fb_multi<T>(ga, blocks, recs, st);
#define SBP_CASE(M_)                                                                                                 \
    if (len == M_) {                                                                                                 \
      if (q == 4) hipLaunchKernelGGL((k_fb<T, M_, B, 4>), grid, dim3(fb_threads<M_, B, 4>()), 0, st, ga, recs, t1); \
      else hipLaunchKernelGGL((k_fb<T, M_, B, 2>), grid, dim3(fb_threads<M_, B, 2>()), 0, st, ga, recs, t1);       \
      return hipGetLastError();                                                                                      \
    }
    SBP_CASE(32) SBP_CASE(64) SBP_CASE(128) SBP_CASE(192) SBP_CASE(256) SBP_CASE(512)
#undef SBP_CASE
    return hipErrorInvalidValue;
  }
  const cplx<T>* t2 = static_cast<const cplx<T>*>(tw2);
  if (len == 0) {
    // a group mixing Ny: float 64-byte rows only, every block takes its box's twiddles
    if (sizeof(T) != 4 || variant != 1 || a != 0) return hipErrorInvalidValue;
    return launch_ac_multi<T>(kind, lin, ga, blocks, recs, st);
  }
#define SBP_CASE(NY_) \
  if (len == NY_) return launch_ac_ny<T, NY_>(kind, a, variant, lin, ga, blocks, recs, t1, t2, st);
  SBP_FUSED_NY(SBP_CASE)
#undef SBP_CASE
  return hipErrorInvalidValue;
}

}  // namespace sbp
