// Host interface of the wide fused schedule: FP32 boxes with Nx and Ny in {512, 1024}, padding 2
// and M in {64, 128, 256, 512}, split four-step as Nx = A * 64 (B = 64 pencils per pass-B item).
// Plans take it on request only (SBP_FLAG_FUSED); its launches carry the tile variant
// kWideVariant in all three passes.
#pragma once

#include "sbp_internal.hpp"

namespace sbp {

constexpr int kWideVariant = 4;

bool fused_wide_ok(int prec, const BoxGeom& g);
// kind 0 pass A, 2 pass C (len = Ny, a = Nx/64; tw: stage-major y twiddles, tw2: x twiddles)
hipError_t launch_fused_wide_ac(int kind, int len, int a, bool lin, GroupArgs ga, int blocks, const BoxRec* recs,
                                const void* tw, const void* tw2, hipStream_t st);
// pass B (len = M, q = padding; tw: stage-major z twiddles)
hipError_t launch_fused_wide_b(int len, int q, GroupArgs ga, int blocks, const BoxRec* recs, const void* tw,
                               hipStream_t st);

}  // namespace sbp
