// Plan internals shared with the autotuner.
#pragma once

#include <string>
#include <vector>

#include "../../include/sbp.h"
#include "sbp_internal.hpp"

namespace sbp {

// 0-4: the five streaming passes; 5-7: the fused three-pass schedule
enum PassKind { kYFwd = 0, kXFwd = 1, kZ = 2, kXInv = 3, kYInv = 4, kFA = 5, kFB = 6, kFC = 7 };
constexpr int kKinds = 8;
// position of each kind in the solve sequence (boxes are independent, so kinds of the same phase
// may run in any order)
constexpr int kPhase[kKinds] = {0, 1, 2, 3, 4, 0, 2, 4};

// one kernel launch of the solve sequence: a group of boxes sharing a kernel shape
struct Launch {
  int kind = 0, len = 0, variant = 0, q = 0, a = 0;
  bool lin = false;  // fused passes A and C: linear remap instantiation
  int blocks = 0;
  size_t ints_off = 0;  // offset (in ints) of box_ids[n] then starts[n+1] in the group int block
  size_t blk_off = 0;   // n > 1: offset (in int2) of the per-block (box id, tile) table
  int n = 0;
  size_t tw = 0, tw64 = 0;  // table offsets
};

struct BoxInfo {
  BoxGeom g;
  int pad = 2;
  size_t tw_x = 0, tw_m = 0, tw_m64 = 0;  // offsets into the table block: plain twiddles
  size_t tws_x = 0, tws_y = 0, tws_m = 0;           // stage-major twiddles, forward then inverse
  size_t zt = 0, zt64[3] = {0, 0, 0}, k0h = 0;
  size_t ws_off = 0;   // half spectrum (plain: padded spectrum)
  size_t ws2_off = 0;  // plain: unpadded half spectrum
  size_t part_off = 0;
  int npartials = 0;    // partial-sum slots reserved (every tiling the plan may launch)
  int first_tiles = 0;  // tiles of the first pass as launched (set with the launch groups)
  size_t data_bytes = 0;
  int var[kKinds] = {1, 1, 1, 1, 1, 0, 0, 0};  // tile variant per pass kind
  int var_src[kKinds] = {0, 0, 0, 0, 0, 0, 0, 0};  // where var[k] came from: kVarSrc*
  bool fused = false;                           // three-pass schedule for this box
};

sbp_status fail(sbp_status st, const char* fmt, ...);

// origin of a box's tile variant for one pass kind
enum VarSrc { kVarDefault = 0, kVarCache = 1, kVarMeasured = 2 };
extern const char* const kVarSrcName[3];

// whether tile variant v exists for pass kind `kind` of a fused box (passes A and C only; the
// launchers reject every other combination)
bool fused_variant_ok(int prec, int kind, const BoxGeom& g, int v);
constexpr int kFusedVariants = 4;

// built-in variant choice (measured on MI355X) for a box
void default_variants(int prec, const BoxGeom& g, int var[kKinds]);
// time the variants of every pass and keep the fastest per (pass, length); cached on disk
sbp_status autotune(sbp_plan p);

// plan access for the autotuner
int plan_prec(sbp_plan p);
int plan_device(sbp_plan p);
std::vector<BoxInfo>& plan_boxes(sbp_plan p);
void plan_set_tune_source(sbp_plan p, const std::string& s);
// while the autotuner times the fused passes, every (Ny, A) keeps its own launch group (float
// plans otherwise merge groups that differ only in A <= 8 into one launch)
void plan_set_nomix(sbp_plan p, bool on);
// index of the first box of a launch group
int plan_group_box(sbp_plan p, const Launch& l);
sbp_status plan_time_groups(sbp_plan p, int reps, std::vector<Launch>& launches, std::vector<double>& ms);

}  // namespace sbp
