// Interface of the two-step launches (fdw_pair.hip) for the fdwave host runtime.
#pragma once

#include "fdw_internal.h"

namespace fdw {

// Arguments of one two-step launch: levels n+1 and n+2 from n-1 and n.  s describes the
// first step as for a one-step launch (s.unew holds u^{n-1} and is only read; s.row_src /
// s.row_rec are the first step's rows; s.blk_off / grp / ev the tile events of the
// 64 x 8 one-cell-per-lane tiles); the second step's rows follow, the two output arrays,
// the kernel terms of the launch (0, 1: the interval n, n+1 alone, 3: both intervals,
// with s.acc_sign, s.part and s.part_mode) and the events of the blocks' rings of level
// n+1 (planes x0 - R .. x1 + R - 1 of each chunk).
struct PairArgs {
    StepArgs s;
    void* out1;              // u^{n+1}
    void* out2;              // u^{n+2}
    int32_t row_src2, row_rec2;
    int32_t terms;
    const int32_t* blk_off_a;
    const EvPlane* grp_a;
    const Event* ev_a;
};

// Tile of the two-step launches: 64 x 8 cells, one per lane (the shape of step variant 1).
constexpr int kPairTZ = 64, kPairTY = 8;

// Two steps of one problem (one shot, 3D, orders 2/4/8) in one launch; see PairArgs.
hipError_t launch_pair(int r, int dtype, int acc_dtype, int nblk, const PairArgs& p, hipStream_t s);

}  // namespace fdw
