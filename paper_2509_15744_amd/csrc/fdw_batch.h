// Launchers of the multi-problem step kernels (fdw_batch.hip): several problems per
// launch, and whole sweeps in one persistent launch.
#pragma once

#include "fdw_internal.h"

namespace fdw {

// One step of several problems in one launch: table[p] holds problem p's
// arguments, block_start[p] its first block (block_start[nprob] = total).
hipError_t launch_step_multi(int ndim, int r, int dtype, int acc_dtype, int variant,
                             const StepArgs* d_table, const int32_t* d_block_start, int nprob,
                             int total_blocks, hipStream_t s);

// Group plans of a persistent launch.  A group is a column of chunks of one tile
// column; plan j groups cand_k[j] consecutive chunks (ncand plans, cand_k ascending, so
// the groups fall with j), group_start[j * (nprob + 1) + p] being the first group of
// problem p under plan j.  groups0, the groups of plan 0, sizes the grid and the
// progress words.  The kernel takes the first plan whose groups do not outnumber the
// blocks that run (the last plan if none fits).
struct GroupPlans {
    const int32_t* cand_k;
    const int32_t* group_start;
    int ncand;
    int groups0;
};

// `nsteps` consecutive steps (table rows of nprob entries each) of several problems in
// one launch whose running blocks each own a fixed set of groups.  A group starts a step
// once its neighbouring groups have finished the previous one.  d_progress:
// kProgressWords words (word 2 the error flag; words 4-6 the arrival count, the number
// of blocks taking part and the number of them ranked; words 8-15 the blocks taking
// part on each XCD; all zeroed), then one zeroed word per group of plan 0; a wait
// longer than timeout_ticks (device wall clock) sets the error flag and ends the launch
// early.  *grid_used receives the number of blocks launched.
constexpr int kProgressWords = 64;
hipError_t launch_step_persistent(int ndim, int r, int dtype, int acc_dtype, int variant, const StepArgs* d_table,
                                  const GroupPlans& gp, int nprob, int nsteps, unsigned* d_progress,
                                  long long timeout_ticks, hipStream_t s, int* grid_used);

// Blocks of the persistent step kernel of this shape that the device holds at once by
// the occupancy calculator (registers, LDS, waves per CU) times the CUs: the grid of
// its launches.
hipError_t persistent_capacity(int ndim, int r, int dtype, int acc_dtype, int variant, int* blocks);

}  // namespace fdw
