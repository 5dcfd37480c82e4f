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

// `nsteps` consecutive steps (table rows of nprob entries each) of several problems in
// one launch whose running blocks each own a fixed set of groups: a group is a column
// of chunks_per_group consecutive chunks of one tile column, group_start[p] the first
// group of problem p (group_start[nprob] = total_groups).  A group starts a step once
// its neighbouring groups have finished the previous one.  d_progress: kProgressWords
// words (word 2 the error flag, words 4-5 the arrival count and the number of blocks
// taking part, all zeroed), then one zeroed word per group; a wait longer than
// timeout_ticks (device wall clock) sets the error flag and ends the launch early.
// *grid_used receives the number of blocks launched.
constexpr int kProgressWords = 64;
hipError_t launch_step_persistent(int ndim, int r, int dtype, int acc_dtype, int variant,
                                  const StepArgs* d_table, const int32_t* d_group_start, int nprob,
                                  int total_groups, int nsteps, int chunks_per_group, unsigned* d_progress,
                                  long long timeout_ticks, hipStream_t s, int* grid_used);

// Blocks of the persistent step kernel of this shape that the device holds at once by
// the occupancy calculator (registers, LDS, waves per CU) times the CUs: the grid of
// its launches.
hipError_t persistent_capacity(int ndim, int r, int dtype, int acc_dtype, int variant, int* blocks);

}  // namespace fdw
