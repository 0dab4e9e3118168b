// dk_round.h -- launch interface of the persistent round kernel.
#pragma once
#include "dk_internal.h"

namespace dk {

// Persistent round kernel: all resident levels of one Algorithm-1 round in one launch.
struct RoundLevel {
    LevelArgs A;            // the level's tables and coefficients (first, count, out unused)
    int kind;               // round_kind(nf, pair)
    int spw;                // samples per block-iteration, round_spw_of(nf)
};
struct RoundTask {
    uint32_t level;         // index into RoundArgs::levels
    uint32_t pad;
    uint64_t first;         // first sample index (absolute) of the task
    uint64_t count;         // samples of the task
};
struct RoundArgs {
    const RoundLevel* levels;   // device
    const RoundTask* tasks;     // device, in the order they are handed out
    const uint32_t* ntasks;     // device scalar
    uint32_t* head;             // device queue counter (reset by the launch)
    double* task_mom;           // device [ntasks][n_obs][DK_NMOM][2] (sum, compensation)
    double* scratch;            // device [grid][scratch_stride] per-sample values of a block-iteration
    uint64_t scratch_stride;    // doubles per block, >= 256 * n_obs * 2
    int n_obs;
};
int round_kind(int nf, bool pair);
int round_spw_of(int nf);
int round_blocks_per_cu(int flux);
int round_max_obs();
// Resets the queue counter, then launches `grid` blocks of the round kernel.
hipError_t launch_round(const RoundArgs& P, int flux, int grid, hipStream_t s);

}  // namespace dk
