// Device-resident tables shared by the step kernel and the host side: one Member per grid of a
// batch, the per-step Control of the scheduler, and the kernel arguments.
#pragma once
#include <stdint.h>

#include "bn2d_physics.h"

namespace bn {

// One grid of the batch.  Lives in device memory and is read through the scalar cache.
struct Member {
    Consts K;                       // grid and model constants
    double *q[2];                   // state buffers; q[cur] holds the current state
    const uint8_t *solid;           // nx*ny mask or null
    const int *jb;                  // first fluid row of each column
    const double *dbot;             // per column: bottom height minus the top of its solid run, or null
    long long *S[3];                // fixed-point free-surface integrals (read m3, accumulate m3+1, clear m3+2)
    unsigned long long *lam[3];     // CFL rate maxima (same rotation), bits of a non-negative double
    double *t;                      // elapsed time
    int *flag;                      // 1: non-physical state, 2: no CFL rate, 4: scheduler error
    double fix_scale, fix_inv;      // fixed-point scale 2^f and 2^-f
    int nstrips;                    // column strips of this grid
    int strip0;                     // global index of its first strip
    long long cost0;                // offset of its first row in the cost arrays
};

// One column strip of the batch: its grid, its index within that grid, the grid's height and the
// offset of its first row in the per-row cost arrays.
struct StripInfo {
    int member;
    int local;
    int ny;
    int pad;
    long long cost_base;
};

// Scheduling state of the whole batch for one combination of the rotations (range lists and
// row costs: slot p mod 2; strip cost totals: m mod 3).
struct Control {
    unsigned long long *desc;       // range descriptors of this step
    int *nranges;                   // published descriptors of this step
    unsigned long long *desc_next;  // range descriptors of the next step (cleared here)
    int *nranges_next;
    const float *cost_in;           // recorded march cost per row (previous step), member by member
    float *cost_out;                // ... recorded by this step
    const double *Ts_in;            // recorded cost per global strip (previous step)
    double *Ts_out;                 // ... accumulated by this step
    double *Ts_clear;               // third buffer, zeroed for the next step
    const StripInfo *strips;        // every global strip
    int *flag;                      // batch-wide scheduler error (4)
    int *unowned;                   // ranges published unowned and not taken yet (0 between steps)
    int nstrips;                    // global strips
    int nmembers;
    int R0;                         // initial descriptors: one per wavefront, one head per strip
    int max_slots;                  // descriptor capacity (initial descriptors and splits)
    int P;                          // wavefronts of the launch
};

struct StepArgs {
    unsigned long long maddr;       // device address of the Member array
    unsigned long long caddr;       // device address of the Control of this step
    double dt_arg;                  // dt of every member (explicit mode)
    int cfl_dt;                     // 1: each member's dt = CFL / its max rate, else dt_arg
    int cur;                        // current state buffer
    int m3;                         // rotation of the 3-way buffers
    int B;                          // rows per claim
    double cost_floor;              // least recorded row cost, as a fraction of its strip's mean
                                    // row cost in the previous step (0: none)
};

// The cost floor where the wavefronts' shares average at least kCostFloorRows rows (rows measured
// cheap still count for most of a typical row, so that no share packs many more rows than its
// strip's average; 0.90 changes nothing on the 2048 x 1024 dam break, 0.95 and above slow the 4096^2
// drop and the ensemble, whose gas rows stay cheap; with a few rows a share, as on a 512 x 256 grid,
// any floor slows the step).
constexpr double kCostFloor = 0.92;
constexpr int kCostFloorRows = 8;

}  // namespace bn
