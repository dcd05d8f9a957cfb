// Kernel argument blocks and launch helpers shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/xpic.h"
#include "xp_tables.h"

namespace xpd {

struct StepArgs {
    const xp_run* runs;
    const int32_t* cell_run;
    const int64_t* e_off;
    const int32_t* e_cap;
    int32_t* e_cnt;
    const int64_t* i_off;
    const int32_t* i_cnt;
    double *ex, *ey, *evx, *evy, *evz;
    uint32_t* ew;
    const double *ix, *iy;
    double *ivx, *ivy, *ivz;
    uint8_t *iz, *ik;
    const double* cell_nhv;
    uint64_t* run_cnt;
    double* run_led;
    int64_t* cell_cnt;
    double* cell_led;
    double* cell_mom;
    uint32_t* status;
    const DevTables* tab;
    const uint32_t* d_step;
    uint32_t step;
    uint32_t flags;
    const int32_t* cell_list;   // optional: cells to process (count in *cell_list_count)
    const int32_t* cell_list_count;
    int32_t* defer_out;         // cells that outgrow this launch's LDS plan
    int32_t* defer_out_count;
    int32_t* stats;             // [0] max electrons per cell after the step, [1] deferrals
    int32_t n_cells;
    int32_t lds_ce, lds_ci;     // LDS capacity per cell (electrons, ions)
};

__global__ void k_step_prep(int32_t* counts, int32_t* stats);

size_t step_lds_bytes(int ce, int ci);

template <int B>
__global__ void k_step(StepArgs a);

}  // namespace xpd

namespace xpd {

// Workspace layout of bin_particles (byte offsets into xp_batch.d_work).
struct BinPlan {
    size_t key_a, val_a, key_b, val_b, hist, scan_aux, cnt_e, cnt_i, start_e, start_i, flags;
    size_t bytes;
};

BinPlan bin_plan(int64_t ne, int64_t ni, int32_t n_cells);
hipError_t bin_launch(const xp_particles* in, xp_batch* b, const xp_capacity* cap,
                      int64_t* d_need, hipStream_t s);

}  // namespace xpd

namespace xpd {

struct DiagArgs {
    const xp_run* runs;
    const int32_t* cell_run;
    const int64_t* e_off;
    const int32_t* e_cnt;
    const int64_t* i_off;
    const int32_t* i_cnt;
    const double *evx, *evy, *evz;
    const uint32_t* ew;
    const uint8_t* iz;
    uint64_t* run_cnt;
    double* run_led;
    double* cell_k;      // workspace [n_cells]
    xp_diag* out;
    int32_t n_runs, n_cells;
};

hipError_t diag_launch(const DiagArgs& a, uint32_t what, hipStream_t s);

}  // namespace xpd

namespace xpd {
hipError_t selftest_launch(int which, int64_t n, const double* x, const uint64_t* u, double* out,
                           uint32_t* words, hipStream_t s);
}  // namespace xpd
