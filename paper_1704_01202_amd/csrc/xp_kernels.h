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
    int32_t* cell_nabs;         // optional [n_cells][XP_MAX_BINS] photon events per bin
    double* cell_nka;           // optional [n_cells][XP_MAX_BINS] K-alpha macro-photons returned
    uint32_t* status;
    uint32_t* run_status;       // optional [n_runs]
    const DevTables* tab;
    const double* run_sig;      // [n_runs][XP_MAX_BINS][3] photo cross sections (k_run_prep)
    const uint32_t* d_step;
    uint32_t step;
    uint32_t flags;
    const int32_t* cell_list;   // optional: cells to process (count in *cell_list_count)
    const int32_t* cell_list_count;
    int32_t* defer_out;         // cells that outgrow this launch's LDS plan
    int32_t* defer_out_count;
    int32_t* big_out;           // cells beyond every LDS plan (global-memory path)
    int32_t* big_out_count;
    int32_t big_out_cap;
    int32_t* stats;             // [0] max electrons per cell after the step, [1] deferrals
    int32_t n_cells;
    int32_t lds_ce, lds_ci;     // LDS capacity per cell (electrons, ions)
};

// Deferral counters of the tiered LDS launches: one per tier, the last one
// counts the cells handed to the global-memory path.
constexpr int STEP_COUNTS = 16;
constexpr int BIG_COUNT_SLOT = STEP_COUNTS - 1;

// Sets status bits for the batch and, when the batch keeps them, for the run.
__device__ __forceinline__ void flag_status(const StepArgs& a, int run, uint32_t bits)
{
    atomicOr(a.status, bits);
    if (a.run_status && run >= 0) atomicOr(&a.run_status[run], bits);
}

__global__ void k_step_prep(int32_t* counts, int32_t* stats);
__global__ void k_run_prep(const xp_run* runs, int n_runs, const DevTables* tb, double* run_sig);

size_t step_lds_bytes(int ce, int ci);
// Largest LDS plan: ions per cell (i_lds) and the electrons that fit beside
// them (e_lds) within the dynamic LDS budget of one workgroup.
void lds_limits(size_t max_lds, int* e_lds, int* i_lds);
size_t lds_budget(size_t max_lds);

// XV: 0 the plain step; 1 compiled with the method's variants (XP_THERM,
// XP_ION_Z, XP_REC_XS, XP_PHOTO_FRAC, XP_KA_FIELD), the per-cell records and
// per-cell photon fields; 2 as 1 plus Nanbu's scattering law (XP_NANBU); 3 as
// 2 plus relativistic collisions (XP_REL).  Each level leaves out the code of
// the next, which keeps its registers for the path it runs.
template <int B, int XV>
__global__ void k_step(StepArgs a);
// 64 / W cells per wave, W lanes per cell (W = 32, 16, 8); plans with at most
// 4 W electrons and 4 W ions.
template <int W, int XV>
__global__ void k_step_g(StepArgs a);

}  // namespace xpd

namespace xpd {

// Workspace layout of bin_particles (byte offsets into xp_batch.d_work).
struct BinPlan {
    size_t key_a, val_a, key_b, val_b, hist, scan_aux, cnt_e, cnt_i, start_e, start_i, flags;
    size_t bytes;
};

BinPlan bin_plan(int64_t ne, int64_t ni, int32_t n_cells);
hipError_t bin_launch(const xp_particles* in, xp_batch* b, const xp_capacity* cap,
                      int64_t* d_need, int32_t e_lds, int32_t i_lds, hipStream_t s);

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
    int32_t e_cap_max;
};

// Kinetic-energy sums of one cell are taken in aligned chunks of DIAG_CHUNK
// electrons (canonical pairwise sums of the chunk sums).
constexpr int DIAG_CHUNK = 8192;
constexpr int DIAG_MAX_CHUNKS = 4096;

hipError_t diag_launch(const DiagArgs& a, uint32_t what, hipStream_t s);

// Reduced radiation transport (transport_photons).
struct TransportArgs {
    const xp_run* runs;
    const int32_t* cell_run;
    double* nhv;            // [n_cells][XP_MAX_BINS], rewritten
    const int32_t* nabs;    // [n_cells][XP_MAX_BINS], photon events of the last step
    const double* nka;      // optional [n_cells][XP_MAX_BINS], K-alpha macro-photons returned
    double* exit;           // workspace [n_cells][XP_MAX_BINS]: exit density at each row start
    double* trans;          // optional [n_runs][XP_MAX_BINS]
    uint32_t* status;
    uint32_t* run_status;   // optional [n_runs]
    int32_t n_runs, n_cells;
};
hipError_t transport_launch(const TransportArgs& a, hipStream_t s);

}  // namespace xpd

namespace xpd {
hipError_t selftest_launch(int which, int64_t n, const double* x, const uint64_t* u, double* out,
                           uint32_t* words, hipStream_t s);
}  // namespace xpd

namespace xpd {

// ---- global-memory path for cells beyond one workgroup's LDS -------------

constexpr int BIG_CH = 1024;          // particle slots per chunk (a power of two)
constexpr int BIG_MAX_CHUNKS = 32768; // chunks per cell and species (33.5 M slots)

// Per-cell state of one step on the global-memory path.
struct BigRec {
    int32_t cell, run;
    int32_t ne0, ne, ni, ecap;
    int32_t ce0, nce, ci0, nci;        // chunk ranges of the current plan
    int64_t eo, io;                    // slab offsets
    int64_t ep0, ip0;                  // offsets in the population arrays
    int32_t state;                     // 0 live, 1 stopped (capacity or size)
    int32_t need;                      // BN_* bits
    int32_t zc, acc, nrec, epn;        // epn: electrons covered by the current chunk plan
    int32_t nnew5, nkeep;              // electrons appended by the source terms; survivors of S4
    int32_t seld, nsub;                // S4 ranks: top-8-bit digit bound, candidates at or below it
    unsigned long long we, wb, sz, sz2, ws, nelig, nfired, we4, wb4, sz4;
    double p, kth, debit, alpha;
    double u[3];
    uint32_t zmask, zeval;             // charge states held by ions (< 13); evaluated in S3
    uint32_t zmask4, pad1;             // charge states held by ions before S4 (XP_REC_XS)
    double prz[14];                    // S4 recombination probability per charge state (XP_REC_XS)
    double ppz[13][5], lnpz[13][5];    // S3 lowered bindings and their logarithms per state
    double pz[13];                     // S3 probability per evaluated state
    double mom[XP_NMOM];
    double sig[XP_MAX_BINS][3];
    double ssum[13][3];
    int32_t cnt[XP_NCOUNT];
    double led[XP_NLEDGER];
    int32_t nabs[XP_MAX_BINS];         // photon events per bin (S5)
    int32_t kz[14];                    // K-alpha photons per charge state Z0 (XP_KA_FIELD)
    int32_t np5, pad5;                 // S5 photo candidates (XP_PHOTO_FRAC)
    // forced thermalization (variant): weight units, lab-frame and drift-frame
    // kinetic energy, draw spread, draw mean, scale; keep: 0 resample, 1 keep
    // the velocities, 2 drift velocity only
    unsigned long long tw;
    double tkin, tkth, tsig, tbeta;
    double tq[3];
    int32_t tkeep, tpad;
};

enum : int32_t {
    BN_PERM_E = 1,      // S1/S2 need the electron permutation
    BN_EI = 2,          // S2 runs
    BN_ION = 4,         // S3 evaluates Lotz and draws
    BN_FIRED = 8,       // S3 has fired ions (drift frame, accept)
    BN_REC = 16,        // S4 recombines
    BN_REC_APPLY = 32,  // S4 drift frame is usable
};

struct BigHdr {
    int32_t n_e_chunks, n_i_chunks;
    int32_t count;      // cells on the path this step
    int32_t pad;
};

struct BigArgs {
    StepArgs s;
    int32_t* list;              // cells on the path
    int32_t* count;             // their number
    BigRec* rec;
    BigHdr* hdr;
    int32_t* e_chunk_cell;      // chunk -> index into list
    int32_t* i_chunk_cell;
    double* part[4];            // per electron chunk partial sums
    uint32_t *key_a, *val_a, *key_b, *val_b, *key_c, *val_c;
    uint32_t* hist;             // [256 * chunks]
    uint8_t* iflag;             // per ion (population)
    int32_t* ccnt;              // per ion chunk counts / bases
    uint32_t* iaux;             // per ion S5 decisions
    uint32_t* wp;               // per electron reduced weights (S4)
    int32_t* sel;               // per ion selected for recombination (S4)
    double* fip;                // per fired ion (rank order) lowered potential (S3)
    double* partz;              // [13][e_chunks_max] per charge state chunk sums (S3)
    double* ev4;                // [e_pop][4] electron (vx, vy, vz, w) in slot order (S1, S2)
    double* iv4;                // [i_pop][4] ion (vx, vy, vz, Z) in slot order (S2)
    double* gev[3];             // electron velocities in permutation-rank order (S1, S2)
    uint32_t* gew;              // electron weights in rank order
    double* giv[3];             // ion velocities in rank order (S2)
    uint8_t* giz;               // ion charge states in rank order
    int32_t big_max;
    int32_t grid;               // chunk-kernel workgroups (0: default)
    int32_t e_chunks_max, i_chunks_max;
    int64_t e_pop_max, i_pop_max;
};

struct BigPlan {
    size_t list, hdr, rec, e_chunk_cell, i_chunk_cell, part, key_a, val_a, key_b, val_b, key_c,
        val_c, hist, iflag, ccnt, iaux, wp, sel, fip, gev, gew, giv, giz, partz, ev4, iv4;
    size_t bytes;
    int32_t e_chunks, i_chunks;
};

BigPlan big_plan(int32_t big_max, int64_t e_pop, int64_t i_pop);
// Enqueues the global-memory step of the cells in a.list (all cells when
// all_cells is set).
hipError_t big_launch(BigArgs& a, bool all_cells, hipStream_t s);

}  // namespace xpd
