// Reduced radiation transport along the beam (x) after a step of the XFEL
// source terms (Sec. II, Sec. III).  Photoionization takes one macro-photon
// (w0 real photons) out of the selected bin per event (Sec. III); here those
// counts set the transmission of each cell,
//   tau = 1 - nabs w0 dx / (V c dt_rad n)   (0 if negative, 1 if n = 0),
// the fraction of the c dt_rad n V / dx photons that crossed the cell's
// entrance face during the step at its density n.  The incident density of
// each bin (the run's nhv) enters every row at its low-x face; cell i's new
// density is the incident density times the transmissions of the cells before
// it, a quasi-static Beer-Lambert profile (the crossing time of a row is taken
// as short against the pulse).  K-alpha photons a cell returned to a bin
// (g macro-photons, when nka is given) join the beam leaving it: the density
// passed on is n_in tau + g w0 dx / (V c dt_rad).  Transmissions are applied
// left to right in each row and rows are summed in order, so results do not
// depend on the launch.
#include <hip/hip_runtime.h>

#include "xp_kernels.h"
#include "xp_physics.h"

namespace xpd {

namespace {

// Row kernel: a block of four waves fetches 512 cells per round trip, two per
// thread.  Row-sum kernel: one wave fetches 512 rows, eight per lane.
constexpr int TR_THREADS = 256;
constexpr int TR_CH = 2;
constexpr int TR_SPAN = TR_THREADS * TR_CH;
constexpr int TS_CH = 8;
constexpr int TS_SPAN = 64 * TS_CH;

// One block per row: the threads fetch and compute the transmissions of 512
// cells at once, thread 0 carries the running product through them in order.
// The grid is a multiple of 8 and workgroup b takes the cells of logical block
// (b mod 8) (grid / 8) + b / 8, a bijection.  Workgroups are handed to the 8
// XCDs in turn, and rows start at a fixed stride of cells (every 8th block
// for rows of 512 cells), so the identity mapping would put every row on one
// XCD and push the whole launch through that XCD's L2.
__global__ __launch_bounds__(TR_THREADS) void k_tr_rows(TransportArgs a)
{
    __shared__ double tau[TR_SPAN];
    __shared__ double gin[TR_SPAN];
    __shared__ double ent[TR_SPAN];
    __shared__ double carry_s;
    __shared__ unsigned long long starts[TR_THREADS / 64];
    const int lane = threadIdx.x;
    const int lb = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
    for (int c0 = lb * TR_THREADS; c0 < a.n_cells; c0 += gridDim.x * TR_THREADS) {
        const int c = c0 + lane;
        bool start = false;
        if (c < a.n_cells) {
            const xp_run& R = a.runs[a.cell_run[c]];
            start = R.field_per_cell && R.n_bins > 0 && R.nx > 0 && (c - R.cell_begin) % R.nx == 0;
        }
        const unsigned long long wm = __ballot(start);
        if ((lane & 63) == 0) starts[lane >> 6] = wm;
        __syncthreads();
        // the row starts of the block's cells, in cell order; every thread reads
        // the same masks, so the loops below are uniform over the block
        for (int w = 0; w < TR_THREADS / 64; ++w) {
        unsigned long long m = starts[w];
        while (m) {
            const int l = __ffsll(m) - 1;
            m &= m - 1;
            const int rc = c0 + w * 64 + l;
            const int run = a.cell_run[rc];
            const xp_run& R = a.runs[run];
            const int nx = R.nx, nb = R.n_bins;
            // the row must lie inside its run's cells, and the run's grid must
            // be its cell count; otherwise the row is left as it is and flagged
            const long long run_end = (long long)R.cell_begin + R.ncells;
            if ((long long)R.nx * R.ny != R.ncells || run_end > a.n_cells || (long long)rc + nx > run_end) {
                if (lane == 0) {
                    atomicOr(a.status, XP_ST_RUN_TABLE);
                    if (a.run_status) atomicOr(&a.run_status[run], XP_ST_RUN_TABLE);
                }
                continue;
            }
            const double cross = (R.volume * (CLIGHT * R.dt_rad)) / R.dx;
            const double w0 = R.w0;
            for (int b = 0; b < nb; ++b) {
                double carry = R.nhv[b];
                for (int i0 = 0; i0 < nx; i0 += TR_SPAN) {
                    double n[TR_CH];
                    int32_t k[TR_CH];
#pragma unroll
                    for (int q = 0; q < TR_CH; ++q) {
                        const int i = i0 + q * TR_THREADS + lane;
                        n[q] = 0.0;
                        k[q] = 0;
                        if (i < nx) {
                            const size_t at = (size_t)(rc + i) * XP_MAX_BINS + b;
                            n[q] = a.nhv[at];
                            k[q] = a.nabs[at];
                        }
                    }
#pragma unroll
                    for (int q = 0; q < TR_CH; ++q) {
                        double t = 1.0;
                        if (n[q] > 0.0) {
                            const double ab = ((double)k[q] * w0) / (cross * n[q]);
                            t = ab < 1.0 ? 1.0 - ab : 0.0;
                        }
                        tau[q * TR_THREADS + lane] = t;
                        if (a.nka) {
                            const int i = i0 + q * TR_THREADS + lane;
                            const double g = i < nx ? a.nka[(size_t)(rc + i) * XP_MAX_BINS + b] : 0.0;
                            gin[q * TR_THREADS + lane] = (g * w0) / cross;
                        }
                    }
                    __syncthreads();
                    if (lane == 0 && a.nka) {
                        // with returned K-alpha photons: n tau + g per cell
                        const int cnt = nx - i0 < TR_SPAN ? nx - i0 : TR_SPAN;
                        for (int q = 0; q < cnt; ++q) {
                            ent[q] = carry;
                            carry = carry * tau[q] + gin[q];
                        }
                        carry_s = carry;
                    } else if (lane == 0) {
                        // eight transmissions fetched ahead of their products; past
                        // the row's end tau = 1, which leaves the carry unchanged
                        const int cnt = nx - i0 < TR_SPAN ? nx - i0 : TR_SPAN;
                        for (int q = 0; q < cnt; q += 8) {
                            double tt[8], ee[8];
#pragma unroll
                            for (int j = 0; j < 8; ++j) tt[j] = tau[q + j];
#pragma unroll
                            for (int j = 0; j < 8; ++j) {
                                ee[j] = carry;
                                carry = carry * tt[j];
                            }
#pragma unroll
                            for (int j = 0; j < 8; ++j) ent[q + j] = ee[j];
                        }
                        carry_s = carry;
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < TR_CH; ++q) {
                        const int i = i0 + q * TR_THREADS + lane;
                        if (i < nx) a.nhv[(size_t)(rc + i) * XP_MAX_BINS + b] = ent[q * TR_THREADS + lane];
                    }
                    carry = carry_s;
                    __syncthreads();
                }
                if (lane == 0) a.exit[(size_t)rc * XP_MAX_BINS + b] = carry;
            }
        }
        }
        __syncthreads();   // starts[] is rewritten by the next round
    }
}

// Mean exit density of a run's rows over its incident density, per bin: the
// lanes fetch 512 rows' exit densities at a time, lane 0 adds them in row
// order.
__global__ __launch_bounds__(64) void k_tr_sum(TransportArgs a)
{
    __shared__ double v[TS_SPAN];
    const int run = blockIdx.x;
    if (run >= a.n_runs || !a.trans) return;
    const xp_run& R = a.runs[run];
    const int lane = threadIdx.x;
    // a run whose grid does not match its cell range (flagged by the row
    // kernel) reports no transmission
    const bool fits = (long long)R.nx * R.ny == R.ncells && (long long)R.cell_begin + R.ncells <= a.n_cells;
    const int nb = fits && R.field_per_cell && R.nx > 0 && R.ny > 0 ? R.n_bins : 0;
    const int ny = R.ny, nx = R.nx, c0 = R.cell_begin;
    if (lane < XP_MAX_BINS && lane >= nb) a.trans[(size_t)run * XP_MAX_BINS + lane] = 0.0;
    for (int b = 0; b < nb; ++b) {
        double s = 0.0;
        for (int j0 = 0; j0 < ny; j0 += TS_SPAN) {
#pragma unroll
            for (int q = 0; q < TS_CH; ++q) {
                const int j = j0 + q * 64 + lane;
                const int c = c0 + j * nx;
                v[q * 64 + lane] = (j < ny && c < a.n_cells) ? a.exit[(size_t)c * XP_MAX_BINS + b] : 0.0;
            }
            __syncthreads();
            if (lane == 0) {
                // past the last row v = +0, which leaves the (non-negative) sum as it is
                const int cnt = ny - j0 < TS_SPAN ? ny - j0 : TS_SPAN;
                for (int q = 0; q < cnt; q += 8) {
                    double vv[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) vv[j] = v[q + j];
#pragma unroll
                    for (int j = 0; j < 8; ++j) s = s + vv[j];
                }
            }
            __syncthreads();
        }
        if (lane == 0) {
            const double inc = R.nhv[b];
            a.trans[(size_t)run * XP_MAX_BINS + b] = inc > 0.0 ? (s / (double)ny) / inc : 0.0;
        }
    }
}

}  // namespace

hipError_t transport_launch(const TransportArgs& a, hipStream_t s)
{
    if (a.n_cells <= 0) return hipSuccess;
    const int64_t blocks = ((int64_t)a.n_cells + TR_THREADS - 1) / TR_THREADS;
    const unsigned g = (unsigned)((blocks < 65536 ? blocks : 65536) + 7) & ~7u;   // multiple of 8
    hipLaunchKernelGGL(k_tr_rows, dim3(g), dim3(TR_THREADS), 0, s, a);
    if (a.trans && a.n_runs > 0) hipLaunchKernelGGL(k_tr_sum, dim3(a.n_runs), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace xpd
