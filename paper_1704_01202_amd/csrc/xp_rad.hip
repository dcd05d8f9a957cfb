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
// as short against the pulse).  Transmissions are multiplied left to right in
// each row and rows are summed in order, so results do not depend on the
// launch.
#include <hip/hip_runtime.h>

#include "xp_kernels.h"
#include "xp_physics.h"

namespace xpd {

namespace {

// One wave per row: the lanes compute the transmissions of 64 cells at once,
// lane 0 carries the running product through them in order.
__global__ __launch_bounds__(64) void k_tr_rows(TransportArgs a)
{
    __shared__ double tau[64];
    __shared__ double ent[64];
    __shared__ double carry_s;
    const int lane = threadIdx.x;
    for (int c0 = blockIdx.x * 64; c0 < a.n_cells; c0 += gridDim.x * 64) {
        const int c = c0 + lane;
        bool start = false;
        if (c < a.n_cells) {
            const xp_run& R = a.runs[a.cell_run[c]];
            start = R.field_per_cell && R.n_bins > 0 && R.nx > 0 && (c - R.cell_begin) % R.nx == 0;
        }
        unsigned long long m = __ballot(start);
        while (m) {
            const int l = __ffsll(m) - 1;
            m &= m - 1;
            const int rc = c0 + l;
            const xp_run& R = a.runs[a.cell_run[rc]];
            const int nx = R.nx, nb = R.n_bins;
            if (rc + nx > a.n_cells) continue;   // inconsistent run table: leave the row
            const double cross = (R.volume * (CLIGHT * R.dt_rad)) / R.dx;
            const double w0 = R.w0;
            for (int b = 0; b < nb; ++b) {
                double carry = R.nhv[b];
                for (int i0 = 0; i0 < nx; i0 += 64) {
                    const int i = i0 + lane;
                    double t = 1.0;
                    if (i < nx) {
                        const size_t k = (size_t)(rc + i) * XP_MAX_BINS + b;
                        const double n = a.nhv[k];
                        if (n > 0.0) {
                            const double ab = ((double)a.nabs[k] * w0) / (cross * n);
                            t = ab < 1.0 ? 1.0 - ab : 0.0;
                        }
                    }
                    tau[lane] = t;
                    __syncthreads();
                    if (lane == 0) {
                        const int cnt = nx - i0 < 64 ? nx - i0 : 64;
#pragma unroll 8
                        for (int q = 0; q < cnt; ++q) {
                            ent[q] = carry;
                            carry = carry * tau[q];
                        }
                        carry_s = carry;
                    }
                    __syncthreads();
                    if (i < nx) a.nhv[(size_t)(rc + i) * XP_MAX_BINS + b] = ent[lane];
                    carry = carry_s;
                    __syncthreads();
                }
                if (lane == 0) a.exit[(size_t)rc * XP_MAX_BINS + b] = carry;
            }
        }
    }
}

// Mean exit density of a run's rows over its incident density, per bin: the
// lanes fetch 64 rows' exit densities at a time, lane 0 adds them in row order.
__global__ __launch_bounds__(64) void k_tr_sum(TransportArgs a)
{
    __shared__ double v[64];
    const int run = blockIdx.x;
    if (run >= a.n_runs || !a.trans) return;
    const xp_run& R = a.runs[run];
    const int lane = threadIdx.x;
    const int nb = R.field_per_cell && R.nx > 0 && R.ny > 0 ? R.n_bins : 0;
    const int ny = R.ny, nx = R.nx, c0 = R.cell_begin;
    if (lane < XP_MAX_BINS && lane >= nb) a.trans[(size_t)run * XP_MAX_BINS + lane] = 0.0;
    for (int b = 0; b < nb; ++b) {
        double s = 0.0;
        for (int j0 = 0; j0 < ny; j0 += 64) {
            const int j = j0 + lane;
            const int c = c0 + j * nx;
            v[lane] = (j < ny && c < a.n_cells) ? a.exit[(size_t)c * XP_MAX_BINS + b] : 0.0;
            __syncthreads();
            if (lane == 0) {
                const int cnt = ny - j0 < 64 ? ny - j0 : 64;
                for (int q = 0; q < cnt; ++q) s = s + v[q];
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
    const int64_t blocks = ((int64_t)a.n_cells + 63) / 64;
    const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_tr_rows, dim3(g), dim3(64), 0, s, a);
    if (a.trans && a.n_runs > 0) hipLaunchKernelGGL(k_tr_sum, dim3(a.n_runs), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace xpd
