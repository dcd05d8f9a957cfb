// diagnostics: per-run charge-state distribution, electron energy histogram,
// weights, Zbar, kinetic energy and T_e = (2/3) K / W_e (Sec. II, Sec. VI.B).
// Integer tallies are exact (atomic adds); the kinetic energy is a canonical
// pairwise sum per cell followed by a canonical pairwise sum over the run's
// cells, so the record does not depend on the launch schedule.
#include <hip/hip_runtime.h>

#include "xp_kernels.h"
#include "xp_physics.h"

namespace xpd {

namespace {

__global__ void k_diag_zero(xp_diag* out, int n_runs)
{
    const int r = blockIdx.x;
    if (r >= n_runs) return;
    int64_t* p = (int64_t*)(out + r);
    const int words = (int)(sizeof(xp_diag) / 8);
    for (int q = threadIdx.x; q < words; q += blockDim.x) p[q] = 0;
}

__global__ __launch_bounds__(64) void k_diag_cells(DiagArgs a)
{
    const int cell = blockIdx.x;
    if (cell >= a.n_cells) return;
    const int run = a.cell_run[cell];
    xp_diag* o = a.out + run;
    const int ne = a.e_cnt[cell], ni = a.i_cnt[cell];
    const int64_t eo = a.e_off[cell], io = a.i_off[cell];
    const double lmin = xlog(0.1);
    const double dl = (xlog(1.0e5) - xlog(0.1)) / 64.0;
    long long we = 0, wi = 0, sz = 0;
    for (int j = threadIdx.x; j < ni; j += 64) {
        const int z = a.iz[io + j];
        atomicAdd((unsigned long long*)&o->csd[z], 1ull);
        wi += 1;
        sz += z;
    }
    for (int j = threadIdx.x; j < ne; j += 64) {
        const double x = a.evx[eo + j], y = a.evy[eo + j], z = a.evz[eo + j];
        const double e = HALF_ME_OVER_QE * ((x * x + y * y) + z * z);
        const uint32_t w = a.ew[eo + j];
        we += w;
        int bin = 0;
        if (e > 0.0) {
            const double u = (xlog(e) - lmin) / dl;
            bin = u < 0.0 ? 0 : (u >= 63.0 ? 63 : (int)u);
        }
        atomicAdd((unsigned long long*)&o->fe_hist[bin], (unsigned long long)w);
    }
    __shared__ double red[2 * (DIAG_CHUNK / 64)];
    extern __shared__ double part[];   // [ceil(e_cap_max / DIAG_CHUNK)]
    auto leaf = [&](int64_t j) {
        const double x = a.evx[eo + j], y = a.evy[eo + j], z = a.evz[eo + j];
        return (double)a.ew[eo + j] * (HALF_ME_OVER_QE * ((x * x + y * y) + z * z));
    };
    double k;
    if (ne <= DIAG_CHUNK) {
        k = block_tree_sum<64>(ne, [&](int j) { return leaf(j); }, red);
    } else {
        // aligned chunks are subtrees of the cell's pairwise sum
        const int nch = (ne + DIAG_CHUNK - 1) / DIAG_CHUNK;
        for (int c = 0; c < nch; ++c) {
            const int64_t base = (int64_t)c * DIAG_CHUNK;
            const int n = ne - base < DIAG_CHUNK ? (int)(ne - base) : DIAG_CHUNK;
            const double t = block_tree_sum<64>(DIAG_CHUNK, [&](int j) { return j < n ? leaf(base + j) : 0.0; }, red);
            if (threadIdx.x == 0) part[c] = t;
        }
        __syncthreads();
        k = block_tree_sum<64>(nch, [&](int j) { return part[j]; }, red);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        we += __shfl_xor(we, off, 64);
        wi += __shfl_xor(wi, off, 64);
        sz += __shfl_xor(sz, off, 64);
    }
    if (threadIdx.x == 0) {
        a.cell_k[cell] = k;
        atomicAdd((unsigned long long*)&o->w_e, (unsigned long long)we);
        atomicAdd((unsigned long long*)&o->w_i, (unsigned long long)wi);
        atomicAdd((unsigned long long*)&o->sum_z, (unsigned long long)sz);
        atomicAdd((unsigned long long*)&o->n_e_macro, (unsigned long long)ne);
    }
}

__global__ __launch_bounds__(256) void k_diag_runs(DiagArgs a, uint32_t what)
{
    extern __shared__ double red[];
    const int r = blockIdx.x;
    if (r >= a.n_runs) return;
    const xp_run* R = a.runs + r;
    const int c0 = R->cell_begin;
    const double k = block_tree_sum<256>(R->ncells, [&](int c) { return a.cell_k[c0 + c]; }, red);
    if (threadIdx.x == 0) {
        xp_diag* o = a.out + r;
        o->ke_ev = k;
        o->zbar = o->w_i > 0 ? (double)o->sum_z / (double)o->w_i : 0.0;
        o->te_ev = o->w_e > 0 ? (2.0 * k) / (3.0 * (double)o->w_e) : 0.0;
    }
    if (threadIdx.x < XP_NCOUNT && a.run_cnt) {
        a.out[r].counters[threadIdx.x] = a.run_cnt[(size_t)r * XP_NCOUNT + threadIdx.x];
        if (what & XP_DIAG_RESET) a.run_cnt[(size_t)r * XP_NCOUNT + threadIdx.x] = 0;
    }
    if (threadIdx.x >= 64 && threadIdx.x < 64 + XP_NLEDGER && a.run_led) {
        const int q = threadIdx.x - 64;
        a.out[r].ledger[q] = a.run_led[(size_t)r * XP_NLEDGER + q];
        if (what & XP_DIAG_RESET) a.run_led[(size_t)r * XP_NLEDGER + q] = 0.0;
    }
}

}  // namespace

hipError_t diag_launch(const DiagArgs& a, uint32_t what, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_zero, dim3(a.n_runs), dim3(64), 0, s, a.out, a.n_runs);
    const int nch_max = (a.e_cap_max + DIAG_CHUNK - 1) / DIAG_CHUNK;
    const size_t cell_smem = sizeof(double) * (size_t)(nch_max > 1 ? nch_max : 1);
    if (a.n_cells > 0) hipLaunchKernelGGL(k_diag_cells, dim3(a.n_cells), dim3(64), cell_smem, s, a);
    int p = 64;
    while (p < a.n_cells) p <<= 1;
    const size_t smem = 2 * sizeof(double) * (size_t)(p / 64);
    if (smem > 65536) hipFuncSetAttribute((const void*)k_diag_runs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    hipLaunchKernelGGL(k_diag_runs, dim3(a.n_runs), dim3(256), smem, s, a, what);
    return hipGetLastError();
}

}  // namespace xpd

namespace xpd {
namespace {

// Evaluates one device building block on n inputs (library self-test).
__global__ void k_selftest(int which, int64_t n, const double* x, const uint64_t* u, double* out,
                           uint32_t* words)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    switch (which) {
    case 0: out[i] = xlog(x[i]); break;
    case 1: out[i] = xexp(x[i]); break;
    case 2: out[i] = xcbrt(x[i]); break;
    case 3: {
        double s, c;
        xsincos2pi(u[i], s, c);
        out[2 * i] = s;
        out[2 * i + 1] = c;
        break;
    }
    case 4: {
        const uint32_t* c = (const uint32_t*)(u + 3 * i);
        const Words w = philox(c[0], c[1], c[2], c[3], c[4], c[5]);
        words[4 * i] = w.x0;
        words[4 * i + 1] = w.x1;
        words[4 * i + 2] = w.x2;
        words[4 * i + 3] = w.x3;
        break;
    }
    case 5: out[i] = sqrt(x[i]); break;
    case 6: out[i] = x[2 * i] / x[2 * i + 1]; break;
    default: break;
    }
}

// Canonical sums of the first m_j leaves of row j (rows of R values of x): a
// block of B threads per row, or (G > 1) G lane groups of 64 / G lanes per
// wave, one row each.  m_j = (j * 37) % R + 1 exercises the padding.
template <int B, int R>
__global__ __launch_bounds__(B) void k_selftest_tree(int64_t rows, const double* x, double* out)
{
    __shared__ double red[2 * (R / 64 > 1 ? R / 64 : 1)];
    const int64_t j = blockIdx.x;
    if (j >= rows) return;
    const int m = (int)((j * 37) % R) + 1;
    const double* row = x + j * R;
    const double t = block_tree_sum<B>(m, [&](int k) { return row[k]; }, red);
    if (threadIdx.x == 0) out[j] = t;
}

template <int W>
__global__ __launch_bounds__(64) void k_selftest_group_tree(int64_t rows, const double* x, double* out)
{
    const int64_t j = (int64_t)blockIdx.x * (64 / W) + threadIdx.x / W;
    const int m = (int)((j * 37) % (4 * W)) + 1;
    const double* row = x + (j < rows ? j : 0) * (4 * W);
    const double t = group_tree_sum<W>(m, [&](int k) { return row[k]; });
    if ((threadIdx.x & (W - 1)) == 0 && j < rows) out[j] = t;
}

}  // namespace

hipError_t selftest_launch(int which, int64_t n, const double* x, const uint64_t* u, double* out,
                           uint32_t* words, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (which == 7) {
        hipLaunchKernelGGL((k_selftest_tree<64, 64>), dim3((unsigned)(n / 64)), dim3(64), 0, s, n / 64, x, out);
    } else if (which == 8) {
        hipLaunchKernelGGL((k_selftest_tree<256, 256>), dim3((unsigned)(n / 256)), dim3(256), 0, s, n / 256, x, out);
    } else if (which == 9) {
        const int64_t rows = n / 64;   // groups of 16 lanes, 64 leaves per row
        hipLaunchKernelGGL(k_selftest_group_tree<16>, dim3((unsigned)((rows + 3) / 4)), dim3(64), 0, s, rows, x, out);
    } else {
        hipLaunchKernelGGL(k_selftest, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, which, n, x, u,
                           out, words);
    }
    return hipGetLastError();
}

}  // namespace xpd
