// bin_particles: stable counting sort of unsorted particles into cell slabs.
//
//   1. cell id of every particle (floor of position / cell size, clamped) and
//      per-cell counts (atomic adds: the totals do not depend on order);
//   2. slab capacities from the counts, exclusive scans -> slab offsets and
//      compact cell starts, required sizes checked against the arrays;
//   3. LSD radix sort of the 32-bit cell ids, 8 bits per pass.  A tile of
//      1024 keys is owned by one wave, which ranks each chunk of 64 keys with
//      ballots over the digit bits (peers with the same digit, popcount below
//      the lane) and keeps running per-digit offsets in LDS, so every pass is
//      stable and the result is the input order within each cell;
//   4. gather of every particle field into its slab slot.
#include <hip/hip_runtime.h>

#include "xp_kernels.h"

namespace xpd {

namespace {

constexpr int TILE = 1024;     // keys per wave in the radix passes
constexpr int SCAN_B = 256;    // threads per scan block
constexpr int SCAN_PER = 4;    // elements per scan thread

__device__ __forceinline__ int cell_of(const xp_run& R, double x, double y)
{
    const double fx = floor((x - R.x0) / R.dx);
    const int ix = fx < 0.0 ? 0 : (fx > (double)(R.nx - 1) ? R.nx - 1 : (int)fx);
    int iy = 0;
    if (R.ny > 1) {
        const double fy = floor((y - R.y0) / R.dy);
        iy = fy < 0.0 ? 0 : (fy > (double)(R.ny - 1) ? R.ny - 1 : (int)fy);
    }
    return R.cell_begin + ix + R.nx * iy;
}

__global__ void k_cell_ids(int64_t n, const int32_t* prun, const double* x, const double* y,
                           const xp_run* runs, uint32_t* key, uint32_t* val, int32_t* count)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n;
    int c = 0;
    if (valid) {
        const int r = prun ? prun[p] : 0;
        c = cell_of(runs[r], x[p], y ? y[p] : 0.0);
        if (key) {
            key[p] = (uint32_t)c;
            val[p] = (uint32_t)p;
        }
    }
    if (!count) return;
    // lanes of a wave that share a cell (inputs are often grouped by cell or
    // run) add their count with one atomic; a few rounds, then one per lane
    const int lane = threadIdx.x & 63;
    bool todo = valid;
    for (int it = 0; it < 4; ++it) {
        const uint64_t act = __ballot(todo);
        if (act == 0) break;
        const int first = __ffsll((unsigned long long)act) - 1;
        const int c0 = __shfl(c, first, 64);
        const bool same = todo && c == c0;
        const uint64_t grp = __ballot(same);
        if (same && lane == first) atomicAdd(&count[c0], (int)__popcll(grp));
        if (same) todo = false;
    }
    if (todo) atomicAdd(&count[c], 1);
}

__global__ void k_caps(int n_cells, const int32_t* ce, const int32_t* ci, int32_t e_per_ion,
                       int32_t e_extra, int32_t* e_cnt, int32_t* i_cnt, int32_t* e_cap,
                       int32_t* i_cap, int64_t* e_off, int64_t* i_off, int64_t* e_start,
                       int64_t* i_start, int64_t* need, int32_t e_lds, int32_t i_lds)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int64_t ne = ce[c], ni = ci[c];
    const int64_t capE = ((ne + (int64_t)e_per_ion * ni + e_extra + 15) / 16) * 16;
    const int64_t capI = ((ni + 15) / 16) * 16;
    e_cnt[c] = (int32_t)ne;
    i_cnt[c] = (int32_t)ni;
    e_cap[c] = (int32_t)capE;
    i_cap[c] = (int32_t)capI;
    e_off[c] = capE;
    i_off[c] = capI;
    e_start[c] = ne;
    i_start[c] = ni;
    atomicMax((unsigned long long*)&need[2], (unsigned long long)capE);
    atomicMax((unsigned long long*)&need[3], (unsigned long long)capI);
    // cells that may outgrow every LDS plan: bounds of the global-memory path
    if (capE > e_lds || ni > i_lds) {
        atomicAdd((unsigned long long*)&need[4], 1ull);
        atomicAdd((unsigned long long*)&need[5], (unsigned long long)capE);
        atomicAdd((unsigned long long*)&need[6], (unsigned long long)capI);
    }
}

// In-place exclusive scan of SCAN_B * SCAN_PER elements per block; block total
// to aux[block].
template <class T>
__global__ void k_scan_local(T* data, int64_t n, T* aux)
{
    __shared__ T part[SCAN_B];
    const int64_t base = (int64_t)blockIdx.x * (SCAN_B * SCAN_PER) + (int64_t)threadIdx.x * SCAN_PER;
    T v[SCAN_PER];
    T s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        v[q] = base + q < n ? data[base + q] : T(0);
        s += v[q];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_B; off <<= 1) {
        T t = threadIdx.x >= off ? part[threadIdx.x - off] : T(0);
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    T run = threadIdx.x > 0 ? part[threadIdx.x - 1] : T(0);
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        if (base + q < n) data[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == SCAN_B - 1 && aux) aux[blockIdx.x] = part[SCAN_B - 1];
}

template <class T>
__global__ void k_scan_add(T* data, int64_t n, const T* aux)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) data[i] += aux[i / (SCAN_B * SCAN_PER)];
}

__global__ void k_need(int n_cells, const int64_t* e_off, const int32_t* e_cap,
                       const int64_t* i_off, const int32_t* i_cap, int64_t e_slots,
                       int64_t i_slots, int64_t* need, uint32_t* status, uint32_t* ok)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t ne = n_cells ? e_off[n_cells - 1] + e_cap[n_cells - 1] : 0;
    const int64_t ni = n_cells ? i_off[n_cells - 1] + i_cap[n_cells - 1] : 0;
    need[0] = ne;
    need[1] = ni;
    const bool fits = ne <= e_slots && ni <= i_slots;
    *ok = fits ? 1u : 0u;
    if (!fits) atomicOr(status, XP_ST_BIN_SIZE);
}

// One wave per tile: per-digit counts of the tile -> hist[digit * ntiles + tile].
__global__ __launch_bounds__(64) void k_radix_hist(const uint32_t* key, int64_t n, int shift,
                                                   int64_t ntiles, uint32_t* hist)
{
    __shared__ uint32_t h[256];
    for (int q = threadIdx.x; q < 256; q += 64) h[q] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x;
    const int64_t b = t * TILE;
    for (int q = threadIdx.x; q < TILE; q += 64) {
        const int64_t i = b + q;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 256; q += 64) hist[(int64_t)q * ntiles + t] = h[q];
}

// One wave per tile: stable scatter with ballot-ranked chunks of 64 keys.
__global__ __launch_bounds__(64) void k_radix_scatter(const uint32_t* key, const uint32_t* val,
                                                      int64_t n, int shift, int64_t ntiles,
                                                      const uint32_t* hist, uint32_t* key_out,
                                                      uint32_t* val_out)
{
    __shared__ uint32_t run[256];
    const int64_t t = blockIdx.x;
    for (int q = threadIdx.x; q < 256; q += 64) run[q] = hist[(int64_t)q * ntiles + t];
    __syncthreads();
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t b = t * TILE;
    for (int c = 0; c < TILE; c += 64) {
        const int64_t i = b + c + lane;
        const bool valid = i < n;
        const uint32_t k = valid ? key[i] : 0u;
        const uint32_t v = valid ? val[i] : 0u;
        const uint32_t d = (k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bal = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t base = valid ? run[d] : 0u;
        __syncthreads();
        if (valid) {
            const uint32_t dst = base + rank;
            key_out[dst] = k;
            val_out[dst] = v;
            if ((peers & lt) == 0) run[d] = base + (uint32_t)__popcll(peers);
        }
        __syncthreads();
    }
}

template <int NF>
struct Gather {
    const double* src[NF];
    double* dst[NF];
};

__global__ void k_gather_e(int64_t n, const uint32_t* key, const uint32_t* val,
                           const int64_t* start, const int64_t* off, Gather<5> g,
                           const uint32_t* w_in, uint32_t* w_out, const uint32_t* ok)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || *ok == 0u) return;
    const uint32_t c = key[s];
    const uint32_t p = val[s];
    const int64_t dst = off[c] + (s - start[c]);
#pragma unroll
    for (int f = 0; f < 5; ++f)
        if (g.dst[f]) g.dst[f][dst] = g.src[f] ? g.src[f][p] : 0.0;
    w_out[dst] = w_in[p];
}

__global__ void k_gather_i(int64_t n, const uint32_t* key, const uint32_t* val,
                           const int64_t* start, const int64_t* off, Gather<5> g,
                           const uint8_t* z_in, const uint8_t* k_in, uint8_t* z_out,
                           uint8_t* k_out, const uint32_t* ok)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || *ok == 0u) return;
    const uint32_t c = key[s];
    const uint32_t p = val[s];
    const int64_t dst = off[c] + (s - start[c]);
#pragma unroll
    for (int f = 0; f < 5; ++f)
        if (g.dst[f]) g.dst[f][dst] = g.src[f] ? g.src[f][p] : 0.0;
    z_out[dst] = z_in[p];
    k_out[dst] = k_in[p];
}

}  // namespace

// -------------------------------------------------------------------------
// host side

BinPlan bin_plan(int64_t ne, int64_t ni, int32_t n_cells)
{
    BinPlan p{};
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t n = ne > ni ? ne : ni;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t hist_n = 256 * (ntiles > 0 ? ntiles : 1);
    size_t o = 0;
    p.key_a = o; o += up(4 * (size_t)(n > 0 ? n : 1));
    p.val_a = o; o += up(4 * (size_t)(n > 0 ? n : 1));
    p.key_b = o; o += up(4 * (size_t)(n > 0 ? n : 1));
    p.val_b = o; o += up(4 * (size_t)(n > 0 ? n : 1));
    p.hist = o; o += up(4 * (size_t)hist_n);
    const int64_t scan_n = hist_n > n_cells ? hist_n : (int64_t)n_cells;
    p.scan_aux = o; o += up(8 * (size_t)(scan_n / (SCAN_B * SCAN_PER) + 64) * 2);
    p.cnt_e = o; o += up(4 * (size_t)n_cells);
    p.cnt_i = o; o += up(4 * (size_t)n_cells);
    p.start_e = o; o += up(8 * (size_t)n_cells);
    p.start_i = o; o += up(8 * (size_t)n_cells);
    p.flags = o; o += up(16);
    p.bytes = o;
    return p;
}

namespace {

template <class T>
hipError_t scan_exclusive(T* data, int64_t n, T* aux, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t per = SCAN_B * SCAN_PER;
    const int64_t nb = (n + per - 1) / per;
    hipLaunchKernelGGL(k_scan_local<T>, dim3((unsigned)nb), dim3(SCAN_B), 0, s, data, n, nb > 1 ? aux : (T*)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    e = scan_exclusive<T>(aux, nb, aux + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, data, n, (const T*)aux);
    return hipGetLastError();
}

hipError_t radix_sort(int64_t n, int bits, uint32_t*& key, uint32_t*& val, uint32_t* key2,
                      uint32_t* val2, uint32_t* hist, uint32_t* aux, hipStream_t s)
{
    const int64_t ntiles = (n + TILE - 1) / TILE;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(64), 0, s, key, n, shift, ntiles, hist);
        hipError_t e = scan_exclusive<uint32_t>(hist, 256 * ntiles, aux, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(64), 0, s, key, val, n, shift,
                           ntiles, hist, key2, val2);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint32_t* tk = key;
        key = key2;
        key2 = tk;
        uint32_t* tv = val;
        val = val2;
        val2 = tv;
    }
    return hipSuccess;
}

}  // namespace

hipError_t bin_launch(const xp_particles* in, xp_batch* b, const xp_capacity* cap,
                      int64_t* d_need, int32_t e_lds, int32_t i_lds, hipStream_t s)
{
    const BinPlan P = bin_plan(in->ne, in->ni, b->n_cells);
    char* w = (char*)b->d_work;
    uint32_t* key_a = (uint32_t*)(w + P.key_a);
    uint32_t* val_a = (uint32_t*)(w + P.val_a);
    uint32_t* key_b = (uint32_t*)(w + P.key_b);
    uint32_t* val_b = (uint32_t*)(w + P.val_b);
    uint32_t* hist = (uint32_t*)(w + P.hist);
    int32_t* cnt_e = (int32_t*)(w + P.cnt_e);
    int32_t* cnt_i = (int32_t*)(w + P.cnt_i);
    int64_t* st_e = (int64_t*)(w + P.start_e);
    int64_t* st_i = (int64_t*)(w + P.start_i);
    uint32_t* ok = (uint32_t*)(w + P.flags);
    int64_t* aux64 = (int64_t*)(w + P.scan_aux);
    uint32_t* aux32 = (uint32_t*)(w + P.scan_aux);
    const int nc = b->n_cells;
    hipError_t e;
    if ((e = hipMemsetAsync(cnt_e, 0, 4 * (size_t)nc, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(cnt_i, 0, 4 * (size_t)nc, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(d_need, 0, 8 * sizeof(int64_t), s)) != hipSuccess) return e;
    int bits = 0;
    while ((1ll << bits) < (long long)nc) ++bits;

    // counts per cell, capacities, slab offsets, compact starts, size check
    if (in->ne > 0)
        hipLaunchKernelGGL(k_cell_ids, dim3((unsigned)((in->ne + 255) / 256)), dim3(256), 0, s, in->ne,
                           in->d_e_run, in->d_ex, in->d_ey, b->d_runs, (uint32_t*)nullptr,
                           (uint32_t*)nullptr, cnt_e);
    if (in->ni > 0)
        hipLaunchKernelGGL(k_cell_ids, dim3((unsigned)((in->ni + 255) / 256)), dim3(256), 0, s, in->ni,
                           in->d_i_run, in->d_ix, in->d_iy, b->d_runs, (uint32_t*)nullptr,
                           (uint32_t*)nullptr, cnt_i);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_caps, dim3((nc + 255) / 256), dim3(256), 0, s, nc, cnt_e, cnt_i,
                       cap->e_per_ion, cap->e_extra, b->d_e_cnt, b->d_i_cnt, b->d_e_cap,
                       b->d_i_cap, b->d_e_off, b->d_i_off, st_e, st_i, d_need, e_lds, i_lds);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive<int64_t>(b->d_e_off, nc, aux64, s)) != hipSuccess) return e;
    if ((e = scan_exclusive<int64_t>(b->d_i_off, nc, aux64, s)) != hipSuccess) return e;
    if ((e = scan_exclusive<int64_t>(st_e, nc, aux64, s)) != hipSuccess) return e;
    if ((e = scan_exclusive<int64_t>(st_i, nc, aux64, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_need, dim3(1), dim3(64), 0, s, nc, b->d_e_off, b->d_e_cap, b->d_i_off,
                       b->d_i_cap, b->e_slots, b->i_slots, d_need, b->d_status, ok);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    // electrons: ids, stable radix sort, gather into slabs
    if (in->ne > 0) {
        hipLaunchKernelGGL(k_cell_ids, dim3((unsigned)((in->ne + 255) / 256)), dim3(256), 0, s, in->ne,
                           in->d_e_run, in->d_ex, in->d_ey, b->d_runs, key_a, val_a, (int32_t*)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        uint32_t *k = key_a, *v = val_a;
        if ((e = radix_sort(in->ne, bits, k, v, key_b, val_b, hist, aux32, s)) != hipSuccess) return e;
        Gather<5> g{{in->d_ex, in->d_ey, in->d_evx, in->d_evy, in->d_evz},
                    {b->d_ex, b->d_ey, b->d_evx, b->d_evy, b->d_evz}};
        hipLaunchKernelGGL(k_gather_e, dim3((unsigned)((in->ne + 255) / 256)), dim3(256), 0, s, in->ne,
                           (const uint32_t*)k, (const uint32_t*)v, (const int64_t*)st_e,
                           (const int64_t*)b->d_e_off, g, in->d_ew, b->d_ew, (const uint32_t*)ok);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // ions
    if (in->ni > 0) {
        hipLaunchKernelGGL(k_cell_ids, dim3((unsigned)((in->ni + 255) / 256)), dim3(256), 0, s, in->ni,
                           in->d_i_run, in->d_ix, in->d_iy, b->d_runs, key_a, val_a, (int32_t*)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        uint32_t *k = key_a, *v = val_a;
        if ((e = radix_sort(in->ni, bits, k, v, key_b, val_b, hist, aux32, s)) != hipSuccess) return e;
        Gather<5> g{{in->d_ix, in->d_iy, in->d_ivx, in->d_ivy, in->d_ivz},
                    {b->d_ix, b->d_iy, b->d_ivx, b->d_ivy, b->d_ivz}};
        hipLaunchKernelGGL(k_gather_i, dim3((unsigned)((in->ni + 255) / 256)), dim3(256), 0, s, in->ni,
                           (const uint32_t*)k, (const uint32_t*)v, (const int64_t*)st_i,
                           (const int64_t*)b->d_i_off, g, in->d_iz, in->d_ik, b->d_iz, b->d_ik,
                           (const uint32_t*)ok);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace xpd
