// The per-cell Monte-Carlo step (Sec. II-V): one workgroup per cell, the
// cell's particles staged in LDS, every stage of the step in one pass.
//
// Work decomposition inside a cell:
//   * moments, Lotz cross sections, per-ion draws and rescales: one thread per
//     particle (strided loops over the block);
//   * random permutations: 64-bit keys (Philox word << 32 | slot) sorted by a
//     bitonic network in LDS;
//   * e-e pairs: one thread per pair, the odd triplet on thread 0;
//   * e-i pairs: one thread per pair within a round, rounds separated by
//     barriers (a round touches every ion at most once);
//   * accept-in-order decisions (ionization energy budget, recombination
//     sequence) on thread 0 over the few selected events;
//   * appends / removals: ordered compaction with wave ballots.
// Global memory is touched twice per particle: one coalesced read of the
// cell's slab at the start, one coalesced write at the end.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "xp_kernels.h"
#include "xp_physics.h"

namespace xpd {

namespace {

template <int RED>
struct CellSharedT {
    double red[RED];
    long long ired[16];
    int sel[16];
    int cnt[XP_NCOUNT];
    int nabs[XP_MAX_BINS];   // photon events per bin (S5)
    double led[XP_NLEDGER];
    double mom[XP_NMOM];
    double sig[XP_MAX_BINS][3];
    double ssum[13][3];
    double pz[13];        // S3 probability per evaluated charge state
    double prz[14];       // S4 (XP_REC_XS) recombination probability per charge state
    double lnp[5];        // S3 logarithms of the lowered bindings, one per subshell
    double dbl[8];
    int ints[8];
    int kz[14];                    // S5 K-alpha photons per charge state (XP_KA_FIELD)
    double pbud[XP_MAX_BINS];      // S5 macro-photons per bin held by the cell (XP_PHOTO_FRAC)
    double pused[XP_MAX_BINS];     // and taken so far
};
using CellShared = CellSharedT<256>;

// A team steps one cell: a whole workgroup of B threads (one or four waves),
// or an aligned group of W lanes of a wave that steps 64 / W cells at once.
// The step is written once against this interface.
template <int B>
struct BlockTeam {
    static constexpr int N = B;
    static constexpr bool REREAD = true;   // see step_args
    // a wave's tree sums keep at most two row sums per 64 leaves in LDS
    using Shared = CellSharedT<B == 64 ? 128 : 256>;
    __device__ static int rank() { return threadIdx.x; }
    __device__ static void sync() { __syncthreads(); }
    __device__ static long long isum(long long v, Shared& S) { return block_isum<B>(v, S.ired); }
    template <class F>
    __device__ static double tree(int n, F f, Shared& S) { return block_tree_sum<B>(n, f, S.red); }
    template <class P, class E>
    __device__ static int select(int n, P pred, E emit, Shared& S)
    {
        return block_ordered_select<B>(n, pred, emit, S.sel);
    }
    __device__ static int prefix(int v, int& tot, Shared& S) { return block_exclusive_sum<B, int>(v, S.sel, tot); }
    // smallest value over the block, returned to every thread
    __device__ static uint64_t umin(uint64_t v, Shared& S)
    {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = shfl_xor_u64(v, off);
            v = o < v ? o : v;
        }
        if (B == 64) return v;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) S.ired[threadIdx.x >> 6] = (long long)v;
        __syncthreads();
        uint64_t m = ~0ull;
#pragma unroll
        for (int w = 0; w < B / 64; ++w) {
            const uint64_t o = (uint64_t)S.ired[w];
            m = o < m ? o : m;
        }
        __syncthreads();
        return m;
    }
};

template <int W>
struct GroupTeam {
    static constexpr int N = W;
    static constexpr bool REREAD = false;   // see step_args
    using Shared = CellSharedT<1>;
    __device__ static int rank() { return threadIdx.x & (W - 1); }
    // the groups of a workgroup share one wave: LDS accesses of a wave are
    // ordered, so a wave barrier with workgroup fences orders the group
    __device__ static void sync()
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __device__ static long long isum(long long v, Shared&)
    {
#pragma unroll
        for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
        return v;
    }
    template <class F>
    __device__ static double tree(int n, F f, Shared&) { return group_tree_sum<W>(n, f); }
    template <class P, class E>
    __device__ static int select(int n, P pred, E emit, Shared&)
    {
        const int t = rank();
        const int sh = threadIdx.x & 63 & ~(W - 1);
        const uint64_t gmask = W == 64 ? ~0ull : ((1ull << W) - 1ull);
        int base = 0;
        for (int c0 = 0; c0 < n; c0 += W) {
            const int j = c0 + t;
            const bool f = j < n && pred(j);
            const uint64_t gm = (__ballot(f) >> sh) & gmask;
            if (f) emit(j, base + __popcll(gm & ((1ull << t) - 1ull)));
            base += __popcll(gm);
        }
        return base;
    }
    __device__ static int prefix(int v, int& tot, Shared&)
    {
        const int t = rank();
        int incl = v;
#pragma unroll
        for (int off = 1; off < W; off <<= 1) {
            const int o = __shfl_up(incl, off, W);
            if (t >= off) incl += o;
        }
        tot = __shfl(incl, W - 1, W);
        return incl - v;
    }
    __device__ static uint64_t umin(uint64_t v, Shared&)
    {
#pragma unroll
        for (int off = W / 2; off > 0; off >>= 1) {
            const uint64_t o = shfl_xor_u64w(v, off, W);
            v = o < v ? o : v;
        }
        return v;
    }
};

struct Lds {
    double *evx, *evy, *evz;
    uint32_t* ew;
    int32_t* eorg;     // position source: >= 0 old slot, < 0 new electron of ion (-1 - i)
    int32_t* perm_e;
    uint8_t* esel;
    double *ivx, *ivy, *ivz;
    uint8_t *iz, *ik;
    int32_t* perm_i;
    int32_t* list;
    uint8_t *z0, *k0, *emask, *fwok;
    uint16_t* ebins;
    uint32_t* fw;      // cached words 1..3 of each ion's RP_ION draw
    uint64_t* sbuf;
};

__device__ __forceinline__ Lds carve(unsigned char* base, int ce, int ci, int ps)
{
    Lds L;
    unsigned char* p = base;
    auto take = [&](size_t bytes) {
        unsigned char* r = p;
        p += (bytes + 15) & ~size_t(15);
        return r;
    };
    L.sbuf = (uint64_t*)take(sizeof(uint64_t) * ps);
    L.evx = (double*)take(sizeof(double) * ce);
    L.evy = (double*)take(sizeof(double) * ce);
    L.evz = (double*)take(sizeof(double) * ce);
    L.ivx = (double*)take(sizeof(double) * ci);
    L.ivy = (double*)take(sizeof(double) * ci);
    L.ivz = (double*)take(sizeof(double) * ci);
    L.ew = (uint32_t*)take(sizeof(uint32_t) * ce);
    L.eorg = (int32_t*)take(sizeof(int32_t) * ce);
    L.perm_e = (int32_t*)take(sizeof(int32_t) * ce);
    L.perm_i = (int32_t*)take(sizeof(int32_t) * ci);
    L.list = (int32_t*)take(sizeof(int32_t) * ci);
    L.ebins = (uint16_t*)take(sizeof(uint16_t) * ci);
    L.fw = (uint32_t*)take(sizeof(uint32_t) * 3 * ci);
    L.esel = (uint8_t*)take(ce);
    L.iz = (uint8_t*)take(ci);
    L.ik = (uint8_t*)take(ci);
    L.z0 = (uint8_t*)take(ci);
    L.k0 = (uint8_t*)take(ci);
    L.emask = (uint8_t*)take(ci);
    L.fwok = (uint8_t*)take(ci);
    return L;
}

__host__ __device__ inline int pow2_at_least(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

}  // namespace

__host__ __device__ size_t step_lds_bytes_dev(int ce, int ci)
{
    const int ps = pow2_at_least(ce > ci ? ce : ci);
    auto r = [](size_t b) { return (b + 15) & ~size_t(15); };
    size_t n = r(8ull * ps) + 3 * r(8ull * ce) + 3 * r(8ull * ci) + 3 * r(4ull * ce) +
               2 * r(4ull * ci) + r(2ull * ci) + r(12ull * ci) + r(ce) + 6 * r(ci);
    return n;
}

using KArgsPtr = const StepArgs __attribute__((address_space(4)))*;
// The launch's step arguments as a stage of the step reads them.  For teams
// with REREAD, a pointer to the kernarg segment (the kernel's only argument,
// at its start) made opaque: loads through it are not hoisted above this
// point, so a stage's argument values need not stay live through the stages
// before it (fewer scalar registers spilled to vector lanes in the wave and
// block kernels).  The lane-group kernels read the kernel's argument as it is.
template <class T>
__device__ __forceinline__ auto step_args(const StepArgs& a)
{
    if constexpr (T::REREAD) {
        uint64_t v = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(v));
        return (KArgsPtr)v;
    } else {
        return &a;
    }
}

template <class T, int XV>
__device__ bool step_cell(const StepArgs& a, int cell, typename T::Shared& S, const Lds& L);

size_t step_lds_bytes(int ce, int ci) { return step_lds_bytes_dev(ce, ci); }

// One workgroup per cell at a time, looping over the cells of the launch:
// all cells (cell_list == nullptr) or the cells listed by an earlier launch
// whose LDS plan they outgrew.  The run counters and tallies of the committed
// cells are summed in LDS and added to the run's records when the run
// changes and at the end, so a launch issues a few atomics per workgroup
// rather than per cell.  Three waves per SIMD: the step is bound by the
// latency of its FP64 chains, and the register budget of three waves holds it
// with almost no spilling.
template <int B, int XV>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(3))) void k_step(StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ typename BlockTeam<B>::Shared S;
    __shared__ unsigned long long acc_cnt[XP_NCOUNT];
    __shared__ double acc_led[XP_NLEDGER];
    __shared__ int acc_run, acc_max;
    __shared__ int acc_hist[64];      // committed cells by electron count (16 per bucket)
    const int tid = threadIdx.x;
    const int ce = a.lds_ce, ci = a.lds_ci;
    const int ps = pow2_at_least(ce > ci ? ce : ci);
    const Lds L = carve(smem, ce, ci, ps);
    for (int q = tid; q < XP_NCOUNT; q += B) acc_cnt[q] = 0;
    for (int q = tid; q < XP_NLEDGER; q += B) acc_led[q] = 0.0;
    for (int q = tid; q < 64; q += B) acc_hist[q] = 0;
    if (tid == 0) {
        acc_run = -1;
        acc_max = 0;
    }
    __syncthreads();
    auto flush = [&]() {
        const int r = acc_run;
        if (r >= 0) {
            if (a.run_cnt)
                for (int q = tid; q < XP_NCOUNT; q += B)
                    if (acc_cnt[q]) atomicAdd((unsigned long long*)&a.run_cnt[(size_t)r * XP_NCOUNT + q], acc_cnt[q]);
            if (a.run_led)
                for (int q = tid; q < XP_NLEDGER; q += B)
                    if (acc_led[q] != 0.0) atomicAdd(&a.run_led[(size_t)r * XP_NLEDGER + q], acc_led[q]);
        }
        for (int q = tid; q < XP_NCOUNT; q += B) acc_cnt[q] = 0;
        for (int q = tid; q < XP_NLEDGER; q += B) acc_led[q] = 0.0;
    };
    const int nitems = a.cell_list ? *a.cell_list_count : a.n_cells;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int cell = a.cell_list ? a.cell_list[item] : item;
        const bool done = step_cell<BlockTeam<B>, XV>(a, cell, S, L);
        __syncthreads();
        if (done) {
            const int run = a.cell_run[cell];
            if (run != acc_run) {
                flush();
                __syncthreads();
                if (tid == 0) acc_run = run;
            }
            for (int q = tid; q < XP_NCOUNT; q += B) acc_cnt[q] += (unsigned long long)S.cnt[q];
            for (int q = tid; q < XP_NLEDGER; q += B) acc_led[q] = acc_led[q] + S.led[q];
            if (tid == 0) {
                const int n = S.ints[6];
                if (n > acc_max) acc_max = n;
                const int bk = (n + 15) / 16;
                acc_hist[bk < 63 ? bk : 63] += 1;
            }
        }
        __syncthreads();
    }
    flush();
    if (a.stats) {
        if (tid == 0 && acc_max > 0) atomicMax(&a.stats[0], acc_max);
        for (int q = tid; q < 64; q += B)
            if (acc_hist[q]) atomicAdd(&a.stats[4 + q], acc_hist[q]);
    }
}

// Several small cells per wave: the wave is cut into 64 / W aligned groups of
// W lanes and every group steps its own cell with its own LDS plan (the same
// step, written against the group team).  Cells are taken G at a time; run
// records are summed per group and flushed like those of k_step.  Per-cell
// values differ between the groups of a wave, so they live in vector
// registers: two waves per SIMD, each carrying G cells.
template <int W, int XV>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_step_g(StepArgs a)
{
    constexpr int G = 64 / W;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ CellSharedT<1> S[G];
    __shared__ unsigned long long acc_cnt[G][XP_NCOUNT];
    __shared__ double acc_led[G][XP_NLEDGER];
    __shared__ int acc_run[G], acc_max[G];
    __shared__ int acc_hist[64];
    using T = GroupTeam<W>;
    const int g = threadIdx.x / W, t = threadIdx.x & (W - 1);
    const int ce = a.lds_ce, ci = a.lds_ci;
    const int ps = pow2_at_least(ce > ci ? ce : ci);
    const size_t cb = (step_lds_bytes_dev(ce, ci) + 15) & ~size_t(15);
    const Lds L = carve(smem + g * cb, ce, ci, ps);
    for (int q = threadIdx.x; q < 64; q += 64) acc_hist[q] = 0;
    for (int q = t; q < XP_NCOUNT; q += W) acc_cnt[g][q] = 0;
    for (int q = t; q < XP_NLEDGER; q += W) acc_led[g][q] = 0.0;
    if (t == 0) {
        acc_run[g] = -1;
        acc_max[g] = 0;
    }
    __syncthreads();
    auto flush = [&]() {
        const int r = acc_run[g];
        if (r >= 0) {
            if (a.run_cnt)
                for (int q = t; q < XP_NCOUNT; q += W)
                    if (acc_cnt[g][q]) atomicAdd((unsigned long long*)&a.run_cnt[(size_t)r * XP_NCOUNT + q], acc_cnt[g][q]);
            if (a.run_led)
                for (int q = t; q < XP_NLEDGER; q += W)
                    if (acc_led[g][q] != 0.0) atomicAdd(&a.run_led[(size_t)r * XP_NLEDGER + q], acc_led[g][q]);
        }
        for (int q = t; q < XP_NCOUNT; q += W) acc_cnt[g][q] = 0;
        for (int q = t; q < XP_NLEDGER; q += W) acc_led[g][q] = 0.0;
    };
    const int nitems = a.cell_list ? *a.cell_list_count : a.n_cells;
    for (int it = blockIdx.x; it * G < nitems; it += gridDim.x) {
        const int item = it * G + g;
        const int cell = item < nitems ? (a.cell_list ? a.cell_list[item] : item) : -1;
        const bool done = step_cell<T, XV>(a, cell, S[g], L);
        T::sync();
        if (done) {
            const int run = a.cell_run[cell];
            if (run != acc_run[g]) {
                flush();
                T::sync();
                if (t == 0) acc_run[g] = run;
            }
            for (int q = t; q < XP_NCOUNT; q += W) acc_cnt[g][q] += (unsigned long long)S[g].cnt[q];
            for (int q = t; q < XP_NLEDGER; q += W) acc_led[g][q] = acc_led[g][q] + S[g].led[q];
            if (t == 0) {
                const int n = S[g].ints[6];
                if (n > acc_max[g]) acc_max[g] = n;
                const int bk = (n + 15) / 16;
                atomicAdd(&acc_hist[bk < 63 ? bk : 63], 1);
            }
        }
        T::sync();
    }
    flush();
    __syncthreads();
    if (a.stats) {
        if (t == 0 && acc_max[g] > 0) atomicMax(&a.stats[0], acc_max[g]);
        if (threadIdx.x < 64 && acc_hist[threadIdx.x]) atomicAdd(&a.stats[4 + threadIdx.x], acc_hist[threadIdx.x]);
    }
}

// Random permutation of slots 0..n-1: out[k] = slot of rank k when the slots
// are sorted by (Philox word, slot); the word of slot i is word i % 4 of the
// call (c0, c1, i / 4, c3).  A team of up to 64 lanes sorts in registers,
// up to 8 keys per lane for a whole wave and 4 for a group: with up to 2 keys
// per lane every lane draws the Philox calls of its own keys; with more, each
// call is drawn once and its four keys pass through sbuf.  Larger cells use
// an LDS bitonic sort in sbuf (>= pow2(n) entries).  Out of line: the step
// calls it four times.
template <class T>
__device__ __noinline__ void make_perm_fn(int n, uint32_t c0, uint32_t c1, uint32_t c3, uint32_t k0,
                                          uint32_t k1, int32_t* out, uint64_t* sbuf)
{
    constexpr int W = T::N;
    const int tid = T::rank();
    constexpr int KMAX = W == 64 ? 8 : 4;
    auto keys_to_lds = [&]() {
        for (int g = tid; 4 * g < n; g += W) {
            const Words w = philox(c0, c1, (uint32_t)g, c3, k0, k1);
            const uint32_t k4[4] = {w.x0, w.x1, w.x2, w.x3};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * g + q;
                if (i < n) sbuf[i] = ((uint64_t)k4[q] << 32) | (uint32_t)i;
            }
        }
    };
    if (W <= 64 && n <= KMAX * W) {
        auto run_k = [&](auto kk) {
            constexpr int K = decltype(kk)::value;
            uint64_t key[K];
            if constexpr (K <= 2) {
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    const int i = tid + W * m;
                    key[m] = ~0ull;
                    if (i < n) {
                        const Words w = philox(c0, c1, (uint32_t)(i >> 2), c3, k0, k1);
                        const uint32_t q = i & 3;
                        const uint32_t kw = q == 0 ? w.x0 : (q == 1 ? w.x1 : (q == 2 ? w.x2 : w.x3));
                        key[m] = ((uint64_t)kw << 32) | (uint32_t)i;
                    }
                }
            } else {
                keys_to_lds();
                T::sync();
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    const int i = tid + W * m;
                    key[m] = i < n ? sbuf[i] : ~0ull;
                }
            }
            group_bitonic<W, K>(key);
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const int r = tid + W * m;
                if (r < n) out[r] = (int32_t)(uint32_t)key[m];
            }
        };
        if (n <= W) run_k(std::integral_constant<int, 1>{});
        else if (n <= 2 * W) run_k(std::integral_constant<int, 2>{});
        else if (n <= 4 * W) run_k(std::integral_constant<int, 4>{});
        else run_k(std::integral_constant<int, KMAX>{});
        T::sync();
        return;
    }
    const int p = pow2_at_least(n);
    keys_to_lds();
    for (int i = n + tid; i < p; i += W) sbuf[i] = ~0ull;
    T::sync();
    bitonic_sort<W>(sbuf, p);
    for (int k = tid; k < n; k += W) out[k] = (int32_t)(uint32_t)sbuf[k];
    T::sync();
}

// The first k ranks of the permutation of make_perm_fn (slots sorted by
// (Philox word, slot)), restricted to the slots with zq[i] > zf when zq is
// given: out[r] = slot of rank r for r < k.  k extractions of the smallest
// remaining key instead of a full sort, for the few recombinations of a step.
// The caller guarantees at least k admissible slots.
template <class T>
__device__ __noinline__ void smallest_fn(int n, int k, uint32_t c0, uint32_t c1, uint32_t c3, uint32_t k0,
                                         uint32_t k1, const uint8_t* zq, int zf, int32_t* out,
                                         uint64_t* sbuf, typename T::Shared& S)
{
    constexpr int W = T::N;
    const int tid = T::rank();
    for (int g = tid; 4 * g < n; g += W) {
        const Words w = philox(c0, c1, (uint32_t)g, c3, k0, k1);
        const uint32_t k4[4] = {w.x0, w.x1, w.x2, w.x3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * g + q;
            if (i < n) sbuf[i] = (zq && !((int)zq[i] > zf)) ? ~0ull : (((uint64_t)k4[q] << 32) | (uint32_t)i);
        }
    }
    T::sync();
    uint64_t last = 0;
    for (int r = 0; r < k; ++r) {
        uint64_t m = ~0ull;
        for (int i = tid; i < n; i += W) {
            const uint64_t v = sbuf[i];
            if ((r == 0 || v > last) && v < m) m = v;
        }
        m = T::umin(m, S);
        if (tid == 0) out[r] = (int32_t)(uint32_t)m;
        last = m;
    }
    T::sync();
}

// XP_KA_FIELD, at the commit of a cell: the K-alpha photons that found a bin
// (counter, lane 0) and the macro-photons returned per bin (d_cell_nka, zeros
// without the variant).  Out of line: the step calls it only with the variant
// or the array set.
__device__ __noinline__ void kalpha_record(const StepArgs& a, int cell, const xp_run* R, const DevTables* tb,
                                           const int* kz, int* cnt, int rank, int width)
{
    const bool on = (a.flags & XP_KA_FIELD) != 0;
    if (on && rank == 0)
        for (int z0 = 0; z0 < 13; ++z0)
            if (kz[z0] && kalpha_bin(R->hv, R->n_bins, tb->e_kalpha[z0]) >= 0) cnt[XP_C_KA_FIELD] += kz[z0];
    if (a.cell_nka)
        for (int q = rank; q < XP_MAX_BINS; q += width)
            a.cell_nka[(size_t)cell * XP_MAX_BINS + q] =
                on && q < R->n_bins ? kalpha_return(tb, R->hv, R->n_bins, kz, q) : 0.0;
}

// Recombinations of a step at most this many select their ions and electrons
// by extraction; more sort the whole permutation.
constexpr int REC_SELECT_MAX = 12;

// Steps one cell; true when its new state was committed (the caller then adds
// S.cnt / S.led to the run records and S.ints[6] holds its electron count).
template <class T, int XV>
__device__ bool step_cell(const StepArgs& a, int cell, typename T::Shared& S, const Lds& L)
{
    auto ka = step_args<T>(a);
    constexpr int B = T::N;
    const int tid = T::rank();
    if (cell < 0 || cell >= ka->n_cells) return false;
    const int run = ka->cell_run[cell];
    const xp_run* R = ka->runs + run;
    const DevTables* tb = ka->tab;
    const uint32_t lcell = (uint32_t)(cell - R->cell_begin);
    const uint32_t step = ka->d_step ? ka->d_step[run] : ka->step;
    const uint32_t key0 = (uint32_t)R->seed, key1 = (uint32_t)(R->seed >> 32);
    const uint32_t flags = ka->flags;
    const double w0 = R->w0, vol = R->volume, dt = R->dt;
    const double mi = tb->mass_ion;

    int ne = ka->e_cnt[cell];
    const int ecap = ka->e_cap[cell];
    const int ni = ka->i_cnt[cell];
    const int64_t eo = ka->e_off[cell], io = ka->i_off[cell];
    const int ce = ka->lds_ce, ci = ka->lds_ci;
    // the LDS plan of this launch bounds the cell; a cell beyond it is passed to
    // the next (larger) plan, a cell beyond its slab capacity is an error
    const int lim = ecap < ce ? ecap : ce;

    // beyond every LDS plan: hand the cell to the global-memory path
    auto to_big = [&]() {
        if (tid == 0) {
            if (ka->big_out) {
                const int k = atomicAdd(ka->big_out_count, 1);
                if (k < ka->big_out_cap) ka->big_out[k] = cell;
                else flag_status(a, run, XP_ST_CAPACITY);
            } else {
                flag_status(a, run, XP_ST_CAPACITY);
            }
        }
    };
    auto defer = [&]() {
        if (!ka->defer_out) {
            to_big();
            return;
        }
        if (tid == 0) {
            const int k = atomicAdd(ka->defer_out_count, 1);
            ka->defer_out[k] = cell;
            if (ka->stats) atomicAdd(&ka->stats[1], 1);
        }
    };
    if (ni > ci) {
        defer();
        return false;
    }
    if (ne > ce || ne > ecap) {
        if (ne > ecap) {
            if (tid == 0) flag_status(a, run, XP_ST_CAPACITY);
        } else {
            defer();
        }
        return false;
    }

    auto rng = [&](uint32_t idx, uint32_t purpose, uint32_t sub) {
        return philox(step, lcell, idx, (purpose << 24) | sub, key0, key1);
    };

    for (int j = tid; j < ne; j += B) {
        L.evx[j] = ka->evx[eo + j];
        L.evy[j] = ka->evy[eo + j];
        L.evz[j] = ka->evz[eo + j];
        L.ew[j] = ka->ew[eo + j];
        L.eorg[j] = j;
    }
    for (int j = tid; j < ni; j += B) {
        L.ivx[j] = ka->ivx[io + j];
        L.ivy[j] = ka->ivy[io + j];
        L.ivz[j] = ka->ivz[io + j];
        L.iz[j] = ka->iz[io + j];
        L.ik[j] = ka->ik[io + j];
        L.fwok[j] = 0;
    }
    for (int q = tid; q < XP_NCOUNT; q += B) S.cnt[q] = 0;
    if (XV) {
        for (int q = tid; q < XP_MAX_BINS; q += B) S.nabs[q] = 0;
        for (int q = tid; q < 14; q += B) S.kz[q] = 0;
    }
    for (int q = tid; q < XP_NLEDGER; q += B) S.led[q] = 0.0;
    for (int q = tid; q < XP_NMOM; q += B) S.mom[q] = 0.0;
    for (int q = tid; q < 8; q += B) S.ints[q] = 0;
    T::sync();

    // ---------------- S0: moments and continuum lowering -----------------
    ka = step_args<T>(a);
    const double ebulk = R->e_bulk;
    auto kin = [&](int j) {
        const double x = L.evx[j], y = L.evy[j], z = L.evz[j];
        return HALF_ME_OVER_QE * ((x * x + y * y) + z * z);
    };
    auto moments_bulk = [&](int n, long long* we, long long& wb, double& ke) {
        long long w_loc = 0, b_loc = 0;
        for (int j = tid; j < n; j += B) {
            const long long w = L.ew[j];
            w_loc += w;
            if (kin(j) < ebulk) b_loc += w;
        }
        if (we) *we = T::isum(w_loc, S);
        wb = T::isum(b_loc, S);
        ke = T::tree(n, [&](int j) {
            const double e = kin(j);
            return e < ebulk ? (double)L.ew[j] * e : 0.0;
        }, S);
    };
    auto ion_sums = [&](long long& sz, long long& sz2) {
        long long s1 = 0, s2 = 0;
        for (int j = tid; j < ni; j += B) {
            const long long z = L.iz[j];
            s1 += z;
            s2 += z * z;
        }
        sz = T::isum(s1, S);
        sz2 = T::isum(s2, S);
    };

    long long we, wb, sz, sz2;
    double ke;
    moments_bulk(ne, &we, wb, ke);
    ion_sums(sz, sz2);
    long long s3_accepted = 0;   // charge added by S3 (one per accepted ionization)
    const long long wi = ni;
    double tmp = 0.01;
    if (wb > 0) {
        tmp = (2.0 * ke) / (3.0 * (double)wb);
        if (tmp < 0.01) tmp = 0.01;
    }
    const double t_e = tmp;
    const double n_e = ((double)we * w0) / vol;
    const double n_i = ((double)wi * w0) / vol;
    const double zbar = wi > 0 ? (double)sz / (double)wi : 0.0;
    const double zstar = sz > 0 ? (double)sz2 / (double)sz : 0.0;
    for (int z = tid; z < 13; z += B) S.mom[16 + z] = ipd(R->ipd_model, z, t_e, n_e, n_i, zbar, zstar);
    if (tid == 13 % B)
        S.mom[10] = R->lnl_fixed > 0.0 ? R->lnl_fixed : coulomb_log(t_e, n_e, zbar);
    if (tid == 0) {
        S.mom[0] = (double)we; S.mom[1] = (double)wi; S.mom[2] = (double)sz;
        S.mom[3] = (double)sz2; S.mom[4] = ke; S.mom[5] = t_e; S.mom[6] = n_e;
        S.mom[7] = n_i; S.mom[8] = zbar; S.mom[9] = zstar;
    }
    T::sync();
    const double* dE = S.mom + 16;
    const double lnl = S.mom[10];

    // ------------- random permutations: sort (Philox key, slot) ---------------
    auto make_perm = [&](uint32_t purpose, int n, int32_t* out) {
        make_perm_fn<T>(n, step, lcell, purpose << 24, key0, key1, out, L.sbuf);
    };

    const double fe_ei = mi / (ME + mi);   // electron side of an e-i pair
    const double fi_ei = ME / (ME + mi);   // ion side
    const double f_ee = ME / (ME + ME);
    const double qe4 = (QE * QE) * (QE * QE);

    // ---------------- S1, S2: binary collisions ----------------
    ka = step_args<T>(a);
    // Every collision of the step goes through one call site (the scattering
    // is the largest code of the step).  Phase 0 is e-e: with an odd count
    // >= 3, item 0 is the triplet (three collisions in sequence at dt/2), the
    // other items are adjacent pairs of the permutation.  Phase 1 is e-i:
    // round robin over the smaller population, round by round.
    const bool do_ee = (flags & XP_EE) && ne >= 2;
    // scattering law bits: 1 Nanbu (else Takizuka-Abe), 2 relativistic (both
    // only in the instances that carry the variants' code)
    const int law = XV == 2 ? ((flags & XP_NANBU) ? 1 : 0)
                  : (XV == 3 ? (((flags & XP_NANBU) ? 1 : 0) | 2) : 0);
    const bool do_ei = (flags & XP_EI) && ne >= 1 && ni >= 1;
    if ((flags & (XP_EE | XP_EI)) && ne >= 1 && (ne >= 2 || ni >= 1)) make_perm(RP_PERM_E, ne, L.perm_e);
    const double mee = (ME * ME) / (ME + ME);
    const double kee = qe4 / (((8.0 * PI) * (EPS0 * EPS0)) * (mee * mee));
    const double afull = (kee * lnl) * dt;
    const double ahalf = (kee * lnl) * (0.5 * dt);
    const int start = (ne % 2 == 1 && ne >= 3) ? 3 : 0;
    const int tri = start == 3 ? 1 : 0;
    const int npairs = (ne - start) / 2;
    const double mei = (ME * mi) / (ME + mi);
    const double kei = qe4 / (((8.0 * PI) * (EPS0 * EPS0)) * (mei * mei));
    const double a1 = (kei * lnl) * dt;
    const int nmin = ne < ni ? ne : ni, nmax = ne < ni ? ni : ne;
#pragma unroll 1
    for (int phase = 0; phase < 2; ++phase) {
        const bool ion = phase == 1;
        if (ion ? !do_ei : !do_ee) continue;
        if (ion) make_perm(RP_PERM_I, ni, L.perm_i);
        double* bvx = ion ? L.ivx : L.evx;
        double* bvy = ion ? L.ivy : L.evy;
        double* bvz = ion ? L.ivz : L.evz;
        const double fa = ion ? fe_ei : f_ee, fb = ion ? fi_ei : f_ee;
        const double nunit = (w0 * (double)(ion ? nmin : ne)) / vol;
        const int items = ion ? nmax : npairs + tri;
        const int per_round = ion ? nmin : items;
#pragma unroll 1
        for (int r0 = 0; r0 < items; r0 += per_round) {
            const int r1 = r0 + per_round < items ? r0 + per_round : items;
            for (int k = r0 + tid; k < r1; k += B) {
                const int nsub = (!ion && tri && k == 0) ? 3 : 1;
#pragma unroll 1
                for (int sub = 0; sub < nsub; ++sub) {
                    int e, bb;
                    uint32_t wb, idx, purpose;
                    double coef;
                    if (ion) {
                        if (ne >= ni) { e = L.perm_e[k]; bb = L.perm_i[k % ni]; }
                        else          { bb = L.perm_i[k]; e = L.perm_e[k % ne]; }
                        const int z = L.iz[bb];
                        if (z == 0) continue;
                        coef = a1 * (double)(z * z);
                        wb = 1u;
                        idx = (uint32_t)k;
                        purpose = RP_EI;
                    } else if (nsub == 3) {
                        e = L.perm_e[sub];
                        bb = L.perm_e[sub == 2 ? 0 : sub + 1];
                        coef = ahalf;
                        wb = L.ew[bb];
                        idx = (uint32_t)sub;
                        purpose = RP_EE_TRI;
                    } else {
                        const int j = k - tri;
                        e = L.perm_e[start + 2 * j];
                        bb = L.perm_e[start + 2 * j + 1];
                        coef = afull;
                        wb = L.ew[bb];
                        idx = (uint32_t)j;
                        purpose = RP_EE;
                    }
                    collide_slots(L.evx, L.evy, L.evz, L.ew, bvx, bvy, bvz, e, bb, wb, fa, fb, coef, nunit,
                                  step, lcell, idx, purpose << 24, key0, key1, S.cnt, law, ME, ion ? mi : ME);
                }
            }
            T::sync();
        }
        if (tid == 0) {
            if (ion) {
                S.cnt[XP_C_EI] += nmax;
            } else {
                S.cnt[XP_C_EE] += npairs;
                S.cnt[XP_C_TRIPLET] += 3 * tri;
            }
        }
    }

    bool overflow = false, deferred = false;

    // ---------------- S3: collisional ionization ----------------
    ka = step_args<T>(a);
    if ((flags & XP_ION) && ne >= 1 && ni >= 1) {
        // charge states are unchanged since the moments: reuse their sum
        const int zc = (int)((2 * sz + wi) / (2 * wi));
        const int ne0 = ne;
        // the charge states whose cross section is evaluated: the average
        // cell ion Z_c, or (XP_ION_Z) every state an ion of the cell holds
        const bool perz = XV && (flags & XP_ION_Z) != 0;
        if (perz) {
            uint32_t ml = 0;
            for (int i = tid; i < ni; i += B)
                if (L.iz[i] < 13) ml |= 1u << L.iz[i];
            if (ml) atomicOr((unsigned*)&S.ints[2], ml);
            T::sync();
        }
        const uint32_t zmask = perz ? (uint32_t)S.ints[2] : (zc < 13 ? 1u << zc : 0u);
        if (tid == 0) S.mom[11] = perz ? (double)__popc(zmask) : (double)zc;
        if (zmask) {
            double pmax = 0.0, pavg = 0.0;
#pragma unroll 1
            for (int z = 0; z < 13; ++z) {
                if (!(zmask & (1u << z))) continue;
                const Occ oc = occupancy(z, 0);
                double pp[5], lnp[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const double raw = tb->bind[z][q] - dE[z];
                    pp[q] = raw < 1.0 ? 1.0 : raw;
                    if (tid == 0 && oc.s[q] > 0 && raw < 1.0) S.cnt[XP_C_IPD_CLAMPED] += 1;
                }
                // the logarithms of the occupied subshells' lowered bindings, one
                // subshell per thread, shared through LDS
                if (tid < 5) {
                    double arg = pp[0];
                    int occ = oc.s[0];
#pragma unroll
                    for (int q = 1; q < 5; ++q)
                        if (tid == q) { arg = pp[q]; occ = oc.s[q]; }
                    S.lnp[tid] = occ > 0 ? xlog(arg) : 0.0;
                }
                T::sync();
#pragma unroll
                for (int q = 0; q < 5; ++q) lnp[q] = S.lnp[q];
                double pmin = __builtin_inf();
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    if (oc.s[q] > 0 && pp[q] < pmin) pmin = pp[q];
                const double ssum = T::tree(ne0, [&](int j) {
                    return lotz_leaf(L.evx[j], L.evy[j], L.evz[j], L.ew[j], oc.s, pp, lnp, pmin, tb);
                }, S);
                double p = ((ssum * w0) * dt) / vol;
                if (p > 1.0) {
                    p = 1.0;
                    if (tid == 0) S.cnt[XP_C_P_CLAMPED] += 1;
                }
                if (perz && tid == 0) S.pz[z] = p;
                if (p > pmax) pmax = p;
                pavg = p;
            }
            if (tid == 0) S.mom[12] = pmax;
            if (perz) T::sync();
            const int nfired = T::select(
                ni,
                [&](int i) {
                    if (L.iz[i] >= 13) return false;
                    const double p = perz ? S.pz[L.iz[i]] : pavg;
                    if (!(p > 0.0)) return false;
                    const Words d = rng((uint32_t)i, RP_ION, 0);
                    L.fw[3 * i] = d.x1;
                    L.fw[3 * i + 1] = d.x2;
                    L.fw[3 * i + 2] = d.x3;
                    L.fwok[i] = 1;
                    return u32(d.x0) < p;
                },
                [&](int i, int pos) { L.list[pos] = i; }, S);
            if (tid == 0) S.cnt[XP_C_ION_FIRED] += nfired;
            T::sync();
            if (nfired > 0) {
                long long ws_loc = 0;
                for (int j = tid; j < ne0; j += B) ws_loc += L.ew[j];
                const long long ws = T::isum(ws_loc, S);
                const double ux = T::tree(ne0, [&](int j) { return (double)L.ew[j] * L.evx[j]; }, S) / (double)ws;
                const double uy = T::tree(ne0, [&](int j) { return (double)L.ew[j] * L.evy[j]; }, S) / (double)ws;
                const double uz = T::tree(ne0, [&](int j) { return (double)L.ew[j] * L.evz[j]; }, S) / (double)ws;
                const double kth = T::tree(ne0, [&](int j) {
                    const double dx = L.evx[j] - ux, dy = L.evy[j] - uy, dz = L.evz[j] - uz;
                    return (double)L.ew[j] * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
                }, S);
                if (tid == 0) {
                    S.mom[13] = kth;
                    double debit = 0.0;
                    int acc = 0;
                    for (int q = 0; q < nfired; ++q) {
                        const int i = L.list[q];
                        const int z = L.iz[i], kv = L.ik[i];
                        const int sv = valence(z, kv);
                        const double ip = lowered(tb, z, sv, dE);
                        if (!(debit + ip <= kth)) break;
                        const int slot = ne0 + acc;
                        if (slot >= lim) {
                            S.ints[0] = slot >= ecap ? 1 : 2;   // 1 over capacity, 2 over the LDS plan
                            break;
                        }
                        debit = debit + ip;
                        L.iz[i] = (uint8_t)(z + 1);
                        if (sv == 0) L.ik[i] = (uint8_t)(kv + 1);
                        L.evx[slot] = 0.0; L.evy[slot] = 0.0; L.evz[slot] = 0.0;
                        L.ew[slot] = 1;
                        L.eorg[slot] = -1 - i;
                        S.led[XP_L_ION_DEBIT] += ip;
                        ++acc;
                    }
                    S.cnt[XP_C_ION_ACCEPTED] += acc;
                    S.cnt[XP_C_ION_STARVED] += nfired - acc;
                    S.cnt[XP_C_E_NEW] += acc;
                    S.mom[14] = debit;
                    S.dbl[0] = debit;
                    S.ints[1] = acc;
                }
                T::sync();
                if (S.ints[0] == 1) overflow = true;
                if (S.ints[0] == 2) deferred = true;
                const double debit = S.dbl[0];
                const int acc = S.ints[1];
                s3_accepted = acc;
                if (debit > 0.0) {
                    const double alpha = sqrt(1.0 - debit / kth);
                    for (int j = tid; j < ne0; j += B) {
                        L.evx[j] = ux + alpha * (L.evx[j] - ux);
                        L.evy[j] = uy + alpha * (L.evy[j] - uy);
                        L.evz[j] = uz + alpha * (L.evz[j] - uz);
                    }
                }
                ne = ne0 + acc;
                T::sync();
            }
        }
    }

    // ---------------- S4: three-body recombination ----------------
    ka = step_args<T>(a);
    if (!overflow && !deferred && (flags & XP_REC) && ne >= 1 && ni >= 1) {
        // charge states changed only by S3 since the moments
        const long long szr = sz + s3_accepted;
        long long wbr;
        double ker;
        moments_bulk(ne, nullptr, wbr, ker);
        double tp = 0.01;
        if (wbr > 0) {
            tp = (2.0 * ker) / (3.0 * (double)wbr);
            if (tp < 0.01) tp = 0.01;
        }
        if (tid == 0) S.mom[15] = tp;
        // Zbar_EOS: its two logarithms on two threads, shared through LDS
        if (tid < 2) S.dbl[2 + tid] = xlog(tid == 0 ? n_i : tp);
        T::sync();
        const int zf = R->z_floor;
        long long nrec = 0;
        bool ions_listed = false;
        if (XV && (flags & XP_REC_XS)) {
            // per ion from its own charge state's rate (detailed balance with
            // the Lotz ionization) at the temperature and electron density
            // after S3; the firing ions recombine in slot order, at most one
            // per electron
            long long wel = 0;
            for (int j = tid; j < ne; j += B) wel += L.ew[j];
            const long long we4 = T::isum(wel, S);
            const double ne4 = ((double)we4 * w0) / vol;
            uint32_t ml = 0;
            for (int i = tid; i < ni; i += B) ml |= 1u << L.iz[i];
            if (ml) atomicOr((unsigned*)&S.ints[3], ml);
            T::sync();
            const uint32_t held = (uint32_t)S.ints[3];
            for (int z = tid; z < 14; z += B) {
                double pz = 0.0;
                if ((held & (1u << z)) && z > zf && z >= 1) {
                    pz = rec_xs_prob(tb, z, tp, ne4, dE, dt);
                    if (pz > 1.0) {
                        pz = 1.0;
                        atomicAdd(&S.cnt[XP_C_P_CLAMPED], 1);
                    }
                }
                S.prz[z] = pz;
            }
            T::sync();
            const int nf = T::select(
                ni,
                [&](int i) {
                    const int z = L.iz[i];
                    if (z <= zf || !(S.prz[z] > 0.0)) return false;
                    return u32(rng((uint32_t)i, RP_REC_XS, 0).x0) < S.prz[z];
                },
                [&](int i, int pos) {
                    if (pos < ne) L.list[pos] = i;
                },
                S);
            nrec = nf < ne ? nf : ne;
            ions_listed = true;
        } else {
            const double zeos = eos_zbar_ln(tb, S.dbl[2], S.dbl[3]);
            const double dd = (double)szr - (double)ni * zeos;
            if (dd > 0.0) {
                nrec = (long long)floor(dd + 0.5);
                long long el = 0;
                for (int j = tid; j < ni; j += B) el += L.iz[j] > zf ? 1 : 0;
                const long long nelig = T::isum(el, S);
                if (nrec > nelig) nrec = nelig;
                if (nrec > ne) nrec = ne;
            }
        }
        {
            if (nrec > 0) {
                const int nr = (int)nrec;
                if (ions_listed) {
                    // the first nr electrons of the REC_E order
                    if (nr <= REC_SELECT_MAX)
                        smallest_fn<T>(ne, nr, step, lcell, RP_REC_E << 24, key0, key1, nullptr, 0, L.perm_e,
                                       L.sbuf, S);
                    else
                        make_perm(RP_REC_E, ne, L.perm_e);
                } else if (nr <= REC_SELECT_MAX) {
                    // the first nr eligible ions of the REC_I order and the
                    // first nr electrons of the REC_E order
                    smallest_fn<T>(ni, nr, step, lcell, RP_REC_I << 24, key0, key1, L.iz, zf, L.list, L.sbuf, S);
                    smallest_fn<T>(ne, nr, step, lcell, RP_REC_E << 24, key0, key1, nullptr, 0, L.perm_e,
                                   L.sbuf, S);
                } else {
                    make_perm(RP_REC_I, ni, L.perm_i);
                    make_perm(RP_REC_E, ne, L.perm_e);
                    T::select(
                        ni, [&](int q) { return (int)L.iz[L.perm_i[q]] > zf; },
                        [&](int q, int pos) {
                            if (pos < nr) L.list[pos] = L.perm_i[q];
                        },
                        S);
                }
                for (int j = tid; j < ne; j += B) L.esel[j] = 0;
                T::sync();
                for (int t = tid; t < nr; t += B) L.esel[L.perm_e[t]] = 1;
                T::sync();
                auto wp = [&](int j) { return (long long)L.ew[j] - (long long)L.esel[j]; };
                long long wsl = 0;
                for (int j = tid; j < ne; j += B) wsl += wp(j);
                const long long ws = T::isum(wsl, S);
                double ux = 0.0, uy = 0.0, uz = 0.0, kth = 0.0;
                if (ws != 0) {
                    ux = T::tree(ne, [&](int j) { return (double)wp(j) * L.evx[j]; }, S) / (double)ws;
                    uy = T::tree(ne, [&](int j) { return (double)wp(j) * L.evy[j]; }, S) / (double)ws;
                    uz = T::tree(ne, [&](int j) { return (double)wp(j) * L.evz[j]; }, S) / (double)ws;
                    kth = T::tree(ne, [&](int j) {
                        const double dx = L.evx[j] - ux, dy = L.evy[j] - uy, dz = L.evz[j] - uz;
                        return (double)wp(j) * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
                    }, S);
                }
                if (ws == 0 || !(kth > 0.0)) {
                    if (tid == 0) S.cnt[XP_C_REC_SKIPPED] += 1;
                } else {
                    if (tid == 0) {
                        const double half_mi = (0.5 * mi) / QE;
                        const double ratio = ME / mi;
                        double eadd = 0.0;
                        for (int t = 0; t < nr; ++t) {
                            const int e = L.perm_e[t], i = L.list[t];
                            const double keu = kin(e);
                            const double v2b = (L.ivx[i] * L.ivx[i] + L.ivy[i] * L.ivy[i]) + L.ivz[i] * L.ivz[i];
                            const double kib = half_mi * v2b;
                            L.ivx[i] = L.ivx[i] + ratio * L.evx[e];
                            L.ivy[i] = L.ivy[i] + ratio * L.evy[e];
                            L.ivz[i] = L.ivz[i] + ratio * L.evz[e];
                            const double v2a = (L.ivx[i] * L.ivx[i] + L.ivy[i] * L.ivy[i]) + L.ivz[i] * L.ivz[i];
                            const double kia = half_mi * v2a;
                            const int z = L.iz[i], kv = L.ik[i];
                            const Occ o0 = occupancy(z, kv);
                            const int kn = (kv >= 1 && o0.s[1] + o0.s[2] == 8) ? kv - 1 : kv;
                            const Occ o1 = occupancy(z - 1, kn);
                            int sl = 0;
                            for (int q = 0; q < 5; ++q)
                                if (o1.s[q] > o0.s[q]) { sl = q; break; }
                            const double ipr = lowered(tb, z - 1, sl, dE);
                            L.iz[i] = (uint8_t)(z - 1);
                            L.ik[i] = (uint8_t)kn;
                            eadd = eadd + ((keu + ipr) + (kib - kia));
                            S.led[XP_L_REC_BIND] += ipr;
                        }
                        S.cnt[XP_C_REC] += nr;
                        S.led[XP_L_REC_ADD] += eadd;
                        S.dbl[1] = eadd;
                    }
                    T::sync();
                    const double alpha = sqrt(1.0 + S.dbl[1] / kth);
                    for (int j = tid; j < ne; j += B) {
                        const long long w2 = wp(j);
                        if (w2 > 0) {
                            L.evx[j] = ux + alpha * (L.evx[j] - ux);
                            L.evy[j] = uy + alpha * (L.evy[j] - uy);
                            L.evz[j] = uz + alpha * (L.evz[j] - uz);
                        }
                        L.ew[j] = (uint32_t)(w2 > 0 ? w2 : 0);
                    }
                    T::sync();
                    // stable compaction of the electrons whose weight reached 0,
                    // chunk by chunk (positions only move down)
                    int out = 0;
                    for (int c0 = 0; c0 < ne; c0 += B) {
                        const int j = c0 + tid;
                        const bool alive = j < ne && L.ew[j] > 0;
                        double vx = 0, vy = 0, vz = 0;
                        uint32_t w = 0;
                        int32_t org = 0;
                        if (alive) {
                            vx = L.evx[j]; vy = L.evy[j]; vz = L.evz[j];
                            w = L.ew[j]; org = L.eorg[j];
                        }
                        int dst = 0;
                        const int tot = T::select(
                            (c0 + B < ne ? B : ne - c0),
                            [&](int q) { return L.ew[c0 + q] > 0; },
                            [&](int q, int pos) { (void)q; dst = pos; }, S);
                        T::sync();
                        if (alive) {
                            const int d = out + dst;
                            L.evx[d] = vx; L.evy[d] = vy; L.evz[d] = vz;
                            L.ew[d] = w; L.eorg[d] = org;
                        }
                        out += tot;
                        T::sync();
                    }
                    if (tid == 0) S.cnt[XP_C_E_REMOVED] += ne - out;
                    ne = out;
                }
                T::sync();
            }
        }
    }

    // ---------------- S5: K-vacancy decay and photoionization ----------------
    ka = step_args<T>(a);
    if (!overflow && !deferred && (flags & (XP_PHOTO | XP_DECAY))) {
        const int nb = R->n_bins;
        const bool photo = (flags & XP_PHOTO) && nb > 0;
        const double* nhv = (XV && R->field_per_cell && ka->cell_nhv) ? ka->cell_nhv + (size_t)cell * XP_MAX_BINS : R->nhv;
        const double dtr = R->dt_rad;
        if (photo) {
            const double* rs = ka->run_sig + (size_t)run * (XP_MAX_BINS * 3);
            for (int q = tid; q < 3 * nb; q += B) S.sig[q / 3][q % 3] = rs[q];
            T::sync();
            for (int q = tid; q < 39; q += B) {
                const int z = q / 3, s = q % 3;
                const double pp = lowered(tb, z, s, dE);
                double acc = 0.0;
                for (int bq = 0; bq < nb; ++bq)
                    if (R->hv[bq] >= pp) acc = acc + nhv[bq] * S.sig[bq][s];
                S.ssum[z][s] = acc;
            }
            T::sync();
        }
        // pass 1: decisions per ion from its pre-S5 state
        for (int i = tid; i < ni; i += B) {
            const int z0 = L.iz[i], k0 = L.ik[i];
            L.z0[i] = (uint8_t)z0;
            L.k0[i] = (uint8_t)k0;
            uint8_t mask = 0;
            uint16_t bins = 0;
            uint32_t pf = 0, dec = 0;
            if (z0 < 13) {
                const Occ o0 = occupancy(z0, k0);
                const int nl0 = o0.s[1] + o0.s[2];
                int z = z0, kv = k0;
                if ((flags & XP_DECAY) && k0 >= 1 && nl0 >= 1) {
                    const double ga = tb->gamma_a[z0][k0], gx = tb->gamma_x[z0][k0];
                    const double rate = ga + gx;
                    if (rate > 0.0) {
                        const Words d = rng((uint32_t)i, RP_DECAY, 0);
                        double pd = dtr * rate;
                        if (pd > 1.0) {
                            pd = 1.0;
                            atomicAdd(&S.cnt[XP_C_P_CLAMPED], 1);
                        }
                        if (u52(d.x0, d.x1) < pd) {
                            kv = k0 - 1;
                            dec = 1;
                            atomicAdd(&S.cnt[XP_C_DECAY], 1);
                            if (nl0 >= 2 && u52(d.x2, d.x3) < ga / rate) {
                                z = z0 + 1;
                                mask |= 1;
                                atomicAdd(&S.cnt[XP_C_AUGER], 1);
                            } else {
                                atomicAdd(&S.cnt[XP_C_KALPHA], 1);
                                atomicAdd(&S.led[XP_L_KALPHA], tb->e_kalpha[z0]);
                                if (XV && (flags & XP_KA_FIELD)) atomicAdd(&S.kz[z0], 1);
                            }
                        }
                    }
                }
                if (photo) {
                    uint32_t fire[3];
                    if (L.fwok[i]) {
                        fire[0] = L.fw[3 * i];
                        fire[1] = L.fw[3 * i + 1];
                        fire[2] = L.fw[3 * i + 2];
                    } else {
                        const Words d = rng((uint32_t)i, RP_ION, 0);
                        fire[0] = d.x1;
                        fire[1] = d.x2;
                        fire[2] = d.x3;
                    }
                    for (int s = 0; s < 3; ++s) {
                        if (o0.s[s] <= 0) continue;
                        const double sum = S.ssum[z0][s];
                        if (!(sum > 0.0)) continue;
                        double p = ((CLIGHT * dtr) * (double)o0.s[s]) * sum;
                        if (p > 1.0) {
                            p = 1.0;
                            atomicAdd(&S.cnt[XP_C_P_CLAMPED], 1);
                        }
                        if (!(u32(fire[s]) < p)) continue;
                        pf |= 1u << s;
                        const Occ on = occupancy(z, kv);
                        if (z >= 13 || on.s[s] <= 0) {
                            atomicAdd(&S.cnt[XP_C_PHOTO_SKIPPED], 1);
                            continue;
                        }
                        const double pp = lowered(tb, z0, s, dE);
                        const Words d = rng((uint32_t)i, RP_BIN, (uint32_t)s);
                        const int sel = photo_bin(R->hv, nhv, S.sig, nb, s, pp, u52(d.x0, d.x1) * sum);
                        z = z + 1;
                        if (s == 0) kv = kv + 1;
                        mask |= (uint8_t)(2u << s);
                        bins |= (uint16_t)(sel << (4 * s));
                        atomicAdd(&S.cnt[XP_C_PHOTO_1S + s], 1);
                    }
                }
                L.iz[i] = (uint8_t)z;
                L.ik[i] = (uint8_t)kv;
            }
            // bits 0..3 the emissions; with XP_PHOTO_FRAC bits 4..6 the photo
            // candidates and bit 7 a decay, for the budget walk below
            if (XV && (flags & XP_PHOTO_FRAC)) {
                mask |= (uint8_t)((pf << 4) | (dec << 7));
                if (pf) atomicAdd(&S.ints[5], __popc(pf));
            }
            L.emask[i] = mask;
            L.ebins[i] = bins;
        }
        T::sync();
        if (XV && photo && (flags & XP_PHOTO_FRAC)) {
            // a bin gives the cell no more macro-photons than it holds: when
            // the candidates outnumber the smallest whole budget, one lane
            // takes the ions again in slot order
            if (tid == 0) {
                double mmin = 1e300;
                for (int bq = 0; bq < nb; ++bq) {
                    const double m = (nhv[bq] * R->volume) / R->w0;
                    S.pbud[bq] = m;
                    S.pused[bq] = 0.0;
                    if (nhv[bq] > 0.0 && floor(m) < mmin) mmin = floor(m);
                }
                if ((double)S.ints[5] > mmin) {
                    int dn[3] = {0, 0, 0}, dskip = 0, dst = 0, dpart = 0;
                    for (int i = 0; i < ni; ++i) {
                        const uint32_t em = L.emask[i];
                        const uint32_t pfi = (em >> 4) & 7u;
                        if (!pfi) continue;
                        const int z0 = L.z0[i], k0 = L.k0[i];
                        int z = z0 + (int)(em & 1u), kv = k0 - (int)(em >> 7);
                        const PhotoWalk w = photo_walk_ion(
                            [&](uint32_t pu, uint32_t sub) { return rng((uint32_t)i, pu, sub); }, tb, R->hv, nhv,
                            S.sig, S.ssum, nb, z0, pfi, dE, S.pbud, S.pused, z, kv);
                        int old = 0;
                        for (int q = 0; q < 3; ++q) {
                            const int f = (int)((em >> (1 + q)) & 1u);
                            dn[q] += w.fired[q] - f;
                            old += f;
                        }
                        dskip += w.skipped - (__popc(pfi) - old);
                        dst += w.starved;
                        dpart += w.partial;
                        L.emask[i] = (uint8_t)((em & 0xF1u) | w.mask);
                        L.ebins[i] = (uint16_t)w.bins;
                        L.iz[i] = (uint8_t)z;
                        L.ik[i] = (uint8_t)kv;
                    }
                    for (int q = 0; q < 3; ++q) S.cnt[XP_C_PHOTO_1S + q] += dn[q];
                    S.cnt[XP_C_PHOTO_SKIPPED] += dskip;
                    S.cnt[XP_C_PHOTO_STARVED] += dst;
                    S.cnt[XP_C_PHOTO_PARTIAL] += dpart;
                }
            }
            T::sync();
        }

        // pass 2: new electrons in ion-slot order (Auger, photo 1s, 2s, 2p)
        int base_pos = ne;
        for (int c0 = 0; c0 < ni; c0 += B) {
            const int i = c0 + tid;
            const int cnt = i < ni ? __popc((unsigned)L.emask[i] & 15u) : 0;
            // exclusive prefix of cnt over the chunk (slot order)
            int tot;
            const int before = T::prefix(cnt, tot, S);
            int pos = base_pos + before;
            if (cnt > 0) {
                const int z0 = L.z0[i], k0 = L.k0[i];
                const Occ o0 = occupancy(z0, k0);
                const uint8_t mask = L.emask[i] & 15u;
                for (int bit = 0; bit < 4; ++bit) {
                    if (!(mask & (1u << bit))) continue;
                    double en;
                    if (bit == 0) {
                        const int nl0 = o0.s[1] + o0.s[2];
                        const double p2s = lowered(tb, z0, 1, dE);
                        const double p2p = lowered(tb, z0, 2, dE);
                        const double num = (double)o0.s[1] * p2s + (double)o0.s[2] * p2p;
                        en = tb->e_kalpha[z0] - num / (double)nl0;
                        if (en < 0.0) en = 0.0;
                        atomicAdd(&S.led[XP_L_AUGER_E], en);
                    } else {
                        const int s = bit - 1;
                        const int sel = (L.ebins[i] >> (4 * s)) & 15;
                        en = R->hv[sel] - lowered(tb, z0, s, dE);
                        atomicAdd(&S.led[XP_L_PHOTO_E], en);
                        atomicAdd(&S.led[XP_L_PHOTON_ABS], R->hv[sel]);
                        if (XV) atomicAdd(&S.nabs[sel], 1);
                    }
                    if (pos < lim) {
                        const Words d = rng((uint32_t)i, RP_DIR, (uint32_t)bit);
                        const double mu = 2.0 * u52(d.x0, d.x1) - 1.0;
                        double sp, cp;
                        xsincos2pi((((uint64_t)d.x2 << 32) | d.x3) >> 12, sp, cp);
                        const double st = sqrt(1.0 - mu * mu);
                        const double sv = sqrt(en * TWO_QE_OVER_ME);
                        L.evx[pos] = sv * (st * cp);
                        L.evy[pos] = sv * (st * sp);
                        L.evz[pos] = sv * mu;
                        L.ew[pos] = 1;
                        L.eorg[pos] = -1 - i;
                    }
                    ++pos;
                }
            }
            base_pos += tot;
            T::sync();
        }
        if (tid == 0) S.cnt[XP_C_E_NEW] += base_pos - ne;
        if (base_pos > ecap) overflow = true;
        else if (base_pos > lim) deferred = true;
        ne = base_pos;
        T::sync();
    }

    // ------------- forced thermalization (variant, Sec. VI.C) -------------
    if (XV && !overflow && !deferred && (flags & XP_THERM)) {
        long long wl = 0;
        for (int j = tid; j < ne; j += B) wl += L.ew[j];
        const long long ws = T::isum(wl, S);
        bool kept = ne < 2 || ws <= 0;
        if (!kept) {
            const double w = (double)ws;
            auto wsum = [&](const double* v) {
                return T::tree(ne, [&](int j) { return (double)L.ew[j] * v[j]; }, S);
            };
            const double kall = T::tree(ne, [&](int j) { return (double)L.ew[j] * kin(j); }, S);
            const double ux = wsum(L.evx) / w, uy = wsum(L.evy) / w, uz = wsum(L.evz) / w;
            const double kth = T::tree(ne, [&](int j) {
                const double dx = L.evx[j] - ux, dy = L.evy[j] - uy, dz = L.evz[j] - uz;
                return (double)L.ew[j] * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
            }, S);
            kept = !(kall > 0.0) || !(kth > 0.0);
            if (!kept) {
                const double sig = sqrt(((2.0 * kall) / (3.0 * w)) * (QE / ME));
                T::sync();
                for (int j = tid; j < ne; j += B) {
                    double gx, gy, gz;
                    therm_normals(rng((uint32_t)j, RP_THERM, 0), gx, gy, gz);
                    L.evx[j] = sig * gx;
                    L.evy[j] = sig * gy;
                    L.evz[j] = sig * gz;
                }
                T::sync();
                const double qx = wsum(L.evx) / w, qy = wsum(L.evy) / w, qz = wsum(L.evz) / w;
                T::sync();
                for (int j = tid; j < ne; j += B) {
                    L.evx[j] = L.evx[j] - qx;
                    L.evy[j] = L.evy[j] - qy;
                    L.evz[j] = L.evz[j] - qz;
                }
                T::sync();
                const double kd = T::tree(ne, [&](int j) { return (double)L.ew[j] * kin(j); }, S);
                T::sync();
                // kd is 0 only if every draw coincides: then every electron
                // gets the drift velocity
                const double beta = kd > 0.0 ? sqrt(kth / kd) : 0.0;
                for (int j = tid; j < ne; j += B) {
                    L.evx[j] = kd > 0.0 ? ux + beta * L.evx[j] : ux;
                    L.evy[j] = kd > 0.0 ? uy + beta * L.evy[j] : uy;
                    L.evz[j] = kd > 0.0 ? uz + beta * L.evz[j] : uz;
                }
                T::sync();
                if (tid == 0) S.cnt[kd > 0.0 ? XP_C_THERM : XP_C_THERM_SKIPPED] += 1;
            }
        }
        if (kept && tid == 0) S.cnt[XP_C_THERM_SKIPPED] += 1;
    }

    // ---------------- commit ----------------
    ka = step_args<T>(a);
    if (overflow) {
        if (tid == 0) flag_status(a, run, XP_ST_CAPACITY);
        return false;
    }
    if (deferred) {
        defer();
        return false;
    }
    bool bad = false;
    for (int j = tid; j < ne; j += B) {
        const double x = L.evx[j], y = L.evy[j], z = L.evz[j];
        bad |= !(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z));
        ka->evx[eo + j] = x;
        ka->evy[eo + j] = y;
        ka->evz[eo + j] = z;
        ka->ew[eo + j] = L.ew[j];
    }
    for (int j = tid; j < ni; j += B) {
        ka->ivx[io + j] = L.ivx[j];
        ka->ivy[io + j] = L.ivy[j];
        ka->ivz[io + j] = L.ivz[j];
        ka->iz[io + j] = L.iz[j];
        ka->ik[io + j] = L.ik[j];
    }
    if (bad) flag_status(a, run, XP_ST_NONFINITE);
    T::sync();
    // positions of moved or new electrons: gather into LDS first, then write
    for (int j = tid; j < ne; j += B) {
        const int org = L.eorg[j];
        if (org == j) continue;
        if (org >= 0) {
            L.evx[j] = ka->ex[eo + org];
            L.evy[j] = ka->ey ? ka->ey[eo + org] : 0.0;
        } else {
            const int i = -1 - org;
            L.evx[j] = ka->ix[io + i];
            L.evy[j] = ka->iy ? ka->iy[io + i] : 0.0;
        }
    }
    T::sync();
    for (int j = tid; j < ne; j += B) {
        if (L.eorg[j] == j) continue;
        ka->ex[eo + j] = L.evx[j];
        if (ka->ey) ka->ey[eo + j] = L.evy[j];
    }
    if (tid == 0) {
        ka->e_cnt[cell] = ne;
        S.ints[6] = ne;
    }
    if (XV && (ka->cell_nka || (flags & XP_KA_FIELD))) {
        kalpha_record(a, cell, R, tb, S.kz, S.cnt, tid, B);
        T::sync();
    }
    if (XV && ka->cell_cnt)
        for (int q = tid; q < XP_NCOUNT; q += B) ka->cell_cnt[(size_t)cell * XP_NCOUNT + q] = S.cnt[q];
    if (XV && ka->cell_led)
        for (int q = tid; q < XP_NLEDGER; q += B) ka->cell_led[(size_t)cell * XP_NLEDGER + q] = S.led[q];
    if (XV && ka->cell_mom)
        for (int q = tid; q < XP_NMOM; q += B) ka->cell_mom[(size_t)cell * XP_NMOM + q] = S.mom[q];
    if (XV && ka->cell_nabs)
        for (int q = tid; q < XP_MAX_BINS; q += B) ka->cell_nabs[(size_t)cell * XP_MAX_BINS + q] = S.nabs[q];
    return true;
}

template __global__ void k_step<64, 0>(StepArgs);
template __global__ void k_step<256, 0>(StepArgs);
template __global__ void k_step_g<32, 0>(StepArgs);
template __global__ void k_step_g<16, 0>(StepArgs);
template __global__ void k_step_g<8, 0>(StepArgs);
template __global__ void k_step<64, 1>(StepArgs);
template __global__ void k_step<256, 1>(StepArgs);
template __global__ void k_step_g<32, 1>(StepArgs);
template __global__ void k_step_g<16, 1>(StepArgs);
template __global__ void k_step_g<8, 1>(StepArgs);
template __global__ void k_step<64, 2>(StepArgs);
template __global__ void k_step<256, 2>(StepArgs);
template __global__ void k_step_g<32, 2>(StepArgs);
template __global__ void k_step_g<16, 2>(StepArgs);
template __global__ void k_step_g<8, 2>(StepArgs);
template __global__ void k_step<64, 3>(StepArgs);
template __global__ void k_step<256, 3>(StepArgs);
template __global__ void k_step_g<32, 3>(StepArgs);
template __global__ void k_step_g<16, 3>(StepArgs);
template __global__ void k_step_g<8, 3>(StepArgs);

__global__ void k_step_prep(int32_t* counts, int32_t* stats)
{
    if (threadIdx.x < STEP_COUNTS && counts) counts[threadIdx.x] = 0;
    if (stats)
        for (int q = threadIdx.x; q < XP_NSTATS; q += blockDim.x) stats[q] = 0;
}

// Per-run photoionization cross sections of every bin and subshell (they
// depend on the run's photon energies only): [run][bin][subshell].
__global__ void k_run_prep(const xp_run* runs, int n_runs, const DevTables* tb, double* run_sig)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = t / (XP_MAX_BINS * 3), q = t % (XP_MAX_BINS * 3);
    if (r >= n_runs) return;
    const xp_run& R = runs[r];
    const int b = q / 3, sh = q % 3;
    run_sig[t] = b < R.n_bins ? photo_sigma(tb, sh, R.hv[b]) : 0.0;
}

size_t lds_budget(size_t max_lds)
{
    // static LDS of k_step (CellShared) plus a margin for the runtime's own
    const size_t fixed = sizeof(CellShared) + 1024;
    return max_lds > fixed ? max_lds - fixed : 0;
}

void lds_limits(size_t max_lds, int* e_lds, int* i_lds)
{
    const int ci = 1024;
    const size_t budget = lds_budget(max_lds);
    int ce = 0;
    while (step_lds_bytes(ce + 16, ci) <= budget) ce += 16;
    *e_lds = ce;
    *i_lds = ci;
}

}  // namespace xpd
