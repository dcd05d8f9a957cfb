// Global-memory step for cells beyond one workgroup's LDS (and for every cell
// when the caller asks for it): the same stages, draws and sums as the LDS
// step, with each cell spread over many workgroups.
//
// * A cell's slots are cut into aligned chunks of BIG_CH.  The canonical
//   pairwise sum over a cell equals the pairwise sum of its chunks' pairwise
//   sums: the chunks are aligned power-of-two subtrees of the same tree, and
//   the extra +0 padding changes at most the sign of a zero, which the final
//   + 0.0 removes.  Every sum that feeds a decision therefore has the bits of
//   the LDS path.
// * The random permutations (slots sorted by Philox word, then slot) come
//   from a segmented LSD radix sort: four stable 8-bit passes whose digit
//   offsets are scanned per cell, so a chunk never mixes cells.
// * e-e pairs are independent: one thread per pair.  In the e-i round robin
//   each slot of the smaller population meets its partners in a fixed
//   sequence (rank q, q + n_min, q + 2 n_min, ...), so one thread per slot of
//   the smaller population runs all rounds without a grid-wide barrier.
// * The ordered parts -- the ionization debit in ion-slot order and the
//   recombination energy sum -- run on one wave per cell over compact lists.
//
// Stage order and every formula follow the LDS step (Sec. II-V of the paper).
#include <hip/hip_runtime.h>

#include "xp_kernels.h"
#include "xp_physics.h"

namespace xpd {

namespace {

constexpr int BT = 256;   // threads of the chunk and per-cell kernels

__device__ __forceinline__ uint32_t step_of(const StepArgs& s, int run)
{
    return s.d_step ? s.d_step[run] : s.step;
}

__device__ __forceinline__ Words draw(const StepArgs& s, const BigRec& r, uint32_t idx,
                                      uint32_t purpose, uint32_t sub)
{
    const xp_run& R = s.runs[r.run];
    const uint32_t lcell = (uint32_t)(r.cell - R.cell_begin);
    return philox(step_of(s, r.run), lcell, idx, (purpose << 24) | sub, (uint32_t)R.seed,
                  (uint32_t)(R.seed >> 32));
}

__device__ __forceinline__ double kin_at(const StepArgs& s, int64_t p)
{
    const double x = s.evx[p], y = s.evy[p], z = s.evz[p];
    return HALF_ME_OVER_QE * ((x * x + y * y) + z * z);
}

__device__ __forceinline__ void flush_counts(BigRec& r, const int* cnt, const double* led)
{
    for (int q = threadIdx.x; q < XP_NCOUNT; q += blockDim.x)
        if (cnt[q]) atomicAdd(&r.cnt[q], cnt[q]);
    if (led)
        for (int q = threadIdx.x; q < XP_NLEDGER; q += blockDim.x)
            if (led[q] != 0.0) atomicAdd(&r.led[q], led[q]);
}

// ---------------------------------------------------------------- set-up

__global__ void k_big_all(BigArgs a, int n_cells)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += gridDim.x * blockDim.x)
        a.list[c] = c;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.count = n_cells;
}

__global__ void k_big_init(BigArgs a)
{
    const int requested = *a.count;
    const int nb = requested < a.big_max ? requested : a.big_max;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.hdr->count = nb;
        a.hdr->n_e_chunks = 0;
        a.hdr->n_i_chunks = 0;
        // cells beyond the list's capacity were flagged with their runs when listed
        if (requested > a.big_max) atomicOr(a.s.status, XP_ST_CAPACITY);
        if (a.s.stats) a.s.stats[2] = nb;
    }
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        BigRec& r = a.rec[b];
        const int cell = a.list[b];
        r.cell = cell;
        r.run = a.s.cell_run[cell];
        r.ne0 = r.ne = a.s.e_cnt[cell];
        r.ni = a.s.i_cnt[cell];
        r.ecap = a.s.e_cap[cell];
        r.eo = a.s.e_off[cell];
        r.io = a.s.i_off[cell];
        r.ce0 = r.nce = r.ci0 = r.nci = 0;
        r.ep0 = r.ip0 = 0;
        r.state = 0;
        r.need = 0;
        r.zc = 0;
        r.zmask = r.zeval = 0;
        r.zmask4 = 0;
        r.acc = 0;
        r.nrec = 0;
        r.epn = 0;
        r.nnew5 = 0;
        r.we = r.wb = r.sz = r.sz2 = r.ws = r.nelig = r.nfired = 0;
        r.we4 = r.wb4 = r.sz4 = 0;
        r.p = r.kth = r.debit = 0.0;
        r.alpha = 1.0;
        r.u[0] = r.u[1] = r.u[2] = 0.0;
        for (int q = 0; q < XP_NMOM; ++q) r.mom[q] = 0.0;
        for (int q = 0; q < XP_NCOUNT; ++q) r.cnt[q] = 0;
        for (int q = 0; q < XP_MAX_BINS; ++q) r.nabs[q] = 0;
        for (int q = 0; q < 14; ++q) r.kz[q] = 0;
        r.np5 = 0;
        for (int q = 0; q < XP_NLEDGER; ++q) r.led[q] = 0.0;
        const int64_t lim = (int64_t)BIG_MAX_CHUNKS * BIG_CH;
        if ((int64_t)r.ecap > lim || (int64_t)r.ni > lim) {
            r.state = 1;
            flag_status(a.s, r.run, XP_ST_CAPACITY);
        }
    }
}

// Chunk plan of one species: chunk ranges, population offsets and the chunk
// -> cell map.  species 0 electrons (current count r.ne), 1 ions.
__global__ __launch_bounds__(1024) void k_big_plan(BigArgs a, int species)
{
    __shared__ long long red[16];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int nb = a.hdr->count;
    if (tid == 0) bad = 0;
    long long carry_c = 0, carry_p = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int b = b0 + tid;
        long long n = 0;
        if (b < nb) {
            const BigRec& r = a.rec[b];
            n = r.state ? 0 : (species == 0 ? r.ne : r.ni);
        }
        const long long nch = (n + BIG_CH - 1) / BIG_CH;
        long long tot_c, tot_p;
        const long long ec = block_exclusive_sum<1024, long long>(nch, red, tot_c);
        const long long ep = block_exclusive_sum<1024, long long>(n, red, tot_p);
        if (b < nb) {
            BigRec& r = a.rec[b];
            if (species == 0) {
                r.ce0 = (int32_t)(carry_c + ec);
                r.nce = (int32_t)nch;
                r.ep0 = carry_p + ep;
                r.epn = (int32_t)n;
            } else {
                r.ci0 = (int32_t)(carry_c + ec);
                r.nci = (int32_t)nch;
                r.ip0 = carry_p + ep;
            }
        }
        carry_c += tot_c;
        carry_p += tot_p;
    }
    const long long cmax = species == 0 ? a.e_chunks_max : a.i_chunks_max;
    const long long pmax = species == 0 ? a.e_pop_max : a.i_pop_max;
    if (carry_c > cmax || carry_p > pmax) {
        // beyond the caller's bounds: stop every cell of the path
        for (int b = tid; b < nb; b += 1024) {
            BigRec& r = a.rec[b];
            r.state = 1;
            if (species == 0) { r.nce = 0; r.epn = 0; } else { r.nci = 0; }
            flag_status(a.s, r.run, XP_ST_CAPACITY);
        }
        if (tid == 0) bad = 1;
    }
    __syncthreads();
    if (tid == 0) {
        if (species == 0) a.hdr->n_e_chunks = bad ? 0 : (int32_t)carry_c;
        else a.hdr->n_i_chunks = bad ? 0 : (int32_t)carry_c;
    }
    if (bad) return;
    int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    for (int b = tid; b < nb; b += 1024) {
        const BigRec& r = a.rec[b];
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int nc = species == 0 ? r.nce : r.nci;
        for (int g = c0; g < c0 + nc; ++g) map[g] = b;
    }
}

// ---------------------------------------------------------------- S0

__global__ __launch_bounds__(BT) void k_big_s0(BigArgs a)
{
    __shared__ double red[2 * (BIG_CH / 64)];
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        BigRec& r = a.rec[a.e_chunk_cell[g]];
        const double ebulk = s.runs[r.run].e_bulk;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        long long wl = 0, bl = 0;
        bool bad = false;
        // the collisions gather electrons in permutation order: one 32-byte
        // record per electron in slot order turns three random reads into one
        const bool stage = (s.flags & (XP_EE | XP_EI)) != 0;
        double* e4 = a.ev4 + 4 * (r.ep0 + base);
        // one pass: every leaf j < n is visited once, so the weight sums, the
        // finiteness check and the staging ride on the bulk-energy tree
        const double ke = block_tree_sum<BT>(BIG_CH, [&](int j) {
            if (j >= n) return 0.0;
            const double x = s.evx[o + j], y = s.evy[o + j], z = s.evz[o + j];
            bad |= !(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z));
            const long long w = s.ew[o + j];
            wl += w;
            const double e = HALF_ME_OVER_QE * ((x * x + y * y) + z * z);
            if (e < ebulk) bl += w;
            if (stage) {
                e4[4 * j] = x;
                e4[4 * j + 1] = y;
                e4[4 * j + 2] = z;
                e4[4 * j + 3] = (double)w;
            }
            return e < ebulk ? (double)w * e : 0.0;
        }, red);
        if (bad) flag_status(s, r.run, XP_ST_NONFINITE);
        const long long we = block_isum<BT>(wl, ired);
        const long long wb = block_isum<BT>(bl, ired);
        if (tid == 0) {
            a.part[0][g] = ke;
            atomicAdd(&r.we, (unsigned long long)we);
            atomicAdd(&r.wb, (unsigned long long)wb);
        }
    }
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        const int64_t o = r.io + base;
        long long s1 = 0, s2 = 0;
        uint32_t zm = 0;
        const bool stage = (s.flags & XP_EI) != 0;
        double* i4 = a.iv4 + 4 * (r.ip0 + base);
        for (int j = tid; j < n; j += BT) {
            const long long z = s.iz[o + j];
            s1 += z;
            s2 += z * z;
            if (z < 13) zm |= 1u << z;
            if (stage) {
                i4[4 * j] = s.ivx[o + j];
                i4[4 * j + 1] = s.ivy[o + j];
                i4[4 * j + 2] = s.ivz[o + j];
                i4[4 * j + 3] = (double)z;
            }
        }
        s1 = block_isum<BT>(s1, ired);
        s2 = block_isum<BT>(s2, ired);
        if (zm) atomicOr(&r.zmask, zm);
        if (tid == 0) {
            atomicAdd(&r.sz, (unsigned long long)s1);
            atomicAdd(&r.sz2, (unsigned long long)s2);
        }
    }
}

// Moments, continuum lowering and the per-cell constants of S3 and S5.
__global__ __launch_bounds__(BT) void k_big_s0fin(BigArgs a)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const uint32_t flags = s.flags;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (r.state) continue;
        const xp_run& R = s.runs[r.run];
        const double ke = block_tree_sum<BT>(r.nce, [&](int j) { return a.part[0][r.ce0 + j]; }, red);
        const long long we = (long long)r.we, wb = (long long)r.wb;
        const long long sz = (long long)r.sz, sz2 = (long long)r.sz2;
        const int ne = r.ne, ni = r.ni;
        const long long wi = ni;
        const double w0 = R.w0, vol = R.volume;
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
        if (tid < 13) r.mom[16 + tid] = ipd(R.ipd_model, tid, t_e, n_e, n_i, zbar, zstar);
        if (tid == 13) r.mom[10] = R.lnl_fixed > 0.0 ? R.lnl_fixed : coulomb_log(t_e, n_e, zbar);
        if (tid == 0) {
            r.mom[0] = (double)we; r.mom[1] = (double)wi; r.mom[2] = (double)sz;
            r.mom[3] = (double)sz2; r.mom[4] = ke; r.mom[5] = t_e; r.mom[6] = n_e;
            r.mom[7] = n_i; r.mom[8] = zbar; r.mom[9] = zstar;
        }
        __syncthreads();
        const double* dE = r.mom + 16;
        if (tid == 0) {
            int need = 0;
            if ((flags & (XP_EE | XP_EI)) && ne >= 1 && (ne >= 2 || ni >= 1)) need |= BN_PERM_E;
            if ((flags & XP_EI) && ne >= 1 && ni >= 1) need |= BN_EI;
            if ((flags & XP_ION) && ne >= 1 && ni >= 1) {
                // charge states are unchanged until S3: the moments' sum serves
                const int zc = (int)((2 * sz + wi) / (2 * wi));
                r.zc = zc;
                // the evaluated charge states: Z_c, or (XP_ION_Z) every state
                // an ion holds
                const bool perz = (flags & XP_ION_Z) != 0;
                const uint32_t ze = perz ? r.zmask : (zc < 13 ? 1u << zc : 0u);
                r.zeval = ze;
                r.mom[11] = perz ? (double)__popc(ze) : (double)zc;
                if (ze) {
                    need |= BN_ION;
                    int clamped = 0;
                    for (int z = 0; z < 13; ++z) {
                        if (!(ze & (1u << z))) continue;
                        const Occ oc = occupancy(z, 0);
                        for (int q = 0; q < 5; ++q) {
                            const double raw = tb->bind[z][q] - dE[z];
                            r.ppz[z][q] = raw < 1.0 ? 1.0 : raw;
                            r.lnpz[z][q] = oc.s[q] > 0 ? xlog(r.ppz[z][q]) : 0.0;
                            if (oc.s[q] > 0 && raw < 1.0) ++clamped;
                        }
                    }
                    r.cnt[XP_C_IPD_CLAMPED] += clamped;
                }
            }
            r.need = need;
        }
        const int nbins = R.n_bins;
        if ((flags & XP_PHOTO) && nbins > 0) {
            const double* rs = s.run_sig + (size_t)r.run * (XP_MAX_BINS * 3);
            for (int q = tid; q < 3 * nbins; q += BT) r.sig[q / 3][q % 3] = rs[q];
            __syncthreads();
            const double* nhv = (R.field_per_cell && s.cell_nhv) ? s.cell_nhv + (size_t)r.cell * XP_MAX_BINS : R.nhv;
            for (int q = tid; q < 39; q += BT) {
                const int z = q / 3, sh = q % 3;
                const double pp = lowered(tb, z, sh, dE);
                double acc = 0.0;
                for (int bq = 0; bq < nbins; ++bq)
                    if (R.hv[bq] >= pp) acc = acc + nhv[bq] * r.sig[bq][sh];
                r.ssum[z][sh] = acc;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- sorting

__device__ __forceinline__ bool big_live(const BigRec& r, int needbit)
{
    return r.state == 0 && (r.need & needbit) != 0;
}

// Philox sort keys of one species in population order: slot j of a cell gets
// word j % 4 of the call with index j / 4.
__global__ __launch_bounds__(BT) void k_big_keys(BigArgs a, int species, int needbit, uint32_t purpose,
                                                 uint32_t* key, uint32_t* val)
{
    const int tid = threadIdx.x;
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, needbit)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int cnt = species == 0 ? r.epn : r.ni;
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int base = (g - c0) * BIG_CH;
        const int end = cnt - base < BIG_CH ? cnt : base + BIG_CH;
        for (int j0 = base + 4 * tid; j0 < end; j0 += 4 * BT) {
            const Words w = draw(a.s, r, (uint32_t)(j0 >> 2), purpose, 0);
            const uint32_t k4[4] = {w.x0, w.x1, w.x2, w.x3};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + q;
                if (j < end) {
                    key[pop + j] = k4[q];
                    val[pop + j] = (uint32_t)j;
                }
            }
        }
    }
}

// One wave per chunk: digit counts -> hist[256 * c0 + digit * nc + chunk].
// sub: sort the first nsub slots of the cell's range (the S4 rank candidates)
// instead of all of them.
__device__ __forceinline__ int big_count(const BigRec& r, int species, int sub)
{
    return sub ? r.nsub : (species == 0 ? r.epn : r.ni);
}

__global__ __launch_bounds__(64) void k_big_rhist(BigArgs a, int species, int needbit, int shift,
                                                  const uint32_t* key, int sub)
{
    __shared__ uint32_t h[256];
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, needbit)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int nc = species == 0 ? r.nce : r.nci;
        const int cnt = big_count(r, species, sub);
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int k = g - c0;
        const int base = k * BIG_CH;
        const int n = cnt - base < BIG_CH ? cnt - base : BIG_CH;
        for (int q = threadIdx.x; q < 256; q += 64) h[q] = 0;
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += 64) atomicAdd(&h[(key[pop + base + q] >> shift) & 255u], 1u);
        __syncthreads();
        uint32_t* hc = a.hist + (size_t)256 * g;
        for (int q = threadIdx.x; q < 256; q += 64) hc[q] = h[q];
        __syncthreads();
    }
}

// Exclusive scan of a cell's digit counts in (digit, chunk) order over the
// chunk-major table hist[chunk][digit].  1024 threads: thread (q, d) runs down
// quarter q of digit d's column (coalesced across d), the quarter totals are
// scanned per digit, the digit totals across digits, and each thread adds
// its offset to its quarter.
__global__ __launch_bounds__(1024) void k_big_rscan(BigArgs a, int species, int needbit, int sub)
{
    __shared__ uint32_t qsum[4][256];
    __shared__ uint32_t red[16];
    const int tid = threadIdx.x, d = tid & 255, qt = tid >> 8;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const BigRec& r = a.rec[b];
        if (!big_live(r, needbit)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        // with sub, only the chunks that hold the nsub candidates have counts
        const int nc = sub ? (r.nsub + BIG_CH - 1) / BIG_CH : (species == 0 ? r.nce : r.nci);
        if (nc == 0) continue;
        const int per = (nc + 3) / 4;
        const int k0 = qt * per, k1 = k0 + per < nc ? k0 + per : nc;
        uint32_t* h = a.hist + (size_t)256 * c0 + d;
        uint32_t run = 0;
        int k = k0;
        // eight loads in flight at a time: the walk is bound by memory latency
        for (; k + 8 <= k1; k += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = h[(size_t)256 * (k + u)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                h[(size_t)256 * (k + u)] = run;
                run += v[u];
            }
        }
        for (; k < k1; ++k) {
            const uint32_t v = h[(size_t)256 * k];
            h[(size_t)256 * k] = run;
            run += v;
        }
        qsum[qt][d] = run;
        __syncthreads();
        // digit totals (threads of quarter 0), exclusive over digits: every
        // thread takes part in the block scan, the other quarters add 0
        uint32_t t = 0;
        if (qt == 0) {
            for (int q = 0; q < 4; ++q) {
                const uint32_t v = qsum[q][d];
                qsum[q][d] = t;
                t += v;
            }
        }
        uint32_t tot;
        const uint32_t dbase = block_exclusive_sum<1024, uint32_t>(t, red, tot);
        if (qt == 0)
            for (int q = 0; q < 4; ++q) qsum[q][d] += dbase;
        __syncthreads();
        const uint32_t off = qsum[qt][d];
        if (off) {
            int k2 = k0;
            for (; k2 + 8 <= k1; k2 += 8) {
                uint32_t v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = h[(size_t)256 * (k2 + u)];
#pragma unroll
                for (int u = 0; u < 8; ++u) h[(size_t)256 * (k2 + u)] = v[u] + off;
            }
            for (; k2 < k1; ++k2) h[(size_t)256 * k2] += off;
        }
        __syncthreads();
    }
}

// One block per chunk: the chunk's keys are ranked stably by digit in LDS
// (first a digit histogram and its scan give each digit's local run, then
// groups of 256 keys are ranked with wave ballots and per-wave digit counts),
// then written out in staged order so that each digit's run lands
// contiguously at the chunk's global offset for that digit.
__global__ __launch_bounds__(256) void k_big_rscatter(BigArgs a, int species, int needbit, int shift,
                                                      const uint32_t* key, const uint32_t* val,
                                                      uint32_t* key_out, uint32_t* val_out, int sub)
{
    __shared__ uint32_t lstart[256];     // local start of each digit's run in the chunk
    __shared__ uint32_t gbase[256];      // global offset of each digit for this chunk
    __shared__ uint32_t seen[256];       // keys of each digit placed so far
    __shared__ uint32_t wcnt[4][256];    // per-wave digit counts of the current group
    __shared__ uint32_t skey[BIG_CH], sval[BIG_CH];
    __shared__ uint32_t red[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, needbit)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int cnt = big_count(r, species, sub);
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int base = (g - c0) * BIG_CH;
        const int n = cnt - base < BIG_CH ? cnt - base : BIG_CH;
        const uint32_t* kin = key + pop + base;
        const uint32_t* vin = val + pop + base;
        // local digit histogram and its exclusive scan
        seen[tid] = 0;
        gbase[tid] = a.hist[(size_t)256 * g + tid];
        __syncthreads();
        for (int q = tid; q < n; q += 256) atomicAdd(&seen[(kin[q] >> shift) & 255u], 1u);
        __syncthreads();
        uint32_t tot;
        lstart[tid] = block_exclusive_sum<256, uint32_t>(seen[tid], red, tot);
        __syncthreads();
        seen[tid] = 0;
        __syncthreads();
        // stable ranking, 256 keys at a time
        for (int c = 0; c < n; c += 256) {
            const int i = c + tid;
            const bool valid = i < n;
            const uint32_t k = valid ? kin[i] : 0u;
            const uint32_t v = valid ? vin[i] : 0u;
            const uint32_t d = (k >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const uint64_t bal = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? bal : ~bal;
            }
            const uint32_t below = (uint32_t)__popcll(peers & lt);
            for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
            __syncthreads();
            if (valid && below == 0) wcnt[wid][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            uint32_t before = 0;
            if (valid)
                for (int w = 0; w < wid; ++w) before += wcnt[w][d];
            if (valid) {
                const uint32_t pos = lstart[d] + seen[d] + before + below;
                skey[pos] = k;
                sval[pos] = v;
            }
            __syncthreads();
            seen[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
            __syncthreads();
        }
        // each digit's run to its global place (consecutive t, consecutive addresses)
        for (int t = tid; t < n; t += 256) {
            const uint32_t k = skey[t];
            const uint32_t d = (k >> shift) & 255u;
            const int64_t dst = pop + gbase[d] + (t - lstart[d]);
            key_out[dst] = k;
            val_out[dst] = sval[t];
        }
        __syncthreads();
    }
}

// ---- S4 ranks: the first nrec ranks of the REC_E permutation (electrons) and
// the first nrec recombination-eligible ions (Z above the run's floor) of the
// REC_I permutation, without sorting the whole population.  The top 8 bits of
// the Philox words of the slots that take part (every electron; the eligible
// ions) are counted per chunk (k_sel_hist); the smallest digit D whose
// cumulative count reaches nrec bounds the candidates: every taking-part slot
// whose word has a top digit <= D (nsub of them, in slot order) is copied to
// key_b / val_b, the radix passes sort those nsub slots by (word, slot), and
// the first nrec ranks are copied out (val_a for electrons, sel for ions).
// Every slot left out has a larger word than every candidate, so the ranks
// are those of the whole permutation, ineligible ions skipped.  species 0
// reads the keys from key_a / val_a, species 1 from key_c / val_c.

__device__ __forceinline__ bool sel_takes_part(const BigArgs& a, const BigRec& r, int species, int j)
{
    return species == 0 || (int)a.s.iz[r.io + j] > a.s.runs[r.run].z_floor;
}

// One wave per chunk: top-digit counts of the taking-part slots -> hist[256 * chunk].
__global__ __launch_bounds__(64) void k_sel_hist(BigArgs a, int species)
{
    __shared__ uint32_t h[256];
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    const uint32_t* key = species == 0 ? a.key_a : a.key_c;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, BN_REC)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int cnt = species == 0 ? r.epn : r.ni;
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int base = (g - c0) * BIG_CH;
        const int n = cnt - base < BIG_CH ? cnt - base : BIG_CH;
        for (int q = threadIdx.x; q < 256; q += 64) h[q] = 0;
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += 64)
            if (sel_takes_part(a, r, species, base + q)) atomicAdd(&h[key[pop + base + q] >> 24], 1u);
        __syncthreads();
        uint32_t* hc = a.hist + (size_t)256 * g;
        for (int q = threadIdx.x; q < 256; q += 64) hc[q] = h[q];
        __syncthreads();
    }
}

// Per cell: the bound D, the candidates nsub, and per chunk the offset of its
// candidates (in hist[256 * chunk], after the chunk's counts are used).  1024
// threads: thread (quarter, digit) adds a quarter of the digit's column with
// eight loads in flight; each wave then counts the candidates of every 16th
// chunk from a coalesced read of the chunk's row.
__global__ __launch_bounds__(1024) void k_sel_find(BigArgs a, int species)
{
    __shared__ uint32_t qsum[4][256];
    __shared__ uint32_t red[16];
    __shared__ uint32_t tots[256];
    __shared__ int dsel;
    const int tid = threadIdx.x, d0 = tid & 255, qt = tid >> 8;
    const int lane = tid & 63, wid = tid >> 6;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, BN_REC)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int nc = species == 0 ? r.nce : r.nci;
        // the digit totals over the cell's chunks
        const int per = (nc + 3) / 4;
        const int k0 = qt * per, k1 = k0 + per < nc ? k0 + per : nc;
        const uint32_t* col = a.hist + (size_t)256 * c0 + d0;
        uint32_t part = 0;
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = col[(size_t)256 * (k + u)];
#pragma unroll
            for (int u = 0; u < 8; ++u) part += v[u];
        }
        for (; k < k1; ++k) part += col[(size_t)256 * k];
        qsum[qt][d0] = part;
        __syncthreads();
        const uint32_t t = tid < 256 ? qsum[0][tid] + qsum[1][tid] + qsum[2][tid] + qsum[3][tid] : 0u;
        uint32_t tot;
        const uint32_t incl = block_exclusive_sum<1024, uint32_t>(t, red, tot) + t;
        if (tid < 256) tots[tid] = incl;
        if (tid == 0) dsel = 255;
        __syncthreads();
        // the smallest digit whose cumulative count reaches nrec
        if (tid < 256 && incl >= (uint32_t)r.nrec && (tid == 0 || tots[tid - 1] < (uint32_t)r.nrec)) dsel = tid;
        __syncthreads();
        const uint32_t d = (uint32_t)dsel;
        // candidates per chunk: a wave reads the chunk's 256 counts and adds
        // those of digits <= d
        for (int kc = wid; kc < nc; kc += 16) {
            uint32_t* h = a.hist + (size_t)256 * (c0 + kc);
            uint32_t c = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t q = (uint32_t)(lane + 64 * u);
                c += q <= d ? h[q] : 0u;
            }
            c = (uint32_t)wave_isum64((long long)c);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) h[0] = c;
        }
        __syncthreads();
        // their exclusive scan over the chunks
        uint32_t carry = 0;
        for (int kb = 0; kb < nc; kb += 1024) {
            const int kc = kb + tid;
            uint32_t* h = a.hist + (size_t)256 * (c0 + kc);
            const uint32_t c = kc < nc ? h[0] : 0u;
            uint32_t ctot;
            const uint32_t ex = block_exclusive_sum<1024, uint32_t>(c, red, ctot);
            if (kc < nc) h[0] = carry + ex;
            carry += ctot;
        }
        if (tid == 0) {
            r.seld = (int32_t)d;
            r.nsub = (int32_t)carry;
        }
        __syncthreads();
    }
}

// The candidates of every chunk to key_b / val_b in slot order.
__global__ __launch_bounds__(BT) void k_sel_compact(BigArgs a, int species)
{
    __shared__ int red[BT / 64];
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    const uint32_t* key = species == 0 ? a.key_a : a.key_c;
    const uint32_t* val = species == 0 ? a.val_a : a.val_c;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, BN_REC)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int cnt = species == 0 ? r.epn : r.ni;
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int base = (g - c0) * BIG_CH;
        const int n = cnt - base < BIG_CH ? cnt - base : BIG_CH;
        if (n <= 0) continue;
        const int64_t in = pop + base;
        const int64_t out = pop + (int64_t)a.hist[(size_t)256 * g];
        const uint32_t d = (uint32_t)r.seld;
        block_ordered_select<BT>(
            n, [&](int q) { return (key[in + q] >> 24) <= d && sel_takes_part(a, r, species, base + q); },
            [&](int q, int pos) {
                a.key_b[out + pos] = key[in + q];
                a.val_b[out + pos] = val[in + q];
            },
            red);
    }
}

// The first nrec sorted candidates (val_b): electrons to val_a, ions to sel.
__global__ __launch_bounds__(BT) void k_sel_copy(BigArgs a, int species)
{
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, BN_REC)) continue;
        const int base = (g - (species == 0 ? r.ce0 : r.ci0)) * BIG_CH;
        if (base >= r.nrec) continue;
        const int n = r.nrec - base < BIG_CH ? r.nrec - base : BIG_CH;
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        if (species == 0)
            for (int q = threadIdx.x; q < n; q += BT) a.val_a[pop + base + q] = a.val_b[pop + base + q];
        else
            for (int q = threadIdx.x; q < n; q += BT) a.sel[pop + base + q] = (int32_t)a.val_b[pop + base + q];
    }
}

// Velocities (and electron weights / ion charge states) copied into
// permutation-rank order before the collisions (scatter = 0) and back to their
// slots afterwards (scatter = 1), so that the collision kernels read and write
// contiguous ranks.  species 0 electrons (PERM_E), 1 ions (PERM_I).
__global__ __launch_bounds__(BT) void k_big_gather(BigArgs a, int species, int scatter)
{
    const StepArgs& s = a.s;
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    const int needbit = species == 0 ? BN_PERM_E : BN_EI;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, needbit)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int cnt = species == 0 ? r.epn : r.ni;
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int base = (g - c0) * BIG_CH;
        const int n = cnt - base < BIG_CH ? cnt - base : BIG_CH;
        // the slot-order side is the 32-byte records staged by k_big_s0 (one
        // random access per particle); the rank-order side is coalesced
        if (species == 0) {
            const uint32_t* perm = a.val_a + pop;
            for (int q = threadIdx.x; q < n; q += BT) {
                const int64_t gi = pop + base + q;
                double* rec = a.ev4 + 4 * (pop + perm[base + q]);
                if (!scatter) {
                    const double2 xy = *(const double2*)rec, zw = *(const double2*)(rec + 2);
                    a.gev[0][gi] = xy.x;
                    a.gev[1][gi] = xy.y;
                    a.gev[2][gi] = zw.x;
                    a.gew[gi] = (uint32_t)zw.y;
                } else {
                    *(double2*)rec = make_double2(a.gev[0][gi], a.gev[1][gi]);
                    *(double2*)(rec + 2) = make_double2(a.gev[2][gi], (double)a.gew[gi]);
                }
            }
        } else {
            const uint32_t* perm = a.val_c + pop;
            for (int q = threadIdx.x; q < n; q += BT) {
                const int64_t gi = pop + base + q;
                double* rec = a.iv4 + 4 * (pop + perm[base + q]);
                if (!scatter) {
                    const double2 xy = *(const double2*)rec, zw = *(const double2*)(rec + 2);
                    a.giv[0][gi] = xy.x;
                    a.giv[1][gi] = xy.y;
                    a.giv[2][gi] = zw.x;
                    a.giz[gi] = (uint8_t)zw.y;
                } else {
                    *(double2*)rec = make_double2(a.giv[0][gi], a.giv[1][gi]);
                    *(double2*)(rec + 2) = make_double2(a.giv[2][gi], (double)a.giz[gi]);
                }
            }
        }
    }
}

// After the collisions: the staged records back into the particle arrays, in
// slot order (coalesced).
__global__ __launch_bounds__(BT) void k_big_unstage(BigArgs a, int species)
{
    const StepArgs& s = a.s;
    const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
    const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
    const int needbit = species == 0 ? BN_PERM_E : BN_EI;
    for (int g = blockIdx.x; g < nch; g += gridDim.x) {
        const BigRec& r = a.rec[map[g]];
        if (!big_live(r, needbit)) continue;
        const int c0 = species == 0 ? r.ce0 : r.ci0;
        const int cnt = species == 0 ? r.epn : r.ni;
        const int64_t pop = species == 0 ? r.ep0 : r.ip0;
        const int base = (g - c0) * BIG_CH;
        const int n = cnt - base < BIG_CH ? cnt - base : BIG_CH;
        const int64_t o = (species == 0 ? r.eo : r.io) + base;
        const double* rec = (species == 0 ? a.ev4 : a.iv4) + 4 * (pop + base);
        double* vx = species == 0 ? s.evx : s.ivx;
        double* vy = species == 0 ? s.evy : s.ivy;
        double* vz = species == 0 ? s.evz : s.ivz;
        for (int q = threadIdx.x; q < n; q += BT) {
            const double2 xy = *(const double2*)(rec + 4 * q);
            vx[o + q] = xy.x;
            vy[o + q] = xy.y;
            vz[o + q] = rec[4 * q + 2];
        }
    }
}

// ---------------------------------------------------------------- S1, S2

// LAW: bit 0 Nanbu's scattering law (XP_NANBU) instead of Takizuka-Abe's,
// bit 1 relativistic kinematics (XP_REL); the plain instance carries none of
// their code.
template <int LAW>
__global__ __launch_bounds__(BT) void k_big_ee(BigArgs a)
{
    __shared__ int cnt[XP_NCOUNT];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const double mi = s.tab->mass_ion;
    (void)mi;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        BigRec& r = a.rec[a.e_chunk_cell[g]];
        const int ne = r.epn;
        if (r.state || !(r.need & BN_PERM_E) || ne < 2) continue;
        const xp_run& R = s.runs[r.run];
        for (int q = tid; q < XP_NCOUNT; q += BT) cnt[q] = 0;
        __syncthreads();
        const double qe4 = (QE * QE) * (QE * QE);
        const double mee = (ME * ME) / (ME + ME);
        const double kee = qe4 / (((8.0 * PI) * (EPS0 * EPS0)) * (mee * mee));
        const double lnl = r.mom[10];
        const double afull = (kee * lnl) * R.dt;
        const double ahalf = (kee * lnl) * (0.5 * R.dt);
        const double nunit = (R.w0 * (double)ne) / R.volume;
        const double f_ee = ME / (ME + ME);
        const int start = (ne % 2 == 1 && ne >= 3) ? 3 : 0;
        const int npairs = (ne - start) / 2;
        const int k = g - r.ce0;
        const int base = k * BIG_CH;
        const int jlo = base <= start ? 0 : (base - start + 1) / 2;
        int jhi = (base + BIG_CH - start + 1) / 2;
        if (jhi > npairs) jhi = npairs;
        // electrons in permutation-rank order
        double* vx = a.gev[0] + r.ep0;
        double* vy = a.gev[1] + r.ep0;
        double* vz = a.gev[2] + r.ep0;
        const uint32_t* w = a.gew + r.ep0;
        const xp_run& RR = R;
        const uint32_t st = step_of(s, r.run);
        const uint32_t lcell = (uint32_t)(r.cell - RR.cell_begin);
        const uint32_t k0 = (uint32_t)RR.seed, k1 = (uint32_t)(RR.seed >> 32);
        if (k == 0 && start == 3 && tid == 0) {
            const int p0 = 0, p1 = 1, p2 = 2;
            collide_slots(vx, vy, vz, w, vx, vy, vz, p0, p1, w[p1], f_ee, f_ee, ahalf, nunit, st, lcell, 0u,
                          RP_EE_TRI << 24, k0, k1, cnt, LAW, ME, ME);
            collide_slots(vx, vy, vz, w, vx, vy, vz, p1, p2, w[p2], f_ee, f_ee, ahalf, nunit, st, lcell, 1u,
                          RP_EE_TRI << 24, k0, k1, cnt, LAW, ME, ME);
            collide_slots(vx, vy, vz, w, vx, vy, vz, p2, p0, w[p0], f_ee, f_ee, ahalf, nunit, st, lcell, 2u,
                          RP_EE_TRI << 24, k0, k1, cnt, LAW, ME, ME);
            cnt[XP_C_TRIPLET] += 3;
        }
        for (int j = jlo + tid; j < jhi; j += BT) {
            const int e = start + 2 * j, f = start + 2 * j + 1;
            collide_slots(vx, vy, vz, w, vx, vy, vz, e, f, w[f], f_ee, f_ee, afull, nunit, st, lcell,
                          (uint32_t)j, RP_EE << 24, k0, k1, cnt, LAW, ME, ME);
        }
        __syncthreads();
        if (tid == 0 && k == 0) cnt[XP_C_EE] += npairs;
        __syncthreads();
        flush_counts(r, cnt, nullptr);
        __syncthreads();
    }
}

template <int LAW>
__global__ __launch_bounds__(BT) void k_big_ei(BigArgs a)
{
    __shared__ int cnt[XP_NCOUNT];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const double mi = s.tab->mass_ion;
    const double fe_ei = mi / (ME + mi);
    const double fi_ei = ME / (ME + mi);
    const double qe4 = (QE * QE) * (QE * QE);
    const double mei = (ME * mi) / (ME + mi);
    const double kei = qe4 / (((8.0 * PI) * (EPS0 * EPS0)) * (mei * mei));
    // species 1: cells with n_e >= n_i, one thread per ion rank;
    // species 0: cells with n_e < n_i, one thread per electron rank
    for (int species = 1; species >= 0; --species) {
        const int nch = species == 0 ? a.hdr->n_e_chunks : a.hdr->n_i_chunks;
        const int32_t* map = species == 0 ? a.e_chunk_cell : a.i_chunk_cell;
        for (int g = blockIdx.x; g < nch; g += gridDim.x) {
            BigRec& r = a.rec[map[g]];
            const int ne = r.epn, ni = r.ni;
            if (r.state || !(r.need & BN_EI)) continue;
            if ((species == 1) != (ne >= ni)) continue;
            const xp_run& R = s.runs[r.run];
            for (int q = tid; q < XP_NCOUNT; q += BT) cnt[q] = 0;
            __syncthreads();
            const double a1 = (kei * r.mom[10]) * R.dt;
            const int nmin = ne < ni ? ne : ni, nmax = ne < ni ? ni : ne;
            const double nunit = (R.w0 * (double)nmin) / R.volume;
            const int c0 = species == 0 ? r.ce0 : r.ci0;
            const int k = g - c0;
            const int base = k * BIG_CH;
            const int n = nmin - base < BIG_CH ? nmin - base : BIG_CH;
            // both species in permutation-rank order
            double* vx = a.gev[0] + r.ep0;
            double* vy = a.gev[1] + r.ep0;
            double* vz = a.gev[2] + r.ep0;
            const uint32_t* w = a.gew + r.ep0;
            double* ix = a.giv[0] + r.ip0;
            double* iy = a.giv[1] + r.ip0;
            double* iz = a.giv[2] + r.ip0;
            const uint8_t* zz = a.giz + r.ip0;
            const uint32_t st = step_of(s, r.run);
            const uint32_t lcell = (uint32_t)(r.cell - R.cell_begin);
            const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
                for (int q = base + tid; q < base + n; q += BT) {
                for (int kk = q; kk < nmax; kk += nmin) {
                    int e, i;
                    if (ne >= ni) { e = kk; i = q; }
                    else          { i = kk; e = q; }
                    const int z = zz[i];
                    if (z == 0) continue;
                    collide_slots(vx, vy, vz, w, ix, iy, iz, e, i, 1u, fe_ei, fi_ei, a1 * (double)(z * z),
                                  nunit, st, lcell, (uint32_t)kk, RP_EI << 24, k0, k1, cnt, LAW, ME, mi);
                }
            }
            __syncthreads();
            if (tid == 0 && k == 0) cnt[XP_C_EI] += nmax;
            __syncthreads();
            flush_counts(r, cnt, nullptr);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- S3

__global__ __launch_bounds__(BT) void k_big_lotz(BigArgs a)
{
    __shared__ double red[2 * (BIG_CH / 64)];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_ION)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        for (int z = 0; z < 13; ++z) {
            if (!(r.zeval & (1u << z))) continue;
            const Occ occ = occupancy(z, 0);
            double pp[5], lnp[5];
            double pmin = __builtin_inf();
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                pp[q] = r.ppz[z][q];
                lnp[q] = r.lnpz[z][q];
                if (occ.s[q] > 0 && pp[q] < pmin) pmin = pp[q];
            }
            const double sum = block_tree_sum<BT>(BIG_CH, [&](int j) {
                if (j >= n) return 0.0;
                return lotz_leaf(s.evx[o + j], s.evy[o + j], s.evz[o + j], s.ew[o + j], occ.s, pp, lnp, pmin, tb);
            }, red);
            if (tid == 0) a.partz[(size_t)z * a.e_chunks_max + g] = sum;
        }
    }
}

__global__ __launch_bounds__(BT) void k_big_s3p(BigArgs a)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    const StepArgs& s = a.s;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, BN_ION)) continue;
        const xp_run& R = s.runs[r.run];
        double pmax = 0.0;
        for (int z = 0; z < 13; ++z) {
            if (!(r.zeval & (1u << z))) continue;
            const double* pz = a.partz + (size_t)z * a.e_chunks_max + r.ce0;
            const double ssum = block_tree_sum<BT>(r.nce, [&](int j) { return pz[j]; }, red);
            double p = ((ssum * R.w0) * R.dt) / R.volume;
            if (p > 1.0) {
                p = 1.0;
                if (threadIdx.x == 0) r.cnt[XP_C_P_CLAMPED] += 1;
            }
            if (threadIdx.x == 0) r.pz[z] = p;
            if (p > pmax) pmax = p;
        }
        if (threadIdx.x == 0) r.mom[12] = pmax;
        __syncthreads();
    }
}

__global__ __launch_bounds__(BT) void k_big_fire(BigArgs a)
{
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (!big_live(r, BN_ION)) continue;
        const bool perz = (s.flags & XP_ION_Z) != 0;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        long long c = 0;
        for (int q = tid; q < n; q += BT) {
            const int i = base + q;
            bool f = false;
            const int zi = s.iz[r.io + i];
            if (zi < 13) {
                const double p = r.pz[perz ? zi : r.zc];
                if (p > 0.0) f = u32(draw(s, r, (uint32_t)i, RP_ION, 0).x0) < p;
            }
            a.iflag[r.ip0 + i] = f ? 1 : 0;
            c += f ? 1 : 0;
        }
        c = block_isum<BT>(c, ired);
        if (tid == 0) {
            a.ccnt[g] = (int32_t)c;
            if (c) atomicAdd(&r.nfired, (unsigned long long)c);
        }
    }
}

// Per-cell exclusive scan of the ion-chunk counts in ccnt.  mode 0: fired
// ions of S3; 2: electrons appended by S5 (with the capacity check); 3: ions
// firing in S4 (XP_REC_XS).
__global__ __launch_bounds__(BT) void k_big_cscan(BigArgs a, int mode)
{
    __shared__ int red[BT / 64];
    const int tid = threadIdx.x;
    const int nb = a.hdr->count;
    const int needbit = mode == 0 ? BN_ION : (mode == 3 ? BN_REC : 0);
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (r.state || (needbit && !(r.need & needbit))) continue;
        int carry = 0;
        for (int k0 = 0; k0 < r.nci; k0 += BT) {
            const int k = k0 + tid;
            const int v = k < r.nci ? a.ccnt[r.ci0 + k] : 0;
            int tot;
            const int ex = block_exclusive_sum<BT, int>(v, red, tot);
            if (k < r.nci) a.ccnt[r.ci0 + k] = carry + ex;
            carry += tot;
        }
        if (tid == 0) {
            if (mode == 0) {
                r.cnt[XP_C_ION_FIRED] += carry;
                if (carry > 0) r.need |= BN_FIRED;
            } else if (mode == 3) {
                // XP_REC_XS: the firing ions recombine in slot order, at most
                // one per electron
                r.nrec = carry < r.ne ? carry : r.ne;
                if (r.nrec == 0) r.need &= ~BN_REC;
            } else if (mode == 2) {
                if ((long long)r.ne + carry > (long long)r.ecap) {
                    r.state = 1;
                    flag_status(a.s, r.run, XP_ST_CAPACITY);
                } else {
                    r.nnew5 = carry;
                    r.cnt[XP_C_E_NEW] += carry;
                }
            }
        }
        __syncthreads();
    }
}

// Drift-frame sums of electrons 0 .. epn-1: weights w (mode 0, S3) or the
// reduced weights wp (mode 1, S4).
__global__ __launch_bounds__(BT) void k_big_drift(BigArgs a, int mode)
{
    __shared__ double red3[6 * (BIG_CH / 64)];
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const int needbit = mode == 0 ? BN_FIRED : BN_REC;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, needbit)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        const uint32_t* wsrc = mode == 0 ? s.ew + o : a.wp + r.ep0 + base;
        // the weights summed in the same pass (every leaf j < n is visited once)
        long long wl = 0;
        const double *vx = s.evx + o, *vy = s.evy + o, *vz = s.evz + o;
        double tx, ty, tz;
        block_tree_sum3<BT>(BIG_CH, [&](int j, double& x, double& y, double& z) {
            if (j < n) {
                const uint32_t wu = wsrc[j];
                wl += wu;
                const double w = (double)wu;
                x = w * vx[j];
                y = w * vy[j];
                z = w * vz[j];
            }
        }, red3, tx, ty, tz);
        wl = block_isum<BT>(wl, ired);
        if (tid == 0) {
            a.part[1][g] = tx;
            a.part[2][g] = ty;
            a.part[3][g] = tz;
        }
        if (tid == 0 && wl) atomicAdd(&r.ws, (unsigned long long)wl);
    }
}

__global__ __launch_bounds__(BT) void k_big_dfin(BigArgs a, int mode)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    const int needbit = mode == 0 ? BN_FIRED : BN_REC;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, needbit)) continue;
        const long long ws = (long long)r.ws;
        for (int d = 0; d < 3; ++d) {
            const double t = block_tree_sum<BT>(r.nce, [&](int j) { return a.part[1 + d][r.ce0 + j]; }, red);
            if (threadIdx.x == 0) r.u[d] = ws != 0 ? t / (double)ws : 0.0;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BT) void k_big_kth(BigArgs a, int mode)
{
    __shared__ double red[2 * (BIG_CH / 64)];
    const StepArgs& s = a.s;
    const int needbit = mode == 0 ? BN_FIRED : BN_REC;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, needbit)) continue;
        if (mode == 1 && r.ws == 0) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        const uint32_t* wsrc = mode == 0 ? s.ew + o : a.wp + r.ep0 + base;
        const double ux = r.u[0], uy = r.u[1], uz = r.u[2];
        const double t = block_tree_sum<BT>(BIG_CH, [&](int j) {
            if (j >= n) return 0.0;
            const double dx = s.evx[o + j] - ux, dy = s.evy[o + j] - uy, dz = s.evz[o + j] - uz;
            return (double)wsrc[j] * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
        }, red);
        if (threadIdx.x == 0) a.part[0][g] = t;
    }
}

// Lowered potential of every fired ion, compacted in ion-slot order:
// fip[ip0 + rank] (ranks from the per-cell scan of the chunk counts).
__global__ __launch_bounds__(BT) void k_big_firelist(BigArgs a)
{
    __shared__ int red[BT / 64];
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        const BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (!big_live(r, BN_FIRED)) continue;
        const int cb = a.ccnt[g];
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        const double* dE = r.mom + 16;
        block_ordered_select<BT>(
            n, [&](int q) { return a.iflag[r.ip0 + base + q] != 0; },
            [&](int q, int pos) {
                const int64_t pi = r.io + base + q;
                const int z = s.iz[pi], kv = s.ik[pi];
                a.fip[r.ip0 + cb + pos] = lowered(tb, z, valence(z, kv), dE);
            },
            red);
    }
}

// One wave per cell: K_th, then the fired ions accepted in slot order while
// the running debit (a left-to-right sum) stays within K_th.  The wave stages
// 64 potentials at a time in LDS (the next 64 already loading) and first adds
// all of them in order: the potentials are positive and rounding is
// monotone, so if the block's running sum stays within K_th (and the slab has
// room) every ion of the block is accepted with exactly that sum.  Only the
// block where the walk stops is walked again ion by ion.
__global__ __launch_bounds__(64) void k_big_accept(BigArgs a)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    __shared__ double blk[64];
    const int lane = threadIdx.x;
    const StepArgs& s = a.s;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, BN_FIRED)) continue;
        const double kth = block_tree_sum<64>(r.nce, [&](int j) { return a.part[0][r.ce0 + j]; }, red);
        const int ne0 = r.ne0;
        const int nfired = (int)r.nfired;
        const int room = r.ecap - ne0;
        const double* fip = a.fip + r.ip0;
        double debit = 0.0;
        int acc = 0;
        bool stop = false, over = false;
        double next = lane < nfired ? fip[lane] : 0.0;
        for (int t0 = 0; t0 < nfired && !stop; t0 += 64) {
            const int m = nfired - t0 < 64 ? nfired - t0 : 64;
            __syncthreads();
            blk[lane] = next;   // +0 beyond the fired ions: adds nothing
            __syncthreads();
            next = t0 + 64 + lane < nfired ? fip[t0 + 64 + lane] : 0.0;
            double run = debit;
#pragma unroll 16
            for (int l = 0; l < 64; ++l) run = run + blk[l];
            if (run <= kth && acc + m <= room) {
                debit = run;
                acc += m;
                continue;
            }
            for (int l = 0; l < m; ++l) {
                const double ipv = blk[l];
                if (!(debit + ipv <= kth)) {
                    stop = true;
                    break;
                }
                if (acc >= room) {
                    over = true;
                    stop = true;
                    break;
                }
                debit = debit + ipv;
                ++acc;
            }
        }
        if (lane == 0) {
            r.kth = kth;
            r.mom[13] = kth;
            if (over) {
                r.state = 1;
                flag_status(s, r.run, XP_ST_CAPACITY);
            } else {
                r.acc = acc;
                r.debit = debit;
                r.mom[14] = debit;
                r.cnt[XP_C_ION_ACCEPTED] += acc;
                r.cnt[XP_C_ION_STARVED] += nfired - acc;
                r.cnt[XP_C_E_NEW] += acc;
                r.led[XP_L_ION_DEBIT] += debit;
                r.alpha = debit > 0.0 ? sqrt(1.0 - debit / kth) : 1.0;
                r.ne = ne0 + acc;
            }
        }
        __syncthreads();
    }
}

// Accepted ions (the first acc fired ones in slot order): Z + 1 (and a K
// vacancy when the valence shell is 1s) and a new electron at rest at the ion.
__global__ __launch_bounds__(BT) void k_big_apply3(BigArgs a)
{
    __shared__ int red[BT / 64];
    const StepArgs& s = a.s;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        const BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (!big_live(r, BN_FIRED)) continue;
        const int cb = a.ccnt[g];
        if (cb >= r.acc) continue;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        block_ordered_select<BT>(
            n, [&](int q) { return a.iflag[r.ip0 + base + q] != 0; },
            [&](int q, int pos) {
                const int rank = cb + pos;
                if (rank >= r.acc) return;
                const int i = base + q;
                const int64_t pi = r.io + i;
                const int z = s.iz[pi], kv = s.ik[pi];
                const int sv = valence(z, kv);
                s.iz[pi] = (uint8_t)(z + 1);
                if (sv == 0) s.ik[pi] = (uint8_t)(kv + 1);
                const int64_t pe = r.eo + r.ne0 + rank;
                s.ex[pe] = s.ix[pi];
                if (s.ey) s.ey[pe] = s.iy ? s.iy[pi] : 0.0;
                s.evx[pe] = 0.0;
                s.evy[pe] = 0.0;
                s.evz[pe] = 0.0;
                s.ew[pe] = 1;
            },
            red);
    }
}

// Drift-frame rescale of S3: electrons 0 .. ne0-1 by sqrt(1 - debit/K_th).
// (S4's rescale by sqrt(1 + E_add/K_th) is applied by k_big_emove as it
// stages the surviving electrons.)
__global__ __launch_bounds__(BT) void k_big_rescale(BigArgs a)
{
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_FIRED)) continue;
        if (!(r.debit > 0.0)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        const double ux = r.u[0], uy = r.u[1], uz = r.u[2], al = r.alpha;
        for (int j = threadIdx.x; j < n; j += BT) {
            s.evx[o + j] = ux + al * (s.evx[o + j] - ux);
            s.evy[o + j] = uy + al * (s.evy[o + j] - uy);
            s.evz[o + j] = uz + al * (s.evz[o + j] - uz);
        }
    }
}

// ---------------------------------------------------------------- S4

__global__ __launch_bounds__(BT) void k_big_s4part(BigArgs a)
{
    __shared__ double red[2 * (BIG_CH / 64)];
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (r.state) continue;
        const double ebulk = s.runs[r.run].e_bulk;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        long long wl = 0, bl = 0;
        // one pass: the weight sums ride on the bulk-energy tree (every leaf
        // j < n is visited once)
        const double ke = block_tree_sum<BT>(BIG_CH, [&](int j) {
            if (j >= n) return 0.0;
            const long long w = s.ew[o + j];
            wl += w;
            const double e = kin_at(s, o + j);
            if (e < ebulk) bl += w;
            return e < ebulk ? (double)w * e : 0.0;
        }, red);
        wl = block_isum<BT>(wl, ired);
        bl = block_isum<BT>(bl, ired);
        if (tid == 0) {
            a.part[0][g] = ke;
            atomicAdd(&r.we4, (unsigned long long)wl);
            atomicAdd(&r.wb4, (unsigned long long)bl);
        }
    }
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (r.state) continue;
        const int zf = s.runs[r.run].z_floor;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        const int64_t o = r.io + base;
        long long s1 = 0, el = 0;
        uint32_t ml = 0;
        for (int j = tid; j < n; j += BT) {
            const int z = s.iz[o + j];
            s1 += z;
            el += z > zf ? 1 : 0;
            ml |= 1u << z;
        }
        s1 = block_isum<BT>(s1, ired);
        el = block_isum<BT>(el, ired);
        if (ml) atomicOr(&r.zmask4, ml);
        if (tid == 0) {
            atomicAdd(&r.sz4, (unsigned long long)s1);
            atomicAdd(&r.nelig, (unsigned long long)el);
        }
    }
}

__global__ __launch_bounds__(BT) void k_big_s4fin(BigArgs a)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    __shared__ double tps;
    __shared__ int any, clamped;
    const StepArgs& s = a.s;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (r.state) continue;
        const int ne = r.ne, ni = r.ni;
        if (ne < 1 || ni < 1) continue;
        const xp_run& R = s.runs[r.run];
        const double ker = block_tree_sum<BT>(r.nce, [&](int j) { return a.part[0][r.ce0 + j]; }, red);
        if (threadIdx.x == 0) {
            const long long wbr = (long long)r.wb4;
            double tp = 0.01;
            if (wbr > 0) {
                tp = (2.0 * ker) / (3.0 * (double)wbr);
                if (tp < 0.01) tp = 0.01;
            }
            r.mom[15] = tp;
            tps = tp;
            any = 0;
            clamped = 0;
            if (!(s.flags & XP_REC_XS)) {
                const double n_i = ((double)ni * R.w0) / R.volume;
                const double zeos = eos_zbar(s.tab, n_i, tp);
                const double dd = (double)(long long)r.sz4 - (double)ni * zeos;
                if (dd > 0.0) {
                    long long nrec = (long long)floor(dd + 0.5);
                    if (nrec > (long long)r.nelig) nrec = (long long)r.nelig;
                    if (nrec > ne) nrec = ne;
                    if (nrec > 0) {
                        r.nrec = (int32_t)nrec;
                        r.need |= BN_REC;
                        r.ws = 0;
                    }
                }
            }
        }
        __syncthreads();
        if (s.flags & XP_REC_XS) {
            // per charge state held by an ion: the recombination probability
            // at the temperature and electron density after S3; the ions
            // draw in k_big_recfire
            const double tp = tps;
            const double ne4 = ((double)(long long)r.we4 * R.w0) / R.volume;
            const int zf = R.z_floor;
            const int z = threadIdx.x;
            if (z < 14) {
                double pz = 0.0;
                if ((r.zmask4 & (1u << z)) && z > zf && z >= 1) {
                    pz = rec_xs_prob(s.tab, z, tp, ne4, r.mom + 16, R.dt);
                    if (pz > 1.0) {
                        pz = 1.0;
                        atomicAdd(&clamped, 1);
                    }
                }
                r.prz[z] = pz;
                if (pz > 0.0) atomicOr(&any, 1);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                r.cnt[XP_C_P_CLAMPED] += clamped;
                if (any) {
                    r.need |= BN_REC;
                    r.ws = 0;
                }
            }
            __syncthreads();
        }
    }
}

// XP_REC_XS: every ion with Z > z_floor draws U32(word 0 of its REC_XS call)
// against the probability of its charge state; the firing ions per chunk go
// to ccnt (scanned per cell by k_big_cscan mode 3).
__global__ __launch_bounds__(BT) void k_big_recfire(BigArgs a)
{
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (!big_live(r, BN_REC)) continue;
        const int zf = s.runs[r.run].z_floor;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        long long c = 0;
        for (int q = tid; q < n; q += BT) {
            const int i = base + q;
            const int z = s.iz[r.io + i];
            bool f = false;
            if (z > zf && r.prz[z] > 0.0) f = u32(draw(s, r, (uint32_t)i, RP_REC_XS, 0).x0) < r.prz[z];
            a.iflag[r.ip0 + i] = f ? 1 : 0;
            c += f ? 1 : 0;
        }
        c = block_isum<BT>(c, ired);
        if (tid == 0) a.ccnt[g] = (int32_t)c;
    }
}

// XP_REC_XS: the firing ions in slot order, sel[ip0 + rank] for ranks below
// the cell's recombination count.
__global__ __launch_bounds__(BT) void k_big_recfirelist(BigArgs a)
{
    __shared__ int red[BT / 64];
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        const BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (!big_live(r, BN_REC)) continue;
        const int cb = a.ccnt[g];
        if (cb >= r.nrec) continue;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        block_ordered_select<BT>(
            n, [&](int q) { return a.iflag[r.ip0 + base + q] != 0; },
            [&](int q, int pos) {
                if (cb + pos < r.nrec) a.sel[r.ip0 + cb + pos] = base + q;
            },
            red);
    }
}

// Reduced weights: every electron's weight in slot order (coalesced copy),
// then k_big_wpdec takes one unit from the electrons of the first nrec REC_E
// ranks (nrec random writes instead of one per electron).
__global__ __launch_bounds__(BT) void k_big_wp(BigArgs a)
{
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_REC)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        for (int j = threadIdx.x; j < n; j += BT) a.wp[r.ep0 + base + j] = s.ew[r.eo + base + j];
    }
}

__global__ __launch_bounds__(BT) void k_big_wpdec(BigArgs a)
{
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_REC)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        if (base >= r.nrec) continue;
        const int n = r.nrec - base < BIG_CH ? r.nrec - base : BIG_CH;
        const uint32_t* perm = a.val_a + r.ep0;
        for (int t = base + threadIdx.x; t < base + n; t += BT) a.wp[r.ep0 + perm[t]] -= 1u;
    }
}

// The recombinations of a cell paired rank by rank (ion sel[t], electron
// REC_E rank t), one thread per pair: the ion takes the electron's momentum
// and drops one charge state; the pair's energy (unit kinetic energy +
// lowered binding + ion kinetic energy change) goes to fip[ip0 + t] for the
// ordered sum of k_big_recsum.  Pairs touch distinct ions and electrons.
__global__ __launch_bounds__(BT) void k_big_recapply(BigArgs a)
{
    __shared__ double red[BT / 64];
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const double mi = tb->mass_ion;
    const double half_mi = (0.5 * mi) / QE;
    const double ratio = ME / mi;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (!big_live(r, BN_REC_APPLY)) continue;
        const int base = (g - r.ci0) * BIG_CH;
        if (base >= r.nrec) continue;
        const int n = r.nrec - base < BIG_CH ? r.nrec - base : BIG_CH;
        const double* dE = r.mom + 16;
        const uint32_t* pe = a.val_a + r.ep0;
        double bind = 0.0;
        for (int t = base + threadIdx.x; t < base + n; t += BT) {
            const int64_t e = r.eo + pe[t];
            const int64_t i = r.io + a.sel[r.ip0 + t];
            const double keu = kin_at(s, e);
            const double vx = s.ivx[i], vy = s.ivy[i], vz = s.ivz[i];
            const double kib = half_mi * ((vx * vx + vy * vy) + vz * vz);
            const double nx = vx + ratio * s.evx[e];
            const double ny = vy + ratio * s.evy[e];
            const double nz = vz + ratio * s.evz[e];
            s.ivx[i] = nx;
            s.ivy[i] = ny;
            s.ivz[i] = nz;
            const double kia = half_mi * ((nx * nx + ny * ny) + nz * nz);
            const int z = s.iz[i], kv = s.ik[i];
            const Occ o0 = occupancy(z, kv);
            const int kn = (kv >= 1 && o0.s[1] + o0.s[2] == 8) ? kv - 1 : kv;
            const Occ o1 = occupancy(z - 1, kn);
            int sl = 0;
            for (int q = 0; q < 5; ++q)
                if (o1.s[q] > o0.s[q]) { sl = q; break; }
            const double ipr = lowered(tb, z - 1, sl, dE);
            s.iz[i] = (uint8_t)(z - 1);
            s.ik[i] = (uint8_t)kn;
            a.fip[r.ip0 + t] = (keu + ipr) + (kib - kia);
            bind = bind + ipr;
        }
        // the released bindings are a tally (any order)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) bind += __shfl_xor(bind, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bind;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < BT / 64; ++w) t += red[w];
            if (t != 0.0) atomicAdd(&r.led[XP_L_REC_BIND], t);
        }
        __syncthreads();
    }
}

// One wave per cell: K_th of the reduced population (canonical sum of the
// chunk partials); with K_th > 0 the recombination can be applied.
__global__ __launch_bounds__(64) void k_big_recfin(BigArgs a)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    const int lane = threadIdx.x;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, BN_REC)) continue;
        const long long ws = (long long)r.ws;
        double kth = 0.0;
        if (ws != 0) kth = block_tree_sum<64>(r.nce, [&](int j) { return a.part[0][r.ce0 + j]; }, red);
        if (lane == 0) {
            r.kth = kth;
            if (ws == 0 || !(kth > 0.0)) r.cnt[XP_C_REC_SKIPPED] += 1;
            else r.need |= BN_REC_APPLY;
        }
        __syncthreads();
    }
}

// One wave per cell: the pairs' energies summed left to right in pair order,
// then the rescale factor of the remaining electrons.  The terms pass through
// LDS 512 at a time; the wave's loads of the next 512 are in flight while
// lane 0 adds the current ones, and lane 0 reads each group of eight terms
// before adding the previous eight, so the sum waits on its additions only.
__global__ __launch_bounds__(64) void k_big_recsum(BigArgs a)
{
    constexpr int SPAN = 512, PER = SPAN / 64;
    __shared__ double v[SPAN + 8];
    const int lane = threadIdx.x;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, BN_REC_APPLY)) continue;
        const int nr = r.nrec;
        const double* term = a.fip + r.ip0;
        double eadd = 0.0;
        double nxt[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = lane + 64 * u;
            nxt[u] = q < nr ? term[q] : 0.0;
        }
        for (int t0 = 0; t0 < nr; t0 += SPAN) {
            const int cnt = nr - t0 < SPAN ? nr - t0 : SPAN;
#pragma unroll
            for (int u = 0; u < PER; ++u) v[lane + 64 * u] = nxt[u];
            if (lane < 8) v[SPAN + lane] = 0.0;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int q = t0 + SPAN + lane + 64 * u;
                nxt[u] = q < nr ? term[q] : 0.0;
            }
            if (lane == 0) {
                int q = 0;
                if (cnt >= 8) {
                    double cur[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) cur[u] = v[u];
                    for (; q + 8 <= cnt; q += 8) {
                        // v[q + 8 .. q + 15] lies within the padded buffer
                        double nx[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) nx[u] = v[q + 8 + u];
#pragma unroll
                        for (int u = 0; u < 8; ++u) eadd = eadd + cur[u];
#pragma unroll
                        for (int u = 0; u < 8; ++u) cur[u] = nx[u];
                    }
                }
                for (; q < cnt; ++q) eadd = eadd + v[q];
            }
            __syncthreads();
        }
        if (lane == 0) {
            r.cnt[XP_C_REC] += nr;
            r.led[XP_L_REC_ADD] += eadd;
            r.alpha = sqrt(1.0 + eadd / r.kth);
        }
        __syncthreads();
    }
}

// Stable removal of the electrons whose reduced weight (wp) reached zero,
// chunk-parallel and out of place: k_big_ecount counts the survivors of each
// electron chunk (into hist), k_big_escan turns the counts into per-cell
// offsets, k_big_emove stages each survivor at its final rank with its reduced
// weight and its velocity rescaled in the drift frame by sqrt(1 + E_add/K_th)
// (x, y in gev[0], gev[1]; vx, vy, vz, w in ev4) and k_big_eback copies the
// staged survivors to the front of the cell's slab.  Survivors keep their
// order.
__global__ __launch_bounds__(BT) void k_big_ecount(BigArgs a)
{
    __shared__ long long ired[BT / 64];
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    uint32_t* cnt = a.hist;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_REC_APPLY)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        long long c = 0;
        for (int j = threadIdx.x; j < n; j += BT) c += a.wp[r.ep0 + base + j] > 0 ? 1 : 0;
        c = block_isum<BT>(c, ired);
        if (threadIdx.x == 0) cnt[g] = (uint32_t)c;
    }
}

__global__ __launch_bounds__(BT) void k_big_escan(BigArgs a)
{
    __shared__ uint32_t red[BT / 64];
    const int tid = threadIdx.x;
    const int nb = a.hdr->count;
    uint32_t* cnt = a.hist;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (!big_live(r, BN_REC_APPLY)) continue;
        uint32_t carry = 0;
        for (int k0 = 0; k0 < r.nce; k0 += BT) {
            const int k = k0 + tid;
            const uint32_t v = k < r.nce ? cnt[r.ce0 + k] : 0u;
            uint32_t tot;
            const uint32_t ex = block_exclusive_sum<BT, uint32_t>(v, red, tot);
            if (k < r.nce) cnt[r.ce0 + k] = carry + ex;
            carry += tot;
        }
        if (tid == 0) {
            r.cnt[XP_C_E_REMOVED] += r.ne - (int32_t)carry;
            r.nkeep = (int32_t)carry;   // r.ne follows in k_big_efin
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BT) void k_big_emove(BigArgs a)
{
    __shared__ int red[BT / 64];
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    const uint32_t* off = a.hist;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_REC_APPLY)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        const uint32_t* wp = a.wp + r.ep0 + base;
        const double ux = r.u[0], uy = r.u[1], uz = r.u[2], al = r.alpha;
        int out = (int)off[g];
        for (int c0 = 0; c0 < n; c0 += BT) {
            const int j = c0 + threadIdx.x;
            const uint32_t w = j < n ? wp[j] : 0u;
            const bool alive = w > 0;
            int tot;
            const int ex = block_exclusive_sum<BT, int>(alive ? 1 : 0, red, tot);
            if (alive) {
                const int64_t d = r.ep0 + out + ex;
                a.gev[0][d] = s.ex[o + j];
                a.gev[1][d] = s.ey ? s.ey[o + j] : 0.0;
                double* rec = a.ev4 + 4 * d;
                const double vx = ux + al * (s.evx[o + j] - ux);
                const double vy = uy + al * (s.evy[o + j] - uy);
                const double vz = uz + al * (s.evz[o + j] - uz);
                *(double2*)rec = make_double2(vx, vy);
                *(double2*)(rec + 2) = make_double2(vz, (double)w);
            }
            out += tot;
        }
    }
}

__global__ __launch_bounds__(BT) void k_big_eback(BigArgs a)
{
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (!big_live(r, BN_REC_APPLY)) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int keep = r.nkeep;
        const int n = keep - base < BIG_CH ? keep - base : BIG_CH;
        const int64_t o = r.eo + base;
        for (int j = threadIdx.x; j < n; j += BT) {
            const int64_t d = r.ep0 + base + j;
            s.ex[o + j] = a.gev[0][d];
            if (s.ey) s.ey[o + j] = a.gev[1][d];
            const double* rec = a.ev4 + 4 * d;
            const double2 xy = *(const double2*)rec, zw = *(const double2*)(rec + 2);
            s.evx[o + j] = xy.x;
            s.evy[o + j] = xy.y;
            s.evz[o + j] = zw.x;
            s.ew[o + j] = (uint32_t)zw.y;
        }
    }
}

// Survivor count of the cells whose electrons were compacted.
__global__ __launch_bounds__(64) void k_big_efin(BigArgs a)
{
    const int nb = a.hdr->count;
    for (int b = blockIdx.x * 64 + threadIdx.x; b < nb; b += gridDim.x * 64) {
        BigRec& r = a.rec[b];
        if (big_live(r, BN_REC_APPLY)) r.ne = r.nkeep;
    }
}

// ---------------------------------------------------------------- S5

// Decisions per ion from its pre-S5 state (K-vacancy decay, then the photo
// events of 1s, 2s, 2p): new Z and k in place, the emission record in iaux
// (bit 0 Auger, bits 1..3 photo 1s 2s 2p, bins at 4 + 4 s, Z0 at 16, k0 at 24)
// and the electrons per chunk in ccnt.
__global__ __launch_bounds__(BT) void k_big_s5a(BigArgs a)
{
    __shared__ int cnt[XP_NCOUNT];
    __shared__ int kz[14];
    __shared__ double led[XP_NLEDGER];
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const uint32_t flags = s.flags;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (r.state) continue;
        const xp_run& R = s.runs[r.run];
        for (int q = tid; q < XP_NCOUNT; q += BT) cnt[q] = 0;
        for (int q = tid; q < XP_NLEDGER; q += BT) led[q] = 0.0;
        for (int q = tid; q < 14; q += BT) kz[q] = 0;
        __syncthreads();
        const int nbins = R.n_bins;
        const bool photo = (flags & XP_PHOTO) && nbins > 0;
        const double* nhv = (R.field_per_cell && s.cell_nhv) ? s.cell_nhv + (size_t)r.cell * XP_MAX_BINS : R.nhv;
        const double dtr = R.dt_rad;
        const double* dE = r.mom + 16;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        long long newe = 0, npf = 0;
        for (int q = tid; q < n; q += BT) {
            const int i = base + q;
            const int64_t pi = r.io + i;
            const int z0 = s.iz[pi], k0 = s.ik[pi];
            uint32_t mask = 0, bins = 0, pf = 0, dec = 0;
            if (z0 < 13) {
                const Occ o0 = occupancy(z0, k0);
                const int nl0 = o0.s[1] + o0.s[2];
                int z = z0, kv = k0;
                if ((flags & XP_DECAY) && k0 >= 1 && nl0 >= 1) {
                    const double ga = tb->gamma_a[z0][k0], gx = tb->gamma_x[z0][k0];
                    const double rate = ga + gx;
                    if (rate > 0.0) {
                        const Words d = draw(s, r, (uint32_t)i, RP_DECAY, 0);
                        double pd = dtr * rate;
                        if (pd > 1.0) {
                            pd = 1.0;
                            atomicAdd(&cnt[XP_C_P_CLAMPED], 1);
                        }
                        if (u52(d.x0, d.x1) < pd) {
                            kv = k0 - 1;
                            dec = 1;
                            atomicAdd(&cnt[XP_C_DECAY], 1);
                            if (nl0 >= 2 && u52(d.x2, d.x3) < ga / rate) {
                                z = z0 + 1;
                                mask |= 1u;
                                atomicAdd(&cnt[XP_C_AUGER], 1);
                            } else {
                                atomicAdd(&cnt[XP_C_KALPHA], 1);
                                atomicAdd(&led[XP_L_KALPHA], tb->e_kalpha[z0]);
                                if (flags & XP_KA_FIELD) atomicAdd(&kz[z0], 1);
                            }
                        }
                    }
                }
                if (photo) {
                    const Words fw = draw(s, r, (uint32_t)i, RP_ION, 0);
                    const uint32_t fire[3] = {fw.x1, fw.x2, fw.x3};
                    for (int sh = 0; sh < 3; ++sh) {
                        if (o0.s[sh] <= 0) continue;
                        const double sum = r.ssum[z0][sh];
                        if (!(sum > 0.0)) continue;
                        double p = ((CLIGHT * dtr) * (double)o0.s[sh]) * sum;
                        if (p > 1.0) {
                            p = 1.0;
                            atomicAdd(&cnt[XP_C_P_CLAMPED], 1);
                        }
                        if (!(u32(fire[sh]) < p)) continue;
                        pf |= 1u << sh;
                        const Occ on = occupancy(z, kv);
                        if (z >= 13 || on.s[sh] <= 0) {
                            atomicAdd(&cnt[XP_C_PHOTO_SKIPPED], 1);
                            continue;
                        }
                        const double pp = lowered(tb, z0, sh, dE);
                        const Words d = draw(s, r, (uint32_t)i, RP_BIN, (uint32_t)sh);
                        const int sel = photo_bin(R.hv, nhv, r.sig, nbins, sh, pp, u52(d.x0, d.x1) * sum);
                        z = z + 1;
                        if (sh == 0) kv = kv + 1;
                        mask |= 2u << sh;
                        bins |= (uint32_t)sel << (4 * sh);
                        atomicAdd(&cnt[XP_C_PHOTO_1S + sh], 1);
                    }
                }
                s.iz[pi] = (uint8_t)z;
                s.ik[pi] = (uint8_t)kv;
            }
            a.iaux[r.ip0 + i] = mask | (bins << 4) | ((uint32_t)z0 << 16) | ((uint32_t)k0 << 24);
            newe += __popc(mask);
            if (flags & XP_PHOTO_FRAC) {
                // the photo candidates and the decay, for k_big_s5fix
                a.iflag[r.ip0 + i] = (uint8_t)(pf | (dec << 3));
                npf += __popc(pf);
            }
        }
        newe = block_isum<BT>(newe, ired);
        if (tid == 0) a.ccnt[g] = (int32_t)newe;
        if (flags & XP_PHOTO_FRAC) {
            npf = block_isum<BT>(npf, ired);
            if (tid == 0 && npf) atomicAdd(&r.np5, (int32_t)npf);
        }
        if (flags & XP_KA_FIELD)
            for (int q = tid; q < 13; q += BT)
                if (kz[q]) atomicAdd(&r.kz[q], kz[q]);
        flush_counts(r, cnt, led);
        __syncthreads();
    }
}

// XP_KA_FIELD: the K-alpha photons a cell returns to the field.  XP_PHOTO_FRAC:
// when a cell's photo candidates outnumber the smallest whole budget of its
// bins, one lane takes its ions again in slot order with the budget (as the
// LDS step does), rewriting their Z, k, emission records and the electrons
// per chunk, and corrects the photo counters.
__global__ __launch_bounds__(64) void k_big_s5fix(BigArgs a)
{
    __shared__ double bud[XP_MAX_BINS], used[XP_MAX_BINS];
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const uint32_t flags = s.flags;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (r.state || threadIdx.x != 0) continue;
        const xp_run& R = s.runs[r.run];
        const int nbins = R.n_bins;
        if (flags & XP_KA_FIELD)
            for (int z0 = 0; z0 < 13; ++z0)
                if (r.kz[z0] && kalpha_bin(R.hv, nbins, tb->e_kalpha[z0]) >= 0) r.cnt[XP_C_KA_FIELD] += r.kz[z0];
        if (!(flags & XP_PHOTO_FRAC) || !(flags & XP_PHOTO) || nbins <= 0) continue;
        const double* nhv = (R.field_per_cell && s.cell_nhv) ? s.cell_nhv + (size_t)r.cell * XP_MAX_BINS : R.nhv;
        double mmin = 1e300;
        for (int bq = 0; bq < nbins; ++bq) {
            const double m = (nhv[bq] * R.volume) / R.w0;
            bud[bq] = m;
            used[bq] = 0.0;
            if (nhv[bq] > 0.0 && floor(m) < mmin) mmin = floor(m);
        }
        if (!((double)r.np5 > mmin)) continue;
        const double* dE = r.mom + 16;
        int dn[3] = {0, 0, 0}, dskip = 0, dst = 0, dpart = 0, chunk_new = 0;
        for (int i = 0; i < r.ni; ++i) {
            const uint32_t aux = a.iaux[r.ip0 + i];
            const uint32_t fl = a.iflag[r.ip0 + i];
            const uint32_t pfi = fl & 7u;
            if (pfi) {
                const int z0 = (aux >> 16) & 255u, k0 = (aux >> 24) & 255u;
                int z = z0 + (int)(aux & 1u), kv = k0 - (int)((fl >> 3) & 1u);
                const PhotoWalk w = photo_walk_ion(
                    [&](uint32_t pu, uint32_t sub) { return draw(s, r, (uint32_t)i, pu, sub); }, tb, R.hv, nhv, r.sig,
                    r.ssum, nbins, z0, pfi, dE, bud, used, z, kv);
                int old = 0;
                for (int q = 0; q < 3; ++q) {
                    const int f = (int)((aux >> (1 + q)) & 1u);
                    dn[q] += w.fired[q] - f;
                    old += f;
                }
                dskip += w.skipped - (__popc(pfi) - old);
                dst += w.starved;
                dpart += w.partial;
                a.iaux[r.ip0 + i] = (aux & 0xFFFF0001u) | w.mask | (w.bins << 4);
                s.iz[r.io + i] = (uint8_t)z;
                s.ik[r.io + i] = (uint8_t)kv;
                chunk_new += __popc((aux & 1u) | w.mask);
            } else {
                chunk_new += (int)(aux & 1u);
            }
            if (((i + 1) & (BIG_CH - 1)) == 0 || i + 1 == r.ni) {
                a.ccnt[r.ci0 + i / BIG_CH] = chunk_new;
                chunk_new = 0;
            }
        }
        for (int q = 0; q < 3; ++q) r.cnt[XP_C_PHOTO_1S + q] += dn[q];
        r.cnt[XP_C_PHOTO_SKIPPED] += dskip;
        r.cnt[XP_C_PHOTO_STARVED] += dst;
        r.cnt[XP_C_PHOTO_PARTIAL] += dpart;
    }
}

// New electrons of S5 in ion-slot order (per ion: Auger, photo 1s, 2s, 2p),
// isotropic with the energies of the decisions in iaux.
__global__ __launch_bounds__(BT) void k_big_s5b(BigArgs a)
{
    __shared__ int red[BT / 64];
    __shared__ double led[XP_NLEDGER];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const DevTables* tb = s.tab;
    const int nci = a.hdr->n_i_chunks;
    for (int g = blockIdx.x; g < nci; g += gridDim.x) {
        BigRec& r = a.rec[a.i_chunk_cell[g]];
        if (r.state || r.nnew5 == 0) continue;
        const xp_run& R = s.runs[r.run];
        for (int q = tid; q < XP_NLEDGER; q += BT) led[q] = 0.0;
        __syncthreads();
        const double* dE = r.mom + 16;
        const int base = (g - r.ci0) * BIG_CH;
        const int n = r.ni - base < BIG_CH ? r.ni - base : BIG_CH;
        int run_pos = r.ne + a.ccnt[g];
        for (int c0 = 0; c0 < n; c0 += BT) {
            const int q = c0 + tid;
            const uint32_t aux = q < n ? a.iaux[r.ip0 + base + q] : 0u;
            const uint32_t mask = aux & 15u;
            const int c = __popc(mask);
            int tot;
            const int ex = block_exclusive_sum<BT, int>(c, red, tot);
            int pos = run_pos + ex;
            if (c > 0) {
                const int i = base + q;
                const int64_t pi = r.io + i;
                const int z0 = (aux >> 16) & 255u, k0 = (aux >> 24) & 255u;
                const Occ o0 = occupancy(z0, k0);
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
                        atomicAdd(&led[XP_L_AUGER_E], en);
                    } else {
                        const int sh = bit - 1;
                        const int sel = (aux >> (4 + 4 * sh)) & 15u;
                        en = R.hv[sel] - lowered(tb, z0, sh, dE);
                        atomicAdd(&led[XP_L_PHOTO_E], en);
                        atomicAdd(&led[XP_L_PHOTON_ABS], R.hv[sel]);
                        if (s.cell_nabs) atomicAdd(&r.nabs[sel], 1);
                    }
                    const Words d = draw(s, r, (uint32_t)i, RP_DIR, (uint32_t)bit);
                    const double mu = 2.0 * u52(d.x0, d.x1) - 1.0;
                    double sp, cp;
                    xsincos2pi((((uint64_t)d.x2 << 32) | d.x3) >> 12, sp, cp);
                    const double st = sqrt(1.0 - mu * mu);
                    const double sv = sqrt(en * TWO_QE_OVER_ME);
                    const int64_t pe = r.eo + pos;
                    s.evx[pe] = sv * (st * cp);
                    s.evy[pe] = sv * (st * sp);
                    s.evz[pe] = sv * mu;
                    s.ew[pe] = 1;
                    s.ex[pe] = s.ix[pi];
                    if (s.ey) s.ey[pe] = s.iy ? s.iy[pi] : 0.0;
                    ++pos;
                }
            }
            run_pos += tot;
        }
        __syncthreads();
        for (int q = tid; q < XP_NLEDGER; q += BT)
            if (led[q] != 0.0) atomicAdd(&r.led[q], led[q]);
        __syncthreads();
    }
}

// ----------------------------------- forced thermalization (variant, Sec. VI.C)
// The LDS step's thermalization over chunks: the cell's electrons now include
// the ones S5 appended; every sum is the chunked canonical sum.  The draws go
// to the rank-order velocity arrays (free after S2), indexed by population.

__global__ __launch_bounds__(64) void k_big_th0(BigArgs a)
{
    const int nb = a.hdr->count;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        BigRec& r = a.rec[b];
        if (r.state) continue;
        r.ne += r.nnew5;
        r.nnew5 = 0;
        r.tw = 0;
        r.tkeep = 0;
        r.tkin = r.tkth = r.tsig = 0.0;
        r.tbeta = 0.0;
        r.tq[0] = r.tq[1] = r.tq[2] = 0.0;
    }
}

// phase 0: weights, w E and w v of the velocities; 1: w E about the drift
// and the draws with their w v; 2: the draws about their mean and their w E.
__global__ __launch_bounds__(BT) void k_big_thpart(BigArgs a, int phase)
{
    __shared__ double red[2 * (BIG_CH / 64)];
    __shared__ long long ired[BT / 64];
    const int tid = threadIdx.x;
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (r.state || r.tkeep) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        const int64_t po = r.ep0 + base;
        const uint32_t* w = s.ew + o;
        if (phase == 0) {
            long long wl = 0;
            for (int j = tid; j < n; j += BT) wl += w[j];
            wl = block_isum<BT>(wl, ired);
            const double k = block_tree_sum<BT>(BIG_CH, [&](int j) {
                return j < n ? (double)w[j] * kin_at(s, o + j) : 0.0;
            }, red);
            if (tid == 0) {
                a.part[0][g] = k;
                if (wl) atomicAdd(&r.tw, (unsigned long long)wl);
            }
            const double* v3[3] = {s.evx + o, s.evy + o, s.evz + o};
            for (int d = 0; d < 3; ++d) {
                const double* v = v3[d];
                const double t = block_tree_sum<BT>(BIG_CH, [&](int j) {
                    return j < n ? (double)w[j] * v[j] : 0.0;
                }, red);
                if (tid == 0) a.part[1 + d][g] = t;
            }
        } else if (phase == 1) {
            const double ux = r.u[0], uy = r.u[1], uz = r.u[2], sig = r.tsig;
            const double k = block_tree_sum<BT>(BIG_CH, [&](int j) {
                if (j >= n) return 0.0;
                const double dx = s.evx[o + j] - ux, dy = s.evy[o + j] - uy, dz = s.evz[o + j] - uz;
                return (double)w[j] * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
            }, red);
            if (tid == 0) a.part[0][g] = k;
            for (int j = tid; j < n; j += BT) {
                double gx, gy, gz;
                therm_normals(draw(s, r, (uint32_t)(base + j), RP_THERM, 0), gx, gy, gz);
                a.gev[0][po + j] = sig * gx;
                a.gev[1][po + j] = sig * gy;
                a.gev[2][po + j] = sig * gz;
            }
            __syncthreads();
            for (int d = 0; d < 3; ++d) {
                const double* v = a.gev[d] + po;
                const double t = block_tree_sum<BT>(BIG_CH, [&](int j) {
                    return j < n ? (double)w[j] * v[j] : 0.0;
                }, red);
                if (tid == 0) a.part[1 + d][g] = t;
            }
        } else {
            const double qx = r.tq[0], qy = r.tq[1], qz = r.tq[2];
            for (int j = tid; j < n; j += BT) {
                a.gev[0][po + j] = a.gev[0][po + j] - qx;
                a.gev[1][po + j] = a.gev[1][po + j] - qy;
                a.gev[2][po + j] = a.gev[2][po + j] - qz;
            }
            __syncthreads();
            const double k = block_tree_sum<BT>(BIG_CH, [&](int j) {
                if (j >= n) return 0.0;
                const double x = a.gev[0][po + j], y = a.gev[1][po + j], z = a.gev[2][po + j];
                return (double)w[j] * (HALF_ME_OVER_QE * ((x * x + y * y) + z * z));
            }, red);
            if (tid == 0) a.part[0][g] = k;
        }
    }
}

// Per-cell ends of the phases: drift velocity, temperature and spread; the
// drift-frame energy and the draws' mean; the scale of the draws.
__global__ __launch_bounds__(BT) void k_big_thfin(BigArgs a, int phase)
{
    __shared__ double red[2 * (BIG_MAX_CHUNKS / 64)];
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        BigRec& r = a.rec[b];
        if (r.state || r.tkeep) continue;
        const long long ws = (long long)r.tw;
        if (phase == 0 && (r.ne < 2 || ws <= 0)) {
            if (threadIdx.x == 0) {
                r.tkeep = 1;
                r.cnt[XP_C_THERM_SKIPPED] += 1;
            }
            __syncthreads();
            continue;
        }
        const double w = (double)ws;
        const double k = block_tree_sum<BT>(r.nce, [&](int j) { return a.part[0][r.ce0 + j]; }, red);
        double m[3];
        if (phase < 2)
            for (int d = 0; d < 3; ++d)
                m[d] = block_tree_sum<BT>(r.nce, [&](int j) { return a.part[1 + d][r.ce0 + j]; }, red) / w;
        if (threadIdx.x == 0) {
            if (phase == 0) {
                r.tkin = k;
                r.u[0] = m[0]; r.u[1] = m[1]; r.u[2] = m[2];
                if (!(k > 0.0)) {
                    r.tkeep = 1;
                    r.cnt[XP_C_THERM_SKIPPED] += 1;
                } else {
                    r.tsig = sqrt(((2.0 * k) / (3.0 * w)) * (QE / ME));
                }
            } else if (phase == 1) {
                r.tkth = k;
                r.tq[0] = m[0]; r.tq[1] = m[1]; r.tq[2] = m[2];
                if (!(k > 0.0)) {
                    r.tkeep = 1;
                    r.cnt[XP_C_THERM_SKIPPED] += 1;
                }
            } else {
                // k is 0 only if every draw coincides: drift velocity for all
                if (k > 0.0) {
                    r.tbeta = sqrt(r.tkth / k);
                    r.cnt[XP_C_THERM] += 1;
                } else {
                    r.tkeep = 2;
                    r.cnt[XP_C_THERM_SKIPPED] += 1;
                }
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(BT) void k_big_thapply(BigArgs a)
{
    const StepArgs& s = a.s;
    const int nce = a.hdr->n_e_chunks;
    for (int g = blockIdx.x; g < nce; g += gridDim.x) {
        const BigRec& r = a.rec[a.e_chunk_cell[g]];
        if (r.state || r.tkeep == 1) continue;
        const int base = (g - r.ce0) * BIG_CH;
        const int n = r.epn - base < BIG_CH ? r.epn - base : BIG_CH;
        const int64_t o = r.eo + base;
        const int64_t po = r.ep0 + base;
        const double ux = r.u[0], uy = r.u[1], uz = r.u[2], be = r.tbeta;
        const bool drift_only = r.tkeep == 2;
        for (int j = threadIdx.x; j < n; j += BT) {
            s.evx[o + j] = drift_only ? ux : ux + be * a.gev[0][po + j];
            s.evy[o + j] = drift_only ? uy : uy + be * a.gev[1][po + j];
            s.evz[o + j] = drift_only ? uz : uz + be * a.gev[2][po + j];
        }
    }
}

// ---------------------------------------------------------------- commit

__global__ __launch_bounds__(64) void k_big_commit(BigArgs a)
{
    const StepArgs& s = a.s;
    const int nb = a.hdr->count;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const BigRec& r = a.rec[b];
        if (r.state) continue;
        const int cell = r.cell;
        const int ne = r.ne + r.nnew5;
        if (threadIdx.x == 0) {
            s.e_cnt[cell] = ne;
            if (s.stats) atomicMax(&s.stats[3], ne);
        }
        if (s.cell_cnt)
            for (int q = threadIdx.x; q < XP_NCOUNT; q += 64) s.cell_cnt[(size_t)cell * XP_NCOUNT + q] = r.cnt[q];
        if (s.cell_led)
            for (int q = threadIdx.x; q < XP_NLEDGER; q += 64) s.cell_led[(size_t)cell * XP_NLEDGER + q] = r.led[q];
        if (s.cell_mom)
            for (int q = threadIdx.x; q < XP_NMOM; q += 64) s.cell_mom[(size_t)cell * XP_NMOM + q] = r.mom[q];
        if (s.cell_nabs)
            for (int q = threadIdx.x; q < XP_MAX_BINS; q += 64)
                s.cell_nabs[(size_t)cell * XP_MAX_BINS + q] = r.nabs[q];
        if (s.cell_nka) {
            const xp_run& R = s.runs[r.run];
            for (int q = threadIdx.x; q < XP_MAX_BINS; q += 64)
                s.cell_nka[(size_t)cell * XP_MAX_BINS + q] =
                    (s.flags & XP_KA_FIELD) && q < R.n_bins ? kalpha_return(s.tab, R.hv, R.n_bins, r.kz, q) : 0.0;
        }
        if (s.run_cnt)
            for (int q = threadIdx.x; q < XP_NCOUNT; q += 64)
                if (r.cnt[q]) atomicAdd((unsigned long long*)&s.run_cnt[(size_t)r.run * XP_NCOUNT + q], (unsigned long long)r.cnt[q]);
        if (s.run_led)
            for (int q = threadIdx.x; q < XP_NLEDGER; q += 64)
                if (r.led[q] != 0.0) atomicAdd(&s.run_led[(size_t)r.run * XP_NLEDGER + q], r.led[q]);
    }
}

}  // namespace

// ---------------------------------------------------------------- host side

BigPlan big_plan(int32_t big_max, int64_t e_pop, int64_t i_pop)
{
    BigPlan p{};
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t bm = big_max > 0 ? big_max : 1;
    const int64_t ep = e_pop > 0 ? e_pop : 1, ip = i_pop > 0 ? i_pop : 1;
    p.e_chunks = (int32_t)(ep / BIG_CH + bm + 1);
    p.i_chunks = (int32_t)(ip / BIG_CH + bm + 1);
    const int64_t cmax = p.e_chunks > p.i_chunks ? p.e_chunks : p.i_chunks;
    const int64_t pmax = ep > ip ? ep : ip;
    size_t o = 0;
    p.list = o; o += up(4 * (size_t)bm);
    p.hdr = o; o += up(sizeof(BigHdr));
    p.rec = o; o += up(sizeof(BigRec) * (size_t)bm);
    p.e_chunk_cell = o; o += up(4 * (size_t)p.e_chunks);
    p.i_chunk_cell = o; o += up(4 * (size_t)p.i_chunks);
    p.part = o; o += 4 * up(8 * (size_t)p.e_chunks);
    p.key_a = o; o += up(4 * (size_t)ep);
    p.val_a = o; o += up(4 * (size_t)ep);
    p.key_b = o; o += up(4 * (size_t)pmax);
    p.val_b = o; o += up(4 * (size_t)pmax);
    p.key_c = o; o += up(4 * (size_t)ip);
    p.val_c = o; o += up(4 * (size_t)ip);
    p.hist = o; o += up(4 * 256 * (size_t)cmax);
    p.iflag = o; o += up((size_t)ip);
    p.ccnt = o; o += up(4 * (size_t)p.i_chunks);
    p.iaux = o; o += up(4 * (size_t)ip);
    p.wp = o; o += up(4 * (size_t)ep);
    p.sel = o; o += up(4 * (size_t)ip);
    p.fip = o; o += up(8 * (size_t)ip);
    p.gev = o; o += 3 * up(8 * (size_t)ep);
    p.gew = o; o += up(4 * (size_t)ep);
    p.giv = o; o += 3 * up(8 * (size_t)ip);
    p.giz = o; o += up((size_t)ip);
    p.partz = o; o += 13 * up(8 * (size_t)p.e_chunks);
    p.ev4 = o; o += up(32 * (size_t)ep);
    p.iv4 = o; o += up(32 * (size_t)ip);
    p.bytes = o;
    return p;
}

namespace {

// Four stable 8-bit radix passes over the words (key) with the slots (val);
// an even number of passes, so the result ends in key / val.
hipError_t big_radix(BigArgs& a, int species, int needbit, uint32_t* key, uint32_t* val, uint32_t* key2,
                     uint32_t* val2, unsigned gch, unsigned gcell, hipStream_t s, int sub)
{
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_big_rhist, dim3(gch), dim3(64), 0, s, a, species, needbit, shift, (const uint32_t*)key,
                           sub);
        hipLaunchKernelGGL(k_big_rscan, dim3(gcell), dim3(1024), 0, s, a, species, needbit, sub);
        hipLaunchKernelGGL(k_big_rscatter, dim3(gch), dim3(256), 0, s, a, species, needbit, shift,
                           (const uint32_t*)key, (const uint32_t*)val, key2, val2, sub);
        uint32_t* t = key; key = key2; key2 = t;
        t = val; val = val2; val2 = t;
    }
    return hipGetLastError();
}

hipError_t big_sort(BigArgs& a, int species, int needbit, uint32_t purpose, uint32_t* key,
                    uint32_t* val, uint32_t* key2, uint32_t* val2, unsigned gch, unsigned gcell,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_big_keys, dim3(gch), dim3(BT), 0, s, a, species, needbit, purpose, key, val);
    return big_radix(a, species, needbit, key, val, key2, val2, gch, gcell, s, 0);
}

// S4 ranks of every recombining cell (see k_sel_find): species 0 the REC_E
// ranks 0 .. nrec - 1 in val_a, species 1 the first nrec eligible ions of
// the REC_I order in sel.  The keys go to key_a / val_a (key_c / val_c), the
// candidates to key_b / val_b.
hipError_t big_select_ranks(BigArgs& a, int species, unsigned gch, unsigned gcell, hipStream_t s)
{
    uint32_t* key = species == 0 ? a.key_a : a.key_c;
    uint32_t* val = species == 0 ? a.val_a : a.val_c;
    hipLaunchKernelGGL(k_big_keys, dim3(gch), dim3(BT), 0, s, a, species, (int)BN_REC,
                       (uint32_t)(species == 0 ? RP_REC_E : RP_REC_I), key, val);
    hipLaunchKernelGGL(k_sel_hist, dim3(gch), dim3(64), 0, s, a, species);
    hipLaunchKernelGGL(k_sel_find, dim3(gcell), dim3(1024), 0, s, a, species);
    hipLaunchKernelGGL(k_sel_compact, dim3(gch), dim3(BT), 0, s, a, species);
    hipError_t e = big_radix(a, species, BN_REC, a.key_b, a.val_b, key, val, gch, gcell, s, 1);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_copy, dim3(gch), dim3(BT), 0, s, a, species);
    return hipGetLastError();
}

}  // namespace

hipError_t big_launch(BigArgs& a, bool all_cells, hipStream_t s)
{
    const int64_t cmax = a.e_chunks_max > a.i_chunks_max ? a.e_chunks_max : a.i_chunks_max;
    const int64_t want = a.grid > 0 ? a.grid : 4096;
    const unsigned gch = (unsigned)(cmax < want ? cmax : want);
    const unsigned gcell = (unsigned)(a.big_max < 1024 ? a.big_max : 1024);
    const uint32_t flags = a.s.flags;
    if (all_cells)
        hipLaunchKernelGGL(k_big_all, dim3((a.s.n_cells + 255) / 256 < 1024 ? (a.s.n_cells + 255) / 256 : 1024),
                           dim3(256), 0, s, a, a.s.n_cells);
    hipLaunchKernelGGL(k_big_init, dim3((gcell + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_big_plan, dim3(1), dim3(1024), 0, s, a, 0);
    hipLaunchKernelGGL(k_big_plan, dim3(1), dim3(1024), 0, s, a, 1);
    hipLaunchKernelGGL(k_big_s0, dim3(gch), dim3(BT), 0, s, a);
    hipLaunchKernelGGL(k_big_s0fin, dim3(gcell), dim3(BT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (flags & (XP_EE | XP_EI)) {
        if ((e = big_sort(a, 0, BN_PERM_E, RP_PERM_E, a.key_a, a.val_a, a.key_b, a.val_b, gch, gcell, s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_big_gather, dim3(gch), dim3(BT), 0, s, a, 0, 0);
        // scattering law: bit 0 Nanbu, bit 1 relativistic
        const int law = ((flags & XP_NANBU) ? 1 : 0) | ((flags & XP_REL) ? 2 : 0);
        if (flags & XP_EE) {
            switch (law) {
            case 0: hipLaunchKernelGGL(k_big_ee<0>, dim3(gch), dim3(BT), 0, s, a); break;
            case 1: hipLaunchKernelGGL(k_big_ee<1>, dim3(gch), dim3(BT), 0, s, a); break;
            case 2: hipLaunchKernelGGL(k_big_ee<2>, dim3(gch), dim3(BT), 0, s, a); break;
            default: hipLaunchKernelGGL(k_big_ee<3>, dim3(gch), dim3(BT), 0, s, a); break;
            }
        }
        if (flags & XP_EI) {
            if ((e = big_sort(a, 1, BN_EI, RP_PERM_I, a.key_c, a.val_c, a.key_b, a.val_b, gch, gcell, s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(k_big_gather, dim3(gch), dim3(BT), 0, s, a, 1, 0);
            switch (law) {
            case 0: hipLaunchKernelGGL(k_big_ei<0>, dim3(gch), dim3(BT), 0, s, a); break;
            case 1: hipLaunchKernelGGL(k_big_ei<1>, dim3(gch), dim3(BT), 0, s, a); break;
            case 2: hipLaunchKernelGGL(k_big_ei<2>, dim3(gch), dim3(BT), 0, s, a); break;
            default: hipLaunchKernelGGL(k_big_ei<3>, dim3(gch), dim3(BT), 0, s, a); break;
            }
            hipLaunchKernelGGL(k_big_gather, dim3(gch), dim3(BT), 0, s, a, 1, 1);
            hipLaunchKernelGGL(k_big_unstage, dim3(gch), dim3(BT), 0, s, a, 1);
        }
        hipLaunchKernelGGL(k_big_gather, dim3(gch), dim3(BT), 0, s, a, 0, 1);
        hipLaunchKernelGGL(k_big_unstage, dim3(gch), dim3(BT), 0, s, a, 0);
    }
    if (flags & XP_ION) {
        hipLaunchKernelGGL(k_big_lotz, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_s3p, dim3(gcell), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_fire, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_cscan, dim3(gcell), dim3(BT), 0, s, a, 0);
        hipLaunchKernelGGL(k_big_firelist, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_drift, dim3(gch), dim3(BT), 0, s, a, 0);
        hipLaunchKernelGGL(k_big_dfin, dim3(gcell), dim3(BT), 0, s, a, 0);
        hipLaunchKernelGGL(k_big_kth, dim3(gch), dim3(BT), 0, s, a, 0);
        hipLaunchKernelGGL(k_big_accept, dim3(gcell), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_big_apply3, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_rescale, dim3(gch), dim3(BT), 0, s, a);
    }
    if (flags & XP_REC) {
        hipLaunchKernelGGL(k_big_plan, dim3(1), dim3(1024), 0, s, a, 0);
        hipLaunchKernelGGL(k_big_s4part, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_s4fin, dim3(gcell), dim3(BT), 0, s, a);
        if (flags & XP_REC_XS) {
            // the ions by their own draws, in slot order
            hipLaunchKernelGGL(k_big_recfire, dim3(gch), dim3(BT), 0, s, a);
            hipLaunchKernelGGL(k_big_cscan, dim3(gcell), dim3(BT), 0, s, a, 3);
            hipLaunchKernelGGL(k_big_recfirelist, dim3(gch), dim3(BT), 0, s, a);
            if ((e = big_select_ranks(a, 0, gch, gcell, s)) != hipSuccess) return e;
        } else {
            if ((e = big_select_ranks(a, 1, gch, gcell, s)) != hipSuccess) return e;
            if ((e = big_select_ranks(a, 0, gch, gcell, s)) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_big_wp, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_wpdec, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_drift, dim3(gch), dim3(BT), 0, s, a, 1);
        hipLaunchKernelGGL(k_big_dfin, dim3(gcell), dim3(BT), 0, s, a, 1);
        hipLaunchKernelGGL(k_big_kth, dim3(gch), dim3(BT), 0, s, a, 1);
        hipLaunchKernelGGL(k_big_recfin, dim3(gcell), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_big_recapply, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_recsum, dim3(gcell), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_big_ecount, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_escan, dim3(gcell), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_emove, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_eback, dim3(gch), dim3(BT), 0, s, a);
        hipLaunchKernelGGL(k_big_efin, dim3((gcell + 63) / 64), dim3(64), 0, s, a);
    }
    if (flags & (XP_PHOTO | XP_DECAY)) {
        hipLaunchKernelGGL(k_big_s5a, dim3(gch), dim3(BT), 0, s, a);
        if (flags & (XP_PHOTO_FRAC | XP_KA_FIELD)) hipLaunchKernelGGL(k_big_s5fix, dim3(gcell), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_big_cscan, dim3(gcell), dim3(BT), 0, s, a, 2);
        hipLaunchKernelGGL(k_big_s5b, dim3(gch), dim3(BT), 0, s, a);
    }
    if (flags & XP_THERM) {
        hipLaunchKernelGGL(k_big_th0, dim3((gcell + 63) / 64), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_big_plan, dim3(1), dim3(1024), 0, s, a, 0);
        for (int ph = 0; ph < 3; ++ph) {
            hipLaunchKernelGGL(k_big_thpart, dim3(gch), dim3(BT), 0, s, a, ph);
            hipLaunchKernelGGL(k_big_thfin, dim3(gcell), dim3(BT), 0, s, a, ph);
        }
        hipLaunchKernelGGL(k_big_thapply, dim3(gch), dim3(BT), 0, s, a);
    }
    hipLaunchKernelGGL(k_big_commit, dim3(gcell), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace xpd
