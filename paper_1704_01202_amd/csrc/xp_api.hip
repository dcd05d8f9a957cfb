// C-ABI entry points of the library: context, table upload, argument checks,
// schedule choice and kernel launches.  No call synchronizes the stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "xp_kernels.h"

struct xp_ctx {
    int device;
    const xpd::DevTables* d_tables;
    bool tables_ready;
    size_t max_lds;               // dynamic LDS limit per workgroup
    int n_cu;                     // compute units
    std::vector<unsigned char> staging;
};

// Workspace of collide_ionize_step_static: one array per device, held by the
// loaded code object until the process ends.  In host code `scratch` only
// names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device when a context is created there.
static __device__ __align__(256) unsigned char scratch[XP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

thread_local std::string g_err;

xp_status fail(xp_status code, const std::string& msg)
{
    g_err = msg;
    return code;
}

xp_status hip_fail(hipError_t e, const char* what)
{
    return fail(XP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t table_layout(const xp_atomic_tables* t, size_t* off_lnsig, size_t* off_eos)
{
    size_t o = (sizeof(xpd::DevTables) + 255) & ~size_t(255);
    *off_lnsig = o;
    o += sizeof(double) * 5 * (size_t)t->photo_nh;
    o = (o + 255) & ~size_t(255);
    *off_eos = o;
    o += sizeof(double) * (size_t)t->eos_nn * (size_t)t->eos_nt;
    return (o + 255) & ~size_t(255);
}

bool finite_all(const double* p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

xp_status check_batch(const xp_ctx* ctx, const xp_batch* b)
{
    if (!ctx) return fail(XP_ERR_INVALID_ARG, "null context");
    if (!ctx->tables_ready) return fail(XP_ERR_NOT_INITIALIZED, "init_species has not been called");
    if (!b) return fail(XP_ERR_INVALID_ARG, "null batch");
    if (b->n_runs <= 0 || b->n_cells < 0) return fail(XP_ERR_INVALID_ARG, "batch needs n_runs > 0 and n_cells >= 0");
    if (!b->d_runs || !b->d_cell_run || !b->d_status) return fail(XP_ERR_INVALID_ARG, "batch run table, cell map or status is null");
    if (b->n_cells > 0 && (!b->d_e_off || !b->d_e_cap || !b->d_e_cnt || !b->d_i_off || !b->d_i_cap || !b->d_i_cnt))
        return fail(XP_ERR_INVALID_ARG, "batch slab arrays are null");
    if (b->e_slots > 0 && (!b->d_ex || !b->d_evx || !b->d_evy || !b->d_evz || !b->d_ew))
        return fail(XP_ERR_INVALID_ARG, "batch electron arrays are null");
    if (b->i_slots > 0 && (!b->d_ix || !b->d_ivx || !b->d_ivy || !b->d_ivz || !b->d_iz || !b->d_ik))
        return fail(XP_ERR_INVALID_ARG, "batch ion arrays are null");
    return XP_OK;
}

}  // namespace

extern "C" {

uint32_t xp_abi_version(void) { return XP_ABI_VERSION; }

const char* xp_last_error(void) { return g_err.c_str(); }

xp_status xp_ctx_create(xp_ctx** out, int32_t device_id)
{
    if (!out) return fail(XP_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device_id < 0 || device_id >= n) return fail(XP_ERR_INVALID_ARG, "device id out of range");
    if ((e = hipSetDevice(device_id)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    int lds = 0;
    if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device_id)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    xp_ctx* c = new xp_ctx();
    c->device = device_id;
    c->d_tables = nullptr;
    c->tables_ready = false;
    c->max_lds = (size_t)lds;
    int ncu = 0;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device_id)) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipDeviceGetAttribute");
    }
    c->n_cu = ncu > 0 ? ncu : 1;
    if (device_id < MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device_id]) {
            void* ptr = nullptr;
            if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) {
                delete c;
                return hip_fail(e, "hipGetSymbolAddress(scratch)");
            }
            g_scratch_ptr[device_id] = ptr;
        }
    }
    *out = c;
    return XP_OK;
}

void xp_ctx_destroy(xp_ctx* ctx) { delete ctx; }

size_t xp_table_bytes(const xp_atomic_tables* t)
{
    if (!t || t->photo_nh < 2 || t->eos_nn < 2 || t->eos_nt < 2) return 0;
    size_t a, b;
    return table_layout(t, &a, &b);
}

xp_status init_species(xp_ctx* ctx, const xp_atomic_tables* t, void* d_buf, size_t bytes, void* stream)
{
    if (!ctx || !t || !d_buf) return fail(XP_ERR_INVALID_ARG, "null context, tables or buffer");
    if (t->z_nuc != 13) return fail(XP_ERR_INVALID_ARG, "only Al (Z = 13) tables are supported");
    if (t->photo_nh < 2 || t->photo_nh > 512 || t->eos_nn < 2 || t->eos_nn > 256 || t->eos_nt < 2 || t->eos_nt > 1024)
        return fail(XP_ERR_INVALID_ARG, "table grid sizes out of range");
    if (!(t->photo_dlnhv > 0) || !(t->eos_dlnn > 0) || !(t->eos_dlnt > 0) || !(t->mass_ion > 0))
        return fail(XP_ERR_INVALID_ARG, "table spacings and ion mass must be positive");
    if (!t->bind || !t->lotz_a || !t->lotz_b || !t->lotz_c || !t->gamma_a || !t->gamma_x || !t->e_kalpha ||
        !t->photo_lnsig || !t->eos_zbar)
        return fail(XP_ERR_INVALID_ARG, "null table array");
    if (!finite_all(t->bind, 70) || !finite_all(t->gamma_a, 42) || !finite_all(t->gamma_x, 42) ||
        !finite_all(t->e_kalpha, 14) || !finite_all(t->photo_lnsig, 5 * (size_t)t->photo_nh) ||
        !finite_all(t->eos_zbar, (size_t)t->eos_nn * t->eos_nt) || !finite_all(t->lotz_a, 5) ||
        !finite_all(t->lotz_b, 5) || !finite_all(t->lotz_c, 5))
        return fail(XP_ERR_INVALID_ARG, "non-finite table value");
    size_t off_lnsig, off_eos;
    const size_t need = table_layout(t, &off_lnsig, &off_eos);
    if (bytes < need) return fail(XP_ERR_TOO_SMALL, "table buffer smaller than xp_table_bytes");
    ctx->staging.assign(need, 0);
    xpd::DevTables* h = (xpd::DevTables*)ctx->staging.data();
    std::memcpy(h->bind, t->bind, sizeof(h->bind));
    std::memcpy(h->lotz_a, t->lotz_a, sizeof(h->lotz_a));
    std::memcpy(h->lotz_b, t->lotz_b, sizeof(h->lotz_b));
    std::memcpy(h->lotz_c, t->lotz_c, sizeof(h->lotz_c));
    std::memcpy(h->gamma_a, t->gamma_a, sizeof(h->gamma_a));
    std::memcpy(h->gamma_x, t->gamma_x, sizeof(h->gamma_x));
    std::memcpy(h->e_kalpha, t->e_kalpha, sizeof(h->e_kalpha));
    h->mass_ion = t->mass_ion;
    h->photo_lnhv0 = t->photo_lnhv0;
    h->photo_dlnhv = t->photo_dlnhv;
    h->eos_lnn0 = t->eos_lnn0;
    h->eos_dlnn = t->eos_dlnn;
    h->eos_lnt0 = t->eos_lnt0;
    h->eos_dlnt = t->eos_dlnt;
    h->photo_nh = t->photo_nh;
    h->eos_nn = t->eos_nn;
    h->eos_nt = t->eos_nt;
    h->off_lnsig = (int64_t)off_lnsig;
    h->off_eos = (int64_t)off_eos;
    std::memcpy(ctx->staging.data() + off_lnsig, t->photo_lnsig, sizeof(double) * 5 * (size_t)t->photo_nh);
    std::memcpy(ctx->staging.data() + off_eos, t->eos_zbar, sizeof(double) * (size_t)t->eos_nn * t->eos_nt);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = hipMemcpyAsync(d_buf, ctx->staging.data(), need, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tables)");
    // the staging copy must outlive the transfer: keep it until the next call
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(tables)");
    ctx->d_tables = (const xpd::DevTables*)d_buf;
    ctx->tables_ready = true;
    return XP_OK;
}

size_t xp_work_bytes(int64_t ne, int64_t ni, int32_t n_cells, int32_t n_runs)
{
    (void)n_runs;
    const xpd::BinPlan p = xpd::bin_plan(ne, ni, n_cells);
    const size_t cells = (size_t)(n_cells > 0 ? n_cells : 1);
    return p.bytes > 8 * cells + 256 ? p.bytes : 8 * cells + 256;
}

xp_status bin_particles(xp_ctx* ctx, const xp_particles* in, xp_batch* b, const xp_capacity* cap,
                        int64_t* d_need, void* stream)
{
    xp_status st = check_batch(ctx, b);
    if (st != XP_OK) return st;
    if (!in || !cap || !d_need) return fail(XP_ERR_INVALID_ARG, "null particles, capacity rule or need buffer");
    if (in->ne < 0 || in->ni < 0 || in->ne >= (1ll << 32) || in->ni >= (1ll << 32))
        return fail(XP_ERR_UNSUPPORTED, "particle counts must be below 2^32 per species");
    if ((in->ne > 0 && (!in->d_ex || !in->d_evx || !in->d_evy || !in->d_evz || !in->d_ew)) ||
        (in->ni > 0 && (!in->d_ix || !in->d_ivx || !in->d_ivy || !in->d_ivz || !in->d_iz || !in->d_ik)))
        return fail(XP_ERR_INVALID_ARG, "null input particle array");
    if (b->n_runs > 1 && ((in->ne > 0 && !in->d_e_run) || (in->ni > 0 && !in->d_i_run)))
        return fail(XP_ERR_INVALID_ARG, "particle run maps are required for more than one run");
    if (cap->e_per_ion < 0 || cap->e_extra < 0) return fail(XP_ERR_INVALID_ARG, "negative capacity rule");
    if (!b->d_work || b->work_bytes < xp_work_bytes(in->ne, in->ni, b->n_cells, b->n_runs))
        return fail(XP_ERR_TOO_SMALL, "workspace smaller than xp_work_bytes");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int e_lds, i_lds;
    xpd::lds_limits(ctx->max_lds, &e_lds, &i_lds);
    e = xpd::bin_launch(in, b, cap, d_need, e_lds, i_lds, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bin_particles launch");
    return XP_OK;
}

// Workspace of the step: two deferral lists, the per-tier counters, then the
// global-memory path's buffers.
struct StepPlan {
    int32_t* lists[2];
    int32_t* counts;   // STEP_COUNTS: one per tier, the last for the big list
    double* run_sig;   // [n_runs][XP_MAX_BINS][3]
    char* big;         // BigPlan region (when the batch has big bounds)
    size_t bytes;
};

static size_t step_lists_bytes(int32_t n_cells)
{
    const size_t n = (size_t)(n_cells > 0 ? n_cells : 1);
    return (8 * n + 4 * xpd::STEP_COUNTS + 255) & ~size_t(255);
}

static size_t step_fixed_bytes(int32_t n_cells, int32_t n_runs)
{
    const size_t r = (size_t)(n_runs > 0 ? n_runs : 1);
    return step_lists_bytes(n_cells) + ((8 * XP_MAX_BINS * 3 * r + 255) & ~size_t(255));
}

static StepPlan step_plan(const xp_batch* b)
{
    StepPlan p;
    char* w = (char*)b->d_work;
    const size_t n = (size_t)(b->n_cells > 0 ? b->n_cells : 1);
    p.lists[0] = (int32_t*)w;
    p.lists[1] = (int32_t*)(w + 4 * n);
    p.counts = (int32_t*)(w + 8 * n);
    p.run_sig = (double*)(w + step_lists_bytes(b->n_cells));
    const size_t fixed = step_fixed_bytes(b->n_cells, b->n_runs);
    p.big = w + fixed;
    p.bytes = fixed;
    if (b->big_cells_max > 0)
        p.bytes += xpd::big_plan(b->big_cells_max, b->big_e_slots, b->big_i_slots).bytes;
    return p;
}

size_t xp_step_work_bytes(const xp_batch* b)
{
    if (!b) return 0;
    // diagnostics: 8 B per cell; transport_photons: one exit density per cell and bin
    const size_t cells = 8 * XP_MAX_BINS * (size_t)(b->n_cells > 0 ? b->n_cells : 1) + 256;
    const StepPlan p = step_plan(b);
    return p.bytes > cells ? p.bytes : cells;
}

xp_status xp_lds_limits(xp_ctx* ctx, int32_t* e_lds, int32_t* i_lds)
{
    if (!ctx || !e_lds || !i_lds) return fail(XP_ERR_INVALID_ARG, "null argument");
    int e, i;
    xpd::lds_limits(ctx->max_lds, &e, &i);
    *e_lds = e;
    *i_lds = i;
    return XP_OK;
}

static xp_status launch_step(xp_ctx* ctx, xp_batch* b, const xp_step_params* p, uint32_t flags, void* stream)
{
    xp_status st = check_batch(ctx, b);
    if (st != XP_OK) return st;
    if (!p) return fail(XP_ERR_INVALID_ARG, "null step parameters");
    if (b->n_cells == 0) return XP_OK;
    if (b->e_cap_max <= 0 || b->i_cap_max < 0) return fail(XP_ERR_INVALID_ARG, "batch e_cap_max / i_cap_max not set");
    if (p->schedule < 0 || p->schedule > 6) return fail(XP_ERR_INVALID_ARG, "unknown schedule");
    if (p->big_grid < 0 || p->big_grid > 65536) return fail(XP_ERR_INVALID_ARG, "big_grid out of range");
    if (b->big_cells_max < 0 || b->big_e_slots < 0 || b->big_i_slots < 0)
        return fail(XP_ERR_INVALID_ARG, "negative big-cell bounds");
    if (!b->d_work || b->work_bytes < xp_step_work_bytes(b))
        return fail(XP_ERR_TOO_SMALL, "workspace smaller than xp_step_work_bytes");
    const bool big_ok = b->big_cells_max > 0;
    const bool all_big = p->schedule == 3;
    if (all_big && (b->big_cells_max < b->n_cells || b->big_e_slots < b->e_slots || b->big_i_slots < b->i_slots))
        return fail(XP_ERR_TOO_SMALL, "schedule 3 needs big-cell bounds covering the whole batch");
    xpd::StepArgs a{};
    a.runs = b->d_runs;
    a.cell_run = b->d_cell_run;
    a.e_off = b->d_e_off;
    a.e_cap = b->d_e_cap;
    a.e_cnt = b->d_e_cnt;
    a.i_off = b->d_i_off;
    a.i_cnt = b->d_i_cnt;
    a.ex = b->d_ex; a.ey = b->d_ey; a.evx = b->d_evx; a.evy = b->d_evy; a.evz = b->d_evz; a.ew = b->d_ew;
    a.ix = b->d_ix; a.iy = b->d_iy; a.ivx = b->d_ivx; a.ivy = b->d_ivy; a.ivz = b->d_ivz;
    a.iz = b->d_iz; a.ik = b->d_ik;
    a.cell_nhv = b->d_cell_nhv;
    a.run_cnt = b->d_run_counters;
    a.run_led = b->d_run_ledger;
    a.cell_cnt = b->d_cell_counters;
    a.cell_led = b->d_cell_ledger;
    a.cell_mom = b->d_cell_moments;
    a.cell_nabs = b->d_cell_nabs;
    a.cell_nka = b->d_cell_nka;
    a.status = b->d_status;
    a.run_status = b->d_run_status;
    a.tab = ctx->d_tables;
    a.d_step = p->d_step;
    a.step = p->step;
    a.flags = flags;
    a.stats = b->d_stats;
    a.n_cells = b->n_cells;
    // LDS plans: ions up to min(i_cap_max, i_lds); electrons doubling from the
    // hint up to what fits beside them
    int e_lds, i_lds;
    xpd::lds_limits(ctx->max_lds, &e_lds, &i_lds);
    const int ci_plan = b->i_cap_max < 1 ? 1 : (b->i_cap_max < i_lds ? b->i_cap_max : i_lds);
    const size_t budget = xpd::lds_budget(ctx->max_lds);
    int ce_fit = 0;
    while (xpd::step_lds_bytes(ce_fit + 16, ci_plan) <= budget) ce_fit += 16;
    const int emax = b->e_cap_max;
    if (!big_ok && (emax > ce_fit || b->i_cap_max > i_lds))
        return fail(XP_ERR_UNSUPPORTED, "cells beyond one workgroup's LDS need the batch's big-cell bounds");
    const int ce_top = emax < ce_fit ? emax : ce_fit;
    a.lds_ci = ci_plan;
    const StepPlan plan = step_plan(b);
    xpd::BigArgs g{};
    if (big_ok) {
        const xpd::BigPlan bp = xpd::big_plan(b->big_cells_max, b->big_e_slots, b->big_i_slots);
        char* w = plan.big;
        g.list = (int32_t*)(w + bp.list);
        g.count = plan.counts + xpd::BIG_COUNT_SLOT;
        g.hdr = (xpd::BigHdr*)(w + bp.hdr);
        g.rec = (xpd::BigRec*)(w + bp.rec);
        g.e_chunk_cell = (int32_t*)(w + bp.e_chunk_cell);
        g.i_chunk_cell = (int32_t*)(w + bp.i_chunk_cell);
        const size_t part_stride = ((8 * (size_t)bp.e_chunks + 255) & ~size_t(255));
        for (int q = 0; q < 4; ++q) g.part[q] = (double*)(w + bp.part + q * part_stride);
        g.key_a = (uint32_t*)(w + bp.key_a);
        g.val_a = (uint32_t*)(w + bp.val_a);
        g.key_b = (uint32_t*)(w + bp.key_b);
        g.val_b = (uint32_t*)(w + bp.val_b);
        g.key_c = (uint32_t*)(w + bp.key_c);
        g.val_c = (uint32_t*)(w + bp.val_c);
        g.hist = (uint32_t*)(w + bp.hist);
        g.iflag = (uint8_t*)(w + bp.iflag);
        g.ccnt = (int32_t*)(w + bp.ccnt);
        g.iaux = (uint32_t*)(w + bp.iaux);
        g.wp = (uint32_t*)(w + bp.wp);
        g.sel = (int32_t*)(w + bp.sel);
        g.fip = (double*)(w + bp.fip);
        g.partz = (double*)(w + bp.partz);
        g.ev4 = (double*)(w + bp.ev4);
        g.iv4 = (double*)(w + bp.iv4);
        const size_t ev_stride = ((8 * (size_t)(b->big_e_slots > 0 ? b->big_e_slots : 1) + 255) & ~size_t(255));
        const size_t iv_stride = ((8 * (size_t)(b->big_i_slots > 0 ? b->big_i_slots : 1) + 255) & ~size_t(255));
        for (int q = 0; q < 3; ++q) {
            g.gev[q] = (double*)(w + bp.gev + q * ev_stride);
            g.giv[q] = (double*)(w + bp.giv + q * iv_stride);
        }
        g.gew = (uint32_t*)(w + bp.gew);
        g.giz = (uint8_t*)(w + bp.giz);
        g.big_max = b->big_cells_max;
        g.grid = p->big_grid;
        g.e_chunks_max = bp.e_chunks;
        g.i_chunks_max = bp.i_chunks;
        g.e_pop_max = b->big_e_slots;
        g.i_pop_max = b->big_i_slots;
        a.big_out = g.list;
        a.big_out_count = g.count;
        a.big_out_cap = b->big_cells_max;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(xpd::k_step_prep, dim3(1), dim3(64), 0, s, plan.counts, b->d_stats);
    a.run_sig = plan.run_sig;
    if (flags & XP_PHOTO) {
        const int nt = b->n_runs * XP_MAX_BINS * 3;
        hipLaunchKernelGGL(xpd::k_run_prep, dim3((nt + 255) / 256), dim3(256), 0, s, b->d_runs, b->n_runs,
                           ctx->d_tables, plan.run_sig);
    }
    if (!all_big) {
        // first plan: the hinted size plus headroom for this step's new electrons
        int ce = ce_top;
        if (p->e_hint > 0) {
            const int head = p->e_hint / 4 > 16 ? p->e_hint / 4 : 16;
            ce = p->e_hint + head;
            ce = ((ce + 15) / 16) * 16;
            if (ce > ce_top) ce = ce_top;
        }
        // the variants, per-cell records and per-cell photon fields are
        // compiled into their own kernels
        const bool xv = (flags & (XP_THERM | XP_ION_Z | XP_NANBU | XP_REL | XP_REC_XS | XP_PHOTO_FRAC |
                                  XP_KA_FIELD)) != 0 ||
                        b->d_cell_counters || b->d_cell_ledger || b->d_cell_moments || b->d_cell_nhv ||
                        b->d_cell_nabs || b->d_cell_nka;
        for (int tier = 0;; ++tier) {
            const bool last = ce >= ce_top || tier >= xpd::BIG_COUNT_SLOT - 1;
            a.lds_ce = ce;
            // ions: the whole batch's bound on the last plan, no more than the
            // electron plan before it (ion-heavy cells move on with the
            // electron-heavy ones)
            a.lds_ci = last || ce >= ci_plan ? ci_plan : ce;
            a.cell_list = tier == 0 ? nullptr : plan.lists[(tier - 1) & 1];
            a.cell_list_count = tier == 0 ? nullptr : plan.counts + (tier - 1);
            a.defer_out = last ? nullptr : plan.lists[tier & 1];
            a.defer_out_count = last ? nullptr : plan.counts + tier;
            const size_t lds1 = xpd::step_lds_bytes(a.lds_ce, a.lds_ci);
            const int m = a.lds_ce > a.lds_ci ? a.lds_ce : a.lds_ci;
            int sched = p->schedule;
            if (sched == 0) {
                // small plans: four cells per wave; a wave per cell while the
                // e-i rounds (at most one pair per ion slot) fit one wave and
                // the LDS of one cell still leaves a few waves per SIMD; a
                // block of four waves per cell for many ions or long slabs
                if (m <= 4 * 16) sched = 5;
                else sched = (a.lds_ci > 128 || a.lds_ce > 384) ? 2 : 1;
            }
            if (sched >= 4) {
                const int w = sched == 4 ? 32 : (sched == 5 ? 16 : 8);
                if (m > 4 * w) sched = m > 128 ? 2 : 1;   // plan too large for the group
            }
            // kernel instance: plain, extended, or extended with Nanbu's law
            const int level = (flags & XP_REL) ? 3 : ((flags & XP_NANBU) ? 2 : (xv ? 1 : 0));
            auto pick = [level](void (*k0)(xpd::StepArgs), void (*k1)(xpd::StepArgs),
                                void (*k2)(xpd::StepArgs), void (*k3)(xpd::StepArgs)) {
                return level == 3 ? (const void*)k3
                                  : (level == 2 ? (const void*)k2 : (level == 1 ? (const void*)k1 : (const void*)k0));
            };
            const void* fn;
            int threads = 64, per_cell_groups = 1;
            switch (sched) {
            case 1: fn = pick(xpd::k_step<64, 0>, xpd::k_step<64, 1>, xpd::k_step<64, 2>, xpd::k_step<64, 3>); break;
            case 2:
                fn = pick(xpd::k_step<256, 0>, xpd::k_step<256, 1>, xpd::k_step<256, 2>, xpd::k_step<256, 3>);
                threads = 256;
                break;
            case 4:
                fn = pick(xpd::k_step_g<32, 0>, xpd::k_step_g<32, 1>, xpd::k_step_g<32, 2>, xpd::k_step_g<32, 3>);
                per_cell_groups = 2;
                break;
            case 5:
                fn = pick(xpd::k_step_g<16, 0>, xpd::k_step_g<16, 1>, xpd::k_step_g<16, 2>, xpd::k_step_g<16, 3>);
                per_cell_groups = 4;
                break;
            default:
                fn = pick(xpd::k_step_g<8, 0>, xpd::k_step_g<8, 1>, xpd::k_step_g<8, 2>, xpd::k_step_g<8, 3>);
                per_cell_groups = 8;
                break;
            }
            const size_t lds = sched >= 4 ? (size_t)per_cell_groups * ((lds1 + 15) & ~size_t(15)) : lds1;
            if (lds > ctx->max_lds) return fail(XP_ERR_UNSUPPORTED, "LDS plan too large");
            if (lds > 65536) hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            // every tier: a few resident rounds of workgroups, each looping
            // over its cells (run records are summed per workgroup); tier 0
            // takes all cells, later tiers the cells deferred to them, read
            // from a list whose length only the device knows, so their grid
            // is sized for the whole batch and surplus workgroups exit at once
            const long long items = ((long long)b->n_cells + per_cell_groups - 1) / per_cell_groups;
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess || per_cu < 1)
                per_cu = 1;
            const long long g0 = 4ll * per_cu * ctx->n_cu;
            const unsigned grid = (unsigned)(items < g0 ? items : g0);
            void* kargs[] = {(void*)&a};
            e = hipLaunchKernel(fn, dim3(grid), dim3(threads), kargs, lds, s);
            if (e != hipSuccess) return hip_fail(e, "step launch");
            e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "step launch");
            if (last) break;
            ce = ce * 2 < ce_top ? ce * 2 : ce_top;
        }
    }
    if (big_ok) {
        g.s = a;
        e = xpd::big_launch(g, all_big, s);
        if (e != hipSuccess) return hip_fail(e, "global-memory step launch");
    }
    return XP_OK;
}

xp_status collide_ionize_step(xp_ctx* ctx, xp_batch* b, const xp_step_params* p, void* stream)
{
    if (!p) return fail(XP_ERR_INVALID_ARG, "null step parameters");
    return launch_step(ctx, b, p, p->flags & (XP_ALL | XP_THERM | XP_ION_Z | XP_NANBU | XP_REL | XP_REC_XS | XP_PHOTO_FRAC | XP_KA_FIELD), stream);
}

xp_status collide_ionize_step_static(xp_ctx* ctx, const xp_batch* b, const xp_step_params* p, void* stream)
{
    if (!ctx) return fail(XP_ERR_INVALID_ARG, "null context");
    if (!b) return fail(XP_ERR_INVALID_ARG, "null batch");
    if (!p) return fail(XP_ERR_INVALID_ARG, "null step parameters");
    const size_t need = xp_step_work_bytes(b);
    if (need > (size_t)XP_STATIC_SCRATCH_BYTES)
        return fail(XP_ERR_UNSUPPORTED, "the batch needs " + std::to_string(need) +
                                            " bytes of step workspace, more than the " +
                                            std::to_string((size_t)XP_STATIC_SCRATCH_BYTES) +
                                            " of the static scratch");
    void* ptr = nullptr;
    if (ctx->device >= 0 && ctx->device < MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ptr = g_scratch_ptr[ctx->device];
    }
    if (!ptr) return fail(XP_ERR_NOT_INITIALIZED, "no static scratch address for the context's device");
    xp_batch v = *b;
    v.d_work = ptr;
    v.work_bytes = (size_t)XP_STATIC_SCRATCH_BYTES;
    return launch_step(ctx, &v, p, p->flags & (XP_ALL | XP_THERM | XP_ION_Z | XP_NANBU | XP_REL | XP_REC_XS | XP_PHOTO_FRAC | XP_KA_FIELD), stream);
}

xp_status photo_auger_step(xp_ctx* ctx, xp_batch* b, const xp_step_params* p, void* stream)
{
    if (!p) return fail(XP_ERR_INVALID_ARG, "null step parameters");
    return launch_step(ctx, b, p, p->flags & (XP_PHOTO | XP_DECAY | XP_THERM | XP_PHOTO_FRAC | XP_KA_FIELD), stream);
}

xp_status diagnostics(xp_ctx* ctx, const xp_batch* b, xp_diag* d_out, uint32_t what, void* stream)
{
    xp_status st = check_batch(ctx, b);
    if (st != XP_OK) return st;
    if (!d_out) return fail(XP_ERR_INVALID_ARG, "null output");
    if ((int64_t)b->e_cap_max > (int64_t)xpd::DIAG_CHUNK * xpd::DIAG_MAX_CHUNKS)
        return fail(XP_ERR_UNSUPPORTED, "diagnostics support cells of up to 2^25 electron slots");
    if (!b->d_work || b->work_bytes < 8 * (size_t)(b->n_cells > 0 ? b->n_cells : 1))
        return fail(XP_ERR_TOO_SMALL, "workspace too small for diagnostics");
    xpd::DiagArgs a{};
    a.runs = b->d_runs;
    a.cell_run = b->d_cell_run;
    a.e_off = b->d_e_off;
    a.e_cnt = b->d_e_cnt;
    a.i_off = b->d_i_off;
    a.i_cnt = b->d_i_cnt;
    a.evx = b->d_evx; a.evy = b->d_evy; a.evz = b->d_evz; a.ew = b->d_ew;
    a.iz = b->d_iz;
    a.run_cnt = b->d_run_counters;
    a.run_led = b->d_run_ledger;
    a.cell_k = (double*)b->d_work;
    a.out = d_out;
    a.n_runs = b->n_runs;
    a.n_cells = b->n_cells;
    a.e_cap_max = b->e_cap_max;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = xpd::diag_launch(a, what, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
    return XP_OK;
}

xp_status transport_photons(xp_ctx* ctx, xp_batch* b, double* d_trans, void* stream)
{
    xp_status st = check_batch(ctx, b);
    if (st != XP_OK) return st;
    if (!b->d_cell_nhv || !b->d_cell_nabs)
        return fail(XP_ERR_INVALID_ARG, "transport_photons needs d_cell_nhv and d_cell_nabs");
    if (!b->d_work || b->work_bytes < xp_step_work_bytes(b))
        return fail(XP_ERR_TOO_SMALL, "workspace smaller than xp_step_work_bytes");
    xpd::TransportArgs a{};
    a.runs = b->d_runs;
    a.cell_run = b->d_cell_run;
    a.nhv = b->d_cell_nhv;
    a.nabs = b->d_cell_nabs;
    a.nka = b->d_cell_nka;
    a.exit = (double*)b->d_work;
    a.trans = d_trans;
    a.status = b->d_status;
    a.run_status = b->d_run_status;
    a.n_runs = b->n_runs;
    a.n_cells = b->n_cells;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = xpd::transport_launch(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "transport launch");
    return XP_OK;
}

xp_status xp_selftest(xp_ctx* ctx, int32_t which, int64_t n, const double* d_x, const uint64_t* d_u,
                      double* d_out, uint32_t* d_words, void* stream)
{
    if (!ctx) return fail(XP_ERR_INVALID_ARG, "null context");
    if (which < 0 || which > 9 || n < 0) return fail(XP_ERR_INVALID_ARG, "unknown self-test");
    if (which == 7 && n % 64 != 0) return fail(XP_ERR_INVALID_ARG, "tree self-test needs rows of 64");
    if (which == 8 && n % 256 != 0) return fail(XP_ERR_INVALID_ARG, "tree self-test needs rows of 256");
    if (which == 9 && n % 64 != 0) return fail(XP_ERR_INVALID_ARG, "tree self-test needs rows of 64");
    if (which >= 7 && n / 64 > 0x7fffffff) return fail(XP_ERR_INVALID_ARG, "too many rows");
    const bool need_x = which <= 2 || which >= 5;
    if ((need_x && !d_x) || ((which == 3 || which == 4) && !d_u) || (which != 4 && !d_out) ||
        (which == 4 && !d_words))
        return fail(XP_ERR_INVALID_ARG, "null self-test array");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = xpd::selftest_launch(which, n, d_x, d_u, d_out, d_words, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "self-test launch");
    return XP_OK;
}

}  // extern "C"
