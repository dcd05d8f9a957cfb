/*
 * xpic: per-cell Monte-Carlo collision / ionization step of the collisional
 * PIC method for XFEL-heated solid-density Al (Royle, Sentoku, Mancini,
 * Paraschiv, Johzaki, "Kinetic modeling of x-ray laser-driven solid Al plasmas
 * via particle-in-cell simulation"), on one AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every pointer named d_* is device memory owned by the caller; every
 * other pointer is host memory, read during the call only.  Streams are passed
 * as `void *` holding a hipStream_t (NULL = the null stream).  All calls that
 * take a stream only enqueue work on it and return without synchronizing,
 * except where stated.  Every call returns an xp_status: XP_OK, or a negative
 * code with a message available from xp_last_error() (thread-local).
 *
 * Conditions found on the device (a cell whose new electrons do not fit its
 * slot capacity, a non-finite velocity) are reported through the batch's
 * d_status word (bit mask XP_ST_*).  A cell stepped in LDS that cannot be
 * completed is left exactly as it was before the step; a cell stepped on the
 * global-memory path (see xp_step_params.schedule) keeps the collisions of that
 * step and skips its later stages.  Either way the batch needs re-binning with
 * more capacity before its results mean anything.  When the batch carries
 * d_run_status, each such bit is also OR-ed into the word of the run the cell
 * belongs to, so that each run sharing a batch reports its own condition.
 *
 * Units: SI for positions, velocities, volumes and densities; energies and
 * temperatures in eV; table cross sections in cm^2.
 */
#ifndef XPIC_H
#define XPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Layout version of the structs below; 2 added xp_batch.d_cell_nabs, 3 added
 * xp_batch.d_run_status, 4 added three counters and xp_batch.d_cell_nka. */
#define XP_ABI_VERSION 4u

typedef int32_t xp_status;
#define XP_OK                   0
#define XP_ERR_INVALID_ARG     -1   /* null or inconsistent argument */
#define XP_ERR_HIP             -2   /* a HIP runtime call failed */
#define XP_ERR_TOO_SMALL       -3   /* a caller buffer is smaller than required */
#define XP_ERR_NOT_INITIALIZED -4   /* init_species has not been called */
#define XP_ERR_UNSUPPORTED     -5   /* size beyond what the library supports */

/* Stage switches (xp_step_params.flags).  Order within a step is always
 * moments -> e-e -> e-i -> ionization -> recombination -> decay/photo
 * [-> forced thermalization]. */
#define XP_EE      0x01u   /* electron-electron binary collisions (Sec. IV) */
#define XP_EI      0x02u   /* electron-ion binary collisions (Sec. IV) */
#define XP_ION     0x04u   /* collisional ionization, Lotz (Sec. IV, Eq. 4) */
#define XP_REC     0x08u   /* three-body recombination to Zbar_EOS (Sec. IV) */
#define XP_PHOTO   0x10u   /* subshell photoionization (Sec. III, Eq. 3) */
#define XP_DECAY   0x20u   /* K-vacancy decay, KLL Auger or K-alpha (Sec. III) */
#define XP_ALL     0x3Fu
/* Variant, not part of XP_ALL: forced thermalization right after S5 (Sec. VI.C).
 * Every free electron of a cell gets a Maxwellian velocity at the cell
 * temperature kT = (2/3) E_ave of all free electrons; the draws' mean is
 * replaced by the cell's drift velocity and their spread scaled to the cell's
 * drift-frame energy before, so momentum and energy are unchanged.  One
 * Philox call per electron slot (purpose 12): Box-Muller on words 0, 1 gives
 * the x and y components, on words 2, 3 the z component.  Cells with fewer
 * than two electrons or no drift-frame energy keep their velocities. */
#define XP_THERM   0x40u
/* Variant, not part of XP_ALL: collisional ionization (S3) with the Lotz cross
 * section of every ion's own charge state instead of the average cell ion
 * (Sec. IV): for each charge state z < 13 held by an ion of the cell,
 * P_z = (w0 dt / V) sum_j w_j sigma(E_j; z) v_j (canonical sum, clamped at 1),
 * and an ion of charge z fires with its ION draw r < P_z.  Acceptance, energy
 * debit and rescale are those of S3.  Moments record: [11] the number of
 * charge states evaluated, [12] the largest P_z. */
#define XP_ION_Z   0x80u
/* Variant, not part of XP_ALL: Nanbu's cumulative scattering law (Nanbu,
 * Phys. Rev. E 55, 4642 (1997)) in the e-e and e-i collisions (Sec. IV cites
 * Monte-Carlo binary collisions without fixing the law).  Pairing, weights and
 * the rotation are those of Takizuka-Abe; the angle chi of one step has the
 * density of cos chi  A exp(A cos chi) / (2 sinh A) with coth A - 1/A =
 * exp(-s), s = 2 <delta^2>, drawn by inverting its distribution function at
 * U52(words 0, 1) of the pair's Philox call.  s >= 15 is isotropic.  Suited
 * to nu dt >> 1, where Takizuka-Abe's single small-angle step is out of its
 * range. */
#define XP_NANBU   0x100u
/* Variant, not part of XP_ALL: relativistic binary collisions in the e-e and
 * e-i stages (Sec. IV cites relativistic weighted binary collisions for the
 * code's collision model), after the centre-of-momentum-frame Monte-Carlo
 * collision of Perez et al. (Phys. Plasmas 19, 083104 (2012)).  Velocities
 * become momenta p = gamma m v, the pair is boosted to its centre-of-momentum
 * frame, p_a* is turned by the angle drawn from the relativistic scattering
 * parameter s (which tends to 2 <delta^2> of Takizuka-Abe for v << c) with
 * Takizuka-Abe's law at <delta^2> = s / 2, or with XP_NANBU Nanbu's law at s,
 * and both momenta are boosted back.  Pairing, draws and weighted acceptance
 * are unchanged; the other stages keep their non-relativistic energies. */
#define XP_REL     0x200u
/* Variant, not part of XP_ALL: three-body recombination (S4) from cross
 * sections instead of the EOS constraint (Sec. IV names it as the model's
 * next step).  The rate per ion of charge Z is the inverse of the Lotz
 * ionization of Z-1 by detailed balance: S_{Z-1}(T) n_e^2 / Phi_Z(T), S the
 * Maxwellian Lotz rate of the ground configuration of Z-1 with lowered
 * bindings (Eq. 4 and its exponential-integral closed form), Phi_Z the Saha
 * factor 2 (g_Z / g_{Z-1}) (m_e k T / (2 pi hbar^2))^{3/2} exp(-P_v / T) with
 * ground-configuration degeneracies g and the lowered valence binding P_v of
 * Z-1; T and n_e of the electrons after S3.  Each ion with Z > z_floor fires
 * when U32(word 0 of its Philox call, purpose 13) is below that probability
 * times dt (clamped at 1); the firing ions recombine in slot order with the
 * electrons of the REC_E permutation, at most one per electron, with S4's
 * energy bookkeeping and rescale. */
#define XP_REC_XS  0x400u

/* Variant of S5 (Sec. III, photoionization): a bin of the photon field can
 * give a cell no more photons than it holds, n_hv V real photons or
 * n_hv V / w0 macro-photons.  The photo events of a cell take one each in ion
 * order (1s, 2s, 2p within an ion) while one is left; the event that finds a
 * fraction f in (0, 1) left is a partial photoionization: the paper's
 * macro-photoelectron of weight f, with f of a unit of charge, which integer
 * weight units carry as an event of probability f (32-bit draw, word 0 of
 * the ion's call of purpose 14, sub = shell), after which the bin is spent;
 * later events of the bin do not happen (XP_C_PHOTO_STARVED).  Without it
 * every event takes its photon whatever the bin holds. */
#define XP_PHOTO_FRAC 0x800u

/* Variant of S5 (Sec. III, K-vacancy decay): the energy of a K-alpha photon
 * goes back into the photon field, to the bin of the largest h nu not above
 * E_Ka(Z0) (the lowest index among equal ones), as E_Ka / h nu photons of
 * that bin, so that energy is kept and no photon is promoted above its own
 * energy; with no such bin it leaves the plasma.  Per cell and bin the step
 * writes g_b = sum over Z0 ascending of (number of K-alpha photons of ions of
 * charge Z0 sent to b) * (E_Ka(Z0) / h nu_b), in macro-photons, to
 * d_cell_nka; transport_photons adds them to the beam leaving the cell.
 * The particle state is that of the step without it. */
#define XP_KA_FIELD   0x1000u

/* Device status bits (xp_batch.d_status, OR-ed by kernels). */
#define XP_ST_CAPACITY  0x1u   /* a cell needed more electron slots than its capacity */
#define XP_ST_NONFINITE 0x2u   /* a non-finite velocity was produced */
#define XP_ST_BIN_SIZE  0x4u   /* bin_particles: output capacity too small, nothing written */
#define XP_ST_RUN_TABLE 0x8u   /* transport_photons: a run's grid does not match its cell range;
                                  its rows were left as they were */

/* Per-cell event counters (indices into counter records). */
enum {
    XP_C_EE = 0, XP_C_EI, XP_C_TRIPLET, XP_C_ACCEPT, XP_C_U0, XP_C_DELTA2_GT1,
    XP_C_ION_FIRED, XP_C_ION_ACCEPTED, XP_C_ION_STARVED,
    XP_C_REC, XP_C_REC_SKIPPED, XP_C_E_REMOVED,
    XP_C_PHOTO_1S, XP_C_PHOTO_2S, XP_C_PHOTO_2P, XP_C_PHOTO_SKIPPED,
    XP_C_DECAY, XP_C_AUGER, XP_C_KALPHA,
    XP_C_P_CLAMPED, XP_C_IPD_CLAMPED, XP_C_E_NEW,
    XP_C_THERM, XP_C_THERM_SKIPPED,   /* cells thermalized / left as they were (XP_THERM) */
    XP_C_PHOTO_STARVED,   /* photo events whose bin was spent (XP_PHOTO_FRAC) */
    XP_C_PHOTO_PARTIAL,   /* partial photoionizations that happened (XP_PHOTO_FRAC) */
    XP_C_KA_FIELD,        /* K-alpha photons returned to the field (XP_KA_FIELD) */
    XP_NCOUNT = 27
};

/* Per-cell energy tallies (eV x weight units). */
enum {
    XP_L_PHOTO_E = 0,   /* kinetic energy given to photoelectrons */
    XP_L_AUGER_E,       /* kinetic energy given to Auger electrons */
    XP_L_ION_DEBIT,     /* lowered potentials paid by collisional ionization */
    XP_L_REC_ADD,       /* energy returned to electrons by recombination */
    XP_L_REC_BIND,      /* lowered binding released by recombination */
    XP_L_KALPHA,        /* K-alpha photon energy emitted */
    XP_L_PHOTON_ABS,    /* photon energy absorbed */
    XP_NLEDGER = 8
};

#define XP_NMOM 32          /* per-cell moment record, see collide_ionize_step */
#define XP_NSTATS 68        /* entries of xp_batch.d_stats */
#define XP_MAX_BINS 16      /* photon energy bins per run */

typedef struct xp_ctx xp_ctx;

/* ---- lifecycle ------------------------------------------------------- */

uint32_t    xp_abi_version(void);
const char *xp_last_error(void);
/* Creates a context bound to HIP device device_id. */
xp_status   xp_ctx_create(xp_ctx **out, int32_t device_id);
void        xp_ctx_destroy(xp_ctx *ctx);

/* ---- atomic data (Sec. III-V; Fig. 2, Fig. 3) ----------------------------
 * Host arrays, copied into the caller's device buffer by init_species.
 *   bind       [14][5]  eV   binding energy of subshell s (1s 2s 2p 3s 3p) of
 *                            charge state Z (tables vs ion charge, Sec. III)
 *   lotz_a,b,c [5]           Lotz constants of Eq. 4 (a in cm^2 eV^2)
 *   gamma_a,x  [14][3]  1/s  Auger and radiative K-vacancy decay rates of
 *                            charge state Z with k K vacancies (Sec. III)
 *   e_kalpha   [14]     eV   K-alpha photon energy of charge state Z
 *   photo_lnsig[5][photo_nh] ln(cm^2) per-electron subshell photoionization
 *                            cross section on the uniform grid ln(hv/eV) =
 *                            photo_lnhv0 + i photo_dlnhv (Fig. 2a)
 *   eos_zbar   [eos_nn][eos_nt] Zbar_EOS on the uniform grid ln(n_i / m^-3) =
 *                            eos_lnn0 + i eos_dlnn, ln(T/eV) = eos_lnt0 + j eos_dlnt
 */
typedef struct {
    int32_t z_nuc;          /* must be 13 (Al) */
    int32_t photo_nh;       /* 2 .. 512 */
    int32_t eos_nn;         /* 2 .. 256 */
    int32_t eos_nt;         /* 2 .. 1024 */
    double mass_ion;        /* kg */
    const double *bind;
    const double *lotz_a;
    const double *lotz_b;
    const double *lotz_c;
    const double *gamma_a;
    const double *gamma_x;
    const double *e_kalpha;
    double photo_lnhv0, photo_dlnhv;
    const double *photo_lnsig;
    double eos_lnn0, eos_dlnn, eos_lnt0, eos_dlnt;
    const double *eos_zbar;
} xp_atomic_tables;

/* Bytes of device memory init_species needs for these tables. */
size_t    xp_table_bytes(const xp_atomic_tables *tab);
/* Validates the tables (z_nuc == 13, grid sizes, positive spacings, finite
 * values) and copies them into d_table_buf (caller-owned, >= xp_table_bytes,
 * kept alive while the context is used).  Enqueued on stream; the host arrays
 * may be freed on return.  Errors: XP_ERR_INVALID_ARG, XP_ERR_TOO_SMALL. */
xp_status init_species(xp_ctx *ctx, const xp_atomic_tables *tab, void *d_table_buf,
                       size_t table_buf_bytes, void *stream);

/* ---- runs, batches and particles ----------------------------------------
 * A batch holds n_runs independent runs; run r owns cells
 * [cell_begin, cell_begin + ncells) of the batch.  Cell c of a run is grid
 * cell (c % nx, c / nx).  Each cell owns a slab of electron slots
 * [e_off[c], e_off[c] + e_cap[c]) of which the first e_cnt[c] are live, in
 * canonical order, and likewise for ions (ion counts never grow).  Every
 * macro-ion is one weight unit (w0 real ions); electrons carry integer units.
 */
typedef struct {
    uint64_t seed;          /* Philox key of the run */
    int32_t nx, ny;         /* grid; cell of (x, y) = floor((x-x0)/dx) + nx floor((y-y0)/dy) */
    double dx, dy, x0, y0;  /* m */
    double volume;          /* cell volume, m^3 */
    double w0;              /* real particles per weight unit */
    double dt;              /* PIC step, s */
    double dt_rad;          /* step of the source terms (decay, photo), s */
    double lnl_fixed;       /* > 0: fixed Coulomb logarithm; else computed per cell */
    double e_bulk;          /* eV; electrons below it form the bulk for T_e (Sec. II) */
    int32_t ipd_model;      /* 0 Stewart-Pyatt (Eq. 6), 1 Ecker-Kroll (Eq. 5) */
    int32_t z_floor;        /* ions with Z > z_floor may recombine (Al3+ floor, Sec. V) */
    int32_t cell_begin;     /* first batch cell of the run */
    int32_t ncells;         /* nx * ny */
    int32_t n_bins;         /* photon energy bins, 0 .. XP_MAX_BINS */
    int32_t field_per_cell; /* 0: nhv below; 1: batch d_cell_nhv[cell][n_bins] */
    double hv[XP_MAX_BINS];  /* eV */
    double nhv[XP_MAX_BINS]; /* photons per m^3, prescribed (Sec. II: RT not modelled) */
} xp_run;

typedef struct {
    int32_t n_runs;
    int32_t n_cells;
    const xp_run *d_runs;           /* [n_runs] */
    const int32_t *d_cell_run;      /* [n_cells] run of each cell */
    int64_t *d_e_off;               /* [n_cells] electron slab offsets */
    int32_t *d_e_cap;               /* [n_cells] */
    int32_t *d_e_cnt;               /* [n_cells] */
    int64_t *d_i_off;               /* [n_cells] */
    int32_t *d_i_cap;               /* [n_cells] */
    int32_t *d_i_cnt;               /* [n_cells] */
    int64_t e_slots, i_slots;       /* lengths of the particle arrays */
    double *d_ex, *d_ey, *d_evx, *d_evy, *d_evz;   /* [e_slots] */
    uint32_t *d_ew;                                /* [e_slots] weight units */
    double *d_ix, *d_iy, *d_ivx, *d_ivy, *d_ivz;   /* [i_slots] */
    uint8_t *d_iz, *d_ik;           /* charge state, K vacancies (0..2) */
    double *d_cell_nhv;             /* optional [n_cells][XP_MAX_BINS] photons / m^3, read by
                                       runs with field_per_cell; rewritten by
                                       transport_photons */
    uint64_t *d_run_counters;       /* [n_runs][XP_NCOUNT], accumulated */
    double *d_run_ledger;           /* [n_runs][XP_NLEDGER], accumulated (order-free) */
    int64_t *d_cell_counters;       /* optional [n_cells][XP_NCOUNT], last step */
    double *d_cell_ledger;          /* optional [n_cells][XP_NLEDGER], last step */
    double *d_cell_moments;         /* optional [n_cells][XP_NMOM], last step */
    uint32_t *d_status;             /* one word, XP_ST_* bits */
    void *d_work;                   /* workspace, >= xp_work_bytes */
    size_t work_bytes;
    int32_t e_cap_max;              /* host copy of max e_cap over cells (d_need[2]) */
    int32_t i_cap_max;              /* host copy of max i_cap over cells (d_need[3]) */
    int32_t *d_stats;               /* optional [XP_NSTATS]: after a step, [0] the largest
                                       electron count of a cell stepped in LDS, [1] cells
                                       re-planned with more LDS, [2] cells stepped on the
                                       global-memory path, [3] the largest electron count
                                       among those, [4 + b] LDS cells ending the step with
                                       16(b-1) < n_e <= 16 b electrons (b = 63: more) */
    /* Bounds of the cells that may take the global-memory path (cells whose
     * slab exceeds what one workgroup's LDS holds): their number and the sums
     * of their e_cap and i_cap (d_need[4..6] of bin_particles).  All zero:
     * the batch has no such cell and the path is never launched. */
    int32_t big_cells_max;
    int32_t reserved0;
    int64_t big_e_slots, big_i_slots;
    int32_t *d_cell_nabs;           /* optional [n_cells][XP_MAX_BINS]: photon events per bin of
                                       the last step (photoionizations, one macro-photon of w0
                                       real photons each, Sec. III); needed by transport_photons */
    uint32_t *d_run_status;         /* optional [n_runs]: the XP_ST_* bits of each run, OR-ed
                                       beside d_status by the step, the global-memory path and
                                       transport_photons (bin_particles sets d_status only);
                                       the caller clears a run's word */
    double *d_cell_nka;             /* optional [n_cells][XP_MAX_BINS]: K-alpha macro-photons
                                       returned per bin in the last step (XP_KA_FIELD; zeros
                                       without it); read by transport_photons if set */
} xp_batch;

/* Unsorted input particles of a batch for bin_particles.  Particle p belongs
 * to run d_e_run[p] (NULL: run 0). */
typedef struct {
    int64_t ne, ni;
    const int32_t *d_e_run, *d_i_run;
    const double *d_ex, *d_ey, *d_evx, *d_evy, *d_evz;
    const uint32_t *d_ew;
    const double *d_ix, *d_iy, *d_ivx, *d_ivy, *d_ivz;
    const uint8_t *d_iz, *d_ik;
} xp_particles;

/* Slab capacity rule used by bin_particles:
 *   e_cap = round_up(cnt_e + e_per_ion * cnt_i + e_extra, 16), i_cap = round_up(cnt_i, 16). */
typedef struct {
    int32_t e_per_ion;
    int32_t e_extra;
} xp_capacity;

/* Workspace bytes bin_particles needs for these input sizes. */
size_t xp_work_bytes(int64_t ne, int64_t ni, int32_t n_cells, int32_t n_runs);
/* Workspace bytes the step, photo_auger_step and diagnostics need on batch b
 * (reads n_cells and the big_* bounds only).  d_work must hold the larger of
 * this and xp_work_bytes of the binning. */
size_t xp_step_work_bytes(const xp_batch *b);
/* Largest electron count a cell stepped in LDS may reach when it holds up to
 * i_lds ions (*e_lds), and the ion limit itself (*i_lds); cells beyond either
 * take the global-memory path.  Depends on the device's LDS size only. */
xp_status xp_lds_limits(xp_ctx *ctx, int32_t *e_lds, int32_t *i_lds);

/* ---- the step ---------------------------------------------------------- */
typedef struct {
    uint32_t flags;            /* XP_* stage switches */
    uint32_t step;             /* step index (Philox counter word 0) */
    const uint32_t *d_step;    /* optional [n_runs] device step index per run; overrides step */
    int32_t schedule;          /* 0 auto, per LDS plan: four cells per wave for plans of at
                                  most 64 slots per species, a wave per cell up to 128, a
                                  block of 256 per cell above; 1 one wave per cell; 2 one
                                  block of 256 per cell; 3 every cell on the global-memory
                                  path (needs big_* bounds covering the whole batch); 4, 5, 6
                                  two, four, eight cells per wave (groups of 32, 16, 8 lanes)
                                  for plans of at most 128, 64, 32 slots per species, as auto
                                  above.  Results never depend on it. */
    int32_t e_hint;            /* expected largest electron count of a cell (e.g. d_stats[0]
                                  of the previous step); 0: plan for e_cap_max.  Plans
                                  before the last hold no more ion than electron slots.
                                  Cells that outgrow a plan are redone with a larger one in
                                  the same call, so the hint changes speed, never results. */
    int32_t big_grid;          /* workgroups of the global-memory path's chunk kernels;
                                  0: library default.  Speed only. */
    int32_t reserved;
} xp_step_params;

/* Stable counting sort of the unsorted particles into the batch's cell slabs
 * (Sec. VI: PIC cells).  The batch's run table, d_cell_run, slab arrays and
 * workspace must be set; offsets, capacities and counts are written from the
 * capacity rule.  Within a cell, particles keep their input order.  d_need is
 * caller-owned device memory of eight int64 receiving the required
 * (e_slots, i_slots), the largest (e_cap, i_cap) of any cell, and the number,
 * summed e_cap and summed i_cap of the cells beyond xp_lds_limits; the caller
 * copies [2], [3] into b->e_cap_max / i_cap_max and [4..6] into the big_*
 * bounds before stepping.  If the particle arrays are too short,
 * XP_ST_BIN_SIZE is set and no particle is written. */
xp_status bin_particles(xp_ctx *ctx, const xp_particles *in, xp_batch *b,
                        const xp_capacity *cap, int64_t *d_need, void *stream);

/* One Monte-Carlo step of every cell of every run in the batch (Sec. II-V):
 * moments and continuum lowering, e-e and e-i binary collisions (Takizuka-Abe,
 * or Nanbu's law with XP_NANBU, relativistic with XP_REL), collisional
 * ionization, three-body recombination, and -- when XP_PHOTO / XP_DECAY are in
 * p->flags -- the XFEL source terms of photo_auger_step, fused in the same
 * pass with dt_rad of the run table, then with XP_THERM the forced
 * thermalization of Sec. VI.C.  Cells stay in canonical slot order:
 * survivors keep their order, new electrons are appended (ionization events
 * in ion-slot order, then per ion Auger, photo 1s, 2s, 2p), electrons whose
 * weight reaches 0 are removed.  Moments record (when d_cell_moments is set):
 * [0] W_e [1] W_i [2] sum Z [3] sum Z^2 [4] K_e [5] T_e [6] n_e [7] n_i
 * [8] Zbar [9] z* [10] lnL [11] Z_c [12] P_ion [13] K_th [14] debit [15] T_e
 * before recombination [16..28] dE[Z] for Z = 0..12.
 * Cells that fit one workgroup's LDS are stepped there, one workgroup per
 * cell; larger cells (and every cell with schedule 3) go through a
 * global-memory path that spreads each cell over many workgroups: chunked
 * canonical sums, a segmented radix sort for the permutations and one thread
 * per pair.  Both give the same bits. */
xp_status collide_ionize_step(xp_ctx *ctx, xp_batch *b, const xp_step_params *p,
                              void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step of
 * collide_ionize_step with its workspace taken from a static device array of
 * XP_STATIC_SCRATCH_BYTES per GPU instead of b->d_work (b->d_work and
 * b->work_bytes are ignored; the batch is not modified).  The array is held
 * by the loaded library until the process ends; its address on a device is
 * taken when a context is created there.  Nothing is allocated and nothing is
 * freed; the caller still owns every other buffer of the batch.  All calls on
 * one GPU share its array and leave their contents in it, so calls that may
 * overlap on one GPU (other streams, other threads, other contexts) race and
 * must be ordered by the caller.  Errors: XP_ERR_UNSUPPORTED when
 * xp_step_work_bytes(b) exceeds XP_STATIC_SCRATCH_BYTES (64 MiB covers a
 * batch of up to about 520,000 cells on the LDS path, or a global-memory path
 * of about 400,000 electron and 400,000 ion slots), plus those of
 * collide_ionize_step. */
#define XP_STATIC_SCRATCH_BYTES (64u << 20)
xp_status collide_ionize_step_static(xp_ctx *ctx, const xp_batch *b, const xp_step_params *p,
                                     void *stream);

/* Source terms alone (Sec. III): moments and continuum lowering of the current
 * state, then K-vacancy decay with KLL Auger / K-alpha branching and subshell
 * photoionization (Eq. 3) with the run's prescribed photon field, over
 * dt_rad, then with XP_THERM the forced thermalization of Sec. VI.C.
 * p->flags is masked to XP_PHOTO | XP_DECAY | XP_THERM | XP_PHOTO_FRAC |
 * XP_KA_FIELD. */
xp_status photo_auger_step(xp_ctx *ctx, xp_batch *b, const xp_step_params *p,
                           void *stream);

/* Reduced radiation transport after a step of the source terms (Sec. II:
 * the radiation field and the plasma exchange energy every dt_rad; Sec. III:
 * every photoionization takes its photon's energy out of the selected bin).
 * For every run with field_per_cell = 1 and n_bins > 0, row by row along x
 * (the beam axis; row j holds cells j nx .. j nx + nx - 1 of the run) and bin
 * by bin: the run's nhv[b] enters the row at its low-x face; cell i passes on
 * the fraction tau_i = 1 - nabs_i w0 dx / (V c dt_rad n_i) (0 if negative, 1
 * if n_i = 0) of the density n_i it had during the step, nabs_i being its
 * photon events of bin b in d_cell_nabs; the density it passes on is
 * n_in tau_i + g_i w0 dx / (V c dt_rad), g_i its K-alpha macro-photons of
 * the bin in d_cell_nka (0 if d_cell_nka is NULL), so without K-alpha return
 * the new density of cell i is the incident density times tau_0 ... tau_{i-1}
 * (multiplied left to right).  The profile
 * is quasi-static: the light crossing time of a row is taken as short
 * against the pulse.  Call after collide_ionize_step / photo_auger_step
 * with d_cell_nabs set.  d_trans (optional, [n_runs][XP_MAX_BINS]) gets
 * each run's mean density leaving its rows over the incident density (0 for
 * an empty bin or a run without a per-cell field; rows summed in order).
 * Needs d_cell_nhv, d_cell_nabs and a workspace of xp_step_work_bytes.
 * Other runs are left as they are. */
xp_status transport_photons(xp_ctx *ctx, xp_batch *b, double *d_trans, void *stream);

/* Run diagnostics (Sec. II, Sec. VI.B, Fig. 7-9): charge-state distribution,
 * electron energy histogram (64 log bins from 0.1 eV to 1e5 eV, weight
 * units), weights, Zbar, total kinetic energy and T_e = (2/3) K / W_e, and a
 * copy of the accumulated counters and tallies.  With XP_DIAG_RESET the
 * accumulated counters are zeroed afterwards.  d_out: [n_runs] records. */
#define XP_DIAG_RESET 0x1u
typedef struct {
    int64_t csd[14];
    int64_t fe_hist[64];
    int64_t w_e, w_i, sum_z, n_e_macro;
    double zbar, ke_ev, te_ev, reserved;
    uint64_t counters[XP_NCOUNT];
    double ledger[XP_NLEDGER];
} xp_diag;

xp_status diagnostics(xp_ctx *ctx, const xp_batch *b, xp_diag *d_out, uint32_t what,
                      void *stream);

/* ---- self-test ----------------------------------------------------------
 * Evaluates one device building block of the step on n caller inputs, so that
 * a test suite can compare it with an independent implementation:
 *   which 0 log(d_x[i]), 1 exp(d_x[i]), 2 cbrt(d_x[i]), 5 sqrt(d_x[i]),
 *         6 d_x[2i] / d_x[2i+1]                          -> d_out[i]
 *   which 3 sin, cos of 2 pi (d_u[i] + 1/2) / 2^52       -> d_out[2i], d_out[2i+1]
 *   which 4 Philox4x32-10 of counter/key words packed as six uint32 in
 *         d_u[3i .. 3i+2] (c0 c1 c2 c3 k0 k1)             -> d_words[4i .. 4i+3]
 *   which 7, 8, 9 the canonical pairwise sum (leaves padded with +0 to a power
 *         of two, summed level by level, + 0.0) of the first m_j = (37 j) % R + 1
 *         values of row j of d_x (rows of R values, n a multiple of R) -> d_out[j]:
 *         7 one wave per row (R = 64), 8 one block of 256 per row (R = 256),
 *         9 groups of 16 lanes, one row each (R = 64).
 * Device arrays are caller-owned; unused ones may be NULL. */
xp_status xp_selftest(xp_ctx *ctx, int32_t which, int64_t n, const double *d_x,
                      const uint64_t *d_u, double *d_out, uint32_t *d_words, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* XPIC_H */
