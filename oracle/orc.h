/*
 * CPU oracle for the per-cell Monte-Carlo collision / ionization step of
 * Royle, Sentoku, Mancini, Paraschiv, Johzaki, "Kinetic modeling of x-ray
 * laser-driven solid Al plasmas via particle-in-cell simulation" (PICLS).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant with the library:
 * both sides implement the same written specification independently.
 *
 * Plain C99, FP64 throughout, slow on purpose: every cell is processed by one
 * loop in the order the paper gives (moments and continuum lowering, binary
 * collisions, collisional ionization, three-body recombination, then the XFEL
 * source terms).  OpenMP is used only across cells, which are independent
 * within a step, so results do not depend on the thread count.
 *
 * Parity status: every function is pinned by tests against closed forms,
 * library routines (libm, rocRAND's Philox, scipy's E1), invariants or brute
 * force, except where a function's comment says "parity unpinned".
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NSUB 5          /* 1s, 2s, 2p, 3s, 3p */
#define ORC_ZMAX 13         /* Al nucleus */
#define ORC_MAX_BINS 16
#define ORC_MAX_NH 128
#define ORC_MAX_EOS (16 * 128)

/* Stage switches for orc_step (same bit values as the library's flags). */
#define ORC_EE      0x01u
#define ORC_EI      0x02u
#define ORC_ION     0x04u
#define ORC_REC     0x08u
#define ORC_PHOTO   0x10u
#define ORC_DECAY   0x20u
#define ORC_THERM   0x40u   /* variant: forced thermalization after S5 (Sec. VI.C) */
#define ORC_ION_Z   0x80u   /* variant: S3 cross section per ion charge state (Sec. IV) */
#define ORC_NANBU   0x100u  /* variant: Nanbu's cumulative scattering law in S1, S2 */
#define ORC_REL     0x200u  /* variant: relativistic binary collisions in S1, S2 */
#define ORC_REC_XS  0x400u  /* variant: S4 per ion from the Lotz rate by detailed balance */
#define ORC_PHOTO_FRAC 0x800u  /* variant: S5 photo events limited by the bin's photons in the cell */
#define ORC_KA_FIELD   0x1000u /* variant: K-alpha photons return to the photon field */

/* Per-cell, per-step event counters. */
enum {
    OC_EE = 0, OC_EI, OC_TRIPLET, OC_ACCEPT, OC_U0, OC_DELTA2_GT1,
    OC_ION_FIRED, OC_ION_ACCEPTED, OC_ION_STARVED,
    OC_REC, OC_REC_SKIPPED, OC_E_REMOVED,
    OC_PHOTO_1S, OC_PHOTO_2S, OC_PHOTO_2P, OC_PHOTO_SKIPPED,
    OC_DECAY, OC_AUGER, OC_KALPHA,
    OC_P_CLAMPED, OC_IPD_CLAMPED, OC_E_NEW,
    OC_THERM, OC_THERM_SKIPPED,
    OC_PHOTO_STARVED, OC_PHOTO_PARTIAL, OC_KA_FIELD,
    OC_NCOUNT = 27
};

/* Per-cell, per-step energy tallies (eV x weight units). */
enum {
    OL_PHOTO_E = 0, OL_AUGER_E, OL_ION_DEBIT, OL_REC_ADD, OL_REC_BIND,
    OL_KALPHA, OL_PHOTON_ABS, OL_NLEDGER = 8
};

typedef struct {
    double bind[ORC_ZMAX + 1][ORC_NSUB];   /* eV, binding of subshell s in charge state Z */
    double lotz_a[ORC_NSUB];               /* cm^2 eV^2 */
    double lotz_b[ORC_NSUB];
    double lotz_c[ORC_NSUB];
    double gamma_a[ORC_ZMAX + 1][3];       /* s^-1, Auger rate for (Z, k) */
    double gamma_x[ORC_ZMAX + 1][3];       /* s^-1, radiative rate for (Z, k) */
    double e_kalpha[ORC_ZMAX + 1];         /* eV */
    double mass_ion;                       /* kg */
    double photo_lnhv0, photo_dlnhv;       /* uniform grid in ln(hv / eV) */
    double photo_lnsig[ORC_NSUB][ORC_MAX_NH]; /* ln(cm^2) per electron */
    int32_t photo_nh;
    int32_t eos_nn, eos_nt;
    int32_t pad0;
    double eos_lnn0, eos_dlnn, eos_lnt0, eos_dlnt;
    double eos_zbar[ORC_MAX_EOS];          /* [nn][nt], uniform in ln n_i and ln T */
} orc_tables;

typedef struct {
    uint64_t seed;
    int32_t nx, ny;
    double dx, dy, x0, y0;
    double volume;          /* cell volume, m^3 */
    double w0;              /* real particles per weight unit */
    double dt, dt_rad;      /* s */
    double lnl_fixed;       /* > 0: fixed Coulomb logarithm */
    double e_bulk;          /* eV, bulk-electron threshold */
    int32_t ipd_model;      /* 0 Stewart-Pyatt, 1 Ecker-Kroll */
    int32_t z_floor;        /* recombination floor */
    int32_t n_bins;         /* photon bins (0: no field) */
    int32_t pad1;
    double hv[ORC_MAX_BINS];    /* eV */
    double nhv[ORC_MAX_BINS];   /* photons / m^3, uniform over cells */
} orc_run;

typedef struct orc_sim orc_sim;

/* --- elementary functions and RNG, exported for the pins --- */
double orc_log(double x);
double orc_exp(double x);
double orc_cbrt(double x);
void   orc_sincos2pi(uint64_t k52, double *s, double *c);
void   orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void   orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out);
double orc_u52(uint32_t hi, uint32_t lo);
double orc_u32(uint32_t x);
void   orc_perm(int32_t n, const uint32_t *keys, int32_t *out);

/* --- single-physics helpers, exported for the pins --- */
void   orc_occupancy(int32_t z, int32_t k, int32_t occ[ORC_NSUB]);
double orc_ipd(int32_t model, int32_t z, double t_ev, double n_e, double n_i,
               double zbar, double zstar);
double orc_lotz(const orc_tables *t, int32_t zc, const double dE[13], double e_ev);
double orc_eos(const orc_tables *t, double n_i, double t_ev);
double orc_photo_sigma(const orc_tables *t, int32_t s, double hv);
double orc_coulomb_log(double t_ev, double n_e, double zbar);
/* One binary collision on explicit velocities (Takizuka-Abe 1977). */
double orc_ta77(double va[3], double vb[3], double ma, double mb, uint32_t wa,
                uint32_t wb, double qq_coef, double nunit, const uint32_t draws[4],
                int32_t *accept_a, int32_t *accept_b);
/* The same collision with the scattering law chosen: 0 Takizuka-Abe, 1 Nanbu. */
double orc_collide(double va[3], double vb[3], double ma, double mb, uint32_t wa,
                   uint32_t wb, double qq_coef, double nunit, const uint32_t draws[4],
                   int32_t law, int32_t *accept_a, int32_t *accept_b);
/* Nanbu (1997): A with coth A - 1/A = exp(-s), and 1 - cos chi for uniform u. */
/* Relativistic binary collision (law bit 2 of orc_collide) on its own, for
 * the tests: returns <delta^2> = s / 2 of the pair, or -1. */
double orc_collide_rel(double va[3], double vb[3], double ma, double mb, uint32_t wa,
                       uint32_t wb, double qq_coef, double nunit, const uint32_t draws[4],
                       int32_t nanbu, int32_t *acc_a, int32_t *acc_b);
/* exp(x) E1(x) for x > 0 (E1 the exponential integral). */
double orc_e1x(double x);
/* Probability per step dt (s) that an ion of charge z recombines to z - 1 by
 * three-body recombination at electron temperature tev (eV) and density n_e
 * (m^-3), the inverse of the Lotz ionization of z - 1 by detailed balance
 * (not clamped). */
double orc_rec_xs(const orc_tables *t, int32_t z, double tev, double n_e, const double dE[13],
                  double dt);
double orc_nanbu_a(double s);
double orc_nanbu_omc(double s, double u);

/* --- simulation of one run --- */
orc_sim *orc_create(const orc_tables *t, const orc_run *r);
void     orc_destroy(orc_sim *s);
/* Stable bin of unsorted particles into cells (input order kept per cell). */
int      orc_bin(orc_sim *s, int64_t ne, const double *ex, const double *ey,
                 const double *evx, const double *evy, const double *evz,
                 const uint32_t *ew, int64_t ni, const double *ix, const double *iy,
                 const double *ivx, const double *ivy, const double *ivz,
                 const uint8_t *iz, const uint8_t *ik);
/* Load already-binned particles (compact cell-major layout with starts). */
int      orc_load(orc_sim *s, const int64_t *e_start, const double *ex, const double *ey,
                  const double *evx, const double *evy, const double *evz,
                  const uint32_t *ew, const int64_t *i_start, const double *ix,
                  const double *iy, const double *ivx, const double *ivy,
                  const double *ivz, const uint8_t *iz, const uint8_t *ik);
/* Per-cell photon densities [ncells][n_bins]; NULL restores the uniform field. */
void     orc_set_cell_field(orc_sim *s, const double *nhv_cells);
/* One step: stages selected by flags, in the order S0 S1 S2 S3 S4 S5. */
void     orc_step(orc_sim *s, uint32_t step, uint32_t flags, int32_t nthreads);
void     orc_counts(const orc_sim *s, int64_t *ne_total, int64_t *ni_total);
void     orc_export(const orc_sim *s, int64_t *e_start, double *ex, double *ey,
                    double *evx, double *evy, double *evz, uint32_t *ew,
                    int64_t *i_start, double *ix, double *iy, double *ivx,
                    double *ivy, double *ivz, uint8_t *iz, uint8_t *ik);
/* Counters and tallies of the last step, [ncells][OC_NCOUNT] / [ncells][OL_NLEDGER]. */
void     orc_last_counters(const orc_sim *s, int64_t *cnt, double *ledger);
/* Photon events per bin of the last step, [ncells][ORC_MAX_BINS]. */
void     orc_last_absorbed(const orc_sim *s, int32_t *nabs);
/* K-alpha photons returned to the field in the last step (ORC_KA_FIELD), in
 * macro-photons of each bin's energy, [ncells][ORC_MAX_BINS]. */
void     orc_last_kalpha_field(const orc_sim *s, double *g);
/* Current photon field per cell, [ncells][n_bins] (the uniform one if unset). */
void     orc_get_cell_field(const orc_sim *s, double *nhv);
/* Reduced radiation transport along x after a step (see orc_step.c):
 * new per-cell field from the incident density and the last step's
 * absorption; trans[n_bins] gets the mean transmission of the rows. */
void     orc_transport(orc_sim *s, double *trans);
/* Cell moments after S0 of the last step: [ncells][16] (see orc_step.c). */
void     orc_last_moments(const orc_sim *s, double *mom);
/* Run diagnostics of the current state. */
void     orc_diag(const orc_sim *s, int64_t csd[ORC_ZMAX + 1], int64_t fe_hist[64],
                  double out[8]);

#ifdef __cplusplus
}
#endif
#endif
