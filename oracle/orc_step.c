/*
 * Oracle: one Monte-Carlo step of every cell of one run.  TEST INFRASTRUCTURE ONLY.
 *
 * Stages per cell, in order (each sees the state the previous one left):
 *   S0 moments: weights, charge sums, bulk temperature k T_e = (2/3) E_ave
 *      (Sec. II), densities, Zbar, z* and the continuum lowering dE[Z] of every
 *      charge state by Ecker-Kroll (Eq. 5) or Stewart-Pyatt (Eq. 6) (Sec. V).
 *   S1 electron-electron and S2 electron-ion binary collisions (Sec. IV), by
 *      Takizuka-Abe's scattering law or (ORC_NANBU) Nanbu's cumulative law,
 *      non-relativistic or (ORC_REL) in the pair's centre-of-momentum frame
 *      with relativistic kinematics.
 *   S3 collisional ionization against the average cell ion with the Lotz cross
 *      section (Eq. 4) and the energy debit of Sec. IV; with ORC_ION_Z every
 *      ion's probability uses the cross section of its own charge state.
 *   S4 three-body recombination constrained by Zbar_EOS(n_i, T_e) (Sec. IV),
 *      or (ORC_REC_XS) per ion from the rate that detailed balance gives the
 *      inverse of the Lotz ionization (orc_rec_xs).
 *   S5 K-vacancy decay with Auger / K-alpha branching and subshell
 *      photoionization (Eq. 3) (Sec. III).  With ORC_PHOTO_FRAC a bin can
 *      give no more macro-photons than the cell holds; the event that finds
 *      less than one left is a partial photoionization.  With ORC_KA_FIELD
 *      the energy of every K-alpha photon goes back into the photon field.
 *   Optionally (ORC_THERM) the forced thermalization of Sec. VI.C right after
 *      S5: every free electron gets a new Maxwellian velocity at the cell
 *      temperature, corrected so that momentum and energy are unchanged.
 * Every random decision uses Philox4x32-10 keyed by the run seed with counter
 * (step, cell, index, purpose << 24 | sub): a uniform r in (0, 1) decides an
 * event with probability P iff r < P (Sec. III).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "orc.h"
#include "orc_internal.h"

/* Random-number purposes.  P_ION is one call per ion and step whose four
 * words decide collisional ionization and the photo events of 1s, 2s, 2p. */
enum { P_PERM_E = 1, P_PERM_I = 2, P_REC_I = 3, P_REC_E = 4, P_EE = 5,
       P_EE_TRI = 6, P_EI = 7, P_ION = 8, P_DECAY = 9, P_DIR = 10, P_BIN = 11,
       P_THERM = 12, P_REC_XS = 13, P_PART = 14 };

#define NMOM 32

typedef struct {
    int ne, ce;
    double *ex, *ey, *evx, *evy, *evz;
    uint32_t *ew;
    int ni;
    double *ix, *iy, *ivx, *ivy, *ivz;
    uint8_t *iz, *ik;
} ocell;

struct orc_sim {
    orc_tables t;
    orc_run r;
    int ncells;
    ocell *cells;
    int64_t *cnt;        /* [ncells][OC_NCOUNT] of the last step */
    double *led;         /* [ncells][OL_NLEDGER] */
    double *mom;         /* [ncells][NMOM] */
    double *cell_nhv;    /* optional [ncells][n_bins] */
    int32_t *nabs;       /* [ncells][ORC_MAX_BINS] photons absorbed per bin, last step */
    double *nka;         /* [ncells][ORC_MAX_BINS] K-alpha macro-photons returned, last step */
    double sigma[ORC_MAX_BINS][3];   /* photo cross section at each bin, m^2 */
};

/* ------------------------------------------------------------------------ */

static void cell_reserve_e(ocell *c, int need)
{
    if (need <= c->ce) return;
    int n = c->ce ? c->ce : 16;
    while (n < need) n *= 2;
    c->ex = realloc(c->ex, sizeof(double) * n);
    c->ey = realloc(c->ey, sizeof(double) * n);
    c->evx = realloc(c->evx, sizeof(double) * n);
    c->evy = realloc(c->evy, sizeof(double) * n);
    c->evz = realloc(c->evz, sizeof(double) * n);
    c->ew = realloc(c->ew, sizeof(uint32_t) * n);
    c->ce = n;
}

static void cell_push_e(ocell *c, double x, double y, double vx, double vy, double vz, uint32_t w)
{
    cell_reserve_e(c, c->ne + 1);
    int j = c->ne++;
    c->ex[j] = x; c->ey[j] = y; c->evx[j] = vx; c->evy[j] = vy; c->evz[j] = vz; c->ew[j] = w;
}

static void cell_alloc_i(ocell *c, int n)
{
    int m = n > 0 ? n : 1;
    c->ix = malloc(sizeof(double) * m);
    c->iy = malloc(sizeof(double) * m);
    c->ivx = malloc(sizeof(double) * m);
    c->ivy = malloc(sizeof(double) * m);
    c->ivz = malloc(sizeof(double) * m);
    c->iz = malloc(m);
    c->ik = malloc(m);
    c->ni = n;
}

static void cell_free(ocell *c)
{
    free(c->ex); free(c->ey); free(c->evx); free(c->evy); free(c->evz); free(c->ew);
    free(c->ix); free(c->iy); free(c->ivx); free(c->ivy); free(c->ivz); free(c->iz); free(c->ik);
    memset(c, 0, sizeof(*c));
}

orc_sim *orc_create(const orc_tables *t, const orc_run *r)
{
    orc_sim *s = calloc(1, sizeof(orc_sim));
    s->t = *t;
    s->r = *r;
    s->ncells = r->nx * r->ny;
    s->cells = calloc((size_t)s->ncells, sizeof(ocell));
    s->cnt = calloc((size_t)s->ncells * OC_NCOUNT, sizeof(int64_t));
    s->led = calloc((size_t)s->ncells * OL_NLEDGER, sizeof(double));
    s->mom = calloc((size_t)s->ncells * NMOM, sizeof(double));
    s->nabs = calloc((size_t)s->ncells * ORC_MAX_BINS, sizeof(int32_t));
    s->nka = calloc((size_t)s->ncells * ORC_MAX_BINS, sizeof(double));
    for (int b = 0; b < r->n_bins; ++b)
        for (int q = 0; q < 3; ++q) s->sigma[b][q] = orc_photo_sigma(t, q, r->hv[b]);
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    for (int c = 0; c < s->ncells; ++c) cell_free(&s->cells[c]);
    free(s->cells); free(s->cnt); free(s->led); free(s->mom); free(s->cell_nhv); free(s->nabs);
    free(s->nka);
    free(s);
}

void orc_set_cell_field(orc_sim *s, const double *nhv)
{
    free(s->cell_nhv);
    s->cell_nhv = NULL;
    if (!nhv) return;
    size_t n = (size_t)s->ncells * (size_t)s->r.n_bins;
    s->cell_nhv = malloc(sizeof(double) * (n ? n : 1));
    memcpy(s->cell_nhv, nhv, sizeof(double) * n);
}

/* Cell index of a position: floor((x - x0)/dx) (+ nx floor((y - y0)/dy)), clamped. */
static int cell_of(const orc_run *r, double x, double y)
{
    double fx = floor((x - r->x0) / r->dx);
    int ix = fx < 0.0 ? 0 : (fx > (double)(r->nx - 1) ? r->nx - 1 : (int)fx);
    int iy = 0;
    if (r->ny > 1) {
        double fy = floor((y - r->y0) / r->dy);
        iy = fy < 0.0 ? 0 : (fy > (double)(r->ny - 1) ? r->ny - 1 : (int)fy);
    }
    return ix + r->nx * iy;
}

int orc_bin(orc_sim *s, int64_t ne, const double *ex, const double *ey,
            const double *evx, const double *evy, const double *evz, const uint32_t *ew,
            int64_t ni, const double *ix, const double *iy, const double *ivx,
            const double *ivy, const double *ivz, const uint8_t *iz, const uint8_t *ik)
{
    for (int c = 0; c < s->ncells; ++c) cell_free(&s->cells[c]);
    int *icount = calloc((size_t)s->ncells, sizeof(int));
    for (int64_t p = 0; p < ne; ++p) {
        ocell *c = &s->cells[cell_of(&s->r, ex[p], ey ? ey[p] : 0.0)];
        cell_push_e(c, ex[p], ey ? ey[p] : 0.0, evx[p], evy[p], evz[p], ew[p]);
    }
    for (int64_t p = 0; p < ni; ++p) icount[cell_of(&s->r, ix[p], iy ? iy[p] : 0.0)]++;
    for (int c = 0; c < s->ncells; ++c) { cell_alloc_i(&s->cells[c], icount[c]); icount[c] = 0; }
    for (int64_t p = 0; p < ni; ++p) {
        int cc = cell_of(&s->r, ix[p], iy ? iy[p] : 0.0);
        ocell *c = &s->cells[cc];
        int j = icount[cc]++;
        c->ix[j] = ix[p]; c->iy[j] = iy ? iy[p] : 0.0;
        c->ivx[j] = ivx[p]; c->ivy[j] = ivy[p]; c->ivz[j] = ivz[p];
        c->iz[j] = iz[p]; c->ik[j] = ik[p];
    }
    free(icount);
    return 0;
}

int orc_load(orc_sim *s, const int64_t *es, const double *ex, const double *ey,
             const double *evx, const double *evy, const double *evz, const uint32_t *ew,
             const int64_t *is, const double *ix, const double *iy, const double *ivx,
             const double *ivy, const double *ivz, const uint8_t *iz, const uint8_t *ik)
{
    for (int c = 0; c < s->ncells; ++c) {
        ocell *cl = &s->cells[c];
        cell_free(cl);
        for (int64_t p = es[c]; p < es[c + 1]; ++p)
            cell_push_e(cl, ex[p], ey ? ey[p] : 0.0, evx[p], evy[p], evz[p], ew[p]);
        int n = (int)(is[c + 1] - is[c]);
        cell_alloc_i(cl, n);
        for (int j = 0; j < n; ++j) {
            int64_t p = is[c] + j;
            cl->ix[j] = ix[p]; cl->iy[j] = iy ? iy[p] : 0.0;
            cl->ivx[j] = ivx[p]; cl->ivy[j] = ivy[p]; cl->ivz[j] = ivz[p];
            cl->iz[j] = iz[p]; cl->ik[j] = ik[p];
        }
    }
    return 0;
}

void orc_counts(const orc_sim *s, int64_t *ne, int64_t *ni)
{
    int64_t a = 0, b = 0;
    for (int c = 0; c < s->ncells; ++c) { a += s->cells[c].ne; b += s->cells[c].ni; }
    *ne = a;
    *ni = b;
}

void orc_export(const orc_sim *s, int64_t *es, double *ex, double *ey, double *evx,
                double *evy, double *evz, uint32_t *ew, int64_t *is, double *ix,
                double *iy, double *ivx, double *ivy, double *ivz, uint8_t *iz, uint8_t *ik)
{
    int64_t pe = 0, pi = 0;
    for (int c = 0; c < s->ncells; ++c) {
        const ocell *cl = &s->cells[c];
        es[c] = pe;
        is[c] = pi;
        for (int j = 0; j < cl->ne; ++j, ++pe) {
            ex[pe] = cl->ex[j]; ey[pe] = cl->ey[j]; evx[pe] = cl->evx[j];
            evy[pe] = cl->evy[j]; evz[pe] = cl->evz[j]; ew[pe] = cl->ew[j];
        }
        for (int j = 0; j < cl->ni; ++j, ++pi) {
            ix[pi] = cl->ix[j]; iy[pi] = cl->iy[j]; ivx[pi] = cl->ivx[j];
            ivy[pi] = cl->ivy[j]; ivz[pi] = cl->ivz[j]; iz[pi] = cl->iz[j]; ik[pi] = cl->ik[j];
        }
    }
    es[s->ncells] = pe;
    is[s->ncells] = pi;
}

void orc_last_counters(const orc_sim *s, int64_t *cnt, double *led)
{
    if (cnt) memcpy(cnt, s->cnt, sizeof(int64_t) * (size_t)s->ncells * OC_NCOUNT);
    if (led) memcpy(led, s->led, sizeof(double) * (size_t)s->ncells * OL_NLEDGER);
}

void orc_last_moments(const orc_sim *s, double *mom)
{
    memcpy(mom, s->mom, sizeof(double) * (size_t)s->ncells * NMOM);
}

void orc_last_kalpha_field(const orc_sim *s, double *g)
{
    memcpy(g, s->nka, sizeof(double) * (size_t)s->ncells * ORC_MAX_BINS);
}

void orc_last_absorbed(const orc_sim *s, int32_t *nabs)
{
    memcpy(nabs, s->nabs, sizeof(int32_t) * (size_t)s->ncells * ORC_MAX_BINS);
}

void orc_get_cell_field(const orc_sim *s, double *nhv)
{
    size_t n = (size_t)s->ncells * (size_t)s->r.n_bins;
    if (s->cell_nhv) {
        memcpy(nhv, s->cell_nhv, sizeof(double) * n);
        return;
    }
    for (int c = 0; c < s->ncells; ++c)
        for (int b = 0; b < s->r.n_bins; ++b) nhv[(size_t)c * s->r.n_bins + b] = s->r.nhv[b];
}

/* Reduced radiation transport along x (the beam axis), after a step of the
 * source terms (Sec. II, Sec. III).  The incident density of each bin, the
 * run's prescribed n_hv, enters every row of cells at its low-x face.  Cell i
 * of a row absorbed nabs photon events of w0 real photons during the step,
 * out of the c dt_rad n (V / dx) photons that crossed its entrance face at its
 * density n of that step, so its transmission is
 *   tau = 1 - nabs w0 dx / (V c dt_rad n)   (0 if negative; 1 if n = 0),
 * the photons the Monte-Carlo events took out of the bin (Sec. III).  The
 * new density of cell i is the density entering it, the incident density
 * times the transmissions of the cells before it in the row (a quasi-static
 * Beer-Lambert profile: the crossing time of a row is taken as short against
 * the pulse).  K-alpha photons that the step returned to bin b of a cell
 * (ORC_KA_FIELD: g macro-photons of the bin's energy) join the beam leaving
 * that cell: the density passed on is n_in tau + g w0 dx / (V c dt_rad).
 * trans[b] (if not NULL) is the mean over rows of the density leaving the
 * row divided by the incident density (0 for an empty bin).
 * The per-cell field is created from the uniform one if not set. */
void orc_transport(orc_sim *s, double *trans)
{
    const orc_run *r = &s->r;
    int nb = r->n_bins;
    if (nb <= 0) return;
    if (!s->cell_nhv) {
        double *f = malloc(sizeof(double) * (size_t)s->ncells * (size_t)nb);
        orc_get_cell_field(s, f);
        s->cell_nhv = f;
    }
    const double cross = (r->volume * (ORC_CLIGHT * r->dt_rad)) / r->dx;
    for (int b = 0; b < nb; ++b) {
        double out_sum = 0.0;
        for (int j = 0; j < r->ny; ++j) {
            double carry = r->nhv[b];
            for (int i = 0; i < r->nx; ++i) {
                size_t c = (size_t)j * (size_t)r->nx + (size_t)i;
                double n = s->cell_nhv[c * nb + b];
                s->cell_nhv[c * nb + b] = carry;
                double tau = 1.0;
                if (n > 0.0) {
                    double a = ((double)s->nabs[c * ORC_MAX_BINS + b] * r->w0) / (cross * n);
                    tau = a < 1.0 ? 1.0 - a : 0.0;
                }
                carry = carry * tau + (s->nka[c * ORC_MAX_BINS + b] * r->w0) / cross;
            }
            out_sum = out_sum + carry;
        }
        if (trans) trans[b] = r->nhv[b] > 0.0 ? (out_sum / (double)r->ny) / r->nhv[b] : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Canonical pairwise sum: leaves padded with +0 to the next power of two,
 * y[i] = y[2i] + y[2i+1] level by level; the result is normalized by + 0.0. */
static double tree_sum(double *y, int n)
{
    if (n <= 0) return 0.0;
    int p = 1;
    while (p < n) p *= 2;
    for (int i = n; i < p; ++i) y[i] = 0.0;
    for (int len = p; len > 1; len /= 2)
        for (int i = 0; i < len / 2; ++i) y[i] = y[2 * i] + y[2 * i + 1];
    return y[0] + 0.0;
}

typedef struct {
    const orc_sim *s;
    uint32_t step, cell;
    uint32_t key[2];
    double *scratch;      /* >= 2 * max particles, padded */
    int32_t *perm_e, *perm_i, *perm_a, *perm_b;
    uint32_t *keys;
    int64_t *cnt;
    double *led;
    int32_t law;          /* S1, S2: bit 0 Nanbu (else Takizuka-Abe), bit 1 relativistic */
    int32_t *nabs;        /* this cell's photons absorbed per bin */
    double *nka;          /* this cell's K-alpha macro-photons returned per bin */
} cctx;

static void rng(const cctx *x, uint32_t idx, uint32_t purpose, uint32_t sub, uint32_t out[4])
{
    uint32_t ctr[4] = {x->step, x->cell, idx, (purpose << 24) | sub};
    orc_philox(ctr, x->key, out);
}

/* Permutation of n slots for one purpose: key of slot i is word i % 4 of the
 * Philox call with index i / 4; slots sorted by (key, slot). */
static void make_perm(const cctx *x, uint32_t purpose, int n, int32_t *out)
{
    uint32_t *k = (uint32_t *)x->keys;
    for (int i = 0; i < n; i += 4) {
        uint32_t w[4];
        rng(x, (uint32_t)(i / 4), purpose, 0, w);
        for (int q = 0; q < 4 && i + q < n; ++q) k[i + q] = w[q];
    }
    orc_perm(n, k, out);
}

static const double HALF_ME_OVER_QE = (0.5 * ORC_ME) / ORC_QE;
static const double TWO_QE_OVER_ME = (2.0 * ORC_QE) / ORC_ME;

static double e_kin(const ocell *c, int j)
{
    double v2 = (c->evx[j] * c->evx[j] + c->evy[j] * c->evy[j]) + c->evz[j] * c->evz[j];
    return HALF_ME_OVER_QE * v2;
}

/* Lowered binding of subshell s of charge state z, clamped at 1 eV. */
static double lowered(const cctx *x, int z, int s, const double *dE, int unused)
{
    (void)unused;
    double p = x->s->t.bind[z][s] - dE[z];
    if (p < 1.0) p = 1.0;
    return p;
}

/* S0: cell moments and continuum lowering. */
static void moments(const cctx *x, ocell *c, double *m)
{
    const orc_run *r = &x->s->r;
    int64_t we = 0, wi = c->ni, sz = 0, sz2 = 0, wb = 0;
    for (int j = 0; j < c->ne; ++j) {
        we += c->ew[j];
        double e = e_kin(c, j);
        int bulk = e < r->e_bulk;
        x->scratch[j] = bulk ? (double)c->ew[j] * e : 0.0;
        if (bulk) wb += c->ew[j];
    }
    double ke = tree_sum(x->scratch, c->ne);
    for (int j = 0; j < c->ni; ++j) { sz += c->iz[j]; sz2 += (int64_t)c->iz[j] * c->iz[j]; }
    double t = 0.01;
    if (wb > 0) {
        t = (2.0 * ke) / (3.0 * (double)wb);
        if (t < 0.01) t = 0.01;
    }
    double n_e = ((double)we * r->w0) / r->volume;
    double n_i = ((double)wi * r->w0) / r->volume;
    double zbar = wi > 0 ? (double)sz / (double)wi : 0.0;
    double zstar = sz > 0 ? (double)sz2 / (double)sz : 0.0;
    m[0] = (double)we; m[1] = (double)wi; m[2] = (double)sz; m[3] = (double)sz2;
    m[4] = ke; m[5] = t; m[6] = n_e; m[7] = n_i; m[8] = zbar; m[9] = zstar;
    m[10] = r->lnl_fixed > 0.0 ? r->lnl_fixed : orc_coulomb_log(t, n_e, zbar);
    for (int z = 0; z < 13; ++z) m[16 + z] = orc_ipd(r->ipd_model, z, t, n_e, n_i, zbar, zstar);
}

static void collide_pair(const cctx *x, ocell *c, int e_a, int is_ion_b, int b,
                         double coef, double nunit, uint32_t idx, uint32_t purpose,
                         uint32_t sub)
{
    double va[3] = {c->evx[e_a], c->evy[e_a], c->evz[e_a]};
    double vb[3];
    uint32_t wa = c->ew[e_a], wb;
    double mb;
    if (is_ion_b) {
        vb[0] = c->ivx[b]; vb[1] = c->ivy[b]; vb[2] = c->ivz[b];
        wb = 1;
        mb = x->s->t.mass_ion;
    } else {
        vb[0] = c->evx[b]; vb[1] = c->evy[b]; vb[2] = c->evz[b];
        wb = c->ew[b];
        mb = ORC_ME;
    }
    uint32_t d[4];
    rng(x, idx, purpose, sub, d);
    int32_t aa, ab;
    double d2 = orc_collide(va, vb, ORC_ME, mb, wa, wb, coef, nunit, d, x->law, &aa, &ab);
    if (d2 < 0.0) { x->cnt[OC_U0]++; return; }
    if (d2 > 1.0) x->cnt[OC_DELTA2_GT1]++;
    x->cnt[OC_ACCEPT] += aa + ab;
    c->evx[e_a] = va[0]; c->evy[e_a] = va[1]; c->evz[e_a] = va[2];
    if (is_ion_b) {
        c->ivx[b] = vb[0]; c->ivy[b] = vb[1]; c->ivz[b] = vb[2];
    } else {
        c->evx[b] = vb[0]; c->evy[b] = vb[1]; c->evz[b] = vb[2];
    }
}

/* Drift velocity and drift-frame thermal energy (eV x units) of electrons
 * 0..n-1 with weights w[] (0 excludes an electron). */
static void drift_frame(const cctx *x, const ocell *c, int n, const uint32_t *w,
                        double u[3], double *kth, int64_t *wsum)
{
    int64_t ws = 0;
    for (int j = 0; j < n; ++j) ws += w[j];
    *wsum = ws;
    if (ws == 0) { u[0] = u[1] = u[2] = 0.0; *kth = 0.0; return; }
    const double *vv[3] = {c->evx, c->evy, c->evz};
    for (int d = 0; d < 3; ++d) {
        for (int j = 0; j < n; ++j) x->scratch[j] = (double)w[j] * vv[d][j];
        u[d] = tree_sum(x->scratch, n) / (double)ws;
    }
    for (int j = 0; j < n; ++j) {
        double dx = c->evx[j] - u[0], dy = c->evy[j] - u[1], dz = c->evz[j] - u[2];
        x->scratch[j] = (double)w[j] * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
    }
    *kth = tree_sum(x->scratch, n);
}

/* Isotropic electron of energy e (eV) from the two draws of a DIR call. */
static void new_electron_dir(const cctx *x, ocell *c, int ion, uint32_t sub, double e)
{
    uint32_t d[4];
    rng(x, (uint32_t)ion, P_DIR, sub, d);
    double mu = 2.0 * orc_u52(d[0], d[1]) - 1.0;
    double sp, cp;
    orc_sincos2pi(((((uint64_t)d[2]) << 32) | d[3]) >> 12, &sp, &cp);
    double st = sqrt(1.0 - mu * mu);
    double sp_ = sqrt(e * TWO_QE_OVER_ME);
    cell_push_e(c, c->ix[ion], c->iy[ion], sp_ * (st * cp), sp_ * (st * sp), sp_ * mu, 1);
    x->cnt[OC_E_NEW]++;
}

/* Forced thermalization (Sec. VI.C).  T from the average kinetic energy of
 * all free electrons, k T = (2/3) K / W (Sec. II); each electron's velocity
 * components are drawn from a normal distribution of zero mean and spread
 * sqrt(k T / m_e) (one Philox call per electron slot: Box-Muller on words 0, 1
 * gives the x and y components, on words 2, 3 the z component).  The draw's
 * mean velocity is replaced by the cell's drift velocity u and its spread
 * about it scaled by beta = sqrt(K_th / K_draw), where K_th is the cell's
 * kinetic energy in the drift frame before, so momentum and energy are those
 * of the cell before (the correction the paper asks for).  Cells with fewer
 * than two electrons or no energy in the drift frame keep their velocities. */
static void thermalize(cctx *x, ocell *c)
{
    int ne = c->ne;
    double *y = x->scratch;
    int64_t ws = 0;
    for (int j = 0; j < ne; ++j) ws += c->ew[j];
    if (ne < 2 || ws <= 0) { x->cnt[OC_THERM_SKIPPED]++; return; }
    double w = (double)ws;
    for (int j = 0; j < ne; ++j) y[j] = (double)c->ew[j] * e_kin(c, j);
    double kin = tree_sum(y, ne);
    double u[3];
    double *vv[3] = {c->evx, c->evy, c->evz};
    for (int d = 0; d < 3; ++d) {
        for (int j = 0; j < ne; ++j) y[j] = (double)c->ew[j] * vv[d][j];
        u[d] = tree_sum(y, ne) / w;
    }
    for (int j = 0; j < ne; ++j) {
        double dx = c->evx[j] - u[0], dy = c->evy[j] - u[1], dz = c->evz[j] - u[2];
        y[j] = (double)c->ew[j] * (HALF_ME_OVER_QE * ((dx * dx + dy * dy) + dz * dz));
    }
    double kth = tree_sum(y, ne);
    if (!(kin > 0.0) || !(kth > 0.0)) { x->cnt[OC_THERM_SKIPPED]++; return; }
    double kt = (2.0 * kin) / (3.0 * w);
    double sig = sqrt(kt * (ORC_QE / ORC_ME));
    /* the draws replace the velocities (the originals are no longer needed) */
    for (int j = 0; j < ne; ++j) {
        uint32_t d[4];
        rng(x, (uint32_t)j, P_THERM, 0, d);
        double s1, c1, s2, c2;
        orc_sincos2pi(((uint64_t)d[1]) << 20, &s1, &c1);
        orc_sincos2pi(((uint64_t)d[3]) << 20, &s2, &c2);
        double r1 = sqrt(-2.0 * orc_log(orc_u32(d[0])));
        double r2 = sqrt(-2.0 * orc_log(orc_u32(d[2])));
        c->evx[j] = sig * (r1 * c1);
        c->evy[j] = sig * (r1 * s1);
        c->evz[j] = sig * (r2 * c2);
    }
    double q[3];
    for (int d = 0; d < 3; ++d) {
        for (int j = 0; j < ne; ++j) y[j] = (double)c->ew[j] * vv[d][j];
        q[d] = tree_sum(y, ne) / w;
    }
    for (int j = 0; j < ne; ++j) {
        c->evx[j] = c->evx[j] - q[0];
        c->evy[j] = c->evy[j] - q[1];
        c->evz[j] = c->evz[j] - q[2];
    }
    for (int j = 0; j < ne; ++j) y[j] = (double)c->ew[j] * e_kin(c, j);
    double kd = tree_sum(y, ne);
    if (!(kd > 0.0)) {
        /* only if every draw coincides: every electron gets the drift velocity */
        for (int j = 0; j < ne; ++j) { c->evx[j] = u[0]; c->evy[j] = u[1]; c->evz[j] = u[2]; }
        x->cnt[OC_THERM_SKIPPED]++;
        return;
    }
    double beta = sqrt(kth / kd);
    for (int j = 0; j < ne; ++j) {
        c->evx[j] = u[0] + beta * c->evx[j];
        c->evy[j] = u[1] + beta * c->evy[j];
        c->evz[j] = u[2] + beta * c->evz[j];
    }
    x->cnt[OC_THERM]++;
}

static void step_cell(cctx *x, ocell *c, uint32_t flags)
{
    const orc_sim *s = x->s;
    const orc_run *r = &s->r;
    const orc_tables *t = &s->t;
    double *m = s->mom + (size_t)x->cell * NMOM;
    memset(m, 0, sizeof(double) * NMOM);
    moments(x, c, m);
    const double *dE = m + 16;
    double lnl = m[10];
    const double mi = t->mass_ion;

    /* S1: electron-electron pairs on a random permutation; odd count -> triplet */
    int ne = c->ne, ni = c->ni;
    int have_pe = 0;
    if ((flags & (ORC_EE | ORC_EI)) && ne >= 1 && (ne >= 2 || ni >= 1)) {
        make_perm(x, P_PERM_E, ne, x->perm_e);
        have_pe = 1;
    }
    if ((flags & ORC_EE) && ne >= 2) {
        const double qe4 = (ORC_QE * ORC_QE) * (ORC_QE * ORC_QE);
        const double mee = (ORC_ME * ORC_ME) / (ORC_ME + ORC_ME);
        const double kee = qe4 / (((8.0 * ORC_PI) * (ORC_EPS0 * ORC_EPS0)) * (mee * mee));
        double a_full = (kee * lnl) * r->dt;
        double a_half = (kee * lnl) * (0.5 * r->dt);
        double nunit = (r->w0 * (double)ne) / r->volume;
        const int32_t *p = x->perm_e;
        int start = 0;
        if (ne % 2 == 1 && ne >= 3) {
            collide_pair(x, c, p[0], 0, p[1], a_half, nunit, 0, P_EE_TRI, 0);
            collide_pair(x, c, p[1], 0, p[2], a_half, nunit, 1, P_EE_TRI, 0);
            collide_pair(x, c, p[2], 0, p[0], a_half, nunit, 2, P_EE_TRI, 0);
            x->cnt[OC_TRIPLET] += 3;
            start = 3;
        }
        for (int j = 0; start + 2 * j + 1 < ne; ++j) {
            collide_pair(x, c, p[start + 2 * j], 0, p[start + 2 * j + 1], a_full, nunit,
                         (uint32_t)j, P_EE, 0);
            x->cnt[OC_EE]++;
        }
    }

    /* S2: electron-ion pairs, round robin over the smaller population */
    if ((flags & ORC_EI) && ne >= 1 && ni >= 1 && have_pe) {
        make_perm(x, P_PERM_I, ni, x->perm_i);
        const double qe4 = (ORC_QE * ORC_QE) * (ORC_QE * ORC_QE);
        const double mei = (ORC_ME * mi) / (ORC_ME + mi);
        const double kei = qe4 / (((8.0 * ORC_PI) * (ORC_EPS0 * ORC_EPS0)) * (mei * mei));
        double a1 = (kei * lnl) * r->dt;
        int nmin = ne < ni ? ne : ni, nmax = ne < ni ? ni : ne;
        double nunit = (r->w0 * (double)nmin) / r->volume;
        for (int kk = 0; kk < nmax; ++kk) {
            int e, i;
            if (ne >= ni) { e = x->perm_e[kk]; i = x->perm_i[kk % ni]; }
            else          { i = x->perm_i[kk]; e = x->perm_e[kk % ne]; }
            int z = c->iz[i];
            x->cnt[OC_EI]++;
            if (z == 0) continue;
            collide_pair(x, c, e, 1, i, a1 * (double)(z * z), nunit, (uint32_t)kk, P_EI, 0);
        }
    }

    /* S3: collisional ionization, average cell ion, Lotz cross section */
    if ((flags & ORC_ION) && ne >= 1 && ni >= 1) {
        int64_t sz = 0;
        for (int j = 0; j < ni; ++j) sz += c->iz[j];
        int64_t wi = ni;
        int zc = (int)((2 * sz + wi) / (2 * wi));
        m[11] = zc;
        int ne0 = ne;
        /* the charge states whose cross section is evaluated: the average cell
         * ion Z_c, or (ORC_ION_Z) every charge state an ion of the cell holds */
        int eval[ORC_ZMAX] = {0};
        if (flags & ORC_ION_Z) {
            for (int i = 0; i < ni; ++i)
                if (c->iz[i] < ORC_ZMAX) eval[c->iz[i]] = 1;
        } else if (zc < ORC_ZMAX) {
            eval[zc] = 1;
        }
        double pz[ORC_ZMAX];
        int nz = 0;
        double pmax = 0.0;
        for (int z = 0; z < ORC_ZMAX; ++z) {
            pz[z] = 0.0;
            if (!eval[z]) continue;
            for (int j = 0; j < ne0; ++j) {
                double v2 = (c->evx[j] * c->evx[j] + c->evy[j] * c->evy[j]) + c->evz[j] * c->evz[j];
                double e = HALF_ME_OVER_QE * v2;
                double sig = orc_lotz(t, z, dE, e);
                x->scratch[j] = ((double)c->ew[j] * sig) * sqrt(v2);
            }
            double ssum = tree_sum(x->scratch, ne0);
            double p = ((ssum * r->w0) * r->dt) / r->volume;
            if (p > 1.0) { p = 1.0; x->cnt[OC_P_CLAMPED]++; }
            pz[z] = p;
            if (p > pmax) pmax = p;
            ++nz;
            /* clamp events of the per-cell lowered levels used by Lotz */
            int occ[ORC_NSUB];
            orc_occupancy(z, 0, occ);
            for (int q = 0; q < ORC_NSUB; ++q)
                if (occ[q] > 0 && t->bind[z][q] - dE[z] < 1.0) x->cnt[OC_IPD_CLAMPED]++;
        }
        if (flags & ORC_ION_Z) m[11] = nz;
        if (nz > 0) {
            m[12] = pmax;
            int nfired = 0;
            for (int i = 0; i < ni; ++i) {
                x->perm_a[i] = 0;
                if (c->iz[i] >= ORC_ZMAX) continue;
                double p = (flags & ORC_ION_Z) ? pz[c->iz[i]] : pz[zc];
                uint32_t d[4];
                rng(x, (uint32_t)i, P_ION, 0, d);
                if (orc_u32(d[0]) < p) { x->perm_a[i] = 1; nfired++; }
            }
            x->cnt[OC_ION_FIRED] += nfired;
            if (nfired > 0) {
                double u[3], kth;
                int64_t wsum;
                drift_frame(x, c, ne0, c->ew, u, &kth, &wsum);
                m[13] = kth;
                double debit = 0.0;
                int accepted = 0;
                for (int i = 0; i < ni; ++i) {
                    if (!x->perm_a[i]) continue;
                    int z = c->iz[i], kv = c->ik[i];
                    int sv = orc_valence(z, kv);
                    double ip = lowered(x, z, sv, dE, 0);
                    if (!(debit + ip <= kth)) break;
                    debit = debit + ip;
                    c->iz[i] = (uint8_t)(z + 1);
                    if (sv == 0) c->ik[i] = (uint8_t)(kv + 1);
                    cell_push_e(c, c->ix[i], c->iy[i], 0.0, 0.0, 0.0, 1);
                    x->cnt[OC_E_NEW]++;
                    x->led[OL_ION_DEBIT] += ip;
                    accepted++;
                }
                x->cnt[OC_ION_ACCEPTED] += accepted;
                x->cnt[OC_ION_STARVED] += nfired - accepted;
                m[14] = debit;
                if (debit > 0.0) {
                    double alpha = sqrt(1.0 - debit / kth);
                    for (int j = 0; j < ne0; ++j) {
                        c->evx[j] = u[0] + alpha * (c->evx[j] - u[0]);
                        c->evy[j] = u[1] + alpha * (c->evy[j] - u[1]);
                        c->evz[j] = u[2] + alpha * (c->evz[j] - u[2]);
                    }
                }
            }
        }
        ne = c->ne;
    }

    /* S4: three-body recombination towards Zbar_EOS(n_i, T_e) */
    if ((flags & ORC_REC) && ne >= 1 && ni >= 1) {
        int64_t sz = 0, we = 0, wb = 0;
        for (int j = 0; j < ni; ++j) sz += c->iz[j];
        for (int j = 0; j < ne; ++j) {
            we += c->ew[j];
            double e = e_kin(c, j);
            int bulk = e < r->e_bulk;
            x->scratch[j] = bulk ? (double)c->ew[j] * e : 0.0;
            if (bulk) wb += c->ew[j];
        }
        double ke = tree_sum(x->scratch, ne);
        double tp = 0.01;
        if (wb > 0) {
            tp = (2.0 * ke) / (3.0 * (double)wb);
            if (tp < 0.01) tp = 0.01;
        }
        m[15] = tp;
        int64_t nrec = 0;
        int *sel_i = x->perm_a;          /* reuse: chosen ions in order */
        if (flags & ORC_REC_XS) {
            /* per ion from its own charge state's rate (orc_rec_xs) at the
             * temperature and electron density after S3: every ion with
             * Z > z_floor draws U32(word 0 of its REC_XS call) against its
             * probability; the firing ions recombine in slot order, at most
             * one per electron */
            double n_e = ((double)we * r->w0) / r->volume;
            double prec[ORC_ZMAX + 1];
            int held[ORC_ZMAX + 1] = {0};
            for (int j = 0; j < ni; ++j) held[c->iz[j]] = 1;
            for (int z = 0; z <= ORC_ZMAX; ++z) {
                prec[z] = 0.0;
                if (!held[z] || z <= r->z_floor || z < 1) continue;
                double pz = orc_rec_xs(t, z, tp, n_e, dE, r->dt);
                if (pz > 1.0) {
                    pz = 1.0;
                    x->cnt[OC_P_CLAMPED]++;
                }
                prec[z] = pz;
            }
            for (int i = 0; i < ni && nrec < ne; ++i) {
                int z = c->iz[i];
                if (z <= r->z_floor || !(prec[z] > 0.0)) continue;
                uint32_t d[4];
                rng(x, (uint32_t)i, P_REC_XS, 0, d);
                if (orc_u32(d[0]) < prec[z]) sel_i[nrec++] = i;
            }
        } else {
            double n_i = ((double)ni * r->w0) / r->volume;
            double zeos = orc_eos(t, n_i, tp);
            double dd = (double)sz - (double)ni * zeos;
            if (dd > 0.0) {
                nrec = (int64_t)floor(dd + 0.5);
                int nelig = 0;
                for (int j = 0; j < ni; ++j) nelig += c->iz[j] > r->z_floor;
                if (nrec > nelig) nrec = nelig;
                if (nrec > ne) nrec = ne;
                if (nrec > 0) {
                    make_perm(x, P_REC_I, ni, x->perm_i);
                    int got = 0;
                    for (int q = 0; q < ni && got < nrec; ++q) {
                        int i = x->perm_i[q];
                        if (c->iz[i] > r->z_floor) sel_i[got++] = i;
                    }
                }
            }
        }
        {
            if (nrec > 0) {
                make_perm(x, P_REC_E, ne, x->perm_b);
                uint32_t *wp = malloc(sizeof(uint32_t) * (size_t)ne);
                for (int j = 0; j < ne; ++j) wp[j] = c->ew[j];
                for (int q = 0; q < nrec; ++q) wp[x->perm_b[q]] -= 1;
                double u[3], kth;
                int64_t wsum;
                drift_frame(x, c, ne, wp, u, &kth, &wsum);
                if (wsum == 0 || !(kth > 0.0)) {
                    x->cnt[OC_REC_SKIPPED]++;
                } else {
                    double eadd = 0.0;
                    const double half_mi = (0.5 * mi) / ORC_QE;
                    const double ratio = ORC_ME / mi;
                    for (int q = 0; q < nrec; ++q) {
                        int e = x->perm_b[q], i = sel_i[q];
                        double keu = e_kin(c, e);
                        double v2b = (c->ivx[i] * c->ivx[i] + c->ivy[i] * c->ivy[i]) + c->ivz[i] * c->ivz[i];
                        double kib = half_mi * v2b;
                        c->ivx[i] = c->ivx[i] + ratio * c->evx[e];
                        c->ivy[i] = c->ivy[i] + ratio * c->evy[e];
                        c->ivz[i] = c->ivz[i] + ratio * c->evz[e];
                        double v2a = (c->ivx[i] * c->ivx[i] + c->ivy[i] * c->ivy[i]) + c->ivz[i] * c->ivz[i];
                        double kia = half_mi * v2a;
                        int z = c->iz[i], kv = c->ik[i];
                        int occ0[ORC_NSUB], occ1[ORC_NSUB];
                        orc_occupancy(z, kv, occ0);
                        int kn = (kv >= 1 && occ0[1] + occ0[2] == 8) ? kv - 1 : kv;
                        orc_occupancy(z - 1, kn, occ1);
                        int sl = 0;
                        for (int q2 = 0; q2 < ORC_NSUB; ++q2)
                            if (occ1[q2] > occ0[q2]) { sl = q2; break; }
                        double ipr = lowered(x, z - 1, sl, dE, 0);
                        c->iz[i] = (uint8_t)(z - 1);
                        c->ik[i] = (uint8_t)kn;
                        eadd = eadd + ((keu + ipr) + (kib - kia));
                        x->led[OL_REC_BIND] += ipr;
                    }
                    x->cnt[OC_REC] += nrec;
                    x->led[OL_REC_ADD] += eadd;
                    double alpha = sqrt(1.0 + eadd / kth);
                    int o = 0;
                    for (int j = 0; j < ne; ++j) {
                        if (wp[j] == 0) continue;
                        c->ex[o] = c->ex[j]; c->ey[o] = c->ey[j];
                        c->evx[o] = u[0] + alpha * (c->evx[j] - u[0]);
                        c->evy[o] = u[1] + alpha * (c->evy[j] - u[1]);
                        c->evz[o] = u[2] + alpha * (c->evz[j] - u[2]);
                        c->ew[o] = wp[j];
                        ++o;
                    }
                    x->cnt[OC_E_REMOVED] += ne - o;
                    c->ne = o;
                }
                free(wp);
            }
        }
        ne = c->ne;
    }

    /* S5: K-vacancy decay (Auger / K-alpha) then subshell photoionization */
    if (flags & (ORC_PHOTO | ORC_DECAY)) {
        int nb = r->n_bins;
        int photo = (flags & ORC_PHOTO) && nb > 0;
        const double *nhv = s->cell_nhv ? s->cell_nhv + (size_t)x->cell * nb : r->nhv;
        double ssum[13][3];
        /* ORC_PHOTO_FRAC: macro-photons of each bin held by the cell, and
         * those taken so far this step */
        double budget[ORC_MAX_BINS], used[ORC_MAX_BINS];
        for (int b = 0; b < nb; ++b) {
            budget[b] = (nhv[b] * r->volume) / r->w0;
            used[b] = 0.0;
        }
        /* ORC_KA_FIELD: K-alpha photons per charge state Z0 */
        int64_t nka_z[ORC_ZMAX] = {0};
        if (photo) {
            for (int z = 0; z < 13; ++z)
                for (int q = 0; q < 3; ++q) {
                    double pp = t->bind[z][q] - dE[z];
                    if (pp < 1.0) pp = 1.0;
                    double acc = 0.0;
                    for (int b = 0; b < nb; ++b)
                        if (r->hv[b] >= pp) acc = acc + nhv[b] * s->sigma[b][q];
                    ssum[z][q] = acc;
                }
        }
        int nion = c->ni;
        for (int i = 0; i < nion; ++i) {
            int z0 = c->iz[i], k0 = c->ik[i];
            if (z0 >= ORC_ZMAX) continue;
            int occ0[ORC_NSUB];
            orc_occupancy(z0, k0, occ0);
            int nl0 = occ0[1] + occ0[2];
            int z = z0, kv = k0;
            if ((flags & ORC_DECAY) && k0 >= 1 && nl0 >= 1) {
                double ga = t->gamma_a[z0][k0], gx = t->gamma_x[z0][k0];
                double rate = ga + gx;
                if (rate > 0.0) {
                    uint32_t d[4];
                    rng(x, (uint32_t)i, P_DECAY, 0, d);
                    double pd = r->dt_rad * rate;
                    if (pd > 1.0) { pd = 1.0; x->cnt[OC_P_CLAMPED]++; }
                    if (orc_u52(d[0], d[1]) < pd) {
                        kv = k0 - 1;
                        x->cnt[OC_DECAY]++;
                        double pa = ga / rate;
                        if (nl0 >= 2 && orc_u52(d[2], d[3]) < pa) {
                            z = z0 + 1;
                            double p2s = lowered(x, z0, 1, dE, 0);
                            double p2p = lowered(x, z0, 2, dE, 0);
                            double num = (double)occ0[1] * p2s + (double)occ0[2] * p2p;
                            double ea = t->e_kalpha[z0] - num / (double)nl0;
                            if (ea < 0.0) ea = 0.0;
                            new_electron_dir(x, c, i, 0, ea);
                            x->cnt[OC_AUGER]++;
                            x->led[OL_AUGER_E] += ea;
                        } else {
                            x->cnt[OC_KALPHA]++;
                            x->led[OL_KALPHA] += t->e_kalpha[z0];
                            nka_z[z0]++;
                        }
                    }
                }
            }
            if (photo) {
                uint32_t fire[4];
                rng(x, (uint32_t)i, P_ION, 0, fire);
                for (int q = 0; q < 3; ++q) {
                    if (occ0[q] <= 0) continue;
                    double sum = ssum[z0][q];
                    if (!(sum > 0.0)) continue;
                    double p = ((ORC_CLIGHT * r->dt_rad) * (double)occ0[q]) * sum;
                    if (p > 1.0) { p = 1.0; x->cnt[OC_P_CLAMPED]++; }
                    if (!(orc_u32(fire[1 + q]) < p)) continue;
                    int occn[ORC_NSUB];
                    orc_occupancy(z, kv, occn);
                    if (z >= ORC_ZMAX || occn[q] <= 0) { x->cnt[OC_PHOTO_SKIPPED]++; continue; }
                    double pp = lowered(x, z0, q, dE, 0);
                    uint32_t d[4];
                    rng(x, (uint32_t)i, P_BIN, (uint32_t)q, d);
                    double target = orc_u52(d[0], d[1]) * sum;
                    double cum = 0.0;
                    int sel = -1, lastpos = -1;
                    for (int b = 0; b < nb; ++b) {
                        if (!(r->hv[b] >= pp)) continue;
                        double term = nhv[b] * s->sigma[b][q];
                        cum = cum + term;
                        if (term > 0.0) lastpos = b;
                        if (cum > target) { sel = b; break; }
                    }
                    if (sel < 0) sel = lastpos;
                    if (flags & ORC_PHOTO_FRAC) {
                        /* one macro-photon per event while the bin has one;
                         * with less than one left (f) the event is a partial
                         * photoionization: a macro-photoelectron of weight f
                         * units taking f of a unit of charge, which integer
                         * weights carry as an event of probability f */
                        double rem = budget[sel] - used[sel];
                        if (rem >= 1.0) {
                            used[sel] = used[sel] + 1.0;
                        } else if (rem > 0.0) {
                            used[sel] = budget[sel];
                            uint32_t e[4];
                            rng(x, (uint32_t)i, P_PART, (uint32_t)q, e);
                            if (!(orc_u32(e[0]) < rem)) {
                                x->cnt[OC_PHOTO_STARVED]++;
                                continue;
                            }
                            x->cnt[OC_PHOTO_PARTIAL]++;
                        } else {
                            x->cnt[OC_PHOTO_STARVED]++;
                            continue;
                        }
                    }
                    z = z + 1;
                    if (q == 0) kv = kv + 1;
                    double ep = r->hv[sel] - pp;
                    new_electron_dir(x, c, i, (uint32_t)(1 + q), ep);
                    x->cnt[OC_PHOTO_1S + q]++;
                    x->led[OL_PHOTO_E] += ep;
                    x->led[OL_PHOTON_ABS] += r->hv[sel];
                    x->nabs[sel]++;
                }
            }
            c->iz[i] = (uint8_t)z;
            c->ik[i] = (uint8_t)kv;
        }
        if (flags & ORC_KA_FIELD) {
            /* each K-alpha photon's energy goes to the bin of the largest
             * h nu not above it, as E_Ka / h nu photons of that bin (energy
             * kept, never promoted above its own energy); with no such bin
             * it leaves the plasma */
            for (int z0 = 0; z0 < ORC_ZMAX; ++z0) {
                if (nka_z[z0] == 0) continue;
                double eka = t->e_kalpha[z0];
                int kb = -1;
                for (int b = 0; b < nb; ++b)
                    if (r->hv[b] <= eka && (kb < 0 || r->hv[b] > r->hv[kb])) kb = b;
                if (kb < 0) continue;
                x->nka[kb] = x->nka[kb] + (double)nka_z[z0] * (eka / r->hv[kb]);
                x->cnt[OC_KA_FIELD] += nka_z[z0];
            }
        }
    }
    if (flags & ORC_THERM) thermalize(x, c);
}

void orc_step(orc_sim *s, uint32_t step, uint32_t flags, int32_t nthreads)
{
    int maxp = 1;
    for (int c = 0; c < s->ncells; ++c) {
        int n = s->cells[c].ne + 5 * s->cells[c].ni + 8;
        if (s->cells[c].ni > n) n = s->cells[c].ni;
        if (n > maxp) maxp = n;
    }
    int pad = 1;
    while (pad < maxp) pad *= 2;
    memset(s->cnt, 0, sizeof(int64_t) * (size_t)s->ncells * OC_NCOUNT);
    memset(s->led, 0, sizeof(double) * (size_t)s->ncells * OL_NLEDGER);
    memset(s->nabs, 0, sizeof(int32_t) * (size_t)s->ncells * ORC_MAX_BINS);
    memset(s->nka, 0, sizeof(double) * (size_t)s->ncells * ORC_MAX_BINS);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        cctx x;
        x.s = s;
        x.step = step;
        x.law = ((flags & ORC_NANBU) ? 1 : 0) | ((flags & ORC_REL) ? 2 : 0);
        x.key[0] = (uint32_t)s->r.seed;
        x.key[1] = (uint32_t)(s->r.seed >> 32);
        x.scratch = malloc(sizeof(double) * (size_t)pad);
        x.perm_e = malloc(sizeof(int32_t) * (size_t)pad);
        x.perm_i = malloc(sizeof(int32_t) * (size_t)pad);
        x.perm_a = malloc(sizeof(int32_t) * (size_t)pad);
        x.perm_b = malloc(sizeof(int32_t) * (size_t)pad);
        x.keys = malloc(sizeof(uint32_t) * (size_t)pad);
#pragma omp for schedule(dynamic, 16)
        for (int c = 0; c < s->ncells; ++c) {
            x.cell = (uint32_t)c;
            x.cnt = s->cnt + (size_t)c * OC_NCOUNT;
            x.led = s->led + (size_t)c * OL_NLEDGER;
            x.nabs = s->nabs + (size_t)c * ORC_MAX_BINS;
            x.nka = s->nka + (size_t)c * ORC_MAX_BINS;
            step_cell(&x, &s->cells[c], flags);
        }
        free(x.scratch); free(x.perm_e); free(x.perm_i); free(x.perm_a); free(x.perm_b); free(x.keys);
    }
}

/* Run diagnostics: charge-state distribution, electron energy histogram
 * (64 log bins from 0.1 eV to 1e5 eV, weight units) and
 * out = {W_e, W_i, sum Z, Zbar, K_e (eV units), T_e, ncells, sum w E^2 / 1e6}. */
void orc_diag(const orc_sim *s, int64_t csd[ORC_ZMAX + 1], int64_t fe[64], double out[8])
{
    memset(csd, 0, sizeof(int64_t) * (ORC_ZMAX + 1));
    memset(fe, 0, sizeof(int64_t) * 64);
    int64_t we = 0, wi = 0, sz = 0;
    int p = 1;
    while (p < s->ncells) p *= 2;
    double *kc = calloc((size_t)p, sizeof(double));
    int maxn = 1;
    for (int c = 0; c < s->ncells; ++c) if (s->cells[c].ne > maxn) maxn = s->cells[c].ne;
    int q = 1;
    while (q < maxn) q *= 2;
    double *sc = calloc((size_t)q, sizeof(double));
    const double lmin = orc_log(0.1), dl = (orc_log(1.0e5) - orc_log(0.1)) / 64.0;
    for (int c = 0; c < s->ncells; ++c) {
        const ocell *cl = &s->cells[c];
        for (int j = 0; j < cl->ni; ++j) { csd[cl->iz[j]]++; wi++; sz += cl->iz[j]; }
        for (int j = 0; j < cl->ne; ++j) {
            double e = e_kin(cl, j);
            we += cl->ew[j];
            sc[j] = (double)cl->ew[j] * e;
            int b = 0;
            if (e > 0.0) {
                double u = (orc_log(e) - lmin) / dl;
                b = u < 0.0 ? 0 : (u >= 63.0 ? 63 : (int)u);
            }
            fe[b] += cl->ew[j];
        }
        kc[c] = tree_sum(sc, cl->ne);
    }
    double ke = tree_sum(kc, s->ncells);
    out[0] = (double)we; out[1] = (double)wi; out[2] = (double)sz;
    out[3] = wi > 0 ? (double)sz / (double)wi : 0.0;
    out[4] = ke;
    out[5] = we > 0 ? (2.0 * ke) / (3.0 * (double)we) : 0.0;
    out[6] = (double)s->ncells;
    out[7] = 0.0;
    free(kc);
    free(sc);
}
