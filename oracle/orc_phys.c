/*
 * Oracle single-physics pieces.  TEST INFRASTRUCTURE ONLY.
 *
 * Constants are CODATA 2018 in SI; energies and temperatures in eV.  Each
 * formula is written with the operand order that the specification of the
 * method fixes, so that an independent implementation can reproduce it bit
 * for bit.
 */
#include <math.h>
#include <stdint.h>

#include "orc.h"
#include "orc_internal.h"

void orc_occupancy(int32_t z, int32_t k, int32_t occ[ORC_NSUB])
{
    /* Lowest-energy configuration of charge state z with k K vacancies
     * (Sec. III: only Z_i and the K-vacancy count are stored per ion). */
    static const int cap[ORC_NSUB] = {2, 2, 6, 2, 6};
    int nb = ORC_ZMAX - z;
    int k1s = 2 - k;
    if (k1s > nb) k1s = nb;
    if (k1s < 0) k1s = 0;
    occ[0] = k1s;
    int rem = nb - k1s;
    for (int s = 1; s < ORC_NSUB; ++s) {
        int c = rem < cap[s] ? rem : cap[s];
        occ[s] = c;
        rem -= c;
    }
}

/* Outermost occupied subshell, or -1 for a bare nucleus. */
int orc_valence(int z, int k)
{
    int occ[ORC_NSUB];
    orc_occupancy(z, k, occ);
    for (int s = ORC_NSUB - 1; s >= 0; --s)
        if (occ[s] > 0) return s;
    return -1;
}

/*
 * Ionization potential depression of charge state z (Sec. V).
 *   Ecker-Kroll (Eq. 5): C = 1, applied when n = n_e + n_i exceeds the critical
 *   density n_crit = (3/4pi)(4 pi eps0 kT / ((z+1)^2 e^2))^3; below it the
 *   Debye-Hueckel shift (z+1) e^2 / (4 pi eps0 lambda_D) is used.
 *   Stewart-Pyatt (Eq. 6) with K = (z+1) e^2 / (4 pi eps0 lambda_D kT),
 *   lambda_D = sqrt(eps0 kT / (e^2 n_e (Zbar + 1))) taking T_i = T_e, and
 *   z* = <Z^2>/<Z>.
 */
double orc_ipd(int32_t model, int32_t z, double t, double n_e, double n_i,
               double zbar, double zstar)
{
    double lamd = INFINITY;
    if (n_e > 0.0) lamd = sqrt((ORC_EPS0 * t) / (ORC_QE * (n_e * (zbar + 1.0))));
    double zp1 = (double)(z + 1);
    if (model == 1) {
        double ntot = n_e + n_i;
        double c = t / ((zp1 * zp1) * ORC_E2);
        double ncrit = ORC_THREE_OVER_4PI * ((c * c) * c);
        if (ntot > ncrit) {
            double rek = orc_cbrt(ORC_THREE_OVER_4PI / ntot);
            return (zp1 * ORC_E2) / rek;
        }
        return (zp1 * ORC_E2) / lamd;
    }
    double kk = (zp1 * ORC_E2) / (lamd * t);
    double zs1 = zstar + 1.0;
    double y = ((3.0 * zs1) * kk) + 1.0;
    double c = orc_cbrt(y);
    return (t / (2.0 * zs1)) * ((c * c) - 1.0);
}

/* Coulomb logarithm per cell: max(2, ln(1 + (lambda_De / b_min)^2) / 2). */
double orc_coulomb_log(double t, double n_e, double zbar)
{
    if (!(n_e > 0.0)) return 2.0;
    double lamde = sqrt((ORC_EPS0 * t) / (ORC_QE * n_e));
    double bcl = (zbar * ORC_E2) / (3.0 * t);
    double bq = ORC_HBAR / (2.0 * sqrt((3.0 * ORC_ME) * (t * ORC_QE)));
    double bmin = bcl > bq ? bcl : bq;
    double ratio = lamde / bmin;
    double lnl = 0.5 * orc_log(1.0 + ratio * ratio);
    return lnl < 2.0 ? 2.0 : lnl;
}

/*
 * Lotz cross section (Eq. 4) of the average cell ion of charge zc in its
 * ground configuration, with binding energies lowered by dE[zc] (clamped at
 * 1 eV); m^2.  ln(E/P) is evaluated as ln E - ln P.
 */
double orc_lotz(const orc_tables *t, int32_t zc, const double dE[13], double e)
{
    if (zc >= ORC_ZMAX || !(e > 0.0)) return 0.0;
    int occ[ORC_NSUB];
    orc_occupancy(zc, 0, occ);
    double lne = orc_log(e);
    double sig = 0.0;
    for (int s = 0; s < ORC_NSUB; ++s) {
        if (occ[s] <= 0) continue;
        double p = t->bind[zc][s] - dE[zc];
        if (p < 1.0) p = 1.0;
        if (!(e > p)) continue;
        double lnp = orc_log(p);
        double term = (((t->lotz_a[s] * 1.0e-4) * (double)occ[s]) * (lne - lnp)) / (e * p);
        if (t->lotz_b[s] != 0.0)
            term = term * (1.0 - t->lotz_b[s] * orc_exp(-(t->lotz_c[s] * (e / p - 1.0))));
        sig = sig + term;
    }
    return sig;
}

/*
 * exp(x) E1(x), x > 0.  E1(x) = -gamma - ln x - sum_{k>=1} (-x)^k / (k k!) for
 * x <= 1 (24 terms), and for x > 1 the continued fraction
 * E1(x) = exp(-x) / (x + 1 - 1/(x + 3 - 4/(x + 5 - 9/(x + 7 - ...)))) evaluated
 * backward from depth 80 (Abramowitz & Stegun 5.1.22 contracted).
 * Pinned against scipy.special.exp1 by tests/test_oracle_recxs.py.
 */
double orc_e1x(double x)
{
    if (x <= 1.0) {
        double sum = 0.0, term = 1.0;
        for (int k = 1; k <= 24; ++k) {
            term = (term * (-x)) / (double)k;
            sum = sum + term / (double)k;
        }
        double e1 = (-0.57721566490153286 - orc_log(x)) - sum;
        return orc_exp(x) * e1;
    }
    double t = x + 161.0;
    for (int k = 80; k >= 1; --k) t = (x + (double)(2 * k - 1)) - (double)(k * k) / t;
    return 1.0 / t;
}

/* Degeneracy of the ground configuration of charge state z: the product over
 * subshells of C(capacity, occupancy). */
static double ground_degeneracy(int32_t z)
{
    static const int cap[ORC_NSUB] = {2, 2, 6, 2, 6};
    int occ[ORC_NSUB];
    orc_occupancy(z, 0, occ);
    double g = 1.0;
    for (int s = 0; s < ORC_NSUB; ++s) {
        double c = 1.0;
        for (int j = 0; j < occ[s]; ++j) c = (c * (double)(cap[s] - j)) / (double)(j + 1);
        g = g * c;
    }
    return g;
}

/*
 * Three-body recombination z -> z-1 from cross sections (Sec. IV names it as
 * the model's next step).  Detailed balance with the collisional ionization
 * of z-1 (Lotz, Eq. 4):  the recombination rate per ion of charge z is
 * S_{z-1}(T) n_e^2 / Phi_z(T), where
 *   S_{z-1} = sum_s a_s N_s vbar / (P_s T) [E1(x_s) - b_s e^{c_s} x_s / (x_s + c_s) E1(x_s + c_s)],
 *     x_s = P_s / T, over the occupied subshells of the ground configuration of
 *     z - 1 with their lowered bindings P_s, vbar = sqrt(8 k T / (pi m_e)),
 *   Phi_z = 2 (g_z / g_{z-1}) (m_e k T / (2 pi hbar^2))^{3/2} exp(-P_v / T),
 *     the Saha factor with the lowered binding P_v of the valence subshell of
 *     z - 1 and ground-configuration degeneracies g.
 * The probability per step is that rate times dt.  Both exponentials are
 * folded together: S e^{x_v} uses exp(x) E1(x) and e^{x_v - x_s} <= 1.
 */
double orc_rec_xs(const orc_tables *t, int32_t z, double tev, double n_e, const double dE[13],
                  double dt)
{
    if (z < 1 || z > ORC_ZMAX || !(n_e > 0.0) || !(tev > 0.0)) return 0.0;
    int zl = z - 1;
    int occ[ORC_NSUB];
    orc_occupancy(zl, 0, occ);
    int v = orc_valence(zl, 0);
    double pv = t->bind[zl][v] - dE[zl];
    if (pv < 1.0) pv = 1.0;
    double xv = pv / tev;
    double vbar = sqrt((8.0 * (tev * ORC_QE)) / (ORC_PI * ORC_ME));
    double sum = 0.0;
    for (int s = 0; s < ORC_NSUB; ++s) {
        if (occ[s] <= 0) continue;
        double p = t->bind[zl][s] - dE[zl];
        if (p < 1.0) p = 1.0;
        double x = p / tev;
        double br = orc_e1x(x);
        if (t->lotz_b[s] != 0.0) {
            double c = t->lotz_c[s];
            br = br - (t->lotz_b[s] * (x / (x + c))) * orc_e1x(x + c);
        }
        double term = ((((t->lotz_a[s] * 1.0e-4) * (double)occ[s]) * vbar) / (p * tev)) * (br * orc_exp(xv - x));
        sum = sum + term;
    }
    double q = (ORC_ME * (tev * ORC_QE)) / ((2.0 * ORC_PI) * (ORC_HBAR * ORC_HBAR));
    double phi0 = (2.0 * (ground_degeneracy(z) / ground_degeneracy(zl))) * (q * sqrt(q));
    return ((sum * (n_e * n_e)) * dt) / phi0;
}

/* Zbar_EOS(n_i, T): bilinear in (ln n_i, ln T) on the table grid, clamped. */
double orc_eos(const orc_tables *t, double n_i, double tev)
{
    double u = (orc_log(n_i) - t->eos_lnn0) / t->eos_dlnn;
    double v = (orc_log(tev) - t->eos_lnt0) / t->eos_dlnt;
    int nn = t->eos_nn, nt = t->eos_nt;
    double fu = floor(u), fv = floor(v);
    int iu = (int)fu, iv = (int)fv;
    double au = u - fu, av = v - fv;
    if (u < 0.0) { iu = 0; au = 0.0; }
    if (v < 0.0) { iv = 0; av = 0.0; }
    if (iu > nn - 2) { iu = nn - 2; au = 1.0; }
    if (iv > nt - 2) { iv = nt - 2; av = 1.0; }
    const double *z = t->eos_zbar;
    double z00 = z[iu * nt + iv], z01 = z[iu * nt + iv + 1];
    double z10 = z[(iu + 1) * nt + iv], z11 = z[(iu + 1) * nt + iv + 1];
    double a = (1.0 - av) * z00 + av * z01;
    double b = (1.0 - av) * z10 + av * z11;
    return (1.0 - au) * a + au * b;
}

/* Neutral-atom subshell photoionization cross section per electron, m^2
 * (Sec. III, Fig. 2a): linear interpolation in ln sigma vs ln hv, clamped. */
double orc_photo_sigma(const orc_tables *t, int32_t s, double hv)
{
    double u = (orc_log(hv) - t->photo_lnhv0) / t->photo_dlnhv;
    double fu = floor(u);
    int iu = (int)fu;
    double a = u - fu;
    if (u < 0.0) { iu = 0; a = 0.0; }
    if (iu > t->photo_nh - 2) { iu = t->photo_nh - 2; a = 1.0; }
    double l0 = t->photo_lnsig[s][iu], l1 = t->photo_lnsig[s][iu + 1];
    double ls = l0 + a * (l1 - l0);
    return orc_exp(ls) * 1.0e-4;
}

/* Nanbu's cumulative small-angle scattering (Nanbu, Phys. Rev. E 55, 4642
 * (1997)): over one step the many small deflections of a pair add up to one
 * angle chi whose cosine has the density A exp(A cos chi) / (2 sinh A), with A
 * fixed by the mean deflection, <cos chi> = coth A - 1/A = exp(-s).
 *
 * orc_nanbu_a(s) returns that A.
 *   s <= 0.05: A >= 20, where coth A differs from 1 by less than 2 exp(-40),
 *     so the equation reads 1 - 1/A = exp(-s): A = 1 / (1 - exp(-s)), with
 *     1 - exp(-s) from its series s (1 - s/2 (1 - s/3 (1 - ... (1 - s/11)))).
 *   0.05 < s < 15: four Newton steps on L(A) = coth A - 1/A = m, m = exp(-s),
 *     from the Pade start A = m (3 - m^2) / (1 - m^2).  L and L' come from the
 *     Laurent series of coth (Bernoulli coefficients 2^2n B_2n / (2n)!,
 *     eleven terms) for A < 0.5 and from E = exp(-2A) above:
 *     L = (1 + E) / (1 - E) - 1/A, L' = 1/A^2 - 4E / (1 - E)^2.
 *   s >= 15: 0, the isotropic limit (<cos chi> = exp(-15) = 3e-7).
 * Pinned by tests/test_oracle_nanbu.py: L(A) against exp(-s) in 50-digit
 * decimal arithmetic, the sampled law against its distribution function, and
 * the composition of deflections over steps. */
static void langevin(double a, double *l, double *dl)
{
    if (a < 0.5) {
        static const double c[11] = {
            1.0 / 3.0, -1.0 / 45.0, 2.0 / 945.0, -1.0 / 4725.0, 2.0 / 93555.0,
            -1382.0 / 638512875.0, 4.0 / 18243225.0, -3617.0 / 162820783125.0,
            87734.0 / 38979295480125.0, -349222.0 / 1531329465290625.0,
            310732.0 / 13447856940643125.0};
        double z = a * a;
        double v = c[10], dv = 21.0 * c[10];
        for (int k = 9; k >= 0; --k) {
            v = c[k] + z * v;
            dv = (double)(2 * k + 1) * c[k] + z * dv;
        }
        *l = a * v;
        *dl = dv;
        return;
    }
    double e = orc_exp(-2.0 * a);
    double ome = 1.0 - e;
    *l = (1.0 + e) / ome - 1.0 / a;
    *dl = 1.0 / (a * a) - (4.0 * e) / (ome * ome);
}

double orc_nanbu_a(double s)
{
    if (s >= 15.0) return 0.0;
    if (s <= 0.05) {
        double q = 1.0;
        for (int k = 11; k >= 2; --k) q = 1.0 - (s * (1.0 / (double)k)) * q;
        return 1.0 / (s * q);
    }
    double m = orc_exp(-s);
    double m2 = m * m;
    double a = (m * (3.0 - m2)) / (1.0 - m2);
    for (int it = 0; it < 4; ++it) {
        double l, dl;
        langevin(a, &l, &dl);
        a = a - (l - m) / dl;
    }
    return a;
}

/* 1 - cos chi for s and a uniform u in (0, 1): inverting the distribution
 * function, cos chi = 1 + ln(u + (1 - u) exp(-2A)) / A; for A = 0 (isotropic)
 * cos chi = 2u - 1.  Clamped to [0, 2]; s <= 0 gives no deflection. */
double orc_nanbu_omc(double s, double u)
{
    if (!(s > 0.0)) return 0.0;
    double a = orc_nanbu_a(s);
    double omc;
    if (a == 0.0) {
        omc = 2.0 * (1.0 - u);
    } else {
        double e2 = orc_exp(-2.0 * a);
        omc = -orc_log(u + (1.0 - u) * e2) / a;
    }
    if (omc < 0.0) omc = 0.0;
    if (omc > 2.0) omc = 2.0;
    return omc;
}

/*
 * One binary Coulomb collision (Takizuka & Abe, J. Comput. Phys. 25, 205
 * (1977)), non-relativistic, with weighted acceptance.
 *   qq_coef = q_a^2 q_b^2 lnL dt / (8 pi eps0^2 m_ab^2)  (per unit density),
 *   <delta^2> = qq_coef * max(w_a, w_b) * nunit / u^3.
 * The relative velocity u = va - vb is turned by the scattering angle Theta
 * and an azimuth Phi = 2 pi r3 (draw 2); each side moves by its reduced-mass
 * fraction of the change.  The scattering law:
 *   law 0 (Takizuka-Abe): delta = sqrt(<delta^2>) sqrt(-2 ln r1) cos(2 pi r2),
 *     r1 from draw 0 and the angle from draw 1; sin(Theta) = 2 delta/(1+delta^2),
 *     1 - cos(Theta) = 2 delta^2/(1+delta^2);
 *   law 1 (Nanbu): 1 - cos(Theta) = orc_nanbu_omc(2 <delta^2>, U52(draws 0, 1)),
 *     sin(Theta) = sqrt((1 - cos)(1 + cos)); s = 2 <delta^2> gives both laws
 *     the same small-angle mean of 1 - cos(Theta).
 * The heavier-weight side accepts with probability w_light / w_heavy (r4 from
 * draw 3, a 32-bit uniform).
 * Returns <delta^2>, or -1 when the relative velocity is zero (no collision).
 */
double orc_collide(double va[3], double vb[3], double ma, double mb, uint32_t wa,
                   uint32_t wb, double qq_coef, double nunit, const uint32_t draws[4],
                   int32_t law, int32_t *acc_a, int32_t *acc_b)
{
    if (law & 2)
        return orc_collide_rel(va, vb, ma, mb, wa, wb, qq_coef, nunit, draws, law & 1, acc_a, acc_b);
    double ux = va[0] - vb[0], uy = va[1] - vb[1], uz = va[2] - vb[2];
    double u2 = (ux * ux + uy * uy) + uz * uz;
    *acc_a = 0;
    *acc_b = 0;
    if (u2 == 0.0) return -1.0;
    uint32_t wmax = wa > wb ? wa : wb;
    double u = sqrt(u2);
    double d2 = ((qq_coef * (double)wmax) * nunit) / (u2 * u);
    double st, omc;
    if (law & 1) {
        omc = orc_nanbu_omc(2.0 * d2, orc_u52(draws[0], draws[1]));
        st = sqrt(omc * (2.0 - omc));
    } else {
        double r1 = orc_u32(draws[0]);
        double s2, c2;
        orc_sincos2pi((uint64_t)draws[1] << 20, &s2, &c2);
        double g = sqrt(-2.0 * orc_log(r1)) * c2;
        double d = sqrt(d2) * g;
        double dd = d * d;
        double den = 1.0 + dd;
        st = (2.0 * d) / den;
        omc = (2.0 * dd) / den;
    }
    double sp, cp;
    orc_sincos2pi((uint64_t)draws[2] << 20, &sp, &cp);
    double a = st * cp;
    double bb = st * sp;
    double up = sqrt(ux * ux + uy * uy);
    double dux, duy, duz;
    if (up > 0.0) {
        dux = ((ux / up) * uz) * a - ((uy / up) * u) * bb - ux * omc;
        duy = ((uy / up) * uz) * a + ((ux / up) * u) * bb - uy * omc;
        duz = -(up * a) - uz * omc;
    } else {
        double auz = fabs(uz);
        dux = auz * a;
        duy = auz * bb;
        duz = -(uz * omc);
    }
    double r4 = orc_u32(draws[3]);
    int ta = (wa <= wb) || (r4 < (double)wb / (double)wa);
    int tb = (wb <= wa) || (r4 < (double)wa / (double)wb);
    double fa = mb / (ma + mb);
    double fb = ma / (ma + mb);
    if (ta) {
        va[0] = va[0] + fa * dux;
        va[1] = va[1] + fa * duy;
        va[2] = va[2] + fa * duz;
    }
    if (tb) {
        vb[0] = vb[0] - fb * dux;
        vb[1] = vb[1] - fb * duy;
        vb[2] = vb[2] - fb * duz;
    }
    *acc_a = ta;
    *acc_b = tb;
    return d2;
}

/*
 * Relativistic binary collision (the COM-frame Monte-Carlo collision of
 * Perez, Gremillet, Decoster, Drouin, Lefebvre, Phys. Plasmas 19, 083104
 * (2012); Sec. IV cites relativistic weighted binary collisions for PICLS).
 * Velocities in, velocities out; c = 299792458 m/s.
 *   1. momenta p = gamma m v, energies E = gamma m c^2, gamma = 1/sqrt(1 - v^2/c^2);
 *   2. centre-of-momentum velocity v_C = (p_a + p_b) c^2 / (E_a + E_b),
 *      gamma_C = 1/sqrt(1 - v_C^2/c^2), and g = (gamma_C - 1)/v_C^2 written as
 *      gamma_C^2 / ((gamma_C + 1) c^2);
 *   3. p_a* = p_a + (g (v_C . p_a) - gamma_C E_a / c^2) v_C, E* = gamma_C (E - v_C . p);
 *   4. the scattering parameter
 *        s = 2 qq n m_ab^2 / (m_a gamma_a m_b gamma_b) * gamma_C |p*| / (m_a gamma_a + m_b gamma_b)
 *            * (m_a gamma_a* m_b gamma_b* c^2 / |p*|^2 + 1)^2 / c^4,
 *      qq = qq_coef of orc_collide (q_a^2 q_b^2 lnL dt / (8 pi eps0^2 m_ab^2)),
 *      n = max(w_a, w_b) nunit; for v << c it tends to 2 <delta^2> of
 *      Takizuka-Abe;
 *   5. the angle of p_a* from <delta^2> = s / 2 by Takizuka-Abe's law (draws
 *      0, 1) or, with nanbu, Nanbu's law with s; the azimuth from draw 2; the
 *      rotation is orc_collide's with u -> p_a*; p_b*' = -p_a*';
 *   6. back to the lab: p' = p*' + (g (v_C . p*') + gamma_C E* / c^2) v_C, and
 *      v' = p' c / sqrt(m^2 c^2 + p'^2);
 *   7. weighted acceptance as in orc_collide (draw 3).
 * |p*| = 0 is no collision (-1).
 */
double orc_collide_rel(double va[3], double vb[3], double ma, double mb, uint32_t wa,
                       uint32_t wb, double qq_coef, double nunit, const uint32_t draws[4],
                       int32_t nanbu, int32_t *acc_a, int32_t *acc_b)
{
    const double c = ORC_CLIGHT, c2 = c * c;
    *acc_a = 0;
    *acc_b = 0;
    double va2 = (va[0] * va[0] + va[1] * va[1]) + va[2] * va[2];
    double vb2 = (vb[0] * vb[0] + vb[1] * vb[1]) + vb[2] * vb[2];
    double ga = 1.0 / sqrt(1.0 - va2 / c2);
    double gb = 1.0 / sqrt(1.0 - vb2 / c2);
    double pa[3], pb[3], vc[3];
    for (int d = 0; d < 3; ++d) {
        pa[d] = (ga * ma) * va[d];
        pb[d] = (gb * mb) * vb[d];
    }
    double ea = (ga * ma) * c2, eb = (gb * mb) * c2;
    double etot = ea + eb;
    for (int d = 0; d < 3; ++d) vc[d] = ((pa[d] + pb[d]) * c2) / etot;
    double vc2 = (vc[0] * vc[0] + vc[1] * vc[1]) + vc[2] * vc[2];
    double gc = 1.0 / sqrt(1.0 - vc2 / c2);
    double g = (gc * gc) / ((gc + 1.0) * c2);
    double vpa = (vc[0] * pa[0] + vc[1] * pa[1]) + vc[2] * pa[2];
    double vpb = (vc[0] * pb[0] + vc[1] * pb[1]) + vc[2] * pb[2];
    double ka = g * vpa - (gc * ea) / c2;
    double ps[3];
    for (int d = 0; d < 3; ++d) ps[d] = pa[d] + ka * vc[d];
    double eas = gc * (ea - vpa), ebs = gc * (eb - vpb);
    double p2 = (ps[0] * ps[0] + ps[1] * ps[1]) + ps[2] * ps[2];
    if (p2 == 0.0) return -1.0;
    double p = sqrt(p2);
    double gas = eas / (ma * c2), gbs = ebs / (mb * c2);
    uint32_t wmax = wa > wb ? wa : wb;
    double mab = (ma * mb) / (ma + mb);
    double x = (((ma * gas) * (mb * gbs)) * c2) / p2 + 1.0;
    double s = ((((2.0 * qq_coef) * ((double)wmax * nunit)) * (mab * mab)) / ((ma * ga) * (mb * gb)))
               * ((gc * p) / (ma * ga + mb * gb)) * ((x * x) / (c2 * c2));
    double d2 = 0.5 * s;
    double st, omc;
    if (nanbu) {
        omc = orc_nanbu_omc(s, orc_u52(draws[0], draws[1]));
        st = sqrt(omc * (2.0 - omc));
    } else {
        double r1 = orc_u32(draws[0]);
        double s2, cc2;
        orc_sincos2pi((uint64_t)draws[1] << 20, &s2, &cc2);
        double gg = sqrt(-2.0 * orc_log(r1)) * cc2;
        double dl = sqrt(d2) * gg;
        double dd = dl * dl;
        double den = 1.0 + dd;
        st = (2.0 * dl) / den;
        omc = (2.0 * dd) / den;
    }
    double sp, cp;
    orc_sincos2pi((uint64_t)draws[2] << 20, &sp, &cp);
    double a = st * cp, bb = st * sp;
    double up = sqrt(ps[0] * ps[0] + ps[1] * ps[1]);
    double dpx, dpy, dpz;
    if (up > 0.0) {
        dpx = ((ps[0] / up) * ps[2]) * a - ((ps[1] / up) * p) * bb - ps[0] * omc;
        dpy = ((ps[1] / up) * ps[2]) * a + ((ps[0] / up) * p) * bb - ps[1] * omc;
        dpz = -(up * a) - ps[2] * omc;
    } else {
        double apz = fabs(ps[2]);
        dpx = apz * a;
        dpy = apz * bb;
        dpz = -(ps[2] * omc);
    }
    double qa[3] = {ps[0] + dpx, ps[1] + dpy, ps[2] + dpz};
    double qb[3] = {-qa[0], -qa[1], -qa[2]};
    double vqa = (vc[0] * qa[0] + vc[1] * qa[1]) + vc[2] * qa[2];
    double vqb = (vc[0] * qb[0] + vc[1] * qb[1]) + vc[2] * qb[2];
    double la = g * vqa + (gc * eas) / c2;
    double lb = g * vqb + (gc * ebs) / c2;
    double na[3], nb[3];
    for (int d = 0; d < 3; ++d) {
        na[d] = qa[d] + la * vc[d];
        nb[d] = qb[d] + lb * vc[d];
    }
    double na2 = (na[0] * na[0] + na[1] * na[1]) + na[2] * na[2];
    double nb2 = (nb[0] * nb[0] + nb[1] * nb[1]) + nb[2] * nb[2];
    double ra = c / sqrt((ma * ma) * c2 + na2);
    double rb = c / sqrt((mb * mb) * c2 + nb2);
    double r4 = orc_u32(draws[3]);
    int ta = (wa <= wb) || (r4 < (double)wb / (double)wa);
    int tb = (wb <= wa) || (r4 < (double)wa / (double)wb);
    if (ta)
        for (int d = 0; d < 3; ++d) va[d] = na[d] * ra;
    if (tb)
        for (int d = 0; d < 3; ++d) vb[d] = nb[d] * rb;
    *acc_a = ta;
    *acc_b = tb;
    return d2;
}

double orc_ta77(double va[3], double vb[3], double ma, double mb, uint32_t wa,
                uint32_t wb, double qq_coef, double nunit, const uint32_t draws[4],
                int32_t *acc_a, int32_t *acc_b)
{
    return orc_collide(va, vb, ma, mb, wa, wb, qq_coef, nunit, draws, 0, acc_a, acc_b);
}
