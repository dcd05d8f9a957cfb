// Device physics of one cell: configurations, continuum lowering, Coulomb
// logarithm, equation of state, photo cross sections and the binary collision.
// Operand order of every expression follows the method's arithmetic contract.
#pragma once

#include "../../include/xpic.h"
#include "xp_device.h"
#include "xp_tables.h"

namespace xpd {

constexpr double E2 = QE / ((4.0 * PI) * EPS0);          // e^2/(4 pi eps0), eV m
constexpr double THREE_OVER_4PI = 3.0 / (4.0 * PI);
constexpr double HALF_ME_OVER_QE = (0.5 * ME) / QE;
constexpr double TWO_QE_OVER_ME = (2.0 * QE) / ME;

// Standard normal velocity components of one electron for the forced
// thermalization (Sec. VI.C), from its RP_THERM draw: Box-Muller on words
// 0, 1 (radius, angle) gives x and y, on words 2, 3 gives z.
__device__ __forceinline__ void therm_normals(const Words& d, double& gx, double& gy, double& gz)
{
    double s1, c1, s2, c2;
    xsincos2pi((uint64_t)d.x1 << 20, s1, c1);
    xsincos2pi((uint64_t)d.x3 << 20, s2, c2);
    const double r1 = sqrt(-2.0 * xlog(u32(d.x0)));
    const double r2 = sqrt(-2.0 * xlog(u32(d.x2)));
    gx = r1 * c1;
    gy = r1 * s1;
    gz = r2 * c2;
}

// Lowest-energy configuration of charge state z with k K vacancies (Sec. III):
// counts of 1s 2s 2p 3s 3p.
struct Occ { int s[5]; };

__device__ __forceinline__ Occ occupancy(int z, int k)
{
    Occ o;
    const int nb = 13 - z;
    int k1 = 2 - k;
    k1 = k1 > nb ? nb : k1;
    k1 = k1 < 0 ? 0 : k1;
    o.s[0] = k1;
    int rem = nb - k1;
    const int cap[5] = {2, 2, 6, 2, 6};
#pragma unroll
    for (int q = 1; q < 5; ++q) {
        const int c = rem < cap[q] ? rem : cap[q];
        o.s[q] = c;
        rem -= c;
    }
    return o;
}

__device__ __forceinline__ int valence(int z, int k)
{
    const Occ o = occupancy(z, k);
    for (int q = 4; q >= 0; --q)
        if (o.s[q] > 0) return q;
    return -1;
}

// Continuum lowering of charge state z: Ecker-Kroll (Eq. 5; Debye-Hueckel
// below n_crit) or Stewart-Pyatt (Eq. 6 with lambda_D including Zbar + 1).
__device__ __noinline__ double ipd(int model, int z, double t, double n_e, double n_i, double zbar,
                      double zstar)
{
    double lamd = __builtin_inf();
    if (n_e > 0.0) lamd = sqrt((EPS0 * t) / (QE * (n_e * (zbar + 1.0))));
    const double zp1 = (double)(z + 1);
    if (model == 1) {
        const double ntot = n_e + n_i;
        const double c = t / ((zp1 * zp1) * E2);
        const double ncrit = THREE_OVER_4PI * ((c * c) * c);
        if (ntot > ncrit) return (zp1 * E2) / xcbrt(THREE_OVER_4PI / ntot);
        return (zp1 * E2) / lamd;
    }
    const double kk = (zp1 * E2) / (lamd * t);
    const double zs1 = zstar + 1.0;
    const double c = xcbrt(((3.0 * zs1) * kk) + 1.0);
    return (t / (2.0 * zs1)) * ((c * c) - 1.0);
}

__device__ __noinline__ double coulomb_log(double t, double n_e, double zbar)
{
    if (!(n_e > 0.0)) return 2.0;
    const double lamde = sqrt((EPS0 * t) / (QE * n_e));
    const double bcl = (zbar * E2) / (3.0 * t);
    const double bq = HBAR / (2.0 * sqrt((3.0 * ME) * (t * QE)));
    const double bmin = bcl > bq ? bcl : bq;
    const double ratio = lamde / bmin;
    const double lnl = 0.5 * xlog(1.0 + ratio * ratio);
    return lnl < 2.0 ? 2.0 : lnl;
}

// Zbar_EOS(n_i, T_e), bilinear in (ln n_i, ln T) on the table grid, from the
// two logarithms.
__device__ __noinline__ double eos_zbar_ln(const DevTables* tb, double ln_ni, double ln_t)
{
    const double* zt = (const double*)((const char*)tb + tb->off_eos);
    const double u = (ln_ni - tb->eos_lnn0) / tb->eos_dlnn;
    const double v = (ln_t - tb->eos_lnt0) / tb->eos_dlnt;
    const int nn = tb->eos_nn, nt = tb->eos_nt;
    const double fu = floor(u), fv = floor(v);
    double au = u - fu, av = v - fv;
    int iu, iv;
    if (u < 0.0) { iu = 0; au = 0.0; } else if (fu > (double)(nn - 2)) { iu = nn - 2; au = 1.0; } else { iu = (int)fu; }
    if (v < 0.0) { iv = 0; av = 0.0; } else if (fv > (double)(nt - 2)) { iv = nt - 2; av = 1.0; } else { iv = (int)fv; }
    const double z00 = zt[iu * nt + iv], z01 = zt[iu * nt + iv + 1];
    const double z10 = zt[(iu + 1) * nt + iv], z11 = zt[(iu + 1) * nt + iv + 1];
    const double a = (1.0 - av) * z00 + av * z01;
    const double b = (1.0 - av) * z10 + av * z11;
    return (1.0 - au) * a + au * b;
}

__device__ __forceinline__ double eos_zbar(const DevTables* tb, double n_i, double tev)
{
    return eos_zbar_ln(tb, xlog(n_i), xlog(tev));
}

// Per-electron subshell photoionization cross section, m^2 (Fig. 2a table).
__device__ __noinline__ double photo_sigma(const DevTables* tb, int s, double hv)
{
    const double* ls = (const double*)((const char*)tb + tb->off_lnsig) + s * tb->photo_nh;
    const double u = (xlog(hv) - tb->photo_lnhv0) / tb->photo_dlnhv;
    const double fu = floor(u);
    double a = u - fu;
    int iu;
    if (u < 0.0) { iu = 0; a = 0.0; } else if (fu > (double)(tb->photo_nh - 2)) { iu = tb->photo_nh - 2; a = 1.0; } else { iu = (int)fu; }
    const double l0 = ls[iu], l1 = ls[iu + 1];
    return xexp(l0 + a * (l1 - l0)) * 1.0e-4;
}

// Lowered binding of subshell s of charge state z, clamped at 1 eV.
__device__ __forceinline__ double lowered(const DevTables* tb, int z, int s, const double* dE)
{
    const double p = tb->bind[z][s] - dE[z];
    return p < 1.0 ? 1.0 : p;
}

// exp(x) E1(x) for x > 0: the series -gamma - ln x - sum (-x)^k / (k k!) to
// k = 24 for x <= 1, the contracted continued fraction
// E1 = exp(-x) / (x + 1 - 1/(x + 3 - 4/(x + 5 - ...))) from depth 80 above.
__device__ __noinline__ double e1x(double x)
{
    if (x <= 1.0) {
        double sum = 0.0, term = 1.0;
        for (int k = 1; k <= 24; ++k) {
            term = (term * (-x)) / (double)k;
            sum = sum + term / (double)k;
        }
        const double e1 = (-0.57721566490153286 - xlog(x)) - sum;
        return xexp(x) * e1;
    }
    double t = x + 161.0;
    for (int k = 80; k >= 1; --k) t = (x + (double)(2 * k - 1)) - (double)(k * k) / t;
    return 1.0 / t;
}

// Degeneracy of the ground configuration of charge state z: the product over
// subshells of C(capacity, occupancy).
__device__ __forceinline__ double ground_degeneracy(int z)
{
    const Occ o = occupancy(z, 0);
    const int cap[5] = {2, 2, 6, 2, 6};
    double g = 1.0;
    for (int s = 0; s < 5; ++s) {
        double c = 1.0;
        for (int j = 0; j < o.s[s]; ++j) c = (c * (double)(cap[s] - j)) / (double)(j + 1);
        g = g * c;
    }
    return g;
}

// Three-body recombination z -> z-1 per step dt (XP_REC_XS): detailed balance
// with the Lotz ionization of z-1 (Eq. 4), S_{z-1}(T) n_e^2 dt / Phi_z(T),
// S the Maxwellian rate of the occupied subshells of the ground configuration
// of z-1 with their lowered bindings, Phi_z = 2 (g_z / g_{z-1})
// (m_e k T / (2 pi hbar^2))^{3/2} exp(-P_v / T) with the lowered binding P_v
// of its valence subshell.  S e^{P_v/T} is formed from exp(x) E1(x) and
// exp(x_v - x_s) <= 1, so nothing overflows.  Not clamped.
__device__ __noinline__ double rec_xs_prob(const DevTables* tb, int z, double tev, double n_e,
                                           const double* dE, double dt)
{
    if (z < 1 || z > 13 || !(n_e > 0.0) || !(tev > 0.0)) return 0.0;
    const int zl = z - 1;
    const Occ o = occupancy(zl, 0);
    const int v = valence(zl, 0);
    double pv = tb->bind[zl][v] - dE[zl];
    if (pv < 1.0) pv = 1.0;
    const double xv = pv / tev;
    const double vbar = sqrt((8.0 * (tev * QE)) / (PI * ME));
    double sum = 0.0;
    for (int s = 0; s < 5; ++s) {
        if (o.s[s] <= 0) continue;
        double p = tb->bind[zl][s] - dE[zl];
        if (p < 1.0) p = 1.0;
        const double x = p / tev;
        double br = e1x(x);
        if (tb->lotz_b[s] != 0.0) {
            const double c = tb->lotz_c[s];
            br = br - (tb->lotz_b[s] * (x / (x + c))) * e1x(x + c);
        }
        const double term = ((((tb->lotz_a[s] * 1.0e-4) * (double)o.s[s]) * vbar) / (p * tev)) * (br * xexp(xv - x));
        sum = sum + term;
    }
    const double q = (ME * (tev * QE)) / ((2.0 * PI) * (HBAR * HBAR));
    const double phi0 = (2.0 * (ground_degeneracy(z) / ground_degeneracy(zl))) * (q * sqrt(q));
    return ((sum * (n_e * n_e)) * dt) / phi0;
}

struct Coll {
    double d2;        // <delta^2>, or -1 when the relative velocity is zero
    int acc_a, acc_b;
};

// Nanbu's cumulative small-angle scattering (Phys. Rev. E 55, 4642 (1997)):
// the deflections of one step add up to one angle chi whose cosine has the
// density A exp(A cos chi) / (2 sinh A), A fixed by <cos chi> = coth A - 1/A
// = exp(-s).  nanbu_a(s):
//   s <= 0.05: A >= 20 and coth A = 1 to working precision, so
//     A = 1 / (1 - exp(-s)), the denominator from its nested series to s/11;
//   0.05 < s < 15: four Newton steps on L(A) = exp(-s) from the Pade start
//     A = m (3 - m^2) / (1 - m^2); L, L' by the Laurent series of coth
//     (eleven Bernoulli terms) below A = 0.5, by E = exp(-2A) above;
//   s >= 15: 0, the isotropic limit.
__device__ __forceinline__ void langevin(double a, double& l, double& dl)
{
    if (a < 0.5) {
        constexpr double c1 = 1.0 / 3.0, c2 = -1.0 / 45.0, c3 = 2.0 / 945.0, c4 = -1.0 / 4725.0,
                         c5 = 2.0 / 93555.0, c6 = -1382.0 / 638512875.0, c7 = 4.0 / 18243225.0,
                         c8 = -3617.0 / 162820783125.0, c9 = 87734.0 / 38979295480125.0,
                         c10 = -349222.0 / 1531329465290625.0, c11 = 310732.0 / 13447856940643125.0;
        const double z = a * a;
        double v = c11;
        v = c10 + z * v; v = c9 + z * v; v = c8 + z * v; v = c7 + z * v; v = c6 + z * v;
        v = c5 + z * v; v = c4 + z * v; v = c3 + z * v; v = c2 + z * v; v = c1 + z * v;
        // derivative coefficients (2k - 1) c_k, each a rounded product
        double dv = 21.0 * c11;
        dv = 19.0 * c10 + z * dv; dv = 17.0 * c9 + z * dv; dv = 15.0 * c8 + z * dv;
        dv = 13.0 * c7 + z * dv;  dv = 11.0 * c6 + z * dv; dv = 9.0 * c5 + z * dv;
        dv = 7.0 * c4 + z * dv;   dv = 5.0 * c3 + z * dv;  dv = 3.0 * c2 + z * dv;
        dv = 1.0 * c1 + z * dv;
        l = a * v;
        dl = dv;
        return;
    }
    const double e = xexp(-2.0 * a);
    const double ome = 1.0 - e;
    l = (1.0 + e) / ome - 1.0 / a;
    dl = 1.0 / (a * a) - (4.0 * e) / (ome * ome);
}

__device__ __noinline__ double nanbu_a(double s)
{
    if (s >= 15.0) return 0.0;
    if (s <= 0.05) {
        double q = 1.0;
        q = 1.0 - (s * (1.0 / 11.0)) * q; q = 1.0 - (s * (1.0 / 10.0)) * q;
        q = 1.0 - (s * (1.0 / 9.0)) * q;  q = 1.0 - (s * (1.0 / 8.0)) * q;
        q = 1.0 - (s * (1.0 / 7.0)) * q;  q = 1.0 - (s * (1.0 / 6.0)) * q;
        q = 1.0 - (s * (1.0 / 5.0)) * q;  q = 1.0 - (s * (1.0 / 4.0)) * q;
        q = 1.0 - (s * (1.0 / 3.0)) * q;  q = 1.0 - (s * (1.0 / 2.0)) * q;
        return 1.0 / (s * q);
    }
    const double m = xexp(-s);
    const double m2 = m * m;
    double a = (m * (3.0 - m2)) / (1.0 - m2);
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
        double l, dl;
        langevin(a, l, dl);
        a = a - (l - m) / dl;
    }
    return a;
}

// 1 - cos chi for s and a uniform u in (0, 1), by inverting the distribution
// function: cos chi = 1 + ln(u + (1 - u) exp(-2A)) / A (A = 0: 2u - 1).
// Clamped to [0, 2]; s <= 0 gives no deflection.
__device__ __forceinline__ double nanbu_omc(double s, double u)
{
    if (!(s > 0.0)) return 0.0;
    const double a = nanbu_a(s);
    double omc;
    if (a == 0.0) {
        omc = 2.0 * (1.0 - u);
    } else {
        const double e2 = xexp(-2.0 * a);
        omc = -xlog(u + (1.0 - u) * e2) / a;
    }
    if (omc < 0.0) omc = 0.0;
    if (omc > 2.0) omc = 2.0;
    return omc;
}

// Binary collision with weighted acceptance (the heavier-weight partner
// accepts with probability w_light / w_heavy).  Scattering law: Takizuka-Abe,
// tan(theta/2) = delta normal with variance <delta^2> (r1 from word 0, the
// Box-Muller angle from word 1), or with nanbu Nanbu's cumulative law with
// s = 2 <delta^2> and u = U52(words 0, 1).  Phi comes from word 2, the
// acceptance draw r4 from word 3.  fa = m_b/(m_a+m_b), fb = m_a/(m_a+m_b).
__device__ __forceinline__ Coll ta77(double& ax, double& ay, double& az, double& bx, double& by,
                                     double& bz, double fa, double fb, uint32_t wa, uint32_t wb,
                                     double coef, double nunit, const Words& d, bool nanbu)
{
    Coll out{-1.0, 0, 0};
    const double ux = ax - bx, uy = ay - by, uz = az - bz;
    const double u2 = (ux * ux + uy * uy) + uz * uz;
    if (u2 == 0.0) return out;
    const uint32_t wmax = wa > wb ? wa : wb;
    const double u = sqrt(u2);
    const double d2 = ((coef * (double)wmax) * nunit) / (u2 * u);
    double st, omc;
    if (nanbu) {
        omc = nanbu_omc(2.0 * d2, u52(d.x0, d.x1));
        st = sqrt(omc * (2.0 - omc));
    } else {
        double s2, c2;
        xsincos2pi((uint64_t)d.x1 << 20, s2, c2);
        const double g = sqrt(-2.0 * xlog(u32(d.x0))) * c2;
        const double dl = sqrt(d2) * g;
        const double dd = dl * dl;
        const double den = 1.0 + dd;
        st = (2.0 * dl) / den;
        omc = (2.0 * dd) / den;
    }
    double sp, cp;
    xsincos2pi((uint64_t)d.x2 << 20, sp, cp);
    const double a = st * cp;
    const double bb = st * sp;
    const double up = sqrt(ux * ux + uy * uy);
    double dux, duy, duz;
    if (up > 0.0) {
        dux = ((ux / up) * uz) * a - ((uy / up) * u) * bb - ux * omc;
        duy = ((uy / up) * uz) * a + ((ux / up) * u) * bb - uy * omc;
        duz = -(up * a) - uz * omc;
    } else {
        const double auz = fabs(uz);
        dux = auz * a;
        duy = auz * bb;
        duz = -(uz * omc);
    }
    bool ta = true, tb = true;
    if (wa != wb) {
        // only the heavier side draws, against w_light / w_heavy
        const double r4 = u32(d.x3);
        const bool lighter_a = wa < wb;
        const double ratio = lighter_a ? (double)wa / (double)wb : (double)wb / (double)wa;
        const bool keep = r4 < ratio;
        ta = lighter_a || keep;
        tb = !lighter_a || keep;
    }
    if (ta) {
        ax = ax + fa * dux;
        ay = ay + fa * duy;
        az = az + fa * duz;
    }
    if (tb) {
        bx = bx - fb * dux;
        by = by - fb * duy;
        bz = bz - fb * duz;
    }
    out.d2 = d2;
    out.acc_a = ta;
    out.acc_b = tb;
    return out;
}

// Relativistic binary collision in the pair's centre-of-momentum frame (the
// Monte-Carlo collision of Perez et al., Phys. Plasmas 19, 083104 (2012)):
// momenta p = gamma m v boosted to the frame moving with v_C = (p_a + p_b)
// c^2 / (E_a + E_b); there p_a* is turned by the angle drawn from the
// scattering parameter
//   s = 2 qq n m_ab^2 / (m_a g_a m_b g_b) * g_C |p*| / (m_a g_a + m_b g_b)
//       * (m_a g_a* m_b g_b* c^2 / |p*|^2 + 1)^2 / c^4
// (qq = coef, n = max(w) nunit; s -> 2 <delta^2> of Takizuka-Abe for v << c),
// by Takizuka-Abe's law with <delta^2> = s / 2 or with nanbu by Nanbu's law;
// p_b*' = -p_a*', both boosted back, v = p c / sqrt(m^2 c^2 + p^2).  Draws,
// rotation and weighted acceptance as in ta77.  (gamma_C - 1) / v_C^2 is
// written gamma_C^2 / ((gamma_C + 1) c^2).
__device__ __noinline__ Coll ta77_rel(double& ax, double& ay, double& az, double& bx, double& by,
                                      double& bz, double ma, double mb, uint32_t wa, uint32_t wb,
                                      double coef, double nunit, const Words& d, bool nanbu)
{
    Coll out{-1.0, 0, 0};
    const double c = CLIGHT, c2 = c * c;
    const double va2 = (ax * ax + ay * ay) + az * az;
    const double vb2 = (bx * bx + by * by) + bz * bz;
    const double ga = 1.0 / sqrt(1.0 - va2 / c2);
    const double gb = 1.0 / sqrt(1.0 - vb2 / c2);
    const double pax = (ga * ma) * ax, pay = (ga * ma) * ay, paz = (ga * ma) * az;
    const double pbx = (gb * mb) * bx, pby = (gb * mb) * by, pbz = (gb * mb) * bz;
    const double ea = (ga * ma) * c2, eb = (gb * mb) * c2;
    const double etot = ea + eb;
    const double vcx = ((pax + pbx) * c2) / etot;
    const double vcy = ((pay + pby) * c2) / etot;
    const double vcz = ((paz + pbz) * c2) / etot;
    const double vc2 = (vcx * vcx + vcy * vcy) + vcz * vcz;
    const double gc = 1.0 / sqrt(1.0 - vc2 / c2);
    const double g = (gc * gc) / ((gc + 1.0) * c2);
    const double vpa = (vcx * pax + vcy * pay) + vcz * paz;
    const double vpb = (vcx * pbx + vcy * pby) + vcz * pbz;
    const double ka = g * vpa - (gc * ea) / c2;
    const double psx = pax + ka * vcx, psy = pay + ka * vcy, psz = paz + ka * vcz;
    const double eas = gc * (ea - vpa), ebs = gc * (eb - vpb);
    const double p2 = (psx * psx + psy * psy) + psz * psz;
    if (p2 == 0.0) return out;
    const double p = sqrt(p2);
    const double gas = eas / (ma * c2), gbs = ebs / (mb * c2);
    const uint32_t wmax = wa > wb ? wa : wb;
    const double mab = (ma * mb) / (ma + mb);
    const double x = (((ma * gas) * (mb * gbs)) * c2) / p2 + 1.0;
    const double s = ((((2.0 * coef) * ((double)wmax * nunit)) * (mab * mab)) / ((ma * ga) * (mb * gb))) *
                     ((gc * p) / (ma * ga + mb * gb)) * ((x * x) / (c2 * c2));
    const double d2 = 0.5 * s;
    double st, omc;
    if (nanbu) {
        omc = nanbu_omc(s, u52(d.x0, d.x1));
        st = sqrt(omc * (2.0 - omc));
    } else {
        double s2, cc2;
        xsincos2pi((uint64_t)d.x1 << 20, s2, cc2);
        const double gg = sqrt(-2.0 * xlog(u32(d.x0))) * cc2;
        const double dl = sqrt(d2) * gg;
        const double dd = dl * dl;
        const double den = 1.0 + dd;
        st = (2.0 * dl) / den;
        omc = (2.0 * dd) / den;
    }
    double sp, cp;
    xsincos2pi((uint64_t)d.x2 << 20, sp, cp);
    const double a = st * cp;
    const double bb = st * sp;
    const double up = sqrt(psx * psx + psy * psy);
    double dpx, dpy, dpz;
    if (up > 0.0) {
        dpx = ((psx / up) * psz) * a - ((psy / up) * p) * bb - psx * omc;
        dpy = ((psy / up) * psz) * a + ((psx / up) * p) * bb - psy * omc;
        dpz = -(up * a) - psz * omc;
    } else {
        const double apz = fabs(psz);
        dpx = apz * a;
        dpy = apz * bb;
        dpz = -(psz * omc);
    }
    const double qax = psx + dpx, qay = psy + dpy, qaz = psz + dpz;
    const double qbx = -qax, qby = -qay, qbz = -qaz;
    const double vqa = (vcx * qax + vcy * qay) + vcz * qaz;
    const double vqb = (vcx * qbx + vcy * qby) + vcz * qbz;
    const double la = g * vqa + (gc * eas) / c2;
    const double lb = g * vqb + (gc * ebs) / c2;
    const double nax = qax + la * vcx, nay = qay + la * vcy, naz = qaz + la * vcz;
    const double nbx = qbx + lb * vcx, nby = qby + lb * vcy, nbz = qbz + lb * vcz;
    const double na2 = (nax * nax + nay * nay) + naz * naz;
    const double nb2 = (nbx * nbx + nby * nby) + nbz * nbz;
    const double ra = c / sqrt((ma * ma) * c2 + na2);
    const double rb = c / sqrt((mb * mb) * c2 + nb2);
    bool ta = true, tb = true;
    if (wa != wb) {
        // only the heavier side draws, against w_light / w_heavy
        const double r4 = u32(d.x3);
        const bool lighter_a = wa < wb;
        const double ratio = lighter_a ? (double)wa / (double)wb : (double)wb / (double)wa;
        const bool keep = r4 < ratio;
        ta = lighter_a || keep;
        tb = !lighter_a || keep;
    }
    if (ta) {
        ax = nax * ra;
        ay = nay * ra;
        az = naz * ra;
    }
    if (tb) {
        bx = nbx * rb;
        by = nby * rb;
        bz = nbz * rb;
    }
    out.d2 = d2;
    out.acc_a = ta;
    out.acc_b = tb;
    return out;
}

// One binary collision between slot e of (avx, avy, avz, aw) and slot b of
// (bvx, bvy, bvz) with weight wb, on LDS arrays; draws from Philox counter
// (c0, c1, idx, c3).  Counts go to cnt (XP_C_* indices).  law: bit 0
// Nanbu's scattering law instead of Takizuka-Abe's, bit 1 relativistic
// kinematics (ta77_rel, with the masses ma and mb).
__device__ __forceinline__ void collide_slots(double* avx, double* avy, double* avz, const uint32_t* aw,
                                           double* bvx, double* bvy, double* bvz, int e, int b,
                                           uint32_t wb, double fa, double fb, double coef,
                                           double nunit, uint32_t c0, uint32_t c1, uint32_t idx,
                                           uint32_t c3, uint32_t k0, uint32_t k1, int* cnt,
                                           int law, double ma = 0.0, double mb = 0.0)
{
    double ax = avx[e], ay = avy[e], az = avz[e];
    double bx = bvx[b], by = bvy[b], bz = bvz[b];
    const Words d = philox(c0, c1, idx, c3, k0, k1);
    const Coll c = (law & 2) ? ta77_rel(ax, ay, az, bx, by, bz, ma, mb, aw[e], wb, coef, nunit, d, (law & 1) != 0)
                             : ta77(ax, ay, az, bx, by, bz, fa, fb, aw[e], wb, coef, nunit, d, (law & 1) != 0);
    if (c.d2 < 0.0) {
        atomicAdd(&cnt[XP_C_U0], 1);
        return;
    }
    if (c.d2 > 1.0) atomicAdd(&cnt[XP_C_DELTA2_GT1], 1);
    atomicAdd(&cnt[XP_C_ACCEPT], c.acc_a + c.acc_b);
    avx[e] = ax; avy[e] = ay; avz[e] = az;
    bvx[b] = bx; bvy[b] = by; bvz[b] = bz;
}

// w sigma v of one electron for the average cell ion (Lotz, Eq. 4): occupied
// subshells oc, lowered bindings pp and their logarithms lnp; pmin is the
// smallest pp of an occupied subshell.  An electron at or below pmin meets no
// subshell term, so its cross section stays 0.0 without the logarithm.
__device__ __forceinline__ double lotz_leaf(double x, double y, double z, uint32_t w, const int* oc,
                                         const double* pp, const double* lnp, double pmin,
                                         const DevTables* tb)
{
    const double v2 = (x * x + y * y) + z * z;
    const double e = HALF_ME_OVER_QE * v2;
    double sig = 0.0;
    if (e > 0.0 && e > pmin) {
        const double lne = xlog(e);
        for (int q = 0; q < 5; ++q) {
            if (oc[q] <= 0 || !(e > pp[q])) continue;
            double term = (((tb->lotz_a[q] * 1.0e-4) * (double)oc[q]) * (lne - lnp[q])) / (e * pp[q]);
            if (tb->lotz_b[q] != 0.0)
                term = term * (1.0 - tb->lotz_b[q] * xexp(-(tb->lotz_c[q] * (e / pp[q] - 1.0))));
            sig = sig + term;
        }
    }
    return ((double)w * sig) * sqrt(v2);
}

// ------------------------------------------- S5 photon field (Sec. III)

// Bin of a photoionization of subshell s: the first bin, in bin order, at
// which the running sum of n_hv sigma over the bins the lowered binding pp
// allows passes target; the last bin with a positive term when rounding
// leaves the sum short of it.
__device__ __forceinline__ int photo_bin(const double* hv, const double* nhv, const double (*sig)[3],
                                         int nb, int s, double pp, double target)
{
    double cum = 0.0;
    int sel = -1, lastpos = -1;
    for (int bq = 0; bq < nb; ++bq) {
        if (!(hv[bq] >= pp)) continue;
        const double term = nhv[bq] * sig[bq][s];
        cum = cum + term;
        if (term > 0.0) lastpos = bq;
        if (cum > target) {
            sel = bq;
            break;
        }
    }
    return sel < 0 ? lastpos : sel;
}

// XP_KA_FIELD: the bin of the largest h nu not above e, the lowest index
// among equal ones; -1 if every bin lies above e.
__device__ __forceinline__ int kalpha_bin(const double* hv, int nb, double e)
{
    int kb = -1;
    for (int b = 0; b < nb; ++b)
        if (hv[b] <= e && (kb < 0 || hv[b] > hv[kb])) kb = b;
    return kb;
}

// XP_KA_FIELD: K-alpha macro-photons a cell returns to bin b, from its
// K-alpha photons per charge state kz[Z0], summed over Z0 ascending.
__device__ __forceinline__ double kalpha_return(const DevTables* tb, const double* hv, int nb, const int32_t* kz,
                                                int b)
{
    double g = 0.0;
    for (int z0 = 0; z0 < 13; ++z0) {
        if (kz[z0] == 0) continue;
        const double e = tb->e_kalpha[z0];
        if (kalpha_bin(hv, nb, e) != b) continue;
        g = g + (double)kz[z0] * (e / hv[b]);
    }
    return g;
}

// XP_PHOTO_FRAC, for a cell whose photo candidates may outnumber what a bin
// holds: one ion's photo shells again, in order, from its state after decay
// (z, kv in and out).  pf: the shells whose draw passed their probability
// (candidates); each candidate that still has an electron takes one
// macro-photon of its bin while one is left (bud[b] held, used[b] taken);
// the one that finds a fraction f left happens with probability f (word 0 of
// its call of purpose RP_PART), after which the bin is spent; later ones
// starve.  draw(purpose, sub) gives the ion's Philox words.
struct PhotoWalk {
    uint32_t mask, bins;   // photo bits 1..3 and bins at 4 s, as the first pass records them
    int fired[3], skipped, starved, partial;
};

template <class D>
__device__ __forceinline__ PhotoWalk photo_walk_ion(D draw, const DevTables* tb, const double* hv, const double* nhv,
                                                 const double (*sig)[3], const double (*ssum)[3], int nb, int z0,
                                                 uint32_t pf, const double* dE, double* bud, double* used, int& z,
                                                 int& kv)
{
    PhotoWalk w = {0u, 0u, {0, 0, 0}, 0, 0, 0};
    for (int s = 0; s < 3; ++s) {
        if (!((pf >> s) & 1u)) continue;
        const Occ on = occupancy(z, kv);
        if (z >= 13 || on.s[s] <= 0) {
            ++w.skipped;
            continue;
        }
        const double pp = lowered(tb, z0, s, dE);
        const Words d = draw(RP_BIN, (uint32_t)s);
        const int sel = photo_bin(hv, nhv, sig, nb, s, pp, u52(d.x0, d.x1) * ssum[z0][s]);
        const double rem = bud[sel] - used[sel];
        if (rem >= 1.0) {
            used[sel] = used[sel] + 1.0;
        } else if (rem > 0.0) {
            used[sel] = bud[sel];
            const Words e = draw(RP_PART, (uint32_t)s);
            if (!(u32(e.x0) < rem)) {
                ++w.starved;
                continue;
            }
            ++w.partial;
        } else {
            ++w.starved;
            continue;
        }
        z = z + 1;
        if (s == 0) kv = kv + 1;
        w.mask |= 2u << s;
        w.bins |= (uint32_t)sel << (4 * s);
        ++w.fired[s];
    }
    return w;
}

}  // namespace xpd

