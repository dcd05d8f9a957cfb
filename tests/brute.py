"""A third, deliberately naive implementation of one step for tiny cells.

Pure Python: Python integers for Philox4x32-10, sorted() for the random
permutations, the math module (libm) for log / sin / cos / cbrt / exp.  It is
written from the method's description, not from the oracle's source, and is
used to check the oracle's pairings, events and velocities on cells of a few
particles.  Because libm and the oracle's own elementary functions can differ
in the last bit, velocities are compared with a relative tolerance.
"""

import math

QE = 1.602176634e-19
ME = 9.1093837015e-31
CLIGHT = 299792458.0
EPS0 = 8.8541878128e-12
HBAR = 1.054571817e-34
CL = 299792458.0
E2 = QE / (4 * math.pi * EPS0)
M32 = 0xFFFFFFFF


def philox(c, k):
    c = list(c)
    k0, k1 = k
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c[3] ^ k1) & M32, p0 & M32]
    return c


def u52(hi, lo):
    return (((hi << 32) | lo) >> 12) / 2.0 ** 52 + 2.0 ** -53


def u32(x):
    return (x + 0.5) / 2.0 ** 32


def nanbu_omc(s, u):
    """1 - cos(chi) of Nanbu's cumulative scattering law (Phys. Rev. E 55, 4642):
    cos(chi) has density A exp(A cos chi) / (2 sinh A) with coth A - 1/A =
    exp(-s); sampled by inverting its distribution function at u.  A is found
    by bracketing (scipy's brentq) on 1 - L(A) = -expm1(-s); s >= 15 is taken
    as isotropic."""
    from scipy.optimize import brentq
    if s <= 0.0:
        return 0.0
    if s >= 15.0:
        cos = 2.0 * u - 1.0
    else:
        target = -math.expm1(-s)

        def one_minus_l(a):
            if a < 0.01:
                return 1.0 - (a / 3.0 - a ** 3 / 45.0 + 2.0 * a ** 5 / 945.0)
            tail = 0.0 if a > 350.0 else 2.0 / math.expm1(2.0 * a)
            return 1.0 / a - tail

        a = brentq(lambda a: one_minus_l(a) - target, 1e-10, 1e12, xtol=1e-300, rtol=1e-15,
                   maxiter=500)
        cos = 1.0 + math.log(u + (1.0 - u) * math.exp(-2.0 * a)) / a
    return min(2.0, max(0.0, 1.0 - cos))


def occ(z, k):
    nb = 13 - z
    o = [max(0, min(2 - k, nb))]
    rem = nb - o[0]
    for cap in (2, 6, 2, 6):
        o.append(min(cap, rem))
        rem -= o[-1]
    return o


class Cell:
    def __init__(self, e, i):
        self.e = [list(p) for p in e]   # [x, y, vx, vy, vz, w]
        self.i = [list(p) for p in i]   # [x, y, vx, vy, vz, Z, k]


class Brute:
    def __init__(self, tables, spec):
        self.t = tables
        self.s = spec
        self.key = (spec.seed & M32, (spec.seed >> 32) & M32)
        self.law = 0   # scattering law: 0 Takizuka-Abe, 1 Nanbu
        self.rel = False   # relativistic kinematics
        self.sig = [[self._sigma(q, h) for q in range(3)] for h in spec.photon_hv]

    def _sigma(self, q, hv):
        t = self.t
        u = (math.log(hv) - t.photo_lnhv0) / t.photo_dlnhv
        iu = int(math.floor(u))
        a = u - iu
        nh = t.photo_lnsig.shape[1]
        if u < 0:
            iu, a = 0, 0.0
        if iu > nh - 2:
            iu, a = nh - 2, 1.0
        l0, l1 = t.photo_lnsig[q, iu], t.photo_lnsig[q, iu + 1]
        return math.exp(l0 + a * (l1 - l0)) * 1e-4

    def rng(self, step, cell, idx, purpose, sub):
        return philox((step, cell, idx, (purpose << 24) | sub), self.key)

    def perm(self, step, cell, purpose, n):
        keys = []
        for i in range(n):
            w = self.rng(step, cell, i // 4, purpose, 0)
            keys.append((w[i % 4], i))
        return [i for _, i in sorted(keys)]

    def ipd(self, z, t, ne, ni, zbar, zstar):
        lam = math.sqrt(EPS0 * t / (QE * ne * (zbar + 1))) if ne > 0 else math.inf
        if self.s.ipd_model == 1:
            ncrit = 3 / (4 * math.pi) * (t / ((z + 1) ** 2 * E2)) ** 3
            if ne + ni > ncrit:
                return (z + 1) * E2 / (3 / (4 * math.pi * (ne + ni))) ** (1 / 3)
            return (z + 1) * E2 / lam
        k = (z + 1) * E2 / (lam * t)
        return t / (2 * (zstar + 1)) * ((3 * (zstar + 1) * k + 1) ** (2 / 3) - 1)

    def eos(self, ni, t):
        T = self.t
        u = (math.log(ni) - T.eos_lnn0) / T.eos_dlnn
        v = (math.log(t) - T.eos_lnt0) / T.eos_dlnt
        nn, nt = T.eos_zbar.shape
        iu, iv = int(math.floor(u)), int(math.floor(v))
        au, av = u - iu, v - iv
        if u < 0:
            iu, au = 0, 0.0
        if v < 0:
            iv, av = 0, 0.0
        if iu > nn - 2:
            iu, au = nn - 2, 1.0
        if iv > nt - 2:
            iv, av = nt - 2, 1.0
        z = T.eos_zbar
        a = (1 - av) * z[iu, iv] + av * z[iu, iv + 1]
        b = (1 - av) * z[iu + 1, iv] + av * z[iu + 1, iv + 1]
        return (1 - au) * a + au * b

    @staticmethod
    def ke(v):
        return 0.5 * ME * (v[2] ** 2 + v[3] ** 2 + v[4] ** 2) / QE

    def collide_rel(self, step, cell, a, b, mb, wb, coef, nunit, idx, purpose, counts):
        """Relativistic pair in its centre-of-momentum frame, written with
        4-momenta and the Lorentz boost matrix (t = E/c component first)."""
        c = CLIGHT
        wa = a[5]
        w = self.rng(step, cell, idx, purpose, 0)
        r4 = u32(w[3])

        def four(v, m):
            g = 1.0 / math.sqrt(1.0 - (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / c ** 2)
            return [g * m * c, g * m * v[0], g * m * v[1], g * m * v[2]], g

        def boost(pv, beta):
            b2 = beta[0] ** 2 + beta[1] ** 2 + beta[2] ** 2
            if b2 == 0.0:
                return list(pv)
            g = 1.0 / math.sqrt(1.0 - b2)
            bx = beta[0] * pv[1] + beta[1] * pv[2] + beta[2] * pv[3]
            t = g * (pv[0] - bx)
            k = (g - 1.0) * bx / b2 - g * pv[0]
            return [t, pv[1] + k * beta[0], pv[2] + k * beta[1], pv[3] + k * beta[2]]

        Pa, ga = four(a[2:5], ME)
        Pb, gb = four(b[2:5], mb)
        beta = [(Pa[q] + Pb[q]) / (Pa[0] + Pb[0]) for q in (1, 2, 3)]
        gc = 1.0 / math.sqrt(1.0 - (beta[0] ** 2 + beta[1] ** 2 + beta[2] ** 2))
        Sa, Sb = boost(Pa, beta), boost(Pb, beta)
        ps = Sa[1:]
        p = math.sqrt(ps[0] ** 2 + ps[1] ** 2 + ps[2] ** 2)
        if p == 0.0:
            return
        gas, gbs = Sa[0] / (ME * c), Sb[0] / (mb * c)
        mab = ME * mb / (ME + mb)
        s = (2.0 * coef * max(wa, wb) * nunit * mab ** 2 / (ME * ga * mb * gb)
             * gc * p / (ME * ga + mb * gb) * (ME * gas * mb * gbs * c * c / p ** 2 + 1.0) ** 2 / c ** 4)
        d2 = 0.5 * s
        if self.law == 1:
            omc = nanbu_omc(s, u52(w[0], w[1]))
            st = math.sqrt(omc * (2.0 - omc))
        else:
            g = math.sqrt(-2 * math.log(u32(w[0]))) * math.cos(2 * math.pi * ((w[1] << 20) + 0.5) / 2 ** 52)
            d = math.sqrt(d2) * g
            st, omc = 2 * d / (1 + d * d), 2 * d * d / (1 + d * d)
        ct = 1.0 - omc
        phi = 2 * math.pi * ((w[2] << 20) + 0.5) / 2 ** 52
        ux, uy, uz = ps[0] / p, ps[1] / p, ps[2] / p
        up = math.hypot(ux, uy)
        if up > 0:
            e1 = [ux * uz / up, uy * uz / up, -up]
            e2 = [-uy / up, ux / up, 0.0]
            n = [ct * [ux, uy, uz][q] + st * math.cos(phi) * e1[q] + st * math.sin(phi) * e2[q]
                 for q in range(3)]
        else:
            n = [st * math.cos(phi), st * math.sin(phi), ct * uz]
        qa = [Sa[0]] + [p * n[q] for q in range(3)]
        qb = [Sb[0]] + [-p * n[q] for q in range(3)]
        back = [-beta[0], -beta[1], -beta[2]]
        La, Lb = boost(qa, back), boost(qb, back)

        def vel(P, m):
            e = math.sqrt((m * c) ** 2 + P[1] ** 2 + P[2] ** 2 + P[3] ** 2)
            return [P[q] * c / e for q in (1, 2, 3)]

        if wa <= wb or r4 < wb / wa:
            a[2:5] = vel(La, ME)
        if wb <= wa or r4 < wa / wb:
            b[2:5] = vel(Lb, mb)
        counts["pairs"] += 1

    def collide(self, step, cell, a, b, mb, wb, coef, nunit, idx, purpose, counts):
        if self.rel:
            return self.collide_rel(step, cell, a, b, mb, wb, coef, nunit, idx, purpose, counts)
        ua = [a[2] - b[2], a[3] - b[3], a[4] - b[4]]
        u2 = ua[0] ** 2 + ua[1] ** 2 + ua[2] ** 2
        if u2 == 0.0:
            return
        wa = a[5]
        w = self.rng(step, cell, idx, purpose, 0)
        r4 = u32(w[3])
        u = math.sqrt(u2)
        d2 = coef * max(wa, wb) * nunit / u ** 3
        g = math.sqrt(-2 * math.log(u32(w[0]))) * math.cos(2 * math.pi * ((w[1] << 20) + 0.5) / 2 ** 52)
        d = math.sqrt(d2) * g
        st, omc = 2 * d / (1 + d * d), 2 * d * d / (1 + d * d)
        if self.law == 1:
            omc = nanbu_omc(2.0 * d2, u52(w[0], w[1]))
            st = math.sqrt(omc * (2.0 - omc))
        phi = 2 * math.pi * ((w[2] << 20) + 0.5) / 2 ** 52
        up = math.hypot(ua[0], ua[1])
        ux, uy, uz = ua
        if up > 0:
            du = [ux / up * uz * st * math.cos(phi) - uy / up * u * st * math.sin(phi) - ux * omc,
                  uy / up * uz * st * math.cos(phi) + ux / up * u * st * math.sin(phi) - uy * omc,
                  -up * st * math.cos(phi) - uz * omc]
        else:
            du = [abs(uz) * st * math.cos(phi), abs(uz) * st * math.sin(phi), -uz * omc]
        if wa <= wb or r4 < wb / wa:
            for q in range(3):
                a[2 + q] += mb / (ME + mb) * du[q]
        if wb <= wa or r4 < wa / wb:
            for q in range(3):
                b[2 + q] -= ME / (ME + mb) * du[q]
        counts["pairs"] += 1

    def drift(self, es, ws):
        wt = sum(ws)
        u = [sum(w * e[2 + q] for e, w in zip(es, ws)) / wt for q in range(3)]
        k = sum(w * 0.5 * ME * sum((e[2 + q] - u[q]) ** 2 for q in range(3)) / QE
                for e, w in zip(es, ws))
        return u, k

    def new_electron(self, step, cell, ion, idx, sub, energy, out):
        w = self.rng(step, cell, idx, 10, sub)
        mu = 2 * u52(w[0], w[1]) - 1
        phi = 2 * math.pi * ((((w[2] << 32) | w[3]) >> 12) + 0.5) / 2 ** 52
        sp = math.sqrt(2 * energy * QE / ME)
        st = math.sqrt(1 - mu * mu)
        out.append([ion[0], ion[1], sp * st * math.cos(phi), sp * st * math.sin(phi), sp * mu, 1])

    def step(self, cell_id, c, step, flags):
        s, t = self.s, self.t
        self.law = 1 if flags & 0x100 else 0
        self.rel = bool(flags & 0x200)
        mi = t.mass_ion
        counts = {"pairs": 0, "ion": 0, "rec": 0, "photo": 0, "decay": 0, "auger": 0}
        es, ions = c.e, c.i
        # S0
        we = sum(e[5] for e in es)
        wi = len(ions)
        sz = sum(i[5] for i in ions)
        sz2 = sum(i[5] ** 2 for i in ions)
        kb = sum(e[5] * self.ke(e) for e in es)
        t_e = max(2 * kb / (3 * we), 0.01) if we else 0.01
        n_e, n_i = we * s.w0 / s.volume, wi * s.w0 / s.volume
        zbar = sz / wi if wi else 0.0
        zstar = sz2 / sz if sz else 0.0
        dE = [self.ipd(z, t_e, n_e, n_i, zbar, zstar) for z in range(13)]
        lnl = s.lnl_fixed
        # S1
        ne, ni = len(es), len(ions)
        pe = self.perm(step, cell_id, 1, ne)
        if flags & 1 and ne >= 2:
            mee = ME / 2
            kee = QE ** 4 / (8 * math.pi * EPS0 ** 2 * mee ** 2)
            nunit = s.w0 * ne / s.volume
            start = 0
            if ne % 2 == 1 and ne >= 3:
                for tix, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
                    self.collide(step, cell_id, es[pe[a]], es[pe[b]], ME, es[pe[b]][5],
                                 kee * lnl * 0.5 * s.dt, nunit, tix, 6, counts)
                start = 3
            j = 0
            while start + 2 * j + 1 < ne:
                a, b = es[pe[start + 2 * j]], es[pe[start + 2 * j + 1]]
                self.collide(step, cell_id, a, b, ME, b[5], kee * lnl * s.dt, nunit, j, 5, counts)
                j += 1
        # S2
        if flags & 2 and ne >= 1 and ni >= 1:
            pi = self.perm(step, cell_id, 2, ni)
            mei = ME * mi / (ME + mi)
            kei = QE ** 4 / (8 * math.pi * EPS0 ** 2 * mei ** 2)
            nunit = s.w0 * min(ne, ni) / s.volume
            for kk in range(max(ne, ni)):
                if ne >= ni:
                    e, i = es[pe[kk]], ions[pi[kk % ni]]
                else:
                    i, e = ions[pi[kk]], es[pe[kk % ne]]
                if i[5] == 0:
                    continue
                self.collide(step, cell_id, e, i, mi, 1, kei * lnl * s.dt * i[5] ** 2, nunit,
                             kk, 7, counts)
        # S3
        if flags & 4 and ne >= 1 and ni >= 1:
            zc = (2 * sz + wi) // (2 * wi)
            if zc < 13:
                o = occ(zc, 0)
                tot = 0.0
                for e in es:
                    en = self.ke(e)
                    sig = 0.0
                    for q in range(5):
                        p = max(t.bind[zc, q] - dE[zc], 1.0)
                        if o[q] and en > p:
                            sig += t.lotz_a[q] * 1e-4 * o[q] * math.log(en / p) / (en * p)
                    tot += e[5] * sig * math.sqrt(2 * en * QE / ME)
                p = min(tot * s.w0 * s.dt / s.volume, 1.0)
                fired = []
                for m, ion in enumerate(ions):
                    if ion[5] < 13 and u32(self.rng(step, cell_id, m, 8, 0)[0]) < p:
                        fired.append(m)
                if fired:
                    u, kth = self.drift(es, [e[5] for e in es])
                    debit, new = 0.0, []
                    for m in fired:
                        ion = ions[m]
                        o2 = occ(ion[5], ion[6])
                        sv = max(q for q in range(5) if o2[q] > 0)
                        ip = max(t.bind[ion[5], sv] - dE[ion[5]], 1.0)
                        if debit + ip > kth:
                            break
                        debit += ip
                        ion[5] += 1
                        if sv == 0:
                            ion[6] += 1
                        new.append([ion[0], ion[1], 0.0, 0.0, 0.0, 1])
                        counts["ion"] += 1
                    if debit > 0:
                        al = math.sqrt(1 - debit / kth)
                        for e in es:
                            for q in range(3):
                                e[2 + q] = u[q] + al * (e[2 + q] - u[q])
                    es.extend(new)
        # S4
        ne = len(es)
        if flags & 8 and ne >= 1 and ni >= 1:
            sz = sum(i[5] for i in ions)
            kb = sum(e[5] * self.ke(e) for e in es)
            t2 = max(2 * kb / (3 * sum(e[5] for e in es)), 0.01)
            d = sz - ni * self.eos(n_i, t2)
            if d > 0:
                nrec = min(int(math.floor(d + 0.5)), sum(1 for i in ions if i[5] > s.z_floor), ne)
                if nrec > 0:
                    pri = [m for m in self.perm(step, cell_id, 3, ni) if ions[m][5] > s.z_floor][:nrec]
                    pre = self.perm(step, cell_id, 4, ne)[:nrec]
                    wp = [e[5] for e in es]
                    for j in pre:
                        wp[j] -= 1
                    alive = [j for j in range(ne) if wp[j] > 0]
                    if alive:
                        u, kth = self.drift([es[j] for j in alive], [wp[j] for j in alive])
                    if alive and kth > 0:
                        eadd = 0.0
                        for j, m in zip(pre, pri):
                            e, ion = es[j], ions[m]
                            keu = self.ke(e)
                            kib = 0.5 * mi * sum(v * v for v in ion[2:5]) / QE
                            for q in range(3):
                                ion[2 + q] += ME / mi * e[2 + q]
                            kia = 0.5 * mi * sum(v * v for v in ion[2:5]) / QE
                            z, k = ion[5], ion[6]
                            o0 = occ(z, k)
                            kn = k - 1 if (k >= 1 and o0[1] + o0[2] == 8) else k
                            o1 = occ(z - 1, kn)
                            sl = next(q for q in range(5) if o1[q] > o0[q])
                            ipr = max(t.bind[z - 1, sl] - dE[z - 1], 1.0)
                            ion[5], ion[6] = z - 1, kn
                            eadd += keu + ipr + (kib - kia)
                            counts["rec"] += 1
                        al = math.sqrt(1 + eadd / kth)
                        kept = []
                        for j in alive:
                            e = es[j]
                            for q in range(3):
                                e[2 + q] = u[q] + al * (e[2 + q] - u[q])
                            e[5] = wp[j]
                            kept.append(e)
                        es[:] = kept
        # S5
        if flags & 0x30:
            nb = len(s.photon_hv)
            new = []
            for m, ion in enumerate(ions):
                z0, k0 = ion[5], ion[6]
                if z0 >= 13:
                    continue
                o0 = occ(z0, k0)
                nl0 = o0[1] + o0[2]
                z, k = z0, k0
                if flags & 0x20 and k0 >= 1 and nl0 >= 1:
                    ga, gx = t.gamma_a[z0, k0], t.gamma_x[z0, k0]
                    if ga + gx > 0:
                        w = self.rng(step, cell_id, m, 9, 0)
                        if u52(w[0], w[1]) < min(s.dt_rad * (ga + gx), 1.0):
                            k = k0 - 1
                            counts["decay"] += 1
                            if nl0 >= 2 and u52(w[2], w[3]) < ga / (ga + gx):
                                z = z0 + 1
                                p2s = max(t.bind[z0, 1] - dE[z0], 1.0)
                                p2p = max(t.bind[z0, 2] - dE[z0], 1.0)
                                ea = max(t.e_kalpha[z0] - (o0[1] * p2s + o0[2] * p2p) / nl0, 0.0)
                                self.new_electron(step, cell_id, ion, m, 0, ea, new)
                                counts["auger"] += 1
                if flags & 0x10 and nb:
                    for q in range(3):
                        if o0[q] == 0:
                            continue
                        pp = max(t.bind[z0, q] - dE[z0], 1.0)
                        terms = [s.photon_n[b] * self.sig[b][q] if s.photon_hv[b] >= pp else 0.0
                                 for b in range(nb)]
                        tot = sum(terms)
                        if tot <= 0:
                            continue
                        fire = self.rng(step, cell_id, m, 8, 0)
                        if not u32(fire[1 + q]) < min(CL * s.dt_rad * o0[q] * tot, 1.0):
                            continue
                        if z >= 13 or occ(z, k)[q] == 0:
                            continue
                        w = self.rng(step, cell_id, m, 11, q)
                        target, cum, sel = u52(w[0], w[1]) * tot, 0.0, None
                        for b in range(nb):
                            cum += terms[b]
                            if terms[b] > 0 and cum > target:
                                sel = b
                                break
                        if sel is None:
                            sel = max(b for b in range(nb) if terms[b] > 0)
                        z += 1
                        if q == 0:
                            k += 1
                        self.new_electron(step, cell_id, ion, m, 1 + q, s.photon_hv[sel] - pp, new)
                        counts["photo"] += 1
                ion[5], ion[6] = z, k
            es.extend(new)
        return counts
