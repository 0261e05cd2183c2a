"""Single-system GFN1-xTB for the oracle: CN, H0, gamma, repulsion, SCC, and
the building blocks of the analytic gradient.

Paper passages followed (section "GFN1-xTB"):
* electronic energy, eq. gfn1_energy_2: sum P H0 + 1/2 dq gamma dq
  - 1/3 sum_A Gamma_A dq_A^3 - T_el S_el;
* shell Mulliken charges; the printed formula sums over the free index, read
  as dq_s = sum_{mu in s} sum_nu P_mu,nu S_mu,nu - q0_s;
* gamma = (R^kg + eta^-kg)^(-1/kg), eta the harmonic mean of (1+kappa) eta_A;
* Fermi smearing of the occupations; the Fock matrix
  F = H0 + 1/2 S (sigma_mu + sigma_nu), sigma_s = sum_t gamma_st dq_t
  - Gamma_A dq_A^2 (+ the embedding potential of section "FMO-xTB");
* H0, eq. h0_hamiltonian, with Pi(R), eq. xtb1_polynomial_correction, and the
  CN-dependent levels, eq. xtb1_diagonal_h0; CN from eq. cn_def;
* repulsion, eq. gfn1_rep_energy (unordered atom pairs of the system).
Gradient building blocks follow eqs. xtb_grad, W_matrix, H0_deriv, cn_grad,
cn_factor.  Readings: Delta q = population minus reference; same-atom
off-diagonal H0 elements are zero; no cutoff in CN; dispersion and halogen
terms are not part of this build.
"""

import math

import numpy as np
from scipy import linalg as sla
from scipy.special import expit

from .integrals import element_basis, pair_blocks, ao_offsets


# --------------------------------------------------------------------------
# coordination number (eq. cn_def) over the whole system

def coordination_numbers(params, Z, xyz, chunk=2048):
    N = len(Z)
    rc = np.array([params.element(int(z))["rcov"] for z in Z])
    cn = np.zeros(N)
    for i0 in range(0, N, chunk):
        i1 = min(N, i0 + chunk)
        d = xyz[i0:i1, None, :] - xyz[None, :, :]
        R = np.sqrt(np.sum(d * d, axis=2))
        rcs = rc[i0:i1, None] + rc[None, :]
        with np.errstate(divide="ignore"):
            x = -params.k1 * (params.k2 * rcs / R - 1.0)
        f = expit(-x)   # 1 / (1 + exp(x))
        f[np.arange(i1 - i0), np.arange(i0, i1)] = 0.0
        cn[i0:i1] = f.sum(axis=1)
    return cn


def cn_gradient(params, Z, xyz, F, chunk=2048):
    """sum_A F_A dCN_A/dR_C for every atom C (eq. cn_grad)."""
    N = len(Z)
    rc = np.array([params.element(int(z))["rcov"] for z in Z])
    g = np.zeros((N, 3))
    for i0 in range(0, N, chunk):
        i1 = min(N, i0 + chunk)
        d = xyz[i0:i1, None, :] - xyz[None, :, :]   # C - A
        R = np.sqrt(np.sum(d * d, axis=2))
        idx = np.arange(i1 - i0)
        R[idx, np.arange(i0, i1)] = 1.0
        rcs = rc[i0:i1, None] + rc[None, :]
        x = -params.k1 * (params.k2 * rcs / R - 1.0)
        f = expit(-x)
        dfdR = -f * (1.0 - f) * params.k1 * params.k2 * rcs / (R * R)
        dfdR[idx, np.arange(i0, i1)] = 0.0
        # CN_A and CN_C both contain f(R_AC); d R_AC / d R_C = (C - A)/R
        w = (F[i0:i1, None] + F[None, :]) * dfdR / R
        g[i0:i1] = np.einsum("ca,cak->ck", w, d)
    return g


# --------------------------------------------------------------------------

class XtbSystem:
    """One GFN1-xTB system (a fragment, a dimer or the whole molecule).

    Z, xyz: atoms in basis order.  cn: coordination numbers of these atoms
    computed in the whole supersystem (FMO reads CN at supersystem level,
    section "Explicit FMO-xTB gradient", coordination number correction)."""

    def __init__(self, params, Z, xyz, cn, charge=0, hop=None):
        """hop: covalent boundary atoms of this system (section "Covalent bond
        fragmentation"), a list of (atom, kind, b) with kind "bda" (a
        detached atom whose partner is outside: it gives up one electron and
        its bond-pointing hybrid is projected out) or "ghost" (a copy of the
        detached atom of a bond whose attached atom is inside: one electron,
        everything but the bond-pointing hybrid projected out); b is the unit
        vector from the detached to the attached atom."""
        self.p = params
        self.Z = np.asarray(Z, dtype=np.int64)
        self.xyz = np.asarray(xyz, dtype=float)
        self.cn = np.asarray(cn, dtype=float)
        self.nat = len(self.Z)
        self.charge = charge
        self.ao_off = ao_offsets(params, self.Z)
        self.nao = int(self.ao_off[-1])
        # shells
        sh_atom, sh_l, sh_level, sh_kcn, sh_kpoly, sh_eta, sh_q0, sh_ao0, sh_nao = ([] for _ in range(9))
        self.atom_sh0 = np.zeros(self.nat + 1, dtype=np.int64)
        for A, z in enumerate(self.Z):
            e = params.element(int(z))
            eb = element_basis(params, z)
            for s, sh in zip(eb.shells, e["shells"]):
                sh_atom.append(A)
                sh_l.append(sh["l"])
                sh_level.append(sh["level"])
                sh_kcn.append(sh["kcn"])
                sh_kpoly.append(sh["kpoly"])
                sh_eta.append((1.0 + sh["kappa"]) * e["eta"])
                sh_q0.append(sh["q0"])
                sh_ao0.append(self.ao_off[A] + s.ao0)
                sh_nao.append(s.nao)
            self.atom_sh0[A + 1] = len(sh_atom)
        self.sh_atom = np.array(sh_atom)
        self.sh_l = np.array(sh_l)
        self.sh_level = np.array(sh_level)
        self.sh_kcn = np.array(sh_kcn)
        self.sh_kpoly = np.array(sh_kpoly)
        self.sh_eta = np.array(sh_eta)
        self.sh_q0 = np.array(sh_q0)
        self.sh_ao0 = np.array(sh_ao0)
        self.sh_nao = np.array(sh_nao)
        self.nsh = len(sh_atom)
        self.ao_sh = np.repeat(np.arange(self.nsh), self.sh_nao)
        self.ao_atom = self.sh_atom[self.ao_sh]
        self.at_EN = np.array([params.element(int(z))["EN"] for z in self.Z])
        self.at_rcov = np.array([params.element(int(z))["rcov"] for z in self.Z])
        self.at_Gamma = np.array([params.element(int(z))["Gamma"] for z in self.Z])
        self.at_zeff = np.array([params.element(int(z))["zeff"] for z in self.Z])
        self.at_arep = np.array([params.element(int(z))["arep"] for z in self.Z])
        self.sh_h = self.sh_level * (1.0 + self.sh_kcn * self.cn[self.sh_atom])
        self.hop = list(hop or [])
        self._apply_hop_references()
        self.nel = float(self.sh_q0.sum()) - charge
        self._build()
        self._build_hop()

    # -- integrals -----------------------------------------------------------
    def _pairs(self):
        A, B = np.triu_indices(self.nat, k=1)
        return A, B

    def _shell_pair_prefactor(self, s, t, R):
        """H0 prefactor of eq. h0_hamiltonian for shell s on A, t on B (A != B),
        without the CN dependence split out: returns (full, Pi, dPi/dR, base)
        where base = K_AB * (k_l + k_l')/2 * EN factor."""
        p = self.p
        A, B = self.sh_atom[s], self.sh_atom[t]
        kll = 0.5 * (p.kl[self.sh_l[s]] + p.kl[self.sh_l[t]])
        den = self.at_EN[A] - self.at_EN[B]
        base = p.KAB * kll * (1.0 + p.kEN * den * den)
        rcov = self.at_rcov[A] + self.at_rcov[B]
        x = np.sqrt(R / rcov)
        pa = 1.0 + self.sh_kpoly[s] * x
        pb = 1.0 + self.sh_kpoly[t] * x
        Pi = pa * pb
        dx = 0.5 / np.sqrt(R * rcov)
        dPi = (self.sh_kpoly[s] * pb + pa * self.sh_kpoly[t]) * dx
        hav = 0.5 * (self.sh_h[s] + self.sh_h[t])
        return base * hav * Pi, Pi, dPi, base

    def _build(self):
        p = self.p
        n = self.nao
        S = np.eye(n)
        H0 = np.zeros((n, n))
        for s in range(self.nsh):
            for k in range(self.sh_nao[s]):
                H0[self.sh_ao0[s] + k, self.sh_ao0[s] + k] = self.sh_h[s]
        self.pair_S = {}
        self.pair_dS = {}
        A, B = self._pairs()
        for za in np.unique(self.Z):
            for zb in np.unique(self.Z):
                sel = np.where((self.Z[A] == za) & (self.Z[B] == zb))[0]
                if len(sel) == 0:
                    continue
                blk, dblk = pair_blocks(p, za, zb, self.xyz[A[sel]] - self.xyz[B[sel]])
                for k, ip in enumerate(sel):
                    self.pair_S[ip] = blk[k]
                    self.pair_dS[ip] = dblk[k]
        for ip in range(len(A)):
            a, b = A[ip], B[ip]
            ia = slice(self.ao_off[a], self.ao_off[a + 1])
            ib = slice(self.ao_off[b], self.ao_off[b + 1])
            blk = self.pair_S[ip]
            S[ia, ib] = blk
            S[ib, ia] = blk.T
            R = float(np.linalg.norm(self.xyz[a] - self.xyz[b]))
            hblk = np.zeros_like(blk)
            for s in range(self.atom_sh0[a], self.atom_sh0[a + 1]):
                for t in range(self.atom_sh0[b], self.atom_sh0[b + 1]):
                    fac = self._shell_pair_prefactor(s, t, R)[0]
                    i0 = self.sh_ao0[s] - self.ao_off[a]
                    j0 = self.sh_ao0[t] - self.ao_off[b]
                    hblk[i0:i0 + self.sh_nao[s], j0:j0 + self.sh_nao[t]] = (
                        fac * blk[i0:i0 + self.sh_nao[s], j0:j0 + self.sh_nao[t]])
            H0[ia, ib] = hblk
            H0[ib, ia] = hblk.T
        self.S = S
        self.H0 = H0
        self.pairA, self.pairB = A, B
        # gamma between shells (shell-resolved; broadcast over the AOs of a shell)
        d = self.xyz[self.sh_atom][:, None, :] - self.xyz[self.sh_atom][None, :, :]
        R = np.sqrt(np.sum(d * d, axis=2))
        self.gamma = gamma_matrix(p, R, self.sh_eta[:, None], self.sh_eta[None, :])
        # repulsion, unordered pairs within the system
        self.erep = 0.0
        for a, b in zip(A, B):
            R = float(np.linalg.norm(self.xyz[a] - self.xyz[b]))
            self.erep += (self.at_zeff[a] * self.at_zeff[b] / R
                          * math.exp(-math.sqrt(self.at_arep[a] * self.at_arep[b]) * R ** p.kf))

    # -- covalent boundaries (HOP) --------------------------------------------
    def _hop_atom_layout(self, A):
        """(s shell, p shell) of a boundary atom; it must have exactly one s
        and one p shell (4 AOs)."""
        shells = list(range(self.atom_sh0[A], self.atom_sh0[A + 1]))
        ls = [int(self.sh_l[t]) for t in shells]
        if ls != [0, 1]:
            raise ValueError("a covalent boundary atom needs one s and one p shell")
        return shells[0], shells[1]

    def _apply_hop_references(self):
        """Reference populations and repulsion charges of boundary atoms: the
        detached atom gives one electron to the bond, taken 1/4 from s and 3/4
        from p (sp3 hybrid weights); the ghost carries 1/4 s + 3/4 p.  The
        repulsion charge is scaled by (v - 1)/v and 1/v (v = valence electrons
        of the element)."""
        for A, kind, _ in self.hop:
            s_sh, p_sh = self._hop_atom_layout(A)
            v = float(self.sh_q0[s_sh] + self.sh_q0[p_sh])
            if kind == "bda":
                self.sh_q0[s_sh] -= 0.25
                self.sh_q0[p_sh] -= 0.75
                self.at_zeff[A] *= (v - 1.0) / v
            elif kind == "ghost":
                self.sh_q0[s_sh] = 0.25
                self.sh_q0[p_sh] = 0.75
                self.at_zeff[A] *= 1.0 / v
            else:
                raise ValueError(kind)

    def hybrid(self, A, b):
        """AO coefficients of the sp3 hybrid 1/2 s + sqrt(3)/2 (b . p) on atom A
        (eq. hybrid), as a length-nao vector."""
        s_sh, p_sh = self._hop_atom_layout(A)
        h = np.zeros(self.nao)
        h[self.sh_ao0[s_sh]] = 0.5
        h[self.sh_ao0[p_sh]:self.sh_ao0[p_sh] + 3] = 0.5 * math.sqrt(3.0) * np.asarray(b, float)
        return h

    def _build_hop(self):
        """V^HOP = S D S (eq. vhop), D = V h h^T on a detached atom (eq. dd_bda)
        and V (1_sp - h h^T) on a ghost (eq. dd_ghost)."""
        n = self.nao
        D = np.zeros((n, n))
        for A, kind, b in self.hop:
            h = self.hybrid(A, b)
            blk = slice(self.ao_off[A], self.ao_off[A + 1])
            if kind == "bda":
                D += self.p.VHOP * np.outer(h, h)
            else:
                one = np.zeros((n, n))
                one[blk, blk] = np.eye(self.ao_off[A + 1] - self.ao_off[A])
                D += self.p.VHOP * (one - np.outer(h, h))
        self.D_hop = D
        self.V_hop = self.S @ D @ self.S if self.hop else np.zeros((n, n))

    # -- Mulliken charges and energy -----------------------------------------
    def shell_charges(self, P):
        pop_ao = np.sum(P * self.S, axis=1)
        return np.bincount(self.ao_sh, weights=pop_ao, minlength=self.nsh) - self.sh_q0

    def atom_sum(self, v):
        return np.bincount(self.sh_atom, weights=v, minlength=self.nat)

    def shift(self, q, phi):
        """Shell potential sigma_s = sum_t gamma_st q_t - Gamma_A q_A^2 + phi_s."""
        qa = self.atom_sum(q)
        return self.gamma @ q - (self.at_Gamma * qa * qa)[self.sh_atom] + phi

    def fock(self, q, phi):
        """F = H0 + 1/2 S (sigma_mu + sigma_nu), plus V^HOP at covalent
        boundaries (eq. fock_hop)."""
        sig = self.shift(q, phi)[self.ao_sh]
        F = self.H0 + 0.5 * self.S * (sig[:, None] + sig[None, :])
        return F + self.V_hop if self.hop else F

    def energy_internal(self, P, q, occ):
        """E'_X of the system without the embedding term (eq. gfn1_energy_2 plus
        the repulsion); a HOP projector is a constraint and not part of it
        (section "FMO-xTB HOP energy")."""
        qa = self.atom_sum(q)
        e = float(np.sum(P * self.H0))
        e += 0.5 * float(q @ self.gamma @ q)
        e -= float(np.sum(self.at_Gamma * qa ** 3)) / 3.0
        e += minus_TS(self.p.kT, occ)
        return e + self.erep


def gamma_matrix(params, R, eta_s, eta_t):
    eta = 2.0 / (1.0 / eta_s + 1.0 / eta_t)
    kg = params.kg
    return (R ** kg + eta ** (-kg)) ** (-1.0 / kg)


def gamma_deriv(params, R, eta_s, eta_t):
    """d gamma / dR."""
    eta = 2.0 / (1.0 / eta_s + 1.0 / eta_t)
    kg = params.kg
    return -R ** (kg - 1.0) * (R ** kg + eta ** (-kg)) ** (-1.0 / kg - 1.0)


def fermi_occupations(eps, nel, kT):
    """Closed-shell Fermi-Dirac occupations n_i = 2 f((eps_i - eF)/kT) with eF
    from bisection so that sum n_i = nel (section "GFN1-xTB", Fermi smearing)."""
    lo, hi = float(eps.min()) - 1.0, float(eps.max()) + 1.0
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        tot = 2.0 * np.sum(expit(-(eps - mid) / kT))
        if tot > nel:
            hi = mid
        else:
            lo = mid
        if hi - lo < 1e-15:
            break
    ef = 0.5 * (lo + hi)
    return 2.0 * expit(-(eps - ef) / kT), ef


def minus_TS(kT, occ):
    """-T_el S_el with S_el = -2 k_B sum [f ln f + (1-f) ln(1-f)], f = n/2."""
    f = np.clip(occ / 2.0, 0.0, 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(f > 0, f * np.log(f), 0.0) + np.where(f < 1, (1 - f) * np.log(1 - f), 0.0)
    return 2.0 * kT * float(np.sum(t))


class SCCResult:
    pass


def scc(sysx, phi=None, q_guess=None, tol=1e-10, etol=1e-11, maxiter=500,
        memory=8, beta=0.5):
    """Self-consistent charges for one system in a fixed external shell
    potential phi (zero for an isolated system).

    Iteration: sigma -> F -> generalized eigenproblem F C = S C eps (LAPACK)
    -> Fermi occupations -> P = C n C^T -> Mulliken charges -> Anderson (Pulay)
    mixing of the charges.  Converged when max|q_out - q_in| < tol and the
    energy change is below etol."""
    nsh = sysx.nsh
    phi = np.zeros(nsh) if phi is None else np.asarray(phi, float)
    q_in = np.zeros(nsh) if q_guess is None else np.asarray(q_guess, float).copy()
    X, Rr = [], []
    e_old = None
    res = SCCResult()
    res.converged = False
    for it in range(1, maxiter + 1):
        F = sysx.fock(q_in, phi)
        eps, C = sla.eigh(F, sysx.S)
        occ, ef = fermi_occupations(eps, sysx.nel, sysx.p.kT)
        P = (C * occ) @ C.T
        q_out = sysx.shell_charges(P)
        e = sysx.energy_internal(P, q_out, occ)
        r = q_out - q_in
        err = float(np.max(np.abs(r))) if nsh else 0.0
        de = abs(e - e_old) if e_old is not None else np.inf
        e_old = e
        if err < tol and de < etol:
            res.converged = True
            break
        X.append(q_in.copy())
        Rr.append(r.copy())
        if len(X) > memory:
            X.pop(0)
            Rr.pop(0)
        m = len(X)
        if m == 1:
            q_in = q_in + beta * r
        else:
            Bm = np.array([[Rr[i] @ Rr[j] for j in range(m)] for i in range(m)])
            M = np.zeros((m + 1, m + 1))
            M[:m, :m] = Bm
            M[:m, m] = 1.0
            M[m, :m] = 1.0
            rhs = np.zeros(m + 1)
            rhs[m] = 1.0
            c = np.linalg.lstsq(M, rhs, rcond=None)[0][:m]
            q_in = sum(c[k] * (X[k] + beta * Rr[k]) for k in range(m))
    res.niter = it
    res.err = err       # final max |q_out - q_in|
    res.de = de         # final |E_k - E_(k-1)|
    res.q = q_out
    res.P = P
    res.C = C
    res.eps = eps
    res.occ = occ
    res.ef = ef
    res.e_int = e
    res.e_emb = e + float(q_out @ phi)
    res.phi = phi
    res.sigma = sysx.shift(q_out, phi)
    res.Wt = (C * (occ * eps)) @ C.T
    return res


# --------------------------------------------------------------------------
# gradient building blocks

def system_gradient(sysx, DH, DS, gx=None, gy=None, with_rep=True):
    """Nuclear gradient of
        sum D_H H0 + sum D_S S + 1/2 sum_{s,t} gx_s gamma_st gy_t + E_rep
    for the atoms of one system at fixed CN, plus the CN sensitivities
    F_A = d/dCN_A of the D_H term (eq. cn_factor).  D_H and D_S symmetric.

    Returns (g (nat, 3), F_cn (nat,))."""
    p = sysx.p
    g = np.zeros((sysx.nat, 3))
    Fcn = np.zeros(sysx.nat)
    # on-site levels h = H (1 + kcn CN)
    for s in range(sysx.nsh):
        a0 = sysx.sh_ao0[s]
        tr = sum(DH[a0 + k, a0 + k] for k in range(sysx.sh_nao[s]))
        Fcn[sysx.sh_atom[s]] += tr * sysx.sh_level[s] * sysx.sh_kcn[s]
    for ip in range(len(sysx.pairA)):
        a, b = sysx.pairA[ip], sysx.pairB[ip]
        Rv = sysx.xyz[a] - sysx.xyz[b]
        R = float(np.linalg.norm(Rv))
        u = Rv / R
        Sblk = sysx.pair_S[ip]
        dSblk = sysx.pair_dS[ip]       # (3, na, nb), d/dR with R = A - B
        ia0, ib0 = sysx.ao_off[a], sysx.ao_off[b]
        gpair = np.zeros(3)
        for s in range(sysx.atom_sh0[a], sysx.atom_sh0[a + 1]):
            for t in range(sysx.atom_sh0[b], sysx.atom_sh0[b + 1]):
                full, Pi, dPi, base = sysx._shell_pair_prefactor(s, t, R)
                i0 = sysx.sh_ao0[s] - ia0
                j0 = sysx.sh_ao0[t] - ib0
                ns, nt = sysx.sh_nao[s], sysx.sh_nao[t]
                dh = DH[ia0 + i0:ia0 + i0 + ns, ib0 + j0:ib0 + j0 + nt]
                ds = DS[ia0 + i0:ia0 + i0 + ns, ib0 + j0:ib0 + j0 + nt]
                sb = Sblk[i0:i0 + ns, j0:j0 + nt]
                dsb = dSblk[:, i0:i0 + ns, j0:j0 + nt]
                # factor 2: (mu,nu) and (nu,mu) entries of the symmetric sums
                gpair += 2.0 * np.einsum("ij,kij->k", full * dh + ds, dsb)
                # Pi derivative (eq. H0_deriv second term)
                gpair += 2.0 * float(np.sum(dh * sb)) * base * 0.5 * (sysx.sh_h[s] + sysx.sh_h[t]) * dPi * u
                # CN dependence of the level average
                w = 2.0 * float(np.sum(dh * sb)) * base * Pi * 0.5
                Fcn[a] += w * sysx.sh_level[s] * sysx.sh_kcn[s]
                Fcn[b] += w * sysx.sh_level[t] * sysx.sh_kcn[t]
        if gx is not None:
            for s in range(sysx.atom_sh0[a], sysx.atom_sh0[a + 1]):
                for t in range(sysx.atom_sh0[b], sysx.atom_sh0[b + 1]):
                    dg = gamma_deriv(p, R, sysx.sh_eta[s], sysx.sh_eta[t])
                    gpair += 0.5 * (gx[s] * gy[t] + gy[s] * gx[t]) * dg * u
        if with_rep:
            za, zb = sysx.at_zeff[a], sysx.at_zeff[b]
            al = math.sqrt(sysx.at_arep[a] * sysx.at_arep[b])
            e = za * zb / R * math.exp(-al * R ** p.kf)
            de = e * (-1.0 / R - al * p.kf * R ** (p.kf - 1.0))
            gpair += de * u
        g[a] += gpair
        g[b] -= gpair
    return g, Fcn
