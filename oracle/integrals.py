"""Minimal-basis overlap integrals and their nuclear derivatives (oracle).

GFN1-xTB uses a Slater-type minimal basis (section "GFN1-xTB"); here every
Slater function is an STO-6G contraction of Cartesian Gaussians taken from
the input parameter file (exponents scaled by zeta^2).  Hydrogen carries a
second s shell that is Gram-Schmidt orthogonalised against the first, so every
on-site overlap block is the identity.

Primitive overlaps follow the Gaussian product theorem, written out for s and
p functions with R = A - B, p = a + b, mu = a b / p:

    <s|s>     = (pi/p)^(3/2) exp(-mu R^2)
    <p_i|s>   = (P - A)_i <s|s>,          (P - A) = -(b/p) R
    <s|p_j>   = (P - B)_j <s|s>,          (P - B) =  (a/p) R
    <p_i|p_j> = [(P-A)_i (P-B)_j + delta_ij / (2p)] <s|s>

Derivatives with respect to centre A are derivatives with respect to R.
AO order within an atom: shells in parameter order, p as x, y, z.
"""

import math

import numpy as np


def _prim_norm(l, a):
    n = (2.0 * a / math.pi) ** 0.75
    if l == 1:
        n = n * 2.0 * math.sqrt(a)
    return n


class Shell:
    __slots__ = ("atom", "l", "n", "zeta", "alpha", "coef", "nao", "ao0", "idx",
                 "level", "q0", "kcn", "kpoly", "kappa", "elem_shell")

    def __init__(self, atom, sh, alpha_unit, coef_unit, elem_shell):
        self.atom = atom
        self.l = sh["l"]
        self.n = sh["n"]
        self.zeta = sh["zeta"]
        self.level = sh["level"]
        self.q0 = sh["q0"]
        self.kcn = sh["kcn"]
        self.kpoly = sh["kpoly"]
        self.kappa = sh["kappa"]
        self.elem_shell = elem_shell
        self.alpha = alpha_unit * self.zeta ** 2
        c = coef_unit * np.array([_prim_norm(self.l, a) for a in self.alpha])
        # renormalise the contraction
        s = 0.0
        for i, ai in enumerate(self.alpha):
            for j, aj in enumerate(self.alpha):
                p = ai + aj
                v = (math.pi / p) ** 1.5
                if self.l == 1:
                    v /= 2.0 * p
                s += c[i] * c[j] * v
        self.coef = c / math.sqrt(s)
        self.nao = 1 if self.l == 0 else 3


def build_shells(params, Z):
    """Shell list for atoms Z (in the given order) and the AO count."""
    shells = []
    ao = 0
    for A, z in enumerate(Z):
        e = params.element(int(z))
        for k, sh in enumerate(e["shells"]):
            a, c = params.basis[(sh["n"], sh["l"])]
            s = Shell(A, sh, a, c, k)
            s.ao0 = ao
            s.idx = len(shells)
            ao += s.nao
            shells.append(s)
    return shells, ao


def prim_block(la, a, ca, lb, b, cb, R):
    """Contracted overlap block between shells (la at A) and (lb at B) and its
    derivative with respect to R = A - B.

    R: (m, 3).  Returns S (m, na, nb) and dS (m, 3, na, nb)."""
    R = np.atleast_2d(R)
    m = R.shape[0]
    na = 1 if la == 0 else 3
    nb = 1 if lb == 0 else 3
    S = np.zeros((m, na, nb))
    dS = np.zeros((m, 3, na, nb))
    R2 = np.sum(R * R, axis=1)
    eye = np.eye(3)
    for i in range(len(a)):
        for j in range(len(b)):
            p = a[i] + b[j]
            mu = a[i] * b[j] / p
            s00 = (math.pi / p) ** 1.5 * np.exp(-mu * R2) * ca[i] * cb[j]  # (m,)
            ds00 = -2.0 * mu * R * s00[:, None]                            # (m,3)
            PA = -(b[j] / p) * R                                           # (m,3)
            PB = (a[i] / p) * R
            if la == 0 and lb == 0:
                S[:, 0, 0] += s00
                dS[:, :, 0, 0] += ds00
            elif la == 1 and lb == 0:
                S[:, :, 0] += PA * s00[:, None]
                # d/dR_k [PA_i s00] = -(b/p) delta_ik s00 + PA_i ds00_k
                dS[:, :, :, 0] += (-(b[j] / p) * eye[None, :, :] * s00[:, None, None]
                                   + ds00[:, :, None] * PA[:, None, :])
            elif la == 0 and lb == 1:
                S[:, 0, :] += PB * s00[:, None]
                dS[:, :, 0, :] += ((a[i] / p) * eye[None, :, :] * s00[:, None, None]
                                   + ds00[:, :, None] * PB[:, None, :])
            else:
                core = PA[:, :, None] * PB[:, None, :] + eye[None] / (2.0 * p)  # (m,3,3)
                S += core * s00[:, None, None]
                # d core_ij / dR_k = -(b/p) d_ik PB_j + (a/p) PA_i d_jk
                dcore = (-(b[j] / p) * eye[None, :, :, None] * PB[:, None, None, :]
                         + (a[i] / p) * PA[:, None, :, None] * eye[None, :, None, :])
                # dcore indices: (m, k, i, j)
                dS += dcore * s00[:, None, None, None] + ds00[:, :, None, None] * core[:, None, :, :]
    return S, dS


class ElementBasis:
    """Shells of one element: exponents, contraction, AO layout and the on-site
    orthogonalisation T (identity except for a second s shell)."""

    def __init__(self, params, Z):
        e = params.element(int(Z))
        self.shells = []
        ao = 0
        for k, sh in enumerate(e["shells"]):
            a, c = params.basis[(sh["n"], sh["l"])]
            s = Shell(0, sh, a, c, k)
            s.ao0 = ao
            s.idx = k
            ao += s.nao
            self.shells.append(s)
        self.nao = ao
        self.T = np.eye(ao)
        ss = [s for s in self.shells if s.l == 0]
        if len(ss) >= 2:
            s1, s2 = ss[0], ss[1]
            Sblk, _ = prim_block(0, s1.alpha, s1.coef, 0, s2.alpha, s2.coef, np.zeros((1, 3)))
            s12 = float(Sblk[0, 0, 0])
            N = 1.0 / math.sqrt(1.0 - s12 * s12)
            self.T[s2.ao0, s2.ao0] = N
            self.T[s1.ao0, s2.ao0] = -N * s12


def element_basis(params, Z):
    """Element basis, cached on the parameter object."""
    cache = params.__dict__.setdefault("_element_basis", {})
    if int(Z) not in cache:
        cache[int(Z)] = ElementBasis(params, Z)
    return cache[int(Z)]


def pair_blocks(params, ZA, ZB, R):
    """Overlap blocks <A|B> (after on-site orthogonalisation) for m atom pairs
    with element ZA at A and ZB at B, R = A - B of shape (m, 3).

    Returns S (m, nA, nB) and dS/dR (m, 3, nA, nB)."""
    ea, eb = element_basis(params, ZA), element_basis(params, ZB)
    m = R.shape[0]
    Sraw = np.zeros((m, ea.nao, eb.nao))
    dSraw = np.zeros((m, 3, ea.nao, eb.nao))
    for sa in ea.shells:
        for sb in eb.shells:
            Sb, dSb = prim_block(sa.l, sa.alpha, sa.coef, sb.l, sb.alpha, sb.coef, R)
            ia = slice(sa.ao0, sa.ao0 + sa.nao)
            ib = slice(sb.ao0, sb.ao0 + sb.nao)
            Sraw[:, ia, ib] = Sb
            dSraw[:, :, ia, ib] = dSb
    S = np.einsum("ai,mab,bj->mij", ea.T, Sraw, eb.T)
    dS = np.einsum("ai,mkab,bj->mkij", ea.T, dSraw, eb.T)
    return S, dS


def onsite_block(params, Z):
    """On-site overlap block of one atom computed from the integrals
    (identity by construction; used as a check)."""
    e = element_basis(params, Z)
    Sraw = np.zeros((e.nao, e.nao))
    for sa in e.shells:
        for sb in e.shells:
            Sb, _ = prim_block(sa.l, sa.alpha, sa.coef, sb.l, sb.alpha, sb.coef, np.zeros((1, 3)))
            Sraw[sa.ao0:sa.ao0 + sa.nao, sb.ao0:sb.ao0 + sb.nao] = Sb[0]
    return e.T.T @ Sraw @ e.T


def ao_offsets(params, Z):
    """First AO of every atom and the AO count, atoms in the given order."""
    off = np.zeros(len(Z) + 1, dtype=np.int64)
    for A, z in enumerate(Z):
        off[A + 1] = off[A] + element_basis(params, z).nao
    return off


def overlap(params, Z, xyz):
    """Overlap matrix of a system, atoms in the given order."""
    Z = np.asarray(Z)
    off = ao_offsets(params, Z)
    n = int(off[-1])
    S = np.zeros((n, n))
    for A in range(len(Z)):
        S[off[A]:off[A + 1], off[A]:off[A + 1]] = np.eye(off[A + 1] - off[A])
    for za in np.unique(Z):
        for zb in np.unique(Z):
            ia = np.where(Z == za)[0]
            ib = np.where(Z == zb)[0]
            AA, BB = np.meshgrid(ia, ib, indexing="ij")
            AA, BB = AA.ravel(), BB.ravel()
            keep = AA != BB
            AA, BB = AA[keep], BB[keep]
            if len(AA) == 0:
                continue
            blk, _ = pair_blocks(params, za, zb, xyz[AA] - xyz[BB])
            na, nb = blk.shape[1], blk.shape[2]
            for k in range(len(AA)):
                a0, b0 = off[AA[k]], off[BB[k]]
                S[a0:a0 + na, b0:b0 + nb] = blk[k]
    return S
