"""Alanine alpha-helices with covalent fragmentation (one residue per fragment).

The paper validates the covalent-boundary treatment on polyalanine helices
("Covalent bond fragmentation" benchmarks); the structures themselves are not
available, so the helix is built from ideal internal coordinates:
phi = -57, psi = -47, omega = 180 degrees; bond lengths N-CA 1.458,
CA-C 1.525, C-N 1.329, C=O 1.231, N-H 1.01, C-H 1.09, CA-CB 1.53 Angstrom;
H2N- and -COOH termini (10 n + 3 atoms).  Bond angles are standard
backbone values.  Each residue's fragment holds its N-H, CA, HA, the methyl
group and the preceding residue's C=O; the CA-C bond of every residue but
the last is cut, CA detached (it stays in its residue's fragment) and C
attached (it belongs to the next fragment).  Coordinates in bohr.
"""

import math

import numpy as np

from .geometry import ANGSTROM_TO_BOHR, System

Z_H, Z_C, Z_N, Z_O = 1, 6, 7, 8


def _place(a, b, c, bond, angle_deg, dihedral_deg):
    """Position of d with |cd| = bond, angle(b, c, d) = angle and
    dihedral(a, b, c, d) = dihedral (natural extension reference frame)."""
    ang = math.radians(angle_deg)
    dih = math.radians(dihedral_deg)
    bc = c - b
    bc /= np.linalg.norm(bc)
    n = np.cross(b - a, bc)
    n /= np.linalg.norm(n)
    m = np.cross(n, bc)
    d2 = np.array([-bond * math.cos(ang), bond * math.sin(ang) * math.cos(dih), bond * math.sin(ang) * math.sin(dih)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * n


def alanine_helix(n_res, phi=-57.0, psi=-47.0, omega=180.0, name=None):
    if n_res < 1:
        raise ValueError("need at least one residue")
    b_nca, b_cac, b_cn, b_co, b_nh, b_ch, b_cacb = 1.458, 1.525, 1.329, 1.231, 1.01, 1.09, 1.53
    a_ncac, a_cacn, a_cnca = 111.2, 116.2, 121.7
    # backbone N, CA, C of every residue
    N = [np.array([0.0, 0.0, 0.0])]
    CA = [np.array([b_nca, 0.0, 0.0])]
    t = math.radians(180.0 - a_ncac)
    C = [CA[0] + b_cac * np.array([math.cos(t), math.sin(t), 0.0])]
    for i in range(1, n_res):
        N.append(_place(N[i - 1], CA[i - 1], C[i - 1], b_cn, a_cacn, psi))
        CA.append(_place(CA[i - 1], C[i - 1], N[i], b_nca, a_cnca, omega))
        C.append(_place(C[i - 1], N[i], CA[i], b_cac, a_ncac, phi))
    atoms, frag = [], []

    def add(z, x, f):
        atoms.append((z, x))
        frag.append(f)
        return len(atoms) - 1

    bonds = []
    for i in range(n_res):
        f = i
        if i > 0:
            # carbonyl of the previous residue (the attached side of its cut bond)
            c_prev = add(Z_C, C[i - 1], f)
            add(Z_O, _place(N[i - 1], CA[i - 1], C[i - 1], b_co, 120.5, psi + 180.0), f)
            bonds.append((ca_prev, c_prev))
        add(Z_N, N[i], f)
        if i == 0:
            add(Z_H, _place(C[0], CA[0], N[0], b_nh, 109.5, 60.0), f)
            add(Z_H, _place(C[0], CA[0], N[0], b_nh, 109.5, -60.0), f)
        else:
            o_prev = _place(N[i - 1], CA[i - 1], C[i - 1], b_co, 120.5, psi + 180.0)
            add(Z_H, _place(o_prev, C[i - 1], N[i], b_nh, 119.5, 180.0), f)
        ca = add(Z_C, CA[i], f)
        add(Z_H, _place(C[i], N[i], CA[i], b_ch, 109.5, 117.9), f)
        cb_x = _place(C[i], N[i], CA[i], b_cacb, 110.5, -122.6)
        add(Z_C, cb_x, f)
        for dih in (60.0, 180.0, -60.0):
            add(Z_H, _place(N[i], CA[i], cb_x, b_ch, 109.5, dih), f)
        ca_prev = ca
        if i == n_res - 1:
            # -COOH terminus stays with the last residue
            add(Z_C, C[i], f)
            add(Z_O, _place(N[i], CA[i], C[i], b_co, 120.5, psi + 180.0), f)
            o2 = _place(N[i], CA[i], C[i], 1.34, 113.0, psi)
            add(Z_O, o2, f)
            add(Z_H, _place(CA[i], C[i], o2, 0.97, 105.0, 180.0), f)
    Z = np.array([z for z, _ in atoms], dtype=np.int32)
    xyz = np.array([x for _, x in atoms]) * ANGSTROM_TO_BOHR
    return System(name=name or f"ala{n_res}-helix", Z=Z, xyz=xyz, frag=np.array(frag, dtype=np.int32),
                  frag_charge=np.zeros(n_res, dtype=np.int32), meta=dict(n_res=n_res),
                  bonds=np.array(bonds, dtype=np.int32).reshape(-1, 2))
