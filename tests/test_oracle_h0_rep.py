"""Pins of the oracle's zeroth-order Hamiltonian, coordination numbers and
repulsion against the paper's formulas evaluated by hand, element by
element, from the raw parameter file (the reference side uses no oracle
code and no oracle parameter object):

* eq. h0_hamiltonian: for mu on A, nu on B (A != B)
      H0_mu,nu / S_mu,nu = K_AB (k_l + k_l')/2 (h_A^l + h_B^l')/2
                           (1 + k_EN (EN_A - EN_B)^2) Pi(R_AB);
* eq. xtb1_polynomial_correction:
      Pi(R) = (1 + k^poly_A,l sqrt(R / Rcov_AB)) (1 + k^poly_B,l' sqrt(R / Rcov_AB)),
      Rcov_AB = Rcov_A + Rcov_B;
* eq. xtb1_diagonal_h0: h_A^l = H_A^l (1 + k_CN,l CN_A), the on-site H0;
* eq. cn_def: CN_A = sum_B 1 / (1 + exp(-k1 (k2 (Rcov_A + Rcov_B) / R_AB - 1)));
* eq. gfn1_rep_energy: E_rep = sum over unordered pairs
      Zeff_A Zeff_B / R exp(-sqrt(alpha_A alpha_B) R^k_f).

The ratio H0/S isolates the prefactor, so the test needs no independent
overlap integral.  C-H, O-H and N-C pairs at several distances give distinct
electronegativity factors, level averages and polynomial factors; the CN
values are chosen freely (the system takes them as input) so that the CN
dependence of the levels is exercised with large, distinct values.  A
mistake in any factor (sign of k_EN, exponent of R/Rcov, a level taken from
the wrong atom or shell, the arithmetic instead of the geometric mean of the
repulsion exponents, ordered instead of unordered pairs) fails these tests.

AO order of a system (the oracle's documented basis order): atoms in the
given order; per atom its shells in parameter-file order; a p shell as
p_x, p_y, p_z.
"""

import json
import math

import numpy as np
import pytest

import workloads as w
from oracle import xtb as X

A2B = w.ANGSTROM_TO_BOHR


@pytest.fixture(scope="module")
def raw():
    with open(w.params_path()) as f:
        return json.load(f)


def _elem(raw, Z):
    for sym, e in raw["elements"].items():
        if int(e["Z"]) == Z:
            return e
    raise KeyError(Z)


def _ao_shells(raw, Zs):
    """(atom, shell dict) of every AO, in basis order."""
    out = []
    for A, Z in enumerate(Zs):
        for sh in _elem(raw, Z)["shells"]:
            out.extend([(A, sh)] * (1 if int(sh["l"]) == 0 else 3))
    return out


def _hand_prefactor(raw, ZA, ZB, R, cnA, cnB, shA, shB):
    g = raw["globals"]
    eA, eB = _elem(raw, ZA), _elem(raw, ZB)
    kl = g["kl"]
    k_ll = 0.5 * (kl[int(shA["l"])] + kl[int(shB["l"])])
    hA = shA["level"] * (1.0 + shA["kcn"] * cnA)
    hB = shB["level"] * (1.0 + shB["kcn"] * cnB)
    dEN = eA["EN"] - eB["EN"]
    en_fac = 1.0 + g["kEN"] * dEN * dEN
    rcov = (eA["rcov_angstrom"] + eB["rcov_angstrom"]) * g["angstrom_to_bohr"]
    x = math.sqrt(R / rcov)
    Pi = (1.0 + shA["kpoly"] * x) * (1.0 + shB["kpoly"] * x)
    return g["KAB"] * k_ll * 0.5 * (hA + hB) * en_fac * Pi


@pytest.mark.parametrize("ZA,ZB,R_ang", [(6, 1, 1.09), (6, 1, 1.9), (8, 1, 0.96), (8, 1, 2.4),
                                         (7, 6, 1.46), (6, 6, 1.40)])
def test_h0_prefactor_by_hand(raw, params, ZA, ZB, R_ang):
    R = R_ang * A2B
    # bond along a general direction so that every p component overlaps
    u = np.array([0.48, -0.36, 0.8])
    u /= np.linalg.norm(u)
    xyz = np.array([[0.3, -0.2, 0.1], [0.3, -0.2, 0.1]]) + np.outer([0.0, 1.0], u * R)
    cn = np.array([2.7, 0.9])
    sx = X.XtbSystem(params, [ZA, ZB], xyz, cn)
    aos = _ao_shells(raw, [ZA, ZB])
    assert len(aos) == sx.nao
    checked = 0
    for mu, (A, shm) in enumerate(aos):
        for nu, (B, shn) in enumerate(aos):
            if A == B:
                continue
            if abs(sx.S[mu, nu]) < 1e-6:
                continue
            if A == 0:
                want = _hand_prefactor(raw, ZA, ZB, R, cn[0], cn[1], shm, shn)
            else:
                want = _hand_prefactor(raw, ZB, ZA, R, cn[1], cn[0], shm, shn)
            got = sx.H0[mu, nu] / sx.S[mu, nu]
            assert abs(got - want) < 1e-12 * max(1.0, abs(want)), (mu, nu, got, want)
            checked += 1
    assert checked >= 8


def test_h0_onsite_by_hand(raw, params):
    """On-site block: diagonal h_A^l with the CN dependence, zero elsewhere
    (same-atom off-diagonal elements are zero; the on-site overlap is the
    identity)."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.1], [1.9, 0.0, -0.6]])
    Zs = [8, 1, 6]
    cn = np.array([1.7, 0.8, 3.2])
    sx = X.XtbSystem(params, Zs, xyz, cn)
    aos = _ao_shells(raw, Zs)
    for mu, (A, shm) in enumerate(aos):
        for nu, (B, shn) in enumerate(aos):
            if A != B:
                continue
            if mu == nu:
                want = shm["level"] * (1.0 + shm["kcn"] * cn[A])
                assert abs(sx.H0[mu, nu] - want) < 1e-15
                assert abs(sx.S[mu, nu] - 1.0) < 1e-12
            else:
                assert sx.H0[mu, nu] == 0.0
                assert abs(sx.S[mu, nu]) < 1e-12


def test_polynomial_factor_at_covalent_distance(raw, params):
    """At R = Rcov_A + Rcov_B, Pi = (1 + k^poly_s)(1 + k^poly_t) exactly;
    for C-C the electronegativity factor is 1, so the prefactor reduces to
    k_ll * (h_s + h_t)/2 * (1 + kpoly_s)(1 + kpoly_t) with the levels at zero
    CN."""
    g = raw["globals"]
    eC = _elem(raw, 6)
    R = 2.0 * eC["rcov_angstrom"] * g["angstrom_to_bohr"]
    xyz = np.array([[0.0, 0.0, 0.0], [R, 0.0, 0.0]])
    sx = X.XtbSystem(params, [6, 6], xyz, np.zeros(2))
    s_sh, p_sh = eC["shells"]
    # AO 0 = 2s of atom 0, AO 4 = 2s of atom 1; AO 5 = p_x of atom 1
    want_ss = g["kl"][0] * s_sh["level"] * (1 + s_sh["kpoly"]) ** 2
    assert abs(sx.H0[0, 4] / sx.S[0, 4] - want_ss) < 1e-13
    want_sp = (0.5 * (g["kl"][0] + g["kl"][1]) * 0.5 * (s_sh["level"] + p_sh["level"])
               * (1 + s_sh["kpoly"]) * (1 + p_sh["kpoly"]))
    assert abs(sx.H0[0, 5] / sx.S[0, 5] - want_sp) < 1e-13


def test_cn_by_hand(raw, params):
    g = raw["globals"]
    Zs = [8, 1, 1, 6]
    xyz = np.array([[0.0, 0.0, 0.0], [1.8, 0.0, 0.0], [-0.5, 1.7, 0.0], [0.4, 0.3, 3.3]])
    got = X.coordination_numbers(params, np.array(Zs), xyz)
    rc = [_elem(raw, z)["rcov_angstrom"] * g["angstrom_to_bohr"] for z in Zs]
    for A in range(4):
        want = 0.0
        for B in range(4):
            if B == A:
                continue
            R = float(np.linalg.norm(xyz[A] - xyz[B]))
            want += 1.0 / (1.0 + math.exp(-g["k1"] * (g["k2"] * (rc[A] + rc[B]) / R - 1.0)))
        assert abs(got[A] - want) < 1e-14


def test_repulsion_by_hand(raw, params):
    g = raw["globals"]
    Zs = [8, 1, 1, 6, 7]
    xyz = np.array([[0.0, 0.0, 0.0], [1.8, 0.0, 0.0], [-0.5, 1.7, 0.0], [0.4, 0.3, 3.3],
                    [2.9, -1.1, 1.4]])
    sx = X.XtbSystem(params, Zs, xyz, np.zeros(len(Zs)))
    want = 0.0
    for A in range(len(Zs)):
        for B in range(A + 1, len(Zs)):
            eA, eB = _elem(raw, Zs[A]), _elem(raw, Zs[B])
            R = float(np.linalg.norm(xyz[A] - xyz[B]))
            want += (eA["zeff"] * eB["zeff"] / R
                     * math.exp(-math.sqrt(eA["alpha_rep"] * eB["alpha_rep"]) * R ** g["kf"]))
    assert abs(sx.erep - want) < 1e-13 * abs(want)
    # a single pair: no factor 1/2 and no double counting
    s2 = X.XtbSystem(params, [8, 1], xyz[:2], np.zeros(2))
    eA, eB = _elem(raw, 8), _elem(raw, 1)
    R = 1.8
    one = eA["zeff"] * eB["zeff"] / R * math.exp(-math.sqrt(eA["alpha_rep"] * eB["alpha_rep"]) * R ** g["kf"])
    assert abs(s2.erep - one) < 1e-15
