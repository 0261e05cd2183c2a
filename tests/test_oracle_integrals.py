"""Pins of the oracle's one-electron pieces against independent mathematics.

* contracted overlaps against 1-D numerical quadrature of the Cartesian
  factors (independent of the Gaussian product theorem used by the oracle);
* the STO-6G fit against the closed-form Slater 1s-1s overlap;
* on-site blocks are the identity, S is symmetric positive definite;
* derivatives against central finite differences;
* gamma, CN and the Fermi/entropy terms against their closed-form limits.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import integrals as I
from oracle import xtb as X
import workloads as w


def _quad_block(sa, sb, R):
    """<sa at R|sb at 0> by 1-D quadrature of each Cartesian factor."""
    A = np.asarray(R, float)
    B = np.zeros(3)
    na, nb = sa.nao, sb.nao
    out = np.zeros((na, nb))
    for i, (ai, ci) in enumerate(zip(sa.alpha, sa.coef)):
        for j, (bj, cj) in enumerate(zip(sb.alpha, sb.coef)):
            def f1(k, pa, pb):
                g = lambda x: ((x - A[k]) ** pa * (x - B[k]) ** pb
                               * math.exp(-ai * (x - A[k]) ** 2 - bj * (x - B[k]) ** 2))
                lo = min(A[k], B[k]) - 12.0
                hi = max(A[k], B[k]) + 12.0
                return integrate.quad(g, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
            for u in range(na):
                for v in range(nb):
                    val = ci * cj
                    for k in range(3):
                        pa = 1 if (sa.l == 1 and u == k) else 0
                        pb = 1 if (sb.l == 1 and v == k) else 0
                        val *= f1(k, pa, pb)
                    out[u, v] += val
    return out


@pytest.mark.parametrize("za,zb", [(8, 1), (6, 6), (1, 8)])
def test_overlap_vs_quadrature(params, za, zb):
    ea, eb = I.element_basis(params, za), I.element_basis(params, zb)
    R = np.array([1.3, -0.7, 1.9])
    Sraw = np.zeros((ea.nao, eb.nao))
    for sa in ea.shells:
        for sb in eb.shells:
            Sraw[sa.ao0:sa.ao0 + sa.nao, sb.ao0:sb.ao0 + sb.nao] = _quad_block(sa, sb, R)
    ref = ea.T.T @ Sraw @ eb.T
    S, _ = I.pair_blocks(params, za, zb, R[None, :])
    assert np.max(np.abs(S[0] - ref)) < 1e-10


def test_sto_fit_against_slater_overlap(params):
    # two H 1s Slater functions with the same exponent: exact overlap
    # exp(-zR) (1 + zR + (zR)^2/3)
    e = I.element_basis(params, 1)
    s1 = e.shells[0]
    for R in (0.5, 1.4, 3.0, 6.0):
        S, _ = I.prim_block(0, s1.alpha, s1.coef, 0, s1.alpha, s1.coef, np.array([[R, 0, 0]]))
        zr = s1.zeta * R
        exact = math.exp(-zr) * (1 + zr + zr * zr / 3.0)
        assert abs(S[0, 0, 0] - exact) < 2e-4


def test_onsite_identity_and_spd(params):
    for z in (1, 6, 7, 8):
        e = I.element_basis(params, z)
        assert np.max(np.abs(I.onsite_block(params, z) - np.eye(e.nao))) < 1e-14
    s = w.water_cluster_cube()
    S = I.overlap(params, s.Z, s.xyz)
    assert np.max(np.abs(S - S.T)) < 1e-15
    np.linalg.cholesky(S)


def test_overlap_derivative_fd(params):
    R = np.array([[1.1, 0.4, -2.0]])
    h = 1e-5
    for za, zb in [(8, 1), (6, 6)]:
        S, dS = I.pair_blocks(params, za, zb, R)
        for k in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[0, k] += h
            Rm[0, k] -= h
            fd = (I.pair_blocks(params, za, zb, Rp)[0] - I.pair_blocks(params, za, zb, Rm)[0]) / (2 * h)
            assert np.max(np.abs(fd[0] - dS[0, k])) < 1e-9


def test_gamma_limits(params):
    eta_s, eta_t = 0.4, 0.6
    # on-site: the harmonic mean of the two shell hardnesses
    assert abs(X.gamma_matrix(params, 0.0, eta_s, eta_t) - 2 / (1 / eta_s + 1 / eta_t)) < 1e-15
    # long range: bare Coulomb 1/R
    R = 1.0e6
    assert abs(X.gamma_matrix(params, R, eta_s, eta_t) * R - 1.0) < 1e-8
    # derivative
    h = 1e-6
    for R in (0.7, 2.5, 9.0):
        fd = (X.gamma_matrix(params, R + h, eta_s, eta_t) - X.gamma_matrix(params, R - h, eta_s, eta_t)) / (2 * h)
        assert abs(fd - X.gamma_deriv(params, R, eta_s, eta_t)) < 1e-9


def test_cn_closed_forms(params):
    # two atoms at R = k2 (Rcov_A + Rcov_B): the counting function is exactly 1/2
    rc = params.element(6)["rcov"] + params.element(1)["rcov"]
    R = params.k2 * rc
    Z = np.array([6, 1])
    xyz = np.array([[0.0, 0.0, 0.0], [R, 0.0, 0.0]])
    cn = X.coordination_numbers(params, Z, xyz)
    assert np.allclose(cn, 0.5, atol=1e-15)
    # isolated atom
    assert X.coordination_numbers(params, np.array([8]), np.zeros((1, 3)))[0] == 0.0
    # gradient of sum_A F_A CN_A vs central differences
    s = w.water_cluster_cube().subset([0, 1])
    rng = np.random.default_rng(3)
    Fw = rng.normal(size=s.n_atoms)
    g = X.cn_gradient(params, s.Z, s.xyz, Fw)
    h = 1e-5
    for A in range(s.n_atoms):
        for k in range(3):
            xp, xm = s.xyz.copy(), s.xyz.copy()
            xp[A, k] += h
            xm[A, k] -= h
            fd = (Fw @ X.coordination_numbers(params, s.Z, xp) - Fw @ X.coordination_numbers(params, s.Z, xm)) / (2 * h)
            assert abs(fd - g[A, k]) < 1e-8


def test_fermi_entropy_half_filled(params):
    # one electron in a spin-degenerate level far below the next: f = 1/2,
    # -T S = -2 kT ln 2
    eps = np.array([-0.5, 0.3])
    occ, _ = X.fermi_occupations(eps, 1.0, params.kT)
    assert abs(occ[0] - 1.0) < 1e-12 and occ[1] < 1e-100
    assert abs(X.minus_TS(params.kT, occ) + 2 * params.kT * math.log(2.0)) < 1e-15
    # integer occupations carry no entropy
    occ, _ = X.fermi_occupations(np.array([-0.5, -0.4, 0.3]), 4.0, params.kT)
    assert abs(X.minus_TS(params.kT, occ)) < 1e-15
