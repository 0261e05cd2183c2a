"""Pins of the oracle's single-system SCC against the mathematics.

* the generalized eigensolve satisfies F C = S C eps and C^T S C = 1;
* the converged density is idempotent (P S P = 2 P), carries N_el electrons
  and the shell charges sum to minus the net charge;
* the fixed point does not depend on the starting charges;
* closed-form single-atom cases (H-, H+, H) of the energy expression;
* two far-apart ions interact through the bare Coulomb law Q1 Q2 / R, which
  fixes the factor 1/2 of the second-order term;
* the analytic gradient of the energy matches central differences, and the
  energy is invariant under rigid translation and rotation.
"""

import math

import numpy as np

from oracle import xtb as X
from oracle import fmo as F
import workloads as w


def _sys(params, s):
    cn = X.coordination_numbers(params, s.Z, s.xyz)
    return X.XtbSystem(params, s.Z, s.xyz, cn, charge=int(s.frag_charge.sum()))


def test_eigensolve_and_density(params):
    s = w.water_cluster_cube().subset([0, 1, 2])
    sx = _sys(params, s)
    r = X.scc(sx)
    assert r.converged
    F_ = sx.fock(r.q, np.zeros(sx.nsh))
    assert np.max(np.abs(F_ @ r.C - sx.S @ r.C * r.eps)) < 1e-10
    assert np.max(np.abs(r.C.T @ sx.S @ r.C - np.eye(sx.nao))) < 1e-12
    assert np.max(np.abs(r.P @ sx.S @ r.P - 2 * r.P)) < 1e-10
    assert abs(np.trace(r.P @ sx.S) - sx.nel) < 1e-10
    assert abs(r.q.sum() + 0.0) < 1e-10


def test_fixed_point_independent_of_start(params):
    s = w.water_cluster_cube().subset([0, 1])
    sx = _sys(params, s)
    r0 = X.scc(sx, tol=1e-12)
    rng = np.random.default_rng(7)
    g = rng.normal(scale=0.2, size=sx.nsh)
    g -= g.mean()
    r1 = X.scc(sx, q_guess=g, tol=1e-12, beta=0.3, memory=4)
    assert np.max(np.abs(r0.q - r1.q)) < 1e-9
    assert abs(r0.e_int - r1.e_int) < 1e-10


def _atom(params, Z, charge):
    s = w.System("atom", np.array([Z], np.int32), np.zeros((1, 3)),
                 np.zeros(1, np.int32), np.array([charge], np.int32))
    sx = _sys(params, s)
    return sx, X.scc(sx, tol=1e-12)


def test_single_atom_closed_forms(params):
    e = params.element(1)
    h1s = e["shells"][0]["level"]
    eta1 = (1 + e["shells"][0]["kappa"]) * e["eta"]
    G = e["Gamma"]
    # H-: two electrons in 1s, dq_1s = +1
    _, r = _atom(params, 1, -1)
    assert abs(r.q[0] - 1.0) < 1e-12
    assert abs(r.e_int - (2 * h1s + 0.5 * eta1 - G / 3.0)) < 1e-12
    # H+: empty, dq_1s = -1
    _, r = _atom(params, 1, +1)
    assert abs(r.e_int - (0.5 * eta1 + G / 3.0)) < 1e-12
    # neutral H: half-filled 1s, entropy -2 kT ln 2
    _, r = _atom(params, 1, 0)
    assert abs(r.e_int - (h1s - 2 * params.kT * math.log(2.0))) < 1e-12


def test_separated_ions_coulomb(params):
    """E(AB) - E(A) - E(B) -> Q_A Q_B / R for two cations far apart (two
    cations cannot lower their energy by transferring charge)."""
    Zw, Xw = w.geometry.water_molecule()
    h3o = np.concatenate([Xw, [[0.0, 0.0, -0.98]]]) * w.ANGSTROM_TO_BOHR
    rot = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    Zb = np.array([8, 1, 1, 1], np.int32)
    res = []
    for R in (60.0, 120.0):
        xyz = np.concatenate([h3o, h3o @ rot.T + np.array([R, 0, 0])])
        s = w.System("ions", np.concatenate([Zb, Zb]), xyz,
                     np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32), np.array([1, 1], np.int32))
        eab = X.scc(_sys(params, s), tol=1e-12).e_int
        ea = X.scc(_sys(params, s.subset([0])), tol=1e-12).e_int
        eb = X.scc(_sys(params, s.subset([1])), tol=1e-12).e_int
        res.append((R, eab - ea - eb))
    for R, de in res:
        # electron-excess charges -1 and -1: +1/R
        assert abs(de * R - 1.0) < 2e-3, (R, de * R)
    # the residual (polarisation) decays faster than 1/R
    assert abs(res[1][1] * res[1][0] - 1.0) < abs(res[0][1] * res[0][0] - 1.0)


def test_xtb_gradient_fd_and_invariance(params):
    s = w.water_cluster_cube().subset([0, 1])
    e, g = F.xtb_gradient(s, params)
    h = 1e-4
    for A in range(s.n_atoms):
        for k in range(3):
            sp = w.System(s.name, s.Z, s.xyz.copy(), s.frag, s.frag_charge)
            sm = w.System(s.name, s.Z, s.xyz.copy(), s.frag, s.frag_charge)
            sp.xyz[A, k] += h
            sm.xyz[A, k] -= h
            fd = (F.xtb_energy(sp, params)[0] - F.xtb_energy(sm, params)[0]) / (2 * h)
            assert abs(fd - g[A, k]) < 2e-8
    assert np.max(np.abs(g.sum(0))) < 1e-10
    assert np.max(np.abs(np.cross(s.xyz, g).sum(0))) < 1e-9
    # rigid motion
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    s2 = w.System(s.name, s.Z, s.xyz @ Rz.T + np.array([3.0, -1.0, 2.0]), s.frag, s.frag_charge)
    assert abs(F.xtb_energy(s2, params)[0] - e) < 1e-10
