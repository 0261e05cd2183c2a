"""Molecular dynamics through the C ABI (fx_md_verlet, fx_set_coordinates)
against the oracle's velocity Verlet on the oracle's FMO surface, plus the
integrator's energy conservation on the GPU surface."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w
from oracle import fmo as F
from oracle import md as M

A2B = w.ANGSTROM_TO_BOHR
KB_AU = 3.166811563e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2606_28022_amd import FmoXtb
    return FmoXtb


def _velocities(s, T, seed):
    m = M.masses_au(s.Z)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(s.n_atoms, 3)) * np.sqrt(KB_AU * T / m)[:, None]
    return v - (m[:, None] * v).sum(0) / m.sum()     # no net momentum


def test_md_matches_oracle(lib, params):
    """Three velocity Verlet steps of four waters (FMO2, 4 A lists rebuilt at
    every step, warm-started charges): positions, velocities and energies
    equal the oracle's trajectory."""
    _say("MD 4 waters vs oracle")
    s = w.water_cluster_cube().subset([0, 1, 2, 3])
    m = M.masses_au(s.Z)
    v0 = _velocities(s, 300.0, 3)
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    x, v, ep, ek = c.md_verlet(3, 10.0, m, s.xyz, v0)
    xo, vo, epo, eko = M.velocity_verlet(M.fmo_energy_grad(s, params, 4 * A2B), s.xyz, v0, m, 10.0, 3)
    assert np.max(np.abs(x - xo)) < 1e-9
    assert np.max(np.abs(v - vo)) < 1e-9
    assert np.max(np.abs(ep - epo)) < 1e-8
    assert np.max(np.abs(ek - eko)) < 1e-10
    # the context holds the last geometry and its results
    assert np.max(np.abs(c.gradient() - M.fmo_energy_grad(s, params, 4 * A2B)(xo)[1])) < 1e-7


def test_md_energy_conservation(lib):
    """Eight waters with every pair an SCC dimer (no list changes): the total
    energy is conserved to second order in the step."""
    _say("MD energy conservation 8 waters")
    s = w.water_cluster_cube()
    m = M.masses_au(s.Z)
    v0 = _velocities(s, 300.0, 4)
    err = []
    for dt, n in ((4.0, 20), (2.0, 40)):
        c = lib()
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
        c.set_options(cutoff_bohr=1e3)
        _, _, ep, ek = c.md_verlet(n, dt, m, s.xyz, v0)
        e = ep + ek
        err.append(np.max(np.abs(e - e[0])))
        assert np.all(np.isfinite(e))
    assert err[1] < err[0] and 2.5 < err[0] / err[1] < 6.0, err


def test_set_coordinates_equals_set_system(lib, params):
    _say("set_coordinates")
    s = w.water_cluster_cube().subset([0, 1, 2])
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.run()
    q = c.charges()
    xyz2 = s.xyz + 0.01
    c.set_coordinates(xyz2)
    c.set_options(guess=2)
    c.set_guess(q)
    r = c.run()
    d = lib()
    d.set_system(s.Z, xyz2, s.frag, s.frag_charge)
    assert abs(r["e_total"] - d.run()["e_total"]) < 1e-9
    from paper_2606_28022_amd.binding import FxError
    with pytest.raises(FxError):
        c.md_verlet(2, -1.0, M.masses_au(s.Z), s.xyz, np.zeros_like(s.xyz))
    with pytest.raises(FxError):
        c.md_verlet(2, 1.0, -M.masses_au(s.Z), s.xyz, np.zeros_like(s.xyz))


def test_warm_clusters_same_fixed_point(lib):
    """Dimers started from the previous geometry's converged solution reach
    the same energy and gradient as a cold start, in fewer SCC iterations;
    fx_set_system forgets the saved solution."""
    _say("warm clusters 8 waters")
    s = w.water_cluster_cube()
    rng = np.random.default_rng(11)
    xyz2 = s.xyz + 0.02 * rng.normal(size=s.xyz.shape)
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(warm_clusters=1)
    r0 = c.run()
    assert r0["warm_dimers"] == 0
    c.set_coordinates(xyz2)
    rw = c.run()
    gw = c.gradient()
    d = lib()
    d.set_system(s.Z, xyz2, s.frag, s.frag_charge)
    rc = d.run()
    n_scc = d.get_counts().n_scc_pairs
    assert n_scc > 0 and rw["warm_dimers"] == n_scc
    assert abs(rw["e_total"] - rc["e_total"]) < 1e-9
    assert np.max(np.abs(gw - d.gradient())) < 1e-7
    assert rw["iters_dimer"] < rc["iters_dimer"], (rw["iters_dimer"], rc["iters_dimer"])
    c.set_system(s.Z, xyz2, s.frag, s.frag_charge)
    assert c.run()["warm_dimers"] == 0
