"""GPU FMO2 analytic gradient vs the FP64 oracle (whose gradient is pinned by
central finite differences in the CPU tests), through the C ABI.

Tolerance: 1e-7 Eh/bohr per component for the FP64 path (both sides solve
the SCC to 1e-10 in the charges; the gradient error is first order in the
charge error times O(1) derivative integrals).  Properties checked at full
size: zero net force and torque.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w
from oracle import fmo as F

A2B = w.ANGSTROM_TO_BOHR


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2606_28022_amd import FmoXtb
    return FmoXtb


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _gpu_grad(lib, s, **opt):
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=1, **opt)
    r = c.run()
    return r, c.gradient(), c


@pytest.mark.parametrize("nfrag,cut_ang", [(4, 4.0), (8, 4.0), (8, 60.0)])
def test_fmo2_gradient_vs_oracle(lib, params, nfrag, cut_ang):
    _say(f"gradient C1[{nfrag}] cutoff {cut_ang} A")
    s = w.water_cluster_cube()
    s = s.subset(list(range(nfrag))) if nfrag < s.n_frag else s
    r, g, _ = _gpu_grad(lib, s, cutoff_bohr=cut_ang * A2B)
    ro = F.fmo(s, params, cut_ang * A2B)
    go, parts = F.fmo2_gradient(s, params, ro)
    assert abs(r["e_total"] - ro.E) < 1e-8
    assert np.max(np.abs(g - go)) < 1e-7, np.max(np.abs(g - go))


def test_fmo2_gradient_without_response(lib, params):
    s = w.water_cluster_cube().subset([0, 1, 2, 3, 4])
    r, g, _ = _gpu_grad(lib, s, want_response=0)
    ro = F.fmo(s, params, 4 * A2B)
    go, _ = F.fmo2_gradient(s, params, ro, with_response=False)
    assert np.max(np.abs(g - go)) < 1e-7


def test_gradient_pentacene_cluster(lib, params):
    """Six pentacene molecules (n = 116 / 232 AOs) against stored oracle values
    (tests/golden/pentacene6.json, written by tests/golden/make_golden.py)."""
    _say("gradient pentacene 6 molecules")
    ref = _golden("pentacene6")
    s = w.pentacene_crystal(reps=(2, 2, 1)).subset(list(range(6)))
    r, g, c = _gpu_grad(lib, s)
    em, ds, de, _ = c.energies()
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag
    assert np.max(np.abs(g - np.array(ref["grad"]))) < 1e-7


def test_gradient_invariances_droplet(lib):
    """Zero net force and torque for the 1024-molecule droplet."""
    _say("gradient droplet 1024")
    s = w.water_droplet()
    r, g, _ = _gpu_grad(lib, s)
    assert np.max(np.abs(g.sum(0))) < 1e-8
    assert np.max(np.abs(np.cross(s.xyz, g).sum(0))) < 1e-6


def test_gradient_deterministic(lib):
    s = w.water_cluster_cube()
    _, g1, c = _gpu_grad(lib, s)
    c.run()
    g2 = c.gradient()
    assert np.array_equal(g1, g2)
