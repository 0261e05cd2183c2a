"""GPU FMO3 analytic gradient (section "Extension to FMO3") vs the FP64
oracle, whose FMO3 gradient is pinned by central finite differences and by
the three-fragment limit (xTB of the union) in the CPU tests.

The cases cover SCC pairs shared by several trimers (negative pair weights
s_IJ = 1 - n_T), ES-DIM sub-pairs inside trimers and the van der Waals
selection rule.  Tolerance as for FMO2: 1e-7 Eh/bohr per component.
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


def _run(lib, s, **opt):
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(order=3, want_gradient=1, **opt)
    r = c.run()
    return r, c.gradient(), c


@pytest.mark.parametrize("response", [1, 0])
def test_fmo3_gradient_vs_oracle(lib, params, response):
    _say(f"FMO3 gradient 5 waters, response {response}")
    s = w.water_cluster_cube().subset([0, 2, 3, 5, 6])
    r, g, c = _run(lib, s, cutoff_bohr=5.5 * A2B, want_response=response)
    ro = F.fmo(s, params, 5.5 * A2B, order=3)
    assert r["solves_trimer"] == len(ro.lists[2]) >= 3
    assert abs(r["e_total"] - ro.E) < 1e-8
    go, _ = F.fmo_gradient(s, params, ro, with_response=bool(response))
    assert np.max(np.abs(g - go)) < 1e-7, np.max(np.abs(g - go))


def test_fmo3_gradient_vdw_selection(lib, params):
    _say("FMO3 gradient, van der Waals selection, 8 waters")
    s = w.water_cluster_cube()
    r, g, c = _run(lib, s, selection=1)
    lists = F.build_lists(s, 0.0, order=3, vdw=(F.vdw_radii(s, params), 2.0, 1.5))
    ro = F.fmo(s, params, 0.0, order=3, lists=lists)
    assert r["solves_trimer"] == len(lists[2]) > 0
    assert abs(r["e_total"] - ro.E) < 1e-8
    go, _ = F.fmo_gradient(s, params, ro)
    assert np.max(np.abs(g - go)) < 1e-7, np.max(np.abs(g - go))


def test_fmo3_gradient_three_fragments_is_xtb(lib, params):
    _say("FMO3 gradient, three fragments")
    s = w.water_cluster_cube().subset([1, 2, 4])
    r, g, _ = _run(lib, s, cutoff_bohr=100.0)
    assert r["solves_trimer"] == 1
    e, gx = F.xtb_gradient(s, params)
    assert abs(r["e_total"] - e) < 1e-8
    assert np.max(np.abs(g - gx)) < 1e-7


def test_fmo3_gradient_invariances_anthracene(lib):
    """Zero net force and torque, and bitwise repeatability, for a small
    anthracene crystal (n = 76 / 152 / 228 AOs)."""
    _say("FMO3 gradient anthracene 2x2x2")
    s = w.anthracene_crystal(reps=(2, 2, 2))
    r, g, c = _run(lib, s)
    assert r["solves_trimer"] > 0
    assert np.max(np.abs(g.sum(0))) < 1e-8
    assert np.max(np.abs(np.cross(s.xyz, g).sum(0))) < 1e-7
    c.run()
    assert np.array_equal(c.gradient(), g)


def test_fmo3_anthracene_golden(lib):
    """Five anthracene molecules (n = 76 / 152 / 228 AOs: FP32 working
    matrices, matrix-core products, the corrected FP32 start basis of the
    trimers) against stored oracle values (tests/golden/anthracene5_fmo3.json,
    written by tests/golden/make_golden.py): energies 1e-8 Eh, gradient
    1e-7 Eh/bohr."""
    import json
    import os
    _say("FMO3 anthracene 5 molecules vs stored oracle values")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "anthracene5_fmo3.json")
    with open(path) as f:
        ref = json.load(f)
    s = w.anthracene_crystal(reps=(2, 2, 1)).subset(list(range(5)))
    r, g, c = _run(lib, s, cutoff_bohr=ref["cutoff_bohr"])
    em, ds, de, dt = c.energies()
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert np.max(np.abs(de - np.array(ref["dE_esd"]))) < 1e-8
    assert np.max(np.abs(dt - np.array(ref["dE_tri"]))) < 1e-8
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag
    assert np.max(np.abs(g - np.array(ref["grad"]))) < 1e-7, np.max(np.abs(g - np.array(ref["grad"])))
