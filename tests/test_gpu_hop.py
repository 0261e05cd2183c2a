"""Covalent fragmentation (hybrid-orbital projectors) on the GPU vs the FP64
oracle, through the C ABI: alanine helices, one residue per fragment, CA-C
bonds cut (section "Covalent bond fragmentation").  Energies to 1e-8 Eh per
fragment term; charges (ghost shells included, after the real ones) to 1e-8.
"""

import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w
from oracle import fmo as F

A2B = w.ANGSTROM_TO_BOHR
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _gpu(s, order=2, **opt):
    from paper_2606_28022_amd import FmoXtb
    c = FmoXtb()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=s.bonds)
    opt.setdefault("want_gradient", 0)
    c.set_options(order=order, **opt)
    r = c.run()
    return r, c


def test_hop_two_fragments(params):
    _say("HOP ala2 FMO2")
    s = w.alanine_helix(2)
    r, c = _gpu(s)
    ro = F.fmo(s, params, 4 * A2B, order=2)
    assert abs(r["e_total"] - ro.E) < 1e-8
    em, ds, de, _ = c.energies()
    assert np.max(np.abs(em - ro.E_mono)) < 1e-8
    q = c.charges()
    assert q.shape == ro.q.shape
    assert np.max(np.abs(q - ro.q)) < 1e-8


def test_hop_ala4_fmo3(params):
    _say("HOP ala4 FMO3")
    ref = _golden("ala4_fmo3")
    s = w.alanine_helix(4)
    r, c = _gpu(s, order=3)
    em, ds, de, dt = c.energies()
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert np.max(np.abs(dt - np.array(ref["dE_tri"]))) < 1e-8
    assert abs(r["e_fmo2"] - ref["E_fmo2"]) < 1e-8 * s.n_frag
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag
    assert np.max(np.abs(c.charges() - np.array(ref["q"]))) < 1e-8


def test_hop_ala10(params):
    _say("HOP ala10 FMO2")
    ref = _golden("ala10")
    s = w.alanine_helix(10)
    r, c = _gpu(s)
    em, ds, de, _ = c.energies()
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert np.max(np.abs(de - np.array(ref["dE_esd"]))) < 1e-9
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag


@pytest.mark.parametrize("name", ["ala20", "ala40", "ala100"])
def test_hop_helices_vs_oracle(name):
    """Helices of the streaming workload (20, 40 and 100 residues, one per
    fragment, every CA-C bond but the last cut) against oracle goldens: every
    fragment and SCC dimer energy within 1e-8 Eh, ES-DIM energies within
    1e-9 Eh, shell charges (ghosts included) within 1e-8 e.  Both sides
    converge to 1e-9 in the charges, the floor that the 1e6 Eh projector
    leaves in FP64."""
    _say(f"HOP {name} FMO2")
    ref = _golden(name)
    s = w.alanine_helix(int(name[3:]))
    r, c = _gpu(s, scc_tol=1e-9, macro_tol=1e-9, energy_tol=1e-10)
    em, ds, de, _ = c.energies()
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert np.max(np.abs(de - np.array(ref["dE_esd"]))) < 1e-9
    assert np.max(np.abs(c.charges() - np.array(ref["q"]))) < 1e-8
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag


@pytest.mark.parametrize("n_res", [2, 4])
def test_hop_gradient_vs_oracle(params, n_res):
    """FMO2 gradient with cut bonds (section "FMO-xTB HOP gradient"): the
    GPU against the oracle's analytic gradient (pinned by central differences
    of the energy plus the projector term in the CPU tests), per component
    within 1e-7 Eh/bohr, with zero net force and torque.  Ala2 heals its bond
    in the dimer; Ala4 also has dimers with a detached atom and a ghost."""
    _say(f"HOP gradient ala{n_res}")
    s = w.alanine_helix(n_res)
    r, c = _gpu(s, scc_tol=1e-9, macro_tol=1e-9, energy_tol=1e-10, want_gradient=1)
    g = c.gradient()
    ro = F.fmo(s, params, 4 * A2B, order=2, scc_tol=1e-9, macro_tol=1e-9, scc_etol=1e-10)
    go, _ = F.fmo_gradient(s, params, ro)
    assert abs(r["e_total"] - ro.E) < 1e-8 * s.n_frag
    assert np.max(np.abs(g.sum(0))) < 1e-8
    assert np.max(np.abs(np.cross(s.xyz, g).sum(0))) < 1e-6
    assert np.max(np.abs(g - go)) < 1e-7, np.max(np.abs(g - go))


def test_hop_gradient_ala10_golden():
    """Ten fragments, nine cut bonds.  The projector term of the gradient
    (section "FMO-xTB HOP gradient") scales rounding-level errors of the
    occupied orbitals in the projector directions by V_HOP = 1e6 Eh, so two
    FP64 computations that differ only in the order of their Jacobi
    rotations, each converged to 3e-11 in the charges, give gradients up to
    about 9e-8 Eh/bohr apart (tighter SCC tolerances change either by less
    than 4e-9).  The bound is 2e-7: twice that floor."""
    _say("HOP gradient ala10")
    ref = _golden("ala10")
    s = w.alanine_helix(10)
    r, c = _gpu(s, scc_tol=1e-9, macro_tol=1e-9, energy_tol=1e-10, want_gradient=1)
    g = c.gradient()
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag
    assert np.max(np.abs(g - np.array(ref["grad"]))) < 2e-7, np.max(np.abs(g - np.array(ref["grad"])))


def test_hop_fmo3_gradient_unsupported():
    from paper_2606_28022_amd import FmoXtb
    from paper_2606_28022_amd.binding import FxError
    s = w.alanine_helix(3)
    c = FmoXtb()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=s.bonds)
    c.set_options(want_gradient=1, order=3)
    with pytest.raises(FxError):
        c.run()


def test_hop_invalid_bonds():
    from paper_2606_28022_amd import FmoXtb
    from paper_2606_28022_amd.binding import FxError
    s = w.alanine_helix(2)
    c = FmoXtb()
    bad = s.bonds.copy()
    bad[0, 1] = bad[0, 0] + 1          # both ends in one fragment
    with pytest.raises(FxError):
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=bad)
    bad = s.bonds.copy()
    bad[0, 0] = s.n_atoms + 5          # out of range
    with pytest.raises(FxError):
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=bad)


def test_hop_set_coordinates_matches_fresh_context():
    """A context that keeps its cluster tables across runs (same clusters
    after fx_set_coordinates) recomputes the projector bond directions: Ala4
    with every atom displaced gives the energies and gradient of a fresh
    context at the new geometry, bit for bit."""
    from paper_2606_28022_amd import FmoXtb
    _say("HOP ala4: set_coordinates vs fresh context")
    s = w.alanine_helix(4)
    rng = np.random.Generator(np.random.PCG64(7))
    x1 = s.xyz + rng.normal(scale=0.02, size=s.xyz.shape)
    c = FmoXtb()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=s.bonds)
    c.set_options(want_gradient=1, scc_tol=1e-9, macro_tol=1e-9, energy_tol=1e-10)
    c.run()
    c.set_coordinates(x1)
    c.build_lists()
    r1 = c.run()
    f = FmoXtb()
    f.set_system(s.Z, x1, s.frag, s.frag_charge, bonds=s.bonds)
    f.set_options(want_gradient=1, scc_tol=1e-9, macro_tol=1e-9, energy_tol=1e-10)
    r2 = f.run()
    assert r1["e_total"] == r2["e_total"]
    for a, b in zip(c.energies(), f.energies()):
        assert np.array_equal(a, b)
    assert np.array_equal(c.gradient(), f.gradient())
