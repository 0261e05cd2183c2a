"""GPU library vs the FP64 oracle, through the C ABI.

Tolerances: integer lists bit-exact; S/H0, CN and the embedding field to
1e-12 (pure FP64 arithmetic, different summation order); fragment energies
within 1e-8 Eh each and charges within 1e-8 e (both sides converge the SCC
to 1e-10 in the charges, so the energies, variational in the density, agree
to second order).
"""

import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w
from oracle import fmo as F
from oracle import xtb as X

A2B = w.ANGSTROM_TO_BOHR


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2606_28022_amd import FmoXtb
    return FmoXtb


def _ctx(lib, s, **opt):
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    if opt:
        c.set_options(**opt)
    return c


@pytest.fixture(scope="module")
def c1():
    return w.water_cluster_cube()


@pytest.fixture(scope="module")
def c4():
    return w.pentacene_crystal()


def test_lists_bit_exact_c1(lib, params, c1):
    _say("lists C1")
    c = _ctx(lib, c1, order=3)
    scc, esd, tri = c.build_lists()
    o_scc, o_esd, o_tri = F.build_lists(c1, 4 * A2B, order=3)
    assert np.array_equal(scc, o_scc) and np.array_equal(esd, o_esd) and np.array_equal(tri, o_tri)


def test_lists_bit_exact_pentacene(lib, params, c4):
    _say("lists pentacene 23760 atoms")
    c = _ctx(lib, c4)
    scc, esd, _ = c.build_lists()
    # oracle classification of every pair from its closest contact
    o_scc, o_esd, _ = F.build_lists(c4, 4 * A2B, order=2)
    assert np.array_equal(scc, o_scc)
    assert np.array_equal(esd, o_esd)


def test_cn_full_size(lib, params, c4):
    _say("cn pentacene")
    c = _ctx(lib, c4)
    cn = c.compute_cn()
    ref = X.coordination_numbers(params, c4.Z, c4.xyz)
    assert np.max(np.abs(cn - ref)) < 1e-12


@pytest.mark.parametrize("frags", [(0,), (1, 2), (0, 3, 5)])
def test_cluster_matrices_water(lib, params, c1, frags):
    c = _ctx(lib, c1)
    S, H = c.cluster_matrices(frags)
    cn = X.coordination_numbers(params, c1.Z, c1.xyz)
    atoms = np.concatenate([np.where(c1.frag == I)[0] for I in frags])
    sx = X.XtbSystem(params, c1.Z[atoms], c1.xyz[atoms], cn[atoms])
    assert np.max(np.abs(S - sx.S)) < 1e-13
    assert np.max(np.abs(H - sx.H0)) < 1e-13


def test_cluster_matrices_pentacene_dimer(lib, params, c4):
    _say("S/H0 pentacene dimer")
    c = _ctx(lib, c4)
    scc, _, _ = c.build_lists()
    I, J = scc[len(scc) // 2]
    S, H = c.cluster_matrices((I, J))
    cn = X.coordination_numbers(params, c4.Z, c4.xyz)
    atoms = np.concatenate([np.where(c4.frag == I)[0], np.where(c4.frag == J)[0]])
    sx = X.XtbSystem(params, c4.Z[atoms], c4.xyz[atoms], cn[atoms])
    assert S.shape == (232, 232)
    assert np.max(np.abs(S - sx.S)) < 1e-13
    assert np.max(np.abs(H - sx.H0)) < 1e-13


@pytest.mark.parametrize("nmol", [256, 250, 5])
def test_embedding_field(lib, params, nmol):
    """Whole 64-atom blocks (768 atoms), a ragged last block (750 atoms) and
    a single partial block (15 atoms, the diagonal block only)."""
    _say(f"embedding field droplet {nmol}")
    s = w.water_droplet(nmol, radius=12.5 * (nmol / 256) ** (1 / 3), seed=21)
    c = _ctx(lib, s)
    rng = np.random.Generator(np.random.PCG64(5))
    q = rng.normal(scale=0.3, size=c.n_shells)
    phi = c.embedding_field(q)
    sh = F.Shells(params, s)
    ref = sh.potential(np.arange(sh.n), q, lambda a, b: sh.frag[a] == sh.frag[b])
    assert np.max(np.abs(phi - ref)) < 1e-11


@pytest.mark.parametrize("sizes", [[1, 2, 3, 8, 16], [31, 64, 76], [116, 152], [232]])
def test_eigh_batched(lib, sizes):
    _say(f"eigh {sizes}")
    rng = np.random.Generator(np.random.PCG64(sum(sizes)))
    mats = []
    for n in sizes:
        a = rng.normal(size=(n, n))
        a = 0.5 * (a + a.T)
        if n > 3:
            a[0, 0] = a[1, 1]  # near-degenerate start
        mats.append(a)
    c = lib()
    out = c.eigh_batched(mats)
    for a, (wv, V) in zip(mats, out):
        n = a.shape[0]
        ref = np.linalg.eigvalsh(a)
        assert np.max(np.abs(np.sort(wv) - ref)) < 1e-12 * max(1.0, np.abs(ref).max()) * n
        assert np.max(np.abs(V @ V.T - np.eye(n))) < 1e-12 * n
        assert np.max(np.abs(a @ V.T - V.T * wv)) < 1e-11 * n


def _compare_fmo(c, r_or, nscc, tol_e=1e-8):
    em, ds, de, dt = c.energies()
    assert np.max(np.abs(em - r_or.E_mono)) < tol_e
    if nscc:
        assert np.max(np.abs(ds - r_or.dE_scc)) < tol_e
    if len(r_or.dE_esd):
        assert np.max(np.abs(de - r_or.dE_esd)) < tol_e
    assert np.max(np.abs(c.charges() - r_or.q)) < 1e-8


def test_fmo2_energy_c1_all_scc(lib, params, c1):
    """Config: 8 waters, every pair a full SCC dimer."""
    _say("FMO2 C1 all-SCC")
    c = _ctx(lib, c1, cutoff_bohr=1e3, want_gradient=0)
    r = c.run()
    ro = F.fmo(c1, params, 1e3)
    assert r["solves_dimer"] == 28
    _compare_fmo(c, ro, 28)
    assert abs(r["e_total"] - ro.E) < 1e-8


def test_fmo2_energy_c1_mixed_pairs(lib, params, c1):
    _say("FMO2 C1 4A cutoff")
    c = _ctx(lib, c1, want_gradient=0)
    r = c.run()
    ro = F.fmo(c1, params, 4 * A2B)
    _compare_fmo(c, ro, len(ro.lists[0]))
    assert abs(r["e_total"] - ro.E) < 1e-8


def test_fmo3_energy_small(lib, params, c1):
    _say("FMO3 C1 subset")
    s = c1.subset([0, 1, 2, 3, 4])
    c = _ctx(lib, s, order=3, cutoff_bohr=6 * A2B, want_gradient=0)
    r = c.run()
    ro = F.fmo(s, params, 6 * A2B, order=3)
    assert r["solves_trimer"] == len(ro.lists[2]) > 0
    em, ds, de, dt = c.energies()
    assert np.max(np.abs(dt - ro.dE_tri)) < 1e-8
    assert abs(r["e_total"] - ro.E) < 1e-8


def test_single_fragment_equals_xtb(lib, params, c1):
    s = c1.subset([2])
    c = _ctx(lib, s, want_gradient=0)
    r = c.run()
    assert abs(r["e_total"] - F.xtb_energy(s, params)[0]) < 1e-8


def test_plain_loop_matches_batched(lib, params, c1):
    _say("plain vs batched")
    c = _ctx(lib, c1, want_gradient=0)
    rb = c.run()
    qb = c.charges()
    c.set_options(schedule=1)
    rp = c.run()
    assert abs(rb["e_total"] - rp["e_total"]) < 1e-9
    assert np.max(np.abs(qb - c.charges())) < 1e-9


def test_error_paths(lib, c1):
    from paper_2606_28022_amd.binding import FxError, FX_E_INVALID, FX_E_UNSUPPORTED, FX_E_STATE, FX_E_NOCONV
    c = lib()
    with pytest.raises(FxError) as e:
        c.run()
    assert e.value.code == FX_E_STATE
    xyz = c1.xyz.copy()
    xyz[3, 1] = np.nan
    with pytest.raises(FxError) as e:
        c.set_system(c1.Z, xyz, c1.frag, c1.frag_charge)
    assert e.value.code == FX_E_INVALID
    Z = c1.Z.copy()
    Z[0] = 26
    with pytest.raises(FxError) as e:
        c.set_system(Z, c1.xyz, c1.frag, c1.frag_charge)
    assert e.value.code == FX_E_UNSUPPORTED
    xyz = c1.xyz.copy()
    xyz[1] = xyz[0] + 0.1
    with pytest.raises(FxError) as e:
        c.set_system(c1.Z, xyz, c1.frag, c1.frag_charge)
    assert e.value.code == FX_E_INVALID
    c.set_system(c1.Z, c1.xyz, c1.frag, c1.frag_charge)
    c.set_options(max_iter=1, want_gradient=0, scc_retry=0)
    with pytest.raises(FxError) as e:
        c.run()
    assert e.value.code == FX_E_NOCONV
    with pytest.raises(FxError) as e:
        c.set_options(scc_retry=2)
    assert e.value.code == FX_E_INVALID


@pytest.mark.parametrize("which", ["c1", "pentacene4"])
def test_graph_schedule_matches_batched(lib, which):
    """FX_BATCHED_GRAPH replays one captured SCC iteration over all systems
    of a solve; converged systems skip themselves on the device.  Energies
    and charges equal the eagerly launched schedule bit for bit, also on a
    second run of the same context (new capture, new replays)."""
    _say(f"graph schedule {which}")
    s = w.water_cluster_cube() if which == "c1" else w.pentacene_crystal(reps=(2, 2, 1)).subset([0, 1, 2, 3])
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=0, schedule=0)
    r0 = c.run()
    e0 = c.energies()
    q0 = c.charges()
    c.set_options(schedule=2)
    for rep in range(2):
        r1 = c.run()
        e1 = c.energies()
        assert r1["e_total"] == r0["e_total"]
        for a, b in zip(e0, e1):
            assert np.array_equal(a, b)
        assert np.array_equal(c.charges(), q0)
        assert r1["iters_dimer"] == r0["iters_dimer"]


@pytest.mark.parametrize("which", ["c1", "pentacene6", "anthracene5"])
def test_device_driven_matches_host_sync(lib, which):
    """FX_BATCHED compacts the active list on the device and launches each
    SCC iteration without waiting for the last one; FX_BATCHED_HOST_SYNC
    compacts on the host after a synchronisation.  Energies, charges,
    iteration counts and the gradient are bitwise identical, also on a
    second run of the same context."""
    _say(f"device-driven vs host-synced {which}")
    if which == "c1":
        s, order = w.water_cluster_cube(), 2
    elif which == "pentacene6":
        s, order = w.pentacene_crystal(reps=(2, 2, 1)).subset([0, 1, 2, 3, 4, 5]), 2
    else:
        s, order = w.anthracene_crystal(reps=(2, 2, 1), seed=3).subset([0, 1, 2, 3, 4]), 3
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=1, order=order, schedule=3)
    r0 = c.run()
    e0, q0, g0 = c.energies(), c.charges(), c.gradient()
    c.set_options(schedule=0)
    for rep in range(2):
        r1 = c.run()
        assert r1["e_total"] == r0["e_total"]
        for a, b in zip(e0, c.energies()):
            assert np.array_equal(a, b)
        assert np.array_equal(c.charges(), q0)
        assert np.array_equal(c.gradient(), g0)
        for k in ("iters_mono", "iters_dimer", "iters_trimer", "macro_iter"):
            assert r1[k] == r0[k], k


def test_rotation_kernel_shapes_bitwise(lib):
    """The rotation kernel's launch shapes (work-group size; one work-group
    per system or the persistent work-queue grid) that the tuner chooses
    among give bitwise identical energies, charges and gradients (six
    pentacenes: 232-AO dimers with the FP32 working matrix, 116-AO monomers
    with the FP64 one)."""
    import os
    s = w.pentacene_crystal(reps=(2, 2, 1)).subset([0, 1, 2, 3, 4, 5])
    out = {}
    for t, p in [(0, -1), (256, 0), (512, 1), (768, 0), (1024, 1)]:
        _say(f"rotation kernel {t} threads, persistent {p}")
        env = {"FX_JACOBI_ROT_THREADS": str(t), "FX_JACOBI_ROT_PERSISTENT": str(p)} if t else {}
        old = {k: os.environ.get(k) for k in ("FX_JACOBI_ROT_THREADS", "FX_JACOBI_ROT_PERSISTENT")}
        os.environ.update(env)
        try:
            c = lib()
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
        c.set_options(want_gradient=1)
        r = c.run()
        out[(t, p)] = (r["e_total"], c.energies(), c.charges(), c.gradient(), r["iters_dimer"])
    ref = out[(0, -1)]
    for k, v in out.items():
        assert v[0] == ref[0], k
        for a, b in zip(v[1], ref[1]):
            assert np.array_equal(a, b), k
        assert np.array_equal(v[2], ref[2]), k
        assert np.array_equal(v[3], ref[3]), k
        assert v[4] == ref[4], k


@pytest.mark.parametrize("which", ["c1", "pentacene6"])
def test_mixed_precision_matches_fp64(lib, which):
    """FX_MIXED (FP32 Fock build and FP32 matrix-core products while an SCC
    residual exceeds 1e-5, FP32 field passes in the early monomer steps and
    response sweeps; FP64 basis, rotation angles, final iterations and
    energies) reaches the FP64 results within the FP64 tolerances: fragment
    energies 1e-8 Eh, gradient 1e-7 Eh/bohr."""
    _say(f"mixed precision {which}")
    s = w.water_cluster_cube() if which == "c1" else w.pentacene_crystal(reps=(2, 2, 1)).subset(list(range(6)))
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=1, precision=0)
    r0 = c.run()
    e0 = c.energies()
    g0 = c.gradient()
    c.set_options(precision=1)
    r1 = c.run()
    e1 = c.energies()
    g1 = c.gradient()
    assert abs(r1["e_total"] - r0["e_total"]) < 1e-8 * s.n_frag
    for a, b in zip(e0, e1):
        if len(a):
            assert np.max(np.abs(a - b)) < 1e-8
    assert np.max(np.abs(g1 - g0)) < 1e-7
    # the FP32 products ran for the pentacene systems (more than 32 AOs),
    # never for the waters
    assert (r1["iters_fp32"] > 0) == (which != "c1")
    assert r0["iters_fp32"] == 0


def test_mixed_precision_vs_oracle(lib):
    """The mixed form against the FP64 oracle (tests/golden/pentacene6.json):
    total energy within 1e-6 Eh and gradient within 1e-5 Eh/bohr (the
    tolerances of the mixed form), and in fact within the FP64 ones (1e-8 Eh
    per fragment, 1e-7 Eh/bohr), since its last iterations are FP64."""
    _say("mixed precision vs oracle, pentacene 6")
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pentacene6.json")
    with open(path) as f:
        ref = json.load(f)
    s = w.pentacene_crystal(reps=(2, 2, 1)).subset(list(range(6)))
    c = lib()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=1, precision=1)
    r = c.run()
    g = c.gradient()
    em, ds, _, _ = c.energies()
    assert abs(r["e_total"] - ref["E"]) < 1e-6
    assert np.max(np.abs(g - np.array(ref["grad"]))) < 1e-5
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert np.max(np.abs(g - np.array(ref["grad"]))) < 1e-7


def test_user_guess_warm_start(lib, params, c1):
    """FX_GUESS_USER starts the monomer loop from given shell charges (an MD
    step from the previous geometry).  The fixed point does not depend on the
    start: from the converged charges the energy and charges are reproduced
    with fewer monomer iterations; after a 0.001 A displacement of every atom
    the warm-started step equals a cold solve and the oracle there."""
    _say("user guess warm start")
    c = _ctx(lib, c1, want_gradient=1)
    r0 = c.run()
    q0 = c.charges()
    g0 = c.gradient()
    c.set_options(guess=2)
    c.set_guess(q0)
    r1 = c.run()
    assert abs(r1["e_total"] - r0["e_total"]) < 1e-9
    assert np.max(np.abs(c.charges() - q0)) < 1e-9
    assert np.max(np.abs(c.gradient() - g0)) < 1e-8
    assert r1["iters_mono"] < r0["iters_mono"]
    rng = np.random.default_rng(11)
    d = rng.normal(size=c1.xyz.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz2 = c1.xyz + 0.001 * A2B * d
    s2 = w.System(name="displaced", Z=c1.Z, xyz=xyz2, frag=c1.frag, frag_charge=c1.frag_charge)
    c.set_system(s2.Z, s2.xyz, s2.frag, s2.frag_charge)
    c.set_guess(q0)
    rw = c.run()
    qw = c.charges()
    c.set_options(guess=0)
    rc = c.run()
    assert abs(rw["e_total"] - rc["e_total"]) < 1e-9
    assert np.max(np.abs(qw - c.charges())) < 1e-9
    assert rw["iters_mono"] < rc["iters_mono"]
    ro = F.fmo(s2, params, 4 * A2B)
    assert abs(rw["e_total"] - ro.E) < 1e-8
    from paper_2606_28022_amd.binding import FxError
    with pytest.raises((FxError, ValueError)):
        c.set_guess(q0[:-1])


@pytest.mark.parametrize("which", ["c1", "anthracene8", "pentacene"])
def test_lists_vdw_bit_exact(lib, params, c1, c4, which):
    """Van der Waals-scaled selection (section "Computational Details"):
    SCC dimers at 2.0 (r_a + r_b), trimers with two of three pairs at 1.5,
    integer lists equal to the oracle's."""
    _say(f"vdW lists {which}")
    s, order = {"c1": (c1, 3), "anthracene8": (None, 3), "pentacene": (c4, 2)}[which]
    if s is None:
        s = w.anthracene_crystal(reps=(2, 2, 2))
    c = _ctx(lib, s, order=order, selection=1, vdw_dimer=2.0, vdw_trimer=1.5)
    scc, esd, tri = c.build_lists()
    o_scc, o_esd, o_tri = F.build_lists(s, 0.0, order=order, vdw=(F.vdw_radii(s, params), 2.0, 1.5))
    assert np.array_equal(scc, o_scc) and np.array_equal(esd, o_esd) and np.array_equal(tri, o_tri)
    assert len(scc) > 0 and len(esd) > 0 and (order < 3 or len(tri) > 0)
    # the rule differs from the fixed cutoff on these systems
    c.set_options(selection=0)
    assert not np.array_equal(c.build_lists()[0], scc) or which == "c1"


def test_fmo3_energy_vdw_selection(lib, params, c1):
    _say("FMO3 vdW selection")
    s = c1.subset([0, 1, 2, 3, 4])
    lists = F.build_lists(s, 0.0, order=3, vdw=(F.vdw_radii(s, params), 2.0, 1.5))
    assert len(lists[2]) > 0
    c = _ctx(lib, s, order=3, selection=1, want_gradient=0)
    r = c.run()
    ro = F.fmo(s, params, 0.0, order=3, lists=lists)
    assert r["solves_trimer"] == len(lists[2])
    _compare_fmo(c, ro, len(lists[0]))
    assert abs(r["e_total"] - ro.E) < 1e-8


def test_multimolecule_fragments(lib, params, c1):
    """Two waters per fragment (fragments need not be contiguous in the atom
    order): FMO2 energy and gradient, FMO3 energy, against the oracle."""
    _say("two waters per fragment")
    s = c1.grouped(2)
    assert s.n_frag == 4
    c = _ctx(lib, s, want_gradient=1)
    r = c.run()
    ro = F.fmo(s, params, 4 * A2B)
    _compare_fmo(c, ro, len(ro.lists[0]))
    assert abs(r["e_total"] - ro.E) < 1e-8
    go, _ = F.fmo2_gradient(s, params, ro)
    assert np.max(np.abs(c.gradient() - go)) < 1e-7
    c.set_options(order=3, want_gradient=0)
    r3 = c.run()
    ro3 = F.fmo(s, params, 4 * A2B, order=3)
    assert abs(r3["e_total"] - ro3.E) < 1e-8
