"""The split eigensolver in the super-block Jacobi ordering (rotation kernel
with the super-block schedule, k_apply_sb applying each super-pair's 16 x 16
rotation product on the FP64 matrix cores) against the FP64 oracle goldens
and against the circle ordering, through the C ABI.  The ordering is a
different cyclic Jacobi order: the fixed point is the same, so the goldens'
tolerances apply (fragment energies 1e-8 Eh, charges 1e-8, gradient 1e-7
Eh/bohr)."""

import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        ref = json.load(f)
    assert ref.get("macro_converged", False) and ref.get("scc_converged", False), "unconverged golden"
    return ref


def _ctx(order, extra=None):
    """A context created with FX_JACOBI_ORDER=order (read when the context
    is created) and any further variables in extra."""
    from paper_2606_28022_amd import FmoXtb
    env = {"FX_JACOBI_ORDER": str(order)}
    env.update(extra or {})
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return FmoXtb()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("name,builder", [
    ("pentacene6", lambda: w.pentacene_crystal(reps=(2, 2, 1)).subset([0, 1, 2, 3, 4, 5])),
    ("pentacene_3x2x2", lambda: w.pentacene_crystal(reps=(3, 2, 2))),
    ("droplet128", lambda: w.water_droplet(128, radius=9.8, seed=22)),
])
def test_sb_order_vs_oracle_golden(name, builder):
    _say(f"super-block ordering: {name} vs oracle golden")
    ref = _golden(name)
    s = builder()
    c = _ctx(1)
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=1)
    r = c.run()
    em, ds, de, _ = c.energies()
    assert np.max(np.abs(em - np.array(ref["E_mono"]))) < 1e-8
    assert np.max(np.abs(ds - np.array(ref["dE_scc"]))) < 1e-8
    assert np.max(np.abs(de - np.array(ref["dE_esd"]))) < 1e-9
    assert np.max(np.abs(c.charges() - np.array(ref["q"]))) < 1e-8
    assert abs(r["e_total"] - ref["E"]) < 1e-8 * s.n_frag
    if "grad" in ref:
        g = c.gradient()
        assert np.max(np.abs(g - np.array(ref["grad"]))) < 1e-7, np.max(np.abs(g - np.array(ref["grad"])))


@pytest.mark.parametrize("which", ["c1", "anthracene5"])
def test_sb_order_matches_circle(which):
    """FMO2 (8 waters, every pair an SCC dimer) and FMO3 (five anthracenes,
    228-AO trimers): both orderings reach the same energies and gradient."""
    _say(f"super-block vs circle ordering: {which}")
    if which == "c1":
        s, order = w.water_cluster_cube(), 2
    else:
        s, order = w.anthracene_crystal(reps=(2, 2, 1), seed=3).subset([0, 1, 2, 3, 4]), 3
    out = []
    for o in (0, 1):
        c = _ctx(o)
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
        c.set_options(order=order, want_gradient=1)
        r = c.run()
        out.append((r["e_total"], c.energies(), c.gradient()))
    assert abs(out[0][0] - out[1][0]) < 1e-8 * s.n_frag
    for a, b in zip(out[0][1], out[1][1]):
        if len(a):
            assert np.max(np.abs(a - b)) < 1e-8
    assert np.max(np.abs(out[0][2] - out[1][2])) < 1e-7


def test_sb_rotation_kernel_shapes_bitwise():
    """Launch shapes of the rotation kernel in the super-block ordering give
    bitwise identical results (232-AO dimers, FP32 working matrix; 116-AO
    monomers, FP64)."""
    s = w.pentacene_crystal(reps=(2, 2, 1)).subset([0, 1, 2, 3, 4, 5])
    out = {}
    for t, p in [(0, -1), (256, 0), (1024, 1)]:
        _say(f"super-block ordering, rotation kernel {t} threads, persistent {p}")
        extra = {"FX_JACOBI_ROT_THREADS": str(t), "FX_JACOBI_ROT_PERSISTENT": str(p)} if t else {}
        c = _ctx(1, extra)
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
        c.set_options(want_gradient=1)
        r = c.run()
        out[(t, p)] = (r["e_total"], c.charges(), c.gradient(), r["iters_dimer"])
    ref = out[(0, -1)]
    for k, v in out.items():
        assert v[0] == ref[0], k
        assert np.array_equal(v[1], ref[1]), k
        assert np.array_equal(v[2], ref[2]), k
        assert v[3] == ref[3], k


@pytest.mark.parametrize("sizes", [[1, 2, 3, 8, 16], [31, 64, 76], [116, 152], [232, 240, 256]])
def test_sb_eigh_batched(sizes):
    _say(f"super-block ordering: eigh {sizes}")
    rng = np.random.Generator(np.random.PCG64(sum(sizes) + 7))
    mats = []
    for n in sizes:
        a = rng.normal(size=(n, n))
        mats.append(0.5 * (a + a.T))
    c = _ctx(1)
    out = c.eigh_batched(mats)
    for a, (wv, V) in zip(mats, out):
        n = a.shape[0]
        ref = np.linalg.eigvalsh(a)
        assert np.max(np.abs(np.sort(wv) - ref)) < 1e-12 * max(1.0, np.abs(ref).max()) * n
        assert np.max(np.abs(V @ V.T - np.eye(n))) < 1e-12 * n
        assert np.max(np.abs(a @ V.T - V.T * wv)) < 1e-11 * n
