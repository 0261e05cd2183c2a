"""Learned initial guess on the GPU vs its oracle (oracle/mlp.py), through
the C ABI: features, bfloat16 forward pass, gradient, Adam step, and FMO runs
started from the learned charges (which must converge to the same energy as
superposition starts, with or without fallbacks)."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w
from oracle import fmo as F
from oracle import mlp as M

A2B = w.ANGSTROM_TO_BOHR


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(s):
    from paper_2606_28022_amd import FmoXtb
    c = FmoXtb()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=s.bonds)
    return c


def _weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=M.NW) * scale).astype(np.float32)


@pytest.mark.parametrize("which", ["c1", "anthracene3", "ala3"])
def test_features(which):
    _say(f"mlp features {which}")
    s = {"c1": lambda: w.water_cluster_cube(),
         "anthracene3": lambda: w.anthracene_crystal(reps=(2, 2, 1)).subset([0, 1, 2]),
         "ala3": lambda: w.alanine_helix(3)}[which]()
    c = _ctx(s)
    g = c.mlp_features().cpu().numpy()
    ref = M.features(s.Z, s.xyz)
    assert g.shape == ref.shape
    assert np.max(np.abs(g - ref)) < 1e-5 * max(1.0, np.abs(ref).max())


def test_forward_gradient_adam():
    import torch
    _say("mlp forward / gradient / Adam")
    s = w.anthracene_crystal(reps=(2, 2, 1)).subset([0, 1, 2, 3])
    c = _ctx(s)
    w0 = _weights(7)
    c.mlp_set_master(w0)
    X = M.features(s.Z, s.xyz)
    rng = np.random.default_rng(8)
    Y = rng.normal(scale=0.2, size=(len(X), 2))
    xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    Xf = X.astype(np.float32)
    # forward
    yg = c.mlp_infer(xd).cpu().numpy()
    yo = M.forward(w0, Xf)
    assert np.max(np.abs(yg - yo)) < 2e-5 * max(1.0, np.abs(yo).max())
    # loss and gradient
    Lg, gg = c.mlp_grad(xd, yd)
    Lo, go = M.loss_and_grad(w0, Xf, Y.astype(np.float32).astype(np.float64))
    assert abs(Lg - Lo) < 1e-5 * max(1.0, Lo)
    assert np.max(np.abs(gg - go)) < 1e-4 * np.abs(go).max()
    # one Adam step of the master weights: entries with a clear gradient
    # sign move by lr; compare where |g| is not at FP32 noise level
    lr = 1e-3
    L1 = c.mlp_train_step(xd, yd, lr)
    assert abs(L1 - Lg) < 1e-12
    w1 = c.mlp_get_master()
    wo, _, _ = M.adam_step(w0.astype(np.float64), np.zeros(M.NW), np.zeros(M.NW), 1, go, lr)
    clear = np.abs(go) > 1e-3 * np.abs(go).max()
    assert clear.sum() > M.NW // 4
    assert np.max(np.abs(w1[clear] - wo[clear])) < 1e-6
    assert np.max(np.abs(w1 - w0)) <= lr * 1.0001
    # save / load round trip (bfloat16)
    blob = c.mlp_save()
    c.mlp_load(blob)
    w2 = c.mlp_get_master()
    assert np.array_equal(w2, M.bf16_round(w1))


def test_learned_guess_converges_to_same_energy(params):
    _say("mlp learned guess FMO2 c1")
    s = w.water_cluster_cube()
    c = _ctx(s)
    c.set_options(want_gradient=0)
    r0 = c.run()
    e0 = r0["e_total"]
    c.mlp_set_master(_weights(11, scale=0.05))
    c.set_options(guess=1, guess_tau=0.0)
    r1 = c.run()
    assert r1["guess_fallbacks"] == 0
    assert abs(r1["e_total"] - e0) < 1e-8
    # a tiny tau sends every monomer back to superposition charges
    c.set_options(guess=1, guess_tau=1e-12)
    r2 = c.run()
    assert r2["guess_fallbacks"] == s.n_frag
    assert abs(r2["e_total"] - e0) < 1e-8
    ro = F.fmo(s, params, 4 * A2B)
    assert abs(r1["e_total"] - ro.E) < 1e-8


def test_mlp_errors():
    from paper_2606_28022_amd.binding import FxError
    s = w.water_cluster_cube()
    c = _ctx(s)
    c.set_options(guess=1)
    with pytest.raises(FxError):
        c.run()                                    # no model loaded
    with pytest.raises(FxError):
        c.mlp_set_master(np.zeros(10, dtype=np.float32))   # wrong size


@pytest.mark.parametrize("which", ["droplet502", "ala10"])
def test_trained_model_same_energy_fewer_iterations(which):
    """The shipped model (trained on water and anthracene) as the start of a
    streaming droplet and of a helix with cut bonds: same converged energy
    as superposition starts; on the droplet, fewer monomer SCC iterations."""
    from paper_2606_28022_amd.binding import trained_guess_model
    _say(f"trained guess model {which}")
    s = w.stream_droplet(502) if which == "droplet502" else w.alanine_helix(10)
    blob, tau = trained_guess_model()
    c = _ctx(s)
    c.set_options(want_gradient=0)
    r0 = c.run()
    c.mlp_load(blob)
    c.set_options(guess=1, guess_tau=tau)
    r1 = c.run()
    assert abs(r1["e_total"] - r0["e_total"]) < 1e-8 * s.n_frag
    if which == "droplet502":
        assert r1["guess_fallbacks"] == 0
        assert r1["iters_mono"] < r0["iters_mono"]
        assert r1["first_residual_median"] < 0.2 * r0["first_residual_median"]
