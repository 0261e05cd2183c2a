"""Oracle of the learned initial guess: bfloat16 rounding, features, forward,
gradient and Adam step, projection (pins by closed forms, brute force and
finite differences)."""

import math

import numpy as np

from oracle import mlp as M


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e38, 1.0 + 2.0 ** -9], np.float32)
    r = M.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # halfway, even mantissa kept
    assert r[2] == 1.0 + 2.0 ** -6           # halfway, rounds up to even
    assert r[3] == -2.5                      # exactly representable
    assert r[5] == 1.0                       # below halfway
    assert np.all(np.abs(r.astype(float) - x) <= np.abs(x) * 2.0 ** -8)


def test_features_two_atoms_closed_form():
    R = 2.3                                   # Angstrom
    Z = np.array([6, 1])
    xyz = np.array([[0.0, 0.0, 0.0], [R / M.BOHR_TO_ANGSTROM, 0.0, 0.0]])
    F = M.features(Z, xyz)
    assert list(F[0, :4]) == [0, 1, 0, 0] and list(F[1, :4]) == [1, 0, 0, 0]
    fc = 0.5 * (math.cos(math.pi * R / 6.0) + 1.0)
    for k in range(16):
        rs = 0.5 + k * 5.5 / 15.0
        assert abs(F[0, 4 + k] - math.exp(-M.ETA * (R - rs) ** 2) * fc) < 1e-14
    assert np.allclose(F[0, 4:], F[1, 4:])
    far = np.array([[0.0, 0.0, 0.0], [6.01 / M.BOHR_TO_ANGSTROM, 0.0, 0.0]])
    assert np.all(M.features(Z, far)[:, 4:] == 0.0)


def test_features_brute_force():
    rng = np.random.default_rng(3)
    Z = rng.choice([1, 6, 7, 8], size=9)
    xyz = rng.uniform(0, 8, size=(9, 3))
    F = M.features(Z, xyz)
    x = xyz * M.BOHR_TO_ANGSTROM
    for i in range(9):
        for k in range(16):
            v = 0.0
            for j in range(9):
                if j == i:
                    continue
                R = float(np.linalg.norm(x[i] - x[j]))
                if R < 6.0:
                    v += math.exp(-M.ETA * (R - M.RS[k]) ** 2) * 0.5 * (math.cos(math.pi * R / 6.0) + 1.0)
            assert abs(F[i, 4 + k] - v) < 1e-12


def test_gradient_finite_differences():
    rng = np.random.default_rng(5)
    w = rng.normal(scale=0.2, size=M.NW)
    X = rng.uniform(0, 2, size=(7, 20))
    Y = rng.normal(scale=0.3, size=(7, 2))
    L, g = M.loss_and_grad(w, X, Y, bf16=False)
    idx = rng.choice(M.NW, size=40, replace=False)
    h = 1e-6
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (M.loss_and_grad(wp, X, Y, bf16=False)[0] - M.loss_and_grad(wm, X, Y, bf16=False)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(fd))


def test_forward_layout_single_unit():
    """With one active path through the net the output is a hand-computable
    composition: W1 row 0 picks feature 3, W2 row 0 picks unit 0, W3 row 1
    reads unit 0."""
    w = np.zeros(M.NW)
    P = M.unpack(np.arange(M.NW, dtype=float))
    off = {}
    k = 0
    for name, shp in M.SHAPES:
        off[name] = k
        k += int(np.prod(shp))
    w[off["W1"] + 0 * 20 + 3] = 0.5
    w[off["W2"] + 0 * 64 + 0] = 2.0
    w[off["W3"] + 1 * 64 + 0] = 1.5
    w[off["b3"] + 0] = 0.25
    X = np.zeros((1, 20))
    X[0, 3] = 1.0
    y = M.forward(w, X)
    assert abs(y[0, 0] - 0.25) < 1e-15
    assert abs(y[0, 1] - 1.5 * math.tanh(2.0 * math.tanh(0.5))) < 1e-12


def test_adam_first_step_is_sign_step():
    g = np.array([0.3, -2.0, 1e-3])
    w = np.array([1.0, 1.0, 1.0])
    w1, m, v = M.adam_step(w, np.zeros(3), np.zeros(3), 1, g, lr=0.01)
    assert np.allclose(w1, w - 0.01 * np.sign(g), atol=1e-7)


def test_projection():
    q = np.array([0.1, 0.2, -0.05, 0.3, 0.0])
    fr = np.array([0, 0, 1, 1, 1])
    out = M.project(q, fr, [0, -1])
    assert abs(out[:2].sum()) < 1e-15 and abs(out[2:].sum() - 1.0) < 1e-15
    assert np.allclose(np.diff(out[:2] - q[:2]), 0.0)
