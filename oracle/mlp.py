"""Learned initial monomer charges (oracle; test infrastructure only).

Not part of the paper (its SCC always starts from superposition charges);
this follows the workload definition of the learned guess:
* per-atom features: one-hot element (H, C, N, O) and 16 radial symmetry
  functions G_k = sum_j exp(-eta (R_ij - Rs_k)^2) fc(R_ij) over all other
  atoms within Rc = 6 Angstrom, Rs_k evenly spaced from 0.5 to 6 Angstrom,
  eta = 1 / (2 * 0.35^2) Angstrom^-2, fc(R) = (cos(pi R / Rc) + 1) / 2;
* a 20 -> 64 -> 64 -> 2 perceptron with tanh hidden units predicting the two
  shell charges of the atom; weights and inputs are rounded to bfloat16
  (round to nearest even) for the forward pass, sums are exact here (FP64);
* per-fragment projection: the guess of each fragment is shifted uniformly
  over its real shells so that its charges sum to minus its net charge
  (ghost shells of covalent boundaries get zero);
* training: mean squared error over atoms and both shells, gradients with
  respect to the bfloat16-rounded weights applied to FP32 master weights by
  Adam (beta1 0.9, beta2 0.999, eps 1e-8).
Weight vector layout (5634 values): W1[64][20], b1[64], W2[64][64], b2[64],
W3[2][64], b3[2].
"""

import math

import numpy as np

ELEMENTS = (1, 6, 7, 8)
NFEAT = 20
NRAD = 16
RC = 6.0
ETA = 1.0 / (2.0 * 0.35 ** 2)
RS = np.linspace(0.5, 6.0, NRAD)
SHAPES = [("W1", (64, 20)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (2, 64)), ("b3", (2,))]
NW = sum(int(np.prod(s)) for _, s in SHAPES)
BOHR_TO_ANGSTROM = 0.529177210903


def unpack(w):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(w[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.reshape(np.shape(x))


def features(Z, xyz_bohr):
    """[N][20] features of every atom (section doc above), FP64."""
    Z = np.asarray(Z)
    x = np.asarray(xyz_bohr, float) * BOHR_TO_ANGSTROM
    N = len(Z)
    F = np.zeros((N, NFEAT))
    for e, z in enumerate(ELEMENTS):
        F[Z == z, e] = 1.0
    for i0 in range(0, N, 1024):
        i1 = min(N, i0 + 1024)
        d = x[i0:i1, None, :] - x[None, :, :]
        R = np.sqrt(np.sum(d * d, axis=2))
        mask = (R < RC)
        mask[np.arange(i1 - i0), np.arange(i0, i1)] = False
        fc = np.where(mask, 0.5 * (np.cos(np.pi * R / RC) + 1.0), 0.0)
        for k in range(NRAD):
            F[i0:i1, 4 + k] = np.sum(np.exp(-ETA * (R - RS[k]) ** 2) * fc, axis=1)
    return F


def forward(w, X, keep=False, bf16=True):
    """Shell charges [N][2] from features X [N][20] with bfloat16-rounded
    weights and inputs (bf16=False: unrounded), exact sums."""
    rnd = (lambda a: bf16_round(a).astype(np.float64)) if bf16 else (lambda a: np.asarray(a, np.float64))
    p = {k: rnd(v) for k, v in unpack(w).items()}
    x = rnd(X)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(a2)
    y = h2 @ p["W3"].T + p["b3"]
    if keep:
        return y, dict(x=x, h1=h1, h2=h2, p=p)
    return y


def loss_and_grad(w, X, Y, bf16=True):
    """Mean squared error over atoms and shells, and its gradient with respect
    to the (bfloat16-rounded) weights, in the weight-vector layout."""
    y, c = forward(w, X, keep=True, bf16=bf16)
    n = y.shape[0] * y.shape[1]
    r = y - Y
    L = float(np.sum(r * r) / n)
    dy = 2.0 * r / n
    p = c["p"]
    g = {}
    g["W3"] = dy.T @ c["h2"]
    g["b3"] = dy.sum(axis=0)
    d2 = (dy @ p["W3"]) * (1.0 - c["h2"] ** 2)
    g["W2"] = d2.T @ c["h1"]
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (1.0 - c["h1"] ** 2)
    g["W1"] = d1.T @ c["x"]
    g["b1"] = d1.sum(axis=0)
    return L, np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])


def adam_step(w, m, v, t, grad, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) of the master weights."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def project(qsh, frag_of_shell, frag_charge):
    """Shift each fragment's shell charges uniformly so that they sum to minus
    its net charge."""
    q = np.array(qsh, dtype=float)
    F = len(frag_charge)
    tot = np.bincount(frag_of_shell, weights=q, minlength=F)
    cnt = np.bincount(frag_of_shell, minlength=F)
    shift = (tot + np.asarray(frag_charge, float)) / np.maximum(cnt, 1)
    return q - shift[frag_of_shell]
