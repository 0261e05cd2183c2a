"""Write the seeded GFN1-like parameter file ``gfn1_like.json``.

The paper states the GFN1-xTB energy expression symbolically (section
"GFN1-xTB", Eqs. gfn1-energy .. gfn1_rep_energy and eq. cn_def) but prints no
parameter values, and its Slater basis is only named.  This script produces a
stand-in parameter set:

* element constants drawn from a seeded generator (seed 0) as a +-5 % uniform
  jitter around textbook anchors (extended-Hueckel ionisation energies, Slater
  exponents, Pauling electronegativities, covalent radii), or uniformly within
  a plausible range where no anchor exists;
* an STO-6G expansion of each Slater radial function r^(n-1) exp(-r)
  (unit exponent) by maximum-overlap least squares on the radial integral.

The output is input data for both the oracle and the GPU library, like a
geometry.  Run once:  python -m workloads.make_params
"""

import json
import math
import os

import numpy as np
from scipy import integrate, optimize

EV_TO_EH = 1.0 / 27.211386245988

# (n, l) pairs that occur in the minimal basis: H 1s/2s, C/N/O 2s/2p.
SHELL_KINDS = [(1, 0), (2, 0), (2, 1)]
NPRIM = 6


def _slater_radial(n):
    return lambda r: r ** (n - 1) * math.exp(-r)


def _gauss_radial(l, a):
    return lambda r: r ** l * math.exp(-a * r * r)


def _radial_dot(f, g):
    val, _ = integrate.quad(lambda r: f(r) * g(r) * r * r, 0.0, np.inf,
                            limit=400, epsabs=1e-14, epsrel=1e-12)
    return val


def _gauss_gauss(l, a, b):
    # integral r^(2l+2) exp(-(a+b) r^2) dr
    m = 2 * l + 2
    return math.gamma((m + 1) / 2.0) / (2.0 * (a + b) ** ((m + 1) / 2.0))


def fit_sto(n, l, nprim=NPRIM):
    """Maximum-overlap fit of r^(n-1) e^(-r) by sum_k d_k r^l e^(-a_k r^2)."""
    fs = _slater_radial(n)
    ss = _radial_dot(fs, fs)

    def neg_overlap(loga):
        a = np.exp(np.sort(loga))
        b = np.array([_radial_dot(fs, _gauss_radial(l, ak)) for ak in a])
        G = np.array([[_gauss_gauss(l, ai, aj) for aj in a] for ai in a])
        try:
            x = np.linalg.solve(G, b)
        except np.linalg.LinAlgError:
            return 1.0
        return -float(b @ x) / ss

    x0 = np.log(np.geomspace(0.02, 25.0, nprim))
    res = optimize.minimize(neg_overlap, x0, method="Nelder-Mead",
                            options={"maxiter": 20000, "xatol": 1e-10,
                                     "fatol": 1e-14})
    res = optimize.minimize(neg_overlap, res.x, method="BFGS",
                            options={"gtol": 1e-12})
    a = np.exp(np.sort(res.x))
    b = np.array([_radial_dot(fs, _gauss_radial(l, ak)) for ak in a])
    G = np.array([[_gauss_gauss(l, ai, aj) for aj in a] for ai in a])
    d = np.linalg.solve(G, b)
    d /= math.sqrt(float(d @ G @ d))  # unit norm in the radial metric
    overlap = float(b @ d) / math.sqrt(ss)
    # express coefficients relative to radially normalised primitives
    dn = d * np.sqrt([_gauss_gauss(l, ak, ak) for ak in a])
    return a.tolist(), dn.tolist(), overlap


# anchors: level (eV), Slater exponent, reference occupation per shell;
# rvdw: Bondi van der Waals radius (Angstrom)
ELEMENTS = {
    "H": dict(Z=1, shells=[(1, 0, 1.20, -13.6, 1.0), (2, 0, 0.75, -3.0, 0.0)],
              EN=2.20, rcov=0.32, eta=0.47, Gamma=0.08, zeff=1.0, arep=2.2, rvdw=1.20),
    "C": dict(Z=6, shells=[(2, 0, 1.625, -21.4, 2.0), (2, 1, 1.625, -11.4, 2.0)],
              EN=2.55, rcov=0.75, eta=0.48, Gamma=0.05, zeff=4.0, arep=1.25, rvdw=1.70),
    "N": dict(Z=7, shells=[(2, 0, 1.95, -26.0, 2.0), (2, 1, 1.95, -13.4, 3.0)],
              EN=3.04, rcov=0.71, eta=0.46, Gamma=0.06, zeff=5.0, arep=1.35, rvdw=1.55),
    "O": dict(Z=8, shells=[(2, 0, 2.275, -32.3, 2.0), (2, 1, 2.275, -14.8, 4.0)],
              EN=3.44, rcov=0.63, eta=0.45, Gamma=0.07, zeff=6.0, arep=1.6, rvdw=1.52),
}


def make(seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))

    def jit(x):
        return float(x * (1.0 + rng.uniform(-0.05, 0.05)))

    basis = {}
    for (n, l) in SHELL_KINDS:
        a, d, ov = fit_sto(n, l)
        basis[f"{n}{'sp'[l]}"] = dict(n=n, l=l, alpha=a, coef=d, overlap=ov)

    elements = {}
    for sym, e in ELEMENTS.items():
        shells = []
        for k, (n, l, zeta, lev, q0) in enumerate(e["shells"]):
            shells.append(dict(
                n=n, l=l, zeta=jit(zeta), level=jit(lev * EV_TO_EH), q0=q0,
                kcn=float(rng.uniform(-0.01, 0.01)),
                kpoly=float(rng.uniform(-0.2, 0.2)),
                kappa=0.0 if k == 0 else float(rng.uniform(-0.3, 0.3)),
            ))
        elements[sym] = dict(
            Z=e["Z"], shells=shells, EN=jit(e["EN"]), rcov_angstrom=jit(e["rcov"]),
            eta=jit(e["eta"]), Gamma=jit(e["Gamma"]), zeff=jit(e["zeff"]),
            alpha_rep=jit(e["arep"]),
            # van der Waals radius of the fragment-pair selection rule: Bondi's
            # values as data, not drawn (no random number is consumed)
            rvdw_angstrom=e["rvdw"],
        )

    return dict(
        name="gfn1-like seeded stand-in (not the fitted GFN1-xTB values)",
        seed=seed,
        globals=dict(kg=2.0, kf=1.5, kEN=-0.007, k1=16.0, k2=4.0 / 3.0,
                     kl=[1.85, 2.6], KAB=1.0, Tel_K=300.0, VHOP=1.0e6,
                     kB_Eh_per_K=3.166811563e-6, angstrom_to_bohr=1.0 / 0.529177210903),
        basis=basis,
        elements=elements,
    )


if __name__ == "__main__":
    p = make(0)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gfn1_like.json")
    with open(out, "w") as f:
        json.dump(p, f, indent=1)
    for k, b in p["basis"].items():
        print(k, "overlap with Slater function:", b["overlap"])
    print("wrote", out)
