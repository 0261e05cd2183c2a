"""Element constants for the oracle.

The paper gives the GFN1-xTB expressions symbolically (section "GFN1-xTB");
the values come from the seeded input file.  Units: Hartree, bohr.
"""

import numpy as np

from workloads import load_params_json


class Params:
    def __init__(self, path=None):
        raw = load_params_json(path)
        g = raw["globals"]
        self.kg = float(g["kg"])
        self.kf = float(g["kf"])
        self.kEN = float(g["kEN"])
        self.k1 = float(g["k1"])
        self.k2 = float(g["k2"])
        self.kl = [float(x) for x in g["kl"]]      # Wolfsberg-Helmholz k_l per l
        self.KAB = float(g["KAB"])
        self.kT = float(g["Tel_K"]) * float(g["kB_Eh_per_K"])
        self.VHOP = float(g["VHOP"])
        a2b = float(g["angstrom_to_bohr"])
        self.basis = {}
        for key, b in raw["basis"].items():
            self.basis[(int(b["n"]), int(b["l"]))] = (
                np.array(b["alpha"], float), np.array(b["coef"], float))
        self.elem = {}
        for sym, e in raw["elements"].items():
            Z = int(e["Z"])
            self.elem[Z] = dict(
                sym=sym,
                shells=[dict(n=int(s["n"]), l=int(s["l"]), zeta=float(s["zeta"]),
                             level=float(s["level"]), q0=float(s["q0"]),
                             kcn=float(s["kcn"]), kpoly=float(s["kpoly"]),
                             kappa=float(s["kappa"])) for s in e["shells"]],
                EN=float(e["EN"]), rcov=float(e["rcov_angstrom"]) * a2b,
                eta=float(e["eta"]), Gamma=float(e["Gamma"]),
                zeff=float(e["zeff"]), arep=float(e["alpha_rep"]),
                rvdw=float(e["rvdw_angstrom"]) * a2b if "rvdw_angstrom" in e else None)

    def element(self, Z):
        if Z not in self.elem:
            raise KeyError(f"element Z={Z} has no parameters")
        return self.elem[Z]


_default = None


def default_params():
    global _default
    if _default is None:
        _default = Params()
    return _default
