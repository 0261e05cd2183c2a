"""Write oracle reference values for GPU parity cases that are too slow to
recompute inside a test.  Calls only the oracle and the seeded workload
generators.  Run:  python tests/golden/make_golden.py [case ...]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as w  # noqa: E402
from oracle import fmo as F  # noqa: E402
from oracle.params import default_params  # noqa: E402

A2B = w.ANGSTROM_TO_BOHR


def case_system(name):
    if name == "pentacene6":
        return w.pentacene_crystal(reps=(2, 2, 1)).subset(list(range(6))), 4 * A2B, 2
    if name == "anthracene5_fmo3":
        return w.anthracene_crystal(reps=(2, 2, 1)).subset(list(range(5))), 4 * A2B, 3
    if name == "droplet128":
        return w.water_droplet(128, radius=9.8, seed=22), 4 * A2B, 2
    if name == "ala4_fmo3":
        return w.alanine_helix(4), 4 * A2B, 3
    if name == "ala10":
        return w.alanine_helix(10), 4 * A2B, 2
    raise KeyError(name)


def make(name):
    s, cut, order = case_system(name)
    p = default_params()
    t = time.time()
    r = F.fmo(s, p, cut, order=order)
    out = dict(case=name, n_atoms=s.n_atoms, n_frag=s.n_frag, cutoff_bohr=cut, order=order,
               E=r.E, E_mono=list(map(float, r.E_mono)), dE_scc=list(map(float, r.dE_scc)),
               dE_esd=list(map(float, r.dE_esd)), q=list(map(float, r.q)),
               scc_pairs=r.lists[0].tolist(), macro_iter=r.macro_iter)
    if order >= 3:
        out["dE_tri"] = list(map(float, r.dE_tri))
        out["trimers"] = r.lists[2].tolist()
    if order >= 3:
        out["E_fmo2"] = r.E_fmo2
    if len(s.bonds):
        out["bonds"] = s.bonds.tolist()
    if not len(s.bonds):
        g, _ = F.fmo_gradient(s, p, r)
        out["grad"] = g.tolist()
    out["oracle_seconds"] = time.time() - t
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f)
    print(name, "E =", r.E, "in", round(out["oracle_seconds"], 1), "s")


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["pentacene6", "anthracene5_fmo3", "droplet128", "ala4_fmo3", "ala10"]):
        make(n)
