"""Write oracle reference values for GPU parity cases that are too slow to
recompute inside a test.  Calls only the oracle and the seeded workload
generators.  Run:  python tests/golden/make_golden.py [case ...]

A result is written only when the oracle's monomer loop and every fragment
SCC converged; the final monomer-loop change is stored with it.  Systems with
cut covalent bonds use tolerances ten times looser (charges 1e-9 for the
monomer loop and every SCC, SCC energy change 1e-10 Eh): the hybrid-orbital
projector carries a 1e6 Eh shift, whose FP64 rounding (about 1e-10 Eh in the
Fock matrix) leaves the charges of some SCC dimers wandering by 3e-10 to
6e-10 from one iteration to the next, above the 1e-10 of molecular
fragments.

Large cases (the 23,760-atom pentacene crystal) run the oracle over a pool of
worker processes (same arithmetic) and store the energies of every fragment
and SCC dimer, the ES-DIM total with a fixed sample of ES-DIM pairs, and a
fixed sample of the monomer shell charges.
"""

import json
import os
import platform
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
HOP_TOL = 1e-9
HOP_ETOL = 1e-10


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
    if name in ("ala20", "ala40", "ala60", "ala100"):
        return w.alanine_helix(int(name[3:])), 4 * A2B, 2
    if name == "pentacene_3x2x2":
        return w.pentacene_crystal(reps=(3, 2, 2)), 4 * A2B, 2
    if name == "pentacene_c4":
        return w.pentacene_crystal(), 4 * A2B, 2
    raise KeyError(name)


# cases too large for a stored gradient and for full per-pair output
LARGE = {"pentacene_c4"}
# helices of the streaming workload: energies and charges, no gradient
HELICES = {"ala20", "ala40", "ala60", "ala100"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make(name, workers=1):
    s, cut, order = case_system(name)
    p = default_params()
    large = name in LARGE
    hop = len(s.bonds) > 0
    macro_tol = HOP_TOL if hop else 1e-10
    scc_tol = HOP_TOL if hop else 1e-10
    scc_etol = HOP_ETOL if hop else 1e-11
    t = time.time()
    r = F.fmo(s, p, cut, order=order, macro_tol=macro_tol, scc_tol=scc_tol, scc_etol=scc_etol,
              workers=workers, keep_clusters=not large)
    t_energy = time.time() - t
    if not r.macro_converged:
        raise RuntimeError(f"{name}: monomer loop not converged (last change {r.macro_delta:.3e})")
    if not r.all_scc_converged:
        raise RuntimeError(f"{name}: a fragment SCC did not converge")
    out = dict(case=name, n_atoms=s.n_atoms, n_frag=s.n_frag, cutoff_bohr=cut, order=order,
               E=r.E, E_mono=list(map(float, r.E_mono)), dE_scc=list(map(float, r.dE_scc)),
               scc_pairs=r.lists[0].tolist(), macro_iter=r.macro_iter, macro_tol=macro_tol,
               scc_tol=scc_tol, scc_etol=scc_etol,
               macro_delta=r.macro_delta, macro_converged=bool(r.macro_converged),
               scc_converged=bool(r.all_scc_converged))
    if large:
        # fixed samples: every 97th ES-DIM pair, every 4th shell charge
        ke = np.arange(0, len(r.dE_esd), 97)
        out["dE_esd_sum"] = F.neumaier_sum(r.dE_esd)
        out["n_esd"] = int(len(r.dE_esd))
        out["esd_sample_index"] = ke.tolist()
        out["dE_esd_sample"] = list(map(float, r.dE_esd[ke]))
        kq = np.arange(0, len(r.q), 4)
        out["q_sample_index"] = kq.tolist()
        out["q_sample"] = list(map(float, r.q[kq]))
        out["q_sum"] = F.neumaier_sum(r.q)
        out["dimer_iters"] = int(sum(d["res"].niter for d in r.dimers))
    else:
        out["dE_esd"] = list(map(float, r.dE_esd))
        out["q"] = list(map(float, r.q))
    if order >= 3:
        out["dE_tri"] = list(map(float, r.dE_tri))
        out["trimers"] = r.lists[2].tolist()
        out["E_fmo2"] = r.E_fmo2
    if len(s.bonds):
        out["bonds"] = s.bonds.tolist()
    if not large and name not in HELICES and (order == 2 or not len(s.bonds)):
        g, _ = F.fmo_gradient(s, p, r)
        out["grad"] = g.tolist()
        if len(s.bonds):
            # the gradient is that of the energy plus the projector term
            out["E_hop_projector"] = F.hop_projector_energy(r)
    out["oracle_seconds"] = time.time() - t
    out["oracle_seconds_energy"] = t_energy
    out["oracle_workers"] = workers
    out["oracle_cpu"] = cpu_model()
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f)
    print(name, "E =", r.E, "macro", r.macro_iter, "in", round(out["oracle_seconds"], 1), "s")


if __name__ == "__main__":
    args = sys.argv[1:]
    workers = 1
    if args and args[0].startswith("--workers="):
        workers = int(args[0].split("=", 1)[1])
        args = args[1:]
    for n in (args or ["pentacene6", "anthracene5_fmo3", "droplet128", "ala4_fmo3", "ala10",
                       "pentacene_3x2x2"]):
        make(n, workers)
