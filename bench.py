"""Benchmark: FMO2-xTB energy + analytic gradient of the 23,760-atom pentacene
crystal (11 x 5 x 6 triclinic herringbone cells, 660 molecules, seeded
+-0.05 A jitter) on one MI355X.

A step is one full pass of the hot path for one geometry: the pair lists
(classification of every fragment pair on the GPU), supersystem CN, the
self-consistent monomer embedding, all SCC dimers, the ES-DIM pairs, the
energy and the FMO2 gradient including the embedding response.  The system
is uploaded before timing (inputs resident in HBM).

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain] [--no-guess] [--no-forms] [--no-warm] [--no-fmo3]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_FP64_PEAK_TFLOPS = 78.6

# HBM traffic of the dominant kernel on this workload, from two rocprofv3 PMC
# passes (FETCH_SIZE scaled by 2 and WRITE_SIZE by 1, the factors a 1 GiB
# device copy gives), bytes per launch averaged over the launches of the
# warm-up and the timed step; valid while the kernel and the SCC schedule are
# unchanged (profiles/k_apply_rot_dual_pentacene_fmo2.md gives the commands)
PMC_TRAFFIC_BYTES = {"fx::k_apply_rot_dual": 2.14e9 + 0.90e9, "fx::k_apply_rot": 0.14e9 + 0.06e9}


def scc_iteration_work(n, n_occ):
    """Algorithmic flops of one SCC iteration of an n-AO system with n_occ
    occupied orbitals: 3.3 n^3 for a dense symmetric eigensolve (reduction and
    back-transformation of the eigenvectors) plus 5 n^2 n_occ for the
    transformations and the density over the occupied orbitals."""
    return 3.3 * n ** 3 + 5.0 * n * n * n_occ


def fragment_sizes(s):
    """(AOs, occupied orbitals) of a neutral fragment of the system (the
    crystal's fragments are identical molecules)."""
    import numpy as np
    from oracle.params import default_params
    p = default_params()
    atoms = np.where(s.frag == 0)[0]
    nao = sum(sum(1 if sh["l"] == 0 else 3 for sh in p.element(int(s.Z[a]))["shells"]) for a in atoms)
    nel = sum(sum(sh["q0"] for sh in p.element(int(s.Z[a]))["shells"]) for a in atoms)
    return nao, int(round(nel / 2))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE = {}


def _oracle_task(args):
    """One unit of oracle work in a pool worker: a monomer SCC, an SCC dimer
    (with its explicit gradient terms) or a chunk of an embedding-field pass
    (all in the zero embedding field where a field is needed)."""
    import numpy as np
    from oracle import fmo as F
    from oracle import xtb as X
    kind, idx = args
    st = _ORACLE
    p, s, fa, cn = st["p"], st["s"], st["fa"], st["cn"]
    t = time.perf_counter()
    if kind == "mono":
        sm = X.XtbSystem(p, s.Z[fa[idx]], s.xyz[fa[idx]], cn[fa[idx]])
        X.scc(sm)
    elif kind == "dimer":
        I, J = idx
        at = np.concatenate([fa[I], fa[J]])
        sd = X.XtbSystem(p, s.Z[at], s.xyz[at], cn[at])
        rd = X.scc(sd)
        DS = 0.5 * (rd.sigma[sd.ao_sh][:, None] + rd.sigma[sd.ao_sh][None, :]) * rd.P - rd.Wt
        X.system_gradient(sd, rd.P, DS, rd.q, rd.q, True)
    else:
        sh = st["sh"]
        same = lambda a, b: sh.frag[a] == sh.frag[b]
        sh.potential(np.arange(idx, min(sh.n, idx + 512)), st["q"], same, chunk=512)
    return time.perf_counter() - t


def cpu_baseline(system, timed_result, workers):
    """Time the FP64 oracle on a bounded sample of the same workload, with a
    process pool over fragments as the oracle runs large systems, and scale it
    to seconds per step: the supersystem CN (timed on 4096 atoms, scaled by
    the square of the atom ratio); one pool round of monomer SCCs, one of SCC
    dimers with their explicit gradient terms and one of field-pass chunks,
    each scaled to the step's counts (monomer solves per sweep times the
    sweeps, SCC dimers, field chunks per pass times the passes).  The oracle's
    response (dense inter-fragment kernel) is not part of the sample."""
    import multiprocessing
    import numpy as np
    from oracle import fmo as F
    from oracle import xtb as X
    from oracle.params import default_params

    p = default_params()
    A2B = 1.0 / 0.529177210903
    nsub = min(4096, system.n_atoms)
    t0 = time.perf_counter()
    X.coordination_numbers(p, system.Z[:nsub], system.xyz[:nsub])
    t_cn = (time.perf_counter() - t0) * (system.n_atoms / nsub) ** 2
    cn = np.zeros(system.n_atoms)
    fa = F.fragment_atoms(system.frag, system.n_frag)
    sub = system.subset(list(range(24)))
    near = np.concatenate([fa[k] for k in range(24)])
    cn[near] = X.coordination_numbers(p, sub.Z, sub.xyz)
    scc_pairs, _, _ = F.build_lists(sub, 4.0 * A2B)
    sh = F.Shells(p, F.ExtendedAtoms(system, cn))
    rng = np.random.Generator(np.random.PCG64(5))
    _ORACLE.update(p=p, s=system, fa=fa, cn=cn, sh=sh, q=rng.normal(0.0, 0.1, sh.n))
    ctx = multiprocessing.get_context("fork")

    def init():
        try:
            from threadpoolctl import threadpool_limits
            threadpool_limits(1)
        except ImportError:
            pass

    def pool_round(tasks):
        with ctx.Pool(workers, initializer=init) as pool:
            t = time.perf_counter()
            pool.map(_oracle_task, tasks, chunksize=1)
            return time.perf_counter() - t

    nw = workers
    t_mono = pool_round([("mono", k % 24) for k in range(nw)])
    dimers = [tuple(map(int, scc_pairs[k % len(scc_pairs)])) for k in range(nw)]
    t_dimer = pool_round([("dimer", d) for d in dimers])
    t_field = pool_round([("field", 512 * k) for k in range(nw)])
    sweeps = timed_result["macro_iter"]
    n_mono = sweeps * system.n_frag
    n_dimers = timed_result["solves_dimer"]
    chunks_per_pass = (sh.n + 511) // 512
    est = (t_cn + t_mono * n_mono / nw + t_dimer * n_dimers / nw
           + t_field * (sweeps + 1) * chunks_per_pass / nw)
    return {
        "value": est, "unit": "s/step", "cores": int(nw), "kind": "oracle",
        "cpu_model": _cpu_model(),
        "sample": (f"FP64 oracle, pool of {nw} worker processes (one BLAS thread each): one round of {nw} "
                   f"monomer SCCs ({t_mono:.2f} s), of {nw} SCC dimers with their explicit gradient terms "
                   f"({t_dimer:.2f} s) and of {nw} field-pass chunks of 512 target shells ({t_field:.2f} s), "
                   f"plus the supersystem CN ({t_cn:.2f} s, timed on {nsub} atoms and scaled by the square of "
                   f"the atom ratio); scaled to {sweeps} sweeps of {system.n_frag} monomer solves, "
                   f"{n_dimers} SCC dimers and {sweeps + 1} field passes of {chunks_per_pass} chunks; the "
                   f"oracle's response is not included"),
    }


def _golden_c4():
    path = os.path.join(ROOT, "tests", "golden", "pentacene_c4.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def forms_c4(c, s, sec_fp64, r64, g64):
    """The forms of the step on the same crystal, each timed after a warm-up
    run (the one-system-at-a-time loop once, without warm-up): the plain
    per-fragment GPU loop (FX_PLAIN_LOOP, FP64), the batched FP64 form (the
    headline, device-compacted active lists), the mixed-precision form, the
    learned initial guess, the batched form with one host synchronisation
    per SCC iteration, the captured-graph schedule, and the combined batched
    + mixed + learned form.
    Each reports |E - E_oracle| against the oracle golden of this crystal and
    max |g - g_FP64| against the batched FP64 gradient (pinned by central
    differences in the tests)."""
    import numpy as np
    import torch
    from paper_2606_28022_amd.binding import trained_guess_model
    ref = _golden_c4()
    blob, tau = trained_guess_model()
    c.mlp_load(blob)
    defaults = dict(schedule=0, precision=0, guess=0, guess_tau=0.0)
    variants = [("plain_loop_fp64", dict(schedule=1), False),
                ("batched_mixed", dict(precision=1), True),
                ("batched_learned_guess", dict(guess=1, guess_tau=tau), True),
                ("host_synced_fp64", dict(schedule=3), True),
                ("graph_fp64", dict(schedule=2), True),
                ("combined_batched_mixed_learned", dict(precision=1, guess=1, guess_tau=tau), True)]
    out = {"workload": "same crystal, FMO2 energy + analytic gradient with response",
           "batched_fp64": {"s_per_step": sec_fp64,
                            "abs_dE_vs_oracle_Eh": abs(r64["e_total"] - ref["E"]) if ref else None}}
    for name, opts, warm in variants:
        c.set_options(**defaults)
        c.set_options(**opts)
        if warm:
            c.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rv = c.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        gv = c.gradient()
        out[name] = {"s_per_step": dt,
                     "abs_dE_vs_oracle_Eh": abs(rv["e_total"] - ref["E"]) if ref else None,
                     "abs_dE_vs_fp64_Eh": abs(rv["e_total"] - r64["e_total"]),
                     "max_abs_dgrad_vs_fp64_Eh_per_bohr": float(np.abs(gv - g64).max()),
                     "iterations": {"monomer": rv["iters_mono"], "dimer": rv["iters_dimer"],
                                    "macro": rv["macro_iter"], "fp32": rv["iters_fp32"]},
                     "phases_ms": {k: round(rv[k], 2) for k in ("ms_monomer", "ms_dimer", "ms_gradient",
                                                                "ms_response")}}
        log(f"form {name}: {dt:.3f} s, E = {rv['e_total']:.8f}")
    c.set_options(**defaults)
    t_plain = out["plain_loop_fp64"]["s_per_step"]
    out["speedup_vs_plain_loop"] = {k: t_plain / v["s_per_step"] for k, v in out.items()
                                    if isinstance(v, dict) and "s_per_step" in v and k != "plain_loop_fp64"}
    return out


def plain_vs_batched():
    """Batched vs one-fragment-at-a-time schedule on the 1024-molecule water
    droplet (FMO2 energy, FP64); returns (speed-up, |dE|)."""
    from paper_2606_28022_amd import FmoXtb
    import workloads as w
    s = w.water_droplet()
    c = FmoXtb()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=0)
    c.run()
    t = time.time()
    rb = c.run()
    tb = time.time() - t
    c.set_options(schedule=1)
    t = time.time()
    rp = c.run()
    tp = time.time() - t
    return tp / tb, abs(rb["e_total"] - rp["e_total"]), tb, tp


def learned_guess_stream(n_droplets=8):
    """Learned initial charges on the streaming workload: the first streaming
    droplets (32-512 waters) and Ala20/Ala40 helices (cut bonds; nitrogen is
    absent from the training set), FMO2 energy, superposition vs learned
    start with the shipped model."""
    import numpy as np
    import workloads as w
    from paper_2606_28022_amd import FmoXtb
    from paper_2606_28022_amd.binding import trained_guess_model
    blob, tau = trained_guess_model()
    systems = [w.stream_droplet(500 + k) for k in range(n_droplets)] + [w.alanine_helix(n) for n in (20, 40)]
    it0 = it1 = mono = fb = 0
    t0 = t1 = 0.0
    dE = 0.0
    res0 = []
    res1 = []
    for s in systems:
        c = FmoXtb()
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge, bonds=s.bonds)
        c.set_options(want_gradient=0)
        c.run()
        t = time.perf_counter()
        r0 = c.run()
        t0 += time.perf_counter() - t
        c.mlp_load(blob)
        c.set_options(guess=1, guess_tau=tau)
        t = time.perf_counter()
        r1 = c.run()
        t1 += time.perf_counter() - t
        it0 += r0["iters_mono"]
        it1 += r1["iters_mono"]
        mono += s.n_frag
        fb += r1["guess_fallbacks"]
        dE = max(dE, abs(r1["e_total"] - r0["e_total"]))
        res0.append(r0["first_residual_median"])
        res1.append(r1["first_residual_median"])
        log(f"  {s.name}: monomer SCC iterations {r0['iters_mono']} -> {r1['iters_mono']}, "
            f"fallbacks {r1['guess_fallbacks']}, dE {r1['e_total'] - r0['e_total']:.2e}")
    return {"workload": f"{n_droplets} streaming droplets (seeds 500-{499 + n_droplets}) + Ala20, Ala40 helices, FMO2 energy",
            "monomer_scc_iterations": {"superposition": it0, "learned": it1},
            "iterations_saved_frac": 1.0 - it1 / max(1, it0), "max_abs_dE_Eh": dE,
            "fallback_rate": fb / max(1, mono), "tau": tau,
            "first_residual_median": {"superposition": float(np.median(res0)), "learned": float(np.median(res1))},
            "seconds": {"superposition": t0, "learned": t1}}


def fmo3_anthracene():
    """FMO3 energy + analytic gradient of the anthracene 8x8x4 crystal (512
    molecules, 12,288 atoms): one warm-up run, one timed run."""
    import numpy as np
    import torch
    import workloads as w
    from paper_2606_28022_amd import FmoXtb
    s = w.anthracene_crystal()
    c = FmoXtb(device=0, stream=C_stream(torch.cuda.current_stream()))
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(order=3, want_gradient=1, want_response=1)
    c.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = c.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    g = c.gradient()
    log(f"FMO3 anthracene: {dt:.3f} s, {r['solves_trimer']} trimers")
    # the same step in the mixed-precision form
    c.set_options(precision=1)
    c.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rm = c.run()
    torch.cuda.synchronize()
    dtm = time.perf_counter() - t
    gm = c.gradient()
    c.close()
    return {"workload": "anthracene 8x8x4 crystal (12,288 atoms, 512 molecules), FMO3 energy + analytic "
                        "gradient with response, fp64",
            "s_per_step": dt, "energy_Eh": r["e_total"],
            "mixed_vs_fp64": {"s_per_step": dtm, "abs_dE_Eh": abs(rm["e_total"] - r["e_total"]),
                              "max_abs_dgrad_Eh_per_bohr": float(np.abs(gm - g).max())},
            "solves": {"monomer": r["solves_mono"], "dimer": r["solves_dimer"], "trimer": r["solves_trimer"]},
            "scc_solves_per_s": (r["solves_mono"] + r["solves_dimer"] + r["solves_trimer"]) / dt,
            "phases_ms": {k: r[k] for k in ("ms_monomer", "ms_dimer", "ms_trimer", "ms_gradient")},
            "net_force": float(np.abs(g.sum(0)).max()),
            "net_torque": float(np.abs(np.cross(s.xyz, g).sum(0)).max())}


def warm_step(c, s, r_prev, sec_cold):
    """One MD-like step: every atom moved 0.001 Angstrom in a seeded random
    direction.  Timed twice at the displaced geometry: the SCC started from
    the previous step's converged monomer shell charges (FX_GUESS_USER), and
    in addition every SCC dimer started from its previous converged charges
    and orbitals (warm_clusters, as fx_md_verlet runs its steps).  A cold
    solve at the displaced geometry checks that all reach the same fixed
    point.  The context is left on the original geometry with the
    superposition guess and warm_clusters off."""
    import numpy as np
    import torch
    import workloads as w
    c.set_options(warm_clusters=1)
    c.run()                       # the previous step, its dimers saved
    q = c.charges()
    rng = np.random.default_rng(4)
    d = rng.normal(size=s.xyz.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz2 = s.xyz + 0.001 * w.ANGSTROM_TO_BOHR * d
    c.set_coordinates(xyz2)

    def timed(warm):
        c.set_options(guess=2, warm_clusters=warm)
        c.set_guess(q)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = c.run()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t, c.gradient()

    rq, tq, gq = timed(0)         # saves nothing: the dimers stay those of the previous step
    rw, tw, gw = timed(1)
    assert rw["warm_dimers"] > 0
    c.set_options(guess=0, warm_clusters=0)
    rc = c.run()
    gc = c.gradient()
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    log(f"warm step: charges {tq:.3f} s, charges + dimers {tw:.3f} s ({rw['warm_dimers']} warm dimers; dimer "
        f"iterations {rw['iters_dimer']} vs {rc['iters_dimer']} cold), "
        f"|E_warm - E_cold| = {max(abs(rw['e_total'] - rc['e_total']), abs(rq['e_total'] - rc['e_total'])):.2e}")
    return {"workload": "same crystal, every atom moved 0.001 A (seeded random directions), "
                        "previous step's monomer charges as the guess; then also its SCC dimers' "
                        "charges and orbitals",
            "s_per_step": tw, "speedup_vs_cold": sec_cold / tw,
            "s_per_step_charges_only": tq,
            "ms_dimer": {"warm_dimers": rw["ms_dimer"], "charges_only": rq["ms_dimer"], "cold": rc["ms_dimer"]},
            "macro_iter": {"warm": rw["macro_iter"], "cold": rc["macro_iter"]},
            "iterations": {"warm_monomer": rw["iters_mono"], "cold_monomer": rc["iters_mono"],
                           "warm_dimer": rw["iters_dimer"], "charges_only_dimer": rq["iters_dimer"],
                           "cold_dimer": rc["iters_dimer"]},
            "warm_dimers": rw["warm_dimers"],
            "abs_dE_warm_vs_cold_Eh": max(abs(rw["e_total"] - rc["e_total"]), abs(rq["e_total"] - rc["e_total"])),
            "max_abs_dgrad_Eh_per_bohr": float(max(np.abs(gw - gc).max(), np.abs(gq - gc).max())),
            "dE_from_previous_step_Eh": rw["e_total"] - r_prev["e_total"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-guess", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--no-fmo3", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(how it would shard is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as w
    from paper_2606_28022_amd import FmoXtb

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    s = w.pentacene_crystal()
    log(f"system {s.name}: {s.n_atoms} atoms, {s.n_frag} fragments")
    c = FmoXtb(device=0, stream=C_stream(stream))
    c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
    c.set_options(want_gradient=1, want_response=1)
    cnt = c.get_counts()

    for k in range(args.warmup):
        c.build_lists_counts()
        r = c.run()
        log(f"warmup {k}: {r['ms_monomer'] + r['ms_dimer'] + r['ms_gradient']:.0f} ms")

    torch.cuda.synchronize()
    times, results = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        c.build_lists_counts()   # the pair lists are part of the step
        r = c.run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        results.append(r)
        log(f"step {k}: {times[-1]:.3f} s, E = {r['e_total']:.8f}")
    g = c.gradient()
    sec = float(np.mean(times))
    r = results[-1]
    solves = r["solves_mono"] + r["solves_dimer"]

    # roofline of the dominant kernel: the library times its hot kernels with
    # HIP events on the context stream (fx_result.kstat, largest first) and
    # credits each with algorithmic work: the eigensolver kernels 3.3 n^3 per
    # SCC iteration (the split form: 1.3 n^3 to the rotation kernel, 2 n^3,
    # the back-transformation of the eigenvectors, to the apply kernel),
    # products 2 n^3 (symmetric ones by the tiles computed, the density over
    # the occupied orbitals 2 n^2 n_occ), field passes 8 flop per shell pair.
    # All compute in FP64 (the FP32-stored Jacobi working matrix aside), so the
    # FP64 peak (78.6 TFLOP/s, vector and matrix alike) is the ceiling.
    kern = {}
    for k in r["kernels"]:
        nl = max(1, k["launches"])
        avg = k["ms"] / nl
        kern[k["name"]] = {"achieved": (k["gflop"] / nl) / avg if avg > 0 else 0.0,  # GFLOP/ms = TFLOP/s
                           "avg_launch_ms": avg, "launches": k["launches"], "total_ms": k["ms"],
                           "share_of_step": k["ms"] / (1000.0 * sec)}
    dom = r["kernels"][0]["name"]
    bound = "mfma" if "gemm" in dom else "alu"
    # whole step: the SCC iterations at 3.3 n^3 + 5 n^2 n_occ each plus the
    # field passes, over the measured step time
    nm, om = fragment_sizes(s)
    field_gflop = sum(k["gflop"] for k in r["kernels"] if k["name"].startswith("fx::k_field"))
    work = (r["iters_mono"] * scc_iteration_work(nm, om) + r["iters_dimer"] * scc_iteration_work(2 * nm, 2 * om)
            + 1e9 * field_gflop)
    step_rate = work / sec / 1e12
    traffic = PMC_TRAFFIC_BYTES.get(dom)
    roofline = {"bound": bound, "kernel": dom,
                "achieved": kern[dom]["achieved"], "peak": MI355X_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": kern[dom]["achieved"] / MI355X_FP64_PEAK_TFLOPS, "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM, PMC)" if traffic else None,
                "avg_launch_ms": kern[dom]["avg_launch_ms"], "launches": kern[dom]["launches"],
                "share_of_step": kern[dom]["share_of_step"],
                "whole_step": {"achieved": step_rate, "frac": step_rate / MI355X_FP64_PEAK_TFLOPS,
                               "algorithmic_tflop": work / 1e12,
                               "accounting": f"SCC iterations x (3.3 n^3 + 5 n^2 n_occ), n = {nm} / {2 * nm}, "
                                             f"n_occ = {om} / {2 * om}, plus field passes"},
                "kernels": kern}

    out = {
        "metric": "FMO2 energy+grad s/step; fragment SCC solves/s; batched vs plain @1e-6 Eh",
        "value": sec, "unit": "s/step", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * sec, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "pentacene 11x5x6 crystal, FMO2 energy + analytic gradient with response",
                   "atoms": s.n_atoms, "fragments": s.n_frag, "scc_dimers": int(cnt.n_scc_pairs),
                   "es_dim_pairs": int(cnt.n_esd_pairs), "cutoff_angstrom": 4.0,
                   "precision": ("fp64: basis, products, rotation angles, energies and gradient; the Jacobi "
                                 "working matrix of the 232-AO dimers is stored in FP32 between FP64 rebuilds "
                                 "of C^T F C"),
                   "schedule": "batched"},
        "scc_solves_per_s": solves / sec,
        "solves_per_s_by_phase": {"monomer": r["solves_mono"] / (1e-3 * r["ms_monomer"]),
                                  "dimer": r["solves_dimer"] / (1e-3 * r["ms_dimer"])},
        "energy_Eh": r["e_total"], "grad_max_Eh_per_bohr": float(np.abs(g).max()),
        "net_force": float(np.abs(g.sum(0)).max()),
        "phases_ms": {k: r[k] for k in ("ms_lists", "ms_monomer", "ms_dimer", "ms_energy", "ms_gradient",
                                        "ms_response")},
        "iterations": {"monomer": r["iters_mono"], "dimer": r["iters_dimer"], "macro": r["macro_iter"]},
        "roofline": roofline,
    }
    if not args.no_warm:
        out["warm_start"] = warm_step(c, s, r, sec)
    if not args.no_fmo3:
        out["fmo3"] = fmo3_anthracene()
    if not args.no_plain:
        sp, de, tb, tp = plain_vs_batched()
        out["batched_vs_plain"] = {"workload": "water droplet 1024 molecules, FMO2 energy, fp64",
                                   "speedup": sp, "abs_dE": de, "batched_s": tb, "plain_s": tp}
    if not args.no_forms:
        out["forms"] = forms_c4(c, s, sec, r, g)
    if not args.no_guess:
        out["learned_guess"] = learned_guess_stream()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, r, workers=min(16, os.cpu_count() or 1))
    print(json.dumps(out), flush=True)


def C_stream(stream):
    """hipStream_t handle of a torch stream (None for the default stream)."""
    import ctypes
    h = stream.cuda_stream
    return ctypes.c_void_p(h) if h else None


if __name__ == "__main__":
    main()
