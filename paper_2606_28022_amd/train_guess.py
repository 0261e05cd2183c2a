"""Train the learned initial-guess model (fx_mlp_*) on converged monomer
charges and write it to paper_2606_28022_amd/data/.

    python -m paper_2606_28022_amd.train_guess [--steps 3000] [--lr 3e-3]

Training systems: the 8-water cube, the 1,024-water droplet and the
512-molecule anthracene crystal (H, C, O only).  Each is solved once (FMO2
energy, superposition start) through the library on the GPU; the rows are the
real atoms' features (fx_mlp_features) and the labels their two converged
monomer shell charges.  Full-batch Adam on the GPU (fx_mlp_train_step), from
seeded Gaussian weights.  The fallback threshold tau is the median, over the
training systems, of the median first SCC residual of superposition starts.
Writes guess_mlp.bf16 (FX_MLP_NW little-endian bfloat16 values) and
guess_mlp.json (tau, loss history, training rows).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

DATA = os.path.join(HERE, "data")


def initial_weights(seed=0):
    """Seeded Gaussian initialisation, 1/sqrt(fan_in) scaled (0.25 for the
    first layer, whose inputs are sums of up to ~20), zero biases."""
    from .binding import FX_MLP_NW
    rng = np.random.default_rng(seed)
    parts = [rng.normal(size=(64, 20)) * 0.25 / np.sqrt(20), np.zeros(64),
             rng.normal(size=(64, 64)) / np.sqrt(64), np.zeros(64),
             rng.normal(size=(2, 64)) / np.sqrt(64), np.zeros(2)]
    w = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert len(w) == FX_MLP_NW
    return w


def training_rows(systems):
    import torch
    from . import FmoXtb
    X, Y, res = [], [], []
    for s in systems:
        c = FmoXtb()
        c.set_system(s.Z, s.xyz, s.frag, s.frag_charge)
        c.set_options(want_gradient=0)
        r = c.run()
        q = c.charges()
        if q.shape[0] != 2 * s.n_atoms:
            raise ValueError("training systems must have two shells per atom")
        X.append(c.mlp_features().cpu())
        Y.append(torch.tensor(q.reshape(-1, 2), dtype=torch.float32))
        res.append(r["first_residual_median"])
        print(f"  {s.name}: {s.n_atoms} atoms, first-iteration residual median {r['first_residual_median']:.3e}",
              flush=True)
    return torch.cat(X).cuda(), torch.cat(Y).cuda(), res


def main():
    import workloads as w
    from . import FmoXtb
    from .binding import FX_MLP_NW
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=DATA)
    args = ap.parse_args()
    t0 = time.time()
    systems = [w.water_cluster_cube(), w.water_droplet(), w.anthracene_crystal()]
    X, Y, first_res = training_rows(systems)
    print(f"{X.shape[0]} training rows in {time.time() - t0:.1f} s", flush=True)
    c = FmoXtb()
    s0 = systems[0]
    c.set_system(s0.Z, s0.xyz, s0.frag, s0.frag_charge)
    c.mlp_set_master(initial_weights(0))
    hist = []
    for k in range(args.steps):
        lr = args.lr if k < args.steps // 2 else args.lr / 3.0
        L = c.mlp_train_step(X, Y, lr)
        if k % 250 == 0 or k == args.steps - 1:
            hist.append([k, L])
            print(f"  step {k}: loss {L:.4e}", flush=True)
    L_final, _ = c.mlp_grad(X, Y)
    blob = c.mlp_save()
    assert len(blob) == FX_MLP_NW
    os.makedirs(args.out, exist_ok=True)
    blob.astype("<u2").tofile(os.path.join(args.out, "guess_mlp.bf16"))
    meta = dict(tau=float(np.median(first_res)), first_residual_medians=first_res,
                rows=int(X.shape[0]), steps=args.steps, lr=args.lr, loss_history=hist,
                final_rmse=float(np.sqrt(L_final)),
                training_systems=[s.name for s in systems], seconds=time.time() - t0)
    with open(os.path.join(args.out, "guess_mlp.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps({k: meta[k] for k in ("tau", "rows", "final_rmse", "seconds")}), flush=True)


if __name__ == "__main__":
    main()
