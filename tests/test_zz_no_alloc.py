"""fx_embedding_field_noalloc (no device allocation; partial sums in the
library's static device scratch) against fx_embedding_field, through the C
ABI: two calls in a row, the second on a smaller system, both compared with
the allocating entry point's FP64 field (eq. v_esp_matrix).  The two passes
sum in different orders (chunked one-direction pass vs. symmetric pass), so
the bound is 1e-12 times the absolute sum sum_t gamma_st |dq_t| of the
shell, computed here with the allocating entry point itself (gamma > 0)."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import workloads as w


def _check(c, seed):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    dq = rng.normal(0.0, 0.2, c.n_shells)
    ref = c.embedding_field(dq)
    scale = c.embedding_field(np.abs(dq))
    tq = torch.tensor(dq, dtype=torch.float64, device="cuda")
    tphi = torch.full_like(tq, float("nan"))
    c.embedding_field_noalloc(tq, tphi)
    torch.cuda.synchronize()
    got = tphi.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref) / np.maximum(scale, 1e-300)) < 1e-12


def test_noalloc_field_two_calls_second_smaller():
    from paper_2606_28022_amd import FmoXtb
    big = w.water_droplet()
    small = w.water_cluster_cube()
    print("no-alloc field: droplet 1024 then cube 8", flush=True)
    sys.stdout.flush()
    c = FmoXtb()
    c.set_system(big.Z, big.xyz, big.frag, big.frag_charge)
    _check(c, 3)
    c2 = FmoXtb()
    c2.set_system(small.Z, small.xyz, small.frag, small.frag_charge)
    _check(c2, 4)
    # the larger system again after the smaller one (scratch keeps the last
    # call's contents; every entry used is rewritten)
    _check(c, 5)


def test_noalloc_field_rejects_bad_arguments():
    import torch
    from paper_2606_28022_amd import FmoXtb
    from paper_2606_28022_amd.binding import FxError
    c = FmoXtb()
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(FxError):
        c.embedding_field_noalloc(t, t)  # no system set
