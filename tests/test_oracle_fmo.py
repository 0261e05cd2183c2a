"""Pins of the oracle's FMO layer.

* exact special cases of the many-body expansion (eqs. fmo2-energy-components,
  fmo3_energy): one fragment equals non-fragmented xTB; two fragments joined by
  an SCC dimer equal xTB of the union; three fragments with all pairs and the
  trimer equal xTB of the union;
* the energy identity E = sum c_I E^emb_I + sum_SCC E^emb_IJ - sum_ESD qγq
  (the reading of E_I as an internal energy);
* the SCC pair energy approaches its ES-DIM value as the pair separates;
* the analytic FMO2 gradient (explicit + response) matches central finite
  differences of the energy with the pair lists frozen, and the response term
  matters (the paper's gradient-error table shows the same pattern);
* the pair/trimer lists equal a brute-force classification, for the fixed
  cutoff and for the van der Waals-scaled rule of section "Computational
  Details" (which reduces to the cutoff rule when every radius is the same,
  and selects more pairs as its scale grows);
* fragments of several molecules: two fragments of four waters each joined
  by an SCC dimer equal xTB of the union;
* the FMO3 gradient (section "Extension to FMO3"): with three fragments, all
  pairs and the trimer it is the xTB gradient of the union; with SCC pairs
  shared by several trimers and ES-DIM sub-pairs inside trimers it matches
  central finite differences of the FMO3 energy, and the response matters.
"""

import numpy as np
import pytest

from oracle import fmo as F
import workloads as w

A2B = w.ANGSTROM_TO_BOHR


@pytest.fixture(scope="module")
def c1():
    return w.water_cluster_cube()


def test_one_fragment_is_xtb(params, c1):
    s = c1.subset([3])
    r = F.fmo(s, params, 4 * A2B)
    assert abs(r.E - F.xtb_energy(s, params)[0]) < 1e-9


def test_two_fragments_fmo2_exact(params, c1):
    s = c1.subset([0, 1])
    r = F.fmo(s, params, 100.0)
    assert len(r.lists[0]) == 1
    assert abs(r.E - F.xtb_energy(s, params)[0]) < 1e-9


def test_three_fragments_fmo3_exact(params, c1):
    s = c1.subset([0, 1, 2])
    r = F.fmo(s, params, 100.0, order=3)
    assert len(r.lists[2]) == 1
    assert abs(r.E - F.xtb_energy(s, params)[0]) < 1e-9


def test_energy_identity(params, c1):
    s = c1.subset([0, 1, 2, 3, 4])
    r = F.fmo(s, params, 4 * A2B)
    assert len(r.lists[0]) > 0 and len(r.lists[1]) > 0
    nscc = np.zeros(s.n_frag)
    for I, J in r.lists[0]:
        nscc[I] += 1
        nscc[J] += 1
    e = sum((1 - nscc[I]) * r.mono[I].e_emb for I in range(s.n_frag))
    e += sum(d["res"].e_emb for d in r.dimers)
    e -= float(np.sum(r.dE_esd))
    assert abs(e - r.E) < 1e-10


def test_separated_pair_limit(params):
    diffs = []
    for d in (4.0, 6.0, 9.0):
        s = w.separated_water_pair(d)
        scc = F.fmo(s, params, 1e3)   # treated as SCC dimer
        esd = F.fmo(s, params, 0.0)   # treated as ES-DIM
        diffs.append(abs(scc.E - esd.E))
    assert diffs[0] > diffs[1] > diffs[2]
    assert diffs[2] < 1e-6


def test_lists_bruteforce(params, c1):
    cut = 4 * A2B
    scc, esd, tri = F.build_lists(c1, cut, order=3)
    near = {}
    for I in range(c1.n_frag):
        for J in range(I + 1, c1.n_frag):
            dmin = min(np.linalg.norm(c1.xyz[a] - c1.xyz[b])
                       for a in np.where(c1.frag == I)[0] for b in np.where(c1.frag == J)[0])
            near[(I, J)] = int(dmin < cut)
    assert [tuple(p) for p in scc] == [k for k, v in near.items() if v]
    assert [tuple(p) for p in esd] == [k for k, v in near.items() if not v]
    exp_tri = [(I, J, K) for I in range(8) for J in range(I + 1, 8) for K in range(J + 1, 8)
               if near[(I, J)] + near[(I, K)] + near[(J, K)] >= 2]
    assert [tuple(t) for t in tri] == exp_tri


def _fd(params, s, res, A, k, h=1e-4, order=2):
    out = []
    for sg in (+1, -1):
        sp = w.System(s.name, s.Z, s.xyz.copy(), s.frag, s.frag_charge)
        sp.xyz[A, k] += sg * h
        out.append(F.fmo(sp, params, 0.0, order=order, lists=res.lists, scc_tol=1e-12, macro_tol=1e-12).E)
    return (out[0] - out[1]) / (2 * h)


def test_fmo2_gradient_fd(params, c1):
    s = c1.subset([0, 1, 2, 3])
    r = F.fmo(s, params, 4 * A2B, scc_tol=1e-12, macro_tol=1e-12)
    assert len(r.lists[0]) > 0 and len(r.lists[1]) > 0
    g, _ = F.fmo2_gradient(s, params, r)
    g0, _ = F.fmo2_gradient(s, params, r, with_response=False)
    err, err0 = [], []
    for A in range(s.n_atoms):
        for k in range(3):
            fd = _fd(params, s, r, A, k)
            err.append(fd - g[A, k])
            err0.append(fd - g0[A, k])
    err, err0 = np.abs(err), np.abs(err0)
    assert err.max() < 2e-8
    assert err0.max() > 1e-6          # the response term is needed
    assert np.max(np.abs(g.sum(0))) < 1e-10
    assert np.max(np.abs(np.cross(s.xyz, g).sum(0))) < 1e-9


def _near_vdw_bruteforce(s, r, lam):
    """Definition, pair by pair: some atom pair closer than lam (r_a + r_b)."""
    out = {}
    for I in range(s.n_frag):
        for J in range(I + 1, s.n_frag):
            out[(I, J)] = int(any(
                float(np.linalg.norm(s.xyz[a] - s.xyz[b])) < lam * (r[a] + r[b])
                for a in np.where(s.frag == I)[0] for b in np.where(s.frag == J)[0]))
    return out


def test_lists_vdw_bruteforce(params, c1):
    r = F.vdw_radii(c1, params)
    assert r[c1.Z == 1][0] == pytest.approx(1.20 * A2B) and r[c1.Z == 8][0] == pytest.approx(1.52 * A2B)
    lam2, lam3 = 2.0, 1.5
    scc, esd, tri = F.build_lists(c1, 0.0, order=3, vdw=(r, lam2, lam3))
    n2 = _near_vdw_bruteforce(c1, r, lam2)
    n3 = _near_vdw_bruteforce(c1, r, lam3)
    assert [tuple(p) for p in scc] == [k for k, v in n2.items() if v]
    assert [tuple(p) for p in esd] == [k for k, v in n2.items() if not v]
    exp_tri = [(I, J, K) for I in range(8) for J in range(I + 1, 8) for K in range(J + 1, 8)
               if n3[(I, J)] + n3[(I, K)] + n3[(J, K)] >= 2]
    assert [tuple(t) for t in tri] == exp_tri
    assert 0 < len(scc) < 28 and 0 < len(tri)


def test_lists_vdw_equal_radii_is_cutoff(c1):
    """With one radius r0 for every atom the scaled test is a closest-contact
    cutoff of 2 lam r0 (geometry checked to have no contact within 1e-6 bohr
    of that distance, so rounding cannot decide a pair)."""
    r0, cut = 1.5, 4 * A2B
    lam = cut / (2 * r0)
    d = np.linalg.norm(c1.xyz[:, None, :] - c1.xyz[None, :, :], axis=2)
    assert np.min(np.abs(d - cut)) > 1e-6
    r = np.full(c1.n_atoms, r0)
    a = F.build_lists(c1, cut, order=3)
    b = F.build_lists(c1, 0.0, order=3, vdw=(r, lam, lam))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_lists_vdw_monotone(params, c1):
    r = F.vdw_radii(c1, params)
    prev = set()
    for lam in (0.01, 0.8, 1.2, 1.6, 2.0, 3.0, 100.0):
        scc = {tuple(p) for p in F.build_lists(c1, 0.0, vdw=(r, lam, lam))[0]}
        assert prev <= scc
        prev = scc
    assert len(F.build_lists(c1, 0.0, vdw=(r, 0.01, 0.01))[0]) == 0
    assert len(prev) == 28


def test_two_multimolecule_fragments_fmo2_exact(params, c1):
    """Fragments of four waters (the paper's fragment-size study uses 1-12
    waters per fragment): with two fragments and their SCC dimer, FMO2 is xTB
    of the union."""
    s = c1.grouped(4)
    assert s.n_frag == 2 and np.all(np.bincount(s.frag) == 12)
    r = F.fmo(s, params, 100.0)
    assert len(r.lists[0]) == 1
    assert abs(r.E - F.xtb_energy(s, params)[0]) < 1e-9


def test_fmo3_gradient_three_fragments_is_xtb(params, c1):
    s = c1.subset([0, 1, 2])
    r = F.fmo(s, params, 100.0, order=3, scc_tol=1e-12, macro_tol=1e-12)
    assert len(r.lists[2]) == 1
    g, _ = F.fmo_gradient(s, params, r)
    _, gx = F.xtb_gradient(s, params, tol=1e-12)
    assert np.max(np.abs(g - gx)) < 1e-8


def test_fmo3_gradient_fd(params, c1):
    s = c1.subset([0, 2, 3, 5, 6])
    r = F.fmo(s, params, 5.5 * A2B, order=3, scc_tol=1e-12, macro_tol=1e-12)
    scc = {tuple(p) for p in r.lists[0]}
    subs = [P for t in r.lists[2] for P in ((t[0], t[1]), (t[0], t[2]), (t[1], t[2]))]
    assert len(r.lists[2]) >= 3
    assert any(P not in scc for P in subs)                  # ES-DIM sub-pair inside a trimer
    assert max(subs.count(P) for P in scc) >= 2             # SCC pair shared by trimers (s_IJ < 0)
    g, _ = F.fmo_gradient(s, params, r)
    g0, _ = F.fmo_gradient(s, params, r, with_response=False)
    rng = np.random.default_rng(5)
    coords = [(int(a), int(k)) for a, k in zip(rng.choice(s.n_atoms, 8, replace=False), rng.integers(0, 3, 8))]
    err, err0 = [], []
    for A, k in coords:
        fd = _fd(params, s, r, A, k, order=3)
        err.append(fd - g[A, k])
        err0.append(fd - g0[A, k])
    err, err0 = np.abs(err), np.abs(err0)
    assert err.max() < 2e-8, err
    assert err0.max() > 1e-7
    assert np.max(np.abs(g.sum(0))) < 1e-10
    assert np.max(np.abs(np.cross(s.xyz, g).sum(0))) < 1e-9
