"""Covalent fragmentation with hybrid-orbital projectors (oracle pins).

Section "Covalent bond fragmentation": the detached atom (BDA) keeps its
fragment and gives one electron to the bond, a ghost copy of it in the
attached atom's fragment carries one electron, and V_HOP = S D S projects the
bond hybrid out of the BDA's occupied space and everything but the bond
hybrid out of the ghost's.  Pins:
* two fragments: the single dimer heals the bond, so FMO2 equals xTB of the
  union (independent of the monomer treatment);
* three fragments in a chain: FMO3 equals xTB of the union (the trimer heals
  both bonds; the non-adjacent dimer keeps one detached atom and one ghost);
* the projected hybrid carries no charge: h^T S P S h -> 0 on the BDA, the
  complement is empty on the ghost (both O(1/V_HOP));
* the projector acts as a penalty: energies approach the V_HOP -> infinity
  limit as 1/V_HOP (successive differences shrink tenfold), with a residual
  below 1e-6 Eh at V_HOP = 1e6 Eh;
* electron bookkeeping: every fragment is closed shell and its Mulliken
  charges sum to minus its net charge.
"""

import copy

import numpy as np
import pytest

import workloads as w
from oracle import fmo as F
from oracle import xtb as X

A2B = w.ANGSTROM_TO_BOHR


def test_helix_geometry():
    s = w.alanine_helix(5)
    assert s.n_atoms == 10 * 5 + 3
    assert s.n_frag == 5 and len(s.bonds) == 4
    d = np.linalg.norm(s.xyz[:, None] - s.xyz[None], axis=2) / A2B
    for a, b in s.bonds:
        assert s.Z[a] == 6 and s.Z[b] == 6
        assert abs(d[a, b] - 1.525) < 1e-9
        assert s.frag[b] == s.frag[a] + 1
    np.fill_diagonal(d, 9.0)
    assert d.min() > 0.95


def _mono_systems(params, s):
    cn = X.coordination_numbers(params, s.Z, s.xyz)
    ext = F.ExtendedAtoms(s, cn)
    out = []
    for I in range(s.n_frag):
        atoms, hop, healed = ext.layout((I,))
        assert len(healed) == 0
        out.append((F._system_for(params, ext, atoms, int(s.frag_charge[I]), hop), hop))
    return out


def test_fmo2_two_fragments_equals_xtb(params):
    s = w.alanine_helix(2)
    e_x = F.xtb_energy(s, params)[0]
    r = F.fmo(s, params, 4 * A2B, order=2)
    assert abs(r.E - e_x) < 1e-9


@pytest.mark.slow
def test_fmo3_three_fragments_equals_xtb(params):
    s = w.alanine_helix(3)
    e_x = F.xtb_energy(s, params)[0]
    r = F.fmo(s, params, 4 * A2B, order=3)
    assert len(r.lists[2]) == 1
    assert abs(r.E - e_x) < 1e-9
    # FMO2 alone is not exact for three fragments
    assert abs(r.E_fmo2 - e_x) > 1e-5


def test_projector_removes_hybrid(params):
    s = w.alanine_helix(3)
    for sx, hop in _mono_systems(params, s):
        res = X.scc(sx)
        SPS = sx.S @ res.P @ sx.S
        nel = res.occ.sum()
        assert abs(nel - sx.nel) < 1e-10 and round(nel) % 2 == 0
        assert abs(res.q.sum() + sx.charge) < 1e-10
        for A, kind, b in hop:
            h = sx.hybrid(A, b)
            pop = float(h @ SPS @ h)
            if kind == "bda":
                assert abs(pop) < 1e-8
            else:
                blk = slice(sx.ao_off[A], sx.ao_off[A + 1])
                comp = float(np.trace(SPS[blk, blk])) - pop
                assert abs(comp) < 1e-8
                assert 0.3 < pop < 2.0


def test_vhop_limit(params):
    """The projector is a penalty V_HOP |h><h|: the energy approaches its
    V -> infinity limit as c / V_HOP (second-order coupling through the
    shifted hybrid), so successive differences for V, 10 V, 100 V shrink by
    10 each, and the residual at 1e6 Eh is below 1e-6 Eh per fragment."""
    s = w.alanine_helix(2)
    E = []
    for scale in (1.0, 10.0, 100.0):
        pp = copy.copy(params)
        pp.VHOP = scale * params.VHOP
        E.append([X.scc(sx).e_int for sx, _ in _mono_systems(pp, s)])
    E = np.array(E)
    d1 = E[0] - E[1]
    d2 = E[1] - E[2]
    assert np.all(np.abs(d1) < 1e-6)
    assert np.allclose(d1 / d2, 10.0, rtol=1e-2)


def _augmented_energy(s, p, cut, lists, **kw):
    r = F.fmo(s, p, cut, lists=lists, **kw)
    return r.E + F.hop_projector_energy(r)


@pytest.mark.parametrize("n_res", [2, 4])
def test_hop_gradient_finite_differences(params, n_res):
    """The FMO2 gradient with cut bonds (section "FMO-xTB HOP gradient") is
    the derivative of the energy plus the projector term sum_X w_X
    Tr(P_X V^HOP_X), the functional every fragment SCC makes stationary.
    Central differences (h = 2e-4 bohr, lists frozen) of that functional at
    V_HOP = 1e4 Eh, where the SCC converges to 1e-11 in the charges: the two
    ends of a cut bond and two other atoms, within 1e-7 Eh/bohr.  Ala2 heals
    its bond in the dimer; Ala4 also has dimers with a detached atom and a
    ghost (partial bonds).  Net force and torque vanish."""
    from threadpoolctl import threadpool_limits
    p = copy.copy(params)
    p.VHOP = 1e4
    s = w.alanine_helix(n_res)
    cut = 4 * A2B
    kw = dict(scc_tol=1e-11, macro_tol=1e-11, scc_etol=1e-12)
    with threadpool_limits(1):
        r = F.fmo(s, p, cut, **kw)
        assert r.macro_converged and r.all_scc_converged
        G, _ = F.fmo_gradient(s, p, r)
        assert np.max(np.abs(G.sum(0))) < 1e-9
        assert np.max(np.abs(np.cross(s.xyz, G).sum(0))) < 1e-8
        a0, a1 = (int(x) for x in s.bonds[0])
        coords = [(a0, 0), (a1, 1), (n_res * 5, 2), (s.n_atoms - 1, 1)]
        h = 2e-4
        for a, k in coords:
            e = []
            for sg in (1.0, -1.0):
                s2 = copy.deepcopy(s)
                s2.xyz[a, k] += sg * h
                e.append(_augmented_energy(s2, p, cut, r.lists, **kw))
            fd = (e[0] - e[1]) / (2 * h)
            assert abs(fd - G[a, k]) < 1e-7, (a, k, fd, G[a, k])
