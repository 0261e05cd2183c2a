"""FMO2 / FMO3 energies and the FMO2 analytic gradient (oracle).

Passages followed:
* fragment pair lists (section "Computational Details"): a pair is a full
  SCC dimer when it passes the contact test, otherwise ES-DIM; a trimer is
  computed when at least two of its three pairs pass the trimer test.  Two
  tests: a fixed closest-contact cutoff (4 Angstrom by default, both tests
  alike), or the paper's van der Waals-scaled contacts: some atom pair closer
  than lam (r_a + r_b), lam = 2.0 for dimers and 1.5 for trimers;
* embedding potential, eq. v_esp_matrix: each fragment sees
  phi_s = sum_{K != I} sum_{t in K} gamma_st dq^K_t in its Fock matrix;
* monomer self-consistency (section "FMO-xTB"): monomers are solved
  repeatedly in the field of the others until all charges are converged
  (sweeps with fully converged inner SCC; the sweep map is driven to its
  fixed point by Anderson mixing of the monomer charges);
* FMO2 energy, eq. fmo2-energy-components, with the embedding correction
  eq. dimer_embedding_correction and the charge transfer eq. ddq_calc;
  E_I, E_IJ are read as internal energies (embedding acts in the Fock matrix
  only), the reading consistent with the printed Delta E^V and ES-DIM forms;
* ES-DIM, eq. esdimer-energy: Delta E_IJ = dq^I gamma_IJ dq^J;
* FMO3 energy, eqs. fmo3_energy, trimer_interaction_energy, trimer_embedding
  (the embedding sum of E^V_{X,Y} read as K not in Y); an ES-DIM sub-pair
  enters the trimer subtraction with its ES-DIM value;
* FMO2 gradient, section "Analytic energy gradients": the explicit terms
  eqs. pair_delta, ctij, esd_grad and the response through the Lagrangian
  potential eq. esp_lagrangian.  The gradient is assembled from the identity
      E = sum_I c_I E^emb_I + sum_SCC E^emb_IJ - sum_ESD dq^I gamma dq^J,
      c_I = 1 - (number of SCC dimers containing I),
  in which every E^emb_X is stationary in its own density, so the only
  implicit dependence is through the monomer charges, whose energy
  derivative is the potential v_K of eq. esp_lagrangian.  The charge response
  is solved in shell-charge space (the shell-summed transition charges Q of
  eq. lagrangian define the fragment susceptibility); this is equivalent to
  the Z-vector equations eq. sczv and gives the Z-vector Z_ai, the AO
  Z-density and the energy-weighted Z-density of eqs. Z_AO and WZ_def, which
  enter the derivative contractions of eqs. ZxHB .. ZxG_inter and the
  Mulliken (Lagrangian) term of eq. resp_addlag.
"""

import math
import multiprocessing

import numpy as np

from .xtb import (XtbSystem, coordination_numbers, cn_gradient, scc, gamma_matrix,
                  gamma_deriv, system_gradient)


def neumaier_sum(values):
    s = 0.0
    c = 0.0
    for v in values:
        v = float(v)
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


# --------------------------------------------------------------------------
# lists

def fragment_atoms(frag, n_frag):
    return [np.where(frag == I)[0] for I in range(n_frag)]


def closest_contact_sq(xyz, atoms_i, atoms_j):
    """Smallest squared interatomic distance between two atom sets, each term
    formed as (dx*dx + dy*dy) + dz*dz in FP64 (no fused multiply-add)."""
    a = xyz[atoms_i]
    b = xyz[atoms_j]
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    xx = dx * dx
    yy = dy * dy
    zz = dz * dz
    d2 = xx + yy
    d2 = d2 + zz
    return float(d2.min())


def vdw_contact(xyz, atoms_i, atoms_j, r, lam):
    """True when some atom pair a in I, b in J is closer than
    lam (r_a + r_b) (section "Computational Details"), compared as
    d2 < (lam (r_a + r_b))^2 with every operation rounded separately."""
    a = xyz[atoms_i]
    b = xyz[atoms_j]
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    t = lam * (r[atoms_i][:, None] + r[atoms_j][None, :])
    return bool(np.any(d2 < t * t))


def vdw_radii(system, params):
    """Van der Waals radius (bohr) of every atom, from the parameter file."""
    r = [params.element(int(z))["rvdw"] for z in system.Z]
    if any(v is None for v in r):
        raise KeyError("van der Waals radius missing from the parameters")
    return np.array(r, dtype=float)


def build_lists(system, cutoff_bohr, order=2, vdw=None):
    """SCC dimers, ES-DIM pairs (lexicographic, I < J) and, for order 3, the
    trimers (I < J < K) with at least two sub-pairs passing the trimer test.
    vdw = None: closest contact below cutoff_bohr for both tests;
    vdw = (radii_bohr, lam_dimer, lam_trimer): van der Waals-scaled contacts."""
    fa = fragment_atoms(system.frag, system.n_frag)
    F = system.n_frag
    c2 = cutoff_bohr * cutoff_bohr
    scc_pairs, esd_pairs = [], []
    near = np.zeros((F, F), dtype=bool)
    for I in range(F):
        for J in range(I + 1, F):
            if vdw is None:
                is_scc = closest_contact_sq(system.xyz, fa[I], fa[J]) < c2
                near[I, J] = near[J, I] = is_scc
            else:
                r, lam2, lam3 = vdw
                is_scc = vdw_contact(system.xyz, fa[I], fa[J], r, lam2)
                if order >= 3:
                    near[I, J] = near[J, I] = vdw_contact(system.xyz, fa[I], fa[J], r, lam3)
            if is_scc:
                scc_pairs.append((I, J))
            else:
                esd_pairs.append((I, J))
    trimers = []
    if order >= 3:
        for I in range(F):
            for J in range(I + 1, F):
                for K in range(J + 1, F):
                    if int(near[I, J]) + int(near[I, K]) + int(near[J, K]) >= 2:
                        trimers.append((I, J, K))
    return (np.array(scc_pairs, dtype=np.int32).reshape(-1, 2),
            np.array(esd_pairs, dtype=np.int32).reshape(-1, 2),
            np.array(trimers, dtype=np.int32).reshape(-1, 3))


# --------------------------------------------------------------------------
# the supersystem's shells

class ExtendedAtoms:
    """The supersystem's atoms followed by one ghost atom per cut covalent bond
    (section "Covalent bond fragmentation"): a copy of the detached atom (same
    element, position and supersystem CN) that belongs to the attached atom's
    fragment.  Without cut bonds this is the system itself."""

    def __init__(self, system, cn):
        b = np.asarray(system.bonds, dtype=np.int64).reshape(-1, 2)
        self.N = system.n_atoms
        self.bonds = b
        self.Z = np.concatenate([system.Z, system.Z[b[:, 0]]])
        self.xyz = np.concatenate([system.xyz, system.xyz[b[:, 0]]])
        self.frag = np.concatenate([system.frag, system.frag[b[:, 1]]]).astype(np.int64)
        self.cn = np.concatenate([cn, cn[b[:, 0]]])
        self.n_atoms = len(self.Z)
        self.frag_charge = system.frag_charge
        self.real_atoms = fragment_atoms(system.frag, system.n_frag)

    def bond_vector(self, k):
        a, b = self.bonds[k]
        v = self.xyz[b] - self.xyz[a]
        return v / np.linalg.norm(v)

    def layout(self, frags):
        """Atoms (extended indices) of the system made of `frags`, in basis
        order: per fragment its real atoms, then the ghosts of its cut bonds
        whose detached atom lies outside; the covalent-boundary list of that
        system; and the ghosts of bonds healed inside it (present in the
        monomers only)."""
        fs = set(int(f) for f in frags)
        fr = self.frag
        atoms = []
        for f in frags:
            atoms.extend(int(a) for a in self.real_atoms[f])
            for k, (a, b) in enumerate(self.bonds):
                if fr[b] == f and fr[a] not in fs:
                    atoms.append(self.N + k)
        pos = {a: i for i, a in enumerate(atoms)}
        hop, healed = [], []
        for k, (a, b) in enumerate(self.bonds):
            ina, inb = fr[a] in fs, fr[b] in fs
            if ina and not inb:
                hop.append((pos[int(a)], "bda", self.bond_vector(k)))
            elif inb and not ina:
                hop.append((pos[self.N + k], "ghost", self.bond_vector(k)))
            elif ina and inb:
                healed.append(self.N + k)
        return np.array(atoms, dtype=np.int64), hop, np.array(healed, dtype=np.int64)


class Shells:
    """Global shell table: shells of atom 0, then atom 1, ... (ghost atoms
    after the real ones); per shell the atom, its fragment and its hardness
    (1 + kappa) eta_A."""

    def __init__(self, params, system):
        self.p = params
        at, eta = [], []
        self.atom_sh0 = np.zeros(system.n_atoms + 1, dtype=np.int64)
        for A, z in enumerate(system.Z):
            e = params.element(int(z))
            for sh in e["shells"]:
                at.append(A)
                eta.append((1.0 + sh["kappa"]) * e["eta"])
            self.atom_sh0[A + 1] = len(at)
        self.atom = np.array(at)
        self.eta = np.array(eta)
        self.frag = system.frag[self.atom]
        self.xyz = system.xyz[self.atom]
        self.n = len(at)

    def of_atoms(self, atoms):
        return np.concatenate([np.arange(self.atom_sh0[a], self.atom_sh0[a + 1]) for a in atoms])

    def gamma_block(self, si, sj):
        d = self.xyz[si][:, None, :] - self.xyz[sj][None, :, :]
        R = np.sqrt(np.sum(d * d, axis=2))
        return gamma_matrix(self.p, R, self.eta[si][:, None], self.eta[sj][None, :])

    def potential(self, targets, q_all, exclude_mask_fn, chunk=4096):
        """phi_s = sum_t gamma_st q_t over sources t allowed by the mask."""
        out = np.zeros(len(targets))
        src = np.arange(self.n)
        for i0 in range(0, len(targets), chunk):
            tg = targets[i0:i0 + chunk]
            G = self.gamma_block(tg, src)
            G = np.where(exclude_mask_fn(tg[:, None], src[None, :]), 0.0, G)
            out[i0:i0 + chunk] = G @ q_all
        return out


# --------------------------------------------------------------------------
# optional process pool over fragments (the oracle's arithmetic is unchanged:
# every task is one monomer SCC, one cluster solve or one chunk of targets of
# an embedding-potential sum; results are gathered in input order)

_POOL_STATE = {}


def _pool_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


class _Runner:
    """map() over tasks, serially or with `workers` forked processes that see
    the module state set before the pool starts."""

    def __init__(self, workers):
        self.workers = int(workers or 1)
        self.pool = None

    def start(self, **state):
        _POOL_STATE.clear()
        _POOL_STATE.update(state)
        if self.workers > 1:
            self.close()
            ctx = multiprocessing.get_context("fork")
            self.pool = ctx.Pool(self.workers, initializer=_pool_init)

    def map(self, fn, tasks):
        if self.pool is None:
            return [fn(t) for t in tasks]
        return self.pool.map(fn, tasks, chunksize=1)

    def close(self):
        if self.pool is not None:
            self.pool.close()
            self.pool.join()
            self.pool = None


def _task_potential(args):
    i0, i1, q_all, mask = args
    sh = _POOL_STATE["sh"]
    if mask == "same_frag":
        fn = lambda s, t: sh.frag[s] == sh.frag[t]
    else:
        fn = lambda s, t: np.zeros_like(s, dtype=bool)
    return sh.potential(np.arange(i0, i1), q_all, fn, chunk=512)


def _field_all(runner, sh, q):
    """phi over every shell from the charges of the other fragments."""
    if runner.pool is None:
        same_frag = lambda s, t: sh.frag[s] == sh.frag[t]
        return sh.potential(np.arange(sh.n), q, same_frag)
    step = 2048
    tasks = [(i0, min(sh.n, i0 + step), q, "same_frag") for i0 in range(0, sh.n, step)]
    return np.concatenate(runner.map(_task_potential, tasks))


def _task_monomer(args):
    I, phi_I, guess = args
    st = _POOL_STATE
    r = scc(st["mono"][I], phi_I, q_guess=guess, tol=st["scc_tol"], etol=st["scc_etol"])
    return r if st["keep"] else SCCResultLight(r)


def _task_cluster(frags):
    st = _POOL_STATE
    out = _solve_cluster(st["params"], st["ext"], st["sh"], st["q"], st["frag_charge"],
                         st["scc_tol"], st["scc_etol"], frags)
    if not st["keep"]:
        sysX, rX, shl, ddq, dEV, atoms, hs = out
        return None, SCCResultLight(rX), shl, ddq, dEV, atoms, hs
    return out


class SCCResultLight:
    """The scalars and charges of a cluster solve (what the energy needs),
    without its matrices, for large runs."""

    def __init__(self, r):
        self.e_int = r.e_int
        self.q = r.q
        self.niter = r.niter
        self.converged = r.converged


def _solve_cluster(params, ext, sh, q, frag_charge, scc_tol, scc_etol, frags):
    """SCC of the cluster made of `frags` in the field of all other monomers
    (eqs. dimer_embedding_correction, ddq_calc; trimers alike)."""
    atoms, hop, healed = ext.layout(frags)
    shl = sh.of_atoms(atoms)
    inside = np.isin(sh.frag, np.asarray(frags))
    no_mask = lambda s, t: np.zeros_like(s, dtype=bool)
    q_out = np.where(inside, 0.0, q)
    phiX = sh.potential(shl, q_out, no_mask)
    sysX = _system_for(params, ext, atoms, int(sum(frag_charge[I] for I in frags)), hop)
    rX = scc(sysX, phiX, q_guess=q[shl], tol=scc_tol, etol=scc_etol)
    ddq = rX.q - q[shl]
    dEV = float(ddq @ phiX)
    hs = np.zeros(0, dtype=np.int64)
    if len(healed):
        # ghosts of bonds healed inside the cluster: their monomer charge is
        # the charge transfer, with the opposite sign (eq. ctij_ghost)
        hs = sh.of_atoms(healed)
        dEV += float(-q[hs] @ sh.potential(hs, q_out, no_mask))
    return sysX, rX, shl, ddq, dEV, atoms, hs


def _system_for(params, ext, atoms, charge, hop=None):
    return XtbSystem(params, ext.Z[atoms], ext.xyz[atoms], ext.cn[atoms], charge=charge, hop=hop)


class FMOResult:
    pass


def fmo(system, params, cutoff_bohr, order=2, lists=None, scc_tol=1e-10,
        macro_tol=1e-10, max_macro=200, verbose=False, workers=1, keep_clusters=True,
        scc_etol=1e-11):
    """FMO2 (order=2) or FMO3 (order=3) energy.  Returns an FMOResult with the
    converged monomer, dimer and trimer results and the energy terms.

    workers > 1 spreads the monomer solves, the cluster solves and the chunks
    of the embedding-potential sums over that many forked processes (same
    arithmetic, same order of every sum).  keep_clusters = False keeps only
    the energies and charges of the monomer and cluster solves (no matrices),
    for large systems whose gradient is not wanted.  The result records whether every
    solve converged (all_scc_converged) and the final monomer-loop change
    (macro_delta).  scc_tol and scc_etol are the charge and energy
    tolerances of every fragment SCC."""
    runner = _Runner(workers)
    try:
        return _fmo(system, params, cutoff_bohr, order, lists, scc_tol, scc_etol, macro_tol, max_macro,
                    verbose, runner, keep_clusters)
    finally:
        runner.close()


def _fmo(system, params, cutoff_bohr, order, lists, scc_tol, scc_etol, macro_tol, max_macro, verbose,
         runner, keep_clusters):
    F = system.n_frag
    cn = coordination_numbers(params, system.Z, system.xyz)
    ext = ExtendedAtoms(system, cn)
    lay = [ext.layout((I,)) for I in range(F)]
    fa = [l[0] for l in lay]
    sh = Shells(params, ext)
    fsh = [sh.of_atoms(fa[I]) for I in range(F)]
    if lists is None:
        lists = build_lists(system, cutoff_bohr, order)
    scc_pairs, esd_pairs, trimers = lists

    mono = [_system_for(params, ext, fa[I], int(system.frag_charge[I]), lay[I][1]) for I in range(F)]
    q = np.zeros(sh.n)   # superposition guess: zero shell charges
    res = [None] * F
    # Monomer self-consistency: every sweep solves all monomers in the field of
    # the current charges; the sweep map q -> q_out is driven to its fixed
    # point with Anderson (Pulay) mixing of the whole charge vector, which
    # also converges where plain repeated sweeps oscillate.
    X_h, R_h = [], []
    beta = 0.5
    runner.start(mono=mono, sh=sh, scc_tol=scc_tol, scc_etol=scc_etol, keep=keep_clusters)
    for it in range(1, max_macro + 1):
        phi = _field_all(runner, sh, q)
        qn = q.copy()
        tasks = [(I, phi[fsh[I]], res[I].q if res[I] is not None else q[fsh[I]]) for I in range(F)]
        res = runner.map(_task_monomer, tasks)
        for I in range(F):
            qn[fsh[I]] = res[I].q
        r = qn - q
        delta = float(np.max(np.abs(r)))
        if verbose:
            print("macro", it, delta)
        if delta < macro_tol:
            q = qn
            break
        X_h.append(q.copy())
        R_h.append(r)
        if len(X_h) > 8:
            X_h.pop(0)
            R_h.pop(0)
        m = len(X_h)
        if m == 1:
            q = q + beta * r
        else:
            M = np.zeros((m + 1, m + 1))
            M[:m, :m] = [[R_h[i] @ R_h[j] for j in range(m)] for i in range(m)]
            M[:m, m] = M[m, :m] = 1.0
            rhs = np.zeros(m + 1)
            rhs[m] = 1.0
            c = np.linalg.lstsq(M, rhs, rcond=None)[0][:m]
            q = sum(c[k] * (X_h[k] + beta * R_h[k]) for k in range(m))
    out = FMOResult()
    out.macro_iter = it
    out.macro_converged = delta < macro_tol
    out.macro_delta = delta
    # final embedding potential of every monomer (consistent with q)
    phi = _field_all(runner, sh, q)
    out.q = q
    out.phi_mono = phi
    out.cn = cn
    out.ext = ext
    out.mono = res
    out.mono_sys = mono
    out.frag_atoms = fa
    out.frag_shells = fsh
    out.shells = sh
    out.lists = lists
    out.E_mono = np.array([r.e_int for r in res])

    runner.start(params=params, ext=ext, sh=sh, q=q, frag_charge=system.frag_charge,
                 scc_tol=scc_tol, scc_etol=scc_etol, keep=keep_clusters)
    conv = [bool(r.converged) for r in res]

    out.dimers = []
    dE_scc = np.zeros(len(scc_pairs))
    solved = runner.map(_task_cluster, [(int(I), int(J)) for I, J in scc_pairs])
    for k, (I, J) in enumerate(scc_pairs):
        sysX, rX, shl, ddq, dEV, atoms, hs = solved[k]
        conv.append(bool(rX.converged))
        dE_scc[k] = rX.e_int - res[I].e_int - res[J].e_int + dEV
        # charge transfer on the cluster's shells and, with the opposite
        # monomer charge, on the ghosts of bonds healed inside it
        out.dimers.append(dict(I=int(I), J=int(J), sys=sysX, res=rX, shells=shl,
                               ddq=ddq, dEV=dEV, atoms=atoms,
                               ct_shells=np.concatenate([shl, hs]),
                               ct_ddq=np.concatenate([ddq, -q[hs]])))
    dE_esd = np.zeros(len(esd_pairs))
    for k, (I, J) in enumerate(esd_pairs):
        dE_esd[k] = float(q[fsh[I]] @ sh.gamma_block(fsh[I], fsh[J]) @ q[fsh[J]])
    out.dE_scc = dE_scc
    out.dE_esd = dE_esd
    out.E_fmo2 = neumaier_sum(list(out.E_mono) + list(dE_scc) + list(dE_esd))
    out.E = out.E_fmo2
    if order >= 3:
        pair_dE = {}
        for k, (I, J) in enumerate(scc_pairs):
            pair_dE[(int(I), int(J))] = dE_scc[k]
        for k, (I, J) in enumerate(esd_pairs):
            pair_dE[(int(I), int(J))] = dE_esd[k]
        out.trimers = []
        dE_tri = np.zeros(len(trimers))
        solved = runner.map(_task_cluster, [(int(I), int(J), int(K)) for I, J, K in trimers])
        for k, (I, J, K) in enumerate(trimers):
            sysX, rX, shl, ddq, dEV, atoms, hs = solved[k]
            conv.append(bool(rX.converged))
            dEIJK = rX.e_int - res[I].e_int - res[J].e_int - res[K].e_int + dEV
            dE_tri[k] = dEIJK - pair_dE[(I, J)] - pair_dE[(I, K)] - pair_dE[(J, K)]
            out.trimers.append(dict(IJK=(int(I), int(J), int(K)), sys=sysX, res=rX, shells=shl,
                                    ddq=ddq, dEIJK=dEIJK, atoms=atoms,
                                    ct_shells=np.concatenate([shl, hs]),
                                    ct_ddq=np.concatenate([ddq, -q[hs]])))
        out.dE_tri = dE_tri
        out.E_fmo3 = neumaier_sum([out.E_fmo2] + list(dE_tri))
        out.E = out.E_fmo3
    out.all_scc_converged = all(conv)
    return out


# --------------------------------------------------------------------------
# FMO2 gradient

def _ds_matrix(sig_ao, P, Wt):
    return 0.5 * (sig_ao[:, None] + sig_ao[None, :]) * P - Wt


def _inter_gamma_force(sh, pair_weights, natoms):
    """sum over listed shell pairs (s, t) of w_st d gamma_st / d R, as atom
    forces; pair_weights: list of (si, tj, W) with W of shape (len si, len tj).
    A pair at zero distance (a ghost shell and its detached atom, in different
    fragments) contributes nothing: gamma is smooth and even in R there."""
    g = np.zeros((natoms, 3))
    for si, tj, W in pair_weights:
        d = sh.xyz[si][:, None, :] - sh.xyz[tj][None, :, :]
        R = np.sqrt(np.sum(d * d, axis=2))
        Rs = np.where(R > 0.0, R, 1.0)
        dg = gamma_deriv(sh.p, Rs, sh.eta[si][:, None], sh.eta[tj][None, :])
        f = (np.where(R > 0.0, W * dg / Rs, 0.0))[:, :, None] * d   # d/dR_s of gamma_st
        np.add.at(g, sh.atom[si], f.sum(axis=1))
        np.add.at(g, sh.atom[tj], -f.sum(axis=0))
    return g


def _many_body_weights(F, scc_pairs, esd_pairs, trimers):
    """Coefficients of the embedded-energy identity.

    Writing every Delta E through embedded energies E^emb_X = E'_X + dq^X phi^X
    (eqs. fmo2-energy-components, dimer_embedding_correction,
    trimer_interaction_energy, fmo3_energy, with ES-DIM sub-pairs entering the
    trimer subtraction by their ES-DIM value) gives
        E = sum_I c_I E^emb_I + sum_SCC s_IJ E^emb_IJ + sum_T E^emb_IJK
            - sum_ESD (1 - n_T(IJ)) dq^I gamma dq^J,
    n_T(IJ) = number of trimers containing I and J, s_IJ = 1 - n_T(IJ),
    c_I = 1 - (SCC pairs containing I)
          + sum over trimers T containing I of (SCC sub-pairs of T containing I - 1).
    Without trimers this is the FMO2 identity (s = 1, c_I = 1 - n_I^SCC)."""
    scc = {(int(I), int(J)) for I, J in scc_pairs}
    nT = {}
    c = np.ones(F)
    for I, J in scc_pairs:
        c[I] -= 1.0
        c[J] -= 1.0
    for T in trimers:
        I, J, K = (int(x) for x in T)
        subs = [(I, J), (I, K), (J, K)]
        for P in subs:
            nT[P] = nT.get(P, 0) + 1
        for L in (I, J, K):
            c[L] += sum(1 for P in subs if L in P and P in scc) - 1.0
    s_scc = np.array([1.0 - nT.get((int(I), int(J)), 0) for I, J in scc_pairs])
    w_esd = np.array([1.0 - nT.get((int(I), int(J)), 0) for I, J in esd_pairs])
    return c, s_scc, w_esd


def _hop_bond_of(ext, atoms, sx, entry):
    """Cut bond (index into the system's bond list) of a boundary entry
    (local atom, kind, b) of system sx whose atoms are `atoms` (extended
    indices)."""
    A, kind, b = entry
    a = int(atoms[A])
    if kind == "ghost":
        return a - ext.N
    for k, (u, v) in enumerate(ext.bonds):
        if int(u) == a and np.allclose(ext.bond_vector(k), b, atol=0.0, rtol=0.0):
            return k
    raise ValueError("boundary atom without its cut bond")


def _hop_derivative_terms(ext, sx, atoms, Dm):
    """Explicit derivative of Tr(Dm V^HOP) at fixed Dm, V^HOP = S D S
    (eq. vhop), for a symmetric density-like matrix Dm of system sx:
    * overlap part (eq. hopsder): sum_mu,nu dS_mu,nu (Dm S D + D S Dm)_mu,nu,
      returned as that matrix, to be contracted with dS like the other
      overlap terms;
    * hybrid-coefficient part (eq. hopcoder): D = +-V h h^T (+ const), h =
      1/2 s + sqrt(3)/2 b.p on the boundary atom, b = (R_attached -
      R_detached) / |...|; d Tr(S Dm S D) = +-2 V (dh)^T (S Dm S) h with
      dh_p = sqrt(3)/2 db, db/dR_attached = (1 - b b^T) / |R|, on the
      attached atom and the opposite on the detached one (global real atoms),
      with + for a detached atom and - for a ghost.
    Returns (DS_add, forces (n_real, 3))."""
    N = ext.N
    g = np.zeros((N, 3))
    if not sx.hop:
        return np.zeros_like(sx.S), g
    D = sx.D_hop
    DS_add = Dm @ sx.S @ D + D @ sx.S @ Dm
    SDS = sx.S @ Dm @ sx.S
    V = sx.p.VHOP
    for entry in sx.hop:
        A, kind, b = entry
        k = _hop_bond_of(ext, atoms, sx, entry)
        a_det, a_att = int(ext.bonds[k][0]), int(ext.bonds[k][1])
        u = ext.xyz[a_att] - ext.xyz[a_det]
        L = float(np.linalg.norm(u))
        h = sx.hybrid(A, b)
        w = SDS @ h
        s_sh, p_sh = sx._hop_atom_layout(A)
        p0 = sx.sh_ao0[p_sh]
        wp = w[p0:p0 + 3]
        sign = 1.0 if kind == "bda" else -1.0
        bb = np.asarray(b, float)
        f = sign * 2.0 * V * (0.5 * math.sqrt(3.0)) / L * (wp - bb * (bb @ wp))
        g[a_att] += f
        g[a_det] -= f
    return DS_add, g


def _scatter_ghosts(ext, v):
    """Values on the extended atoms (real atoms, then one ghost per cut bond)
    summed onto the real atoms: a ghost sits on its detached atom."""
    out = np.array(v[:ext.N], copy=True)
    for k in range(len(ext.bonds)):
        out[int(ext.bonds[k][0])] += v[ext.N + k]
    return out


def hop_projector_energy(res):
    """sum_X w_X Tr(P_X V^HOP_X) over the monomers (w = c_I) and SCC dimers
    (w = 1) of an FMO2 result: the constraint term that the reported energy
    leaves out (section "FMO-xTB HOP energy") and that the SCC of every
    fragment makes stationary together with the energy."""
    F = len(res.mono)
    c, _, _ = _many_body_weights(F, res.lists[0], res.lists[1], [])
    e = 0.0
    for I in range(F):
        sx, r = res.mono_sys[I], res.mono[I]
        if sx.hop:
            e += c[I] * float(np.sum(r.P * sx.V_hop))
    for d in res.dimers:
        sx, r = d["sys"], d["res"]
        if sx.hop:
            e += float(np.sum(r.P * sx.V_hop))
    return e


def fmo_gradient(system, params, res, with_response=True):
    """Analytic FMO2 or FMO3 gradient (Eh/bohr, shape (natoms, 3)) for a
    converged result `res` (lists frozen).  From the identity of
    _many_body_weights, with every E^emb_X stationary in its own density:
        dE/dxi = sum_X w_X g^emb_X (explicit, at fixed monomer charges)
                 + sum_ESD (1 - n_T) dq^I dgamma dq^J
                 + sum_SCC s_IJ ddq^IJ . dphi^IJ + sum_T ddq^T . dphi^T
                 + response of the monomer charges,
    the response driven by v_K = sum over clusters X not containing K of
    w_X gamma_{K,X} ddq^X (eq. esp_lagrangian; for trimers the generalized
    accumulated charge transfer of section "Extension to FMO3").

    Cut covalent bonds (FMO2; section "FMO-xTB HOP gradient"): the systems
    are stationary for E^emb_X + Tr(P_X V^HOP_X), so this is the gradient of
    the reported energy plus hop_projector_energy (the two differ by terms
    of order 1/V_HOP).  Ghost shells are part of their monomer's charges;
    the ghost of a bond healed in a dimer carries the charge transfer
    -dq^ghost (eq. ctij_ghost); the projector derivative (eqs. hop_grad,
    hopsder, hopcoder) enters every system with the density and the
    response with the Z-vector density (eq. hop_resp); every ghost force
    acts on its detached atom."""
    if len(getattr(system, "bonds", ())) and len(res.lists[2]):
        raise NotImplementedError("FMO3 gradient with covalent boundaries")
    sh = res.shells
    ext = res.ext
    F = system.n_frag
    fa, fsh = res.frag_atoms, res.frag_shells
    q = res.q
    N = system.n_atoms
    Ne = ext.n_atoms
    scc_pairs, esd_pairs, trimers = res.lists
    tri = getattr(res, "trimers", [])
    if len(trimers) and len(tri) != len(trimers):
        raise ValueError("the result holds no trimer solutions (run fmo with order=3)")
    c, s_scc, w_esd = _many_body_weights(F, scc_pairs, esd_pairs, trimers if len(tri) else [])
    clusters = [(d, s_scc[k]) for k, d in enumerate(res.dimers)] + [(t, 1.0) for t in tri]

    G = np.zeros((N, 3))
    Fcn = np.zeros(Ne)
    parts = {}

    # explicit fragment terms: sum_X w_X g^emb_X (fixed CN), with sigma containing
    # the embedding potential (eqs. xtb_grad, W_matrix, pair_delta), plus the
    # projector derivative of systems with boundary atoms
    gm = np.zeros((Ne, 3))
    g_hop = np.zeros((N, 3))
    systems = [(res.mono_sys[I], res.mono[I], fa[I], c[I]) for I in range(F)]
    systems += [(d["sys"], d["res"], d["atoms"], wx) for d, wx in clusters]
    for sx, r, atoms, wx in systems:
        if wx == 0.0:
            continue
        DS = _ds_matrix(r.sigma[sx.ao_sh], r.P, r.Wt)
        dsh, gh = _hop_derivative_terms(ext, sx, atoms, r.P)
        g, f = system_gradient(sx, r.P, DS + dsh, r.q, r.q, True)
        gm[atoms] += wx * g
        Fcn[atoms] += wx * f
        g_hop += wx * gh
    parts["fragments"] = _scatter_ghosts(ext, gm) + g_hop
    G += parts["fragments"]

    # ES-DIM (eq. esd_grad) and charge-transfer embedding (eqs. ctij,
    # ctij_ghost and the FMO3 charge transfer) terms
    wl = []
    for k, (I, J) in enumerate(esd_pairs):
        if w_esd[k] != 0.0:
            wl.append((fsh[I], fsh[J], w_esd[k] * np.outer(q[fsh[I]], q[fsh[J]])))
    g_esd = _scatter_ghosts(ext, _inter_gamma_force(sh, wl, Ne))
    wl = []
    for d, wx in clusters:
        frags = d["IJK"] if "IJK" in d else (d["I"], d["J"])
        others = np.where(~np.isin(sh.frag, frags))[0]
        if wx != 0.0 and len(others):
            wl.append((d["ct_shells"], others, wx * np.outer(d["ct_ddq"], q[others])))
    g_ct = _scatter_ghosts(ext, _inter_gamma_force(sh, wl, Ne))
    parts["esd"] = g_esd
    parts["ct"] = g_ct
    G += g_esd + g_ct

    if with_response:
        g_resp, f_resp, info = _response(system, params, res, clusters)
        G += g_resp
        Fcn += f_resp
        parts["response"] = g_resp
        parts.update(info)

    # a ghost's CN is its detached atom's
    g_cn = cn_gradient(params, system.Z, system.xyz, _scatter_ghosts(ext, Fcn))
    parts["cn"] = g_cn
    G += g_cn
    return G, parts


def fmo2_gradient(system, params, res, with_response=True):
    """The FMO2 gradient (fmo_gradient of an FMO2 result)."""
    return fmo_gradient(system, params, res, with_response)


def lagrangian_potential(res, clusters=None):
    """v_K on the shells of every monomer K: the potential of the weighted
    charge transfer of all clusters not containing K (eq. esp_lagrangian;
    FMO2: all SCC dimers with weight 1)."""
    sh = res.shells
    if clusters is None:
        clusters = [(d, 1.0) for d in res.dimers]
    v = np.zeros(sh.n)
    for d, wx in clusters:
        frags = d["IJK"] if "IJK" in d else (d["I"], d["J"])
        tg = np.where(~np.isin(sh.frag, frags))[0]
        v[tg] += wx * (sh.gamma_block(tg, d["ct_shells"]) @ d["ct_ddq"])
    return v


def _monomer_response_blocks(sx, r):
    """Shell-summed transition charges Q_ai,s (eq. lagrangian), the
    susceptibility kernel M = sum_ai Q Q^T / (eps_a - eps_i) and the charge
    Hessian G = gamma - 2 Gamma_A dq_A (same-atom shell blocks)."""
    occ_mask = r.occ > 1.0
    Co = r.C[:, occ_mask]
    Cv = r.C[:, ~occ_mask]
    eo = r.eps[occ_mask]
    ev = r.eps[~occ_mask]
    SCo = sx.S @ Co
    SCv = sx.S @ Cv
    # per AO: C_mu,a (S C)_mu,i + C_mu,i (S C)_mu,a, summed over the AOs of a shell
    T = Cv[:, :, None] * SCo[:, None, :] + SCv[:, :, None] * Co[:, None, :]   # (n, nv, no)
    Q = np.zeros((sx.nsh, Cv.shape[1], Co.shape[1]))
    np.add.at(Q, sx.ao_sh, T)
    Q = Q.reshape(sx.nsh, -1)                                                   # (nsh, nv*no)
    D = (ev[:, None] - eo[None, :]).reshape(-1)
    M = (Q / D) @ Q.T
    qa = sx.atom_sum(r.q)
    Gm = sx.gamma.copy()
    same = sx.sh_atom[:, None] == sx.sh_atom[None, :]
    Gm -= np.where(same, 2.0 * (sx.at_Gamma * qa)[sx.sh_atom][:, None], 0.0)
    return dict(Q=Q, D=D, M=M, G=Gm, Co=Co, Cv=Cv, eo=eo, ev=ev)


def _response(system, params, res, clusters):
    sh = res.shells
    F = system.n_frag
    fa, fsh = res.frag_atoms, res.frag_shells
    N = system.n_atoms
    q = res.q
    v = lagrangian_potential(res, clusters)
    blocks = [_monomer_response_blocks(res.mono_sys[I], res.mono[I]) for I in range(F)]
    # susceptibility chi_K = -(1 + M G)^-1 M, block diagonal over fragments
    ns = sh.n
    chi = np.zeros((ns, ns))
    for I in range(F):
        b = blocks[I]
        k = len(fsh[I])
        chi[np.ix_(fsh[I], fsh[I])] = -np.linalg.solve(np.eye(k) + b["M"] @ b["G"], b["M"])
    # inter-fragment Coulomb coupling
    Goff = sh.gamma_block(np.arange(ns), np.arange(ns))
    Goff[sh.frag[:, None] == sh.frag[None, :]] = 0.0
    # adjoint of the monomer self-consistency: y = v + Goff chi y
    y = np.linalg.solve(np.eye(ns) - Goff @ chi, v)
    u = chi @ y
    ext = res.ext
    Ne = ext.n_atoms
    g = np.zeros((Ne, 3))
    g_hop = np.zeros((N, 3))
    Fcn = np.zeros(Ne)
    zinfo = []
    for I in range(F):
        sx, r, b = res.mono_sys[I], res.mono[I], blocks[I]
        yI = y[fsh[I]]
        w = np.linalg.solve(np.eye(len(yI)) + b["G"] @ b["M"], yI)
        Z = (-2.0 * (w @ b["Q"]) / b["D"]).reshape(b["Cv"].shape[1], b["Co"].shape[1])
        Zt = b["Cv"] @ Z @ b["Co"].T
        Zb = 0.5 * (Zt + Zt.T)
        WZ = b["Cv"] @ (Z * b["eo"][None, :]) @ b["Co"].T
        WZs = 0.5 * (WZ + WZ.T)
        QZ = np.bincount(sx.ao_sh, weights=np.sum(Zb * sx.S, axis=1), minlength=sx.nsh)
        sig = r.sigma[sx.ao_sh]
        wa = w[sx.ao_sh]
        P = r.P
        PSDP = P @ sx.S @ (wa[:, None] * P)
        DS = (0.5 * (sig[:, None] + sig[None, :]) * Zb - WZs
              + 0.5 * (wa[:, None] + wa[None, :]) * P - 0.25 * (PSDP + PSDP.T))
        # the projector derivative with the Z-vector density (eq. hop_resp)
        dsh, gh = _hop_derivative_terms(ext, sx, fa[I], Zb)
        gI, fI = system_gradient(sx, Zb, DS + dsh, 2.0 * QZ, r.q, with_rep=False)
        g[fa[I]] += gI
        Fcn[fa[I]] += fI
        g_hop += gh
        zinfo.append(dict(Z=Z, w=w))
    # inter-fragment kernel derivative with the response charges u
    wl = []
    for I in range(F):
        for K in range(I + 1, F):
            W = np.outer(u[fsh[I]], q[fsh[K]]) + np.outer(q[fsh[I]], u[fsh[K]])
            wl.append((fsh[I], fsh[K], W))
    g += _inter_gamma_force(sh, wl, Ne)
    return _scatter_ghosts(ext, g) + g_hop, Fcn, dict(v=v, y=y, u=u, zinfo=zinfo)


# --------------------------------------------------------------------------
# non-fragmented xTB of a whole system (reference for the exact special cases)

def xtb_energy(system, params, tol=1e-11):
    cn = coordination_numbers(params, system.Z, system.xyz)
    sx = XtbSystem(params, system.Z, system.xyz, cn, charge=int(system.frag_charge.sum()))
    r = scc(sx, tol=tol)
    return r.e_int, sx, r


def xtb_gradient(system, params, tol=1e-11):
    """Analytic gradient of a non-fragmented xTB system (eq. xtb_grad)."""
    e, sx, r = xtb_energy(system, params, tol)
    DS = _ds_matrix(r.sigma[sx.ao_sh], r.P, r.Wt)
    g, f = system_gradient(sx, r.P, DS, r.q, r.q, True)
    g += cn_gradient(params, system.Z, system.xyz, f)
    return e, g
