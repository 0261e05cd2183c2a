"""Molecular dynamics on the FMO energy surface (oracle; test infrastructure
only, never called by the GPU library).

The paper derives the analytic gradient to make molecular dynamics of large
systems routine (section "Analytic energy gradients"; the conclusion).  The
integrator is plain velocity Verlet in atomic units (bohr, electron masses,
hbar/Eh):
    x_{n+1} = x_n + v_n dt - g_n / (2 m) dt^2,
    v_{n+1} = v_n - (g_n + g_{n+1}) / (2 m) dt,
with g = dE/dx.  Pinned in the CPU tests by exactness under a constant force,
time reversibility and the second-order energy error for a harmonic
potential.
"""

import numpy as np

from . import fmo as F

AMU_TO_ME = 1822.888486209        # atomic mass unit in electron masses (CODATA 2018)
MASS_AMU = {1: 1.00794, 6: 12.0107, 7: 14.0067, 8: 15.9994}


def masses_au(Z):
    return np.array([MASS_AMU[int(z)] for z in Z]) * AMU_TO_ME


def velocity_verlet(energy_grad, x0, v0, m, dt, n_steps):
    """energy_grad(x) -> (E, dE/dx); x, v of shape (N, 3), m of shape (N,).
    Returns the final x, v and the potential and kinetic energies of every
    step (n_steps + 1 values)."""
    x = np.array(x0, dtype=float)
    v = np.array(v0, dtype=float)
    mm = np.asarray(m, dtype=float)[:, None]
    E, g = energy_grad(x)
    e_pot = [E]
    e_kin = [0.5 * float(np.sum(mm * v * v))]
    for _ in range(n_steps):
        x = x + v * dt - 0.5 * g / mm * dt * dt
        E, gn = energy_grad(x)
        v = v - 0.5 * (g + gn) / mm * dt
        g = gn
        e_pot.append(E)
        e_kin.append(0.5 * float(np.sum(mm * v * v)))
    return x, v, np.array(e_pot), np.array(e_kin)


def fmo_energy_grad(system, params, cutoff_bohr, order=2, vdw=None):
    """x -> (FMO energy, analytic gradient) of `system` moved to x, with the
    pair and trimer lists rebuilt at every geometry."""
    def f(x):
        s = type(system)(system.name, system.Z, np.array(x, dtype=float), system.frag, system.frag_charge)
        lists = F.build_lists(s, cutoff_bohr, order, vdw=vdw)
        r = F.fmo(s, params, cutoff_bohr, order=order, lists=lists)
        g, _ = F.fmo_gradient(s, params, r)
        return r.E, g
    return f
