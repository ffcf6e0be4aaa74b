"""Velocity-Verlet NVE reference driven by the C FP64 oracle's forces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One step: v += dt/2 F/m; x += dt v; F = F(x); v += dt/2 F/m, with
positions in Angstrom, velocities in Angstrom/fs, masses in amu and forces
in eV/Angstrom (1 eV/(Angstrom amu) = 9.648533212331e-3 Angstrom/fs^2).
Parity: the forces are the pinned force oracle's; the integrator is pinned
by second-order energy conservation on a smooth cluster (the error falls
as dt^2) and by time reversibility.
"""

import numpy as np

from . import d3_ref

ACC = 9.648533212331e-3
KE = 103.642691


def run(pos, vel, mass, types, cell, pbc, table, n_steps, dt, force_fn=None, **prm):
    """n_steps steps; forces from the C oracle, or from force_fn(pos) (a dict
    with "energy" and "forces") when it is given."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)[:, None]

    def forces(p):
        if force_fn is not None:
            return force_fn(p)
        return d3_ref.d3(p, types, cell, pbc, table, **prm)

    res = forces(pos)
    f = res["forces"]
    thermo = [(res["energy"], 0.5 * KE * float((m * vel * vel).sum()))]
    for _ in range(n_steps):
        vel += 0.5 * dt * ACC * f / m
        pos += dt * vel
        res = forces(pos)
        f = res["forces"]
        vel += 0.5 * dt * ACC * f / m
        thermo.append((res["energy"], 0.5 * KE * float((m * vel * vel).sum())))
    return pos, vel, np.array(thermo)
