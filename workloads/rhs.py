"""Boundary data from exact Stokes flows.

A point force g at z (the 2D Stokeslet, unit viscosity) generates the velocity
    u(x) = (1/(4 pi)) * ( -ln|r| I + r r^T / |r|^2 ) g,   r = x - z,
which solves the Stokes equations away from z.  With every z outside the
fluid (beyond the outer curve or inside a hole), u restricted to the boundary
is Dirichlet data whose interior solution is u itself; this is the workload's
right-hand side.  Random draws are seeded and documented with each function.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from .geometry import Geometry


@dataclass
class PointForce:
    z: np.ndarray      # (2,) location, outside the fluid
    g: np.ndarray      # (2,) force vector
    hole: int          # 0 = beyond the outer curve, h = inside hole h (1-based)


def stokeslet_velocity(targets: np.ndarray, forces: Sequence[PointForce]) -> np.ndarray:
    """Velocity (M, 2) at targets (M, 2) due to a list of point forces."""
    x = np.asarray(targets, dtype=np.float64)
    u = np.zeros_like(x)
    for pf in forces:
        r = x - pf.z[None, :]
        r2 = np.einsum("ij,ij->i", r, r)
        rg = r @ pf.g
        u += (-0.5 * np.log(r2)[:, None] * pf.g[None, :] + r * (rg / r2)[:, None]) / (4.0 * np.pi)
    return u


def boundary_data(geom: Geometry, columns: Sequence[Sequence[PointForce]]) -> np.ndarray:
    """Right-hand sides f, shape (2N, ncols), DOF 2j = x-velocity of node j, 2j+1 = y."""
    f = np.empty((geom.n_dofs, len(columns)), dtype=np.float64)
    for c, forces in enumerate(columns):
        f[:, c] = stokeslet_velocity(geom.xy, forces).reshape(-1)
    return f


def exterior_forces_for_geometry(geom: Geometry, ncols: int, seed: int) -> List[List[PointForce]]:
    """Seeded point forces for `ncols` right-hand sides.

    Generator: numpy PCG64 seeded with [seed, 1].  Forces g ~ N(0, I2).
    * No holes: each column sums 3 forces at radius rho ~ U[1.5 E, 3 E],
      angle ~ U[0, 2 pi), E = outer curve's largest semi-axis.
    * With holes: each column sums one force beyond the outer curve at
      rho ~ U[1.1 R, 1.5 R] plus one inside each of two distinct holes (one if
      p = 1), at c_h + R_theta (0.4 a cos phi, 0.4 b sin phi).
    """
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    outer = geom.curves[0]
    holes = [c for c in geom.curves if c.hole]
    E = outer.extent
    cols: List[List[PointForce]] = []
    for _ in range(ncols):
        forces: List[PointForce] = []
        if not holes:
            for _k in range(3):
                rho = rng.uniform(1.5 * E, 3.0 * E)
                phi = rng.uniform(0.0, 2.0 * np.pi)
                z = np.array([outer.cx + rho * np.cos(phi), outer.cy + rho * np.sin(phi)])
                forces.append(PointForce(z, rng.standard_normal(2), 0))
        else:
            rho = rng.uniform(1.1 * E, 1.5 * E)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            z = np.array([outer.cx + rho * np.cos(phi), outer.cy + rho * np.sin(phi)])
            forces.append(PointForce(z, rng.standard_normal(2), 0))
            k = min(2, len(holes))
            pick = rng.choice(len(holes), size=k, replace=False)
            for h in pick:
                cv = holes[int(h)]
                phi = rng.uniform(0.0, 2.0 * np.pi)
                c, s = np.cos(cv.theta), np.sin(cv.theta)
                lx, ly = 0.4 * cv.a * np.cos(phi), 0.4 * cv.b * np.sin(phi)
                z = np.array([cv.cx + c * lx - s * ly, cv.cy + s * lx + c * ly])
                forces.append(PointForce(z, rng.standard_normal(2), int(h) + 1))
        cols.append(forces)
    return cols


def neumann_flux(curve_id) -> np.ndarray:
    """The heat-flux data of the Laplace Neumann workload (eq. (neumanndata) of
    Section 4.4.1): 0 on the outer curve, +1 on the first hole, -1 on the
    second."""
    c = np.asarray(curve_id)
    return np.where(c == 1, 1.0, np.where(c == 2, -1.0, 0.0))
