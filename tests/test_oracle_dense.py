"""Pins of the dense augmented system (eq. backwardeq) against exact Stokes flows.

* Point forces outside the fluid (Section 3.1): the solved representation
  reproduces the exact interior velocity, and the augmented unknowns equal
  the force (alpha_h) and torque (beta_h, about c_h) of the forces enclosed
  by hole h, which is how the paper characterises Stokeslet and rotlet
  strengths.
* Couette flow between concentric circles (Section 4.1): closed-form
  velocity, alpha = 0, beta = 4 pi B (tests/golden/couette_r1_1_r2_2.txt).
"""

import os

import numpy as np

from oracle import stokes
from workloads import (boundary_data, concentric_annulus, exterior_forces_for_geometry,
                       stokeslet_velocity, workload_small, single_ellipse)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals


def _interior_targets(g, n=40, seed=0, margin=0.45):
    rng = np.random.Generator(np.random.PCG64(seed))
    R = g.curves[0].a
    out = []
    while len(out) < n:
        p = rng.uniform(-R, R, size=2)
        if np.hypot(*p) > R - margin:
            continue
        ok = True
        for c in g.curves[1:]:
            # distance test in the ellipse frame, with a margin
            cs, sn = np.cos(c.theta), np.sin(c.theta)
            d = p - np.array([c.cx, c.cy])
            lx, ly = cs * d[0] + sn * d[1], -sn * d[0] + cs * d[1]
            if (lx / (c.a + margin)) ** 2 + (ly / (c.b + margin)) ** 2 < 1.0:
                ok = False
                break
        if ok:
            out.append(p)
    return np.array(out)


def test_point_force_solution_multiply_connected():
    g = workload_small(seed=11, n_outer=256, n_holes=2, nodes_per_hole=128, radius=3.0)
    cols = exterior_forces_for_geometry(g, 3, seed=5)
    f = boundary_data(g, cols)
    x = stokes.dense_solve(g, f)
    n = g.n_dofs
    tg = _interior_targets(g)
    u = stokes.evaluate_interior(g, x, tg)
    for c, forces in enumerate(cols):
        ex = stokeslet_velocity(tg, forces)
        assert np.abs(u[:, :, c] - ex).max() < 1e-9 * np.abs(ex).max()
        lam = x[n:, c].reshape(-1, 3)
        for h in range(g.n_holes):
            F = sum((pf.g for pf in forces if pf.hole == h + 1), np.zeros(2))
            cc = g.hole_xy[h]
            tq = sum(((pf.z - cc)[0] * pf.g[1] - (pf.z - cc)[1] * pf.g[0]
                      for pf in forces if pf.hole == h + 1), 0.0)
            assert np.allclose(lam[h, :2], F, atol=1e-10)
            assert abs(lam[h, 2] - tq) < 1e-10
    # residual of the dense solve itself
    res = stokes.apply_system(g, x) - np.vstack([f, np.zeros((3 * g.n_holes, 3))])
    assert np.linalg.norm(res) < 1e-12 * np.linalg.norm(f)


def test_point_force_solution_simply_connected():
    g = single_ellipse(512, 1.0, 0.6)
    cols = exterior_forces_for_geometry(g, 2, seed=1)
    f = boundary_data(g, cols)
    x = stokes.dense_solve(g, f)
    tg = np.array([[0.0, 0.0], [0.5, 0.1], [-0.4, -0.2], [0.2, 0.3]])
    u = stokes.evaluate_interior(g, x, tg)
    for c, forces in enumerate(cols):
        ex = stokeslet_velocity(tg, forces)
        assert np.abs(u[:, :, c] - ex).max() < 1e-10 * np.abs(ex).max()


def test_couette_closed_form():
    gv = _golden("couette_r1_1_r2_2.txt")
    r1, r2, v1, v2 = gv["r1"], gv["r2"], gv["v1"], gv["v2"]
    A = (v2 * r2 - v1 * r1) / (r2 ** 2 - r1 ** 2)
    B = r1 * r2 * (v1 * r2 - v2 * r1) / (r2 ** 2 - r1 ** 2)
    assert abs(A - gv["A"]) < 1e-15 and abs(B - gv["B"]) < 1e-15
    g = concentric_annulus(512, 256, r_outer=r2, r_inner=r1)
    # tangential data: counter-clockwise unit tangent e_theta times the wall speed
    et = np.stack([-g.xy[:, 1], g.xy[:, 0]], axis=1) / np.hypot(g.xy[:, 0], g.xy[:, 1])[:, None]
    speed = np.where(g.curve_id == 0, v2, v1)
    f = (speed[:, None] * et).reshape(-1)
    x = stokes.dense_solve(g, f)
    n = g.n_dofs
    assert np.allclose(x[n:n + 2], [gv["alpha1"], gv["alpha2"]], atol=1e-10)
    assert abs(x[n + 2] - gv["beta"]) < 1e-9 * gv["beta"]
    rr = np.linspace(1.2, 1.8, 7)
    th = np.linspace(0.1, 6.0, 7)
    tg = np.stack([rr * np.cos(th), rr * np.sin(th)], axis=1)
    u = stokes.evaluate_interior(g, x, tg)[:, :, 0]
    ut = (A * rr + B / rr)[:, None] * np.stack([-np.sin(th), np.cos(th)], axis=1)
    assert np.abs(u - ut).max() < 1e-10
