"""Boundary discretisations and the seeded random geometries.

Curves are circles and ellipses, discretised by equispaced parameter values
with the trapezoid rule (weight = parameter step times speed), as the paper
does for its spline curves in Section 4 ("non-uniform trapezoid quadrature"),
but with analytic curves since the paper's spline knots are not given.

Orientation convention: the normal at every node points out of the fluid
domain, i.e. outward on the outer curve and into each hole.  Curvature is
signed: positive where the curve bends away from that normal (outer circle of
radius R: +1/R), negative on holes.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class Curve:
    """One closed curve: an ellipse with semi-axes (a, b) rotated by theta."""

    n: int
    a: float
    b: float
    theta: float
    cx: float
    cy: float
    hole: bool

    @property
    def extent(self) -> float:
        return max(self.a, self.b)


@dataclass
class Geometry:
    """Concatenated boundary nodes of an outer curve followed by its holes."""

    xy: np.ndarray          # (N, 2) float64 node positions
    normal: np.ndarray      # (N, 2) unit normals, out of the fluid
    weight: np.ndarray      # (N,) trapezoid weights
    curvature: np.ndarray   # (N,) signed curvature
    curve_id: np.ndarray    # (N,) int32: 0 = outer curve, h = hole h (1-based)
    hole_xy: np.ndarray     # (p, 2) one interior point per hole (its centre)
    curves: List[Curve] = field(default_factory=list)
    root: Optional[np.ndarray] = None  # optional fixed root square (cx, cy, side)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_holes(self) -> int:
        return int(self.hole_xy.shape[0])

    @property
    def n_dofs(self) -> int:
        return 2 * self.n_nodes

    @property
    def n_system(self) -> int:
        return 2 * self.n_nodes + 3 * self.n_holes


def ellipse_nodes(n: int, a: float, b: float, theta: float, cx: float, cy: float,
                  hole: bool):
    """Nodes, normals, weights and signed curvature of one ellipse.

    Parameter t_k = 2 pi k / n, position c + R_theta (a cos t, b sin t).
    """
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    ct, st = np.cos(t), np.sin(t)
    c, s = np.cos(theta), np.sin(theta)
    px, py = a * ct, b * st
    dx, dy = -a * st, b * ct                      # d/dt of (px, py)
    ox, oy = b * ct, a * st                       # outward (unnormalised) normal
    speed = np.hypot(dx, dy)
    xy = np.stack([cx + c * px - s * py, cy + s * px + c * py], axis=1)
    nrm = np.stack([c * ox - s * oy, s * ox + c * oy], axis=1) / speed[:, None]
    w = 2.0 * np.pi * speed / n
    kap = a * b / speed ** 3
    if hole:
        nrm = -nrm
        kap = -kap
    return xy, nrm, w, kap


def starfish_nodes(n: int, radius: float, amp: float, arms: int, theta: float, cx: float, cy: float,
                   hole: bool):
    """Nodes, normals, weights and signed curvature of a starfish curve.

    Polar radius r(t) = radius (1 + amp cos(arms t)) at parameter t_k = 2 pi k / n,
    rotated by theta about its centre (cx, cy); trapezoid weights, analytic
    normal and curvature (the convention of the module docstring).
    """
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    r = radius * (1.0 + amp * np.cos(arms * t))
    r1 = -radius * amp * arms * np.sin(arms * t)
    r2 = -radius * amp * arms * arms * np.cos(arms * t)
    ct, st = np.cos(t), np.sin(t)
    px, py = r * ct, r * st
    dx, dy = r1 * ct - r * st, r1 * st + r * ct
    ddx = r2 * ct - 2.0 * r1 * st - r * ct
    ddy = r2 * st + 2.0 * r1 * ct - r * st
    speed = np.hypot(dx, dy)
    c, s = np.cos(theta), np.sin(theta)
    xy = np.stack([cx + c * px - s * py, cy + s * px + c * py], axis=1)
    ox, oy = dy / speed, -dx / speed                 # outward for the counter-clockwise curve
    nrm = np.stack([c * ox - s * oy, s * ox + c * oy], axis=1)
    w = 2.0 * np.pi * speed / n
    kap = (dx * ddy - dy * ddx) / speed ** 3
    if hole:
        nrm = -nrm
        kap = -kap
    return xy, nrm, w, kap


def starfish_geometry(n_total: int = 16384, theta1: float = 0.0, theta2: float = np.pi,
                      amp: float = 0.25, arms: int = 5, hole_scale: float = 0.16) -> Geometry:
    """The Laplace Neumann workload's boundary: a starfish (radius 1) holding two
    starfish holes 16 % of its size, with 2/3 of the nodes on the outer curve
    and 1/6 on each hole.  Hole h sits on the outer curve scaled by 1/2 at
    polar angle theta_h (the path the holes move along)."""
    n_out = int(round(2 * n_total / 3))
    n_h = (n_total - n_out) // 2
    n_out = n_total - 2 * n_h
    parts = [starfish_nodes(n_out, 1.0, amp, arms, 0.0, 0.0, 0.0, False)]
    holes = []
    for th in (theta1, theta2):
        rr = 0.5 * (1.0 + amp * np.cos(arms * th))
        cx, cy = rr * np.cos(th), rr * np.sin(th)
        parts.append(starfish_nodes(n_h, hole_scale, amp, arms, th, cx, cy, True))
        holes.append((cx, cy))
    xy = np.concatenate([q[0] for q in parts])
    return Geometry(
        xy=np.ascontiguousarray(xy),
        normal=np.ascontiguousarray(np.concatenate([q[1] for q in parts])),
        weight=np.concatenate([q[2] for q in parts]),
        curvature=np.concatenate([q[3] for q in parts]),
        curve_id=np.concatenate([np.full(n_out, 0, np.int32), np.full(n_h, 1, np.int32),
                                 np.full(n_h, 2, np.int32)]),
        hole_xy=np.array(holes, dtype=np.float64),
        curves=[],
    )


def build_geometry(curves: Sequence[Curve], root=None) -> Geometry:
    xs, ns, ws, ks, ids, holes = [], [], [], [], [], []
    h = 0
    for cv in curves:
        xy, nrm, w, kap = ellipse_nodes(cv.n, cv.a, cv.b, cv.theta, cv.cx, cv.cy, cv.hole)
        if cv.hole:
            h += 1
            holes.append((cv.cx, cv.cy))
            cid = h
        else:
            cid = 0
        xs.append(xy)
        ns.append(nrm)
        ws.append(w)
        ks.append(kap)
        ids.append(np.full(cv.n, cid, dtype=np.int32))
    return Geometry(
        xy=np.ascontiguousarray(np.concatenate(xs)),
        normal=np.ascontiguousarray(np.concatenate(ns)),
        weight=np.concatenate(ws),
        curvature=np.concatenate(ks),
        curve_id=np.concatenate(ids),
        hole_xy=np.array(holes, dtype=np.float64).reshape(-1, 2),
        curves=list(curves),
        root=None if root is None else np.asarray(root, dtype=np.float64),
    )


def single_ellipse(n: int = 2048, a: float = 1.0, b: float = 0.6) -> Geometry:
    return build_geometry([Curve(n, a, b, 0.0, 0.0, 0.0, False)])


def concentric_annulus(n_outer: int, n_inner: int, r_outer: float = 2.0,
                       r_inner: float = 1.0) -> Geometry:
    """Outer circle r_outer with one circular hole r_inner, both centred at 0."""
    return build_geometry([
        Curve(n_outer, r_outer, r_outer, 0.0, 0.0, 0.0, False),
        Curve(n_inner, r_inner, r_inner, 0.0, 0.0, 0.0, True),
    ])


def _place_holes(rng: np.random.Generator, radius: float, sizes: Sequence[int],
                 wall_gap: float = 0.5, hole_gap: float = 0.25,
                 axis_lo: float = 0.3, axis_hi: float = 0.8) -> List[Curve]:
    """Random non-overlapping ellipses inside a circle of the given radius.

    Semi-axes ~ U[axis_lo, axis_hi], angle ~ U[0, pi); centres by rejection so
    that |c| + max(a, b) <= radius - wall_gap and, for every pair,
    |c_i - c_j| >= max(a_i, b_i) + max(a_j, b_j) + hole_gap.
    """
    out: List[Curve] = []
    for n in sizes:
        while True:
            a = rng.uniform(axis_lo, axis_hi)
            b = rng.uniform(axis_lo, axis_hi)
            th = rng.uniform(0.0, np.pi)
            e = max(a, b)
            ok = False
            for _ in range(2000):
                c = rng.uniform(-radius, radius, size=2)
                if np.hypot(c[0], c[1]) + e > radius - wall_gap:
                    continue
                if all(np.hypot(c[0] - o.cx, c[1] - o.cy) >= e + o.extent + hole_gap
                       for o in out):
                    ok = True
                    break
            if ok:
                out.append(Curve(int(n), a, b, th, float(c[0]), float(c[1]), True))
                break
    return out


def random_holes_geometry(seed: int, radius: float, n_outer: int,
                          hole_sizes: Sequence[int]) -> Geometry:
    rng = np.random.Generator(np.random.PCG64(seed))
    curves = [Curve(n_outer, radius, radius, 0.0, 0.0, 0.0, False)]
    curves += _place_holes(rng, radius, hole_sizes)
    return build_geometry(curves)


def workload_small(seed: int = 11, n_outer: int = 256, n_holes: int = 2,
                   nodes_per_hole: int = 128, radius: float = 3.0) -> Geometry:
    """A small multiply-connected geometry for quick parity cases."""
    return random_holes_geometry(seed, radius, n_outer, [nodes_per_hole] * n_holes)


def workload_ellipse_2048() -> Geometry:
    """Single ellipse, semi-axes 1.0 and 0.6, 2048 nodes (4096 unknowns)."""
    return single_ellipse(2048, 1.0, 0.6)


def workload_circle10_8holes() -> Geometry:
    """Circle of radius 10 (4096 nodes) plus 8 random ellipses of 1024 nodes."""
    return random_holes_geometry(2, 10.0, 4096, [1024] * 8)


def workload_circle40_64holes() -> Geometry:
    """Circle of radius 40 (16384 nodes) plus 64 random ellipses of 1792 nodes."""
    return random_holes_geometry(3, 40.0, 16384, [1792] * 64)


def workload_batch_member(i: int, n_members: int = 512, radius: float = 10.0,
                          max_dofs: int = 65536) -> Geometry:
    """Member i of the many-geometry batch.

    p ~ U{1..16} holes; every curve gets U{8..64} * 64 nodes; the draw is
    repeated while the total unknown count 2 * sum(n) exceeds max_dofs.
    """
    ss = np.random.SeedSequence(4).spawn(n_members)[i]
    rng = np.random.Generator(np.random.PCG64(ss))
    while True:
        p = int(rng.integers(1, 17))
        sizes = [int(rng.integers(8, 65)) * 64 for _ in range(p + 1)]
        if 2 * sum(sizes) <= max_dofs:
            break
    curves = [Curve(sizes[0], radius, radius, 0.0, 0.0, 0.0, False)]
    curves += _place_holes(rng, radius, sizes[1:])
    return build_geometry(curves)


def move_hole(geom: Geometry, hole: int, rng: np.random.Generator,
              step: float = 0.05, dtheta: float = 0.1, radius: Optional[float] = None,
              wall_gap: float = 0.5, hole_gap: float = 0.25):
    """Translate hole `hole` (1-based) by step*N(0, I) and rotate it by U[-dtheta, dtheta].

    The move is redrawn while it violates the wall or hole gap.  Returns
    (new_geometry, moved_node_indices).  The root square is kept.
    """
    curves = list(geom.curves)
    outer = curves[0]
    R = outer.a if radius is None else radius
    ci = [i for i, c in enumerate(curves) if c.hole][hole - 1]
    old = curves[ci]
    while True:
        d = step * rng.standard_normal(2)
        th = old.theta + rng.uniform(-dtheta, dtheta)
        cand = Curve(old.n, old.a, old.b, th, old.cx + d[0], old.cy + d[1], True)
        if np.hypot(cand.cx, cand.cy) + cand.extent > R - wall_gap:
            continue
        if any(np.hypot(cand.cx - o.cx, cand.cy - o.cy) < cand.extent + o.extent + hole_gap
               for j, o in enumerate(curves) if o.hole and j != ci):
            continue
        break
    curves[ci] = cand
    new = build_geometry(curves, root=geom.root)
    start = sum(c.n for c in curves[:ci])
    return new, np.arange(start, start + old.n, dtype=np.int64)


def insert_hole(geom: Geometry, rng: np.random.Generator, n: int, radius: Optional[float] = None,
                wall_gap: float = 0.5, hole_gap: float = 0.25):
    """Add one random ellipse of n nodes (semi-axes U[0.3, 0.8], angle U[0, pi),
    centre by rejection against the wall and the other holes), appended after
    the existing curves.  Returns (new_geometry, old_of_new): old_of_new[j] is
    the old index of new node j, -1 for the new hole's nodes.  The root square
    is kept."""
    curves = list(geom.curves)
    R = curves[0].a if radius is None else radius
    others = [c for c in curves if c.hole]
    new_curve = None
    while new_curve is None:
        a, b = rng.uniform(0.3, 0.8), rng.uniform(0.3, 0.8)
        th = rng.uniform(0.0, np.pi)
        e = max(a, b)
        for _ in range(2000):
            c = rng.uniform(-R, R, size=2)
            if np.hypot(c[0], c[1]) + e > R - wall_gap:
                continue
            if all(np.hypot(c[0] - o.cx, c[1] - o.cy) >= e + o.extent + hole_gap for o in others):
                new_curve = Curve(int(n), a, b, th, float(c[0]), float(c[1]), True)
                break
    new = build_geometry(curves + [new_curve], root=geom.root)
    old_of_new = np.concatenate([np.arange(geom.n_nodes), np.full(n, -1)]).astype(np.int64)
    return new, old_of_new


def delete_hole(geom: Geometry, hole: int):
    """Remove hole `hole` (1-based).  The later curves' nodes move down in the
    numbering, keeping their order.  Returns (new_geometry, old_of_new)."""
    curves = list(geom.curves)
    ci = [i for i, c in enumerate(curves) if c.hole][hole - 1]
    start = sum(c.n for c in curves[:ci])
    cut = curves[ci].n
    new = build_geometry(curves[:ci] + curves[ci + 1:], root=geom.root)
    old_of_new = np.concatenate([np.arange(start), np.arange(start + cut, geom.n_nodes)]).astype(np.int64)
    return new, old_of_new
