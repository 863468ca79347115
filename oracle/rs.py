"""Level-parallel recursive skeletonization with the bordered root solve.

TEST INFRASTRUCTURE ONLY (see the package header).

The factorization of Sections 2.2-2.7 applied to the top-left block
lam I + D + N of the augmented Stokes system, with H and Psi^T carried
through the transforms as in Section 3.2 (eq. bigskel, eq. partition).

Per box B of level l (l = L ... 1, all boxes of a level reading the
level-start set of active unknowns, Section 2.7):
  1. I_B: the box's active unknowns in ascending order (all unknowns of a
     leaf, else the union of its children's skeletons).
  2. Proxy circle (Section 2.5): centre of B, radius ratio * side, n_p
     equispaced points, outward normals.
  3. F_int: active unknowns not in I_B whose node lies strictly inside it.
  4. M_B = [A(F_int, B); A(B, F_int)^T; D(P, B); D(B, P)^T; S(B, P)^T;
            (w_j n_j^T)_B; w_B (n_j^T)_B]   (the stacked two-sided ID of
     Section 2.4 with the proxy rows of eq. greens; the last two rows carry
     the global rank-one N exactly).  Every row block is on the scale of one
     boundary interaction: the proxy points act as targets of B's sources
     with no weight of their own, and as sources for B's targets with weight
     w_B, the largest quadrature weight of B's active nodes, which also
     scales the target-side rank-one row.  The ID's relative tolerance is then
     relative to the size of the operator's own entries (a unit-scale row
     would set |R_11| and loosen the truncation of every kernel row by the
     ratio of the two scales).
  5. Pivoted QR of M_B -> rank k, skeleton S, redundant R, T (eq. lowrank).
  6. A_BB: leaf -> lam I + D + N; otherwise children's X_SS on their own
     diagonal blocks and original kernel entries between different children
     (eq. levelcompress).
  7. X_SR = A_SR - A_SS T, X_RS = A_RS - T^T A_SS,
     X_RR = A_RR - A_RS T - T^T X_SR                          (eq. tmat)
  8. LU of X_RR; if its reciprocal 1-norm condition number is below
     rcond_min, the next pivot moves from R to S and 7 repeats (the guard
     the paper asks for after eq. schurmat).
  9. E = X_SR X_RR^{-1}, F = X_RR^{-1} X_RS, X_SS = A_SS - X_SR F (eq. schurmat).
Root (eq. partition): p = 0 -> LU of X_SS; p > 0 -> Hh = U H, Ph = Psi^T V,
G = sum_B Ph(:, R_B) X_RR^{-1} Hh(R_B, :) and the LU of
Z = [[X_SS, Hh_S], [Ph_S, -I - G]].
Solve x = V X_D^{-1} U f (eq. kinv) with U applied leaf level first and V
level 1 first.

Updating (Section 2.8): after nodes move, the tree is rebuilt on the same
root square and, level by level, a box is recompressed exactly when an input
of its compression changed; every other box keeps its stored factors:
  * leaf: it is new, its node set changed, or one of its nodes moved;
  * parent: it is new, its set of children changed, or a child was
    recompressed (its skeleton or X_SS may differ);
  * any box: its near field F_int (ids, in order) changed, or a node of
    F_int moved.
Moved nodes outside the proxy circle act only through the proxy rows, which
is the locality the paper's updating relies on.  The root (and H, Psi^T)
is always redone.  With the same root the result equals a fresh
factorization of the new geometry.

Pins: dense LU agreement to O(eps) (P5), explicit U A V block-diagonal on
tiny inputs (P6), exact point-force solutions, update == refactor (P8).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla

from . import stokes
from .cpqr import PivotedQR
from .tree import Box, build_tree, depth


@dataclass
class RSParams:
    lam: float = -0.5
    tol: float = 1e-10
    leaf_size: int = 64
    n_proxy: int = 64
    proxy_ratio: float = 1.5
    rcond_min: float = 1e-12
    pivot: str = "max"            # pivot rule of the ID's QR (oracle.cpqr.PIVOT_RULES)
    level_parallel: bool = True   # False: the sequential scheme (each box sees the
                                  # active set left by the boxes before it)


@dataclass
class BoxFactor:
    box: int
    level: int
    I: np.ndarray                 # active unknowns of the box, ascending
    perm: np.ndarray              # positions into I: first k are S, the rest R
    k: int
    T: np.ndarray                 # k x r
    E: np.ndarray                 # k x r
    F: np.ndarray                 # r x k
    lu: Optional[tuple]           # LU of X_RR (None when r == 0)
    Xss: np.ndarray               # k x k, in S order
    Fint: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    rank0: int = 0                # rank from the tolerance alone (before the guard)
    m: int = 0                    # rows of the box's ID matrix M_B

    @property
    def S(self) -> np.ndarray:
        return self.I[self.perm[: self.k]]

    @property
    def R(self) -> np.ndarray:
        return self.I[self.perm[self.k:]]

    @property
    def r(self) -> int:
        return self.I.size - self.k


def proxy_circle(cx, cy, side, n_proxy, ratio):
    rp = ratio * side
    th = 2.0 * np.pi * np.arange(n_proxy) / n_proxy
    nrm = np.stack([np.cos(th), np.sin(th)], axis=1)
    pts = np.array([cx, cy])[None, :] + rp * nrm
    w = np.full(n_proxy, 2.0 * np.pi * rp / n_proxy)
    return pts, nrm, w, rp


def _cols(blk, cpos, ccomp):
    """(Mt, Mc, 2, 2) node blocks -> rows (2 i + a) x chosen columns (node cpos, comp ccomp)."""
    sel = blk[:, cpos, :, ccomp]            # (n, Mt, 2) after advanced indexing
    sel = np.moveaxis(sel, 0, -1)           # (Mt, 2, n)
    return sel.reshape(-1, cpos.size)


def _rows_t(blk, rpos, rcomp):
    """(Mb, Mt, 2, 2) blocks of K(B <- P) -> K(B, P)^T as rows (2 k + a) x columns of B."""
    sel = blk[rpos, :, rcomp, :]            # (n, Mt, 2): [b, k, a]
    sel = np.moveaxis(sel, 0, -1)           # (Mt, 2, n)
    return sel.reshape(-1, rpos.size)


def id_matrix(geom, box: Box, I: np.ndarray, Fint: np.ndarray, prm: RSParams) -> np.ndarray:
    """M_B of step 4 (all blocks without lam I, as I and F_int are disjoint)."""
    nodes, cpos = np.unique(I // 2, return_inverse=True)
    comp = I % 2
    P, Pn, _, _ = proxy_circle(box.cx, box.cy, box.side, prm.n_proxy, prm.proxy_ratio)
    wB = geom.weight[nodes].max()
    Pw = np.full(prm.n_proxy, wB)
    xy = geom.xy[nodes]
    blocks = []
    if Fint.size:
        blocks.append(stokes.operator_entries(geom, Fint, I, 0.0))
        blocks.append(stokes.operator_entries(geom, I, Fint, 0.0).T)
    blocks.append(_cols(stokes.double_layer_blocks(P, xy, geom.normal[nodes], geom.weight[nodes]), cpos, comp))
    blocks.append(_rows_t(stokes.double_layer_blocks(xy, P, Pn, Pw), cpos, comp))
    blocks.append(_rows_t(stokes.stokeslet_blocks(xy, P, Pw), cpos, comp))
    blocks.append((geom.weight[I // 2] * geom.normal[I // 2, comp])[None, :])
    blocks.append(wB * geom.normal[I // 2, comp][None, :])
    return np.vstack(blocks)


class RSFactorization:
    def __init__(self, geom, prm: Optional[RSParams] = None, root=None):
        self.geom = geom
        self.prm = prm or RSParams()
        if root is None and getattr(geom, "root", None) is not None:
            root = tuple(geom.root)
        self.boxes: List[Box] = build_tree(geom.xy, self.prm.leaf_size, root)
        self.root = (self.boxes[0].cx, self.boxes[0].cy, self.boxes[0].side)
        self.L = depth(self.boxes)
        self.fac: Dict[int, BoxFactor] = {}
        self.factored = False

    # ---- per-box steps -------------------------------------------------
    def leaf_dofs(self, b: Box) -> np.ndarray:
        return np.sort(np.concatenate([2 * b.nodes, 2 * b.nodes + 1]))

    def box_dofs(self, b: Box) -> np.ndarray:
        if b.is_leaf:
            return self.leaf_dofs(b)
        return np.sort(np.concatenate([self.fac[c].S for c in b.children]))

    def far_near(self, b: Box, I: np.ndarray, active: np.ndarray) -> np.ndarray:
        _, _, _, rp = proxy_circle(b.cx, b.cy, b.side, self.prm.n_proxy, self.prm.proxy_ratio)
        cand = np.nonzero(active)[0]
        d = self.geom.xy[cand // 2] - np.array([b.cx, b.cy])[None, :]
        inside = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] < rp * rp   # |x - c_B| < r_p
        cand = cand[inside]
        return cand[~np.isin(cand, I)]

    def diag_block(self, b: Box, I: np.ndarray) -> np.ndarray:
        A = stokes.operator_entries(self.geom, I, I, self.prm.lam)
        if not b.is_leaf:
            for c in b.children:
                fc = self.fac[c]
                S = fc.S
                pos = np.searchsorted(I, S)
                A[np.ix_(pos, pos)] = fc.Xss
        return A

    def compress(self, b: Box, active: np.ndarray) -> BoxFactor:
        prm = self.prm
        I = self.box_dofs(b)
        n = I.size
        Fint = self.far_near(b, I, active)
        if n == 0:
            z = np.zeros((0, 0))
            return BoxFactor(b.id, b.level, I, np.zeros(0, np.int64), 0, z, z, z, None, z, Fint)
        M = id_matrix(self.geom, b, I, Fint, prm)
        qr = PivotedQR(M, prm.pivot)
        k = qr.rank(prm.tol)
        k0 = k
        A = self.diag_block(b, I)
        while True:
            T = qr.interpolation(k)
            perm = qr.perm.copy()
            s, r = perm[:k], perm[k:]
            Ass, Asr = A[np.ix_(s, s)], A[np.ix_(s, r)]
            Ars, Arr = A[np.ix_(r, s)], A[np.ix_(r, r)]
            Xsr = Asr - Ass @ T
            Xrs = Ars - T.T @ Ass
            Xrr = Arr - Ars @ T - T.T @ Xsr
            if r.size == 0:
                lu = None
                E = np.zeros((k, 0))
                Fm = np.zeros((0, k))
                Xss = Ass.copy()
                break
            lu = sla.lu_factor(Xrr)
            Xinv = sla.lu_solve(lu, np.eye(r.size))
            rcond = 1.0 / (np.linalg.norm(Xrr, 1) * np.linalg.norm(Xinv, 1))
            if not np.isfinite(rcond) or rcond < prm.rcond_min:
                k += 1
                continue
            Fm = sla.lu_solve(lu, Xrs)
            E = sla.lu_solve(lu, Xsr.T, trans=1).T
            Xss = Ass - Xsr @ Fm
            break
        return BoxFactor(b.id, b.level, I, perm, k, T, E, Fm, lu, Xss, Fint, k0, M.shape[0])

    # ---- factorization ----------------------------------------------------
    def levels(self, l: int) -> List[Box]:
        return [b for b in self.boxes if b.level == l]

    def factor(self, only: Optional[set] = None):
        """Compress every box of levels L..1, then factor the root.

        `only`, when given, restricts recompression to that set of box ids
        (the other boxes keep their stored factors); used by update().
        """
        N2 = self.geom.n_dofs
        active = np.ones(N2, dtype=bool)
        seq = not self.prm.level_parallel
        if seq and only is not None:
            raise ValueError("updating is defined for the level-parallel scheme")
        for l in range(self.L, 0, -1):
            bl = self.levels(l)
            snap = active.copy()
            for b in bl:
                if only is None or b.id in only or b.id not in self.fac:
                    # sequential scheme (Section 2.2): a box's near field holds
                    # only what the boxes compressed before it left active
                    self.fac[b.id] = self.compress(b, active if seq else snap)
                if seq:
                    active[self.fac[b.id].R] = False
            for b in bl:
                active[self.fac[b.id].R] = False
        self._factor_root()
        self.factored = True
        return self

    def _factor_root(self):
        b = self.boxes[0]
        I0 = self.box_dofs(b)
        self.I0 = I0
        self.X0 = self.diag_block(b, I0)
        p = self.geom.n_holes
        if p == 0:
            self.lu0 = sla.lu_factor(self.X0)
            return
        H = stokes.h_matrix(self.geom)
        Pt = stokes.psi_t_matrix(self.geom)
        self.Hh = self.apply_U(H)
        self.Ph = self.apply_Vt_rows(Pt)
        G = np.zeros((3 * p, 3 * p))
        for l in range(self.L, 0, -1):
            for b in self.levels(l):
                fb = self.fac[b.id]
                if fb.r == 0:
                    continue
                R = fb.R
                G += self.Ph[:, R] @ sla.lu_solve(fb.lu, self.Hh[R, :])
        n0 = I0.size
        Z = np.zeros((n0 + 3 * p, n0 + 3 * p))
        Z[:n0, :n0] = self.X0
        Z[:n0, n0:] = self.Hh[I0, :]
        Z[n0:, :n0] = self.Ph[:, I0]
        Z[n0:, n0:] = -np.eye(3 * p) - G
        self.Z = Z
        self.luZ = sla.lu_factor(Z)

    # ---- transforms --------------------------------------------------------
    def apply_U(self, C: np.ndarray) -> np.ndarray:
        """U C: per box, leaf level first: c_R -= T^T c_S; c_S -= E c_R."""
        C = np.array(C, dtype=np.float64, copy=True)
        for l in range(self.L, 0, -1):
            for b in self.levels(l):
                fb = self.fac[b.id]
                if fb.I.size == 0:
                    continue
                S, R = fb.S, fb.R
                C[R] -= fb.T.T @ C[S]
                C[S] -= fb.E @ C[R]
        return C

    def apply_V(self, Y: np.ndarray) -> np.ndarray:
        """V Y: per box, level 1 first: y_R -= F y_S; y_S -= T y_R."""
        Y = np.array(Y, dtype=np.float64, copy=True)
        for l in range(1, self.L + 1):
            for b in self.levels(l):
                fb = self.fac[b.id]
                if fb.I.size == 0:
                    continue
                S, R = fb.S, fb.R
                Y[R] -= fb.F @ Y[S]
                Y[S] -= fb.T @ Y[R]
        return Y

    def apply_Vt_rows(self, G: np.ndarray) -> np.ndarray:
        """G V for row vectors G: per box, leaf level first: g_R -= g_S T; g_S -= g_R F."""
        G = np.array(G, dtype=np.float64, copy=True)
        for l in range(self.L, 0, -1):
            for b in self.levels(l):
                fb = self.fac[b.id]
                if fb.I.size == 0:
                    continue
                S, R = fb.S, fb.R
                G[:, R] -= G[:, S] @ fb.T
                G[:, S] -= G[:, R] @ fb.F
        return G

    # ---- solve ---------------------------------------------------------------
    def solve(self, f: np.ndarray) -> np.ndarray:
        """[mu; lambda] for right-hand sides f of 2N rows (border rows zero, as
        in eq. backwardeq) or 2N + 3p rows [f; g] (a general right-hand side of
        the augmented system, e.g. a refinement residual): g enters the border
        rows of the root system, Z [y_0; lambda] = [c_0; g - sum_B Ph_R z_R]."""
        assert self.factored
        f = np.asarray(f, dtype=np.float64)
        one = f.ndim == 1
        Fm = f.reshape(f.shape[0], -1)
        N2 = self.geom.n_dofs
        p = self.geom.n_holes
        if Fm.shape[0] not in (N2, N2 + 3 * p):
            raise ValueError("right-hand side must have 2N or 2N + 3p rows")
        gb = Fm[N2:] if Fm.shape[0] > N2 else np.zeros((3 * p, Fm.shape[1]))
        c = self.apply_U(Fm[:N2])
        y = np.zeros_like(c)
        z: Dict[int, np.ndarray] = {}
        for l in range(self.L, 0, -1):
            for b in self.levels(l):
                fb = self.fac[b.id]
                if fb.r:
                    z[b.id] = sla.lu_solve(fb.lu, c[fb.R])
        I0 = self.I0
        if p == 0:
            y[I0] = sla.lu_solve(self.lu0, c[I0])
            lam = np.zeros((0, c.shape[1]))
            for bid, zr in z.items():
                y[self.fac[bid].R] = zr
        else:
            rhs2 = gb.copy()
            for bid, zr in z.items():
                rhs2 -= self.Ph[:, self.fac[bid].R] @ zr
            sol = sla.lu_solve(self.luZ, np.vstack([c[I0], rhs2]))
            y[I0] = sol[: I0.size]
            lam = sol[I0.size:]
            for bid, zr in z.items():
                fb = self.fac[bid]
                y[fb.R] = zr - sla.lu_solve(fb.lu, self.Hh[fb.R] @ lam)
        x = self.apply_V(y)
        out = np.vstack([x, lam]) if p else x
        assert out.shape[0] == N2 + 3 * p
        return out[:, 0] if one else out

    # ---- updating (Section 2.8) -------------------------------------------------
    def update(self, new_geom, moved_nodes):
        """Refactor for new_geom (same root square) recompressing only the boxes
        whose compression inputs changed.  Returns the set of recompressed box ids."""
        moved = np.zeros(new_geom.n_nodes, dtype=bool)
        moved[np.asarray(moved_nodes, dtype=np.int64)] = True
        return self._update(new_geom, moved, np.arange(self.geom.n_nodes))

    def update_geometry(self, new_geom, old_of_new):
        """The update of Section 2.8 when curves are inserted or deleted (the
        experiment of Section 4.2): new_geom has its own node numbering and
        number of holes; old_of_new[j] is the old index of new node j, or -1
        for a node that did not exist.  Kept nodes must keep their relative
        order and their data.  A box is recompressed exactly when an input of
        its compression changed (new or deleted nodes count as changed), and
        the root, H and Psi^T are rebuilt for the new holes.  Returns the set
        of recompressed box ids."""
        old_of_new = np.asarray(old_of_new, dtype=np.int64)
        if old_of_new.shape != (new_geom.n_nodes,):
            raise ValueError("old_of_new must have one entry per new node")
        kept = np.nonzero(old_of_new >= 0)[0]
        ko = old_of_new[kept]
        if np.any(np.diff(ko) <= 0) or (ko.size and (ko[0] < 0 or ko[-1] >= self.geom.n_nodes)):
            raise ValueError("kept nodes must keep their relative order")
        g0 = self.geom
        for a in ("xy", "normal"):
            if not np.array_equal(getattr(new_geom, a)[kept], getattr(g0, a)[ko]):
                raise ValueError("kept nodes must keep their data")
        for a in ("weight", "curvature"):
            if not np.array_equal(getattr(new_geom, a)[kept], getattr(g0, a)[ko]):
                raise ValueError("kept nodes must keep their data")
        new_of_old = np.full(g0.n_nodes, -1, dtype=np.int64)
        new_of_old[ko] = kept
        moved = old_of_new < 0
        return self._update(new_geom, moved, new_of_old)

    def _update(self, new_geom, moved, new_of_old):
        """moved: per new node, True if its data are new; new_of_old: per old
        node, its new index or -1 (deleted).  Old index sets are carried into
        the new numbering before they are compared or kept."""
        if not self.prm.level_parallel:
            raise ValueError("updating is defined for the level-parallel scheme")

        def nodes_new(nodes):      # deleted nodes map below -1, so sets with them never match
            m = new_of_old[nodes]
            return np.where(m >= 0, m, -2 - nodes)

        def dofs_new(d):
            m = new_of_old[d // 2]
            return np.where(m >= 0, 2 * m + d % 2, -2 - d)

        old_boxes, old_fac = self.boxes, self.fac
        old_by_key = {b.key: b for b in old_boxes}
        self.geom = new_geom
        self.boxes = build_tree(new_geom.xy, self.prm.leaf_size, self.root)
        self.L = depth(self.boxes)
        self.fac = {}
        recomputed = set()
        active = np.ones(new_geom.n_dofs, dtype=bool)
        for l in range(self.L, 0, -1):
            bl = self.levels(l)
            snap = active.copy()
            for b in bl:
                ob = old_by_key.get(b.key)
                ofb = old_fac.get(ob.id) if ob is not None else None
                changed = ob is None or ofb is None or ob.is_leaf != b.is_leaf
                if not changed:
                    kI = dofs_new(ofb.I)
                    changed = bool(np.any(kI < 0))
                if not changed:
                    if b.is_leaf:
                        changed = not np.array_equal(nodes_new(ob.nodes), b.nodes) or bool(moved[b.nodes].any())
                    else:
                        okeys = sorted(old_boxes[c].key for c in ob.children)
                        nkeys = sorted(self.boxes[c].key for c in b.children)
                        changed = okeys != nkeys or any(c in recomputed for c in b.children)
                if not changed:
                    I = self.box_dofs(b)
                    Fint = self.far_near(b, I, snap)
                    changed = (not np.array_equal(Fint, dofs_new(ofb.Fint))) or bool(moved[Fint // 2].any())
                if changed:
                    self.fac[b.id] = self.compress(b, snap)
                    recomputed.add(b.id)
                else:
                    self.fac[b.id] = BoxFactor(b.id, ofb.level, kI, ofb.perm, ofb.k, ofb.T, ofb.E, ofb.F, ofb.lu,
                                               ofb.Xss, dofs_new(ofb.Fint), ofb.rank0, ofb.m)
            for b in bl:
                active[self.fac[b.id].R] = False
        self._factor_root()
        self.factored = True
        return recomputed

    # ---- statistics -----------------------------------------------------------
    def ranks(self):
        return {bid: (fb.I.size, fb.k) for bid, fb in self.fac.items()}
