"""Adaptive quadtree (paper Section 2.3, Figure 1).

TEST INFRASTRUCTURE ONLY (see the package header).

Reading of the paper: boxes split while they hold more than `leaf_size`
points ("no more than" a prescribed number per leaf); only non-empty boxes
are kept.  Root square: centred on the bounding box of the nodes with side
(1 + 2^-20) times its larger extent, unless a fixed root is given (a fixed
root is what makes an updated factorization identical to a fresh one,
Section 2.8).  A node goes to the east child when x >= cx and to the north
child when y >= cy; children are kept in the order SW, SE, NW, NE.

Pinned by tests/test_oracle_rs.py::test_tree_partition_and_leaf_bound
(partition, leaf bound, containment, child levels).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MAX_DEPTH = 48


@dataclass
class Box:
    id: int
    level: int
    cx: float
    cy: float
    side: float
    parent: int
    nodes: np.ndarray                    # sorted node indices inside the box
    children: List[int] = field(default_factory=list)
    ix: int = 0                          # integer position of the box on its level's grid
    iy: int = 0

    @property
    def key(self):
        return (self.level, self.ix, self.iy)

    @property
    def is_leaf(self) -> bool:
        return not self.children


def default_root(xy: np.ndarray):
    xmin, ymin = xy.min(axis=0)
    xmax, ymax = xy.max(axis=0)
    cx = 0.5 * (xmin + xmax)
    cy = 0.5 * (ymin + ymax)
    side = (1.0 + 2.0 ** -20) * max(xmax - xmin, ymax - ymin)
    if side == 0.0:
        side = 1.0
    return float(cx), float(cy), float(side)


def build_tree(xy: np.ndarray, leaf_size: int, root: Optional[tuple] = None) -> List[Box]:
    """Boxes in breadth-first order (so every level is a contiguous run)."""
    cx, cy, side = default_root(xy) if root is None else tuple(float(v) for v in root)
    boxes = [Box(0, 0, cx, cy, side, -1, np.arange(xy.shape[0], dtype=np.int64))]
    head = 0
    while head < len(boxes):
        b = boxes[head]
        head += 1
        if b.nodes.size <= leaf_size:
            continue
        if b.level >= MAX_DEPTH:
            raise ValueError("quadtree deeper than %d levels (coincident nodes?)" % MAX_DEPTH)
        pts = xy[b.nodes]
        q = (pts[:, 0] >= b.cx).astype(np.int64) + 2 * (pts[:, 1] >= b.cy).astype(np.int64)
        h = b.side / 4.0
        for quad in range(4):
            sel = b.nodes[q == quad]
            if sel.size == 0:
                continue
            ccx = b.cx - h if quad % 2 == 0 else b.cx + h
            ccy = b.cy - h if quad < 2 else b.cy + h
            child = Box(len(boxes), b.level + 1, ccx, ccy, b.side / 2.0, b.id, sel,
                        ix=2 * b.ix + (quad & 1), iy=2 * b.iy + (quad >> 1))
            b.children.append(child.id)
            boxes.append(child)
    return boxes


def depth(boxes: List[Box]) -> int:
    return max(b.level for b in boxes)
