"""Keyframe selection for mapping windows (Sec. III-F "Keyframe Selection").

Keyframes live in a spatial grid of resolution g = 200 m, coarser than and
independent of the chunk grid: K(p) is the set of keyframes whose grid cell
(element-wise floor of position / g) equals that of p (the equation defining
the spatial candidate set).  Each step draws its keyframes from
K(p_latest), the cell of the most recently added keyframe.  Overlap(k) (the
chunk-overlap equation of the same section) is the fraction of keyframe k's
visible chunks already resident.

Inside the candidate set the paper applies CaRtGS's usage-based,
loss-weighted choice without restating it.  This module's reading: every
keyframe starts with `usage` uses; a step takes the candidates that still
have uses, highest last loss first (ties: higher Overlap, then the more
recent keyframe), and spends one use of each; when no candidate has uses
left, the candidates whose last loss is at least the median of the set get
`usage` more uses (high-loss views get more optimisation), the others one.
Host-side bookkeeping only: the visible chunk sets come from
dcgs_select_chunks and the residency from the pool.
"""
from __future__ import annotations

import math

import numpy as np


def grid_cell(p, g: float = 200.0) -> tuple:
    """floor(p / g) element-wise."""
    return tuple(int(math.floor(float(x) / g)) for x in p)


def overlap(visible: set, active: set) -> float:
    """|C_v(k) & C_active| / |C_v(k)| (1 for a keyframe that sees nothing)."""
    if not visible:
        return 1.0
    return len(visible & active) / len(visible)


class KeyframeScheduler:
    def __init__(self, grid: float = 200.0, usage: int = 3):
        self.g = float(grid)
        self.usage = int(usage)
        self.pos = {}        # keyframe -> position
        self.vis = {}        # keyframe -> set of visible chunk ids
        self.cells = {}      # grid cell -> keyframes (insertion order)
        self.left = {}       # keyframe -> remaining uses
        self.loss = {}       # keyframe -> last loss (inf until measured)
        self.latest = None

    def add(self, k, position, visible_chunks) -> None:
        self.pos[k] = np.asarray(position, np.float64)
        self.vis[k] = set(int(c) for c in visible_chunks)
        self.cells.setdefault(grid_cell(position, self.g), []).append(k)
        self.left[k] = self.usage
        self.loss[k] = math.inf
        self.latest = k

    def candidates(self, p=None) -> list:
        """K(p) (p defaults to the latest keyframe's position)."""
        if p is None:
            if self.latest is None:
                return []
            p = self.pos[self.latest]
        return list(self.cells.get(grid_cell(p, self.g), []))

    def report_loss(self, k, loss: float) -> None:
        self.loss[k] = float(loss)

    def select(self, n: int, active_chunks=()) -> list:
        """Up to n keyframes for the next window, spending one use each."""
        cand = self.candidates()
        if not cand:
            return []
        active = set(int(c) for c in active_chunks)
        if all(self.left[k] <= 0 for k in cand):
            losses = [self.loss[k] for k in cand]
            finite = [x for x in losses if math.isfinite(x)]
            med = float(np.median(finite)) if finite else math.inf
            for k in cand:
                self.left[k] += self.usage if self.loss[k] >= med else 1
        order = {k: i for i, k in enumerate(cand)}
        ready = [k for k in cand if self.left[k] > 0]
        ready.sort(key=lambda k: (-self.loss[k], -overlap(self.vis[k], active), -order[k]))
        chosen = ready[:n]
        for k in chosen:
            self.left[k] -= 1
        return chosen
