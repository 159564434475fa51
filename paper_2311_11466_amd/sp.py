"""Orders for sequential projections.

Any order of the positions is a valid SP order (the paper lets it be fixed or
shuffled).  The library turns an order into batches of pairwise disjoint
windows by dependency level, so the order decides how much of it can run at
once: ascending raster order chains every position to its neighbour (about
raster columns + (N / step) x raster rows batches), while the colour order
below puts every position of one colour class, whose windows are pairwise
disjoint, into one batch (about (N / step + 1)^2 batches).
"""
from __future__ import annotations

import numpy as np


def colour_classes(pos, n: int) -> np.ndarray:
    """First-fit colouring of the window-overlap graph in ascending index
    order: positions of one colour have pairwise disjoint windows."""
    pos = np.asarray(pos, dtype=np.int64)
    j = len(pos)
    colour = np.full(j, -1, dtype=np.int64)
    for i in range(j):
        near = (np.abs(pos[:i, 0] - pos[i, 0]) < n) & (np.abs(pos[:i, 1] - pos[i, 1]) < n)
        used = set(colour[:i][near].tolist())
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


def disjoint_order(pos, n: int) -> np.ndarray:
    """Positions sorted by colour class (colour_classes); within a colour,
    ascending index.  The library runs each class as one batch."""
    colour = colour_classes(pos, n)
    return np.lexsort((np.arange(len(colour)), colour)).astype(np.int32)


def shuffled_orders(n_pos: int, n_iter: int, seed: int) -> list:
    """One seeded random permutation per iteration (the shuffled form)."""
    rng = np.random.default_rng(seed)
    return [rng.permutation(n_pos).astype(np.int32) for _ in range(n_iter)]


__all__ = ["colour_classes", "disjoint_order", "shuffled_orders"]
