"""Tile binning: (tile, depth) keys, their sorted order and per-tile ranges
(test infrastructure only).

Every visible Gaussian is duplicated once per screen tile its opacity-aware
bounding box touches (rect from the FP32 key path).  Each copy carries the
64-bit key (global tile id << 32) | bits(camera-space depth), where bits() is
the FP32 bit pattern (monotone for the positive depths kept), and the value
is the Gaussian's index.  Sorting the copies by key, ties by index, groups
them by tile in front-to-back order; ranges[t] = [first, last+1) of tile t in
that order, (0, 0) when empty.  The global tile id of view k is
k * TX * TY + ty * TX + tx.
"""
from __future__ import annotations

import numpy as np


def duplicate(kp: dict, gauss_index: np.ndarray, tile_offset: int):
    """Keys and values of one view's copies, in Gaussian order.

    kp is the key-path dict of the view; gauss_index maps its rows to the
    global Gaussian index used as the value."""
    TX = kp["TX"]
    vis = np.nonzero(kp["visible"])[0]
    keys, vals = [], []
    for i in vis:
        x0, y0, x1, y1 = kp["rect"][i]
        ty, tx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        tid = (tile_offset + ty * TX + tx).ravel().astype(np.uint64)
        keys.append((tid << np.uint64(32)) | np.uint64(kp["zbits"][i]))
        vals.append(np.full(tid.shape[0], gauss_index[i], np.int64))
    if not keys:
        return np.zeros(0, np.uint64), np.zeros(0, np.int64)
    return np.concatenate(keys), np.concatenate(vals)


def sort_keys(keys: np.ndarray, vals: np.ndarray):
    """Ascending (key, value) order."""
    order = np.lexsort((vals, keys))
    return keys[order], vals[order]


def tile_ranges(sorted_keys: np.ndarray, n_tiles: int) -> np.ndarray:
    """ranges[t] = (first, last+1) of tile t in the sorted list, else (0,0)."""
    rng = np.zeros((n_tiles, 2), np.int64)
    if sorted_keys.shape[0] == 0:
        return rng
    tid = (sorted_keys >> np.uint64(32)).astype(np.int64)
    starts = np.searchsorted(tid, np.arange(n_tiles), side="left")
    ends = np.searchsorted(tid, np.arange(n_tiles), side="right")
    nz = ends > starts
    rng[nz, 0] = starts[nz]
    rng[nz, 1] = ends[nz]
    return rng
