"""Oracle: spherical real-space grid, blockwise Hilbert ordering, neighbours.

Paper: the domain is a sphere around the nanocluster with the wavefunctions
vanishing outside (the confined-system discussion); grid points are ordered
along blockwise Hilbert space-filling curves to speed up the sparse H-times-
vector products (the SFC discussion before Table I's description).

Readings where the paper is silent:
* grid points (i, j, k) * h, origin on the centre atom, kept when
  i^2 + j^2 + k^2 <= floor((R_dom / h)^2 + 1e-9);
* blocks of 8^3 points counted from the bounding-box minimum corner
  (I = i + n_r with n_r = floor(R_dom / h)); blocks ranked by a 3-D Hilbert
  index computed with Skilling's transpose algorithm (J. Skilling,
  "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004), x the most
  significant axis, order = ceil(log2(blocks per edge)) (at least 1);
  points inside a block in x-fastest order; empty blocks skipped;
* padded rows: row = slot * 512 + local index; rows of outside points are
  unused (zero);
* the Cartesian baseline orders points z-slowest, x-fastest with row = rank;
* neighbour table: 36 offsets, axis-major (x, y, z), each axis -6..-1 then
  +1..+6; the entry is the neighbour's rank or -1 when it is outside.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BLOCK = 8
HALF_ORDER = 6
ORDER_HILBERT, ORDER_LEX = 0, 1


@dataclass
class Grid:
    h: float
    radius: float          # R_dom, bohr
    n_r: int               # floor(R_dom / h)
    ijk: np.ndarray        # [N, 3] int64 integer coordinates, rank order
    row_of_rank: np.ndarray  # [N] int64
    n_rows: int
    ordering: int
    blocks: np.ndarray     # [n_blocks, 3] block coordinates in slot order (Hilbert only)

    @property
    def n(self) -> int:
        return int(self.ijk.shape[0])

    @property
    def xyz(self) -> np.ndarray:
        """Cartesian coordinates (bohr) of the points, rank order."""
        return self.ijk.astype(np.float64) * self.h


def sphere_points(radius: float, h: float) -> tuple[int, np.ndarray]:
    """All integer (i, j, k) inside the sphere, in no particular order."""
    n_r = int(math.floor(radius / h))
    thr = math.floor((radius / h) ** 2 + 1e-9)
    g = np.arange(-n_r, n_r + 1, dtype=np.int64)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    inside = (i * i + j * j + k * k) <= thr
    return n_r, np.stack([i[inside], j[inside], k[inside]], axis=1)


def hilbert_index3(x: np.ndarray, y: np.ndarray, z: np.ndarray, nbits: int) -> np.ndarray:
    """Hilbert index of integer cell coordinates (Skilling's transpose method).

    Step 1 turns the axes into the "transposed" Hilbert index by undoing the
    excess work (inversions / exchanges of low bits, highest level first),
    then Gray-encodes; step 2 interleaves the bits, axis x first at each level.
    """
    X = [np.asarray(x, np.int64).copy(), np.asarray(y, np.int64).copy(), np.asarray(z, np.int64).copy()]
    top = 1 << (nbits - 1)
    q = top
    while q > 1:
        p = q - 1
        for i in range(3):
            hit = (X[i] & q) != 0
            X[0] = np.where(hit, X[0] ^ p, X[0])
            t = np.where(hit, 0, (X[0] ^ X[i]) & p)
            X[0] = X[0] ^ t
            X[i] = X[i] ^ t
        q >>= 1
    X[1] = X[1] ^ X[0]
    X[2] = X[2] ^ X[1]
    t = np.zeros_like(X[0])
    q = top
    while q > 1:
        t = np.where((X[2] & q) != 0, t ^ (q - 1), t)
        q >>= 1
    X = [v ^ t for v in X]
    idx = np.zeros_like(X[0])
    for lvl in range(nbits - 1, -1, -1):
        for i in range(3):
            idx = (idx << 1) | ((X[i] >> lvl) & 1)
    return idx


def hilbert_bits(n_blocks_edge: int) -> int:
    return max(1, int(n_blocks_edge - 1).bit_length())


def build_grid(radius: float, h: float, ordering: int = ORDER_HILBERT) -> Grid:
    n_r, pts = sphere_points(radius, h)
    if ordering == ORDER_LEX:
        order = np.lexsort((pts[:, 0], pts[:, 1], pts[:, 2]))
        ijk = pts[order]
        return Grid(h, radius, n_r, ijk, np.arange(len(ijk), dtype=np.int64), len(ijk), ordering,
                    np.zeros((0, 3), np.int64))
    I = pts + n_r
    B = I // BLOCK
    nb = (2 * n_r) // BLOCK + 1
    key = hilbert_index3(B[:, 0], B[:, 1], B[:, 2], hilbert_bits(nb))
    ukey, first = np.unique(key, return_index=True)
    slot = np.searchsorted(ukey, key)
    local = (I[:, 0] % BLOCK) + BLOCK * (I[:, 1] % BLOCK) + BLOCK * BLOCK * (I[:, 2] % BLOCK)
    row = slot * BLOCK ** 3 + local
    order = np.argsort(row, kind="stable")
    return Grid(h, radius, n_r, pts[order], row[order], len(ukey) * BLOCK ** 3, ordering, B[first])


def offsets() -> list[tuple[int, int]]:
    """(axis, k) for the 36 neighbour columns, in table order."""
    out = []
    for axis in range(3):
        for k in list(range(-HALF_ORDER, 0)) + list(range(1, HALF_ORDER + 1)):
            out.append((axis, k))
    return out


def neighbour_table(g: Grid) -> np.ndarray:
    """[N, 36] int32 neighbour ranks (-1 outside), via a dense lookup cube."""
    n = 2 * g.n_r + 1
    cube = -np.ones((n, n, n), dtype=np.int64)
    I = g.ijk + g.n_r
    cube[I[:, 0], I[:, 1], I[:, 2]] = np.arange(g.n)
    out = -np.ones((g.n, 36), dtype=np.int64)
    for c, (axis, k) in enumerate(offsets()):
        J = I.copy()
        J[:, axis] += k
        ok = (J[:, axis] >= 0) & (J[:, axis] < n)
        out[ok, c] = cube[J[ok, 0], J[ok, 1], J[ok, 2]]
    return out.astype(np.int32)
