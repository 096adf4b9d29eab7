"""Grid hierarchy and FP64 per-dimension operator constants (oracle).

Reading of the paper's "multilevel decomposition on a multigrid hierarchy"
(Sec. 2) for structured tensor-product grids, uniform or not, dyadic or not:

* a side of n nodes coarsens to floor(n/2)+1 nodes: the even indices plus the
  last index n-1.  For even n the last coarse interval [n-2, n-1] keeps no
  midpoint.  New (fine-only) nodes are the odd indices below n-1;
* a side is decomposed only while it has more than 3 nodes; all decomposed
  sides coarsen together, so the number of levels L is the smallest number of
  coarsenings that brings one of them to 3 nodes;
* sides of 1 or 2 nodes are not decomposed (they act as batch dimensions);
* coarse coordinates are the subset of fine coordinates at the coarse nodes.

Per level and decomposed dimension the piecewise-linear (P1) operators are

* interpolation of a new node i from its coarse neighbours i-1, i+1 with
  weights wl = (x[i+1]-x[i]) / (x[i+1]-x[i-1]) and wr = (x[i]-x[i-1]) / (x[i+1]-x[i-1]);
* the exact (consistent) P1 mass matrix on the fine nodes:
  diagonal (h[i-1]+h[i])/3, off-diagonals h/6 of the shared interval;
* the restriction (transpose of the interpolation): coarse node j at fine
  index c gathers g[c] plus wr of new node c-1 times g[c-1] and wl of new
  node c+1 times g[c+1];
* the coarse mass matrix, factored for the Thomas algorithm:
  r[0] = 1/b[0], cp[0] = c[0]*r[0],
  r[i] = 1/(b[i] - a[i]*cp[i-1]), cp[i] = c[i]*r[i].

All constants are computed in float64 and cast to the working type by the
caller.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def coarsen(n: int) -> int:
    """Coarse node count of a side of n nodes."""
    return n // 2 + 1


def dim_levels(n: int):
    """Coarsenings of a side until 3 nodes remain; None if the side is not decomposed (n <= 2)."""
    if n <= 2:
        return None
    k = 0
    while n > 3:
        n = coarsen(n)
        k += 1
    return k


def num_levels(shape) -> int:
    ls = [dim_levels(n) for n in shape]
    ls = [v for v in ls if v is not None]
    return min(ls) if ls else 0


def coarse_index(n: int) -> np.ndarray:
    idx = list(range(0, n, 2))
    if (n - 1) % 2 == 1:
        idx.append(n - 1)
    return np.asarray(idx, dtype=np.int64)


def new_index(n: int) -> np.ndarray:
    return np.arange(1, n - 1, 2, dtype=np.int64)


@dataclass
class DimOp:
    """Operators of one decomposed dimension at one level (fine side nf -> coarse side nc)."""

    nf: int
    nc: int
    cidx: np.ndarray  # fine indices of the coarse nodes (nc)
    fidx: np.ndarray  # fine indices of the new nodes (nf - nc)
    wl: np.ndarray  # interpolation weight of the left coarse neighbour, per new node
    wr: np.ndarray  # interpolation weight of the right coarse neighbour, per new node
    ma: np.ndarray  # fine mass matrix, sub-diagonal a[i] (row i, column i-1); a[0] unused
    mb: np.ndarray  # fine mass matrix diagonal
    mc: np.ndarray  # fine mass matrix super-diagonal c[i] (row i, column i+1); c[nf-1] unused
    rl: np.ndarray  # restriction weight from fine c-1 (0 when c-1 is not a new node)
    rr: np.ndarray  # restriction weight from fine c+1 (0 when c+1 is not a new node)
    has_l: np.ndarray  # bool: left new neighbour exists
    has_r: np.ndarray  # bool: right new neighbour exists
    ta: np.ndarray  # coarse mass sub-diagonal (Thomas a)
    tr: np.ndarray  # Thomas reciprocal pivots r
    tcp: np.ndarray  # Thomas modified super-diagonal c'
    coarse_mass: tuple = field(default=None)  # (a, b, c) of the coarse mass matrix


def mass_bands(x: np.ndarray):
    """Exact P1 mass matrix bands on coordinates x (float64)."""
    n = len(x)
    h = np.diff(x)
    a = np.zeros(n)
    b = np.zeros(n)
    c = np.zeros(n)
    hl = np.concatenate([[0.0], h])  # h[i-1], 0 at the left end
    hr = np.concatenate([h, [0.0]])  # h[i], 0 at the right end
    b[:] = (hl + hr) / 3.0
    a[1:] = h / 6.0
    c[:-1] = h / 6.0
    return a, b, c


def thomas_factors(a: np.ndarray, b: np.ndarray, c: np.ndarray):
    """Reciprocal pivots r and modified super-diagonal c' of a tridiagonal matrix (float64)."""
    n = len(b)
    r = np.zeros(n)
    cp = np.zeros(n)
    r[0] = 1.0 / b[0]
    cp[0] = c[0] * r[0]
    for i in range(1, n):
        r[i] = 1.0 / (b[i] - a[i] * cp[i - 1])
        cp[i] = c[i] * r[i]
    return r, cp


def make_dimop(x: np.ndarray) -> DimOp:
    """Operators for coarsening the side with fine coordinates x (float64, strictly increasing)."""
    nf = len(x)
    cidx = coarse_index(nf)
    fidx = new_index(nf)
    nc = len(cidx)
    xl = x[fidx - 1]
    xm = x[fidx]
    xr = x[fidx + 1]
    wl = (xr - xm) / (xr - xl)
    wr = (xm - xl) / (xr - xl)
    ma, mb, mc = mass_bands(x)
    # restriction weights per coarse node
    is_new = np.zeros(nf, dtype=bool)
    is_new[fidx] = True
    wl_full = np.zeros(nf)
    wr_full = np.zeros(nf)
    wl_full[fidx] = wl
    wr_full[fidx] = wr
    has_l = np.array([c - 1 >= 0 and is_new[c - 1] for c in cidx], dtype=bool)
    has_r = np.array([c + 1 < nf and is_new[c + 1] for c in cidx], dtype=bool)
    rl = np.zeros(nc)
    rr = np.zeros(nc)
    rl[has_l] = wr_full[cidx[has_l] - 1]  # new node c-1 weights its right neighbour c by wr
    rr[has_r] = wl_full[cidx[has_r] + 1]  # new node c+1 weights its left neighbour c by wl
    xc = x[cidx]
    ta, tb, tc = mass_bands(xc)
    tr, tcp = thomas_factors(ta, tb, tc)
    return DimOp(nf=nf, nc=nc, cidx=cidx, fidx=fidx, wl=wl, wr=wr, ma=ma, mb=mb, mc=mc,
                 rl=rl, rr=rr, has_l=has_l, has_r=has_r, ta=ta, tr=tr, tcp=tcp,
                 coarse_mass=(ta, tb, tc))


class Hierarchy:
    """Level sizes, coordinates and operators of a tensor grid.

    Level L is the input grid, level 0 the coarsest.  ``ops[l][d]`` holds the
    operators that take level l to level l-1 along dimension d (None for a
    dimension that is not decomposed).
    """

    def __init__(self, shape, coords=None):
        self.shape = tuple(int(s) for s in shape)
        if len(self.shape) == 0 or any(s < 1 for s in self.shape):
            raise ValueError("bad shape")
        D = len(self.shape)
        self.D = D
        if coords is None:
            coords = [None] * D
        xs = []
        for d in range(D):
            if coords[d] is None:
                xs.append(np.arange(self.shape[d], dtype=np.float64))
            else:
                x = np.asarray(coords[d], dtype=np.float64)
                if x.shape != (self.shape[d],) or np.any(np.diff(x) <= 0):
                    raise ValueError("coordinates must be strictly increasing with one value per node")
                xs.append(x)
        self.decomposed = [dim_levels(n) is not None for n in self.shape]
        self.L = num_levels(self.shape)
        L = self.L
        self.sizes = [None] * (L + 1)
        self.coords = [None] * (L + 1)
        self.sizes[L] = list(self.shape)
        self.coords[L] = xs
        self.ops = [None] * (L + 1)
        for l in range(L, 0, -1):
            ops = []
            cs = []
            sz = []
            for d in range(D):
                if self.decomposed[d]:
                    op = make_dimop(self.coords[l][d])
                    ops.append(op)
                    cs.append(self.coords[l][d][op.cidx])
                    sz.append(op.nc)
                else:
                    ops.append(None)
                    cs.append(self.coords[l][d])
                    sz.append(self.sizes[l][d])
            self.ops[l] = ops
            self.coords[l - 1] = cs
            self.sizes[l - 1] = sz

    def cidx(self, l, d):
        op = self.ops[l][d]
        return np.arange(self.sizes[l][d]) if op is None else op.cidx

    def fidx(self, l, d):
        op = self.ops[l][d]
        return np.zeros(0, dtype=np.int64) if op is None else op.fidx

    def count(self, l) -> int:
        return int(np.prod(self.sizes[l]))

    def level_counts(self):
        """Number of stream entries per level: coarsest grid, then new nodes of levels 1..L."""
        out = [self.count(0)]
        for l in range(1, self.L + 1):
            out.append(self.count(l) - self.count(l - 1))
        return out
