"""Multilevel decomposition and recomposition (oracle).

Reading of the paper's recursive decomposition (Sec. 2) as the P1
finite-element multilevel transform of the cited multilevel theory:

  level l holds nodal values u_l on grid l.  Its multilevel coefficients are
  the interpolation residual at the new nodes, c = u_l - Pi u_l, where Pi is
  the multilinear interpolant from the coarse nodes.  The next level is the
  L2 projection u_{l-1} = Q u_l = u_l|coarse + z with z solving
  M_{l-1} z = P^T M_l cbar, cbar being c extended by zeros at the coarse
  nodes.  Recomposition runs the same steps backwards.

Operation order (fixed here so that any implementation can reproduce the
rounding bit for bit; every step is rounded to the working type T):

* Pi is a sweep of 1D interpolations over dimensions D-1 down to 0: each
  sweep fills the new nodes of its dimension by (wl*left) + (wr*right) and
  copies the coarse nodes.  In the result the coarse nodes equal u exactly,
  so cbar = u - Pi u is exactly zero there;
* the load vector applies, for d = D-1 down to 0, the fine mass matrix along
  d, summed ((a*g[i-1] + b*g[i]) + c*g[i+1]), then the restriction along d,
  summed ((rl*g[c-1] + g[c]) + rr*g[c+1]); terms outside the side or at
  non-new neighbours are left out;
* the solve runs the Thomas algorithm along d = 0 up to D-1:
  forward d'[0] = d[0]*r[0], d'[i] = (d[i] - a[i]*d'[i-1])*r[i];
  backward x[i] = d'[i] - c'[i]*x[i+1];
* decomposition: u_{l-1} = u_l|coarse + z;
  recomposition: u_l|coarse = u_{l-1} - z, then u_l = c + Pi(u_l|coarse) at
  new nodes and u_l|coarse at coarse nodes.

Numpy float32/float64 elementwise arithmetic is IEEE round-to-nearest per
operation with no fused multiply-add, which is exactly what the order above
asks for.
"""
from __future__ import annotations

import numpy as np

from .grid import Hierarchy


def _front(a, axis):
    return np.moveaxis(a, axis, 0)


def _col(v, T, ndim):
    """Constant vector along axis 0, broadcast over the remaining axes."""
    return np.asarray(v, dtype=np.float64).astype(T).reshape((-1,) + (1,) * (ndim - 1))


def interp_axis(W, axis, op, T):
    """Expand ``axis`` from op.nc coarse nodes to op.nf fine nodes (copy + linear fill)."""
    a = _front(W, axis)
    out = np.empty((op.nf,) + a.shape[1:], dtype=T)
    out[op.cidx] = a
    jl = (op.fidx - 1) // 2  # coarse index of the left neighbour
    wl = _col(op.wl, T, a.ndim)
    wr = _col(op.wr, T, a.ndim)
    out[op.fidx] = wl * a[jl] + wr * a[jl + 1]
    return np.moveaxis(out, 0, axis)


def interpolant(uc, hier: Hierarchy, l: int, T):
    """Pi: multilinear interpolant on grid l from the dense coarse grid uc (grid l-1)."""
    W = uc
    for d in reversed(range(hier.D)):
        op = hier.ops[l][d]
        if op is not None:
            W = interp_axis(W, d, op, T)
    return W


def mass_axis(g, axis, op, T):
    a = _front(g, axis)
    ma = _col(op.ma, T, a.ndim)
    mb = _col(op.mb, T, a.ndim)
    mc = _col(op.mc, T, a.ndim)
    s = mb * a
    s[1:] = ma[1:] * a[:-1] + s[1:]
    s[:-1] = s[:-1] + mc[:-1] * a[1:]
    return np.moveaxis(s, 0, axis)


def restrict_axis(g, axis, op, T):
    a = _front(g, axis)
    f = a[op.cidx].copy()
    rl = _col(op.rl, T, a.ndim)
    rr = _col(op.rr, T, a.ndim)
    L = np.nonzero(op.has_l)[0]
    R = np.nonzero(op.has_r)[0]
    f[L] = rl[L] * a[op.cidx[L] - 1] + f[L]
    f[R] = f[R] + rr[R] * a[op.cidx[R] + 1]
    return np.moveaxis(f, 0, axis)


def thomas_axis(f, axis, op, T):
    a = _front(f, axis).copy()
    n = a.shape[0]
    ta = np.asarray(op.ta).astype(T)
    tr = np.asarray(op.tr).astype(T)
    tcp = np.asarray(op.tcp).astype(T)
    a[0] = a[0] * tr[0]
    for i in range(1, n):
        a[i] = (a[i] - ta[i] * a[i - 1]) * tr[i]
    for i in range(n - 2, -1, -1):
        a[i] = a[i] - tcp[i] * a[i + 1]
    return np.moveaxis(a, 0, axis)


def correction(cbar, hier: Hierarchy, l: int, T):
    """z = M_{l-1}^{-1} P^T M_l cbar on grid l-1 (tensor form, fixed order)."""
    g = cbar
    for d in reversed(range(hier.D)):
        op = hier.ops[l][d]
        if op is not None:
            g = mass_axis(g, d, op, T)
            g = restrict_axis(g, d, op, T)
    for d in range(hier.D):
        op = hier.ops[l][d]
        if op is not None:
            g = thomas_axis(g, d, op, T)
    return g


def coarse_part(u, hier: Hierarchy, l: int):
    return u[np.ix_(*[hier.cidx(l, d) for d in range(hier.D)])]


def decompose_level(u, hier: Hierarchy, l: int, T):
    """One level: returns (cbar on grid l, u_{l-1} on grid l-1)."""
    uc = coarse_part(u, hier, l)
    cbar = u - interpolant(uc, hier, l, T)
    z = correction(cbar, hier, l, T)
    return cbar, uc + z


def recompose_level(cbar, ucoarse, hier: Hierarchy, l: int, T):
    """Inverse of decompose_level: cbar (zeros at coarse nodes) and u_{l-1} -> u_l."""
    z = correction(cbar, hier, l, T)
    uc = ucoarse - z
    P = interpolant(uc, hier, l, T)
    u = cbar + P
    u[np.ix_(*[hier.cidx(l, d) for d in range(hier.D)])] = uc
    return u


def coefficient_at(u, hier: Hierarchy, p, T):
    """Finest-level coefficient at one node p of the input grid (0 at coarse nodes).

    The interpolant is evaluated at p alone, with the same nesting as
    ``interpolant``: the highest odd dimension innermost.
    """
    l = hier.L
    odd = [d for d in range(hier.D)
           if hier.ops[l][d] is not None and p[d] % 2 == 1 and p[d] < hier.sizes[l][d] - 1]

    def nest(q, k):
        if k == len(odd):
            return T(u[tuple(q)])
        d = odd[k]
        op = hier.ops[l][d]
        j = (q[d] - 1) // 2
        left = list(q)
        right = list(q)
        left[d] -= 1
        right[d] += 1
        a = nest(left, k + 1)
        b = nest(right, k + 1)
        return T(T(op.wl[j]) * a) + T(T(op.wr[j]) * b)

    if not odd:
        return T(0)
    return T(T(u[tuple(p)]) - nest(list(p), 0))


def decompose(u, hier: Hierarchy, T=None):
    """Full decomposition; returns (coarsest grid, [cbar_1, ..., cbar_L])."""
    T = np.dtype(T or u.dtype).type
    cur = np.ascontiguousarray(u, dtype=T)
    cbars = [None] * (hier.L + 1)
    for l in range(hier.L, 0, -1):
        cbars[l], cur = decompose_level(cur, hier, l, T)
    return cur, cbars


def recompose(coarsest, cbars, hier: Hierarchy, T=None):
    T = np.dtype(T or coarsest.dtype).type
    cur = np.ascontiguousarray(coarsest, dtype=T)
    for l in range(1, hier.L + 1):
        cur = recompose_level(np.asarray(cbars[l], dtype=T), cur, hier, l, T)
    return cur
