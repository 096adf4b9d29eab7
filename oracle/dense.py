"""Brute-force dense finite-element objects on tiny tensor grids (oracle pins).

Used only to pin the tensor/Thomas implementation in ``transform`` against an
independent construction of the same L2 projection (the finite-element
guarantee the paper relies on, Sec. 1 and Sec. 2.3):

* mass matrices are assembled cell by cell from the multilinear hat basis with
  2-point Gauss quadrature per dimension, which integrates products of two
  linear factors exactly;
* the prolongation evaluates each coarse hat function at the fine nodes with
  ``numpy.interp`` (piecewise-linear interpolation of unit vectors);
* the correction is ``numpy.linalg.solve(M_coarse, P^T M_fine cbar)``.
"""
from __future__ import annotations

import itertools

import numpy as np

_GAUSS = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def mass_1d_quadrature(x):
    """1D P1 mass matrix assembled by 2-point Gauss quadrature per cell."""
    n = len(x)
    M = np.zeros((n, n))
    for e in range(n - 1):
        h = x[e + 1] - x[e]
        for t in _GAUSS:
            phi = (1.0 - t, t)
            for a in range(2):
                for b in range(2):
                    M[e + a, e + b] += 0.5 * h * phi[a] * phi[b]
    return M


def mass_nd_quadrature(xs):
    """Tensor-grid mass matrix assembled cell by cell (dense, C-order node numbering)."""
    shape = [len(x) for x in xs]
    D = len(xs)
    N = int(np.prod(shape))
    M = np.zeros((N, N))
    strides = [int(np.prod(shape[d + 1:])) for d in range(D)]
    cells = itertools.product(*[range(max(n - 1, 0)) for n in shape])
    corners = list(itertools.product(*[(0, 1)] * D))
    for cell in cells:
        hs = [xs[d][cell[d] + 1] - xs[d][cell[d]] for d in range(D)]
        idx = [sum((cell[d] + c[d]) * strides[d] for d in range(D)) for c in corners]
        for qp in itertools.product(*[_GAUSS] * D):
            wq = np.prod([0.5 * hs[d] for d in range(D)])
            vals = [np.prod([(qp[d] if c[d] else 1.0 - qp[d]) for d in range(D)]) for c in corners]
            for a in range(len(corners)):
                for b in range(len(corners)):
                    M[idx[a], idx[b]] += wq * vals[a] * vals[b]
    return M


def prolongation_1d(xf, xc):
    """Values of each coarse hat function at the fine nodes (nf x nc)."""
    nc = len(xc)
    P = np.zeros((len(xf), nc))
    for j in range(nc):
        e = np.zeros(nc)
        e[j] = 1.0
        P[:, j] = np.interp(xf, xc, e)
    return P


def kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def correction_dense(cbar, xs_fine, xs_coarse):
    """z on the coarse grid from the L2 projection of cbar (all dimensions decomposed)."""
    Mf = mass_nd_quadrature(xs_fine)
    Mc = mass_nd_quadrature(xs_coarse)
    P = kron_all([prolongation_1d(xf, xc) for xf, xc in zip(xs_fine, xs_coarse)])
    rhs = P.T @ (Mf @ np.ravel(cbar))
    z = np.linalg.solve(Mc, rhs)
    return z.reshape([len(x) for x in xs_coarse]), (Mf, Mc, P)


def interpolant_dense(uc, xs_fine, xs_coarse):
    P = kron_all([prolongation_1d(xf, xc) for xf, xc in zip(xs_fine, xs_coarse)])
    return (P @ np.ravel(uc)).reshape([len(x) for x in xs_fine])
