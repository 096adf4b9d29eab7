"""Error control in the L2 norm and the s-norms (oracle; test infrastructure only).

The paper quantizes the multilevel coefficients level by level with bin
widths derived from error estimators in several norms, selected by a
smoothness parameter s (Sec. 2; the tolerance, s and error-bound type of the
high-level call, Sec. 3 first listing; its cosmology case bounds the relative
L2 error, Sec. 4).  Reading used here, for the P1 hierarchy of the
decomposition (grid.py, transform.py):

* L2 norm of a grid function: that of its multilinear interpolant,
  ||u||^2 = u^T M u with M = kron_d M_d, the consistent P1 mass matrix of each
  decomposed side; a side that is not decomposed (1 or 2 nodes) acts as a
  batch dimension and contributes the identity (a sum over its slices);
* the decomposition computes the nodal values of u_l = Q_l u, the L2
  projection onto level l (u_L = u, u_{l-1} = coarse part + correction).  The
  s-norm is ||u||_s^2 = sum_{l=0..L} 4^(s l) ||(Q_l - Q_{l-1}) u||^2 with
  Q_{-1} = 0 (level 0 the coarsest); by orthogonality
  ||(Q_l - Q_{l-1}) u||^2 = ||u_l||^2 - ||u_{l-1}||^2, and ||u||_0 = ||u||;
* estimator: a coefficient error delta_l (values at level l's new nodes, zero
  at its coarse nodes; every node at level 0) changes the recomposed field by
  (I - Q_{l-1}) delta_l, and these changes are orthogonal across levels, so
  ||e||_s^2 <= sum_l 4^(s l) ||delta_l||^2 <= sum_l 4^(s l) W_l max|delta_l|^2,
  where W_l is the sum, over the level's new nodes, of the integral of their
  level-l hat function (delta^T M delta <= sum_i delta_i^2 (M 1)_i for the
  nonnegative symmetric M);
* allocation: with |delta_l| <= b_l / 2, the widths that keep the most bits
  (maximize sum_l N_l log b_l) under sum_l 4^(s l) W_l b_l^2 / 4 <= tau^2 are
  b_l = 2 tau g_l with g_l = sqrt(N_l / ((N 4^(s l)) W_l));
* rounding: the transform's rounding, at most rho = 4 (L+1) eps ||u||_inf per
  node (the reserve of the L-infinity bound), adds at most
  max(1, 2^(s L)) rho sqrt(W_0) in the s-norm (W_0 = |Omega|); tau_eff = tau
  minus that, and a tolerance whose reserve exceeds tau / 2 is refused, as is
  one with ||u||_inf / b_l >= 2^49;
* relative bound (s = 0 only): tau = tol ||u||.

Sums run in index order and products in dimension order, so the host code of
the library, which writes the same expressions, gets the same float64 values.
"""
from __future__ import annotations

import math

import numpy as np

from . import alloc as A
from . import transform as X
from .grid import Hierarchy, mass_bands


def hat_integrals(x) -> list:
    """Integral of each P1 hat function on nodes x: (h_left + h_right) / 2."""
    x = [float(v) for v in x]
    n = len(x)
    out = []
    for i in range(n):
        hl = x[i] - x[i - 1] if i > 0 else 0.0
        hr = x[i + 1] - x[i] if i + 1 < n else 0.0
        out.append((hl + hr) / 2.0)
    return out


def _seq_sum(vals) -> float:
    s = 0.0
    for v in vals:
        s += v
    return s


def level_weights(hier: Hierarchy) -> list:
    """W_l, l = 0..L: the sum of the hat integrals of level l's new nodes (all nodes at l = 0)."""
    W = [0.0] * (hier.L + 1)
    for l in range(hier.L, -1, -1):
        all_p, coarse_p = 1.0, 1.0
        for d in range(hier.D):
            if hier.decomposed[d]:
                w = hat_integrals(hier.coords[l][d])
                a = _seq_sum(w)
                c = _seq_sum(w[i] for i in hier.cidx(l, d)) if l > 0 else 0.0
            else:
                a = c = float(hier.sizes[l][d])
            all_p *= a
            coarse_p *= c
        W[l] = all_p - coarse_p if l > 0 else all_p
    return W


def level_factors(hier: Hierarchy, s: float) -> list:
    """g_l = sqrt(N_l / ((N 4^(s l)) W_l)): the bin width per unit of 2 tau."""
    W = level_weights(hier)
    N = hier.level_counts()
    tot = float(sum(N))
    return [math.sqrt(float(N[l]) / ((tot * float(np.power(2.0, 2.0 * s * l))) * W[l])) for l in range(hier.L + 1)]


def reserve_factor(hier: Hierarchy, s: float) -> float:
    """max(1, 2^(s L)) sqrt(W_0): multiplies the per-node rounding reserve."""
    W0 = level_weights(hier)[0]
    return max(1.0, float(np.power(2.0, s * hier.L))) * math.sqrt(W0)


def tau_effective(tau: float, maxabs: float, hier: Hierarchy, s: float, T) -> float:
    rho = 4.0 * (hier.L + 1) * A.eps_of(T) * maxabs
    rs = rho * reserve_factor(hier, s)
    return tau - min(rs, 0.5 * tau)


def out_of_range(tau: float, maxabs: float, hier: Hierarchy, s: float, T, bins) -> bool:
    if not tau_effective(tau, maxabs, hier, s, T) > 0.0:
        return False
    rho = 4.0 * (hier.L + 1) * A.eps_of(T) * maxabs
    return rho * reserve_factor(hier, s) > 0.5 * tau or any(not maxabs < A.MAX_SCALE * b for b in bins)


def bins_for(hier: Hierarchy, tau_eff: float, s: float) -> list:
    if not tau_eff > 0.0:
        return [1.0] * (hier.L + 1)
    return [2.0 * tau_eff * g for g in level_factors(hier, s)]


def estimate_sq(hier: Hierarchy, bins, s: float) -> float:
    """The a-priori bound of ||e||_s^2 for widths b_l: sum_l 4^(s l) W_l b_l^2 / 4."""
    W = level_weights(hier)
    return sum(float(np.power(2.0, 2.0 * s * l)) * W[l] * bins[l] * bins[l] / 4.0 for l in range(hier.L + 1))


def mass_apply(u, hier: Hierarchy, l: int = None):
    """M u for a grid function on level l (the input grid by default), in float64."""
    l = hier.L if l is None else l
    g = np.asarray(u, dtype=np.float64)
    for d in range(hier.D):
        if not hier.decomposed[d]:
            continue
        a, b, c = mass_bands(np.asarray(hier.coords[l][d], dtype=np.float64))
        g = np.moveaxis(g, d, 0)
        out = b.reshape((-1,) + (1,) * (g.ndim - 1)) * g
        if g.shape[0] > 1:
            out[1:] += a[1:].reshape((-1,) + (1,) * (g.ndim - 1)) * g[:-1]
            out[:-1] += c[:-1].reshape((-1,) + (1,) * (g.ndim - 1)) * g[1:]
        g = np.moveaxis(out, 0, d)
    return g


def l2_norm_sq(u, hier: Hierarchy, l: int = None) -> float:
    """u^T M u on level l (the input grid by default)."""
    u64 = np.asarray(u, dtype=np.float64)
    return float(np.sum(u64 * mass_apply(u64, hier, l)))


def level_norms_sq(u, hier: Hierarchy) -> list:
    """||u_l||^2 for l = 0..L, with u_l = Q_l u from the float64 decomposition."""
    out = [0.0] * (hier.L + 1)
    cur = np.asarray(u, dtype=np.float64)
    out[hier.L] = l2_norm_sq(cur, hier, hier.L)
    for l in range(hier.L, 0, -1):
        _, cur = X.decompose_level(cur, hier, l, np.float64)
        out[l - 1] = l2_norm_sq(cur, hier, l - 1)
    return out


def s_norm_sq(u, hier: Hierarchy, s: float) -> float:
    """||u||_s^2 = sum_l 4^(s l) (||u_l||^2 - ||u_{l-1}||^2)."""
    nl = level_norms_sq(u, hier)
    tot = 0.0
    for l in range(hier.L + 1):
        prev = nl[l - 1] if l > 0 else 0.0
        tot += float(np.power(2.0, 2.0 * s * l)) * (nl[l] - prev)
    return tot
