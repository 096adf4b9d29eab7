"""Bin-width allocation for the L-infinity bound (oracle).

The paper states that the quantization error of the multilevel coefficients
is controlled in a chosen norm by error estimators (Sec. 2) and that the loss
is guaranteed by finite-element theory (Sec. 1, Sec. 2.3).  The reading used
here for the L-infinity norm:

  with coefficient errors |delta_l| <= b_l/2, recomposition adds at level l
  the correction error A_l delta_l on the coarse nodes and delta_l plus a
  convex interpolation of the coarse error on the new nodes.  With
  A_l = kron_d A_{d,l}, A_{d,l} = T_{d,l}^{-1} P_d^T M_{d,l} and
  ||kron A_d||_inf = prod ||A_d||_inf, induction over the levels gives

      ||u - u~||_inf <= b_0/2 + sum_{l=1..L} (1 + K_l) b_l / 2,
      K_l = prod_d ||A_{d,l}||_inf.

* plain allocation: one bin width b = 2 tau_eff / S for every level,
  S = 1 + sum_l (1 + K_l);
* count-weighted allocation (ablation): b_l = 2 tau_eff N_l / ((1+K_l) sum N),
  with K_0 = 0 for the coarsest grid; it meets the same bound.

tau_eff leaves room for the rounding of the transform in the working type:
tau_eff = tau - min(rho, tau/2), rho = 4 (L+1) eps_T ||u||_inf, eps_T the
machine epsilon of T.  A field that is identically zero gets b = 1.

Supported range (a reading: the bound above is only worth stating when the
rounding reserve is a small part of tau, and the quantizer's integers must be
exact): a tolerance is rejected when rho > tau/2, or when ||u||_inf / b_l
reaches 2^49 for some level.  The multilevel coefficients stay within a small
multiple of ||u||_inf (convex interpolation, L2 projections stable in the
maximum norm), so with that cap |c / b| stays far below 2^63 even for learned
widths down to exp(-3) b.
"""
from __future__ import annotations

import numpy as np

from .grid import DimOp, Hierarchy


def tridiag_dense(a, b, c):
    n = len(b)
    M = np.diag(np.asarray(b, dtype=np.float64))
    if n > 1:
        M += np.diag(np.asarray(a[1:], dtype=np.float64), -1)
        M += np.diag(np.asarray(c[:-1], dtype=np.float64), 1)
    return M


def prolongation_dense(op: DimOp):
    """P (nf x nc): coarse nodal values -> fine nodal values by linear interpolation."""
    P = np.zeros((op.nf, op.nc))
    P[op.cidx, np.arange(op.nc)] = 1.0
    jl = (op.fidx - 1) // 2
    P[op.fidx, jl] = op.wl
    P[op.fidx, jl + 1] = op.wr
    return P


def correction_matrix(op: DimOp):
    """Dense A = T^{-1} P^T M for one dimension and level (LAPACK solve; used to pin below)."""
    M = tridiag_dense(op.ma, op.mb, op.mc)
    Tm = tridiag_dense(*op.coarse_mass)
    P = prolongation_dense(op)
    return np.linalg.solve(Tm, P.T @ M)


def norm_inf(A) -> float:
    return float(np.abs(A).sum(axis=1).max())


def correction_norm(op: DimOp) -> float:
    """||T^{-1} P^T M||_inf as the method applies the operator: column k of A is the
    1D mass, restriction and Thomas steps applied to the unit vector e_k (float64),
    and the row sums of |A| accumulate over k = 0, 1, ... in order."""
    from .transform import mass_axis, restrict_axis, thomas_axis

    rows = np.zeros(op.nc)
    for k in range(op.nf):
        e = np.zeros(op.nf)
        e[k] = 1.0
        col = thomas_axis(restrict_axis(mass_axis(e, 0, op, np.float64), 0, op, np.float64), 0, op,
                          np.float64)
        rows = rows + np.abs(col)
    return float(rows.max())


def level_K(hier: Hierarchy):
    """K_l for l = 1..L (index 0 unused, set to 0)."""
    K = [0.0]
    for l in range(1, hier.L + 1):
        k = 1.0
        for op in hier.ops[l]:
            if op is not None:
                k *= correction_norm(op)
        K.append(k)
    return K


def S_constant(hier: Hierarchy) -> float:
    K = level_K(hier)
    return 1.0 + sum(1.0 + K[l] for l in range(1, hier.L + 1))


def eps_of(T) -> float:
    return float(np.finfo(T).eps)


def tau_effective(tau: float, maxabs: float, L: int, T) -> float:
    rho = 4.0 * (L + 1) * eps_of(T) * maxabs
    return tau - min(rho, 0.5 * tau)


def tau_abs(tol: float, maxabs: float, rel: bool) -> float:
    return tol * maxabs if rel else tol


def plain_bins(hier: Hierarchy, tau_eff: float):
    if tau_eff <= 0.0:
        return [1.0] * (hier.L + 1)
    b = 2.0 * tau_eff / S_constant(hier)
    return [b] * (hier.L + 1)


def count_weighted_bins(hier: Hierarchy, tau_eff: float):
    if tau_eff <= 0.0:
        return [1.0] * (hier.L + 1)
    K = level_K(hier)
    N = hier.level_counts()
    tot = float(sum(N))
    return [2.0 * tau_eff * N[l] / ((1.0 + K[l]) * tot) for l in range(hier.L + 1)]


def error_bound(hier: Hierarchy, bins) -> float:
    """The a-priori L-infinity bound of a bin allocation."""
    K = level_K(hier)
    return bins[0] / 2.0 + sum((1.0 + K[l]) * bins[l] / 2.0 for l in range(1, hier.L + 1))


MAX_SCALE = 2.0 ** 49


def out_of_range(tau: float, maxabs: float, L: int, T, bins) -> bool:
    """True when the tolerance lies outside the supported range (see above)."""
    tau_eff = tau_effective(tau, maxabs, L, T)
    if not tau_eff > 0.0:
        return False
    rho = 4.0 * (L + 1) * eps_of(T) * maxabs
    return rho > 0.5 * tau or any(not maxabs < MAX_SCALE * b for b in bins)
