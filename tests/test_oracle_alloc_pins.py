"""Pins of the oracle's bin-width allocation (the L-infinity guarantee).

The plain allocation rests on the constant S = 1 + sum_l (1 + K_l), with K_l
the product over dimensions of ||T^-1 P^T M||_inf for the level (the loss is
guaranteed by finite-element theory, Sec. 1 and Sec. 2.3; the bin width is
derived from an error estimator, Sec. 2).  These pins tie it to values that
do not come from the oracle's own band and Thomas code:

* ||A||_inf in exact rational arithmetic from the hat-function definitions
  (mass integrals, interpolation weights, Gaussian elimination over Q);
* K_l as the infinity norm of the dense Kronecker product of the per-dimension
  matrices (a sum over dimensions, or a missing dimension, fails it);
* the exact worst case of the whole recomposition: the largest row abs-sum of
  the dense map from coefficient errors to the recomposed field, built by
  recomposing unit vectors, never exceeds S (nor the bound of per-level widths);
* hand-derived constants in tests/golden/hand_values.json;
* the edges of the supported tolerance range.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import fieldgen
from oracle import alloc as A
from oracle import codec, grid, quant as Q
from oracle import transform as X

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_values.json")))


def _coarse_new(n):
    coarse = list(range(0, n, 2))
    if (n - 1) % 2:
        coarse.append(n - 1)
    return coarse, list(range(1, n - 1, 2))


def _mass(x):
    """P1 mass matrix on nodes x: the integrals of products of hat functions."""
    n = len(x)
    zero = x[0] - x[0]
    M = [[zero] * n for _ in range(n)]
    for i in range(n - 1):
        h = x[i + 1] - x[i]
        M[i][i] += h / 3
        M[i + 1][i + 1] += h / 3
        M[i][i + 1] += h / 6
        M[i + 1][i] += h / 6
    return M


def _solve(Mc, B):
    """Gaussian elimination (no pivoting needed: Mc is symmetric positive definite)."""
    n = len(Mc)
    M = [row[:] + brow[:] for row, brow in zip(Mc, B)]
    for k in range(n):
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            M[i] = [a - f * b for a, b in zip(M[i], M[k])]
    X_ = [None] * n
    for i in range(n - 1, -1, -1):
        row = M[i][n:]
        for j in range(i + 1, n):
            row = [a - M[i][j] * b for a, b in zip(row, X_[j])]
        X_[i] = [a / M[i][i] for a in row]
    return X_


def correction_matrix_from_definitions(x):
    """A = Mc^-1 P^T Mf for fine nodes x (Fractions or floats), as a list of rows."""
    n = len(x)
    coarse, new = _coarse_new(n)
    nc = len(coarse)
    zero = x[0] - x[0]
    P = [[zero] * nc for _ in range(n)]
    for j, c in enumerate(coarse):
        P[c][j] = zero + 1
    for i in new:
        jl = coarse.index(i - 1)
        P[i][jl] = (x[i + 1] - x[i]) / (x[i + 1] - x[i - 1])
        P[i][jl + 1] = (x[i] - x[i - 1]) / (x[i + 1] - x[i - 1])
    Mf = _mass(x)
    Mc = _mass([x[c] for c in coarse])
    PtM = [[sum(P[k][j] * Mf[k][i] for k in range(n)) for i in range(n)] for j in range(nc)]
    return _solve(Mc, PtM)


def row_norm(Am):
    return max(sum(abs(v) for v in row) for row in Am)


@pytest.mark.parametrize("n", list(range(3, 11)))
def test_correction_norm_equals_exact_rational_value(n):
    exact = row_norm(correction_matrix_from_definitions([Fraction(i) for i in range(n)]))
    got = A.correction_norm(grid.make_dimop(np.arange(float(n))))
    assert abs(got - float(exact)) <= 1e-14 * float(exact), (n, got, exact)
    g = GOLD["correction_norm_uniform_exact"]["values"]
    assert abs(float(exact) - g[str(n)]) <= 5e-5, n  # the 4-decimal table of the derivation


def test_correction_norm_n5_hand_value():
    g = GOLD["correction_norm_uniform_exact"]
    exact = row_norm(correction_matrix_from_definitions([Fraction(i) for i in range(5)]))
    assert exact == Fraction(g["n5_numerator"], g["n5_denominator"])
    assert abs(A.correction_norm(grid.make_dimop(np.arange(5.0))) - 1.75) <= 1e-15


def test_correction_norm_nonuniform_exact():
    rng = np.random.default_rng(11)
    for n in (4, 6, 7, 9):
        x = np.cumsum(rng.integers(1, 9, size=n)).astype(float)
        exact = row_norm(correction_matrix_from_definitions([Fraction(int(v)) for v in x]))
        got = A.correction_norm(grid.make_dimop(x))
        assert abs(got - float(exact)) <= 1e-14 * float(exact), (n, got, exact)


@pytest.mark.parametrize("shape", [(9,), (6, 7), (5, 9), (5, 6, 7), (2, 9), (9, 1, 5), (4, 5, 4, 5)])
def test_level_K_is_norm_of_kronecker_product(shape):
    rng = np.random.default_rng(sum(shape) * 7 + len(shape))
    coords = [fieldgen.random_coords(n, rng, jitter=0.5) for n in shape]
    h = grid.Hierarchy(shape, coords)
    K = A.level_K(h)
    assert K[0] == 0.0
    for l in range(1, h.L + 1):
        mats = [np.array(correction_matrix_from_definitions(list(h.coords[l][d])), dtype=np.float64)
                for d in range(h.D) if h.decomposed[d]]
        big = mats[0]
        for m in mats[1:]:
            big = np.kron(big, m)
        ref = float(np.abs(big).sum(axis=1).max())
        assert abs(K[l] - ref) <= 1e-12 * ref, (shape, l, K[l], ref)


def _error_map(h):
    """Dense map from stream coefficient errors to the recomposed field (float64)."""
    n = int(np.prod(h.shape))
    E = np.zeros((n, n))
    for j in range(n):
        s = np.zeros(n)
        s[j] = 1.0
        coarsest, cbars = Q.from_stream(s, h, np.float64)
        E[:, j] = X.recompose(coarsest, cbars, h, np.float64).ravel()
    return E


@pytest.mark.parametrize("shape", [(9,), (10,), (17,), (9, 9), (6, 10), (5, 6, 7), (2, 9, 5)])
def test_worst_case_error_within_the_a_priori_bound(shape):
    rng = np.random.default_rng(len(shape) * 100 + shape[0])
    coords = [fieldgen.random_coords(n, rng, jitter=0.5) for n in shape]
    for cc in (None, coords):
        h = grid.Hierarchy(shape, cc)
        E = _error_map(h)
        worst = float(np.abs(E).sum(axis=1).max())  # max |e| for |delta| <= 1/2 is worst / 2
        S = A.S_constant(h)
        assert worst <= S * (1 + 1e-12), (shape, worst, S)
        # per-level widths: sum_j |E_ij| b_l(j) / 2 stays within the bound of the widths
        off = Q.level_offsets(h)
        for bins in (A.count_weighted_bins(h, 1.0), list(rng.uniform(0.5, 2.0, h.L + 1))):
            w = np.concatenate([np.full(off[l + 1] - off[l], bins[l] / 2) for l in range(h.L + 1)])
            worst_b = float((np.abs(E) * w[None, :]).sum(axis=1).max())
            assert worst_b <= A.error_bound(h, bins) * (1 + 1e-12), (shape, worst_b)


def _dense_A(x):
    """A = Mc^-1 P^T Mf in float64 with numpy, assembled from the definitions."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    coarse, new = _coarse_new(n)

    def mass(y):
        h = np.diff(y)
        M = np.diag(np.concatenate([h, [0.0]]) / 3 + np.concatenate([[0.0], h]) / 3)
        return M + np.diag(h / 6, 1) + np.diag(h / 6, -1)

    P = np.zeros((n, len(coarse)))
    P[coarse, np.arange(len(coarse))] = 1.0
    for i in new:
        j = coarse.index(i - 1)
        P[i, j] = (x[i + 1] - x[i]) / (x[i + 1] - x[i - 1])
        P[i, j + 1] = (x[i] - x[i - 1]) / (x[i + 1] - x[i - 1])
    return np.linalg.solve(mass(x[coarse]), P.T @ mass(x)), np.asarray(coarse)


def S_from_definitions(shape, coords=None):
    """1 + sum over levels of (1 + product over decomposed sides of ||A||_inf)."""
    xs = [np.arange(float(n)) if coords is None or coords[d] is None else np.asarray(coords[d], float)
          for d, n in enumerate(shape)]
    dec = [n > 2 for n in shape]
    levels = []
    for n, ok in zip(shape, dec):
        if ok:
            k = 0
            while n > 3:
                n, k = n // 2 + 1, k + 1
            levels.append(k)
    S = 1.0
    for _ in range(min(levels)):
        K = 1.0
        for d in range(len(shape)):
            if dec[d]:
                Am, coarse = _dense_A(xs[d])
                K *= float(np.abs(Am).sum(axis=1).max())
                xs[d] = xs[d][coarse]
        S += 1.0 + K
    return S


@pytest.mark.parametrize("key", ["S_c1_129x129", "S_c2_513cubed", "S_257cubed", "S_c3_500cubed_geometric"])
def test_S_constant_hand_values(key):
    g = GOLD[key]
    shape = tuple(g["shape"])
    coords = None
    if g.get("coords") == "geometric":
        x = fieldgen.geometric_coords(shape[0])
        coords = [x] * len(shape)
        assert abs(A.correction_norm(grid.make_dimop(x)) - g["finest_norm"]) <= g["abs_tol"]
    S = A.S_constant(grid.Hierarchy(shape, coords))
    assert abs(S - g["S"]) <= g["abs_tol"], (key, S)
    Sd = S_from_definitions(shape, coords)
    assert abs(S - Sd) <= 1e-12 * Sd, (key, S, Sd)


def test_count_weighted_bins_hand_value():
    g = GOLD["count_weighted_1d_n5"]
    h = grid.Hierarchy((5,))
    b = A.count_weighted_bins(h, g["tau_eff"])
    assert np.allclose(b, g["bins"], rtol=1e-14, atol=0)
    assert abs(A.error_bound(h, b) - g["tau_eff"]) <= 1e-15


def test_tolerance_range_edges():
    """Rounding reserve above tau/2 (float32) and max|u|/b at 2^49 (float64) are refused."""
    u = np.array([1.0, -0.5, 0.25, 0.75, -1.0])
    h = grid.Hierarchy((5,))
    # float32, L = 1: rho = 8 eps32 max|u| = 9.54e-7; refused below tol 1.91e-6
    for tol, bad in ((1.8e-6, True), (2.0e-6, False)):
        T = np.float32
        tau = tol
        tau_eff = A.tau_effective(tau, 1.0, h.L, T)
        assert A.out_of_range(tau, 1.0, h.L, T, A.plain_bins(h, tau_eff)) == bad, tol
    # float64, L = 1, S = 3.75: accepted only for tol in (1.78e-15 * 2, ...) with b > 2^-49
    for tol, bad in ((3.0e-15, True), (4.5e-15, True), (6.0e-15, False), (1e-13, False)):
        tau_eff = A.tau_effective(tol, 1.0, h.L, np.float64)
        assert A.out_of_range(tol, 1.0, h.L, np.float64, A.plain_bins(h, tau_eff)) == bad, tol
    with pytest.raises(ValueError):
        codec.compress(u, 4.5e-15)
    codec.compress(u, 6.0e-15)
    with pytest.raises(ValueError):
        codec.compress(u.astype(np.float32), 1.8e-6)
