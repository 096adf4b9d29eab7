"""Pins of the oracle's L2 / s-norm error control (Sec. 2: bin widths from error
estimators in several norms chosen by the smoothness s; Sec. 3, first listing).

Independent of the oracle's own code paths:

* the L2 norm equals the dense quadratic form u^T (kron_d M_d) u with M_d
  assembled here from hat-function integrals, and matches closed forms
  (constants, linear functions);
* the s = 0 level decomposition of the norm adds up to the L2 norm
  (orthogonality of the L2 projections), and the level norms grow with l;
* W_l equals the explicit sum over the level's new nodes, and its closed form
  on uniform odd grids;
* the estimator bounds the s-norm of the recomposed error for random and
  sign-pattern coefficient errors, for negative, zero and positive s;
* end to end, the compressed field meets the bound.
"""
import math

import numpy as np
import pytest

import fieldgen
from oracle import codec, grid
from oracle import quant as Q
from oracle import snorm as SN
from oracle import transform as X


def dense_mass(x):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    M = np.zeros((n, n))
    for i in range(n - 1):
        h = x[i + 1] - x[i]
        M[i:i + 2, i:i + 2] += h * np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    return M


def dense_kron_mass(hier, l=None):
    l = hier.L if l is None else l
    big = np.ones((1, 1))
    for d in range(hier.D):
        Md = dense_mass(hier.coords[l][d]) if hier.decomposed[d] else np.eye(hier.sizes[l][d])
        big = np.kron(big, Md)
    return big


SHAPES = [(9,), (10,), (5, 9), (6, 7), (5, 6, 7), (2, 9, 5), (9, 1, 6)]


@pytest.mark.parametrize("shape", SHAPES)
def test_l2_norm_equals_dense_quadratic_form(shape):
    rng = np.random.default_rng(sum(shape))
    coords = [fieldgen.random_coords(n, rng, jitter=0.5) for n in shape]
    for cc in (None, coords):
        h = grid.Hierarchy(shape, cc)
        u = rng.standard_normal(shape)
        ref = float(u.ravel() @ dense_kron_mass(h) @ u.ravel())
        assert abs(SN.l2_norm_sq(u, h) - ref) <= 1e-12 * ref


def test_l2_norm_closed_forms():
    x = np.linspace(0.0, 2.0, 17) ** 1.5  # nonuniform on [0, 2^1.5]
    h = grid.Hierarchy((17,), [x])
    assert abs(SN.l2_norm_sq(np.ones(17), h) - x[-1]) <= 1e-13  # int 1 = |Omega|
    # the P1 interpolant of a linear function is itself: int_0^1 y^2 dy = 1/3
    y = np.linspace(0.0, 1.0, 33)
    h = grid.Hierarchy((33,), [y])
    assert abs(SN.l2_norm_sq(y, h) - 1.0 / 3.0) <= 1e-14
    # 2D: int int (x y)^2 over [0,1]^2 = 1/9
    h2 = grid.Hierarchy((33, 33), [y, y])
    assert abs(SN.l2_norm_sq(np.outer(y, y), h2) - 1.0 / 9.0) <= 1e-14


@pytest.mark.parametrize("shape", SHAPES)
def test_level_norms_add_up_to_the_l2_norm(shape):
    rng = np.random.default_rng(3 + sum(shape))
    coords = [fieldgen.random_coords(n, rng, jitter=0.5) for n in shape]
    h = grid.Hierarchy(shape, coords)
    u = rng.standard_normal(shape)
    nl = SN.level_norms_sq(u, h)
    assert all(nl[l] >= nl[l - 1] * (1 - 1e-12) for l in range(1, h.L + 1))
    total = SN.l2_norm_sq(u, h)
    assert abs(SN.s_norm_sq(u, h, 0.0) - total) <= 1e-12 * total
    # a level-0 function has no finer components: every s gives its L2 norm
    if h.L >= 1:
        coarse = np.zeros(h.sizes[0])
        coarse[...] = rng.standard_normal(h.sizes[0])
        cb = [None] + [np.zeros(h.sizes[l]) for l in range(1, h.L + 1)]
        v = X.recompose(coarse, cb, h, np.float64)
        for s in (-1.0, 0.5, 2.0):
            assert abs(SN.s_norm_sq(v, h, s) - SN.l2_norm_sq(v, h)) <= 1e-11 * SN.l2_norm_sq(v, h)


@pytest.mark.parametrize("shape", SHAPES)
def test_level_weights_equal_explicit_sums(shape):
    rng = np.random.default_rng(7 + sum(shape))
    coords = [fieldgen.random_coords(n, rng, jitter=0.5) for n in shape]
    h = grid.Hierarchy(shape, coords)
    W = SN.level_weights(h)
    for l in range(h.L + 1):
        ones = np.ones(h.sizes[l])
        integ = (dense_kron_mass(h, l) @ ones.ravel()).reshape(h.sizes[l])  # (M 1)_i = int phi_i
        if l == 0:
            ref = float(integ.sum())
        else:
            new = np.ones(h.sizes[l], dtype=bool)
            new[np.ix_(*[h.cidx(l, d) for d in range(h.D)])] = False
            ref = float(integ[new].sum())
        assert abs(W[l] - ref) <= 1e-12 * max(1.0, ref), (shape, l)


def test_level_weights_uniform_hand_value():
    # 2D 9x9 on unit spacing: every level spans 8 x 8; the coarse nodes hold half of each side's
    # hat integrals, so W_l = 64 (1 - 1/4) = 48 for l = 1, 2 and W_0 = 64
    h = grid.Hierarchy((9, 9))
    assert SN.level_weights(h) == [64.0, 48.0, 48.0]
    # 3D 5x5x5: W_1 = 64 (1 - 1/8) = 56, W_0 = 64
    assert SN.level_weights(grid.Hierarchy((5, 5, 5))) == [64.0, 56.0]


def test_mass_inequality_of_the_estimator():
    rng = np.random.default_rng(4)
    for shape in [(9,), (6, 7), (5, 6, 7)]:
        h = grid.Hierarchy(shape, [fieldgen.random_coords(n, rng) for n in shape])
        M = dense_kron_mass(h)
        row = M.sum(axis=1)
        for _ in range(20):
            d = rng.standard_normal(M.shape[0])
            assert d @ M @ d <= float((d * d) @ row) * (1 + 1e-12)


@pytest.mark.parametrize("s", [-1.0, -0.5, 0.0, 0.5, 1.0])
@pytest.mark.parametrize("shape", [(17,), (9, 10), (6, 7, 5)])
def test_estimator_bounds_the_recomposed_error(shape, s):
    """Coefficient errors within b_l/2 (uniform random and +-b_l/2 sign patterns)
    recompose to an error whose s-norm stays within the a-priori bound."""
    rng = np.random.default_rng(int(10 * s) + sum(shape) + 50)
    coords = [fieldgen.random_coords(n, rng, jitter=0.5) for n in shape]
    h = grid.Hierarchy(shape, coords)
    bins = SN.bins_for(h, 1.0, s)
    assert abs(SN.estimate_sq(h, bins, s) - 1.0) <= 1e-12
    off = Q.level_offsets(h)
    half = np.concatenate([np.full(off[l + 1] - off[l], bins[l] / 2) for l in range(h.L + 1)])
    for trial in range(12):
        if trial % 2:
            delta = half * rng.choice([-1.0, 1.0], size=len(half))
        else:
            delta = half * rng.uniform(-1.0, 1.0, size=len(half))
        coarsest, cbars = Q.from_stream(delta, h, np.float64)
        e = X.recompose(coarsest, cbars, h, np.float64)
        assert SN.s_norm_sq(e, h, s) <= 1.0 + 1e-12


@pytest.mark.parametrize("s,rel,tol", [(0.0, True, 1e-3), (0.0, True, 1e-5), (0.0, False, 1e-3), (1.0, False, 1e-3),
                                       (-1.0, False, 1e-3)])
def test_compressed_field_meets_the_snorm_bound(s, rel, tol):
    u = fieldgen.bumps2d(65, seed=2)
    x = np.linspace(0.0, 1.0, 65)  # the unit square: an absolute bound in the field's own units
    cc = [x, x]
    buf = codec.compress(u, tol, rel=rel, coords=cc, norm="s", s=s)
    hd = codec.parse(buf)
    assert hd.norm == codec.NORM_S and hd.s == s
    h = grid.Hierarchy(u.shape, cc)
    tau = tol * math.sqrt(SN.l2_norm_sq(u, h)) if rel else tol
    assert hd.tau_abs == tau
    r = codec.decompress(buf)
    e = r.astype(np.float64) - u
    assert SN.s_norm_sq(e, h, s) <= tau * tau
    # float32 as well, where its rounding reserve leaves room (it is refused at rel 1e-5)
    if tol < 1e-4:
        return
    u32 = u.astype(np.float32)
    r32 = codec.decompress(codec.compress(u32, tol, rel=rel, coords=cc, norm="s", s=s))
    assert SN.s_norm_sq(r32.astype(np.float64) - u32.astype(np.float64), h, s) <= tau * tau * (1 + 1e-6)


def test_snorm_refusals():
    u = fieldgen.bumps2d(33)
    with pytest.raises(ValueError):
        codec.compress(u, 1e-3, rel=True, norm="s", s=1.0)
    with pytest.raises(ValueError):
        codec.compress(u, 1e-3, norm="s", alloc="count")
    with pytest.raises(ValueError):
        codec.compress(u.astype(np.float32), 1e-8, norm="s")
