"""Pins of the CPU oracle against what the method and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a hand
derivation (tests/golden/hand_values.json), a closed form, an invariant of
the finite-element projection, an independent dense construction, or a
textbook algorithm.
"""
import heapq
import json
import math
import os

import numpy as np
import pytest

import fieldgen
from oracle import alloc as A
from oracle import codec, dense, grid, huffman as H, mlp, quant as Q
from oracle import transform as X

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_values.json")))


# ---------------------------------------------------------------- hierarchy
@pytest.mark.parametrize("n,sizes", [
    (129, [129, 65, 33, 17, 9, 5, 3]),
    (513, [513, 257, 129, 65, 33, 17, 9, 5, 3]),
    (500, [500, 251, 126, 64, 33, 17, 9, 5, 3]),
    (257, [257, 129, 65, 33, 17, 9, 5, 3]),
    (4, [4, 3]),
])
def test_level_sizes(n, sizes):
    h = grid.Hierarchy((n,))
    assert h.L == len(sizes) - 1
    assert [h.sizes[l][0] for l in range(h.L, -1, -1)] == sizes


def test_level_counts_partition():
    h = grid.Hierarchy((129, 129))
    assert h.level_counts() == [9, 16, 56, 208, 800, 3136, 12416]
    h = grid.Hierarchy((513, 513, 513))
    c = h.level_counts()
    assert c[-1] == 118_031_104 and c[-2] == 14_827_904 and c[0] == 27
    assert sum(c) == 513 ** 3


def test_levels_stop_at_smallest_side_and_batch_dims():
    h = grid.Hierarchy((65, 2049))
    assert h.L == 5 and h.sizes[0] == [3, 65]
    h = grid.Hierarchy((2, 9, 1))
    assert h.decomposed == [False, True, False] and h.L == 2 and h.sizes[0] == [2, 3, 1]


def test_coarse_sets_even_side_keeps_last_node():
    assert list(grid.coarse_index(8)) == [0, 2, 4, 6, 7]
    assert list(grid.new_index(8)) == [1, 3, 5]
    assert list(grid.coarse_index(9)) == [0, 2, 4, 6, 8]


# ---------------------------------------------------------------- transform
def _multilinear(xs, rng):
    """a + sum b_d x_d + sum c_de x_d x_e (+ x0 x1 x2 term): multilinear in physical coordinates."""
    D = len(xs)
    grids = np.meshgrid(*xs, indexing="ij")
    u = np.full(grids[0].shape, rng.normal())
    for d in range(D):
        u = u + rng.normal() * grids[d]
    for d in range(D):
        for e in range(d + 1, D):
            u = u + rng.normal() * grids[d] * grids[e]
    if D >= 3:
        u = u + rng.normal() * grids[0] * grids[1] * grids[2]
    return u


@pytest.mark.parametrize("shape", [(17,), (9, 12), (10, 9, 7), (5, 6, 5, 5)])
def test_multilinear_input_has_zero_coefficients(shape):
    rng = np.random.default_rng(11)
    xs = [fieldgen.random_coords(n, rng) for n in shape]
    h = grid.Hierarchy(shape, xs)
    u = _multilinear(xs, rng)
    l = h.L
    cbar, ucoarse = X.decompose_level(u, h, l, np.float64)
    scale = np.abs(u).max()
    assert np.abs(cbar).max() <= 1e-13 * scale
    # the projection of a coarse-representable function is itself
    assert np.abs(ucoarse - X.coarse_part(u, h, l)).max() <= 1e-13 * scale


@pytest.mark.parametrize("shape", [(9,), (10, 7), (9, 12, 8), (5, 6, 5, 4)])
def test_coefficient_at_is_residual_of_multilinear_interpolation(shape):
    """At every new node of the finest level: u(p) minus the tensor-product
    linear interpolation of the coarse nodes (scipy's RegularGridInterpolator),
    and exactly the value the full decomposition places in the stream."""
    from scipy.interpolate import RegularGridInterpolator

    rng = np.random.default_rng(17)
    xs = [fieldgen.random_coords(n, rng) for n in shape]
    h = grid.Hierarchy(shape, xs)
    u = rng.standard_normal(shape)
    l = h.L
    cs = [h.cidx(l, d) for d in range(h.D)]
    interp = RegularGridInterpolator([xs[d][cs[d]] for d in range(h.D)], u[np.ix_(*cs)], method="linear")
    cbar, _ = X.decompose_level(u, h, l, np.float64)
    fine = [set(h.fidx(l, d).tolist()) for d in range(h.D)]
    seen = 0
    for p in np.ndindex(*shape):
        got = X.coefficient_at(u, h, p, np.float64)
        if not any(p[d] in fine[d] for d in range(h.D)):
            assert got == 0.0
            continue
        seen += 1
        want = u[p] - interp([xs[d][p[d]] for d in range(h.D)])[0]
        assert abs(got - want) <= 1e-12 * (1 + abs(u).max())
        assert got == cbar[p]
    assert seen == np.prod(shape) - np.prod([len(c) for c in cs])


def test_constant_input():
    h = grid.Hierarchy((33, 17))
    u = np.full((33, 17), 2.5)
    c0, cbars = X.decompose(u, h)
    assert np.all(c0 == 2.5)
    for l in range(1, h.L + 1):
        assert np.abs(cbars[l]).max() <= 1e-15


@pytest.mark.parametrize("shape", [(3,), (4,), (5,), (6,), (9,), (10,), (5, 4), (6, 5), (4, 5, 6), (5, 4, 5)])
def test_correction_equals_dense_projection(shape):
    """Tensor Thomas correction == dense L2 projection assembled by quadrature."""
    rng = np.random.default_rng(sum(shape) * 7 + len(shape))
    xs = [fieldgen.random_coords(n, rng, jitter=0.6) for n in shape]
    h = grid.Hierarchy(shape, xs)
    if h.L == 0:
        pytest.skip("not decomposed")
    l = h.L
    u = rng.standard_normal(shape)
    uc = X.coarse_part(u, h, l)
    Pi = X.interpolant(uc, h, l, np.float64)
    assert np.abs(Pi - dense.interpolant_dense(uc, h.coords[l], h.coords[l - 1])).max() <= 1e-14
    cbar = u - Pi
    z = X.correction(cbar, h, l, np.float64)
    zd, (Mf, Mc, P) = dense.correction_dense(cbar, h.coords[l], h.coords[l - 1])
    assert np.abs(z - zd).max() <= 1e-13 * max(1.0, np.abs(zd).max())
    # orthogonality: cbar - P z is L2-orthogonal to every coarse basis function
    resid = P.T @ (Mf @ (np.ravel(cbar) - P @ np.ravel(z)))
    assert np.abs(resid).max() <= 1e-13


def test_interpolant_is_not_dimensionwise_surplus():
    """Pi uses coarse corners only; the dimension-by-dimension in-place surplus differs at (odd, odd)."""
    rng = np.random.default_rng(3)
    u = rng.standard_normal((5, 5))
    h = grid.Hierarchy((5, 5))
    cbar, _ = X.decompose_level(u, h, 1, np.float64)
    # direct bilinear residual at (1, 1)
    bil = 0.25 * (u[0, 0] + u[0, 2] + u[2, 0] + u[2, 2])
    assert abs(cbar[1, 1] - (u[1, 1] - bil)) <= 1e-15
    # in-place surplus along x then y gives another value at (1, 1)
    v = u.copy()
    v[1::2, :] -= 0.5 * (u[0:-1:2, :] + u[2::2, :])
    w = v.copy()
    w[:, 1::2] -= 0.5 * (v[:, 0:-1:2] + v[:, 2::2])
    assert abs(w[1, 1] - cbar[1, 1]) > 1e-6


@pytest.mark.parametrize("n", [5, 8, 9, 12, 17])
def test_oracle_bands_match_quadrature_and_galerkin(n):
    rng = np.random.default_rng(n)
    x = fieldgen.random_coords(n, rng, jitter=0.5)
    op = grid.make_dimop(x)
    Mf = A.tridiag_dense(op.ma, op.mb, op.mc)
    assert np.abs(Mf - dense.mass_1d_quadrature(x)).max() <= 1e-14
    Mc = A.tridiag_dense(*op.coarse_mass)
    assert np.abs(Mc - dense.mass_1d_quadrature(x[op.cidx])).max() <= 1e-14
    P = A.prolongation_dense(op)
    assert np.abs(P - dense.prolongation_1d(x, x[op.cidx])).max() <= 1e-15
    assert np.abs(P.T @ Mf @ P - Mc).max() <= 1e-14


def test_roundtrip_fp64_c1_field():
    u = fieldgen.bumps2d()
    h = grid.Hierarchy(u.shape)
    c0, cb = X.decompose(u, h)
    r = X.recompose(c0, cb, h)
    assert np.abs(r - u).max() / np.abs(u).max() <= 1e-12


@pytest.mark.parametrize("shape", [(33,), (20, 17), (9, 10, 11), (5, 6, 5, 6), (2, 17, 9)])
def test_roundtrip_fp64_random_nonuniform(shape):
    rng = np.random.default_rng(len(shape) * 100 + shape[0])
    xs = [fieldgen.random_coords(n, rng) for n in shape]
    h = grid.Hierarchy(shape, xs)
    u = fieldgen.random_field(shape, rng)
    c0, cb = X.decompose(u, h)
    s = Q.to_stream(c0, cb, h)
    assert len(s) == u.size
    c0b, cbb = Q.from_stream(s, h, np.float64)
    r = X.recompose(c0b, cbb, h)
    assert np.abs(r - u).max() / np.abs(u).max() <= 1e-12


def test_linearity_and_affine_coordinate_invariance():
    rng = np.random.default_rng(5)
    shape = (13, 9)
    xs = [fieldgen.random_coords(n, rng) for n in shape]
    h = grid.Hierarchy(shape, xs)
    u = rng.standard_normal(shape)
    v = rng.standard_normal(shape)
    su = Q.to_stream(*X.decompose(u, h), h)
    sv = Q.to_stream(*X.decompose(v, h), h)
    sw = Q.to_stream(*X.decompose(2.0 * u - 3.0 * v, h), h)
    assert np.abs(sw - (2.0 * su - 3.0 * sv)).max() <= 1e-12
    h2 = grid.Hierarchy(shape, [7.0 * x + 3.0 for x in xs])
    su2 = Q.to_stream(*X.decompose(u, h2), h2)
    assert np.abs(su2 - su).max() <= 1e-12


# ------------------------------------------------------------- allocation
def test_correction_matrix_hand_value_n3():
    g = GOLD["correction_matrix_n3_uniform"]
    op = grid.make_dimop(np.arange(3.0))
    Am = A.correction_matrix(op)
    assert np.allclose(Am, np.array(g["A"]), atol=1e-15)
    assert abs(A.norm_inf(Am) - g["norm_inf"]) <= 1e-15


def test_correction_norm_closed_form_limit():
    g = GOLD["correction_norm_uniform_limit"]
    assert abs(g["value"] - (1.0 + math.sqrt(3.0) / 2.0)) < 1e-15
    op = grid.make_dimop(np.arange(257.0))
    Am = A.correction_matrix(op)
    assert abs(A.norm_inf(Am) - g["value"]) <= 1e-12
    assert abs(Am[64, 128] - g["centre_entry"]) <= 1e-12


@pytest.mark.parametrize("n", [3, 4, 5, 8, 17, 64, 129])
def test_column_norm_equals_dense_lapack_norm(n):
    """The column-by-column operator norm used by the allocation equals the dense LAPACK one."""
    rng = np.random.default_rng(n)
    for x in (np.arange(float(n)), fieldgen.random_coords(n, rng, jitter=0.5)):
        op = grid.make_dimop(x)
        dense_norm = A.norm_inf(A.correction_matrix(op))
        assert abs(A.correction_norm(op) - dense_norm) <= 1e-14 * dense_norm


def test_norm_invariant_to_uniform_scale():
    a = A.norm_inf(A.correction_matrix(grid.make_dimop(np.arange(9.0))))
    b = A.norm_inf(A.correction_matrix(grid.make_dimop(0.01 * np.arange(9.0) - 4.0)))
    assert abs(a - b) <= 1e-13


def test_plain_bins_meet_a_priori_bound():
    h = grid.Hierarchy((129, 129))
    b = A.plain_bins(h, 1e-3)
    assert abs(A.error_bound(h, b) - 1e-3) <= 1e-15
    bw = A.count_weighted_bins(h, 1e-3)
    assert abs(A.error_bound(h, bw) - 1e-3) <= 1e-15


# ------------------------------------------------------------- quantization
def test_quantize_ties_and_bound():
    g = GOLD["quantize_ties"]
    assert list(Q.quantize(np.array(g["c"]), g["b"])) == g["q"]
    rng = np.random.default_rng(2)
    c = rng.standard_normal(10000).astype(np.float32)
    b = 0.013
    q = Q.quantize(c, b)
    ch = Q.dequantize(q, b, np.float32)
    assert np.abs(c.astype(np.float64) - ch).max() <= b / 2 * (1 + 1e-6)


def test_stream_order_by_hand():
    """5x4 grid, one level: coarsest 3x3 (rows 0,2,4 x cols 0,2,3), then mask 1 (rows 1,3 x cols 0,2,3),
    mask 2 (rows 0,2,4 x col 1), mask 3 (rows 1,3 x col 1)."""
    h = grid.Hierarchy((5, 4))
    assert h.L == 1
    lab = np.arange(20.0).reshape(5, 4)
    coarsest = lab[np.ix_([0, 2, 4], [0, 2, 3])]
    s = Q.to_stream(coarsest, [None, lab], h)
    expect = [0, 2, 3, 8, 10, 11, 16, 18, 19,
              4, 6, 7, 12, 14, 15,
              1, 9, 17,
              5, 13]
    assert list(s) == expect


def test_symbols_escape_edges():
    q = np.array([0, 4095, -4095, 4096, -4096, 100000])
    s, o = Q.to_symbols(q, 8192)
    assert list(s) == [4096, 8191, 1, 0, 0, 0]
    assert list(o) == [4096, -4096, 100000]
    assert list(Q.from_symbols(s, o, 8192)) == list(q)


# ------------------------------------------------------------------ Huffman
def test_huffman_hand_example():
    g = GOLD["huffman_small"]
    L = H.code_lengths(g["counts"])
    assert list(L) == g["lengths"]
    assert [int(c) for c in H.canonical_codes(L)] == g["codes"]
    for key in ("bitpack_small", "bitpack_two_chunks"):
        b = GOLD[key]
        bits, words = H.encode(b["symbols"], L, H.canonical_codes(L), b.get("chunk", 4096))
        assert bits == b["chunk_bits"] and words == b["words"]


def _textbook_cost(counts):
    heap = [c for c in counts if c > 0]
    if len(heap) <= 1:
        return sum(heap)
    heapq.heapify(heap)
    cost = 0
    while len(heap) > 1:
        a = heapq.heappop(heap)
        b = heapq.heappop(heap)
        cost += a + b
        heapq.heappush(heap, a + b)
    return cost


@pytest.mark.parametrize("seed", range(6))
def test_huffman_optimal_kraft_roundtrip(seed):
    rng = np.random.default_rng(seed)
    dict_size = 256
    n = int(rng.integers(1, 5000))
    if seed == 0:
        sym = np.full(n, 17)
    else:
        sym = np.clip(np.round(rng.laplace(128, 4 + 10 * seed, size=n)), 0, 255).astype(np.int64)
    hist = H.histogram(sym, dict_size)
    L = H.code_lengths(hist)
    codes = H.canonical_codes(L)
    used = L > 0
    kraft = sum(2.0 ** -int(v) for v in L[used])
    assert kraft == 1.0 or used.sum() == 1
    if used.sum() > 1:
        assert int((hist * L).sum()) == _textbook_cost(hist)
    # prefix-free canonical codes
    pairs = sorted((int(L[s]), int(codes[s])) for s in range(dict_size) if used[s])
    for (l1, c1), (l2, c2) in zip(pairs, pairs[1:]):
        assert (c2 >> (l2 - l1)) != c1
    bits, words = H.encode(sym, L, codes, 97)
    out = H.decode(words, bits, L, codes, n, 97)
    assert np.array_equal(out, sym)


# -------------------------------------------------------------- end to end
@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-4])
def test_c1_bound_and_roundtrip(tol):
    u = fieldgen.bumps2d()
    buf = codec.compress(u, tol)
    r = codec.decompress(buf)
    tau = tol * np.abs(u).max()
    assert np.abs(r - u).max() <= tau
    assert len(buf) < u.nbytes


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_bound_adversarial_signs(dtype):
    """Checkerboard and random sign fields on small nonuniform grids."""
    rng = np.random.default_rng(9)
    for shape in [(17, 17), (9, 10, 11), (33,)]:
        xs = [fieldgen.random_coords(n, rng) for n in shape]
        idx = np.indices(shape).sum(axis=0)
        for u in ((-1.0) ** idx, rng.choice([-1.0, 1.0], size=shape), rng.standard_normal(shape)):
            u = u.astype(dtype)
            for tol in (1e-1, 1e-3):
                buf = codec.compress(u, tol, coords=xs, dict_size=256, chunk=64)
                r = codec.decompress(buf)
                assert r.dtype == dtype
                err = np.abs(r.astype(np.float64) - u.astype(np.float64)).max()
                assert err <= tol * np.abs(u).max()


def test_format_parse_and_errors():
    rng = np.random.default_rng(1)
    u = rng.standard_normal((9, 12))
    xs = [None, fieldgen.random_coords(12, rng)]
    buf = codec.compress(u, 1e-2, coords=xs, dict_size=1024, chunk=50)
    hd = codec.parse(buf)
    assert hd.shape == (9, 12) and hd.coords[0] is None and np.array_equal(hd.coords[1], xs[1])
    assert hd.offsets["end"] == len(buf) and hd.dict_size == 1024 and hd.chunk == 50
    with pytest.raises(ValueError):
        codec.parse(buf[:-1])
    with pytest.raises(ValueError):
        codec.parse(b"XXXX" + buf[4:])
    with pytest.raises(ValueError):
        codec.compress(np.array([1.0, np.nan, 2.0]), 1e-3)


def test_zero_field():
    u = np.zeros((9, 9))
    r = codec.decompress(codec.compress(u, 1e-3))
    assert np.all(r == 0)


# --------------------------------------------------------------------- MLP
def test_mlp_gradients_central_difference():
    rng = np.random.default_rng(0)
    params = mlp.init(3, sizes=(4, 8, 8, 1))
    X_ = rng.standard_normal((16, 4))
    y = rng.standard_normal(16)

    def loss_of(ps):
        out, _ = mlp.forward(ps, X_)
        return mlp.mse(out, y)[0]

    out, cache = mlp.forward(params, X_)
    _, dout = mlp.mse(out, y)
    grads = mlp.backward(params, cache, dout)
    h = 1e-6
    for k in range(3):
        for j in range(2):
            P = params[k][j]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                i = it.multi_index
                old = P[i]
                P[i] = old + h
                lp = loss_of(params)
                P[i] = old - h
                lm = loss_of(params)
                P[i] = old
                fd = (lp - lm) / (2 * h)
                g = grads[k][j][i]
                assert abs(fd - g) <= 1e-6 * max(1.0, abs(g))


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step moves every weight by lr*sign(g) (for |g| >> eps)."""
    params = [[np.array([[1.0, -2.0]]), np.array([0.5])]]
    grads = [[np.array([[0.3, -4.0]]), np.array([2.0])]]
    m = mlp.adam_init(params)
    v = mlp.adam_init(params)
    mlp.adam_step(params, grads, m, v, 1, lr=0.1)
    assert np.allclose(params[0][0], [[0.9, -1.9]], atol=1e-7)
    assert np.allclose(params[0][1], [0.4], atol=1e-7)


# ----------------------------------------------------------------- out-of-core chunks
def test_chunked_slab_plan_covers_the_array_in_slabs_of_three_or_more():
    from oracle import chunked as K

    for n0 in range(3, 70):
        for slab in (3, 4, 7, 16, 64):
            b = K.slab_bounds(n0, slab)
            assert b[0][0] == 0 and b[-1][1] == n0
            assert all(b[i][1] == b[i + 1][0] for i in range(len(b) - 1))
            assert all(p1 - p0 >= 3 for p0, p1 in b)
            assert all(p1 - p0 == slab for p0, p1 in b[:-1])
            assert b[-1][1] - b[-1][0] < slab + 3  # a remainder below 3 planes joined the last slab
    with pytest.raises(ValueError):
        K.slab_bounds(10, 2)


def test_chunked_single_slab_is_the_plain_format_at_the_arrays_tolerance():
    from oracle import chunked as K

    rng = np.random.default_rng(41)
    u = fieldgen.random_field((12, 9, 10), rng).astype(np.float32)
    buf = K.compress_chunked(u, 1e-3, 64)
    c = K.parse_chunked(buf)
    assert c["n_slabs"] == 1 and c["tau_abs"] == 1e-3 * float(np.abs(u).max())
    assert buf[c["offsets"][0]:] == codec.compress(u, c["tau_abs"], rel=False)


def test_chunked_slabs_share_the_global_tolerance_and_meet_it():
    from oracle import chunked as K

    rng = np.random.default_rng(42)
    shape = (23, 11, 9)
    u = fieldgen.random_field(shape, rng)
    u[:8] *= 1e-3  # the first slab's own max is far below the array's
    xs = [fieldgen.random_coords(n, rng) for n in shape]
    buf = K.compress_chunked(u, 1e-4, 8, coords=xs)
    c = K.parse_chunked(buf)
    tau = 1e-4 * float(np.abs(u).max())
    assert c["tau_abs"] == tau and c["n_slabs"] == 3  # 8 + 8 + 7 planes
    for k in range(c["n_slabs"]):
        hd = codec.parse(buf[c["offsets"][k]:c["offsets"][k + 1]])
        assert hd.tau_abs == tau and not hd.rel
    r = K.decompress_chunked(buf)
    assert float(np.abs(r - u).max()) <= tau


# ------------------------------------------------------- escaped values
def test_escape_packing_hand_example():
    g = GOLD["escape_packing_small"]
    h = grid.Hierarchy(tuple(g["shape"]))
    q = np.array(g["q"], dtype=np.int64)
    counts, widths, words = Q.pack_escapes(q, h, g["dict_size"])
    assert counts == g["counts"] and widths == g["widths"]
    assert [int(w) for w in words] == g["words"]
    sym, outl = Q.to_symbols(q, g["dict_size"])
    assert list(sym) == g["symbols"]
    back = Q.unpack_escapes(words, counts, widths, g["dict_size"])
    assert list(back) == list(outl)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_escape_packing_roundtrip_extremes(seed):
    """Random escapes (both signs, |q| from R to 2^62, a level whose codes are all
    0, a level without escapes) come back in stream order; widths are the bit
    lengths of each level's largest code, and each level starts on a word."""
    rng = np.random.default_rng(seed)
    h = grid.Hierarchy((9, 17))
    n = 9 * 17
    dict_size = 256
    R = dict_size // 2
    off = Q.level_offsets(h)
    q = rng.integers(-R + 1, R, size=n)
    lv = [l for l in range(h.L + 1)]
    big = rng.choice(n, size=n // 3, replace=False)
    q[big] = np.sign(rng.standard_normal(len(big))).astype(np.int64) * (R + rng.integers(0, 2 ** 62, size=len(big)))
    q[off[1]:off[2]] = R  # every escape of level 1 has code 0
    counts, widths, words = Q.pack_escapes(q, h, dict_size)
    for l in lv:
        ql = q[off[l]:off[l + 1]]
        e = ql[np.abs(ql) >= R]
        assert counts[l] == len(e)
        if len(e):
            vmax = max(2 * (abs(int(x)) - R) + (1 if x < 0 else 0) for x in e)
            assert widths[l] == vmax.bit_length()
    assert len(words) == sum((c * w + 31) // 32 for c, w in zip(counts, widths))
    _, outl = Q.to_symbols(q, dict_size)
    assert np.array_equal(Q.unpack_escapes(words, counts, widths, dict_size, block=7), outl)
