"""Pins of the fp64 oracle against facts independent of its own code.

Each test checks the oracle (stencil definition of SPIDER Sec. 2.2, zero halo,
Jacobi steps) against a library routine that reduces to the same operation, a
closed form, or an invariant of the definition, chosen so that a dropped tap, a
flipped or transposed kernel, a wrong halo or a wrong step count fails at least
one of them.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import stencil_inputs as si

pytestmark = pytest.mark.filterwarnings("ignore")


def _scipy_steps(w, x, steps):
    y = np.asarray(x, dtype=np.float64)
    for _ in range(steps):
        y = ndimage.correlate(y, w, mode="constant", cval=0.0)
    return y


@pytest.mark.parametrize("ndim,r,kind,shape,steps", [
    (2, 1, "box", (17, 23), 3), (2, 2, "box", (20, 31), 2), (2, 3, "box", (32, 29), 4),
    (2, 3, "star", (25, 40), 3), (2, 1, "star", (9, 7), 5), (3, 1, "box", (8, 9, 11), 3),
    (3, 1, "star", (7, 8, 6), 4), (3, 2, "box", (9, 10, 12), 2), (2, 3, "box", (4, 5), 2),
    (2, 1, "box", (1, 1), 2), (3, 1, "box", (1, 3, 1), 2)])
def test_matches_scipy_correlate(oracle_mod, ndim, r, kind, shape, steps):
    # scipy.ndimage.correlate with mode='constant', cval=0 is this stencil with a zero halo.
    rng = np.random.default_rng(7 + r + ndim)
    w = np.zeros((2 * r + 1,) * ndim)
    m = si.shape_mask(ndim, r, kind)
    w[m] = rng.uniform(-1, 1, int(m.sum()))   # asymmetric: a flip or transpose fails
    x = rng.uniform(-1, 1, shape)
    got = oracle_mod.apply(w, x, steps)
    ref = _scipy_steps(w, x, steps)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_delta_response_is_unflipped_kernel(oracle_mod):
    # One step on a unit impulse at p0 gives out[p0 - o] = w[o]: correlation, not convolution.
    r = 3
    rng = np.random.default_rng(1)
    w = rng.uniform(-2, 2, (2 * r + 1, 2 * r + 1))
    x = np.zeros((21, 19))
    x[10, 9] = 1.0
    y = oracle_mod.apply(w, x, 1)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            assert y[10 - dy, 9 - dx] == w[dy + r, dx + r]
    mask = np.ones_like(y, dtype=bool)
    mask[10 - r:10 + r + 1, 9 - r:9 + r + 1] = False
    assert np.all(y[mask] == 0.0)


def test_delta_response_3d(oracle_mod):
    rng = np.random.default_rng(2)
    w = rng.uniform(-2, 2, (3, 3, 3))
    x = np.zeros((7, 8, 9))
    x[3, 4, 4] = 1.0
    y = oracle_mod.apply(w, x, 1)
    for o in np.ndindex(3, 3, 3):
        assert y[3 - (o[0] - 1), 4 - (o[1] - 1), 4 - (o[2] - 1)] == w[o]


@pytest.mark.parametrize("n", [1, 5, 12, 20])
def test_binomial_closed_form(oracle_mod, n):
    # Taps [1/4, 1/2, 1/4] along x only: n steps on a delta give C(2n, k) / 4^n, exact in fp64.
    w = np.zeros((3, 3))
    w[1] = [0.25, 0.5, 0.25]
    x = np.zeros((3, 2 * n + 41))
    c = n + 20
    x[1, c] = 1.0
    y = oracle_mod.apply(w, x, n)
    expect = np.zeros(x.shape[1])
    for k in range(2 * n + 1):
        expect[c - n + k] = math.comb(2 * n, k) / 4.0 ** n
    assert np.array_equal(y[1], expect)
    assert np.all(y[0] == 0) and np.all(y[2] == 0)


@pytest.mark.parametrize("modes,steps", [((1, 1, 1), 7), ((2, 3, 1), 4), ((3, 1, 2), 10)])
def test_heat3d_zero_halo_eigenvector(oracle_mod, modes, steps):
    # u = prod_i sin(pi m_i (j_i + 1) / (N_i + 1)) is an eigenvector of the zero-halo 7-point
    # update with eigenvalue 1 - 2 alpha sum_i (1 - cos(pi m_i / (N_i + 1))).
    alpha = 0.1
    shape = (9, 11, 13)
    w = si.heat3d_coeffs(alpha)
    axes = [np.sin(np.pi * m * (np.arange(N) + 1) / (N + 1)) for m, N in zip(modes, shape)]
    u = axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]
    lam = 1.0 - 2.0 * alpha * sum(1.0 - np.cos(np.pi * m / (N + 1)) for m, N in zip(modes, shape))
    y = oracle_mod.apply(w, u, steps)
    assert np.max(np.abs(y - lam ** steps * u)) <= 1e-13


def test_separable_kernel_equals_two_passes(oracle_mod):
    # w = u (x) v: one step equals a 1-D pass along x with v then along y with u.
    rng = np.random.default_rng(3)
    r = 3
    u = rng.uniform(-1, 1, 2 * r + 1)
    v = rng.uniform(-1, 1, 2 * r + 1)
    w = np.outer(u, v)
    x = rng.uniform(-1, 1, (30, 33))
    y = oracle_mod.apply(w, x, 1)
    t = np.zeros_like(x)
    xp = np.pad(x, ((0, 0), (r, r)))
    for dx in range(2 * r + 1):
        t += v[dx] * xp[:, dx:dx + x.shape[1]]
    z = np.zeros_like(x)
    tp = np.pad(t, ((r, r), (0, 0)))
    for dy in range(2 * r + 1):
        z += u[dy] * tp[dy:dy + x.shape[0], :]
    assert np.max(np.abs(y - z)) <= 1e-14 * 49


def test_linearity(oracle_mod):
    rng = np.random.default_rng(4)
    w = rng.uniform(-1, 1, (5, 5))
    a = rng.uniform(-1, 1, (24, 27))
    b = rng.uniform(-1, 1, (24, 27))
    al, be = 0.75, -1.25
    lhs = oracle_mod.apply(w, al * a + be * b, 6)
    rhs = al * oracle_mod.apply(w, a, 6) + be * oracle_mod.apply(w, b, 6)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


@pytest.mark.parametrize("ndim,r,steps", [(2, 1, 5), (2, 3, 4), (3, 1, 3)])
def test_constant_preserved_in_interior(oracle_mod, ndim, r, steps):
    # Taps summing to 1 keep a constant field wherever the steps*r neighbourhood stays inside.
    w = si.coeffs_uniform01(ndim, r, 11)
    shape = (40,) * ndim if ndim == 2 else (20, 21, 22)
    x = np.full(shape, 3.5)
    y = oracle_mod.apply(w, x, steps)
    m = steps * r
    inner = y[tuple(slice(m, s - m) for s in shape)]
    assert np.max(np.abs(inner - 3.5)) <= 1e-13
    # ...and loses mass at the zero halo
    assert y[(0,) * ndim] < 3.5


def test_restart_is_bitwise(oracle_mod):
    rng = np.random.default_rng(5)
    w = rng.uniform(-1, 1, (7, 7)) / 20
    x = rng.uniform(0, 1, (31, 26))
    once = oracle_mod.apply(w, x, 9)
    twice = oracle_mod.apply(w, oracle_mod.apply(w, x, 4), 5)
    assert np.array_equal(once, twice)


def test_zero_steps_copies_and_thread_count_invariance(oracle_mod):
    rng = np.random.default_rng(6)
    w = rng.uniform(-1, 1, (3, 3, 3))
    x = rng.uniform(0, 1, (10, 12, 14))
    assert np.array_equal(oracle_mod.apply(w, x, 0), x)
    assert np.array_equal(oracle_mod.apply(w, x, 3, nthreads=1), oracle_mod.apply(w, x, 3, nthreads=4))


def test_rel_errors_metric(oracle_mod):
    ref = np.array([3.0, 4.0])
    y = np.array([3.0, 4.5])
    rms, mx = oracle_mod.rel_errors(y, ref)
    assert rms == pytest.approx(0.5 / 5.0) and mx == pytest.approx(0.5 / 4.0)


def test_sampled_point_matches_full_grid(oracle_mod):
    # A point's value after T steps depends only on inputs within T*r: the oracle on the
    # cone sub-grid reproduces the full-grid value (this is how full-size GPU runs are sampled).
    rng = np.random.default_rng(8)
    r, T = 2, 4
    w = rng.uniform(-1, 1, (5, 5)) / 10
    x = rng.uniform(0, 1, (60, 70))
    full = oracle_mod.apply(w, x, T)
    for (py, px) in [(30, 35), (3, 4), (59, 69), (10, 66)]:
        y0, y1 = max(0, py - T * r), min(60, py + T * r + 1)
        x0, x1 = max(0, px - T * r), min(70, px + T * r + 1)
        sub = oracle_mod.apply(w, x[y0:y1, x0:x1], T)
        assert sub[py - y0, px - x0] == full[py, px]


# ------------------------------------------------------------------ 1-D (the paper's d = 1 stencils)


@pytest.mark.parametrize("r,n,steps", [(1, 37, 4), (2, 64, 3), (3, 5, 2), (1, 1, 3), (2, 1000, 6)])
def test_1d_matches_scipy_correlate(oracle_mod, r, n, steps):
    rng = np.random.default_rng(30 + r)
    w = rng.uniform(-1, 1, 2 * r + 1)   # asymmetric: a flip fails
    x = rng.uniform(-1, 1, n)
    got = oracle_mod.apply(w, x, steps)
    ref = _scipy_steps(w, x, steps)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_1d_delta_response_is_unflipped(oracle_mod):
    w = np.array([0.5, -1.25, 2.0, 0.75, -3.0])
    x = np.zeros(15)
    x[7] = 1.0
    y = oracle_mod.apply(w, x, 1)
    for o in range(-2, 3):
        assert y[7 - o] == w[o + 2]
    assert np.count_nonzero(y) == 5


@pytest.mark.parametrize("n", [1, 7, 20])
def test_1d_binomial_closed_form(oracle_mod, n):
    x = np.zeros(2 * n + 31)
    c = n + 15
    x[c] = 1.0
    y = oracle_mod.apply(np.array([0.25, 0.5, 0.25]), x, n)
    expect = np.zeros_like(x)
    for k in range(2 * n + 1):
        expect[c - n + k] = math.comb(2 * n, k) / 4.0 ** n
    assert np.array_equal(y, expect)


@pytest.mark.parametrize("m,steps", [(1, 9), (4, 5), (11, 3)])
def test_1d_heat_zero_halo_eigenvector(oracle_mod, m, steps):
    # u_j = sin(pi m (j + 1) / (N + 1)) is an eigenvector of [a, 1 - 2a, a] with the zero
    # halo, eigenvalue 1 - 2a (1 - cos(pi m / (N + 1))).
    a, N = 0.2, 23
    u = np.sin(np.pi * m * (np.arange(N) + 1) / (N + 1))
    lam = 1.0 - 2.0 * a * (1.0 - np.cos(np.pi * m / (N + 1)))
    y = oracle_mod.apply(np.array([a, 1 - 2 * a, a]), u, steps)
    assert np.max(np.abs(y - lam ** steps * u)) <= 1e-14


def test_1d_equals_2d_single_row(oracle_mod):
    # a 1-D stencil on a line is the 2-D stencil with only the centre kernel row on a 1 x n grid
    rng = np.random.default_rng(44)
    w1 = rng.uniform(-1, 1, 5)
    w2 = np.zeros((5, 5))
    w2[2] = w1
    x = rng.uniform(-1, 1, 301)
    assert np.array_equal(oracle_mod.apply(w1, x, 4), oracle_mod.apply(w2, x[None, :], 4)[0])


def test_1d_linearity_and_constant_interior(oracle_mod):
    rng = np.random.default_rng(45)
    w = rng.uniform(0, 1, 5)
    w /= w.sum()
    a, b = rng.uniform(-1, 1, 200), rng.uniform(-1, 1, 200)
    lhs = oracle_mod.apply(w, 2.5 * a - 0.75 * b, 3)
    rhs = 2.5 * oracle_mod.apply(w, a, 3) - 0.75 * oracle_mod.apply(w, b, 3)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14
    y = oracle_mod.apply(w, np.full(200, 3.0), 5)
    assert np.max(np.abs(y[10:-10] - 3.0)) <= 1e-14
