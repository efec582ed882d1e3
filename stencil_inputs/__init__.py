"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws numbers: coefficients, grids and request streams.  It
applies no stencil and holds none of the strided-swap method's arithmetic, so
both the GPU path's tests and the fp64 oracle can take their inputs from it.

Stencil shapes follow SPIDER Sec. 2.2: "box" stencils use every offset in
[-r, r]^d, "star" stencils only the offsets on the coordinate axes.  Coefficient
arrays are (2r+1,)*d, w[dz][dy][dx] multiplying x[p + offset], zero where the
shape has no tap.

The paper's own workloads are synthetic grids (Sec. 4.1 "Benchmarks": 1-D and
2-D star/box stencils of radius 1..3 on (10240, 10240) grids).  The recipes
below give the shapes, sizes and value distributions of the five workloads this
library is measured on; `stable_*` helpers reject seeds whose stencil would grow
without bound (see `symbol_max`).
"""
import numpy as np

# --------------------------------------------------------------------------- shapes


def shape_mask(ndim, r, kind):
    """Boolean (2r+1,)*ndim mask of the taps of a 'box' or 'star' stencil."""
    k = 2 * r + 1
    if kind == "box":
        return np.ones((k,) * ndim, dtype=bool)
    if kind == "star":
        m = np.zeros((k,) * ndim, dtype=bool)
        for ax in range(ndim):
            idx = [r] * ndim
            for t in range(k):
                idx[ax] = t
                m[tuple(idx)] = True
        return m
    raise ValueError(kind)


def symbol_max(w, n=256):
    """max over a n^d frequency grid of |sum_o w[o] exp(i theta . o)|.

    A value <= 1 means repeated application cannot amplify any Fourier mode (the
    zero-halo operator is a compression of the infinite-grid one, so its 2-norm
    is bounded by this too).  Computed with the FFT of the zero-padded taps.
    """
    w = np.asarray(w, dtype=np.float64)
    pad = np.zeros((n,) * w.ndim)
    pad[tuple(slice(0, s) for s in w.shape)] = w
    return float(np.max(np.abs(np.fft.fftn(pad))))


def _normalise(v):
    s = float(np.sum(v))
    return v / s


def coeffs_uniform01(ndim, r, seed, kind="box"):
    """Taps ~ U[0,1), rescaled to sum 1 (non-negative, hence always stable)."""
    m = shape_mask(ndim, r, kind)
    rng = np.random.default_rng(seed)
    w = np.zeros(m.shape)
    w[m] = rng.random(int(m.sum()))
    return _normalise(w)


def _stable(draw, ndim, r, kind, seed0, max_tries=10000):
    m = shape_mask(ndim, r, kind)
    for s in range(seed0, seed0 + max_tries):
        rng = np.random.default_rng(s)
        w = np.zeros(m.shape)
        w[m] = draw(rng, int(m.sum()))
        tot = float(np.sum(w))
        if abs(tot) < 1e-6:
            continue
        w = w / tot
        if symbol_max(w) <= 1.0 + 1e-9:
            return w, s
    raise RuntimeError("no stable seed found")


def stable_coeffs_uniform_pm1(ndim, r, seed0, kind="star"):
    """Taps ~ U[-1,1], rescaled to sum 1; first seed >= seed0 that is stable.

    Returns (w, accepted_seed)."""
    return _stable(lambda g, n: g.uniform(-1.0, 1.0, n), ndim, r, kind, seed0)


def stable_coeffs_gaussian(ndim, r, seed0, kind="box"):
    """Taps ~ N(0,1), rescaled to sum 1; first seed >= seed0 that is stable.

    Returns (w, accepted_seed)."""
    return _stable(lambda g, n: g.standard_normal(n), ndim, r, kind, seed0)


def heat3d_coeffs(alpha=0.1):
    """Explicit 7-point heat update: centre 1 - 6 alpha, six face neighbours alpha."""
    w = np.zeros((3, 3, 3))
    w[1, 1, 1] = 1.0 - 6.0 * alpha
    for d in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        w[d] = alpha
    return w


def integer_coeffs(ndim, r, lo, hi, seed, kind="box"):
    """Integer taps drawn uniformly from [lo, hi] (for exactness tests)."""
    m = shape_mask(ndim, r, kind)
    rng = np.random.default_rng(seed)
    w = np.zeros(m.shape)
    w[m] = rng.integers(lo, hi + 1, int(m.sum()))
    return w


# --------------------------------------------------------------------------- grids


def grid_uniform01(shape, seed, dtype=np.float32):
    """Grid values ~ U[0,1)."""
    rng = np.random.default_rng(seed)
    return rng.random(shape, dtype=np.float64 if dtype == np.float64 else np.float32).astype(dtype, copy=False)


def grid_integer(shape, lo, hi, seed, dtype=np.float32):
    """Integer grid values drawn uniformly from [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, shape).astype(dtype)


def grid_integer_int8(shape, lo, hi, seed):
    """Integer grid values drawn uniformly from [lo, hi] (-128 <= lo <= hi <= 127),
    drawn directly as int8 so grids of 2^31 points stay at one byte per point."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, shape, dtype=np.int8)


def grid_sinusoids(shape, seed, dtype=np.float32, nwaves=8, noise=0.01):
    """Smooth 2-D field: mean of `nwaves` random plane sinusoids plus uniform noise.

    f(y, x) = (1/nwaves) sum_k a_k sin(2 pi (kx_k x / Nx + ky_k y / Ny) + phi_k)
              + noise * U[-1, 1),
    a_k ~ U[0.5, 1], kx_k, ky_k ~ U{1..16}, phi_k ~ U[0, 2 pi).
    Evaluated as sin(u + v) = sin u cos v + cos u sin v, i.e. one (Ny x 2n) @ (2n x Nx)
    product, row block by row block.
    """
    ny, nx = shape
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.0, nwaves)
    kx = rng.integers(1, 17, nwaves)
    ky = rng.integers(1, 17, nwaves)
    ph = rng.uniform(0.0, 2.0 * np.pi, nwaves)
    u = 2.0 * np.pi * kx[:, None] * (np.arange(nx, dtype=np.float64) / nx)[None, :] + ph[:, None]  # n x Nx
    right = np.concatenate([np.sin(u), np.cos(u)], axis=0)                                         # 2n x Nx
    out = np.empty((ny, nx), dtype=dtype)
    nrng = np.random.default_rng(seed + 1_000_003)
    blk = 1024
    for y0 in range(0, ny, blk):
        ys = np.arange(y0, min(ny, y0 + blk), dtype=np.float64) / ny
        v = 2.0 * np.pi * ys[:, None] * ky[None, :]                                                 # b x n
        left = np.concatenate([a * np.cos(v), a * np.sin(v)], axis=1) / nwaves                       # b x 2n
        f = left @ right
        f += noise * nrng.uniform(-1.0, 1.0, f.shape)
        out[y0:y0 + ys.shape[0]] = f.astype(dtype)
    return out


# --------------------------------------------------------------------------- workloads


def workload(name, small=False):
    """Coefficients, grid shape, steps and grid generator of a named workload.

    Returns a dict: name, ndim, r, kind, coeffs, shape, steps, make_grid(dtype),
    seeds.  `small=True` gives the same recipe on a grid the oracle finishes in
    seconds (used for parity tests).
    """
    if name == "box2d9p_256_f64":
        w = coeffs_uniform01(2, 1, 1)
        shape = (256, 256)
        return dict(name=name, ndim=2, r=1, kind="box", coeffs=w, shape=shape, steps=10,
                    make_grid=lambda dt=np.float64, s=shape: grid_uniform01(s, 2, dt),
                    seeds=dict(coeffs=1, grid=2))
    if name == "star2d13p_8192":
        w, s = stable_coeffs_uniform_pm1(2, 3, 0, "star")
        shape = (384, 320) if small else (8192, 8192)
        steps = 12 if small else 100
        return dict(name=name, ndim=2, r=3, kind="star", coeffs=w, shape=shape, steps=steps,
                    make_grid=lambda dt=np.float32, s=shape: grid_uniform01(s, 2, dt),
                    seeds=dict(coeffs=s, grid=2))
    if name == "box2d49p_10240":
        w, s = stable_coeffs_gaussian(2, 3, 0, "box")
        shape = (300, 520) if small else (10240, 10240)
        steps = 10 if small else 50
        return dict(name=name, ndim=2, r=3, kind="box", coeffs=w, shape=shape, steps=steps,
                    make_grid=lambda dt=np.float32, s=shape: grid_sinusoids(s, 3, dt),
                    seeds=dict(coeffs=s, grid=3))
    if name == "box2d7r_10240":
        # Box-2D7R (r = 7, 225 taps), the stencil of the paper's row-swap comparison
        # (Table 3); it states no size or recipe there, so the Box-2D49P recipe is used
        w, s = stable_coeffs_gaussian(2, 7, 0, "box")
        shape = (300, 520) if small else (10240, 10240)
        steps = 10 if small else 50
        return dict(name=name, ndim=2, r=7, kind="box", coeffs=w, shape=shape, steps=steps,
                    make_grid=lambda dt=np.float32, s=shape: grid_sinusoids(s, 3, dt),
                    seeds=dict(coeffs=s, grid=3))
    if name == "box3d27p_512":
        w = coeffs_uniform01(3, 1, 4)
        shape = (40, 36, 300) if small else (512, 512, 512)
        steps = 5 if small else 20
        return dict(name=name, ndim=3, r=1, kind="box", coeffs=w, shape=shape, steps=steps,
                    make_grid=lambda dt=np.float32, s=shape: grid_uniform01(s, 5, dt),
                    seeds=dict(coeffs=4, grid=5))
    if name == "heat3d_256":
        w = heat3d_coeffs(0.1)
        shape = (24, 40, 280) if small else (256, 256, 256)
        steps = 5 if small else 20
        return dict(name=name, ndim=3, r=1, kind="star", coeffs=w, shape=shape, steps=steps,
                    make_grid=lambda dt=np.float32, s=shape: grid_uniform01(s, 6, dt),
                    seeds=dict(coeffs=None, grid=6))
    if name in ("1d3p_10240000", "1d5p_10240000"):
        # the paper's 1-D benchmarks: r = 1 and r = 2 on (1, 10 240 000); it states no step
        # count or coefficient recipe, so: U[0,1) taps normalised to sum 1, U[0,1) values, 100 steps
        r = 1 if name.startswith("1d3p") else 2
        w = coeffs_uniform01(1, r, 7 + r)
        shape = (50000,) if small else (10240000,)
        steps = 20 if small else 100
        return dict(name=name, ndim=1, r=r, kind="box", coeffs=w, shape=shape, steps=steps,
                    make_grid=lambda dt=np.float32, s=shape: grid_uniform01(s, 8, dt),
                    seeds=dict(coeffs=7 + r, grid=8))
    raise KeyError(name)


SERVING_STENCILS = ("box2d9p", "star2d13p", "box2d49p", "box3d27p")


def serving_requests(n, rate_per_s, seed):
    """Poisson request stream for the serving mix.

    Each request: arrival time (exponential gaps at `rate_per_s`), a stencil drawn
    uniformly from SERVING_STENCILS, a 2-D side log-uniform on [512, 8192]
    rounded to a multiple of 64 or a 3-D side log-uniform on [64, 384] rounded to
    a multiple of 16, steps uniform on 1..100, and a grid seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        st = SERVING_STENCILS[int(rng.integers(0, len(SERVING_STENCILS)))]
        if st == "box3d27p":
            side = int(round(np.exp(rng.uniform(np.log(64), np.log(384))) / 16.0)) * 16
            shape = (side, side, side)
        else:
            side = int(round(np.exp(rng.uniform(np.log(512), np.log(8192))) / 64.0)) * 64
            shape = (side, side)
        steps = int(rng.integers(1, 101))
        reqs.append(dict(id=i, t=t, stencil=st, shape=shape, steps=steps, seed=int(rng.integers(0, 2**31))))
    return reqs


def serving_coeffs(stencil):
    """Coefficients used for each serving-mix stencil (fixed seeds)."""
    if stencil == "box2d9p":
        return coeffs_uniform01(2, 1, 1)
    if stencil == "star2d13p":
        return stable_coeffs_uniform_pm1(2, 3, 0, "star")[0]
    if stencil == "box2d49p":
        return stable_coeffs_gaussian(2, 3, 0, "box")[0]
    if stencil == "box3d27p":
        return coeffs_uniform01(3, 1, 4)
    raise KeyError(stencil)
