"""GPU parity of the explicit row swap (the comparison of Sec. 3.2 / Table 3).

With row_swap="explicit" the 16-point sparse band kernel copies every staged
line into an LDS operand tile whose rows are already in the swapped order and
gathers from it at plain offsets, instead of folding the swap into the gather
offsets.  The products and their order are unchanged, so the result must equal
the implicit kernel's bit for bit, and integer cases must equal the oracle.
"""
import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si
from gpu_helpers import empty_like_dev, from_dev, to_dev

pytestmark = pytest.mark.gpu


def run(plan, x_dev, steps):
    y = empty_like_dev(x_dev)
    plan.apply(x_dev, y, steps)
    return from_dev(y)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("shape", [(70, 520), (41, 301), (3, 5)])
def test_integer_exact_f16(oracle_mod, r, shape):
    # |taps| <= 1 and |x| <= 4: partial sums stay below 225 * 4 < 2^11 for r <= 7
    w = si.integer_coeffs(2, r, -1, 1, 50 + r, "box")
    x = si.grid_integer(shape, -4, 4, 60 + r)
    xd, x64 = to_dev(x, "f16")
    plan = sp.Plan(w, shape, carry="f16", engine="sparse", row_swap="explicit")
    assert plan.info()["band_height"] == 16 and plan.info()["time_block"] == 1
    got = run(plan, xd, 1)
    ref = oracle_mod.apply(w, x64, 1)
    assert np.array_equal(got, ref), np.argwhere(got != ref)[:5]


@pytest.mark.parametrize("shape", [(70, 520), (41, 301)])
def test_integer_exact_bf16(oracle_mod, shape):
    for kind, r in [("box", 1), ("star", 3), ("box", 2)]:
        w = si.integer_coeffs(2, r, -2, 2, 70 + r, kind)
        x = si.grid_integer(shape, -2, 2, 80)
        xd, x64 = to_dev(x, "bf16")
        plan = sp.Plan(w, shape, carry="bf16", engine="sparse", row_swap="explicit")
        got = run(plan, xd, 1)
        assert np.array_equal(got, oracle_mod.apply(w, x64, 1)), (kind, r)


@pytest.mark.parametrize("carry", ["f16", "bf16"])
@pytest.mark.parametrize("name,r", [("box2d49p_10240", 3), ("star2d13p_8192", 3), ("box7", 7), ("box5", 5)])
def test_explicit_equals_implicit(name, r, carry):
    shape = (517, 1000)
    if name.startswith("box2") or name.startswith("star"):
        w = si.workload(name, small=True)["coeffs"]
    else:
        w, _ = si.stable_coeffs_gaussian(2, r, 0, "box")
    x = si.grid_sinusoids(shape, 3)
    xd, _ = to_dev(x, carry)
    tiles = [0, 37]
    outs = []
    for swap in ("implicit", "explicit"):
        for t in tiles:
            plan = sp.Plan(w, shape, carry=carry, engine="sparse", band_height=16, time_block=1, tile_h=t,
                           row_swap=swap)
            outs.append(run(plan, xd, 7))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_full_size_box7r_equals_implicit():
    """Box-2D7R (the paper's Table 3 stencil) at 10240^2, a few steps, explicit vs implicit bit for bit."""
    w, _ = si.stable_coeffs_gaussian(2, 7, 0, "box")
    shape = (10240, 10240)
    x = si.grid_sinusoids(shape, 3)
    xd, _ = to_dev(x, "f16")
    got = []
    for swap in ("implicit", "explicit"):
        plan = sp.Plan(w, shape, carry="f16", engine="sparse", time_block=1, row_swap=swap)
        got.append(run(plan, xd, 3))
        plan.close()
    assert np.array_equal(got[0], got[1])


def test_batch_and_server_run_explicit_alone():
    # the batched kernel holds the implicit swap only: batched apply and the server
    # run an explicit-swap plan with its own time loop, equal to spider_apply
    import time
    shape = (64, 64)
    w = si.integer_coeffs(2, 1, -1, 1, 5, "box")
    x = si.grid_integer(shape, -2, 2, 6)
    xd, _ = to_dev(x, "f16")
    plan = sp.Plan(w, shape, carry="f16", engine="sparse", row_swap="explicit")
    ref = empty_like_dev(xd)
    plan.apply(xd, ref, 3)
    ref = from_dev(ref)
    y = empty_like_dev(xd)
    sp.apply_batch([plan], [xd], [y], [3])
    assert np.array_equal(from_dev(y), ref)
    srv = sp.Server(1 << 28)
    try:
        y2 = empty_like_dev(xd)
        t = srv.submit(plan, xd, y2, 3)
        t0 = time.time()
        while not srv.poll(t)[0]:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        assert srv.poll(t)[1] == 0
        assert np.array_equal(from_dev(y2), ref)
    finally:
        srv.close()