"""spider_apply_noalloc (through the C ABI) against spider_apply.

The no-allocation entry point runs the same kernels in the same launch sequence
as spider_apply, with the ping-pong buffer taken from the library's fixed device
array, so its results must equal spider_apply's bit for bit.  Two calls in a row
(the second on a smaller grid) must both be right, and after the first call no
call may change the device's free memory.
"""
import ctypes

import numpy as np
import pytest

import paper_2506_22035_amd as sp
import stencil_inputs as si

pytestmark = pytest.mark.gpu

LIMIT = 128 << 20   # SPIDER_NOALLOC_SCRATCH_BYTES


def _noalloc(plan, x, y, steps):
    import torch
    st = sp.lib().spider_apply_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       int(steps), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _case(name, carry, small):
    import torch
    wl = si.workload(name, small=small)
    x = torch.from_numpy(wl["make_grid"](np.float32)).to(sp.torch_dtype(carry)).to("cuda:0")
    return wl, x


@pytest.mark.parametrize("carry,engine", [("f16", "sparse"), ("bf16", "dense"), ("f32", "sparse"), ("f32", "direct")])
def test_noalloc_equals_apply_two_calls(carry, engine):
    import torch
    # first call: a 2-D grid whose loop fuses several steps per launch; second: a smaller grid
    cases = [("star2d13p_8192", (2048, 2048), 37), ("box2d49p_10240", (300, 520), 10)]
    for name, shape, steps in cases:
        wl = si.workload(name)
        x = torch.from_numpy(si.grid_uniform01(shape, 3)).to(sp.torch_dtype(carry)).to("cuda:0")
        split = 3 if (carry == "f32" and engine != "direct") else 2
        plan = sp.Plan(wl["coeffs"], shape, carry=carry, engine=engine, split=split)
        ref = torch.empty_like(x)
        plan.apply(x, ref, steps)
        got = torch.full_like(x, float("nan"))
        assert _noalloc(plan, x, got, steps) == 0, sp.lib().spider_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (name, carry, engine)
        # in place and zero steps
        y = x.clone()
        assert _noalloc(plan, y, y, steps) == 0
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        z = torch.empty_like(x)
        assert _noalloc(plan, x, z, 0) == 0
        torch.cuda.synchronize()
        assert torch.equal(z, x)
        plan.close()


def test_noalloc_3d_1d_and_no_device_allocation():
    import torch
    plans = []
    for name in ("box3d27p_512", "1d5p_10240000"):
        wl, x = _case(name, "f16", small=True)
        plans.append((wl, x, sp.Plan(wl["coeffs"], wl["shape"], carry="f16")))
    wl, x, p = plans[0]
    y = torch.empty_like(x)
    assert _noalloc(p, x, y, 3) == 0          # first call on the device: address lookup
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for wl, x, p in plans:                    # fresh plans, never applied before
        y = torch.empty_like(x)
        ref = torch.empty_like(x)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert _noalloc(p, x, y, wl["steps"]) == 0
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free1, wl["name"]
        p.apply(x, ref, wl["steps"])
        torch.cuda.synchronize()
        assert torch.equal(y, ref), wl["name"]
    assert free0 > 0


def test_noalloc_rejects_grids_beyond_its_array():
    import torch
    w = np.ones((3, 3)) / 9
    shape = (8192, 8193)                       # 134 234 112 bytes of fp16 > 128 MiB
    plan = sp.Plan(w, shape, carry="f16")
    x = torch.zeros(16, dtype=torch.float16, device="cuda:0")
    assert 2 * shape[0] * shape[1] > LIMIT
    assert _noalloc(plan, x, x, 1) == 1
    assert b"exceeds" in sp.lib().spider_last_error()
    ok = sp.Plan(w, (8192, 8192), carry="f16")  # exactly the limit: accepted
    xs = torch.rand((8192, 8192), device="cuda:0").to(torch.float16)
    ys = torch.empty_like(xs)
    ref = torch.empty_like(xs)
    assert _noalloc(ok, xs, ys, 5) == 0
    ok.apply(xs, ref, 5)
    torch.cuda.synchronize()
    assert torch.equal(ys, ref)
