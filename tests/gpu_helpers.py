"""Shared helpers for the GPU tests (inputs to device, results back, error metrics)."""
import numpy as np


def torch_mod():
    import torch
    return torch


def to_dev(x, carry):
    """Round a host array to the carry dtype and place it on cuda:0; also return the
    exact fp64 values of what the device holds (the oracle's input)."""
    torch = torch_mod()
    dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[carry]
    src = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64 if carry == "f64" else np.float32))
    t = src.to(dt)
    host64 = t.to(torch.float64).numpy()
    return t.to("cuda:0").contiguous(), host64


def host_rounded(x, carry):
    """The exact fp64 values of host array `x` rounded to the carry dtype (what to_dev
    places on the device), computed on the host only."""
    torch = torch_mod()
    dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[carry]
    src = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64 if carry == "f64" else np.float32))
    return src.to(dt).to(torch.float64).numpy()


def from_dev(t):
    torch = torch_mod()
    torch.cuda.synchronize()
    return t.to(torch.float64).cpu().numpy()


def empty_like_dev(t):
    torch = torch_mod()
    return torch.empty_like(t)


def rel_errors(y, ref):
    d = y - ref
    return float(np.sqrt((d * d).sum() / (ref * ref).sum())), float(np.abs(d).max() / np.abs(ref).max())
