"""Shared helpers of the GPU parity tests (inputs come from the seeded generators; expected
values from the oracle or closed forms only)."""

import numpy as np
import torch


def rel_l2(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))


def to_gpu(a, dtype=torch.complex64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda:0")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def f32(a):
    """The float32 (or complex64) cast the GPU receives, back in float64 for the oracle."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return a.astype(np.complex64).astype(np.complex128)
    return a.astype(np.float32).astype(np.float64)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
