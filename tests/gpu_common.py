"""Shared helpers of the GPU parity tests (inputs come from the seeded generators; expected
values from the oracle or closed forms only)."""

import contextlib

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


@contextlib.contextmanager
def forced_gemm_tile(tile, tmp_path):
    """Every MFT GEMM on one tile configuration for the duration: the default choice and every
    shape an earlier autotune call gave its own line. Restores the previous choices after."""
    from paper_1806_06467_amd import fresnel as fb
    saved = tmp_path / "gemm_saved.txt"
    fb.autotune_save(str(saved))
    lines = ["gemm_default %d 0" % tile]
    for ln in saved.read_text().splitlines():
        t = ln.split()
        if t and t[0] == "gemm":
            lines.append(" ".join(t[:6] + [str(tile), "0"]))
    forced = tmp_path / "gemm_forced.txt"
    forced.write_text("\n".join(lines) + "\n")
    fb.autotune_load(str(forced))
    try:
        yield
    finally:
        forced.write_text("gemm_default -1 0\n")
        fb.autotune_load(str(forced))
        fb.autotune_load(str(saved))


def grid_plane_wave_sum(n, waves, dtype=np.complex128):
    """sum_j a_j exp(2 pi i (kx_j x + ky_j y) / n) on the n x n grid, for integer frequencies
    (kx_j, ky_j, a_j): each term is an exact eigenvector of every shift-invariant step on the
    grid. The index products are reduced modulo n in integers before the float64 exponential."""
    x = np.arange(n, dtype=np.int64)
    out = np.zeros((n, n), dtype=dtype)
    for kx, ky, a in waves:
        ex = np.exp(2j * np.pi * ((kx * x) % n) / n)
        ey = np.exp(2j * np.pi * ((ky * x) % n) / n)
        out += (complex(a) * ey)[:, None].astype(dtype) * ex[None, :].astype(dtype)
    return out
