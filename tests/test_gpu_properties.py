"""Property tests on the GPU (hypothesis, derandomised so that every run draws the same cases,
kept small): the angular-spectrum step over 7-smooth edges (power-of-two and mixed-radix
sweeps), the direct step over power-of-two edges and both MFT directions over random shapes and
samplings, each against the FP64 oracle at the parity bar (relative L2 <= 1e-5)."""

import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

import oracle
from paper_1806_06467_amd import fresnel as fb
from tests.gpu_common import f32, rel_l2, to_gpu, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-5
SETTINGS = settings(max_examples=12, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


def _smooth7(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


EDGES = [n for n in range(16, 257, 2) if _smooth7(n)]   # the library's own check decides (assume)


def _field(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))


@SETTINGS
@given(n=st.sampled_from(EDGES), z_frac=st.floats(-0.9, 0.9), seed=st.integers(0, 2 ** 16),
       adjoint=st.booleans())
def test_angular_spectrum_step_any_smooth_edge(n, z_frac, seed, adjoint):
    assume(fb.lib().fr_fft_size_supported(n) == 1)
    dx, lam = 1.7e-5, 633e-9
    z = z_frac * n * dx * dx / lam
    u = _field(n, seed)
    t = to_gpu(u)
    fb.fresnel_step(t, dx, lam, z, adjoint=adjoint)
    ref = oracle.fresnel_step(f32(u), dx, lam, z, adjoint=adjoint)
    assert rel_l2(to_np(t), ref) <= TOL


@SETTINGS
@given(n=st.sampled_from([64, 128, 256, 512]), z_mult=st.floats(0.3, 6.0), sign=st.sampled_from([1, -1]),
       seed=st.integers(0, 2 ** 16))
def test_direct_step_power_of_two_edges(n, z_mult, sign, seed):
    dx, lam = 2.2e-5, 550e-9
    z = sign * z_mult * n * dx * dx / lam
    u = _field(n, seed)
    t = to_gpu(u)
    fb.fresnel_direct(t, dx, lam, z)
    ref, _ = oracle.direct_fresnel(f32(u), dx, lam, z)
    assert rel_l2(to_np(t), ref) <= TOL


@SETTINGS
@given(n=st.integers(8, 300), m=st.integers(4, 200), du=st.floats(0.05, 2.0), seed=st.integers(0, 2 ** 16))
def test_mft_both_directions_random_shapes(n, m, du, seed):
    n_d = float(n) * 0.6
    e = _field(n, seed)
    got = to_np(fb.mft_forward(to_gpu(e), n_d, m, du))
    assert rel_l2(got, oracle.mft(f32(e), n_d, m, du)) <= TOL
    eb = _field(m, seed + 1)
    got = to_np(fb.mft_adjoint(to_gpu(eb), n_d, n, du))
    assert rel_l2(got, oracle.mft_adjoint(f32(eb), n_d, n, du)) <= TOL
