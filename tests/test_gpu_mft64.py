"""GPU parity of mft_f64 (the MFT in float64, forward and adjoint) against the FP64 oracle (O4).
Bar: relative L2 <= 1e-12 (float64 sums in another order; the oracle's and the library's
matrices agree to the last bits of their cosines); the adjoint identity <A x, y> = <x, A^H y> to
1e-12 of |A x| |y|."""

import numpy as np
import pytest
import torch

import oracle
from paper_1806_06467_amd import fresnel as fb
from paper_1806_06467_amd import synth
from tests.gpu_common import banner, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-12

# (pupil edge, focal edge, pupil diameter in pixels, focal pitch in lambda/D): tile multiples,
# ragged edges below and above one 64-wide tile, and the occulter and detector shapes of the
# 4096^2 train, and a ragged product of 33 x 33 tiles of 64 (the large-tile kernel)
CASES = [(64, 16, 32.0, 0.5), (300, 77, 150.0, 0.37), (33, 130, 20.0, 0.11), (1024, 256, 512.0, 0.125),
         (4096, 256, 1024.0, 0.03125), (1024, 512, 1024.0, 0.25), (2100, 40, 700.0, 0.3)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,m,n_d,du", CASES)
def test_mft_f64_forward(n, m, n_d, du):
    banner(f"mft_f64 forward {n}->{m} n_d={n_d} du={du}")
    e = synth.random_field(n, 3 * n + m)
    got = _host(fb.mft_f64(_dev(e), n_d, m, du))
    assert rel_l2(got, oracle.mft(e, n_d, m, du)) <= TOL


@pytest.mark.parametrize("n,m,n_d,du", CASES)
def test_mft_f64_adjoint(n, m, n_d, du):
    banner(f"mft_f64 adjoint {m}->{n} n_d={n_d} du={du}")
    eb = synth.random_field(m, 5 * n + m)
    got = _host(fb.mft_f64(_dev(eb), n_d, n, du, adjoint=True))
    assert rel_l2(got, oracle.mft_adjoint(eb, n_d, n, du)) <= TOL


@pytest.mark.parametrize("n,m,n_d,du", [(300, 77, 150.0, 0.37), (1024, 256, 512.0, 0.125)])
def test_mft_f64_inner_product(n, m, n_d, du):
    x = synth.random_field(n, 11)
    y = synth.random_field(m, 12)
    ax = _host(fb.mft_f64(_dev(x), n_d, m, du))
    ahy = _host(fb.mft_f64(_dev(y), n_d, n, du, adjoint=True))
    assert abs(np.vdot(y, ax) - np.vdot(ahy, x)) <= TOL * np.linalg.norm(ax) * np.linalg.norm(y)


def test_mft_f64_matches_float32_mft_within_its_bar():
    """The float64 and float32 library paths on one field agree to the float32 path's bar."""
    n, m, n_d, du = 1024, 256, 512.0, 0.125
    e = synth.random_field(n, 21)
    got64 = _host(fb.mft_f64(_dev(e), n_d, m, du))
    got32 = fb.mft_forward(torch.from_numpy(e.astype(np.complex64)).to("cuda:0"), n_d, m, du)
    torch.cuda.synchronize()
    assert rel_l2(got32.cpu().numpy().astype(np.complex128), got64) <= 1e-5
