"""The C-ABI library loads and exports every function include/fresnel.h declares, and its
host-side argument checks answer without launching anything (no GPU needed)."""

import ctypes
import os
import subprocess

import pytest

from paper_1806_06467_amd import fresnel as fb

EXPECTED = {
    "fr_create", "fr_destroy", "fr_set_cache_limit", "fr_status_string", "fr_fft_size_supported", "fresnel_step",
    "fresnel_step_batched", "fresnel_step_batched_graph", "fresnel_step_exact", "fresnel_step_exact_batched", "fresnel_step_f64", "mft_f64", "mft_f64_workspace_bytes", "fresnel_direct", "fr_plan_route", "fr_plan_system", "propagate_system", "mft_workspace_bytes", "mft_forward", "mft_adjoint",
    "propagate_train_workspace_bytes", "propagate_train_ckpt_bytes", "propagate_train", "mft_forward_noalloc", "fr_profile_enable", "fr_profile_read",
    "fr_autotune", "fr_autotune_save", "fr_autotune_load",
}


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fb.LIB_PATH):
        pytest.fail("libfresnel.so is not built (run __graft_entry__.build())")
    return fb.lib()


def test_header_declares_the_boundary():
    assert set(fb.declared_symbols()) == EXPECTED


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", fb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = set(fb.declared_symbols()) - exported
    assert not missing, missing
    for name in fb.declared_symbols():
        assert getattr(L, name) is not None


def test_status_strings(L):
    assert fb.status_string(0) == "ok"
    for st in (-1, -2, -3, -5):
        assert len(fb.status_string(st)) > 5
    assert fb.status_string(-99) == "unknown status"
    assert "warning" in fb.status_string(1)


def test_supported_sizes(L):
    # powers of two up to 8192; other edges up to 4096 that factor into radices 2..16
    # (6 passes at most); the per-wavelength grids of the broadband workload among them
    for n in (64, 128, 256, 512, 1024, 2048, 4096, 8192, 2, 3, 30, 100, 3000,
              3584, 3600, 3840, 3888, 3920, 4000, 4032):
        assert L.fr_fft_size_supported(n) == 1, n
    # 4095 = 3^2 5 7 13 and 17 have a prime factor above 16; 4097 and 6000 exceed 4096
    for n in (0, 1, -4, 17, 4095, 4097, 6000, 16384):
        assert L.fr_fft_size_supported(n) == 0, n


def test_workspace_query(L):
    # the n x m c64 intermediate plus 16 float64 complex split-K slices
    assert L.mft_workspace_bytes(4096, 256) == 4096 * 256 * 8 + 16 * 4096 * 256 * 16
    assert L.mft_workspace_bytes(0, 256) == 0


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def test_fresnel_step_argument_errors(L):
    null = ctypes.c_void_p()
    st = L.fresnel_step(null, null, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null)
    assert st == fb.FR_EINVAL
    st = L.fresnel_step(null, FAKE, 4095, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null)
    assert st == fb.FR_EUNSUPPORTED
    st = L.fresnel_step(null, FAKE, 256, -1e-4, 5e-7, 1.0, null, null, 0.0, 0, null)
    assert st == fb.FR_EINVAL
    st = L.fresnel_step(null, FAKE, 256, 1e-4, 0.0, 1.0, null, null, 0.0, 0, null)
    assert st == fb.FR_EINVAL
    st = L.fresnel_step(null, FAKE, 256, 1e-4, 5e-7, float("nan"), null, null, 0.0, 0, null)
    assert st == fb.FR_EINVAL
    st = L.fresnel_step(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 4, null)
    assert st == fb.FR_EINVAL
    # valid arguments but no context
    st = L.fresnel_step(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null)
    assert st == fb.FR_EINVAL


def test_fresnel_direct_argument_errors(L):
    null = ctypes.c_void_p()
    out = ctypes.c_double(-7.0)
    ref = ctypes.byref(out)
    assert L.fresnel_direct(null, null, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, ref, null) == fb.FR_EINVAL
    assert L.fresnel_direct(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, None, null) == fb.FR_EINVAL
    assert L.fresnel_direct(null, FAKE, 256, 1e-4, 5e-7, 0.0, null, null, 0.0, 0, ref, null) == fb.FR_EINVAL
    assert L.fresnel_direct(null, FAKE, 256, 1e-4, 5e-7, float("nan"), null, null, 0.0, 0, ref, null) == fb.FR_EINVAL
    assert L.fresnel_direct(null, FAKE, 256, 0.0, 5e-7, 1.0, null, null, 0.0, 0, ref, null) == fb.FR_EINVAL
    assert L.fresnel_direct(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, float("inf"), 0, ref, null) == fb.FR_EINVAL
    assert L.fresnel_direct(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 2, ref, null) == fb.FR_EINVAL
    # power-of-two edges only (the mixed-radix sweeps have no direct variant)
    assert L.fresnel_direct(null, FAKE, 3584, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, ref, null) == fb.FR_EUNSUPPORTED
    assert L.fresnel_direct(null, FAKE, 32, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, ref, null) == fb.FR_EUNSUPPORTED
    # valid arguments but no context; the output pitch is written only on success
    assert L.fresnel_direct(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, ref, null) == fb.FR_EINVAL
    assert out.value == -7.0


def test_fresnel_step_exact_argument_errors(L):
    null = ctypes.c_void_p()
    assert L.fresnel_step_exact(null, null, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EINVAL
    assert L.fresnel_step_exact(null, FAKE, 0, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EINVAL
    assert L.fresnel_step_exact(null, FAKE, 256, 0.0, 5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EINVAL
    assert L.fresnel_step_exact(null, FAKE, 256, 1e-4, -5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EINVAL
    assert L.fresnel_step_exact(null, FAKE, 256, 1e-4, 5e-7, float("nan"), null, null, 0.0, 0, null) == fb.FR_EINVAL
    assert L.fresnel_step_exact(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, float("inf"), 0, null) == fb.FR_EINVAL
    assert L.fresnel_step_exact(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 2, null) == fb.FR_EINVAL
    # power-of-two edges from 64 only
    assert L.fresnel_step_exact(null, FAKE, 3584, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EUNSUPPORTED
    assert L.fresnel_step_exact(null, FAKE, 32, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EUNSUPPORTED
    # valid arguments but no context
    assert L.fresnel_step_exact(null, FAKE, 256, 1e-4, 5e-7, 1.0, null, null, 0.0, 0, null) == fb.FR_EINVAL


def test_mft_f64_argument_errors(L):
    null = ctypes.c_void_p()
    assert L.mft_f64(null, null, FAKE, 64, 16, 32.0, 0.5, 0, FAKE, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, null, 64, 16, 32.0, 0.5, 0, FAKE, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, FAKE, 64, 16, 32.0, 0.5, 0, null, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, FAKE, 0, 16, 32.0, 0.5, 0, FAKE, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, FAKE, 64, -1, 32.0, 0.5, 0, FAKE, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, FAKE, 64, 16, 0.0, 0.5, 0, FAKE, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, FAKE, 64, 16, 32.0, float("inf"), 0, FAKE, 1 << 30, null) == fb.FR_EINVAL
    assert L.mft_f64(null, FAKE, FAKE, 64, 16, 32.0, 0.5, 2, FAKE, 1 << 30, null) == fb.FR_EINVAL
    # workspace below mft_f64_workspace_bytes: 16 n m, four times that where the first product
    # is split over k, plus 16 partial m x m products where the second is
    assert L.mft_f64_workspace_bytes(64, 16) == 16 * 64 * 16
    assert L.mft_f64_workspace_bytes(4096, 256) == 4 * 16 * 4096 * 256 + 32 * 16 * 256 * 256
    assert L.mft_f64_workspace_bytes(0, 16) == 0
    assert L.mft_f64(null, FAKE, FAKE, 64, 16, 32.0, 0.5, 0, FAKE, 16 * 64 * 16 - 1, null) == fb.FR_EWORKSPACE
    # valid arguments but no context
    assert L.mft_f64(null, FAKE, FAKE, 64, 16, 32.0, 0.5, 0, FAKE, 1 << 30, null) == fb.FR_EINVAL


def test_batched_argument_errors(L):
    null = ctypes.c_void_p()
    arr = (fb.FrPlane * 2)()
    arr[0] = fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, 1.0, 0.0, 256, 0)
    arr[1] = fb.FrPlane(0x2000, None, None, 1e-4, 5e-7, 1.0, 0.0, 512, 0)
    for fn in (L.fresnel_step_batched, L.fresnel_step_batched_graph):
        assert fn(null, arr, 2, null) == fb.FR_EINVAL   # valid planes, no context
        assert fn(null, arr, 0, null) == fb.FR_EINVAL
        bad = (fb.FrPlane * 1)()
        bad[0] = fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, 1.0, 0.0, 4097, 0)
        assert fn(null, bad, 1, null) == fb.FR_EUNSUPPORTED


def test_create_argument_errors(L):
    assert L.fr_create(None, 0, None) == fb.FR_EINVAL     # no handle to fill


def test_exact_batched_argument_errors(L):
    null = ctypes.c_void_p()
    fn = L.fresnel_step_exact_batched
    good = (fb.FrPlane * 2)()
    good[0] = fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, 1.0, 0.0, 256, 0)
    good[1] = fb.FrPlane(0x2000, None, None, 2e-4, 6e-7, -1.0, 0.0, 256, fb.FR_ADJOINT)
    assert fn(null, good, 2, null) == fb.FR_EINVAL     # valid planes, no context
    assert fn(null, good, 0, null) == fb.FR_EINVAL
    assert fn(null, None, 1, null) == fb.FR_EINVAL
    mixed = (fb.FrPlane * 2)()
    mixed[0] = fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, 1.0, 0.0, 256, 0)
    mixed[1] = fb.FrPlane(0x2000, None, None, 1e-4, 5e-7, 1.0, 0.0, 512, 0)
    assert fn(null, mixed, 2, null) == fb.FR_EINVAL    # one edge per call
    odd = (fb.FrPlane * 1)()
    odd[0] = fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, 1.0, 0.0, 3584, 0)
    assert fn(null, odd, 1, null) == fb.FR_EUNSUPPORTED   # power-of-two edges only
    for plane, want in ((fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, 1.0, 0.0, 256, 2), fb.FR_EINVAL),
                        (fb.FrPlane(None, None, None, 1e-4, 5e-7, 1.0, 0.0, 256, 0), fb.FR_EINVAL),
                        (fb.FrPlane(0x1000, None, None, 1e-4, 5e-7, float("nan"), 0.0, 256, 0), fb.FR_EINVAL),
                        (fb.FrPlane(0x1000, None, None, 1e-4, 0.0, 1.0, 0.0, 256, 0), fb.FR_EINVAL)):
        one = (fb.FrPlane * 2)()
        one[0] = good[0]
        one[1] = plane
        assert fn(null, one, 2, null) == want


def test_mft_argument_errors(L):
    null = ctypes.c_void_p()
    st = L.mft_forward(null, FAKE, 256, 256, FAKE, 128, 128, 256.0, 0.25, null, null, 0, null)
    assert st == fb.FR_EWORKSPACE
    st = L.mft_forward(null, FAKE, 256, 200, FAKE, 128, 128, 256.0, 0.25, null, FAKE, 1 << 30, null)
    assert st == fb.FR_EINVAL          # row stride shorter than a row
    st = L.mft_forward(null, FAKE, 256, 256, FAKE, 128, 128, 256.0, -0.25, null, FAKE, 1 << 30, null)
    assert st == fb.FR_EINVAL
    st = L.mft_adjoint(null, FAKE, 128, 128, FAKE, 256, 256, 256.0, 0.25, 1.0, float("inf"), null,
                       FAKE, 1 << 30, null)
    assert st == fb.FR_EINVAL
    st = L.mft_adjoint(null, FAKE, 128, 128, FAKE, 256, 256, 256.0, 0.25, 1.0, 0.0, null, FAKE, 16, null)
    assert st == fb.FR_EWORKSPACE


def test_profile_argument_errors(L):
    null = ctypes.c_void_p()
    assert L.fr_profile_enable(null, 1) == fb.FR_EINVAL
    n = ctypes.c_int32()
    assert L.fr_profile_read(null, 0, None, 0, None, None, ctypes.byref(n)) == fb.FR_EINVAL


def test_cache_limit_argument_errors(L):
    null = ctypes.c_void_p()
    assert L.fr_set_cache_limit(null, 16) == fb.FR_EINVAL
    assert L.fr_set_cache_limit(FAKE, 0) == fb.FR_EINVAL
    assert L.fr_set_cache_limit(FAKE, -3) == fb.FR_EINVAL


def test_train_checkpoint_size_and_mode_errors(L):
    import torch
    null = ctypes.c_void_p()
    d = fb.FrTrainDesc()
    d.n_d, d.d_m = 64, 64 * 25e-6
    d.pupil_amp = 0x1000
    d.n_dm, d.n_act, d.dm_heights_m = 1, 8, 0x2000
    d.z_m = 0.05
    d.occ_m, d.occ_du_c, d.occ_mask, d.lyot = 64, 0.125, 0x3000, 0x4000
    d.det_m, d.det_du_c, d.lambda_c_m = 64, 0.5, 550e-9
    nl = 2
    npd = (ctypes.c_int32 * nl)(128, 120)
    lam = (ctypes.c_double * nl)(500e-9, 600e-9)
    w = (ctypes.c_float * nl)(0.5, 0.5)
    # per wavelength the last-DM plane (n^2 c64) and the detector field (det^2 c64), 256-aligned
    want = sum(((n * n * 8 + 255) // 256) * 256 for n in (128, 120)) + 2 * 64 * 64 * 8
    assert L.propagate_train_ckpt_bytes(ctypes.byref(d), nl, npd) == want
    assert L.propagate_train_ckpt_bytes(None, nl, npd) == 0
    big = 1 << 40

    def call(mode, ckpt, ckpt_bytes, psf=0x5000, gpsf=0x6000, gh=0x7000):
        return L.propagate_train(null, ctypes.byref(d), nl, lam, npd, w, mode, psf, gpsf, gh, ckpt, ckpt_bytes,
                                 0x8000, big, null)
    # two phases in one call
    assert call(fb.FR_TRAIN_GRAD | fb.FR_TRAIN_BWD, 0x9000, big) == fb.FR_EINVAL
    assert call(fb.FR_TRAIN_FWD_SAVE | fb.FR_TRAIN_BWD, 0x9000, big) == fb.FR_EINVAL
    # a checkpoint missing or too small
    assert call(fb.FR_TRAIN_FWD_SAVE, None, 0) == fb.FR_EWORKSPACE
    assert call(fb.FR_TRAIN_BWD, 0x9000, want - 1) == fb.FR_EWORKSPACE
    # the backward needs grad_psf and grad_heights, not psf
    assert call(fb.FR_TRAIN_BWD, 0x9000, want, gpsf=None) == fb.FR_EINVAL
    assert call(fb.FR_TRAIN_BWD, 0x9000, want, psf=None) == fb.FR_EINVAL   # valid, but no context
    # without a DM there is nothing to save for
    d.n_dm = 0
    assert call(fb.FR_TRAIN_FWD_SAVE, 0x9000, want) == fb.FR_EINVAL


def test_fresnel_step_f64_argument_errors(L):
    null = ctypes.c_void_p()
    f = L.fresnel_step_f64
    assert f(null, None, 256, 1e-5, 5e-7, 1.0, None, None, 0.0, 0, null) == fb.FR_EINVAL
    assert f(null, FAKE, 0, 1e-5, 5e-7, 1.0, None, None, 0.0, 0, null) == fb.FR_EINVAL
    assert f(null, FAKE, 256, -1e-5, 5e-7, 1.0, None, None, 0.0, 0, null) == fb.FR_EINVAL
    assert f(null, FAKE, 256, 1e-5, 5e-7, float("nan"), None, None, 0.0, 0, null) == fb.FR_EINVAL
    assert f(null, FAKE, 256, 1e-5, 5e-7, 1.0, None, None, 0.0, 4, null) == fb.FR_EINVAL
    for n in (3, 96, 3840, 16384):
        assert f(null, FAKE, n, 1e-5, 5e-7, 1.0, None, None, 0.0, 0, null) == fb.FR_EUNSUPPORTED
    assert f(null, FAKE, 4096, 1e-5, 5e-7, 1.0, None, None, 0.0, 0, null) == fb.FR_EINVAL   # no context


def test_system_argument_errors(L):
    null = ctypes.c_void_p()
    ops = (fb.FrOptic * 2)()
    ops[0] = fb.FrOptic(0.0, 2.0, None, None)
    ops[1] = fb.FrOptic(1.0, 0.0, None, None)
    out = ctypes.c_double()
    tr = ctypes.c_int32()
    pitches = (ctypes.c_double * 2)()
    assert L.fr_plan_system(256, 1e-4, 5e-7, 2e-3, ops, 2, pitches, ctypes.byref(tr)) == 0
    assert tr.value > 0 and pitches[0] == 1e-4
    assert L.fr_plan_system(256, 1e-4, 5e-7, 2e-3, None, 2, pitches, None) == fb.FR_EINVAL
    assert L.fr_plan_system(256, 1e-4, 5e-7, 2e-3, ops, 0, pitches, None) == fb.FR_EINVAL
    assert L.fr_plan_system(256, -1e-4, 5e-7, 2e-3, ops, 2, pitches, None) == fb.FR_EINVAL
    assert L.fr_plan_system(256, 1e-4, 5e-7, 0.0, ops, 2, pitches, None) == fb.FR_EINVAL
    assert L.fr_plan_system(96, 1e-4, 5e-7, 2e-3, ops, 2, pitches, None) == fb.FR_EUNSUPPORTED
    ops[1] = fb.FrOptic(-1.0, 0.0, None, None)   # a negative distance
    assert L.fr_plan_system(256, 1e-4, 5e-7, 2e-3, ops, 2, pitches, None) == fb.FR_EINVAL
    ops[1] = fb.FrOptic(1.0, 0.0, None, None)
    assert L.propagate_system(null, FAKE, 256, 1e-4, 5e-7, 2e-3, ops, 2, None, null) == fb.FR_EINVAL
    assert L.propagate_system(null, None, 256, 1e-4, 5e-7, 2e-3, ops, 2, ctypes.byref(out), null) == fb.FR_EINVAL
    assert L.propagate_system(null, FAKE, 256, 1e-4, 5e-7, 2e-3, ops, 2, ctypes.byref(out), null) == fb.FR_EINVAL
