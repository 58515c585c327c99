"""ctypes binding of libfresnel.so (C ABI: include/fresnel.h).

Argument marshalling only: torch tensors supply device memory and the current HIP stream,
every step of the computation runs in the library's kernels. There is no CPU fallback: if
the library is not built, or a tensor is not on the GPU, the call raises.
"""

import ctypes
import os
import re
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfresnel.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "fresnel.h")

FR_OK = 0
FR_EINVAL = -1
FR_EUNSUPPORTED = -2
FR_EWORKSPACE = -3
FR_EHIP = -4
FR_ENOMEM = -5
FR_ESTATE = -6
FR_W_AS_UNDERSAMPLED = 1
FR_W_MFT_ALIASED = 2
FR_W_DIRECT_UNDERSAMPLED = 4
FR_ADJOINT = 1
FR_INVERSE = 2
FR_ROUTE_AS, FR_ROUTE_DIRECT, FR_ROUTE_DIRECT_INVERSE = 1, 2, 3
FR_TRAIN_NO_OCCULTER = 1
FR_TRAIN_GRAD = 2
FR_TRAIN_BATCHED = 4
FR_TRAIN_GRAPH = 8
FR_TRAIN_FWD_SAVE = 16
FR_TRAIN_BWD = 32

_c = ctypes
_vp = _c.c_void_p


class FrError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


class FrRouteStep(_c.Structure):
    _fields_ = [("kind", _c.c_int32), ("z_m", _c.c_double), ("dx_in_m", _c.c_double), ("dx_out_m", _c.c_double)]


class FrOptic(_c.Structure):
    _fields_ = [("z_m", _c.c_double), ("lens_focal_m", _c.c_double), ("amp", _vp), ("opd_m", _vp)]


class FrPlane(_c.Structure):
    _fields_ = [("field", _vp), ("amp", _vp), ("opd_m", _vp), ("dx_m", _c.c_double),
                ("wavelength_m", _c.c_double), ("z_m", _c.c_double), ("lens_focal_m", _c.c_double),
                ("n", _c.c_int32), ("flags", _c.c_int32)]


class FrTrainDesc(_c.Structure):
    _fields_ = [("n_d", _c.c_int32), ("d_m", _c.c_double), ("pupil_amp", _vp),
                ("pupil_opd_m", _vp), ("n_dm", _c.c_int32), ("n_act", _c.c_int32),
                ("dm_heights_m", _vp), ("z_m", _c.c_double), ("occ_m", _c.c_int32),
                ("occ_du_c", _c.c_double), ("occ_mask", _vp), ("lyot", _vp),
                ("det_m", _c.c_int32), ("det_du_c", _c.c_double), ("lambda_c_m", _c.c_double)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libfresnel.so once (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = _c.CDLL(LIB_PATH)
        i32, f64, f32, sz = _c.c_int32, _c.c_double, _c.c_float, _c.c_size_t
        sig = {
            "fr_create": (_c.c_int, [_c.POINTER(_vp), _c.c_int, _c.c_char_p]),
            "fr_destroy": (_c.c_int, [_vp]),
            "fr_set_cache_limit": (_c.c_int, [_vp, i32]),
            "fr_status_string": (_c.c_char_p, [_c.c_int]),
            "fr_fft_size_supported": (_c.c_int, [i32]),
            "fresnel_step": (_c.c_int, [_vp, _vp, i32, f64, f64, f64, _vp, _vp, f64, i32, _vp]),
            "fresnel_step_batched": (_c.c_int, [_vp, _c.POINTER(FrPlane), i32, _vp]),
            "fresnel_step_batched_graph": (_c.c_int, [_vp, _c.POINTER(FrPlane), i32, _vp]),
            "fresnel_step_exact": (_c.c_int, [_vp, _vp, i32, f64, f64, f64, _vp, _vp, f64, i32, _vp]),
            "fresnel_step_exact_batched": (_c.c_int, [_vp, _c.POINTER(FrPlane), i32, _vp]),
            "fresnel_direct": (_c.c_int, [_vp, _vp, i32, f64, f64, f64, _vp, _vp, f64, i32, _c.POINTER(f64), _vp]),
            "fr_plan_route": (_c.c_int, [f64, f64, f64, i32, f64, f64, f64, _c.POINTER(FrRouteStep), i32]),
            "fr_plan_system": (_c.c_int, [i32, f64, f64, f64, _c.POINTER(FrOptic), i32, _c.POINTER(f64),
                                          _c.POINTER(i32)]),
            "propagate_system": (_c.c_int, [_vp, _vp, i32, f64, f64, f64, _c.POINTER(FrOptic), i32,
                                            _c.POINTER(f64), _vp]),
            "mft_workspace_bytes": (sz, [i32, i32]),
            "mft_f64_workspace_bytes": (sz, [i32, i32]),
            "mft_f64": (_c.c_int, [_vp, _vp, _vp, i32, i32, f64, f64, i32, _vp, sz, _vp]),
            "mft_forward": (_c.c_int, [_vp, _vp, i32, i32, _vp, i32, i32, f64, f64, _vp, _vp, sz, _vp]),
            "mft_forward_noalloc": (_c.c_int, [_vp, _vp, i32, i32, _vp, i32, i32, f64, f64, _vp, _vp]),
            "fresnel_step_f64": (_c.c_int, [_vp, _vp, i32, f64, f64, f64, _vp, _vp, f64, i32, _vp]),
            "mft_adjoint": (_c.c_int, [_vp, _vp, i32, i32, _vp, i32, i32, f64, f64, f32, f32, _vp,
                                       _vp, sz, _vp]),
            "fr_profile_enable": (_c.c_int, [_vp, _c.c_int]),
            "fr_profile_read": (_c.c_int, [_vp, i32, _c.c_char_p, i32, _c.POINTER(f64),
                                           _c.POINTER(_c.c_int64), _c.POINTER(i32)]),
            "fr_autotune": (_c.c_int, [_vp, i32, i32, i32, _vp]),
            "fr_autotune_save": (_c.c_int, [_vp, _c.c_char_p]),
            "fr_autotune_load": (_c.c_int, [_vp, _c.c_char_p]),
            "propagate_train_workspace_bytes": (sz, [_c.POINTER(FrTrainDesc), i32, _c.POINTER(i32), i32]),
            "propagate_train_ckpt_bytes": (sz, [_c.POINTER(FrTrainDesc), i32, _c.POINTER(i32)]),
            "propagate_train": (_c.c_int, [_vp, _c.POINTER(FrTrainDesc), i32, _c.POINTER(f64),
                                           _c.POINTER(i32), _c.POINTER(f32), i32, _vp, _vp, _vp, _vp,
                                           sz, _vp, sz, _vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def declared_symbols():
    """Function names declared in include/fresnel.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\([^;{]*\)\s*;", text)) - {"if", "return"})


def status_string(status):
    return lib().fr_status_string(int(status)).decode()


def _check(status, where):
    if status < 0:
        raise FrError(status, where)
    return status


# ---- contexts and streams -------------------------------------------------------------------

class Context:
    """An fr_ctx bound to one HIP device (owns the cached float64-built tables)."""

    def __init__(self, device=0, tune_file=None):
        self.device = int(device)
        h = _vp()
        path = None if tune_file is None else os.fsencode(tune_file)
        _check(lib().fr_create(_c.byref(h), self.device, path), "fr_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().fr_destroy(self.handle)
            self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def context(device=None):
    dev = torch.cuda.current_device() if device is None else int(device)
    ctx = _contexts.get(dev)
    if ctx is None:
        ctx = _contexts[dev] = Context(dev)
    return ctx


def _stream(device, stream):
    """The torch stream a call runs on: the given one, else the device's current stream."""
    return torch.cuda.current_stream(device) if stream is None else stream


def _stream_handle(device, stream):
    return _vp(_stream(device, stream).cuda_stream)


_workspaces = {}


def workspace(nbytes, device, stream=None):
    """A cached device byte buffer of at least nbytes, one per (device, stream) and allocated on
    that stream, so that the caching allocator never hands it (or a buffer it outgrew) to other
    work while the library's kernels on that stream may still use it."""
    s = _stream(device, stream)
    key = (int(device), s.cuda_stream)
    buf = _workspaces.get(key)
    if buf is None or buf.numel() < nbytes:
        with torch.cuda.stream(s):
            buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=f"cuda:{device}")
        _workspaces[key] = buf
    return buf


def _empty(shape, dtype, device, stream):
    """An output allocated on the stream the library writes it from."""
    with torch.cuda.stream(_stream(device.index, stream)):
        return torch.empty(shape, dtype=dtype, device=device)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp()


def _need(t, dtype, shape, name, contiguous=True):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if contiguous and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _row_stride(t, name):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D view with unit column stride")
    return t.stride(0)


# ---- Fresnel plane ----------------------------------------------------------------------------

def fresnel_step(field, dx, wavelength, z, amp=None, opd=None, lens_focal=0.0, adjoint=False,
                 stream=None):
    """In place: field <- AS_z(field * optic) (or its adjoint). Returns the warning bits."""
    _need(field, torch.complex64, None, "field")
    n = field.shape[0]
    _need(field, torch.complex64, (n, n), "field")
    for t, nm in ((amp, "amp"), (opd, "opd")):
        if t is not None:
            _need(t, torch.float32, (n, n), nm)
    dev = field.device.index
    st = lib().fresnel_step(context(dev).handle, _ptr(field), n, float(dx), float(wavelength),
                            float(z), _ptr(amp), _ptr(opd), float(lens_focal),
                            FR_ADJOINT if adjoint else 0, _stream_handle(dev, stream))
    return _check(st, "fresnel_step")


def fresnel_step_exact(field, dx, wavelength, z, amp=None, opd=None, lens_focal=0.0, adjoint=False,
                       stream=None):
    """In place: field <- the angular-spectrum step with the exact transfer function (as
    fresnel_step otherwise). Returns the warning bits."""
    _need(field, torch.complex64, None, "field")
    n = field.shape[0]
    _need(field, torch.complex64, (n, n), "field")
    for t, nm in ((amp, "amp"), (opd, "opd")):
        if t is not None:
            _need(t, torch.float32, (n, n), nm)
    dev = field.device.index
    st = lib().fresnel_step_exact(context(dev).handle, _ptr(field), n, float(dx), float(wavelength), float(z),
                                  _ptr(amp), _ptr(opd), float(lens_focal), FR_ADJOINT if adjoint else 0,
                                  _stream_handle(dev, stream))
    return _check(st, "fresnel_step_exact")


def fresnel_direct(field, dx, wavelength, z, amp=None, opd=None, lens_focal=0.0, adjoint=False,
                   inverse=False, stream=None):
    """In place: field <- the direct (single-transform) Fresnel step of field * optic over z != 0
    (or its exact adjoint, from the output grid back). Returns (output pitch lambda z / (n dx),
    warning bits)."""
    _need(field, torch.complex64, None, "field")
    n = field.shape[0]
    _need(field, torch.complex64, (n, n), "field")
    for t, nm in ((amp, "amp"), (opd, "opd")):
        if t is not None:
            _need(t, torch.float32, (n, n), nm)
    dev = field.device.index
    out = _c.c_double(0.0)
    st = lib().fresnel_direct(context(dev).handle, _ptr(field), n, float(dx), float(wavelength), float(z),
                              _ptr(amp), _ptr(opd), float(lens_focal),
                              (FR_ADJOINT if adjoint else 0) | (FR_INVERSE if inverse else 0),
                              _c.byref(out), _stream_handle(dev, stream))
    return out.value, _check(st, "fresnel_direct")


def plan_route(w0, z_waist, wavelength, n, dx, z_from, z_to):
    """fr_plan_route: the steps (kind, z, dx_in, dx_out) carrying a field from z_from to z_to
    under a Gaussian pilot beam of waist w0 at z_waist."""
    steps = (FrRouteStep * 2)()
    k = _check(lib().fr_plan_route(float(w0), float(z_waist), float(wavelength), int(n), float(dx),
                                   float(z_from), float(z_to), steps, 2), "fr_plan_route")
    return [(steps[i].kind, steps[i].z_m, steps[i].dx_in_m, steps[i].dx_out_m) for i in range(k)]


def follow_route(field, wavelength, steps, stream=None):
    """Run planned steps on `field` in place (fresnel_step / fresnel_direct, one call each);
    returns the final pitch."""
    dx = None
    for kind, z, dx_in, dx_out in steps:
        if kind == FR_ROUTE_AS:
            fresnel_step(field, dx_in, wavelength, z, stream=stream)
        elif kind == FR_ROUTE_DIRECT:
            fresnel_direct(field, dx_in, wavelength, z, stream=stream)
        elif kind == FR_ROUTE_DIRECT_INVERSE:
            fresnel_direct(field, dx_out, wavelength, z, inverse=True, stream=stream)
        else:
            raise ValueError("unknown route step")
        dx = dx_out
    return dx


def _optics(optics, n=None):
    """optics: sequence of (z_m, lens_focal_m, amp or None, opd or None) -> FrOptic array."""
    arr = (FrOptic * len(optics))()
    for i, (z, f, amp, opd) in enumerate(optics):
        for t, name in ((amp, "amp"), (opd, "opd")):
            if t is not None and n is not None:
                _need(t, torch.float32, (n, n), f"optics[{i}].{name}")
        arr[i] = FrOptic(float(z), float(f), amp.data_ptr() if amp is not None else None,
                         opd.data_ptr() if opd is not None else None)
    return arr


def plan_system(n, dx, wavelength, beam_radius, optics):
    """fr_plan_system: ([pitch of each plane], 2-D transforms of the system). optics as for
    propagate_system (masks may be None: only distances and lenses matter)."""
    arr = _optics(optics)
    pitches = (_c.c_double * len(optics))()
    tr = _c.c_int32()
    _check(lib().fr_plan_system(int(n), float(dx), float(wavelength), float(beam_radius), arr, len(optics),
                                pitches, _c.byref(tr)), "fr_plan_system")
    return list(pitches), tr.value


def propagate_system(field, dx, wavelength, beam_radius, optics, stream=None):
    """In place on an n x n complex64 GPU tensor: the system of optics (z_m from the previous
    plane, lens focal length, amp, opd: maps on each plane's pitch from plan_system); returns the
    pitch of the last plane."""
    n = field.shape[0] if field.dim() == 2 else -1
    _need(field, torch.complex64, (n, n), "field")
    arr = _optics(optics, n)
    dx_out = _c.c_double()
    dev = field.device.index
    _check(lib().propagate_system(context(dev).handle, _ptr(field), n, float(dx), float(wavelength),
                                  float(beam_radius), arr, len(optics), _c.byref(dx_out),
                                  _stream_handle(dev, stream)), "propagate_system")
    return dx_out.value


def fresnel_step_f64(field, dx, wavelength, z, amp=None, opd=None, lens_focal=0.0, adjoint=False,
                     stream=None):
    """In place on an n x n complex128 GPU tensor: the Fresnel step of fresnel_step in float64
    (float64 amp / opd maps). Returns the status (warning bits) or raises."""
    n = field.shape[0] if field.dim() == 2 else -1
    _need(field, torch.complex128, (n, n), "field")
    for t, name in ((amp, "amp"), (opd, "opd")):
        if t is not None:
            _need(t, torch.float64, (n, n), name)
    dev = field.device.index
    st = lib().fresnel_step_f64(context(dev).handle, _ptr(field), n, float(dx), float(wavelength), float(z),
                                _ptr(amp), _ptr(opd), float(lens_focal), FR_ADJOINT if adjoint else 0,
                                _stream_handle(dev, stream))
    return _check(st, "fresnel_step_f64")


def _planes(fields, dx, wavelengths, zs, amps, opds, lens_focals, adjoints):
    """FrPlane array of a batch: per-plane sequences (or scalars)."""
    count = len(fields)
    if count == 0:
        raise ValueError("empty batch")

    def seq(v, default):
        if v is None:
            return [default] * count
        if isinstance(v, (list, tuple)):
            if len(v) != count:
                raise ValueError("per-plane sequence length mismatch")
            return list(v)
        return [v] * count

    dxs, lams, zz = seq(dx, None), seq(wavelengths, None), seq(zs, None)
    amps, opds = seq(amps, None), seq(opds, None)
    lf, adj = seq(lens_focals, 0.0), seq(adjoints, False)
    arr = (FrPlane * count)()
    for i, f in enumerate(fields):
        n = f.shape[0] if f.dim() == 2 else -1
        _need(f, torch.complex64, (n, n), f"fields[{i}]")
        for t, nm in ((amps[i], "amp"), (opds[i], "opd")):
            if t is not None:
                _need(t, torch.float32, (n, n), nm)
        arr[i] = FrPlane(f.data_ptr(), amps[i].data_ptr() if amps[i] is not None else None,
                         opds[i].data_ptr() if opds[i] is not None else None, float(dxs[i]),
                         float(lams[i]), float(zz[i]), float(lf[i]), n,
                         FR_ADJOINT if adj[i] else 0)
    return arr


def fresnel_step_batched(fields, dx, wavelengths, zs, amps=None, opds=None, lens_focals=None,
                         adjoints=None, stream=None, graph=False):
    """Many planes in one launch per sweep; per-plane sequences (or scalars). Planes may have
    different edges (power-of-two edges take the two-sweep kernels, one launch per sweep for
    the planes of each edge; the others the mixed-radix sweeps).
    graph: the library records the call's launches as one graph the first time these plane
    entries (field / map addresses, parameters) and stream are seen, and replays it later."""
    arr = _planes(fields, dx, wavelengths, zs, amps, opds, lens_focals, adjoints)
    count = len(fields)
    dev = fields[0].device.index
    fn = lib().fresnel_step_batched_graph if graph else lib().fresnel_step_batched
    st = fn(context(dev).handle, arr, count, _stream_handle(dev, stream))
    return _check(st, "fresnel_step_batched_graph" if graph else "fresnel_step_batched")


def fresnel_step_exact_batched(fields, dx, wavelengths, zs, amps=None, opds=None, lens_focals=None,
                               adjoints=None, stream=None):
    """Many planes of the exact-transfer-function step in one call (one power-of-two edge);
    per-plane sequences (or scalars). Returns the warning bits."""
    arr = _planes(fields, dx, wavelengths, zs, amps, opds, lens_focals, adjoints)
    dev = fields[0].device.index
    st = lib().fresnel_step_exact_batched(context(dev).handle, arr, len(fields), _stream_handle(dev, stream))
    return _check(st, "fresnel_step_exact_batched")


# ---- MFT ----------------------------------------------------------------------------------

def mft_forward(inp, n_d, m_out, du, mask=None, out=None, stream=None):
    """(du/n_d) W inp W^T (* mask): n_in x n_in (view allowed) -> m_out x m_out."""
    if inp.dtype != torch.complex64 or not inp.is_cuda:
        raise TypeError("inp must be a complex64 GPU tensor")
    n_in = inp.shape[0]
    if inp.shape != (n_in, n_in):
        raise ValueError("inp must be square")
    ld_in = _row_stride(inp, "inp")
    dev = inp.device.index
    if out is None:
        out = _empty((m_out, m_out), torch.complex64, inp.device, stream)
    ld_out = _row_stride(out, "out")
    if mask is not None:
        _need(mask, torch.float32, (m_out, m_out), "mask")
    L = lib()
    nbytes = L.mft_workspace_bytes(n_in, m_out)
    ws = workspace(nbytes, dev, stream)
    st = L.mft_forward(context(dev).handle, _ptr(inp), n_in, ld_in, _ptr(out), m_out, ld_out,
                       float(n_d), float(du), _ptr(mask), _ptr(ws), ws.numel(),
                       _stream_handle(dev, stream))
    _check(st, "mft_forward")
    return out


def mft_f64(inp, n_d, size_out, du, adjoint=False, stream=None):
    """The MFT in float64: (du/n_d) W inp W^T (n x n -> size_out x size_out), or with adjoint its
    exact adjoint (du/n_d) W^H inp conj(W) (m x m -> size_out x size_out). inp: dense complex128
    GPU tensor."""
    if inp.dtype != torch.complex128 or not inp.is_cuda or not inp.is_contiguous():
        raise TypeError("inp must be a contiguous complex128 GPU tensor")
    k = inp.shape[0]
    if inp.shape != (k, k):
        raise ValueError("inp must be square")
    n, m = (size_out, k) if adjoint else (k, size_out)
    dev = inp.device.index
    out = _empty((size_out, size_out), torch.complex128, inp.device, stream)
    L = lib()
    nbytes = L.mft_f64_workspace_bytes(n, m)
    ws = workspace(nbytes, dev, stream)
    st = L.mft_f64(context(dev).handle, _ptr(inp), _ptr(out), n, m, float(n_d), float(du),
                   FR_ADJOINT if adjoint else 0, _ptr(ws), ws.numel(), _stream_handle(dev, stream))
    _check(st, "mft_f64")
    return out


def mft_forward_noalloc(inp, n_d, m_out, du, out, mask=None, stream=None):
    """mft_forward through the allocation-free entry point (the library's own device scratch
    array, no workspace): the caller passes the output; the MFT matrix of the geometry must have
    been built by an earlier mft_forward call. Returns the status (warning bits) or raises."""
    if inp.dtype != torch.complex64 or not inp.is_cuda:
        raise TypeError("inp must be a complex64 GPU tensor")
    n_in = inp.shape[0]
    if inp.shape != (n_in, n_in):
        raise ValueError("inp must be square")
    _need(out, torch.complex64, (m_out, m_out), "out")
    if mask is not None:
        _need(mask, torch.float32, (m_out, m_out), "mask")
    dev = inp.device.index
    st = lib().mft_forward_noalloc(context(dev).handle, _ptr(inp), n_in, _row_stride(inp, "inp"), _ptr(out),
                                   m_out, _row_stride(out, "out"), float(n_d), float(du), _ptr(mask),
                                   _stream_handle(dev, stream))
    return _check(st, "mft_forward_noalloc")


def mft_adjoint(inp, n_d, n_out, du, alpha=1.0, beta=0.0, mask=None, out=None, stream=None):
    """alpha (du/n_d) W^H inp conj(W) + beta out (* mask): m x m -> n_out x n_out (view allowed)."""
    if inp.dtype != torch.complex64 or not inp.is_cuda:
        raise TypeError("inp must be a complex64 GPU tensor")
    m_in = inp.shape[0]
    ld_in = _row_stride(inp, "inp")
    dev = inp.device.index
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs an out tensor")
        out = _empty((n_out, n_out), torch.complex64, inp.device, stream)
    if tuple(out.shape) != (n_out, n_out):
        raise ValueError("out shape mismatch")
    ld_out = _row_stride(out, "out")
    if mask is not None:
        _need(mask, torch.float32, (n_out, n_out), "mask")
    L = lib()
    nbytes = L.mft_workspace_bytes(n_out, m_in)
    ws = workspace(nbytes, dev, stream)
    st = L.mft_adjoint(context(dev).handle, _ptr(inp), m_in, ld_in, _ptr(out), n_out, ld_out,
                       float(n_d), float(du), float(alpha), float(beta), _ptr(mask), _ptr(ws),
                       ws.numel(), _stream_handle(dev, stream))
    _check(st, "mft_adjoint")
    return out


def set_cache_limit(max_tables, device=None):
    """fr_set_cache_limit: bound of the device context's table cache (applied at call starts)."""
    _check(lib().fr_set_cache_limit(context(device).handle, int(max_tables)), "fr_set_cache_limit")


# ---- autotuner -------------------------------------------------------------------------------

FR_TUNE_FRESNEL = 1
FR_TUNE_MFT = 2


def autotune_fresnel(n, device=None, stream=None):
    """Time the sweep configurations for plane edge n and keep the fastest in the context."""
    dev = torch.cuda.current_device() if device is None else device
    _check(lib().fr_autotune(context(dev).handle, FR_TUNE_FRESNEL, int(n), 0, _stream_handle(dev, stream)),
           "fr_autotune")


def autotune_mft(n, m, device=None, stream=None):
    """Time the GEMM tile configurations of the n <-> m MFTs and keep the fastest."""
    dev = torch.cuda.current_device() if device is None else device
    _check(lib().fr_autotune(context(dev).handle, FR_TUNE_MFT, int(n), int(m), _stream_handle(dev, stream)),
           "fr_autotune")


def autotune_save(path, device=None):
    _check(lib().fr_autotune_save(context(device).handle, os.fsencode(path)), "fr_autotune_save")


def autotune_load(path, device=None):
    _check(lib().fr_autotune_load(context(device).handle, os.fsencode(path)), "fr_autotune_load")


# ---- kernel timing ---------------------------------------------------------------------------

def profile_enable(enable=True, device=None):
    """Bracket every kernel launch of the device's context with HIP events on its stream."""
    _check(lib().fr_profile_enable(context(device).handle, 1 if enable else 0), "fr_profile_enable")


def profile_read(device=None, max_entries=64):
    """{kernel/tag: (total_ms, launches)} since the last read (waits for the events)."""
    name_len = 96
    names = _c.create_string_buffer(max_entries * name_len)
    tot = (_c.c_double * max_entries)()
    cnt = (_c.c_int64 * max_entries)()
    n = _c.c_int32()
    _check(lib().fr_profile_read(context(device).handle, max_entries, names, name_len, tot, cnt,
                                 _c.byref(n)), "fr_profile_read")
    out = {}
    raw = names.raw
    for i in range(n.value):
        nm = raw[i * name_len:(i + 1) * name_len].split(b"\0", 1)[0].decode()
        out[nm] = (tot[i], cnt[i])
    return out


# ---- Lyot coronagraph train ----------------------------------------------------------------

class Train:
    """Geometry and optics of a Lyot coronagraph train (device tensors) for propagate_train.

    pupil_amp, pupil_opd, lyot: n_d x n_d float32; occ_mask: occ_m x occ_m float32 (1 = blocked).
    """

    def __init__(self, n_d, d_m, z_m, pupil_amp, lyot, occ_mask, occ_du_c, det_m, det_du_c,
                 lambda_c_m=550e-9, pupil_opd=None, n_act=0, n_dm=0):
        self.n_d, self.d_m, self.z_m = int(n_d), float(d_m), float(z_m)
        self.pupil_amp, self.pupil_opd, self.lyot, self.occ_mask = pupil_amp, pupil_opd, lyot, occ_mask
        self.occ_m = int(occ_mask.shape[0]) if occ_mask is not None else 1
        self.occ_du_c, self.det_m, self.det_du_c = float(occ_du_c), int(det_m), float(det_du_c)
        self.lambda_c_m, self.n_act, self.n_dm = float(lambda_c_m), int(n_act), int(n_dm)
        nd = self.n_d
        _need(pupil_amp, torch.float32, (nd, nd), "pupil_amp")
        _need(lyot, torch.float32, (nd, nd), "lyot")
        if pupil_opd is not None:
            _need(pupil_opd, torch.float32, (nd, nd), "pupil_opd")
        if occ_mask is not None:
            _need(occ_mask, torch.float32, (self.occ_m, self.occ_m), "occ_mask")

    def desc(self, heights):
        d = FrTrainDesc()
        d.n_d, d.d_m = self.n_d, self.d_m
        d.pupil_amp = self.pupil_amp.data_ptr()
        d.pupil_opd_m = self.pupil_opd.data_ptr() if self.pupil_opd is not None else None
        d.n_dm, d.n_act = self.n_dm, self.n_act
        d.dm_heights_m = heights.data_ptr() if heights is not None else None
        d.z_m = self.z_m
        d.occ_m, d.occ_du_c = self.occ_m, self.occ_du_c
        d.occ_mask = self.occ_mask.data_ptr() if self.occ_mask is not None else None
        d.lyot = self.lyot.data_ptr()
        d.det_m, d.det_du_c, d.lambda_c_m = self.det_m, self.det_du_c, self.lambda_c_m
        return d


def propagate_train(train, wavelengths, n_pad, weights, heights=None, occulter=True,
                    grad_psf=None, batched=False, graph=False, out=None, grad_out=None,
                    stream=None, ckpt=None, phase=None):
    """Broadband PSF (det_m x det_m float32) of the train; with grad_psf = dL/dPSF also returns
    dL/dheights (n_dm x n_act x n_act float32).

    batched: the Fresnel planes of all wavelengths in one launch per sweep (one plane per
    wavelength held in the workspace; same results).
    graph: the library records the whole call as one graph and replays it on later calls with
    the same arguments, which includes the addresses of heights, grad_psf, the outputs and the
    workspace; pass out= / grad_out= (and keep heights in place) so that they stay fixed.
    phase="save": forward only, keeping what the adjoint needs in `ckpt` (a uint8 GPU tensor of
    at least train_ckpt_bytes(...) bytes; returns the PSF); phase="backward": the gradient from
    that checkpoint (grad_psf required; returns dL/dheights only)."""
    dev = train.pupil_amp.device.index
    nl = len(wavelengths)
    if len(n_pad) != nl or len(weights) != nl:
        raise ValueError("wavelengths, n_pad and weights must have one entry per wavelength")
    if train.n_dm:
        _need(heights, torch.float32, (train.n_dm, train.n_act, train.n_act), "heights")
    if phase not in (None, "save", "backward"):
        raise ValueError("phase must be None, 'save' or 'backward'")
    mode = ((0 if occulter else FR_TRAIN_NO_OCCULTER) | (FR_TRAIN_BATCHED if batched else 0)
            | (FR_TRAIN_GRAPH if graph else 0))
    if phase is not None:
        if ckpt is None or ckpt.dtype != torch.uint8 or not ckpt.is_cuda:
            raise TypeError("ckpt must be a uint8 GPU tensor")
        mode |= FR_TRAIN_FWD_SAVE if phase == "save" else FR_TRAIN_BWD
    gh = None
    if grad_psf is not None:
        if phase == "save":
            raise ValueError("phase='save' takes no grad_psf")
        _need(grad_psf, torch.float32, (train.det_m, train.det_m), "grad_psf")
        if phase is None:
            mode |= FR_TRAIN_GRAD
        if grad_out is not None:
            _need(grad_out, torch.float32, (train.n_dm, train.n_act, train.n_act), "grad_out")
            gh = grad_out
        else:
            gh = _empty((train.n_dm, train.n_act, train.n_act), torch.float32, train.pupil_amp.device,
                        stream)
    elif phase == "backward":
        raise ValueError("phase='backward' needs grad_psf")
    lam = (_c.c_double * nl)(*[float(x) for x in wavelengths])
    npd = (_c.c_int32 * nl)(*[int(x) for x in n_pad])
    w = (_c.c_float * nl)(*[float(x) for x in weights])
    d = train.desc(heights)
    L = lib()
    nbytes = L.propagate_train_workspace_bytes(_c.byref(d), nl, npd, mode)
    if nbytes == 0:
        raise ValueError("invalid train geometry")
    ws = workspace(nbytes, dev, stream)
    psf = None
    if phase != "backward":
        if out is not None:
            _need(out, torch.float32, (train.det_m, train.det_m), "out")
            psf = out
        else:
            psf = _empty((train.det_m, train.det_m), torch.float32, train.pupil_amp.device, stream)
    st = L.propagate_train(context(dev).handle, _c.byref(d), nl, lam, npd, w, mode, _ptr(psf),
                           _ptr(grad_psf), _ptr(gh), _ptr(ckpt), ckpt.numel() if ckpt is not None else 0,
                           _ptr(ws), ws.numel(), _stream_handle(dev, stream))
    _check(st, "propagate_train")
    if phase == "backward":
        return gh
    return (psf, gh) if grad_psf is not None else psf


def train_ckpt_bytes(train, n_pad):
    """Bytes of the checkpoint that propagate_train(phase='save') fills for these grids."""
    nl = len(n_pad)
    npd = (_c.c_int32 * nl)(*[int(x) for x in n_pad])
    d = train.desc(None)
    return int(lib().propagate_train_ckpt_bytes(_c.byref(d), nl, npd))


class DMHeightsToPSF(torch.autograd.Function):
    """heights (n_dm x n_act x n_act) -> broadband PSF, with the library's adjoint as backward.

    apply(heights, train, wavelengths, n_pad, weights[, batched]). The forward keeps the
    library's checkpoint (per wavelength the field at the last DM plane and the detector field)
    and the backward runs only the adjoint chain from it."""

    @staticmethod
    def forward(ctx, heights, train, wavelengths, n_pad, weights, batched=False):
        h = heights.detach().contiguous()
        ctx.train, ctx.args = train, (list(wavelengths), list(n_pad), list(weights), bool(batched))
        ck = torch.empty(train_ckpt_bytes(train, n_pad), dtype=torch.uint8, device=h.device)
        ctx.save_for_backward(h, ck)
        return propagate_train(train, wavelengths, n_pad, weights, h, batched=batched, ckpt=ck, phase="save")

    @staticmethod
    def backward(ctx, grad_out):
        h, ck = ctx.saved_tensors
        wl, npd, w, batched = ctx.args
        gh = propagate_train(ctx.train, wl, npd, w, h, grad_psf=grad_out.contiguous().float(), batched=batched,
                             ckpt=ck, phase="backward")
        return gh, None, None, None, None, None
