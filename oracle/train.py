"""FP64 Lyot-coronagraph train, deformable mirrors, gradient and finite differences.

TEST INFRASTRUCTURE (see the package docstring): never imported by the product path.

The train is the paper's statement of a coronagraph model (Sec. 1.1: Fresnel steps between
optics, then the semi-analytic Lyot coronagraph of Soummer et al. by matrix DFTs; Sec. 1.2:
the whole sequence is repeated for every wavelength), reduced to a fixed topology:

  pupil A exp(2 pi i phi/lambda) [x DM1 phasor]  --AS over z-->  x DM phasor = E_dm
  E_occ = MFT(E_dm: full padded plane -> occ_m^2)
  E_L   = Lyot . ( window(E_dm) - MFT^H(M_occ . E_occ -> n_d^2 window) )   (Babinet form)
  E_det = MFT(E_L -> det_m^2);   I = |E_det|^2

Focal grids are fixed in units of lambda_c/D, so the per-wavelength sampling is
du_lambda = du_c lambda_c / lambda and every mask is one lambda-independent array.
The deformable mirrors and the gradient are additions on top of the paper's forward model;
their definitions are the ordinary chain rule of that model.
"""

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from .core import as_propagate, centred, mft, mft_adjoint


def embed(a, n):
    """Place an n_d x n_d array in the centre of an n x n zero array (offset (n - n_d)//2)."""
    nd = a.shape[0]
    off = (n - nd) // 2
    out = np.zeros((n, n), dtype=np.result_type(a.dtype, np.complex128))
    out[off:off + nd, off:off + nd] = a
    return out


def extract(a, nd):
    """The centred nd x nd window of an n x n array (inverse of embed)."""
    off = (a.shape[0] - nd) // 2
    return a[off:off + nd, off:off + nd]


# --------------------------------------------------------------------------------------------
# O6. Deformable mirror: separable Gaussian influence functions (Sec. 1.2: 32x32 to 196x196
#     actuator mirrors sampled by hundreds of pixels).
# --------------------------------------------------------------------------------------------

def dm_influence(n, n_d, n_act):
    """G[i, a] = exp(-(c(i) - xi_a)^2 / (2 sigma^2)), xi_a = (a - (n_act-1)/2) p, sigma = p = n_d/n_act."""
    p = float(n_d) / float(n_act)
    xi = (np.arange(n_act, dtype=np.float64) - (n_act - 1) / 2.0) * p
    c = centred(n).astype(np.float64)
    return np.exp(-((c[:, None] - xi[None, :]) ** 2) / (2.0 * p * p))


def dm_surface(heights, n, n_d):
    """Mirror surface s = G A G^T [m] over the full n x n grid (A: n_act x n_act heights)."""
    g = dm_influence(n, n_d, heights.shape[0])
    return g @ np.asarray(heights, dtype=np.float64) @ g.T


@dataclass
class TrainGeometry:
    n_d: int                 # pupil pixels across D
    d_m: float               # pupil diameter [m]; dx = d_m / n_d
    z_m: float               # Fresnel distance pupil -> (last) DM plane [m]
    occ_m: int               # occulter grid edge
    occ_du_c: float          # occulter pitch [lambda_c / D]
    det_m: int               # detector grid edge
    det_du_c: float          # detector pitch [lambda_c / D]
    lambda_c: float          # reference wavelength [m]
    pupil_amp: np.ndarray    # n_d x n_d
    occ_mask: np.ndarray     # occ_m x occ_m, 1 where the spot blocks (Babinet subtraction)
    lyot: np.ndarray         # n_d x n_d
    pupil_opd: Optional[np.ndarray] = None   # n_d x n_d OPD [m]

    @property
    def dx(self):
        return self.d_m / self.n_d


@dataclass
class TrainForward:
    e_det: np.ndarray
    e_dm: List[np.ndarray] = field(default_factory=list)    # field just after each DM
    dm_phasors: List[np.ndarray] = field(default_factory=list)


def _dm_phasor(surface, wavelength):
    turns = 2.0 * surface / float(wavelength)              # reflection: OPD = 2 x surface
    return np.exp(2j * np.pi * (turns - np.round(turns)))


def train_forward(geom: TrainGeometry, wavelength, n, heights: Sequence[np.ndarray], occulter=True,
                  step_cache=None):
    """One wavelength through the train on an n x n padded grid.

    heights: one array (the DM after the Fresnel step) or two (DM1 at the pupil, DM2 after
    the step), each n_act x n_act surface heights in m.
    step_cache: optional dict; the Fresnel step's result is remembered there per (wavelength,
    n) and, with two DMs, the pupil DM's heights (the only heights it depends on), and reused
    (memoisation only: the arithmetic is unchanged).
    """
    lam = float(wavelength)
    nd = geom.n_d
    pupil = np.asarray(geom.pupil_amp, dtype=np.float64).astype(np.complex128)
    if geom.pupil_opd is not None:
        t = np.asarray(geom.pupil_opd, dtype=np.float64) / lam
        pupil = pupil * np.exp(2j * np.pi * (t - np.round(t)))
    e = embed(pupil, n)
    out = TrainForward(e_det=None)
    hs = list(heights)
    if len(hs) == 2:
        ph1 = _dm_phasor(dm_surface(hs[0], n, nd), lam)
        e = e * ph1
        out.e_dm.append(e)
        out.dm_phasors.append(ph1)
    key = (lam, n) if len(hs) < 2 else (lam, n, np.asarray(hs[0], dtype=np.float64).tobytes())
    if step_cache is not None and key in step_cache:
        e = step_cache[key]
    else:
        e = as_propagate(e, geom.dx, lam, geom.z_m)
        if step_cache is not None:
            step_cache[key] = e
    if hs:
        ph = _dm_phasor(dm_surface(hs[-1], n, nd), lam)
        e = e * ph
        out.e_dm.append(e)
        out.dm_phasors.append(ph)
    else:
        out.e_dm.append(e)
    out.e_det = dm_to_detector(geom, lam, e, occulter)
    return out


def dm_to_detector(geom: TrainGeometry, wavelength, e_dm, occulter=True):
    """The linear map F_lambda from the field after the last DM (n x n) to the detector field:
    Babinet occulter (Soummer et al.), Lyot stop, detector MFT."""
    lam = float(wavelength)
    nd = geom.n_d
    du_occ = geom.occ_du_c * geom.lambda_c / lam
    e_l = extract(e_dm, nd).copy()
    if occulter:
        e_occ = mft(e_dm, nd, geom.occ_m, du_occ)
        e_l = e_l - mft_adjoint(geom.occ_mask * e_occ, nd, nd, du_occ)
    e_l = geom.lyot * e_l
    return mft(e_l, nd, geom.det_m, geom.det_du_c * geom.lambda_c / lam)


def dm_to_detector_adjoint(geom: TrainGeometry, wavelength, n, y, occulter=True):
    """F_lambda^H: detector field (det_m^2) -> DM-plane field (n x n). Each piece of
    dm_to_detector is replaced by its adjoint, in reverse order (the masks are real)."""
    lam = float(wavelength)
    nd = geom.n_d
    du_occ = geom.occ_du_c * geom.lambda_c / lam
    du_det = geom.det_du_c * geom.lambda_c / lam
    y = geom.lyot * mft_adjoint(y, nd, nd, du_det)
    b = embed(y, n)
    if occulter:
        b = b - mft_adjoint(geom.occ_mask * mft(y, nd, geom.occ_m, du_occ), nd, n, du_occ)
    return b


def train_psf(geom, wavelengths, ns, weights, heights, occulter=True, step_cache=None):
    """Broadband PSF sum_lambda w_lambda |E_det,lambda|^2 (det_m x det_m, float64)."""
    psf = np.zeros((geom.det_m, geom.det_m))
    for lam, n, w in zip(wavelengths, ns, weights):
        e = train_forward(geom, lam, n, heights, occulter, step_cache).e_det
        psf += float(w) * (e.real ** 2 + e.imag ** 2)
    return psf


def train_loss(geom, wavelengths, ns, weights, heights, dh_mask, max_ref, step_cache=None):
    """Mean normalised contrast over the dark hole: sum_DH PSF / (|DH| max I_ref)."""
    psf = train_psf(geom, wavelengths, ns, weights, heights, True, step_cache)
    return float(np.sum(psf * dh_mask) / (np.sum(dh_mask) * max_ref))


# --------------------------------------------------------------------------------------------
# O7. Backward: adjoints of every linear piece in reverse order, then the phase-to-height chain.
# --------------------------------------------------------------------------------------------

def train_backward(geom, wavelength, n, heights, fwd: TrainForward, grad_intensity, occulter=True):
    """Gradients of L w.r.t. each DM's actuator heights for one wavelength, given
    grad_intensity = dL/dI (det_m x det_m, real). Returns a list aligned with heights."""
    lam = float(wavelength)
    nd = geom.n_d
    b = dm_to_detector_adjoint(geom, lam, n, grad_intensity * fwd.e_det, occulter)
    kappa = 4.0 * np.pi / lam
    hs = list(heights)
    grads = [None] * len(hs)
    g_inf = None
    if hs:
        g_inf = dm_influence(n, nd, hs[0].shape[0])
        gs = -2.0 * kappa * np.imag(fwd.e_dm[-1] * np.conj(b))
        grads[-1] = g_inf.T @ gs @ g_inf
    if len(hs) == 2:
        b1 = as_propagate(np.conj(fwd.dm_phasors[-1]) * b, geom.dx, lam, -geom.z_m)
        gs1 = -2.0 * kappa * np.imag(fwd.e_dm[0] * np.conj(b1))
        grads[0] = g_inf.T @ gs1 @ g_inf
    return grads


def train_grad(geom, wavelengths, ns, weights, heights, dh_mask, max_ref):
    """dL/d(heights) of the mean dark-hole contrast, summed over wavelengths (max_ref fixed)."""
    hs = list(heights)
    total = [np.zeros_like(np.asarray(h, dtype=np.float64)) for h in hs]
    cnt = float(np.sum(dh_mask))
    for lam, n, w in zip(wavelengths, ns, weights):
        fwd = train_forward(geom, lam, n, hs, True)
        g_i = (float(w) / (cnt * max_ref)) * dh_mask
        for acc, g in zip(total, train_backward(geom, lam, n, hs, fwd, g_i, True)):
            acc += g
    return total


def fd_grad(geom, wavelengths, ns, weights, heights, dh_mask, max_ref, actuators, h=1e-12,
            step_cache=None):
    """Central differences of train_loss on single actuators: actuators = [(dm, row, col), ...]."""
    out = []
    for dm, r, c in actuators:
        plus = [np.array(a, dtype=np.float64, copy=True) for a in heights]
        minus = [np.array(a, dtype=np.float64, copy=True) for a in heights]
        plus[dm][r, c] += h
        minus[dm][r, c] -= h
        lp = train_loss(geom, wavelengths, ns, weights, plus, dh_mask, max_ref, step_cache)
        lm = train_loss(geom, wavelengths, ns, weights, minus, dh_mask, max_ref, step_cache)
        out.append((lp - lm) / (2.0 * h))
    return np.array(out)
