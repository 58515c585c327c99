"""Core FP64 definitions: DFT, optic phasor, angular-spectrum step, MFT.

TEST INFRASTRUCTURE (see the package docstring): never imported by the product path.

Conventions (fixed readings of points the paper leaves open):
  * arrays are indexed [y, x]; the optical axis sits on pixel n//2 of every
    plane, so the centred coordinate of index i is c(i) = i - n//2 (the
    fftshift discussion of Sec. 2.4 is about exactly this re-centring);
  * the signed frequency index of DFT bin k is k if k < n/2, else k - n;
  * no e^{ikz} piston and no 1/(i lambda z) factor are applied (intensity-
    invariant; Sec. 1.1 does not state them).
"""

from functools import lru_cache

import numpy as np


def centred(n):
    """c(i) = i - n//2 as int64 (axis on pixel n//2)."""
    return np.arange(n, dtype=np.int64) - n // 2


def signed_index(n):
    """Signed DFT frequency index: k for k < n/2, k - n otherwise."""
    k = np.arange(n, dtype=np.int64)
    return np.where(2 * k < n, k, k - n)


# --------------------------------------------------------------------------------------------
# O1. Discrete Fourier transform (Sec. 1.2: the transform the FFT evaluates in O(n log n)).
# --------------------------------------------------------------------------------------------

@lru_cache(maxsize=4)
def _dft_matrix_cached(n):
    k = np.arange(n, dtype=np.int64)
    p = np.outer(k, k) % n                      # exact integer index reduction
    w = np.exp((-2j * np.pi / n) * p)
    w.setflags(write=False)
    return w


def dft_matrix(n):
    """W[k, m] = exp(-2 pi i ((k m) mod n) / n), the n-point DFT matrix (symmetric)."""
    return _dft_matrix_cached(int(n))


def dft2(u):
    """Unnormalised 2-D DFT, W U W^T (first along y, then along x)."""
    n = u.shape[0]
    if u.shape != (n, n):
        raise ValueError("square arrays only")
    w = dft_matrix(n)
    return w @ u @ w.T


def idft2(u):
    """Inverse 2-D DFT, conj(W) U conj(W)^T / n^2."""
    n = u.shape[0]
    if u.shape != (n, n):
        raise ValueError("square arrays only")
    wc = dft_matrix(n).conj()
    return (wc @ u @ wc.T) / (n * n)


# --------------------------------------------------------------------------------------------
# O3. Angular-spectrum plane-to-plane step, paraxial transfer function
#     (Sec. 1.1: angular spectrum propagation after Lawrence Eqs. 82-89).
# --------------------------------------------------------------------------------------------

def transfer_function(n, dx, wavelength, z):
    """H[ky, kx] = exp(-i pi lambda z (fx^2 + fy^2)), f = signed index / (n dx).

    Formed per pixel (not factored): the integer kx^2 + ky^2 is exact, the phase
    is taken in turns in float64 and reduced to [-1/2, 1/2] before the exponential.
    """
    k = signed_index(n)
    q = k[:, None] ** 2 + k[None, :] ** 2
    turns = q * (-float(wavelength) * float(z) / (2.0 * (n * float(dx)) ** 2))
    turns = turns - np.round(turns)
    return np.exp(2j * np.pi * turns)


def as_propagate(u, dx, wavelength, z):
    """U(z) = IDFT2( H . DFT2(U) ): one angular-spectrum step over signed distance z."""
    n = u.shape[0]
    return idft2(transfer_function(n, dx, wavelength, z) * dft2(np.asarray(u, dtype=np.complex128)))


def as_propagate_rows(u, dx, wavelength, z, rows):
    """Rows `rows` of as_propagate(u, dx, wavelength, z), at O(len(rows) n^2) cost.

    The paraxial H is the outer product h (x) h with h[k] = exp(-i pi lambda z k~^2/(n dx)^2),
    so IDFT2(H . DFT2(U)) = K U K^T with the circulant K = IDFT diag(h) DFT, whose entries are
    K[y, r] = kappa[(y - r) mod n] for kappa = IDFT(h) (1-D). Rows of the result are then
    K[rows, :] U K^T: no 2-D transform of the whole plane is needed.
    """
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[0]
    k = signed_index(n)
    turns = (k * k) * (-float(wavelength) * float(z) / (2.0 * (n * float(dx)) ** 2))
    turns = turns - np.round(turns)
    h = np.exp(2j * np.pi * turns)
    kappa = (dft_matrix(n).conj() @ h) / n
    rows = np.asarray(rows, dtype=np.int64)
    i = np.arange(n, dtype=np.int64)
    left = kappa[(rows[:, None] - i[None, :]) % n] @ u
    return left @ kappa[(i[:, None] - i[None, :]) % n].T


# --------------------------------------------------------------------------------------------
# O2. Optic multiply: the complex phasor of Eq. (3), A exp(2 pi i phi / lambda), plus a
#     reflective surface (OPD = 2 x surface) and a thin lens exp(-i pi r^2 / (lambda f))
#     (Sec. 1.1: powered optics as thin lenses, Goodman Eq. 5-10; Eq. (2) is the
#     quadratic-phase exponential).
# --------------------------------------------------------------------------------------------

def optic_phasor(n, dx, wavelength, amp=None, opd=None, surface=None, lens_focal=0.0):
    """A exp(2 pi i (opd + 2 surface) / lambda) exp(-i pi r^2 / (lambda f)) on an n x n grid.

    amp, opd, surface: n x n real arrays or None. lens_focal: focal length in m (0: no lens).
    """
    lam = float(wavelength)
    turns = np.zeros((n, n))
    if opd is not None:
        turns = turns + np.asarray(opd, dtype=np.float64) / lam
    if surface is not None:
        turns = turns + 2.0 * np.asarray(surface, dtype=np.float64) / lam
    if lens_focal:
        c = centred(n)
        r2 = (c[:, None] ** 2 + c[None, :] ** 2) * (float(dx) ** 2)
        turns = turns - r2 / (2.0 * lam * float(lens_focal))
    turns = turns - np.round(turns)
    ph = np.exp(2j * np.pi * turns)
    if amp is not None:
        ph = ph * np.asarray(amp, dtype=np.float64)
    return ph


def fresnel_step(u, dx, wavelength, z, amp=None, opd=None, lens_focal=0.0, adjoint=False):
    """One Fresnel plane: optic multiply (Eq. 3 + thin lens) then AS step over z.

    adjoint=True applies the exact adjoint of that linear map: AS over -z, then
    multiply by the conjugate optic phasor.
    """
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[0]
    ph = optic_phasor(n, dx, wavelength, amp, opd, None, lens_focal)
    if adjoint:
        return as_propagate(u, dx, wavelength, -z) * np.conj(ph)
    return as_propagate(u * ph, dx, wavelength, z)


# --------------------------------------------------------------------------------------------
# O4. Matrix Fourier transform (Sec. 1.1: the semi-analytic coronagraph of Soummer et al. uses
#     matrix DFTs of modest arrays; Sec. 2.3: the sin/cos arrays of the matrix DFT).
# --------------------------------------------------------------------------------------------

def mft_matrix(m_out, n_in, n_d, du):
    """W[k, m] = exp(-2 pi i u_k x_m), u_k = (k - m_out//2) du  [lambda/D],
    x_m = (m - n_in//2) / n_d  [D].  The index product is an exact integer."""
    p = np.outer(centred(m_out), centred(n_in))
    turns = p * (float(du) / float(n_d))
    turns = turns - np.round(turns)
    return np.exp(-2j * np.pi * turns)


def mft(e, n_d, m_out, du):
    """E_B = (du / n_d) W E W^T: n_in x n_in pupil field -> m_out x m_out focal field."""
    e = np.asarray(e, dtype=np.complex128)
    w = mft_matrix(m_out, e.shape[0], n_d, du)
    return (float(du) / float(n_d)) * (w @ e @ w.T)


def mft_adjoint(eb, n_d, n_out, du):
    """Exact adjoint of mft: E_A = (du / n_d) W^H E_B conj(W), focal m x m -> pupil n_out x n_out."""
    eb = np.asarray(eb, dtype=np.complex128)
    w = mft_matrix(eb.shape[0], n_out, n_d, du)
    return (float(du) / float(n_d)) * (w.conj().T @ eb @ w.conj())


# --------------------------------------------------------------------------------------------
# O9. Direct (single-transform) Fresnel step (Sec. 1.1: POPPY's direct Fresnel method beside
#     the angular spectrum; Sec. 2.3, Eq. 2: the quadratic phase factor, read as
#     exp(+i pi (x^2 + y^2) / (lambda z)) since the printed form drops pi / lambda and its sign).
# --------------------------------------------------------------------------------------------

def direct_pitch(n, dx, wavelength, z):
    """Output pixel pitch of the direct step: lambda |z| / (n dx)."""
    return float(wavelength) * abs(float(z)) / (n * float(dx))


def quadratic_phase(n, pitch, wavelength, z):
    """q(i) = exp(+i pi (c(i) pitch)^2 / (lambda z)); the integer c(i)^2 is exact and the phase
    is taken in turns in float64, reduced before the exponential."""
    c = centred(n)
    turns = (c * c) * (float(pitch) ** 2 / (2.0 * float(wavelength) * float(z)))
    turns = turns - np.round(turns)
    return np.exp(2j * np.pi * turns)


def direct_kernel_matrix(n, sign=1):
    """F[k, i] = exp(-2 pi i sign c(k) c(i) / n): the Fresnel transform kernel exp(-2 pi i x u /
    (lambda z)) between the centred input grid x = c(i) dx and the centred output grid
    u = c(k) lambda |z| / (n dx); sign = the sign of z."""
    p = np.outer(centred(n), centred(n)) % n      # exact integer index reduction
    return np.exp((-2j * np.pi * (1 if sign > 0 else -1) / n) * p)


def direct_fresnel(u, dx, wavelength, z):
    """The Fresnel integral over a distance z > 0 evaluated with one transform:

        U2(u, v) = dx^2 / (i lambda z) q2(u) q2(v) sum_{x, y} U1(x, y) q1(x) q1(y)
                   exp(-2 pi i (x u + y v) / (lambda z)),

    input pitch dx, output pitch dx2 = lambda |z| / (n dx), q1 / q2 the quadratic phase on the
    input / output grid, z of either sign (z < 0: towards the source; then the kernel's sign
    flips with z). No e^{ikz} piston (as for the angular-spectrum step).
    Returns (U2, dx2)."""
    if not float(z) != 0.0:
        raise ValueError("the direct step takes z != 0")
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[0]
    if u.shape != (n, n):
        raise ValueError("square arrays only")
    dx2 = direct_pitch(n, dx, wavelength, z)
    q1 = quadratic_phase(n, dx, wavelength, z)
    q2 = quadratic_phase(n, dx2, wavelength, z)
    f = direct_kernel_matrix(n, np.sign(z))
    c = float(dx) ** 2 / (1j * float(wavelength) * float(z))
    inner = (q1[:, None] * u * q1[None, :])
    return c * (q2[:, None] * (f @ inner @ f.T) * q2[None, :]), dx2


def direct_fresnel_rows(u, dx, wavelength, z, rows):
    """Rows `rows` of direct_fresnel(u, dx, wavelength, z)[0], at O(len(rows) n^2) cost (the
    kernel matrix's rows, not the whole matrix)."""
    u = np.asarray(u, dtype=np.complex128)
    n = u.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    dx2 = direct_pitch(n, dx, wavelength, z)
    q1 = quadratic_phase(n, dx, wavelength, z)
    q2 = quadratic_phase(n, dx2, wavelength, z)
    c = float(dx) ** 2 / (1j * float(wavelength) * float(z))
    sgn = 1 if float(z) > 0 else -1
    fr = np.exp((-2j * np.pi * sgn / n) * (np.outer(centred(n)[rows], centred(n)) % n))   # len(rows) x n
    f = direct_kernel_matrix(n, sgn)
    inner = (q1[:, None] * u * q1[None, :])
    return c * (q2[rows][:, None] * ((fr @ inner) @ f.T) * q2[None, :])


def direct_fresnel_adjoint(v, dx, wavelength, z):
    """Exact adjoint of direct_fresnel over the same (dx, wavelength, z): from the output grid
    (pitch lambda z / (n dx)) back to the input grid,

        U1(x, y) = conj(dx^2 / (i lambda z)) conj(q1(x) q1(y)) sum_{u, v} V(u, v) conj(q2(u) q2(v))
                   exp(+2 pi i (x u + y v) / (lambda z)),

    so that <direct_fresnel(u), v> = <u, direct_fresnel_adjoint(v)>. Scaled by (dx2 / dx)^2 it
    is the inverse step (the forward one is unitary up to the pitch change)."""
    if not float(z) != 0.0:
        raise ValueError("the direct step takes z != 0")
    v = np.asarray(v, dtype=np.complex128)
    n = v.shape[0]
    if v.shape != (n, n):
        raise ValueError("square arrays only")
    dx2 = direct_pitch(n, dx, wavelength, z)
    q1 = quadratic_phase(n, dx, wavelength, z)
    q2 = quadratic_phase(n, dx2, wavelength, z)
    fh = direct_kernel_matrix(n, np.sign(z)).conj()   # the kernel matrix is symmetric: F^H = conj(F)
    c = float(dx) ** 2 / (1j * float(wavelength) * float(z))
    inner = q2.conj()[:, None] * v * q2.conj()[None, :]
    return np.conj(c) * (q1.conj()[:, None] * (fh @ inner @ fh.T) * q1.conj()[None, :])


# --------------------------------------------------------------------------------------------
# O10. Angular-spectrum step with the exact (non-paraxial) transfer function (Sec. 1.1: the
#      angular-spectrum method after Lawrence, here without the paraxial approximation).
# --------------------------------------------------------------------------------------------

def transfer_function_exact(n, dx, wavelength, z):
    """H[ky, kx] = exp(2 pi i z (sqrt(1/lambda^2 - f^2) - 1/lambda)) for f^2 = fx^2 + fy^2 below
    1/lambda^2 (the piston exp(2 pi i z / lambda) left out, as for the paraxial form, which is
    this phase to second order in lambda f); evanescent components (f^2 > 1/lambda^2) decay as
    exp(-2 pi |z| sqrt(f^2 - 1/lambda^2)) in either direction. The phase is taken in turns as
    -z f^2 / (sqrt(1/lambda^2 - f^2) + 1/lambda) (no cancellation) and reduced before the
    exponential."""
    k = signed_index(n)
    lam = float(wavelength)
    f2 = (k[:, None] ** 2 + k[None, :] ** 2).astype(np.float64) / (n * float(dx)) ** 2
    inv2 = 1.0 / (lam * lam)
    prop = f2 < inv2
    root = np.sqrt(np.where(prop, inv2 - f2, 0.0))
    turns = np.where(prop, -float(z) * f2 / (root + 1.0 / lam), 0.0)
    turns = turns - np.round(turns)
    decay = np.where(prop, 1.0, np.exp(-2.0 * np.pi * abs(float(z)) * np.sqrt(np.where(prop, 0.0, f2 - inv2))))
    # the piston is left out of the evanescent part too
    piston = np.where(prop, 1.0, np.exp(-2j * np.pi * ((float(z) / lam) - np.round(float(z) / lam))))
    return np.where(prop, np.exp(2j * np.pi * turns), decay * piston)


def as_propagate_exact(u, dx, wavelength, z):
    """U(z) = IDFT2( H_exact . DFT2(U) ): one angular-spectrum step with the exact transfer
    function."""
    n = u.shape[0]
    return idft2(transfer_function_exact(n, dx, wavelength, z) * dft2(np.asarray(u, dtype=np.complex128)))
