"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no lattice-Boltzmann arithmetic: it produces velocity, density-fluctuation
and force fields (and plain random arrays) on a grid. Both the FP64 oracle and the HIP
library build their populations from these fields with their own code.

Every field has shape (3, nz, ny, nx) (x fastest) for vectors and (nz, ny, nx) for scalars;
velocity gradients have shape (3, 3, nz, ny, nx) with grad[a, b] = d u_b / d x_a. All
arrays are float64 and C-contiguous.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0  # lattice equation of state p = c_s^2 delta_rho used to turn p into delta_rho


def coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))


def tgv_rotated(shape, u0: float = 0.05, rho0: float = 1.0, plane=(0, 1)):
    """Taylor-Green vortex turned by 45 degrees, at t = 0.

    u_a = u0 sin(k x_b), u_b = u0 sin(k x_a), p = rho0 u0^2 cos(k x_a) cos(k x_b),
    k = 2 pi / N along the plane's axes (both must have N nodes).
    Returns (delta_rho, u, grad_u).
    """
    a, b = plane
    X = coords(shape)
    N = shape[2 - a]
    assert shape[2 - b] == N
    k = 2.0 * np.pi / N
    u = np.zeros((3,) + tuple(shape))
    u[a] = u0 * np.sin(k * X[b])
    u[b] = u0 * np.sin(k * X[a])
    p = rho0 * u0 * u0 * np.cos(k * X[a]) * np.cos(k * X[b])
    grad = np.zeros((3, 3) + tuple(shape))
    grad[b, a] = u0 * k * np.cos(k * X[b])   # d u_a / d x_b
    grad[a, b] = u0 * k * np.cos(k * X[a])   # d u_b / d x_a
    return p / CS2, u, grad


def tgv_axis(shape, u0: float = 0.05, rho0: float = 1.0, plane=(0, 1)):
    """Axis-aligned Taylor-Green vortex at t = 0.

    u_a = u0 sin(k x_a) cos(k x_b), u_b = -u0 cos(k x_a) sin(k x_b),
    p = rho0 u0^2 / 4 (cos 2k x_a + cos 2k x_b). Returns (delta_rho, u, grad_u).
    """
    a, b = plane
    X = coords(shape)
    N = shape[2 - a]
    assert shape[2 - b] == N
    k = 2.0 * np.pi / N
    sa, ca = np.sin(k * X[a]), np.cos(k * X[a])
    sb, cb = np.sin(k * X[b]), np.cos(k * X[b])
    u = np.zeros((3,) + tuple(shape))
    u[a] = u0 * sa * cb
    u[b] = -u0 * ca * sb
    p = 0.25 * rho0 * u0 * u0 * (np.cos(2 * k * X[a]) + np.cos(2 * k * X[b]))
    grad = np.zeros((3, 3) + tuple(shape))
    grad[a, a] = u0 * k * ca * cb
    grad[b, a] = -u0 * k * sa * sb
    grad[a, b] = u0 * k * sa * sb
    grad[b, b] = -u0 * k * ca * cb
    return p / CS2, u, grad


def spectrum_velocity(shape, seed: int = 1704, u_rms: float = 0.04, k0: float = 4.0) -> np.ndarray:
    """Random solenoidal velocity with energy spectrum E(k) ~ k^4 exp(-2 (k/k0)^2).

    Gaussian white noise (3 components) -> FFT -> projection onto divergence-free modes
    (I - k k / |k|^2) -> amplitude sqrt(E(k) / (4 pi k^2)) with k the integer wavenumber
    magnitude; the k = 0 and Nyquist modes are zeroed -> inverse FFT -> scaled so that
    sqrt(<u.u>/3) = u_rms.
    """
    import scipy.fft as sfft

    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3,) + tuple(shape))
    uh = sfft.fftn(noise, axes=(1, 2, 3), workers=-1)
    del noise
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    K = np.stack([KX, KY, KZ])
    k2 = (K * K).sum(axis=0)
    kmag = np.sqrt(k2)
    safe = np.where(k2 > 0, k2, 1.0)
    kdotu = (K * uh).sum(axis=0)
    uh = uh - K * kdotu[None] / safe[None]
    E = kmag**4 * np.exp(-2.0 * (kmag / k0) ** 2)
    amp = np.sqrt(E / (4.0 * np.pi * np.where(k2 > 0, k2, 1.0)))
    amp[k2 == 0] = 0.0
    nyq = np.zeros_like(amp, dtype=bool)
    if nx % 2 == 0:
        nyq |= np.abs(KX) == nx // 2
    if ny % 2 == 0:
        nyq |= np.abs(KY) == ny // 2
    if nz % 2 == 0:
        nyq |= np.abs(KZ) == nz // 2
    amp[nyq] = 0.0
    uh *= amp[None]
    del amp, K, KX, KY, KZ, k2, kmag, safe, kdotu, E, nyq
    u = np.real(sfft.ifftn(uh, axes=(1, 2, 3), workers=-1))
    del uh
    rms = np.sqrt((u * u).sum(axis=0).mean() / 3.0)
    return np.ascontiguousarray(u * (u_rms / rms))


def uniform_random_force(shape, seed: int = 7559, amp: float = 1e-6) -> np.ndarray:
    """Body-force field with i.i.d. components drawn from U(-amp, amp)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(3,) + tuple(shape))


def random_state(q: int, shape, seed: int = 0, scale: float = 0.01, mean=None) -> np.ndarray:
    """Plain random array of shape (q, nz, ny, nx): mean + scale * N(0, 1).

    ``mean`` (length q) lets a caller centre each population; it carries no physics here.
    """
    rng = np.random.default_rng(seed)
    a = scale * rng.standard_normal((q,) + tuple(shape))
    if mean is not None:
        a = a + np.asarray(mean, dtype=np.float64).reshape((q,) + (1,) * len(shape))
    return a


def random_vector(shape, seed: int = 0, scale: float = 0.01) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((3,) + tuple(shape))
