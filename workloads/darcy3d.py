"""Seeded synthetic 3-D variable-coefficient Poisson (Darcy) systems (input generation only).

The 3-D counterpart of ``workloads.darcy``: -div(a grad u) = 1 on the unit cube with u = 0 on the
boundary, 7-point finite differences on the N x N x N interior grid, h = 1/(N + 1), unknown
(x, y, z) (1-based interior node coordinates) at index (x-1) + N*((y-1) + N*(z-1)). The coefficient
on the face between nodes P and Q is the harmonic mean 2 a_P a_Q/(a_P + a_Q), and a = exp(theta)
with theta a unit-variance Gaussian random field on the (N+2)^3 periodic node lattice, filtered by
the square root of S(kappa) = (tau^2 + |kappa|^2)^-2, tau = 3 (the 2-D spectral density carried
over to 3-D). System i draws its noise from ``numpy.random.default_rng([2401, 3, i])``.

Face arrays (C order, matching the 7-point operator of the C ABI):
  ax[z, y, f]: face between x-nodes f and f+1 (f = 0..N), shape (N, N, N+1)
  ay[z, f, x]: face between y-nodes f and f+1, shape (N, N+1, N)
  az[f, y, x]: face between z-nodes f and f+1, shape (N+1, N, N)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

GRF_TAU = 3.0
SEED_ROOT = 2401


def grf_field3d(M: int, seed: int, tau: float = GRF_TAU) -> np.ndarray:
    """Unit-variance periodic Gaussian random field on an M x M x M lattice (float64)."""
    rng = np.random.default_rng([SEED_ROOT, 3, int(seed)])
    xi = rng.standard_normal((M, M, M))
    kf = 2.0 * np.pi * np.fft.fftfreq(M, d=1.0 / M)
    k2 = kf[:, None, None] ** 2 + kf[None, :, None] ** 2 + kf[None, None, :] ** 2
    S = (tau * tau + k2) ** -2.0
    theta = np.real(np.fft.ifftn(np.sqrt(S) * np.fft.fftn(xi)))
    theta /= np.sqrt(S.mean())
    return theta


def _harmonic(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    return 2.0 * p * q / (p + q)


@dataclass
class Darcy3DSystem:
    """One assembled 3-D system. ``A`` is CSR (int32 indices, float64 values)."""

    N: int
    a: np.ndarray          # (N+2)^3 node permeability: the sort key
    ax: np.ndarray
    ay: np.ndarray
    az: np.ndarray
    inv_h2: float
    A: sp.csr_matrix
    b: np.ndarray

    @property
    def n(self) -> int:
        return self.N ** 3


def faces3d_from_nodes(a: np.ndarray):
    """Harmonic-mean face coefficients for the interior unknowns of node field ``a`` ((N+2)^3)."""
    N = a.shape[0] - 2
    I = slice(1, N + 1)
    ax = _harmonic(a[I, I, :-1], a[I, I, 1:])     # (N, N, N+1)
    ay = _harmonic(a[I, :-1, I], a[I, 1:, I])     # (N, N+1, N)
    az = _harmonic(a[:-1, I, I], a[1:, I, I])     # (N+1, N, N)
    return ax, ay, az


def assemble_csr3d(ax: np.ndarray, ay: np.ndarray, az: np.ndarray, inv_h2: float) -> sp.csr_matrix:
    """7-point CSR matrix with sorted column indices from the face arrays."""
    N = ax.shape[0]
    n = N ** 3
    idx = np.arange(n).reshape(N, N, N)           # [z, y, x]
    diag = (ax[:, :, :-1] + ax[:, :, 1:] + ay[:, :-1, :] + ay[:, 1:, :] + az[:-1, :, :] + az[1:, :, :]) * inv_h2
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [diag.ravel()]
    fx, fy, fz = ax[:, :, 1:N], ay[:, 1:N, :], az[1:N, :, :]   # interior faces
    for (ra, ca, f) in ((idx[:, :, 1:], idx[:, :, :-1], fx), (idx[:, :, :-1], idx[:, :, 1:], fx),
                        (idx[:, 1:, :], idx[:, :-1, :], fy), (idx[:, :-1, :], idx[:, 1:, :], fy),
                        (idx[1:, :, :], idx[:-1, :, :], fz), (idx[:-1, :, :], idx[1:, :, :], fz)):
        rows.append(ra.ravel())
        cols.append(ca.ravel())
        vals.append((-f * inv_h2).ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def darcy3d_from_nodes(a: np.ndarray, with_csr: bool = True) -> Darcy3DSystem:
    N = a.shape[0] - 2
    h = 1.0 / (N + 1)
    inv_h2 = 1.0 / (h * h)
    ax, ay, az = faces3d_from_nodes(a)
    A = assemble_csr3d(ax, ay, az, inv_h2) if with_csr else None
    return Darcy3DSystem(N=N, a=a, ax=ax, ay=ay, az=az, inv_h2=inv_h2, A=A, b=np.ones(N ** 3))


def darcy3d_system(N: int, seed: int, with_csr: bool = True) -> Darcy3DSystem:
    return darcy3d_from_nodes(np.exp(grf_field3d(N + 2, seed)), with_csr)


def darcy3d_sequence(N: int, count: int, first_seed: int = 0, with_csr: bool = True) -> list:
    return [darcy3d_system(N, first_seed + i, with_csr) for i in range(count)]
