"""Seeded synthetic Darcy-flow systems (input generation only).

The paper's Darcy dataset (App. D.2, "Darcy Flow") solves -div(K grad h) = f with a
permeability K drawn from a Gaussian random field, and sorts the systems on the GRF
parameters (Alg. 1). That dataset is not available, so this module stands in for it:

* GRF: i.i.d. N(0,1) noise on an M x M periodic lattice (M = N_g + 2, the full node grid
  including the Dirichlet boundary), filtered in Fourier space by the square root of the
  spectral density S(kappa) = (tau^2 + |kappa|^2)^-2, tau = 3, kappa = 2*pi*(integer FFT
  frequency), then scaled so that the field has unit variance. The permeability is
  a = exp(theta) at the nodes. System i draws its noise from
  ``numpy.random.default_rng([2401, i])``.
* Discretisation: -div(a grad u) = 1 on the unit square with u = 0 on the boundary, 5-point
  finite differences on the N_g x N_g interior grid, h = 1/(N_g + 1), unknown (i, j) at index
  (i-1)*N_g + (j-1) (row-major, as in the paper's worked FDM example, Sec. 3.1 and App. A).
  The coefficient on the face between nodes P and Q is the harmonic mean 2 a_P a_Q/(a_P + a_Q).
  Row (i, j): diagonal = sum of its four face coefficients / h^2, off-diagonal = -face / h^2 for
  each interior neighbour. With a == 1 this is -(1/h^2) times the paper's Poisson example matrix.

Nothing here is part of the method (sort or solver): the outputs are plain inputs handed to both
the oracle and the GPU library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

GRF_TAU = 3.0
SEED_ROOT = 2401


def grf_field(M: int, seed: int, tau: float = GRF_TAU) -> np.ndarray:
    """Unit-variance periodic Gaussian random field on an M x M lattice (float64)."""
    rng = np.random.default_rng([SEED_ROOT, int(seed)])
    xi = rng.standard_normal((M, M))
    kf = 2.0 * np.pi * np.fft.fftfreq(M, d=1.0 / M)
    k2 = kf[:, None] ** 2 + kf[None, :] ** 2
    S = (tau * tau + k2) ** -2.0
    theta = np.real(np.fft.ifft2(np.sqrt(S) * np.fft.fft2(xi)))
    theta /= np.sqrt(S.mean())
    return theta


def permeability(N_g: int, seed: int, tau: float = GRF_TAU) -> np.ndarray:
    """a = exp(GRF) on the (N_g+2) x (N_g+2) node grid (boundary nodes included)."""
    return np.exp(grf_field(N_g + 2, seed, tau))


def _harmonic(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    return 2.0 * p * q / (p + q)


@dataclass
class DarcySystem:
    """One assembled system. ``A`` is CSR (int32 indices, float64 values)."""

    N_g: int
    a: np.ndarray          # (N_g+2, N_g+2) node permeability: the sort key (parameter matrix)
    ax: np.ndarray         # (N_g, N_g+1) x-direction face coefficients, ax[i-1, j] between (i,j),(i,j+1)
    ay: np.ndarray         # (N_g+1, N_g) y-direction face coefficients, ay[i, j-1] between (i,j),(i+1,j)
    inv_h2: float
    A: sp.csr_matrix
    b: np.ndarray

    @property
    def n(self) -> int:
        return self.N_g * self.N_g


def faces_from_nodes(a: np.ndarray):
    """Harmonic-mean face coefficients for the interior unknowns of node field ``a``."""
    N_g = a.shape[0] - 2
    inner = a[1:N_g + 1, :]                      # rows i = 1..N_g, all columns
    ax = _harmonic(inner[:, :-1], inner[:, 1:])  # (N_g, N_g+1)
    cols = a[:, 1:N_g + 1]                       # all rows, columns j = 1..N_g
    ay = _harmonic(cols[:-1, :], cols[1:, :])    # (N_g+1, N_g)
    return ax, ay


def assemble_csr(ax: np.ndarray, ay: np.ndarray, inv_h2: float) -> sp.csr_matrix:
    """5-point CSR matrix with sorted column indices from the face arrays."""
    N_g = ax.shape[0]
    n = N_g * N_g
    idx = np.arange(n).reshape(N_g, N_g)
    west = ax[:, :-1]
    east = ax[:, 1:]
    north = ay[:-1, :]
    south = ay[1:, :]
    diag = (west + east + north + south) * inv_h2
    rows = [idx.ravel()]
    colsl = [idx.ravel()]
    vals = [diag.ravel()]
    # west neighbour (i, j-1)
    rows.append(idx[:, 1:].ravel()); colsl.append(idx[:, :-1].ravel()); vals.append((-west[:, 1:] * inv_h2).ravel())
    # east neighbour (i, j+1)
    rows.append(idx[:, :-1].ravel()); colsl.append(idx[:, 1:].ravel()); vals.append((-east[:, :-1] * inv_h2).ravel())
    # north neighbour (i-1, j)
    rows.append(idx[1:, :].ravel()); colsl.append(idx[:-1, :].ravel()); vals.append((-north[1:, :] * inv_h2).ravel())
    # south neighbour (i+1, j)
    rows.append(idx[:-1, :].ravel()); colsl.append(idx[1:, :].ravel()); vals.append((-south[:-1, :] * inv_h2).ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(colsl))), shape=(n, n)).tocsr()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def darcy_from_nodes(a: np.ndarray) -> DarcySystem:
    N_g = a.shape[0] - 2
    h = 1.0 / (N_g + 1)
    inv_h2 = 1.0 / (h * h)
    ax, ay = faces_from_nodes(a)
    A = assemble_csr(ax, ay, inv_h2)
    b = np.ones(N_g * N_g)
    return DarcySystem(N_g=N_g, a=a, ax=ax, ay=ay, inv_h2=inv_h2, A=A, b=b)


def darcy_system(N_g: int, seed: int) -> DarcySystem:
    return darcy_from_nodes(permeability(N_g, seed))


def darcy_sequence(N_g: int, count: int, first_seed: int = 0) -> list[DarcySystem]:
    """``count`` systems with seeds first_seed .. first_seed+count-1."""
    return [darcy_system(N_g, first_seed + i) for i in range(count)]


def param_matrix(systems) -> np.ndarray:
    """Row-major (N, p) float64 sort keys: each row is vec(a_i) over the full node grid."""
    return np.ascontiguousarray(np.stack([s.a.ravel() for s in systems]))
