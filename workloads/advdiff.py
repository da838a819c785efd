"""Seeded nonsymmetric systems: 2-D unsteady advection-diffusion, backward Euler, upwind.

(I/dt - nu Lap_h + b . grad_h) u = rhs on the N x N interior grid of the unit square, zero Dirichlet
data, h = 1/(N+1), unknown (i, j) at index i*N + j. Lap_h is the 5-point Laplacian; the advection
term uses first-order upwinding of the velocity b = (bx, by) sampled at the nodes. The velocity is
the divergence-free field b = curl(psi) of a seeded smooth stream function psi (a few low Fourier
modes). Input generation only: nothing of the solver lives here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SEED_ROOT = 2401


def stream_velocity(N: int, seed: int, amp: float = 1.0):
    """Velocity (bx, by) = (d psi/dy, -d psi/dx) at the N x N interior nodes, psi = sum of seeded modes."""
    rng = np.random.default_rng([SEED_ROOT, 7, int(seed)])
    h = 1.0 / (N + 1)
    x = h * np.arange(1, N + 1)
    X, Y = np.meshgrid(x, x, indexing="xy")          # X varies along j (columns), Y along i (rows)
    bx = np.zeros((N, N))
    by = np.zeros((N, N))
    for kx in range(1, 4):
        for ky in range(1, 4):
            c = rng.standard_normal() / (kx * kx + ky * ky)
            # psi = c sin(pi kx X) sin(pi ky Y)
            bx += c * np.pi * ky * np.sin(np.pi * kx * X) * np.cos(np.pi * ky * Y)
            by += -c * np.pi * kx * np.cos(np.pi * kx * X) * np.sin(np.pi * ky * Y)
    scale = amp / max(np.abs(bx).max(), np.abs(by).max(), 1e-300)
    return bx * scale, by * scale


def advdiff_matrix(N: int, nu: float, bx: np.ndarray, by: np.ndarray, dt: float) -> sp.csr_matrix:
    """CSR matrix of I/dt - nu Lap_h + upwind(b . grad_h) (int32 indices, sorted columns)."""
    h = 1.0 / (N + 1)
    n = N * N
    idx = np.arange(n).reshape(N, N)
    bxp, bxm = np.maximum(bx, 0.0), np.minimum(bx, 0.0)
    byp, bym = np.maximum(by, 0.0), np.minimum(by, 0.0)
    diag = 1.0 / dt + 4.0 * nu / (h * h) + (bxp - bxm + byp - bym) / h
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [diag.ravel()]
    # west (j-1): -nu/h^2 - bx+/h ; east (j+1): -nu/h^2 + bx-/h ; south (i-1), north (i+1) likewise with by
    for di, dj, coef in ((0, -1, -nu / h ** 2 - bxp / h), (0, 1, -nu / h ** 2 + bxm / h),
                         (-1, 0, -nu / h ** 2 - byp / h), (1, 0, -nu / h ** 2 + bym / h)):
        i0, i1 = max(0, -di), N - max(0, di)
        j0, j1 = max(0, -dj), N - max(0, dj)
        src = idx[i0:i1, j0:j1]
        dst = idx[i0 + di:i1 + di, j0 + dj:j1 + dj]
        c = coef if np.isscalar(coef) else coef[i0:i1, j0:j1]
        rows.append(src.ravel()); cols.append(dst.ravel()); vals.append(np.broadcast_to(c, src.shape).ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


class AdvDiffSystem:
    def __init__(self, N, nu, seed, dt=1e-2, amp=1.0):
        self.N_g = N
        self.nu = nu
        self.bx, self.by = stream_velocity(N, seed, amp)
        self.A = advdiff_matrix(N, nu, self.bx, self.by, dt)
        x = (np.arange(1, N + 1) / (N + 1))
        X, Y = np.meshgrid(x, x, indexing="xy")
        self.b = (np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel() / dt   # x^t / dt with a smooth x^t

    @property
    def n(self):
        return self.N_g * self.N_g


def advdiff_sequence(N: int, count: int, first_seed: int = 0, dt: float = 1e-2, amp: float = 1.0):
    """``count`` systems with nu ~ U[1e-3, 1e-2] and a velocity field per seed."""
    out = []
    for s in range(first_seed, first_seed + count):
        nu = 1e-3 + 9e-3 * np.random.default_rng([SEED_ROOT, 8, s]).random()
        out.append(AdvDiffSystem(N, nu, s, dt, amp))
    return out


class AdvDiffChain:
    """One time-stepping chain: a fixed operator A = I/dt - nu Lap_h + upwind(b . grad_h) with its own
    nu ~ U[1e-3, 1e-2] and seeded divergence-free velocity b = curl(psi), and a seeded smooth initial
    state x0 (a few low sine modes). Its systems are the backward-Euler steps A x^{t+1} = x^t / dt, so
    the right-hand side of step t + 1 is the solution of step t divided by dt.

    ``params`` identifies the operator (nu, then the two velocity components at the nodes): the
    vector a chain's systems are admitted by.
    """

    def __init__(self, N: int, seed: int, dt: float = 1e-2, amp: float = 1.0):
        self.N_g = N
        self.dt = dt
        self.nu = 1e-3 + 9e-3 * np.random.default_rng([SEED_ROOT, 9, int(seed)]).random()
        self.bx, self.by = stream_velocity(N, 10_000 + int(seed), amp)
        self.A = advdiff_matrix(N, self.nu, self.bx, self.by, dt)
        rng = np.random.default_rng([SEED_ROOT, 10, int(seed)])
        x = np.arange(1, N + 1) / (N + 1)
        X, Y = np.meshgrid(x, x, indexing="xy")
        x0 = np.zeros((N, N))
        for kx in range(1, 4):
            for ky in range(1, 4):
                x0 += rng.standard_normal() / (kx * ky) * np.sin(np.pi * kx * X) * np.sin(np.pi * ky * Y)
        self.x0 = x0.ravel()
        self.b = self.x0 / dt             # right-hand side of the first step
        self.params = np.concatenate([[self.nu], self.bx.ravel(), self.by.ravel()])

    @property
    def n(self):
        return self.N_g * self.N_g


def advdiff_chains(N: int, count: int, first_seed: int = 0, dt: float = 1e-2, amp: float = 1.0):
    """``count`` independent time-stepping chains on an N x N grid."""
    return [AdvDiffChain(N, s, dt, amp) for s in range(first_seed, first_seed + count)]

