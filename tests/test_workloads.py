"""Input generators: the FDM assembly pinned to the paper's worked example, and structural checks."""
import os

import numpy as np

from workloads import darcy_from_nodes, darcy_sequence, grf_field, param_matrix


def _load_golden(path):
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return np.array(rows, dtype=np.float64)


def test_fdm_matches_paper_2x2_example(golden_dir):
    # a == 1, N_g = 2: -div(grad u) discretised; the paper prints Delta x^2 * (nabla^2 operator).
    M_paper = _load_golden(os.path.join(golden_dir, "fdm_poisson_2x2.txt"))
    sysm = darcy_from_nodes(np.ones((4, 4)))
    h = 1.0 / 3.0
    A = sysm.A.toarray()
    np.testing.assert_allclose(A, -(1.0 / h ** 2) * M_paper, rtol=1e-14, atol=0)


def test_structure_and_symmetry():
    for N_g in (1, 2, 7, 32):
        s = darcy_sequence(N_g, 1, first_seed=3)[0]
        A = s.A
        assert A.shape == (N_g * N_g, N_g * N_g)
        assert A.nnz == 5 * N_g * N_g - 4 * N_g
        assert A.indptr.dtype == np.int32 and A.indices.dtype == np.int32
        assert abs(A - A.T).max() == 0.0
        d = A.diagonal()
        off = np.asarray(abs(A).sum(axis=1)).ravel() - d
        assert np.all(d >= off * (1 - 1e-15))           # weak diagonal dominance
        assert np.all(d > 0)


def test_faces_reproduce_csr():
    s = darcy_sequence(9, 1, first_seed=5)[0]
    N_g = s.N_g
    x = np.random.default_rng(0).standard_normal((N_g, N_g))
    xp = np.zeros((N_g + 2, N_g + 2))
    xp[1:-1, 1:-1] = x
    ax, ay = s.ax, s.ay
    y = (ax[:, :-1] * (x - xp[1:-1, :-2]) + ax[:, 1:] * (x - xp[1:-1, 2:])
         + ay[:-1, :] * (x - xp[:-2, 1:-1]) + ay[1:, :] * (x - xp[2:, 1:-1])) * s.inv_h2
    np.testing.assert_allclose(y.ravel(), s.A @ x.ravel(), rtol=1e-12, atol=1e-9 * s.inv_h2)


def test_grf_is_seeded_and_unit_variance():
    f1 = grf_field(66, 7)
    f2 = grf_field(66, 7)
    assert np.array_equal(f1, f2)
    assert not np.array_equal(f1, grf_field(66, 8))
    v = np.mean([grf_field(34, s).var() + grf_field(34, s).mean() ** 2 for s in range(200)])
    assert 0.8 < v < 1.2


def test_param_matrix_layout():
    seq = darcy_sequence(4, 3)
    P = param_matrix(seq)
    assert P.shape == (3, 36) and P.flags.c_contiguous
    assert np.array_equal(P[1], seq[1].a.ravel())


def test_advdiff_operator():
    from workloads.advdiff import advdiff_matrix, advdiff_sequence, stream_velocity
    Nf = 64
    hf = 1.0 / (Nf + 1)
    bxf, byf = stream_velocity(Nf, 3)
    # the sampled velocity of a stream function is divergence-free up to the O(h^2) difference error
    dbx = np.gradient(bxf, hf, axis=1)
    div = dbx + np.gradient(byf, hf, axis=0)
    assert np.abs(div[2:-2, 2:-2]).max() < 0.02 * np.abs(dbx).max()
    N = 9
    h = 1.0 / (N + 1)
    bx, by = stream_velocity(N, 3)
    A = advdiff_matrix(N, 0.01, bx, by, 1e-2).toarray()
    # constant velocity check against a hand-built upwind row
    A2 = advdiff_matrix(N, 0.5, np.full((N, N), 2.0), np.full((N, N), -1.0), 0.1).toarray()
    r = 4 * N + 4
    assert np.isclose(A2[r, r], 10 + 2.0 / h ** 2 + 3.0 / h)
    assert np.isclose(A2[r, r - 1], -0.5 / h ** 2 - 2.0 / h)       # west, bx > 0 upwind
    assert np.isclose(A2[r, r + 1], -0.5 / h ** 2)                 # east
    assert np.isclose(A2[r, r + N], -0.5 / h ** 2 - 1.0 / h)       # north, by < 0 upwind
    assert np.isclose(A2[r, r - N], -0.5 / h ** 2)                 # south
    assert not np.allclose(A, A.T)
    seq = advdiff_sequence(6, 3)
    assert all(1e-3 <= s.nu <= 1e-2 for s in seq) and seq[0].A.shape == (36, 36)


def test_advdiff_time_stepping_chains():
    from workloads.advdiff import advdiff_chains
    ch = advdiff_chains(12, 3, first_seed=5, dt=1e-2)
    again = advdiff_chains(12, 3, first_seed=5, dt=1e-2)
    N, n = 12, 144
    interior = np.array([i * N + j for i in range(1, N - 1) for j in range(1, N - 1)])
    for c, d in zip(ch, again):
        assert 1e-3 <= c.nu <= 1e-2
        assert np.array_equal(c.params, d.params) and np.array_equal(c.x0, d.x0)    # seeded
        assert c.params.shape == (1 + 2 * n,) and c.params[0] == c.nu
        # upwind advection and the Laplacian cancel in the row sums of interior rows: 1/dt
        assert np.allclose(np.asarray(c.A.sum(axis=1)).ravel()[interior], 1.0 / c.dt, rtol=1e-12)
        assert not np.allclose(c.A.toarray(), c.A.toarray().T)
    assert len({c.nu for c in ch}) == 3


def test_3d_structure_and_symmetry():
    from workloads import darcy3d_sequence
    for N in (1, 2, 5):
        s = darcy3d_sequence(N, 1, first_seed=4)[0]
        A = s.A
        assert A.shape == (N ** 3, N ** 3)
        assert A.nnz == 7 * N ** 3 - 6 * N ** 2
        assert A.indptr.dtype == np.int32 and A.indices.dtype == np.int32
        assert abs(A - A.T).max() == 0.0
        d = A.diagonal()
        off = np.asarray(abs(A).sum(axis=1)).ravel() - d
        assert np.all(d >= off * (1 - 1e-15)) and np.all(d > 0)
        assert s.ax.shape == (N, N, N + 1) and s.ay.shape == (N, N + 1, N) and s.az.shape == (N + 1, N, N)


def test_3d_faces_reproduce_csr():
    from workloads import darcy3d_sequence
    s = darcy3d_sequence(6, 1, first_seed=2)[0]
    N = s.N
    x = np.random.default_rng(1).standard_normal((N, N, N))        # [z, y, x]
    xp = np.zeros((N + 2, N + 2, N + 2))
    xp[1:-1, 1:-1, 1:-1] = x
    c = xp[1:-1, 1:-1, 1:-1]
    y = (s.ax[:, :, :-1] * (c - xp[1:-1, 1:-1, :-2]) + s.ax[:, :, 1:] * (c - xp[1:-1, 1:-1, 2:])
         + s.ay[:, :-1, :] * (c - xp[1:-1, :-2, 1:-1]) + s.ay[:, 1:, :] * (c - xp[1:-1, 2:, 1:-1])
         + s.az[:-1, :, :] * (c - xp[:-2, 1:-1, 1:-1]) + s.az[1:, :, :] * (c - xp[2:, 1:-1, 1:-1])) * s.inv_h2
    np.testing.assert_allclose(y.ravel(), s.A @ x.ravel(), rtol=1e-12, atol=1e-9 * s.inv_h2)


def test_3d_constant_coefficient_closed_form():
    # a == 1: the 7-point Dirichlet Laplacian, whose eigenvalues are
    # (4/h^2) (sin^2(p pi h/2) + sin^2(q pi h/2) + sin^2(r pi h/2)), p, q, r = 1..N
    from workloads.darcy3d import darcy3d_from_nodes
    N = 5
    h = 1.0 / (N + 1)
    A = darcy3d_from_nodes(np.ones((N + 2, N + 2, N + 2))).A.toarray()
    lam = np.sort(np.linalg.eigvalsh(A))
    s1 = np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    ref = np.sort((4 / h ** 2) * (s1[:, None, None] + s1[None, :, None] + s1[None, None, :]).ravel())
    np.testing.assert_allclose(lam, ref, rtol=1e-12)


def test_grf3d_is_seeded_and_unit_variance():
    from workloads import grf_field3d
    assert np.array_equal(grf_field3d(10, 3), grf_field3d(10, 3))
    assert not np.array_equal(grf_field3d(10, 3), grf_field3d(10, 4))
    v = np.mean([grf_field3d(12, s).var() + grf_field3d(12, s).mean() ** 2 for s in range(60)])
    assert 0.8 < v < 1.2
