"""Pins of the oracle's P1 assembly (Sec. 2.1.2-2.1.3; capacity matrix Sec. 2.2.2)
against closed forms, textbook stencils and exact invariants."""
import math

import numpy as np
import pytest

from paper_1506_08435_amd import workloads as W


def _single(coords, D, f=1.0):
    coords = np.asarray(coords, dtype=np.float64)
    d = coords.shape[1]
    return W.Problem(name="one", dim=d, coords=coords,
                     elems=np.arange(d + 1, dtype=np.int32)[None, :],
                     D=np.asarray(D, dtype=np.float64).reshape(1, d, d), kscale=None,
                     f_elem=np.array([f]), dirichlet=np.zeros(d + 1, dtype=np.uint8),
                     cells=(1,) * d, h=1.0)


def _all_free(p):
    q = W.Problem(**{**p.__dict__})
    q.dirichlet = np.zeros_like(p.dirichlet)
    return q


def test_right_triangle_closed_form(oracle_mod):
    # isotropic right triangle, right angle at vertex 0: K = 1/2 [[2,-1,-1],[-1,1,0],[-1,0,1]]
    S = oracle_mod.assemble(_single([[0, 0], [1, 0], [0, 1]], np.eye(2)), with_mass=True)
    K = S.to_scipy().toarray()
    np.testing.assert_array_equal(K, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]))
    M = S.to_scipy("M").toarray()
    np.testing.assert_allclose(M, (0.5 / 12) * (np.ones((3, 3)) + np.eye(3)), rtol=1e-15)
    np.testing.assert_allclose(S.F, [1 / 6] * 3, rtol=1e-15)


def test_reference_tet_closed_form(oracle_mod):
    X = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    S = oracle_mod.assemble(_single(X, np.eye(3), f=2.0), with_mass=True)
    K = S.to_scipy().toarray()
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    np.testing.assert_allclose(K, ref, atol=1e-16)
    M = S.to_scipy("M").toarray()
    np.testing.assert_allclose(M, (1 / 6 / 20) * (np.ones((4, 4)) + np.eye(4)), rtol=1e-15)
    np.testing.assert_allclose(S.F, [2 / 6 / 4] * 4, rtol=1e-15)


def test_anisotropic_triangle_scaled_axes(oracle_mod):
    # D = diag(a, b) on the right triangle: K = 1/2 [[a+b, -a, -b], [-a, a, 0], [-b, 0, b]]
    a, b = 3.0, 0.25
    S = oracle_mod.assemble(_single([[0, 0], [1, 0], [0, 1]], np.diag([a, b])))
    K = S.to_scipy().toarray()
    np.testing.assert_allclose(K, 0.5 * np.array([[a + b, -a, -b], [-a, a, 0], [-b, 0, b]]), rtol=1e-15)


def test_2d_isotropic_is_five_point(oracle_mod):
    n = 8
    p = W.square2d(n, theta=0.0, ratio=1.0)
    p.f_elem = np.ones(p.n_elems)
    S = oracle_mod.assemble(p)
    A = S.to_scipy().toarray()
    m = n - 1
    idx = lambda i, j: i + m * j
    for j in range(m):
        for i in range(m):
            r = idx(i, j)
            assert A[r, r] == 4.0
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                if 0 <= i + di < m and 0 <= j + dj < m:
                    assert A[r, idx(i + di, j + dj)] == -1.0
            for di, dj in ((1, 1), (-1, -1)):
                if 0 <= i + di < m and 0 <= j + dj < m:
                    assert A[r, idx(i + di, j + dj)] == 0.0   # structural zero of the diagonal edge
            assert np.count_nonzero(A[r]) == 1 + sum(
                1 for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1))
                if 0 <= i + di < m and 0 <= j + dj < m)
    np.testing.assert_allclose(S.F, 1.0 / n ** 2, rtol=1e-13)
    # structural pattern holds 7 entries per interior row
    assert S.rowptr[idx(3, 3) + 1] - S.rowptr[idx(3, 3)] == 7


def test_3d_kuhn_isotropic_is_seven_point(oracle_mod):
    n = 6
    p = W.cube3d(n, eigs=(1.0, 1.0, 1.0))
    p.D = np.eye(3)[None]
    p.f_elem = np.ones(p.n_elems)
    S = oracle_mod.assemble(p)
    A = S.to_scipy()
    h = 1.0 / n
    m = n - 1
    r = 2 + m * (2 + m * 2)           # interior DOF (2,2,2)
    row = A.getrow(r)
    cols, vals = row.indices, row.data
    assert len(cols) == 15             # Kuhn pattern: 15 structural entries
    steps = {0: 6 * h, 1: -h, -1: -h, m: -h, -m: -h, m * m: -h, -m * m: -h}
    for c, v in zip(cols, vals):
        expect = steps.get(c - r, 0.0)
        assert abs(v - expect) <= 1e-15, (c - r, v, expect)
    np.testing.assert_allclose(S.F, h ** 3, rtol=1e-12)


@pytest.mark.parametrize("maker", [lambda: W.square2d(16), lambda: W.cube3d(8),
                                   lambda: W.config_transient3d(12, 10, 6, ell=2.0)])
def test_symmetry_rowsum_patch(oracle_mod, maker):
    p = maker()
    S = oracle_mod.assemble(p)
    A = S.to_scipy()
    assert (A - A.T).count_nonzero() == 0             # bitwise symmetric
    full = oracle_mod.assemble(_all_free(p), with_mass=True)
    Af = full.to_scipy()
    one = np.ones(full.n)
    scale = np.abs(Af).max()
    assert np.abs(Af @ one).max() <= 1e-14 * scale     # K_full 1 = 0
    # patch test: for l(x) = a.x, l.K l = |Omega| a.D a (element-constant D)
    rng = np.random.default_rng(0)
    a = rng.standard_normal(p.dim)
    l = p.coords @ a
    if p.kscale is None:
        D = p.D[0]
        exact = a @ D @ a * 1.0
    else:
        vol = np.prod(np.array(p.cells) * p.h) / p.n_elems
        exact = vol * np.sum(p.kscale) * (a @ p.D[0] @ a)
    # (K l has heavy cancellation in the interior, hence the looser bound)
    np.testing.assert_allclose(l @ (Af @ l), exact, rtol=1e-10)
    if p.kscale is None:
        # with a constant D, interior rows annihilate linear functions
        interior = p.dirichlet == 0
        assert np.abs((Af @ l)[interior]).max() <= 1e-13 * scale
    # consistent mass integrates P1 products exactly: x.Mx = int x^2 = |Omega|/3 along x
    Mf = full.to_scipy("M")
    x = p.coords[:, 0]
    extent = np.array(p.cells) * p.h
    vol_omega = float(np.prod(extent))
    np.testing.assert_allclose(one @ (Mf @ one), vol_omega, rtol=1e-13)
    np.testing.assert_allclose(x @ (Mf @ x), vol_omega * extent[0] ** 2 / 3.0, rtol=1e-12)


def test_elimination_is_submatrix(oracle_mod):
    p = W.square2d(10)
    S = oracle_mod.assemble(p)
    full = oracle_mod.assemble(_all_free(p))
    free = np.flatnonzero(p.dirichlet == 0)
    sub = full.to_scipy()[free][:, free]
    assert abs(sub - S.to_scipy()).max() == 0.0
    assert np.array_equal(S.dof[free], np.arange(free.size))
    assert (S.dof[p.dirichlet == 1] == -1).all()


def test_load_integrates_source(oracle_mod):
    assert abs(oracle_mod.assemble(W.config_small()).F.sum() - 0.0625) < 1e-15
    assert abs(oracle_mod.assemble(W.cube3d(16)).F.sum() - 0.015625) < 1e-15


def test_config_small_matrix_facts(oracle_mod):
    S = oracle_mod.assemble(W.config_small())
    assert S.n == 3969 and S.nnz == 27281
    A = S.to_scipy()
    off = A - __import__("scipy.sparse", fromlist=["diags"]).diags(A.diagonal())
    # not an M-matrix: some off-diagonal entries are positive
    assert (off.data > 0).sum() > 1000
