"""Input generators: mesh counts, conformity, volumes, seeded fields."""
import math
from collections import Counter
from itertools import combinations

import numpy as np
import pytest

from paper_1506_08435_amd import workloads as W


def _volumes(p):
    X = p.coords[p.elems.astype(np.int64)]
    B = X[:, 1:, :] - X[:, :1, :]
    return np.abs(np.linalg.det(B)) / math.factorial(p.dim)


def test_small_config_counts():
    p = W.config_small()
    assert p.n_nodes == 4225 and p.n_elems == 8192 and p.n_free == 3969
    assert p.f_elem.sum() == 2 * 16 * 16        # f = 1 on cells [24, 40)^2
    np.testing.assert_allclose(_volumes(p).sum(), 1.0, rtol=1e-14)


def test_cube_counts_formula():
    for n in (3, 8, 16):
        p = W.cube3d(n)
        assert p.n_nodes == (n + 1) ** 3
        assert p.n_elems == 6 * n ** 3
        assert p.n_free == (n - 1) ** 3
        np.testing.assert_allclose(_volumes(p).sum(), 1.0, rtol=1e-13)
        assert (_volumes(p) > 0).all()


@pytest.mark.parametrize("maker", [lambda: W.square2d(6), lambda: W.cube3d(4)])
def test_conforming(maker):
    """Every interior facet is shared by exactly two simplices, every facet on
    the box boundary by one."""
    p = maker()
    d = p.dim
    facets = Counter()
    for e in p.elems:
        for f in combinations(sorted(int(v) for v in e), d):
            facets[f] += 1
    X = p.coords
    for f, cnt in facets.items():
        pts = X[list(f)]
        on_bnd = any(np.all(pts[:, k] == 0.0) or np.all(np.isclose(pts[:, k], 1.0))
                     for k in range(d))
        assert cnt == (1 if on_bnd else 2), (f, cnt)


def test_cube128_sizes_without_building():
    n = 128
    assert (n + 1) ** 3 == 2146689 and (n - 1) ** 3 == 2048383 and 6 * n ** 3 == 12582912


def test_tensors():
    D = W.aniso2d_tensor()
    # R(pi/6) diag(1, 1e-3) R^T: cos^2 + 1e-3 sin^2, (1 - 1e-3) sin cos, sin^2 + 1e-3 cos^2
    d12 = 0.999 * math.sqrt(3.0) / 4.0
    np.testing.assert_allclose(D, [[0.75025, d12], [d12, 0.25075]], rtol=1e-14)
    D3 = W.aniso3d_tensor()
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(D3)), [1e-4, 1e-2, 1.0], rtol=1e-12)
    v = np.linalg.eigh(D3)[1][:, -1]
    np.testing.assert_allclose(np.abs(v), [2 ** -0.5, 2 ** -0.5, 0.0], atol=1e-12)


def test_grf_statistics():
    G = W.gaussian_random_field((64, 64, 32), 8.0, 1506)
    assert abs(G.mean()) < 1e-12 and abs(G.std() - 1.0) < 1e-12
    # squared-exponential correlation at lag ell is exp(-1/2) ~ 0.61
    lag = 8
    rho = np.mean(G[:-lag] * G[lag:])
    assert 0.35 < rho < 0.85
    G2 = W.gaussian_random_field((64, 64, 32), 8.0, 1506)
    assert np.array_equal(G, G2)


def test_batch_problem_seeded_ranges():
    for i in (0, 1, 511):
        p = W.batch_problem(i)
        q = W.batch_problem(i)
        assert np.array_equal(p.f_elem, q.f_elem) and np.array_equal(p.D, q.D)
        n = p.cells[0]
        assert 32 <= n <= 256
        ev = np.linalg.eigvalsh(p.D[0])
        assert 1e-4 <= ev[0] / ev[1] <= 1e-1
        assert p.f_elem.sum() > 0


def test_transient_nodes_numbered_shortest_axis_first():
    """The transient workload renumbers nodes z fastest: every element keeps
    its geometry, Dirichlet flags follow their nodes, and the widest coupling
    is (nz + 1)(ny + 1) + nz + 2 (16,771 at 256 x 256 x 64, within int16)."""
    nx, ny, nz = 9, 7, 4
    p = W.config_transient3d(nx, ny, nz, ell=2.0)
    q = W.box_problem("lex", (nx, ny, nz), 1.0 / nx, W.aniso3d_tensor((1.0, 0.1, 1e-3)))
    assert np.array_equal(p.coords[p.elems], q.coords[q.elems])
    # a node's new id follows z, then y, then x
    ijk = np.rint(p.coords / p.h).astype(np.int64)
    assert np.array_equal(np.arange(p.n_nodes), ijk[:, 2] + (nz + 1) * (ijk[:, 1] + (ny + 1) * ijk[:, 0]))
    on_box = (ijk == 0).any(1) | (ijk == [nx, ny, nz]).any(1)
    assert np.array_equal(p.dirichlet.astype(bool), on_box)
    e = p.elems.astype(np.int64)
    assert (e.max(1) - e.min(1)).max() == (nz + 1) * (ny + 1) + nz + 2
    assert (64 + 1) * (256 + 1) + 64 + 2 == 16771 < 32767
