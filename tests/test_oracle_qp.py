"""Pins of the oracle's QP solution (Sec. 2.1.3, eq. non-negative; Sec. 2.2.2)
against brute force, library solves of special cases, the KKT definition, a
manufactured solution's convergence rate and limits of the transient step."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import brute
from paper_1506_08435_amd import workloads as W


def _system_from_dense(oracle_mod, K, F):
    A = sp.csr_matrix(K)
    A.sort_indices()
    return oracle_mod.System(n=K.shape[0], rowptr=A.indptr.astype(np.int64),
                             col=A.indices.astype(np.int32), K=A.data.astype(np.float64), M=None,
                             F=np.asarray(F, dtype=np.float64), dof=np.arange(K.shape[0]))


@pytest.mark.parametrize("maker", [W.tiny2d, W.tiny3d])
def test_tiny_meshes_match_brute_force(oracle_mod, maker):
    S = oracle_mod.assemble(maker())
    assert S.n <= 12
    K = S.to_scipy().toarray()
    gal = np.linalg.solve(K, S.F)
    assert gal.min() < 0.0                    # the constraint matters here
    c_bf, sets = brute.brute_force(K, S.F)
    r = oracle_mod.solve(S, tol=1e-13)
    assert r.certified and r.status == 0
    np.testing.assert_allclose(r.c, c_bf, rtol=0, atol=1e-13 * np.abs(c_bf).max())
    assert (r.c >= 0).all()
    assert len(sets) == 1                    # non-degenerate: one KKT face


def test_random_dense_qps_match_brute_force(oracle_mod):
    rng = np.random.default_rng(1506)
    for trial in range(40):
        n = int(rng.integers(1, 11))
        A = rng.standard_normal((n, n))
        K = A @ A.T + 0.3 * np.eye(n)
        F = rng.standard_normal(n)
        c_bf, _ = brute.brute_force(K, F)
        S = _system_from_dense(oracle_mod, K, F)
        r = oracle_mod.solve(S, tol=1e-13)
        scale = max(np.abs(c_bf).max(), 1e-300)
        np.testing.assert_allclose(r.c, c_bf, rtol=0, atol=1e-11 * scale, err_msg=f"trial {trial}")
        assert (r.c >= 0).all()


def _isotropic(p):
    p.D = np.eye(p.dim)[None].copy()
    return p


@pytest.mark.parametrize("maker", [
    lambda: _isotropic(W.square2d(32)),               # isotropic: 5-point M-matrix
    lambda: W.square2d(32, theta=0.0, ratio=1e-3),    # axis-aligned anisotropy: D12 = 0
    lambda: _isotropic(W.cube3d(10)),                 # isotropic Kuhn: 7-point M-matrix
])
def test_m_matrix_cases_equal_direct_solve(oracle_mod, maker):
    """K is a Stieltjes matrix and F >= 0, so K^-1 F >= 0 solves the QP."""
    S = oracle_mod.assemble(maker())
    A = S.to_scipy().tocsc()
    off = (A - sp.diags(A.diagonal())).tocoo()
    assert off.data.max() <= 0.0
    ref = spl.spsolve(A, S.F)
    assert ref.min() > 0.0
    r = oracle_mod.solve(S, tol=1e-13)
    np.testing.assert_allclose(r.c, ref, rtol=0, atol=1e-12 * ref.max())
    assert (r.c > 0).all()                    # active set empty


def test_nonnegative_galerkin_is_the_minimiser(oracle_mod):
    # mild anisotropy + a broad source: the Galerkin solution is already >= 0
    p = W.square2d(24, theta=math.pi / 6, ratio=0.5)
    p.f_elem = np.ones(p.n_elems)
    S = oracle_mod.assemble(p)
    ref = spl.spsolve(S.to_scipy().tocsc(), S.F)
    assert ref.min() > 0.0
    r = oracle_mod.solve(S, tol=1e-13)
    np.testing.assert_allclose(r.c, ref, rtol=0, atol=1e-12 * ref.max())


def test_config_small_certificate(oracle_mod):
    S = oracle_mod.assemble(W.config_small())
    r = oracle_mod.solve(S, tol=1e-12)
    k = oracle_mod.kkt(S, r.c)
    assert r.certified and k.r <= 1e-12 and k.min_c >= 0.0 and k.nonfinite == 0
    assert k.nat_inf <= 1e-11 * np.abs(S.F).max()
    assert k.min_g_active >= -1e-11 * np.abs(S.F).max()
    assert abs(r.c.max() - 0.0739059) < 1e-6
    # the Galerkin solution violates non-negativity on ~32% of the nodes
    gal = spl.spsolve(S.to_scipy().tocsc(), S.F)
    assert 0.25 < (gal < 0).mean() < 0.40
    # first-order optimality differs: the QP solution is not the Galerkin one
    assert np.abs(r.c - gal).max() > 1e-5


def test_oracle_deterministic(oracle_mod):
    S = oracle_mod.assemble(W.square2d(40))
    oracle_mod.set_num_threads(1)
    a = oracle_mod.solve(S, tol=1e-12).c
    oracle_mod.set_num_threads(max(2, oracle_mod.num_threads()))
    b = oracle_mod.solve(S, tol=1e-12).c
    assert np.array_equal(a, b)


def test_nonpositive_source_gives_zero(oracle_mod):
    p = W.square2d(16)
    p.f_elem = -p.f_elem
    S = oracle_mod.assemble(p)
    r = oracle_mod.solve(S, c0=np.full(S.n, 0.3))
    assert r.certified and np.array_equal(r.c, np.zeros(S.n))


def test_mms_rate_2d(oracle_mod):
    errs = []
    for n in (16, 32, 64):
        p = W.mms_problem(2, n)
        S = oracle_mod.assemble(p)
        r = oracle_mod.solve(S, tol=1e-13)
        free = W.free_node_ids(p)
        errs.append(np.abs(r.c - p.exact(p.coords[free])).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(1.8 <= q <= 2.25 for q in rates), rates


def test_mms_rate_3d(oracle_mod):
    errs = []
    for n in (8, 16, 32):
        p = W.mms_problem(3, n)
        S = oracle_mod.assemble(p)
        r = oracle_mod.solve(S, tol=1e-13)
        free = W.free_node_ids(p)
        errs.append(np.abs(r.c - p.exact(p.coords[free])).max())
    rate = math.log2(errs[-2] / errs[-1])
    assert 1.8 <= rate <= 2.3, errs


def test_transient_huge_dt_is_steady(oracle_mod):
    p = W.square2d(24)
    S = oracle_mod.assemble(p, with_mass=True)
    steady = oracle_mod.solve(S, tol=1e-13).c
    r = oracle_mod.transient_step(S, 1e12, np.zeros(S.n), tol=1e-13)
    assert r.certified
    np.testing.assert_allclose(r.c, steady, rtol=0, atol=1e-9 * steady.max())


def test_transient_steps_certified_and_warm_equals_cold(oracle_mod):
    p = W.cube3d(8)
    S = oracle_mod.assemble(p, with_mass=True)
    dt = 1e-3
    c = np.zeros(S.n)
    for step in range(3):
        Kt, ft = oracle_mod.transient_system(S, dt, c)
        warm = oracle_mod.transient_step(S, dt, c, tol=1e-13)
        cold = oracle_mod.solve(S, tol=1e-13, F=ft, vals=Kt)
        assert warm.certified and cold.certified
        k = oracle_mod.kkt(S, warm.c, F=ft, vals=Kt)
        assert k.r <= 1e-13 and k.min_c >= 0.0
        np.testing.assert_allclose(warm.c, cold.c, rtol=0, atol=1e-11 * max(cold.c.max(), 1e-30))
        c = warm.c
    assert c.max() > 0


def test_transient_system_definition(oracle_mod):
    """K~ = M/dt + K and f~ = F + M c^n / dt, checked through scipy products."""
    p = W.square2d(12)
    S = oracle_mod.assemble(p, with_mass=True)
    rng = np.random.default_rng(3)
    cn = rng.random(S.n)
    Kt, ft = oracle_mod.transient_system(S, 0.01, cn)
    A = S.to_scipy()
    Mm = S.to_scipy("M")
    np.testing.assert_allclose(Kt, Mm.data / 0.01 + A.data, rtol=1e-15)
    np.testing.assert_allclose(ft, S.F + (Mm @ cn) / 0.01, rtol=1e-13)


def test_kkt_report_special_points(oracle_mod):
    """At c = 0 with F >= 0 the projected gradient is -F, so r = 1 exactly; at
    the brute-force minimiser every KKT measure vanishes to rounding; a point
    with a negative entry is reported by min_c."""
    S = oracle_mod.assemble(W.tiny2d())
    k0 = oracle_mod.kkt(S, np.zeros(S.n))
    assert k0.r == 1.0 and k0.min_c == 0.0 and k0.n_zero == S.n
    # min(c, g) at c = 0 is min(0, -F): its largest magnitude is max(F)
    assert k0.nat_inf == S.F.max()
    c_bf, _ = brute.brute_force(S.to_scipy().toarray(), S.F)
    k1 = oracle_mod.kkt(S, c_bf)
    assert k1.r <= 1e-13 and k1.comp_inf <= 1e-15 and k1.min_c >= 0.0
    bad = c_bf.copy()
    bad[np.argmax(bad)] *= -1.0
    k2 = oracle_mod.kkt(S, bad)
    assert k2.min_c < 0.0 and k2.r > 1e-3
    nanc = c_bf.copy()
    nanc[0] = np.nan
    assert oracle_mod.kkt(S, nanc).nonfinite >= 1


@pytest.mark.parametrize("maker", [
    W.config_small,
    lambda: W.square2d(37, theta=1.1, ratio=3e-3),
    lambda: W.cube3d(10),
])
def test_galerkin_oracle_equals_direct_solve(oracle_mod, maker):
    """The oracle's unconstrained solve (Sec. 2.1.2, eq. Single_field_formulation,
    by Jacobi-PCG) against a sparse direct factorisation of the same K; the
    Galerkin solution takes negative values on these anisotropic problems
    (the DMP violation of Table Tab:S5_cube_dmp)."""
    S = oracle_mod.assemble(maker())
    ref = spl.spsolve(S.to_scipy().tocsc(), S.F)
    c = oracle_mod.galerkin(S, rtol=1e-13)
    assert np.abs(c - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.linalg.norm(S.to_scipy() @ c - S.F) <= 1.01e-13 * np.linalg.norm(S.F)
    assert c.min() < 0.0 and (c < 0).sum() == (ref < 0).sum()


def test_galerkin_oracle_m_matrix_is_nonnegative(oracle_mod):
    """Isotropic Kuhn mesh: K is a Stieltjes matrix, K^-1 >= 0, so the Galerkin
    solution of a non-negative load is non-negative and equals the QP's."""
    p = _isotropic(W.cube3d(9))
    S = oracle_mod.assemble(p)
    c = oracle_mod.galerkin(S, rtol=1e-13)
    assert c.min() > 0.0
    r = oracle_mod.solve(S, tol=1e-13)
    np.testing.assert_allclose(c, r.c, rtol=0, atol=1e-11 * r.c.max())


# ---------------------------------------------------------------- two-sided bounds, lifting
def test_box_random_dense_qps_match_brute_force(oracle_mod):
    """lo <= c <= hi (Sec. 2.2.2, eq. Eq:non-negative): random SPD QPs with
    random bounds against exhaustive enumeration of lower/free/upper."""
    rng = np.random.default_rng(2015)
    uppers = 0
    for trial in range(40):
        n = int(rng.integers(1, 8))
        A = rng.standard_normal((n, n))
        K = A @ A.T + 0.3 * np.eye(n)
        F = 2.0 * rng.standard_normal(n)
        lo = float(rng.uniform(-0.5, 0.2))
        hi = lo + float(rng.uniform(0.1, 1.0))
        c_bf, sets = brute.brute_force(K, F, lo=lo, hi=hi)
        S = _system_from_dense(oracle_mod, K, F)
        r = oracle_mod.solve(S, tol=1e-13, lo=lo, hi=hi)
        assert r.status == 0 and r.certified
        scale = max(np.abs(c_bf).max(), 1e-300)
        np.testing.assert_allclose(r.c, c_bf, rtol=0, atol=1e-11 * scale, err_msg=f"trial {trial}")
        assert r.c.min() >= lo and r.c.max() <= hi
        uppers += int((r.c == hi).sum())
    assert uppers > 0          # the upper bound was exercised


@pytest.mark.parametrize("maker", [W.tiny2d, W.tiny3d])
def test_tiny_meshes_capped_match_brute_force(oracle_mod, maker):
    S = oracle_mod.assemble(maker())
    K = S.to_scipy().toarray()
    hi = 0.6 * oracle_mod.solve(S, tol=1e-13).c.max()
    c_bf, sets = brute.brute_force(K, S.F, hi=hi)
    r = oracle_mod.solve(S, tol=1e-13, hi=hi)
    assert r.certified and (r.c == hi).any() and (r.c == 0).any()
    np.testing.assert_allclose(r.c, c_bf, rtol=0, atol=1e-13 * hi)


def test_box_reflection_swaps_the_bounds(oracle_mod):
    """c* solves (F, [0, 1]) iff 1 - c* solves (K 1 - F, [0, 1]): the map
    c -> 1 - c exchanges the two bounds and the sign of the gradient, so a
    mistake on either side of the box breaks the identity."""
    p = W.square2d(24, theta=1.0, ratio=1e-3)
    p.f_elem = 30.0 * p.f_elem
    S = oracle_mod.assemble(p)
    r = oracle_mod.solve(S, tol=1e-13, hi=1.0)
    assert (r.c == 1.0).sum() > 0 and (r.c == 0.0).sum() > 0
    F2 = oracle_mod.spmv(S, np.ones(S.n)) - S.F
    r2 = oracle_mod.solve(S, tol=1e-13, F=F2, hi=1.0)
    np.testing.assert_allclose(r2.c, 1.0 - r.c, rtol=0, atol=1e-11)
    k = oracle_mod.kkt(S, r.c, lo=0.0, hi=1.0)
    assert k.r <= 1e-12 and k.n_upper == (r.c == 1.0).sum() and k.max_g_upper <= 0.0
    assert k.min_g_active >= -1e-12 * np.abs(S.F).max()


@pytest.mark.parametrize("maker", [
    lambda: W.square2d(9, theta=0.4, ratio=1e-2),
    lambda: W.cube3d(6),
])
def test_lifting_reproduces_linear_boundary_data(oracle_mod, maker):
    """P1 reproduces linear functions: with f = 0 and Dirichlet values a.x + b
    on the whole boundary, the lifted system K c = F - K_FD c_D has the linear
    function itself as its solution at the free nodes, for any constant D."""
    p = maker()
    p.f_elem = np.zeros_like(p.f_elem)
    a = np.array([0.7, -1.3, 0.4][:p.dim])
    lin = p.coords @ a + 0.25
    p.dirichlet_values = np.where(p.dirichlet == 1, lin, 0.0)
    S = oracle_mod.assemble(p)
    c = spl.spsolve(S.to_scipy().tocsc(), S.F)
    free_nodes = np.flatnonzero(S.dof >= 0)
    np.testing.assert_allclose(c, lin[free_nodes], rtol=0, atol=1e-12)
    assert np.abs(oracle_mod.galerkin(S, rtol=1e-14) - lin[free_nodes]).max() <= 1e-11


def test_cube_hole_workload_and_dmp(oracle_mod):
    """The structured cube-with-hole stand-in (Sec. 5.1): geometry, the
    dispersion tensor (eq. S5_dispersion_tensor), Galerkin DMP violation and
    a certified [0, 1] solution."""
    k = 2
    p = W.cube_hole(k)
    n = 9 * k
    assert p.n_elems == 6 * (n ** 3 - k ** 3)
    used = np.zeros(p.n_nodes, dtype=bool)
    used[p.elems.ravel()] = True
    assert (p.dirichlet[~used] == 1).all() and (p.dirichlet_values[~used] == 1.0).all()
    x = p.coords
    on_hole = np.all((x >= 4.0 / 9 - 1e-12) & (x <= 5.0 / 9 + 1e-12), axis=1)
    assert np.array_equal(p.dirichlet_values == 1.0, on_hole)
    D = p.D[0]
    v = np.ones(3) / math.sqrt(3.0)
    np.testing.assert_allclose(D @ v, math.sqrt(3.0) * v, rtol=1e-14)
    u = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
    np.testing.assert_allclose(D @ u, math.sqrt(3.0) * 1e-3 * u, atol=1e-15)
    S = oracle_mod.assemble(p)
    gal = spl.spsolve(S.to_scipy().tocsc(), S.F)
    assert (gal < 0).mean() > 0.2                    # DMP violated by Galerkin
    r = oracle_mod.solve(S, tol=1e-12, lo=0.0, hi=1.0)
    assert r.certified and r.c.min() >= 0.0 and r.c.max() <= 1.0
    kk = oracle_mod.kkt(S, r.c, lo=0.0, hi=1.0)
    assert kk.r <= 1e-12 and kk.n_zero > 0


def test_isotropic_hole_dmp_box_equals_galerkin(oracle_mod):
    """Isotropic D on the Kuhn mesh: K is a Stieltjes matrix and the lifted
    data lie in [0, 1], so the Galerkin solution keeps the maximum principle
    and the [0, 1]-bounded QP returns it."""
    p = W.cube_hole(2)
    p.D = np.eye(3)[None].copy()
    S = oracle_mod.assemble(p)
    gal = spl.spsolve(S.to_scipy().tocsc(), S.F)
    assert gal.min() > 0.0 and gal.max() < 1.0
    r = oracle_mod.solve(S, tol=1e-13, lo=0.0, hi=1.0)
    np.testing.assert_allclose(r.c, gal, rtol=0, atol=1e-12)


def test_transient_box_large_dt_is_steady(oracle_mod):
    p = W.square2d(16, theta=0.5, ratio=1e-2)
    p.f_elem = 20.0 * p.f_elem
    S = oracle_mod.assemble(p, with_mass=True)
    steady = oracle_mod.solve(S, tol=1e-13, hi=0.5)
    assert (steady.c == 0.5).any()
    r = oracle_mod.transient_step(S, 1e12, np.zeros(S.n), tol=1e-13, hi=0.5)
    np.testing.assert_allclose(r.c, steady.c, rtol=0, atol=1e-10)


# ---------------------------------------------------------------- nondegenerate masks
def _kkt_problem(c_star, g_star, seed):
    """A dense SPD K and the load F = K c* - g* for which c* is the minimiser
    whenever (c*, g*) satisfy the KKT conditions of the box."""
    rng = np.random.default_rng(seed)
    n = c_star.size
    A = rng.standard_normal((n, n))
    K = A @ A.T + n * np.eye(n)
    return K, K @ c_star - g_star


def test_nondegenerate_masks_hand_built_lower_bound(oracle_mod):
    """Free, strictly active and degenerate nodes known by construction
    (c >= 0, g >= 0, c.g = 0; Sec. 2.1.3, eq. non-negative), with ||c||_inf
    = 2e-3 and ||F||_inf ~ 1e3: nodes 0, 3 and 6 free; node 4 free with c far
    below the F scale but above 1e-8 ||c||_inf; node 1 strictly active; node
    2 degenerate (c = g = 0); node 5 at zero with g above 1e-8 ||c||_inf but
    below 1e-8 ||F||_inf, which the masks leave undecided (the two scales
    swapped would call node 4 undecided and node 5 strict).  Brute force
    confirms the minimiser, and its surviving assignments differ on the
    degenerate node 2 only."""
    c_star = np.array([1e-3, 0.0, 0.0, 2e-3, 1e-9, 0.0, 5e-4])
    g_star = np.array([0.0, 4.0, 0.0, 0.0, 0.0, 1e-6, 0.0])
    rng = np.random.default_rng(5)
    A = rng.standard_normal((7, 7))
    K = 1e5 * (A @ A.T + 7 * np.eye(7))
    F = K @ c_star - g_star
    assert 1e2 < np.abs(F).max() < 1e4
    free, strict = oracle_mod.nondegenerate_masks(c_star, g_star, F)
    assert free.tolist() == [True, False, False, True, True, False, True]
    assert strict.tolist() == [False, True, False, False, False, False, False]
    # the masks of the minimiser as brute force finds it
    c_bf, survivors = brute.brute_force(K, F)
    assert np.abs(c_bf - c_star).max() <= 1e-12 * np.abs(c_star).max()
    g_bf = K @ c_bf - F
    free_bf, strict_bf = oracle_mod.nondegenerate_masks(c_bf, g_bf, F)
    assert np.array_equal(free_bf, free) and np.array_equal(strict_bf, strict)
    sets = [set(a) for a in survivors]
    assert len(sets) == 2 and set.union(*sets) - set.intersection(*sets) == {2}


def test_nondegenerate_masks_hand_built_two_sided(oracle_mod):
    """Box [lo, hi] = [-0.5, 1]: strict at lo needs g > 0, strict at hi needs
    g < 0 (a sign slip on either side fails); nodes at a bound with g = 0 are
    degenerate; free nodes are inside both bounds by more than 1e-8 ||c||_inf."""
    lo, hi = -0.5, 1.0
    c_star = np.array([lo, hi, 0.3, hi, lo, 0.9999, -0.2])
    g_star = np.array([2.0, -3.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    K, F = _kkt_problem(c_star, g_star, 9)
    free, strict = oracle_mod.nondegenerate_masks(c_star, g_star, F, lo=lo, hi=hi)
    assert free.tolist() == [False, False, True, False, False, True, True]
    assert strict.tolist() == [True, True, False, False, False, False, False]
    c_bf, _ = brute.brute_force(K, F, lo=lo, hi=hi)
    assert np.abs(c_bf - c_star).max() <= 1e-12
    # the wrong sign on the upper side turns the strict upper node away
    flipped = g_star.copy()
    flipped[1] = 3.0
    _, strict_f = oracle_mod.nondegenerate_masks(c_star, flipped, F, lo=lo, hi=hi)
    assert not strict_f[1]


def test_nondegenerate_masks_on_tiny_meshes(oracle_mod):
    """On the brute-force meshes every node is decided (no degeneracy), the
    masks partition the nodes, and the active ones are exactly the nodes the
    unique surviving assignment puts at the bound."""
    for p in (W.tiny2d(), W.tiny3d()):
        S = oracle_mod.assemble(p)
        Kd = S.to_scipy().toarray()
        c_bf, survivors = brute.brute_force(Kd, S.F)
        assert len(survivors) == 1
        g = Kd @ c_bf - S.F
        free, strict = oracle_mod.nondegenerate_masks(c_bf, g, S.F)
        assert free.any() and strict.any()
        assert not (free & strict).any() and (free | strict).all()
        assert np.array_equal(strict, c_bf == 0.0)
