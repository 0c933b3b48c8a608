"""Seeded synthetic inputs for the non-negative diffusion QP.

This module produces *inputs only*: simplicial meshes, per-element diffusivity
tensors, per-element source values and the Dirichlet node mask.  It holds none
of the method's arithmetic (no element matrices, no assembly, no solver); the
CPU oracle and the HIP library each assemble and solve from these arrays on
their own.

Problem statement (steady diffusion BVP, Sec. 2.1 eq. LargeScale_BVP): find c
with -div(D grad c) = f in Omega, c = 0 on the Dirichlet boundary, D symmetric
and uniformly elliptic.  The paper's cube-with-hole meshes and the chromium
data set are not available, so every workload here is a seeded structured
stand-in of the same kind (P1 simplices, anisotropic D, compact sources):

* 2D: n x n square cells of side h, each split along its (i,j)-(i+1,j+1)
  diagonal into the triangles (v00, v10, v11) and (v00, v11, v01).
* 3D: cuboid grid of cubic cells, each split into the six Kuhn tetrahedra
  v000 -> +e_a -> +e_a+e_b -> v111 over the six axis orders (a, b, c).
* Nodes are numbered lexicographically, x fastest; elements cell by cell
  (x fastest) and then by sub-simplex.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

# Axis orders of the six Kuhn tetrahedra of a cube (fixed order).
KUHN_ORDERS: Tuple[Tuple[int, int, int], ...] = (
    (0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclasses.dataclass
class Problem:
    """One QP instance as plain host arrays.

    coords     float64 [n_nodes, dim]
    elems      int32   [n_elems, dim+1]   node ids of each simplex
    D          float64 [nD, dim, dim]     nD == 1 (one tensor) or n_elems
    kscale     float64 [n_elems] or None  per-element scalar multiplying D
    f_elem     float64 [n_elems]          source value on each element
    dirichlet  uint8   [n_nodes]          1 = Dirichlet node
    cells      cell counts per axis of the structured grid
    dirichlet_values float64 [n_nodes] or None: c at the Dirichlet nodes
               (None: homogeneous, c = 0)
    bounds     (lo, hi) of the constrained problem: (0, inf) is the
               non-negative QP, (0, 1) the DMP variant
    """
    name: str
    dim: int
    coords: np.ndarray
    elems: np.ndarray
    D: np.ndarray
    kscale: Optional[np.ndarray]
    f_elem: np.ndarray
    dirichlet: np.ndarray
    cells: Tuple[int, ...]
    h: float
    exact: Optional[Callable[[np.ndarray], np.ndarray]] = None
    dirichlet_values: Optional[np.ndarray] = None
    bounds: Tuple[float, float] = (0.0, math.inf)

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    @property
    def n_free(self) -> int:
        return int(self.n_nodes - int(self.dirichlet.sum()))


# ---------------------------------------------------------------- meshes
def structured_simplex_mesh(cells: Sequence[int], h: float):
    """Nodes and simplices of a structured grid with `cells` cells per axis."""
    cells = tuple(int(c) for c in cells)
    dim = len(cells)
    npts = [c + 1 for c in cells]
    axes = [np.arange(p, dtype=np.float64) * h for p in npts]
    if dim == 2:
        yy, xx = np.meshgrid(axes[1], axes[0], indexing="ij")
        coords = np.stack([xx.ravel(), yy.ravel()], axis=1)
        nx, ny = cells
        j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        v00 = (i + (nx + 1) * j).ravel().astype(np.int64)
        v10 = v00 + 1
        v01 = v00 + (nx + 1)
        v11 = v01 + 1
        tri = np.empty((v00.size, 2, 3), dtype=np.int64)
        tri[:, 0] = np.stack([v00, v10, v11], axis=1)
        tri[:, 1] = np.stack([v00, v11, v01], axis=1)
        elems = tri.reshape(-1, 3)
    elif dim == 3:
        zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        coords = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
        nx, ny, nz = cells
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                              indexing="ij")
        step = np.array([1, nx + 1, (nx + 1) * (ny + 1)], dtype=np.int64)
        v000 = (i + (nx + 1) * (j + (ny + 1) * k)).ravel().astype(np.int64)
        v111 = v000 + step.sum()
        tet = np.empty((v000.size, 6, 4), dtype=np.int64)
        for t, (a, b, _c) in enumerate(KUHN_ORDERS):
            tet[:, t, 0] = v000
            tet[:, t, 1] = v000 + step[a]
            tet[:, t, 2] = v000 + step[a] + step[b]
            tet[:, t, 3] = v111
        elems = tet.reshape(-1, 4)
    else:
        raise ValueError("dim must be 2 or 3")
    return np.ascontiguousarray(coords), np.ascontiguousarray(elems.astype(np.int32))


def box_dirichlet(cells: Sequence[int]) -> np.ndarray:
    """uint8 mask of the nodes on the boundary of the box (all faces)."""
    npts = [c + 1 for c in cells]
    grids = np.meshgrid(*[np.arange(p) for p in reversed(npts)], indexing="ij")
    on = np.zeros(grids[0].shape, dtype=bool)
    for g, p in zip(grids, reversed(npts)):
        on |= (g == 0) | (g == p - 1)
    return on.ravel().astype(np.uint8)


def subelems_per_cell(dim: int) -> int:
    return 2 if dim == 2 else 6


def cell_box_indicator(cells: Sequence[int], lo: Sequence[int], hi: Sequence[int]) -> np.ndarray:
    """Per-element 1.0 on the cells with lo <= index < hi per axis, else 0."""
    dim = len(cells)
    grids = np.meshgrid(*[np.arange(c) for c in reversed(cells)], indexing="ij")
    inside = np.ones(grids[0].shape, dtype=bool)
    for ax in range(dim):
        g = grids[dim - 1 - ax]
        inside &= (g >= lo[ax]) & (g < hi[ax])
    per_cell = inside.ravel().astype(np.float64)
    return np.repeat(per_cell, subelems_per_cell(dim))


def central_box(cells: Sequence[int]):
    """Cell ranges [3n/8, 5n/8) per axis: the central box of half the extent."""
    lo = [(3 * c) // 8 for c in cells]
    hi = [(5 * c) // 8 for c in cells]
    return lo, hi


# ---------------------------------------------------------------- tensors
def rot2(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def rot_x(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_z(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def principal_tensor(R: np.ndarray, eigs: Sequence[float]) -> np.ndarray:
    """Diffusivity with principal axes the columns of R: R diag(eigs) R^T."""
    D = R @ np.diag(np.asarray(eigs, dtype=np.float64)) @ R.T
    return 0.5 * (D + D.T)


def aniso2d_tensor(theta: float = math.pi / 6, ratio: float = 1e-3) -> np.ndarray:
    return principal_tensor(rot2(theta), [1.0, ratio])


def aniso3d_rotation() -> np.ndarray:
    """pi/6 about x, then pi/4 about z."""
    return rot_z(math.pi / 4) @ rot_x(math.pi / 6)


def aniso3d_tensor(eigs=(1.0, 1e-2, 1e-4)) -> np.ndarray:
    return principal_tensor(aniso3d_rotation(), eigs)


def dispersion_tensor(v: Sequence[float], alpha_L: float, alpha_T: float,
                      D_M: float = 0.0) -> np.ndarray:
    """Velocity-dependent dispersion (Sec. 5, eq. S5_dispersion_tensor):
    (alpha_T |v| + D_M) I + (alpha_L - alpha_T) v v^T / |v|; principal values
    alpha_L |v| + D_M along v and alpha_T |v| + D_M across it."""
    v = np.asarray(v, dtype=np.float64)
    speed = float(np.linalg.norm(v))
    D = (alpha_T * speed + D_M) * np.eye(v.size) + (alpha_L - alpha_T) * np.outer(v, v) / speed
    return 0.5 * (D + D.T)


# ---------------------------------------------------------------- problems
def box_problem(name: str, cells: Sequence[int], h: float, D: np.ndarray,
                f_elem: Optional[np.ndarray] = None, kscale=None) -> Problem:
    cells = tuple(int(c) for c in cells)
    dim = len(cells)
    coords, elems = structured_simplex_mesh(cells, h)
    if f_elem is None:
        lo, hi = central_box(cells)
        f_elem = cell_box_indicator(cells, lo, hi)
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64).reshape(-1, dim, dim))
    return Problem(name=name, dim=dim, coords=coords, elems=elems, D=D,
                   kscale=None if kscale is None else np.ascontiguousarray(kscale, dtype=np.float64),
                   f_elem=np.ascontiguousarray(f_elem, dtype=np.float64),
                   dirichlet=box_dirichlet(cells), cells=cells, h=h)


def square2d(n: int = 64, theta: float = math.pi / 6, ratio: float = 1e-3) -> Problem:
    """Unit square, n x n cells, f = 1 on the central box [3/8, 5/8)^2 of cells."""
    return box_problem(f"square2d_n{n}", (n, n), 1.0 / n, aniso2d_tensor(theta, ratio))


def cube3d(n: int = 128, eigs=(1.0, 1e-2, 1e-4)) -> Problem:
    """Unit cube, n^3 cells x 6 Kuhn tets, f = 1 on the central cube of side 1/4."""
    return box_problem(f"cube3d_n{n}", (n, n, n), 1.0 / n, aniso3d_tensor(eigs))


def cube_hole(k: int = 14, alpha_L: float = 1.0, alpha_T: float = 1e-3, D_M: float = 0.0,
              v=(1.0, 1.0, 1.0), inner: float = 1.0, bounds=(0.0, 1.0)) -> Problem:
    """Structured stand-in for the unit cube with the cubic hole
    [4/9, 5/9]^3 (Sec. 5.1): n = 9k cells per side, the k^3 cells of the hole
    removed, c = 0 on the outer boundary, c = `inner` on the hole's boundary,
    f = 0, D the dispersion tensor of velocity v = (1, 1, 1) with alpha_L = 1,
    alpha_T = 1e-3, D_M = 0, bounds [0, 1] (the DMP variant of the non-negative
    method).  Nodes strictly inside the hole belong to no element; they are
    flagged Dirichlet (value `inner`) so that node ids stay lexicographic.
    The grid is mirrored in x (x -> 1 - x; the domain is symmetric), so every
    cell's Kuhn diagonal runs along (-1, 1, 1), across the flow: with the
    diagonal along v = (1, 1, 1) the P1 stiffness of this tensor is an
    M-matrix and the Galerkin solution keeps the maximum principle, which the
    paper's unstructured meshes do not."""
    n = 9 * int(k)
    cells = (n, n, n)
    coords, elems = structured_simplex_mesh(cells, 1.0 / n)
    coords[:, 0] = 1.0 - coords[:, 0]
    lo, hi = 4 * k, 5 * k
    in_hole = cell_box_indicator(cells, (lo, lo, lo), (hi, hi, hi)) > 0.0
    elems = np.ascontiguousarray(elems[~in_hole])
    npts = n + 1
    kk, jj, ii = np.meshgrid(np.arange(npts), np.arange(npts), np.arange(npts), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    outer = box_dirichlet(cells).astype(bool)
    hole = ((ii >= lo) & (ii <= hi) & (jj >= lo) & (jj <= hi) & (kk >= lo) & (kk <= hi))
    dirichlet = (outer | hole).astype(np.uint8)
    dvals = np.where(hole, float(inner), 0.0)
    D = dispersion_tensor(v, alpha_L, alpha_T, D_M).reshape(1, 3, 3)
    return Problem(name=f"cube_hole_k{k}", dim=3, coords=coords, elems=elems,
                   D=np.ascontiguousarray(D), kscale=None,
                   f_elem=np.zeros(elems.shape[0]), dirichlet=dirichlet, cells=cells, h=1.0 / n,
                   dirichlet_values=np.ascontiguousarray(dvals), bounds=tuple(bounds))


def config_small() -> Problem:
    """2D unit square, 64x64 cells, theta = pi/6, ratio 1e-3 (3,969 free DOF)."""
    return square2d(64)


def config_cube128() -> Problem:
    """3D unit cube, 128^3 cells (2,146,689 nodes, 2,048,383 free DOF)."""
    return cube3d(128)


def gaussian_random_field(shape: Sequence[int], ell: float, seed: int,
                          pad: Optional[int] = None) -> np.ndarray:
    """Zero-mean, unit-sample-variance field with squared-exponential covariance
    exp(-r^2 / (2 ell^2)) (r, ell in cells), by FFT filtering of iid N(0,1)
    noise on a grid padded by 3*ell cells per side, then cropped.
    Returned array is indexed [x, y, z]."""
    shape = tuple(int(s) for s in shape)
    pad = int(math.ceil(3 * ell)) if pad is None else pad
    pshape = tuple(s + 2 * pad for s in shape)
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(pshape)
    # kernel = Gaussian with std ell/sqrt(2): its self-convolution has std ell.
    sig = ell / math.sqrt(2.0)
    freq = [np.fft.fftfreq(p) for p in pshape[:-1]] + [np.fft.rfftfreq(pshape[-1])]
    grids = np.meshgrid(*freq, indexing="ij", sparse=True)
    k2 = sum(g * g for g in grids)
    transfer = np.exp(-2.0 * (math.pi ** 2) * (sig ** 2) * k2)
    field = np.fft.irfftn(np.fft.rfftn(noise) * transfer, s=pshape, axes=tuple(range(len(pshape))))
    crop = field[tuple(slice(pad, pad + s) for s in shape)]
    crop = crop - crop.mean()
    crop = crop / crop.std()
    return np.ascontiguousarray(crop)


def renumber_nodes(p: Problem, new_id: np.ndarray) -> Problem:
    """The same problem with node o renamed new_id[o] (a permutation):
    coordinates, Dirichlet flags and values move with their nodes, elements
    keep their order and are rewritten in the new ids."""
    new_id = np.asarray(new_id, dtype=np.int64)
    assert new_id.shape == (p.n_nodes,) and np.array_equal(np.sort(new_id), np.arange(p.n_nodes))
    coords = np.empty_like(p.coords)
    coords[new_id] = p.coords
    dirichlet = np.empty_like(p.dirichlet)
    dirichlet[new_id] = p.dirichlet
    dvals = None
    if p.dirichlet_values is not None:
        dvals = np.empty_like(p.dirichlet_values)
        dvals[new_id] = p.dirichlet_values
    return dataclasses.replace(p, coords=coords, dirichlet=dirichlet, dirichlet_values=dvals,
                               elems=np.ascontiguousarray(new_id[p.elems].astype(np.int32)))


def config_transient3d(nx=256, ny=256, nz=64, seed=1506, ell=8.0) -> Problem:
    """256 x 256 x 64 cubic cells (h = 1/256), D_e = exp(G_e) R diag(1, .1, 1e-3) R^T,
    G a seeded Gaussian random field (one value per cell, shared by its 6 tets),
    f = 1 on the central box of each extent; used with backward Euler, dt = 1e-3.
    Nodes are numbered z fastest, then y, then x (the shortest axis first), so
    the widest coupling of the stiffness is (nz + 1)(ny + 1) + nz + 2 = 16771
    rows: column offsets fit int16 (with x fastest they would reach 66307)."""
    cells = (nx, ny, nz)
    G = gaussian_random_field(cells, ell, seed)          # [x, y, z]
    kcell = np.exp(G).transpose(2, 1, 0).ravel()         # cell order: x fastest
    kscale = np.repeat(kcell, 6)
    D0 = aniso3d_tensor((1.0, 0.1, 1e-3))
    p = box_problem(f"transient3d_{nx}x{ny}x{nz}", cells, 1.0 / nx, D0, kscale=kscale)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    new_id = (k + (nz + 1) * (j + (ny + 1) * i)).ravel()   # old ids run x fastest
    return renumber_nodes(p, new_id)


def batch_problem(index: int, seed: int = 8435, nprob: int = 512,
                  n_range=(32, 256)) -> Problem:
    """One member of the seeded batch of independent 2D problems: n ~ U{32..256},
    theta ~ U[0, pi), ratio 10^-a with a ~ U(1, 4), f = 1 on the cells whose
    centroid lies in a random square of side U[0.1, 0.3]."""
    ss = np.random.SeedSequence(seed).spawn(nprob)[index]
    rng = np.random.default_rng(ss)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    theta = float(rng.uniform(0.0, math.pi))
    a = float(rng.uniform(1.0, 4.0))
    side = float(rng.uniform(0.1, 0.3))
    corner = rng.uniform(0.0, 1.0 - side, size=2)
    h = 1.0 / n
    cx = (np.arange(n) + 0.5) * h
    inx = (cx >= corner[0]) & (cx <= corner[0] + side)
    iny = (cx >= corner[1]) & (cx <= corner[1] + side)
    cell_f = (iny[:, None] & inx[None, :]).astype(np.float64).ravel()  # [y, x] -> x fastest
    f_elem = np.repeat(cell_f, 2)
    return box_problem(f"batch{seed}_{index}_n{n}", (n, n), h,
                       aniso2d_tensor(theta, 10.0 ** (-a)), f_elem=f_elem)


# ---------------------------------------------------------------- served request stream
def serve_problem(index: int, seed: int = 50, dof_range=(1e3, 1e6)) -> Problem:
    """One request of the served stream: 2D or 3D with probability 1/2, free
    DOF log-uniform in dof_range.  2D as a batch member (random theta,
    anisotropy 10^-U(1,4), source on a random square of side U[0.1, 0.3]);
    3D with the cube tensor (1, 1e-2, 1e-4) and the source on a random cube
    of side U[0.1, 0.3]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, index]))
    dim = 2 if rng.uniform() < 0.5 else 3
    dof = math.exp(rng.uniform(math.log(dof_range[0]), math.log(dof_range[1])))
    n = max(2, int(round(dof ** (1.0 / dim))) + 1)      # (n-1)^dim free DOF
    side = float(rng.uniform(0.1, 0.3))
    corner = rng.uniform(0.0, 1.0 - side, size=dim)
    h = 1.0 / n
    cx = (np.arange(n) + 0.5) * h
    ins = [(cx >= corner[k]) & (cx <= corner[k] + side) for k in range(dim)]
    if dim == 2:
        theta = float(rng.uniform(0.0, math.pi))
        a = float(rng.uniform(1.0, 4.0))
        cell_f = (ins[1][:, None] & ins[0][None, :]).astype(np.float64).ravel()
        return box_problem(f"serve{seed}_{index}_2d_n{n}", (n, n), h,
                           aniso2d_tensor(theta, 10.0 ** (-a)), f_elem=np.repeat(cell_f, 2))
    cell_f = (ins[2][:, None, None] & ins[1][None, :, None] & ins[0][None, None, :])
    cell_f = cell_f.astype(np.float64).ravel()                      # [z, y, x] -> x fastest
    return box_problem(f"serve{seed}_{index}_3d_n{n}", (n, n, n), h, aniso3d_tensor(),
                       f_elem=np.repeat(cell_f, 6))


def serve_arrivals(nreq: int, rate: float, seed: int = 50) -> np.ndarray:
    """Poisson arrival times (seconds) of nreq requests at `rate` per second."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1 << 20]))
    return np.cumsum(rng.exponential(1.0 / rate, size=nreq))


# ---------------------------------------------------------------- manufactured solution
def mms_problem(dim: int, n: int) -> Problem:
    """c = prod sin(pi x_k) with constant anisotropic D; f = -div(D grad c)
    in closed form, sampled at element centroids."""
    if dim == 2:
        D = aniso2d_tensor(math.pi / 6, 1e-1)
        cells = (n, n)
    else:
        D = aniso3d_tensor((1.0, 0.3, 0.1))
        cells = (n, n, n)
    coords, elems = structured_simplex_mesh(cells, 1.0 / n)
    cen = coords[elems.astype(np.int64)].mean(axis=1)
    pi = math.pi
    s = np.sin(pi * cen)
    co = np.cos(pi * cen)
    # -div(D grad c) = pi^2 [ sum_k D_kk prod s - sum_{k!=l} D_kl co_k co_l prod_{m!=k,l} s_m ]
    f = np.zeros(cen.shape[0])
    prod_s = np.prod(s, axis=1)
    for k in range(dim):
        f += D[k, k] * prod_s
    for k in range(dim):
        for l in range(dim):
            if k == l:
                continue
            term = co[:, k] * co[:, l]
            for m in range(dim):
                if m != k and m != l:
                    term = term * s[:, m]
            f -= D[k, l] * term
    f *= pi * pi

    def exact(x):
        return np.prod(np.sin(pi * x), axis=1)

    p = box_problem(f"mms{dim}d_n{n}", cells, 1.0 / n, D, f_elem=f)
    p.exact = exact
    return p


def tiny2d() -> Problem:
    """4 x 4 cells (9 free DOF), theta = pi/6, ratio 1e-3, f = 1 on cell (1, 1)."""
    return square2d(4)


def tiny3d() -> Problem:
    """3 x 3 x 3 cells (8 free DOF), the cube tensor, f = 1 on the corner cell (0, 0, 0)."""
    cells = (3, 3, 3)
    f = cell_box_indicator(cells, (0, 0, 0), (1, 1, 1))
    return box_problem("tiny3d", cells, 1.0 / 3, aniso3d_tensor(), f_elem=f)


def free_node_ids(p: Problem) -> np.ndarray:
    """Node ids of the free DOFs, in DOF order (ascending node id)."""
    return np.flatnonzero(p.dirichlet == 0)


def solution_on_nodes(p: Problem, c_free: np.ndarray) -> np.ndarray:
    """Scatter a free-DOF vector onto all nodes (Dirichlet nodes hold 0)."""
    out = np.zeros(p.n_nodes)
    out[free_node_ids(p)] = c_free
    return out
