"""Seeded synthetic workloads shared by the kernels' tests, the oracle's tests and the benchmark.

This module only builds inputs: mesh incidence, renumberings, face velocities, cell fields and
time steps.  It holds none of the flux-limiter arithmetic (no face selection, gradient ratio,
limiter, flux or divergence); both the HIP library and the CPU oracle receive the arrays built
here and nothing else from it.

Mesh model (Section 2 of the paper): a mesh is given by its oriented face-to-cell incidence.
Every face f joins the two cells ``face_cells[f] = (own, nbr)`` and carries a unit normal
``face_normal[f]`` that points from ``own`` into ``nbr``; the oriented incidence is then
``E[f, nbr] = +1`` and ``E[f, own] = -1`` (the difference ``E theta`` is taken along the normal).
A boundary face has one cell: ``face_cells[f] = (own, -1)`` with the normal pointing out of the
mesh (``open_box``); every other mesh built here is periodic, so every face has two cells.

Workload recipes (sizes and distributions of the paper's advection study, Section 4):

* 1-D periodic line of N uniform cells: square wave on [0.2, 0.4] plus a Gaussian of width
  0.05 at x = 0.7, unit velocity, Euler step at CFL 0.5.
* 3-D periodic hexahedral box n^3 in natural or seeded random cell/face numbering with random
  face orientation flips: a solenoidal face velocity from the discrete curl of a seeded random
  edge potential built from Fourier modes with max-norm wavenumber <= 4, and a Gaussian blob at
  the paper's sphere centre (0.35, 0.35, 0.35) plus a sharp tanh step in x.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_VELOCITY = 0
SEED_RENUMBER = 1
SEED_TARGET = 2
SEED_BATCH = 3


@dataclasses.dataclass
class MeshArrays:
    """Plain arrays describing a mesh by its face-to-cell incidence."""

    face_cells: np.ndarray  # int32 [F, 2] (own, nbr)
    face_normal: np.ndarray  # float64 [F, 3], unit, own -> nbr
    face_area: np.ndarray  # float64 [F]
    cell_volume: np.ndarray  # float64 [C]
    n: int = 0  # cells per side of the box it was built from
    dim: int = 0
    # Maps from the natural (lexicographic) numbering to this numbering; identity if None.
    cell_new_of_old: Optional[np.ndarray] = None  # int64 [C]
    face_new_of_old: Optional[np.ndarray] = None  # int64 [F]
    face_flip_old: Optional[np.ndarray] = None  # bool [F], indexed by old face
    # distance between the cell centres across each face (a boundary face: to the mirror image
    # of its cell), for the distance-weighted upstream difference; None: not given
    face_dist: Optional[np.ndarray] = None

    @property
    def n_cells(self) -> int:
        return int(self.cell_volume.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_cells.shape[0])

    def cell_field_from_natural(self, x: np.ndarray) -> np.ndarray:
        """Re-index a cell field given in natural numbering (axis 0) into this mesh's numbering."""
        if self.cell_new_of_old is None:
            return np.ascontiguousarray(x)
        out = np.empty_like(x)
        out[self.cell_new_of_old] = x
        return out

    def cell_field_to_natural(self, x: np.ndarray) -> np.ndarray:
        if self.cell_new_of_old is None:
            return np.ascontiguousarray(x)
        return np.ascontiguousarray(x[self.cell_new_of_old])

    def face_field_from_natural(self, x: np.ndarray) -> np.ndarray:
        """Re-index face data that does not change sign with the orientation (axis 0)."""
        if self.face_new_of_old is None:
            return np.ascontiguousarray(x)
        out = np.empty_like(x)
        out[self.face_new_of_old] = x
        return out

    def face_velocity_from_natural(self, u: np.ndarray) -> np.ndarray:
        """Re-index a normal face velocity from natural numbering; flipped faces change sign."""
        if self.face_new_of_old is None:
            return np.ascontiguousarray(u)
        v = np.where(self.face_flip_old, -u, u) if self.face_flip_old is not None else u
        out = np.empty_like(v)
        out[self.face_new_of_old] = v
        return out


def periodic_box(n: int, dim: int = 3) -> MeshArrays:
    """Periodic box [0,1)^dim with n cells per side in natural numbering.

    Cell (i0, i1, i2) has index i0 + n*i1 + n*n*i2.  Faces come in ``dim`` blocks of C faces:
    face ``a*C + c`` joins cell c (own) to its +e_a neighbour (nbr, wrapped), normal +e_a.
    """
    if dim not in (1, 2, 3):
        raise ValueError("dim must be 1, 2 or 3")
    if n < 1:
        raise ValueError("n must be positive")
    C = n**dim
    c = np.arange(C, dtype=np.int64)
    idx = [(c // n**a) % n for a in range(dim)]
    own = np.empty(dim * C, dtype=np.int32)
    nbr = np.empty(dim * C, dtype=np.int32)
    nrm = np.zeros((dim * C, 3), dtype=np.float64)
    for a in range(dim):
        sl = slice(a * C, (a + 1) * C)
        own[sl] = c
        nbr[sl] = c - idx[a] * n**a + ((idx[a] + 1) % n) * n**a
        nrm[sl, a] = 1.0
    h = 1.0 / n
    face_cells = np.stack([own, nbr], axis=1)
    area = np.full(dim * C, h ** (dim - 1), dtype=np.float64)
    vol = np.full(C, h**dim, dtype=np.float64)
    return MeshArrays(face_cells, nrm, area, vol, n=n, dim=dim)


def open_box(n: int, dim: int = 3, open_axes=(0,)) -> MeshArrays:
    """The box of ``periodic_box(n, dim)`` cut open along ``open_axes``: there the wrapped faces
    become boundary faces on the high side (own = the last cell, normal +e_a) and new boundary
    faces close the low side (own = the first cell, normal -e_a), appended after the dim blocks
    of C faces.  Along the other axes the box stays periodic."""
    base = periodic_box(n, dim)
    C = base.n_cells
    c = np.arange(C, dtype=np.int64)
    fc = base.face_cells.copy()
    nrm = [base.face_normal]
    extra_fc = []
    for a in open_axes:
        if not 0 <= a < dim:
            raise ValueError("open axis out of range")
        ia = (c // n**a) % n
        last = a * C + c[ia == n - 1]
        fc[last, 1] = -1
        first = c[ia == 0]
        extra_fc.append(np.stack([first, -np.ones_like(first)], axis=1).astype(np.int32))
        e = np.zeros((first.shape[0], 3))
        e[:, a] = -1.0
        nrm.append(e)
    face_cells = np.concatenate([fc] + extra_fc, axis=0).astype(np.int32)
    face_normal = np.concatenate(nrm, axis=0)
    area = np.full(face_cells.shape[0], base.face_area[0], dtype=np.float64)
    return MeshArrays(face_cells, face_normal, area, base.cell_volume.copy(), n=n, dim=dim)


def stretched_box(n: int, dim: int = 3, amp: float = 0.5, open_axes=()) -> MeshArrays:
    """periodic_box (open_box along open_axes) with cell widths along x proportional to
    1 + amp sin(2 pi (i + 1/2) / n), summing to 1, and uniform widths 1/n along the other axes:
    face areas, cell volumes and the face distances between cell centres follow (a boundary
    face's distance is its cell's width along the face normal: to the cell's mirror image)."""
    m = open_box(n, dim, tuple(open_axes)) if open_axes else periodic_box(n, dim)
    i = np.arange(n)
    hx = 1.0 + amp * np.sin(2 * np.pi * (i + 0.5) / n)
    hx /= hx.sum()
    h = 1.0 / n
    C = m.n_cells
    c = np.arange(C, dtype=np.int64)
    wx = hx[c % n]  # x width of every cell
    own = m.face_cells[:, 0].astype(np.int64)
    nbr = m.face_cells[:, 1].astype(np.int64)
    axis = np.abs(m.face_normal).argmax(axis=1)
    dist = np.full(m.n_faces, h)
    x = axis == 0
    inner = nbr >= 0
    dist[x & inner] = 0.5 * (wx[own[x & inner]] + wx[nbr[x & inner]])
    dist[x & ~inner] = wx[own[x & ~inner]]
    area = np.where(x, h ** (dim - 1), wx[own] * h ** max(dim - 2, 0))
    vol = wx * h ** (dim - 1)
    return dataclasses.replace(m, face_area=area, cell_volume=vol, face_dist=dist)


def face_centres(mesh: MeshArrays) -> np.ndarray:
    """Face centres [F, 3] of a box built by periodic_box or open_box (natural numbering): the
    own cell's centre moved half a cell along the face normal."""
    n, dim = mesh.n, mesh.dim
    c = mesh.face_cells[:, 0].astype(np.int64)
    x = np.zeros((mesh.n_faces, 3))
    for a in range(dim):
        x[:, a] = ((c // n**a) % n + 0.5) / n
    return x + 0.5 / n * mesh.face_normal


def velocity_open_box(mesh: MeshArrays) -> np.ndarray:
    """A smooth face velocity on a box cut open along x: u_x = 0.3 + cos(2 pi y) cos(2 pi z)
    (every open side has inflow and outflow faces), u_y = 0.5 sin(2 pi x + 1),
    u_z = 0.4 cos(2 pi (x + y)); the normal component of that field on each face."""
    x = face_centres(mesh)
    v = np.stack([0.3 + np.cos(2 * np.pi * x[:, 1]) * np.cos(2 * np.pi * x[:, 2]),
                  0.5 * np.sin(2 * np.pi * x[:, 0] + 1.0),
                  0.4 * np.cos(2 * np.pi * (x[:, 0] + x[:, 1]))], axis=1)
    return np.einsum("fa,fa->f", v, mesh.face_normal)


def inflow_values(mesh: MeshArrays, u: Optional[np.ndarray] = None, S: int = 1) -> np.ndarray:
    """Inflow values [F] (or [F, S]) of a box's boundary faces: 0.8 + 0.15 sin(2 pi (y + 2z))
    (+0.1 per extra scalar); NaN on the interior faces, and on the outflow boundary faces
    (u_f > 0) when u is given, so that a read of a value the boundary rule never uses shows."""
    x = face_centres(mesh)
    v = 0.8 + 0.15 * np.sin(2 * np.pi * (x[:, 1] + 2 * x[:, 2]))
    out = np.stack([v + 0.1 * k for k in range(S)], axis=1) if S > 1 else v.copy()
    unused = mesh.face_cells[:, 1] >= 0
    if u is not None:
        unused |= u > 0.0
    out[unused] = np.nan
    return out


def periodic_triangles(n: int) -> MeshArrays:
    """Periodic square [0,1)^2 cut into n x n squares, each split by its diagonal from (i, j) to
    (i+1, j+1) into a lower triangle (cell 2 (i + n j)) and an upper one (cell 2 (i + n j) + 1).

    Faces (3 n^2, each block in square order i + n j): horizontal edges (own = the upper triangle
    below, nbr = the lower triangle above, normal +y), vertical edges (own = the lower triangle
    to the left, nbr = the upper triangle to the right, normal +x), diagonals (own = lower,
    nbr = upper, normal (-1, 1)/sqrt(2)).  Face areas are edge lengths, cell volumes h^2 / 2.
    The faces of a triangle do not come in opposite pairs, and each face side projects on one or
    two faces with weights +-1/sqrt(2): the general cells of the upstream difference.
    """
    if n < 3:
        raise ValueError("n must be at least 3")
    C2 = n * n
    sq = np.arange(C2, dtype=np.int64)
    i, j = sq % n, sq // n
    lower = lambda ii, jj: 2 * ((ii % n) + n * (jj % n))
    upper = lambda ii, jj: 2 * ((ii % n) + n * (jj % n)) + 1
    own = np.concatenate([upper(i, j - 1), lower(i - 1, j), lower(i, j)]).astype(np.int32)
    nbr = np.concatenate([lower(i, j), upper(i, j), upper(i, j)]).astype(np.int32)
    nrm = np.zeros((3 * C2, 3))
    nrm[:C2, 1] = 1.0
    nrm[C2:2 * C2, 0] = 1.0
    r2 = 1.0 / math.sqrt(2.0)
    nrm[2 * C2:, 0] = -r2
    nrm[2 * C2:, 1] = r2
    h = 1.0 / n
    area = np.concatenate([np.full(2 * C2, h), np.full(C2, h * math.sqrt(2.0))])
    vol = np.full(2 * C2, 0.5 * h * h)
    return MeshArrays(np.stack([own, nbr], axis=1), nrm, area, vol, n=n, dim=2)


def triangle_centroids(n: int) -> np.ndarray:
    """Centroids [2 n^2, 2] of periodic_triangles(n)."""
    sq = np.arange(n * n)
    i, j = sq % n, sq // n
    h = 1.0 / n
    out = np.empty((2 * n * n, 2))
    out[0::2, 0], out[0::2, 1] = (i + 2.0 / 3.0) * h, (j + 1.0 / 3.0) * h
    out[1::2, 0], out[1::2, 1] = (i + 1.0 / 3.0) * h, (j + 2.0 / 3.0) * h
    return out


def velocity_stream_triangles(n: int, seed: int = SEED_VELOCITY, kmax: int = 3) -> np.ndarray:
    """Solenoidal face velocity of periodic_triangles(n): a seeded periodic stream function psi
    sampled at the vertices (rounded to multiples of 2^-40), the flux through an edge from A to B
    with normal (t_y, -t_x) is psi(B) - psi(A), and u_f is that flux over the edge length.  The
    fluxes of every triangle sum to zero exactly; scaled so that max |u_f| is about 1."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="ij")  # X[i, j] = i h
    psi = np.zeros((n, n))
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if (kx, ky) == (0, 0):
                continue
            a, b = rng.standard_normal(2) / (kx * kx + ky * ky)
            ph = 2 * np.pi * (kx * X + ky * Y)
            psi += a * np.cos(ph) + b * np.sin(ph)
    P = lambda ii, jj: psi[ii % n, jj % n]
    sq = np.arange(n * n)
    i, j = sq % n, sq // n
    q = np.concatenate([P(i, j) - P(i + 1, j), P(i, j + 1) - P(i, j), P(i, j) - P(i + 1, j + 1)])
    ln = np.concatenate([np.full(2 * n * n, h), np.full(n * n, h * math.sqrt(2.0))])
    scale = 1.0 / float(np.abs(q / ln).max())
    psi = np.round(psi * scale * 2.0**40) / 2.0**40
    q = np.concatenate([P(i, j) - P(i + 1, j), P(i, j + 1) - P(i, j), P(i, j) - P(i + 1, j + 1)])
    return q / ln


def periodic_skewed_box(n: int, shear: float = 0.3) -> MeshArrays:
    """periodic_box(n, 3)'s incidence on a sheared lattice: cell (i, j, k) spans
    i a1 + j a2 + k a3 with a1 = (h, 0, 0), a2 = (shear h, h, 0), a3 = (0, shear h, h).  Faces
    are parallelograms with unit normals a2 x a3, a3 x a1, a1 x a2 (normalised, pointing to the
    + neighbour), areas |a2 x a3| etc., volumes a1 . (a2 x a3).  Opposite faces still pair up, but
    neighbouring faces are no longer orthogonal: every face side projects on five faces."""
    m = periodic_box(n, 3)
    h = 1.0 / n
    a = [np.array([h, 0.0, 0.0]), np.array([shear * h, h, 0.0]), np.array([0.0, shear * h, h])]
    C = n**3
    nrm = np.empty((3 * C, 3))
    area = np.empty(3 * C)
    for d in range(3):
        cr = np.cross(a[(d + 1) % 3], a[(d + 2) % 3])
        if cr @ a[d] < 0:
            cr = -cr
        nrm[d * C:(d + 1) * C] = cr / np.linalg.norm(cr)
        area[d * C:(d + 1) * C] = np.linalg.norm(cr)
    vol = np.full(C, abs(a[0] @ np.cross(a[1], a[2])))
    return MeshArrays(m.face_cells, nrm, area, vol, n=n, dim=3)


def renumber(mesh: MeshArrays, seed: int = SEED_RENUMBER, flip: bool = True) -> MeshArrays:
    """Randomly renumber cells and faces (and flip each face's orientation with probability 1/2).

    The result describes the same mesh; fields move with ``cell_field_from_natural`` and
    ``face_velocity_from_natural``.
    """
    rng = np.random.default_rng(seed)
    C, F = mesh.n_cells, mesh.n_faces
    cnew = rng.permutation(C).astype(np.int64)
    fnew = rng.permutation(F).astype(np.int64)
    flips = (rng.random(F) < 0.5) if flip else np.zeros(F, dtype=bool)
    bnd = mesh.face_cells[:, 1] < 0
    flips &= ~bnd  # a boundary face keeps its one cell as own (normal pointing out)
    own = cnew[mesh.face_cells[:, 0]]
    nbr = np.where(bnd, -1, cnew[np.maximum(mesh.face_cells[:, 1], 0)])
    own2 = np.where(flips, nbr, own)
    nbr2 = np.where(flips, own, nbr)
    fc = np.empty((F, 2), dtype=np.int32)
    fc[fnew, 0] = own2
    fc[fnew, 1] = nbr2
    nrm = np.empty_like(mesh.face_normal)
    nrm[fnew] = np.where(flips[:, None], -mesh.face_normal, mesh.face_normal)
    area = np.empty_like(mesh.face_area)
    area[fnew] = mesh.face_area
    vol = np.empty_like(mesh.cell_volume)
    vol[cnew] = mesh.cell_volume
    dist = None
    if mesh.face_dist is not None:
        dist = np.empty_like(mesh.face_dist)
        dist[fnew] = mesh.face_dist
    return MeshArrays(fc, nrm, area, vol, n=mesh.n, dim=mesh.dim,
                      cell_new_of_old=cnew, face_new_of_old=fnew, face_flip_old=flips,
                      face_dist=dist)


# ---------------------------------------------------------------------------------------------
# Velocities
# ---------------------------------------------------------------------------------------------

def velocity_uniform(mesh: MeshArrays, direction=(1.0, 0.0, 0.0), speed: float = 1.0) -> np.ndarray:
    """Normal face velocity u_f = speed * (direction . n_f) of a constant vector field."""
    d = np.asarray(direction, dtype=np.float64)
    return speed * (mesh.face_normal @ d)


def _edge_potential(n: int, seed: int, kmax: int) -> list:
    """Seeded random edge potential A_d sampled at the midpoints of the d-directed edges.

    A_d(x) = sum over integer wavevectors k with 1 <= |k|_inf <= kmax of Re(a_{d,k} e^{2 pi i k.x}),
    a_{d,k} complex standard normal.  Edge (d, v) runs from vertex v*h to v*h + h*e_d; its
    midpoint carries the half-cell phase shift along d.
    """
    rng = np.random.default_rng(seed)
    K = 2 * kmax + 1
    ks = np.arange(-kmax, kmax + 1)
    out = []
    for d in range(3):
        coef = rng.standard_normal((K, K, K)) + 1j * rng.standard_normal((K, K, K))
        coef[kmax, kmax, kmax] = 0.0
        kd = [ks, ks, ks][d]
        shape = [1, 1, 1]
        shape[d] = K
        coef = coef * np.exp(1j * math.pi * kd / n).reshape(shape)  # midpoint shift along d
        spec = np.zeros((n, n, n), dtype=np.complex128)
        ii = np.mod(ks, n)
        np.add.at(spec, np.ix_(ii, ii, ii), coef)
        field = np.fft.ifftn(spec) * float(n**3)
        out.append(np.ascontiguousarray(field.real))  # indexed [i0, i1, i2]
        del spec, field
    return out


def velocity_curl(n: int, seed: int = SEED_VELOCITY, kmax: int = 4) -> np.ndarray:
    """Solenoidal normal face velocity of ``periodic_box(n, 3)`` (natural face numbering).

    u_f is the circulation of the edge potential around face f divided by the face area: the
    discrete curl, so the discrete divergence of u vanishes (exact sequence, Section 2).  The
    potential is scaled so max|u_f| is about 1 and rounded to multiples of 2^-40 so that every
    circulation, and every cell's flux balance, is computed without rounding.
    """
    if n < 3:
        raise ValueError("n must be >= 3")
    A = _edge_potential(n, seed, kmax)

    def circulation(A):
        circ = []
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            # face (a, cell i) sits at vertex v = i + e_a; edges b at v, c at v+e_b, b at v+e_c, c at v
            v = lambda arr, sh: np.roll(arr, shift=[-s for s in sh], axis=(0, 1, 2))
            ea = [0, 0, 0]; ea[a] = 1
            eab = list(ea); eab[b] += 1
            eac = list(ea); eac[c] += 1
            s = v(A[b], ea) + v(A[c], eab) - v(A[b], eac) - v(A[c], ea)
            circ.append(s)
        return circ

    circ = circulation(A)
    umax = max(float(np.abs(cc).max()) for cc in circ) * n
    q = 2.0**-40
    A = [np.round(a / umax / q) * q for a in A]
    circ = circulation(A)
    # natural face numbering: face a*C + c with c = i0 + n*i1 + n^2*i2 -> Fortran order of [i0,i1,i2]
    u = np.concatenate([(cc * n).ravel(order="F") for cc in circ])
    return u


def velocity_deformation(n: int) -> np.ndarray:
    """Normal face velocity of the deformation flow of Section 4.1 on periodic_box(n, 3):
    u = 2 sin^2(pi x) sin(2 pi y) sin(2 pi z), v = -sin(2 pi x) sin^2(pi y) sin(2 pi z),
    w = -sin(2 pi x) sin(2 pi y) sin^2(pi z) (times cos(pi t / T), applied per stage).

    Each face carries the exact integral of the field over the face divided by its area, so the
    flux balance of every cell is the integral of div u = 0 (to rounding).  The normal component
    vanishes on the planes x, y, z in {0, 1}, so the periodic wrap carries no flux."""
    h = 1.0 / n
    lo = np.arange(n) * h
    hi = lo + h
    sin2_at = np.sin(np.pi * hi) ** 2                  # sin^2 at the +face plane of cell i
    isin = (np.cos(2 * np.pi * lo) - np.cos(2 * np.pi * hi)) / (2 * np.pi)  # int of sin(2 pi t)
    out = []
    # axis 0 (x-faces at x = (i+1)h): 2 sin^2(pi x_f) * isin(y) * isin(z)
    fx = 2.0 * sin2_at[:, None, None] * isin[None, :, None] * isin[None, None, :]
    fy = -isin[:, None, None] * sin2_at[None, :, None] * isin[None, None, :]
    fz = -isin[:, None, None] * isin[None, :, None] * sin2_at[None, None, :]
    for f in (fx, fy, fz):
        out.append((f / (h * h)).ravel(order="F"))  # index i + n j + n^2 k
    return np.concatenate(out)


def deformation_scales(n_steps: int, dt: float, period: float, scheme: str) -> np.ndarray:
    """cos(pi t / period) at every stage time (Euler: t_i; SSP-RK3: t_i, t_i + dt, t_i + dt/2),
    t_i = i dt."""
    offs = [0.0] if scheme == "euler" else [0.0, 1.0, 0.5]
    t = np.array([i * dt + c * dt for i in range(n_steps) for c in offs])
    return np.cos(np.pi * t / period)


def workload_deformation(n: int, cfl: float = 0.4, period: float = 3.0,
                         scheme: str = "ssprk3") -> Workload:
    """Section 4.1 benchmark: sphere of radius 0.15 at (0.35, 0.35, 0.35) in the deformation
    flow, reversed by cos(pi t / T) so it returns to its initial shape at t = T = 3."""
    mesh = periodic_box(n, 3)
    u = velocity_deformation(n)
    dt0 = cfl_dt(mesh, u, cfl)
    steps = int(math.ceil(period / dt0))
    return Workload(mesh, field_sphere(n), u, period / steps, steps, scheme, f"deformation{n}")


def velocity_1d(mesh: MeshArrays, speed: float = 1.0) -> np.ndarray:
    return velocity_uniform(mesh, (1.0, 0.0, 0.0), speed)


# ---------------------------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------------------------

def cell_centres(n: int, dim: int) -> np.ndarray:
    """Cell centres [C, dim] of periodic_box(n, dim) in natural numbering."""
    C = n**dim
    c = np.arange(C, dtype=np.int64)
    return np.stack([((c // n**a) % n + 0.5) / n for a in range(dim)], axis=1)


def field_square_gauss_1d(n: int) -> np.ndarray:
    """Square wave on [0.2, 0.4] plus a Gaussian (sigma 0.05) centred at 0.7."""
    x = cell_centres(n, 1)[:, 0]
    sq = ((x >= 0.2) & (x <= 0.4)).astype(np.float64)
    return sq + np.exp(-((x - 0.7) ** 2) / (2 * 0.05**2))


def field_blob_step(n: int, centre=(0.35, 0.35, 0.35), sigma: float = 0.08, width: float = 0.01,
                    step_at: float = 0.5, x: Optional[np.ndarray] = None) -> np.ndarray:
    """Periodic Gaussian blob plus a tanh step in x (natural numbering of periodic_box(n, 3));
    x may pass precomputed cell_centres(n, 3)."""
    if x is None:
        x = cell_centres(n, 3)
    d = np.abs(x - np.asarray(centre)[None, :])
    d = np.minimum(d, 1.0 - d)
    r2 = (d * d).sum(axis=1)
    return np.exp(-r2 / (2 * sigma**2)) + 0.5 * (1.0 + np.tanh((x[:, 0] - step_at) / width))


def field_sphere(n: int, centre=(0.35, 0.35, 0.35), radius: float = 0.15) -> np.ndarray:
    """Indicator of the sphere used by the paper's deformation benchmark (Section 4.1)."""
    x = cell_centres(n, 3)
    r2 = ((x - np.asarray(centre)[None, :]) ** 2).sum(axis=1)
    return (r2 <= radius * radius).astype(np.float64)


def field_smooth_random(n: int, dim: int, seed: int, kmax: int = 3) -> np.ndarray:
    """Seeded smooth periodic field: a few low Fourier modes, O(1) amplitude."""
    rng = np.random.default_rng(seed)
    x = cell_centres(n, dim)
    out = np.zeros(x.shape[0])
    for _ in range(8):
        k = rng.integers(-kmax, kmax + 1, size=dim)
        ph = rng.uniform(0, 2 * math.pi)
        out += rng.standard_normal() * np.cos(2 * math.pi * (x @ k) + ph)
    return 0.25 * out


def multi_scalar(fields: list) -> np.ndarray:
    """Stack S cell fields into the [C][S] layout (scalar index fastest)."""
    return np.ascontiguousarray(np.stack(fields, axis=1))


# ---------------------------------------------------------------------------------------------
# Time step
# ---------------------------------------------------------------------------------------------

def cfl_dt(mesh: MeshArrays, u: np.ndarray, cfl: float) -> float:
    """dt = cfl / max_c (1/V_c) * sum of the outgoing volumetric fluxes of cell c."""
    own = mesh.face_cells[:, 0].astype(np.int64)
    nbr = mesh.face_cells[:, 1].astype(np.int64)
    q = mesh.face_area * u
    inner = nbr >= 0  # a boundary face's inflow leaves no cell
    # one pass in the order of a loop over the own sides, then the nbr sides of the faces
    out = np.bincount(np.concatenate([own, nbr[inner]]),
                      weights=np.concatenate([np.maximum(q, 0.0), np.maximum(-q[inner], 0.0)]),
                      minlength=mesh.n_cells)
    rate = float((out / mesh.cell_volume).max())
    if rate <= 0.0:
        raise ValueError("velocity is zero everywhere")
    return cfl / rate


# ---------------------------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    mesh: MeshArrays
    theta0: np.ndarray  # [C] or [C][S], mesh numbering
    u: np.ndarray  # [F], mesh numbering
    dt: float
    steps: int
    scheme: str  # "euler" | "ssprk3"
    name: str
    inflow: Optional[np.ndarray] = None  # [F] or [F][S] inflow values of the boundary faces


def workload_line(n: int = 200, cfl: float = 0.5, steps: int = 400) -> Workload:
    """1-D periodic line, square wave + Gaussian, u = 1, Euler, dt = cfl*h (one period at 400)."""
    mesh = periodic_box(n, 1)
    u = velocity_1d(mesh)
    return Workload(mesh, field_square_gauss_1d(n), u, cfl / n, steps, "euler", f"line{n}")


def workload_box(n: int, renumbered: bool = False, cfl: float = 0.4, steps: int = 100,
                 seed_velocity: int = SEED_VELOCITY, seed_renumber: int = SEED_RENUMBER) -> Workload:
    """3-D periodic hex box with the curl velocity and the blob + step field, SSP-RK3."""
    mesh = periodic_box(n, 3)
    u = velocity_curl(n, seed_velocity)
    th = field_blob_step(n)
    if renumbered:
        mesh = renumber(mesh, seed_renumber)
        u = mesh.face_velocity_from_natural(u)
        th = mesh.cell_field_from_natural(th)
    dt = cfl_dt(mesh, u, cfl)
    name = f"box{n}" + ("_random" if renumbered else "")
    return Workload(mesh, th, u, dt, steps, "ssprk3", name)


def workload_open_box(n: int, renumbered: bool = False, cfl: float = 0.4, steps: int = 40,
                      S: int = 1) -> Workload:
    """A box cut open along x (boundary faces on both x sides, periodic in y and z) with the
    smooth velocity of velocity_open_box, the blob + step field (S scalars: shifted copies) and
    SSP-RK3; the inflow values come from inflow_values(mesh, u, S)."""
    mesh = open_box(n, 3, (0,))
    u = velocity_open_box(mesh)
    th = field_blob_step(n)
    if S > 1:
        th = multi_scalar([th + 0.1 * k for k in range(S)])
    inflow = inflow_values(mesh, u, S)
    if renumbered:
        mesh = renumber(mesh, SEED_RENUMBER)
        u = mesh.face_velocity_from_natural(u)
        th = mesh.cell_field_from_natural(th)
        inflow = mesh.face_field_from_natural(inflow)
    dt = cfl_dt(mesh, u, cfl)
    return Workload(mesh, th, u, dt, steps, "ssprk3",
                    f"openbox{n}" + ("_random" if renumbered else ""), inflow)


def box_shared_cache(n: int) -> MeshArrays:
    """periodic_box(n, 3), memoised: batched workloads reuse one mesh per side length."""
    m = _BOX_CACHE.get(n)
    if m is None:
        m = periodic_box(n, 3)
        _BOX_CACHE[n] = m
    return m


_BOX_CACHE: dict = {}


@dataclasses.dataclass
class BatchProblem:
    n: int
    n_scalars: int
    limiter: int
    cfl: float
    seed: int


def batch_recipe(count: int = 512, side_min: int = 12, side_max: int = 96, s_max: int = 8,
                 limiters=(1, 2, 3, 4, 5), cfl_range=(0.2, 0.5), seed: int = SEED_BATCH) -> list:
    """Per-problem side, scalar count, limiter id, CFL and velocity seed of a batched workload."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(BatchProblem(
            n=int(rng.integers(side_min, side_max + 1)),
            n_scalars=int(rng.integers(1, s_max + 1)),
            limiter=int(rng.choice(np.asarray(limiters))),
            cfl=float(rng.uniform(*cfl_range)),
            seed=1000 + i,
        ))
    return out


def batch_fields(p: BatchProblem) -> np.ndarray:
    """[C][S] initial fields of one batched problem: shifted blobs plus steps, seeded."""
    rng = np.random.default_rng(p.seed)
    x = cell_centres(p.n, 3)
    fs = []
    for s in range(p.n_scalars):
        c = tuple(rng.uniform(0.2, 0.8, size=3))
        fs.append(field_blob_step(p.n, centre=c, sigma=0.08 + 0.02 * s, width=0.02,
                                  step_at=float(rng.uniform(0.3, 0.7)), x=x))
    return multi_scalar(fs)
