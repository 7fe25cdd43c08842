"""Literal-matrix mini-oracle: the paper's algebraic operators built as sparse matrices.

TEST INFRASTRUCTURE ONLY (tiny meshes).  This is a second, independent CPU path next to the
gather oracle in oracle.c: it builds the incidence, degree, shift, adjacency and normal matrices
of Section 2 and evaluates the face reconstruction theta_f = Pi theta + F(r) d_u and the update
theta + dt M U(u) theta_f of Section 3.1 with those matrices (sparse products and pointwise
operations), a check of the operator equations that Algorithms 3 and 4 evaluate.

Readings (where the printed formulas disagree with each other or with the printed example):
  * oriented incidence E[f, nbr] = +1, E[f, own] = -1, so E theta is the difference along the
    face normal (own -> nbr);
  * face adjacency A_FF = B_CF B_FC - W_FF (non-negative, as printed in the example and as the
    text states);
  * directed adjacency A^D_FF = offdiag(E_CF B_FC): -1 for the faces of the cell the normal
    leaves (behind the face), +1 for the faces of the cell it enters (ahead), as the text says;
  * upstream difference d_U = Q N (I_d (x) A^U) N^T E theta with A^U = (A - Q A^D)/2, i.e.
    d_U = (Q T_CF - S_CF) theta with S_CF = N (I_d (x) A^D) N^T E / 2 and
    T_CF = N (I_d (x) A) N^T E / 2, so that d_U = theta_C - theta_U along the flow (this
    restores the one-dimensional gradient ratio, which the printed (Q S + T) form does not);
  * F(r) = (psi(r) - 1)/2 (Table 1), theta_f = Pi theta + F(r) d_u, with theta_f = Pi theta where
    d_u = 0;
  * divergence M = Omega^{-1} E^T A_F (net inflow per unit volume), theta^{n+1} =
    theta^n + dt M U(u) theta_f.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

R_BIG = 1.0e18


def psi_np(limiter: str, r: np.ndarray) -> np.ndarray:
    """Limiter functions of Sweby's family (superbee as in Table 1), vectorised."""
    r = np.asarray(r, dtype=np.float64)
    big = ~(np.abs(r) <= R_BIG)
    rr = np.where(big, 0.0, r)
    if limiter == "upwind":
        v = np.zeros_like(rr)
        inf_pos, inf_neg = 0.0, 0.0
    elif limiter == "central":
        v = np.ones_like(rr)
        inf_pos, inf_neg = 1.0, 1.0
    elif limiter == "minmod":
        v = np.maximum(0.0, np.minimum(1.0, rr))
        inf_pos, inf_neg = 1.0, 0.0
    elif limiter == "vanleer":
        v = (rr + np.abs(rr)) / (1.0 + np.abs(rr))
        inf_pos, inf_neg = 2.0, 0.0
    elif limiter == "vanalbada":
        v = (rr * rr + rr) / (rr * rr + 1.0)
        inf_pos, inf_neg = 1.0, 1.0
    elif limiter == "superbee":
        v = np.maximum(0.0, np.maximum(np.minimum(1.0, 2.0 * rr), np.minimum(rr, 2.0)))
        inf_pos, inf_neg = 2.0, 0.0
    elif limiter == "smart":
        v = np.maximum(0.0, np.minimum(np.minimum(2.0 * rr, 0.25 + 0.75 * rr), 4.0))
        inf_pos, inf_neg = 4.0, 0.0
    else:
        raise ValueError(limiter)
    return np.where(big, np.where(r > 0, inf_pos, inf_neg), v)


class AlgebraicMesh:
    """The matrices of Section 2 for a mesh given by (own, nbr) and unit normals."""

    def __init__(self, face_cells, face_normal, face_area=None, cell_volume=None, n_cells=None,
                 dim=3):
        fc = np.asarray(face_cells, dtype=np.int64)
        F = fc.shape[0]
        C = int(n_cells) if n_cells is not None else int(fc.max()) + 1
        self.F, self.C, self.d = F, C, dim
        rows = np.repeat(np.arange(F), 2)
        cols = fc.reshape(-1)
        vals = np.tile([-1.0, 1.0], F)
        # oriented incidence E_{C->F} (|F| x |C|), Section 2 incidence matrices
        self.E = sp.csr_matrix((vals, (rows, cols)), shape=(F, C))
        # undirected incidence B = |E| (undirected-incidence equation)
        self.B = abs(self.E).tocsr()
        # degree W_FF = diag(B 1_C) (degree equation)
        w = np.asarray(self.B.sum(axis=1)).ravel()
        self.W = sp.diags(w)
        # shift Pi_{C->F} = W^-1 B (shift equation)
        self.Pi = (sp.diags(1.0 / w) @ self.B).tocsr()
        # face adjacency A_FF = B B^T - W (adjacency-of-faces equation, sign of the printed matrix)
        self.A = (self.B @ self.B.T - self.W).tocsr()
        self.A.eliminate_zeros()
        # directed adjacency A^D_FF = offdiag(E B^T) (directed-adjacency equation, text's sign)
        AD = (self.E @ self.B.T).tolil()
        AD.setdiag(0.0)
        self.AD = AD.tocsr()
        self.AD.eliminate_zeros()
        # normal matrix N_F = (N_1 | ... | N_d) (normal-matrix equation)
        nrm = np.asarray(face_normal, dtype=np.float64)[:, :dim]
        self.N = sp.hstack([sp.diags(nrm[:, k]) for k in range(dim)]).tocsr()
        Id = sp.identity(dim, format="csr")
        # precomputed upstream matrices (simplified upstream-difference equation)
        self.S = (0.5 * self.N @ sp.kron(Id, self.AD) @ self.N.T @ self.E).tocsr()
        self.T = (0.5 * self.N @ sp.kron(Id, self.A) @ self.N.T @ self.E).tocsr()
        a = np.ones(F) if face_area is None else np.asarray(face_area, dtype=np.float64)
        v = np.ones(C) if cell_volume is None else np.asarray(cell_volume, dtype=np.float64)
        # divergence M = Omega^-1 E^T A_F (net inflow per unit volume)
        self.M = (sp.diags(1.0 / v) @ self.E.T @ sp.diags(a)).tocsr()

    @classmethod
    def from_incidence(cls, E, face_normal=None, dim=2) -> "AlgebraicMesh":
        """Matrices from an explicit oriented incidence E_{C->F} (boundary faces allowed)."""
        self = cls.__new__(cls)
        E = sp.csr_matrix(np.asarray(E, dtype=np.float64))
        F, C = E.shape
        self.F, self.C, self.d = F, C, dim
        self.E = E
        self.B = abs(E).tocsr()
        w = np.asarray(self.B.sum(axis=1)).ravel()
        self.W = sp.diags(w)
        self.Pi = (sp.diags(1.0 / w) @ self.B).tocsr()
        self.A = (self.B @ self.B.T - self.W).tocsr()
        self.A.eliminate_zeros()
        AD = (self.E @ self.B.T).tolil()
        AD.setdiag(0.0)
        self.AD = AD.tocsr()
        self.AD.eliminate_zeros()
        return self

    @classmethod
    def from_arrays(cls, m) -> "AlgebraicMesh":
        return cls(m.face_cells, m.face_normal, m.face_area, m.cell_volume, n_cells=m.n_cells,
                   dim=max(m.dim, 1))

    def face_values(self, limiter: str, theta: np.ndarray, u: np.ndarray) -> np.ndarray:
        """theta_f = Pi theta + F(r) o d_u with F = (psi - 1)/2 (Section 3.1 and Table 1), one
        scalar: the face interpolation of Section 2's shift plus the limited correction, from
        d_u = Q E theta (the face-difference equation), d_U from upstream_difference and
        r = d_U / d_u (the gradient-ratio equation; r = 0 where d_u = 0, where the correction
        vanishes whatever r is)."""
        q = np.where(u > 0, 1.0, -1.0)
        d_u = q * (self.E @ theta)
        d_U = self.upstream_difference(theta, u)
        flat = d_u == 0.0
        r = np.where(flat, 0.0, d_U / np.where(flat, 1.0, d_u))
        correction = np.where(flat, 0.0, 0.5 * (psi_np(limiter, r) - 1.0) * d_u)
        return correction + self.Pi @ theta

    def upstream_difference(self, theta: np.ndarray, u: np.ndarray) -> np.ndarray:
        q = np.where(u > 0, 1.0, -1.0)
        return q * (self.T @ theta) - self.S @ theta

    def upstream_difference_unsimplified(self, theta: np.ndarray, u: np.ndarray) -> np.ndarray:
        """d_U = Q N (I (x) A^U) N^T E theta with A^U = (A - Q A^D)/2, built as a matrix."""
        q = np.where(u > 0, 1.0, -1.0)
        Q = sp.diags(q)
        AU = 0.5 * (self.A - Q @ self.AD)
        Id = sp.identity(self.d, format="csr")
        op = Q @ self.N @ sp.kron(Id, AU) @ self.N.T @ self.E
        return op @ theta

    def rhs(self, limiter: str, theta: np.ndarray, u: np.ndarray) -> np.ndarray:
        return self.M @ (u * self.face_values(limiter, theta, u))

    def euler_run(self, limiter: str, dt: float, theta0: np.ndarray, u: np.ndarray, nsteps: int):
        """Algorithm 4 repeated nsteps times."""
        th = np.array(theta0, dtype=np.float64)
        for _ in range(nsteps):
            th = th + dt * self.rhs(limiter, th, u)
        return th
