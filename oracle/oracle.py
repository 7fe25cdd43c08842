"""ctypes binding of the CPU FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU
baseline.  The HIP library and its Python binding never import this module.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

UPWIND, MINMOD, VANLEER, VANALBADA, SUPERBEE, SMART, CENTRAL = range(7)
EULER, SSPRK3 = 1, 3
LIMITERS = {"upwind": UPWIND, "minmod": MINMOD, "vanleer": VANLEER, "vanalbada": VANALBADA,
            "superbee": SUPERBEE, "smart": SMART, "central": CENTRAL}
R_BIG = 1.0e18


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", LIB_PATH, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_mesh_new.restype = _P
        L.orc_mesh_new.argtypes = [_I64, _I64, _P, _P, _P, _P]
        L.orc_mesh_free.argtypes = [_P]
        L.orc_cell_degree.restype = _I64
        L.orc_cell_degree.argtypes = [_P, _I64]
        L.orc_boundary_faces.restype = _I64
        L.orc_boundary_faces.argtypes = [_P]
        L.orc_mesh_set_inflow.argtypes = [_P, _P, _I]
        L.orc_mesh_set_distances.argtypes = [_P, _P]
        L.orc_psi.restype = _D
        L.orc_psi.argtypes = [_I, _D]
        L.orc_dpsi.restype = _D
        L.orc_dpsi.argtypes = [_I, _D]
        L.orc_psi_inf.restype = _D
        L.orc_psi_inf.argtypes = [_I, _I]
        L.orc_select.argtypes = [_P, _P, _P]
        L.orc_side_weights.restype = _I
        L.orc_side_weights.argtypes = [_P, _I64, _I, _P, _P, _I]
        L.orc_face_values.argtypes = [_P, _I, _I, _P, _P, _P]
        L.orc_rhs.argtypes = [_P, _I, _I, _P, _P, _P]
        L.orc_rhs_cells.argtypes = [_P, _I, _I, _P, _P, _I64, _P, _P]
        L.orc_run.restype = _I
        L.orc_run.argtypes = [_P, _I, _I, _D, _I, _I64, _P, _P]
        L.orc_rhs_jvp.argtypes = [_P, _I, _I, _P, _P, _P, _P, _P]
        L.orc_face_values_jvp.argtypes = [_P, _I, _I, _P, _P, _P, _P, _P]
        L.orc_rhs_vjp.argtypes = [_P, _I, _I, _P, _P, _P, _P, _P]
        L.orc_run_tangent.restype = _I
        L.orc_run_tangent.argtypes = [_P, _I, _I, _D, _I, _I64, _P, _P, _P, _P]
        L.orc_run_adjoint.restype = _I
        L.orc_run_adjoint.argtypes = [_P, _I, _I, _D, _I, _I64, _P, _P, _P, _P, _P]
        L.orc_run_scaled.restype = _I
        L.orc_run_scaled.argtypes = [_P, _I, _I, _D, _I, _I64, _P, _P, _P]
        L.orc_num_threads.restype = _I
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def lim_id(limiter) -> int:
    return LIMITERS[limiter] if isinstance(limiter, str) else int(limiter)


def psi(limiter, r: float) -> float:
    return lib().orc_psi(lim_id(limiter), float(r))


def dpsi(limiter, r: float) -> float:
    return lib().orc_dpsi(lim_id(limiter), float(r))


def num_threads() -> int:
    return lib().orc_num_threads()


class OracleMesh:
    """Oracle view of a mesh; keeps its own copies of the arrays alive."""

    def __init__(self, face_cells, face_normal, face_area=None, cell_volume=None, n_cells=None):
        self.fc = np.ascontiguousarray(face_cells, dtype=np.int32)
        self.nrm = _f64(face_normal)
        F = self.fc.shape[0]
        C = int(n_cells) if n_cells is not None else int(self.fc.max()) + 1
        self.area = _f64(face_area) if face_area is not None else np.ones(F)
        self.vol = _f64(cell_volume) if cell_volume is not None else np.ones(C)
        self.n_cells, self.n_faces = C, F
        h = lib().orc_mesh_new(C, F, _ptr(self.fc), _ptr(self.nrm), _ptr(self.area), _ptr(self.vol))
        if not h:
            raise ValueError("oracle rejected the mesh (index out of range or own == nbr)")
        self._h = h
        self.n_boundary = int(lib().orc_boundary_faces(h))
        self._inflow = None
        self._dist = None

    def set_distances(self, dist) -> None:
        """Face distances [F] (Algorithm 1D / UNS weighting of the upstream difference), or
        None for the unweighted form.  Forward functions only."""
        if dist is None:
            self._dist = None
            lib().orc_mesh_set_distances(self._h, None)
            return
        d = _f64(dist)
        if d.shape != (self.n_faces,) or not np.all(d > 0) or not np.all(np.isfinite(d)):
            raise ValueError("distances must be finite, positive, one per face")
        self._dist = d
        lib().orc_mesh_set_distances(self._h, _ptr(d))

    def set_inflow(self, values) -> None:
        """Inflow values of the boundary faces ([F] or [F, S], read where u_f <= 0 on boundary
        faces only), or None: the exterior then repeats the interior cell's value.  Every later
        call must use the same number of scalars."""
        if values is None:
            self._inflow = None
            lib().orc_mesh_set_inflow(self._h, None, 0)
            return
        v = _f64(values)
        if v.shape[0] != self.n_faces:
            raise ValueError("inflow values need one row per face")
        self._inflow = v
        lib().orc_mesh_set_inflow(self._h, _ptr(v), self._S(v))

    def _check_S(self, theta: np.ndarray) -> None:
        if self._inflow is not None and self._S(self._inflow) != self._S(theta):
            raise ValueError("the inflow values were set for another number of scalars")

    @classmethod
    def from_arrays(cls, m) -> "OracleMesh":
        return cls(m.face_cells, m.face_normal, m.face_area, m.cell_volume, n_cells=m.n_cells)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_mesh_free(h)
            self._h = None

    def degree(self, c: int) -> int:
        return int(lib().orc_cell_degree(self._h, c))

    # -- operator -----------------------------------------------------------------------------
    @staticmethod
    def _S(theta: np.ndarray) -> int:
        return 1 if theta.ndim == 1 else int(theta.shape[1])

    def select(self, u) -> np.ndarray:
        u = _f64(u)
        out = np.empty((self.n_faces, 3), dtype=np.int32)
        lib().orc_select(self._h, _ptr(u), _ptr(out))
        return out

    def side_weights(self, f: int, side_nbr: bool):
        w = np.zeros(64)
        fa = np.zeros(64, dtype=np.int32)
        k = lib().orc_side_weights(self._h, f, int(side_nbr), _ptr(w), _ptr(fa), 64)
        return fa[:k].copy(), w[:k].copy()

    def face_values(self, limiter, theta, u) -> np.ndarray:
        theta, u = _f64(theta), _f64(u)
        self._check_S(theta)
        out = np.empty((self.n_faces,) + theta.shape[1:])
        lib().orc_face_values(self._h, lim_id(limiter), self._S(theta), _ptr(theta), _ptr(u),
                              _ptr(out))
        return out

    def face_values_jvp(self, limiter, theta, u, dtheta):
        """(theta_f, its tangent along dtheta), u held fixed."""
        self._check_S(theta)
        theta, u, dtheta = _f64(theta), _f64(u), _f64(dtheta)
        tf = np.empty((self.n_faces,) + theta.shape[1:])
        dtf = np.empty_like(tf)
        lib().orc_face_values_jvp(self._h, lim_id(limiter), self._S(theta), _ptr(theta), _ptr(u),
                                  _ptr(dtheta), _ptr(tf), _ptr(dtf))
        return tf, dtf

    def rhs(self, limiter, theta, u) -> np.ndarray:
        theta, u = _f64(theta), _f64(u)
        self._check_S(theta)
        out = np.empty_like(theta)
        lib().orc_rhs(self._h, lim_id(limiter), self._S(theta), _ptr(theta), _ptr(u), _ptr(out))
        return out

    def rhs_cells(self, limiter, theta, u, cells) -> np.ndarray:
        theta, u = _f64(theta), _f64(u)
        self._check_S(theta)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((cells.shape[0],) + theta.shape[1:])
        lib().orc_rhs_cells(self._h, lim_id(limiter), self._S(theta), _ptr(theta), _ptr(u),
                            cells.shape[0], _ptr(cells), _ptr(out))
        return out

    def run(self, limiter, scheme, dt, theta0, u, nsteps) -> np.ndarray:
        th = _f64(theta0).copy()
        self._check_S(th)
        u = _f64(u)
        sc = {"euler": EULER, "ssprk3": SSPRK3}.get(scheme, scheme)
        rc = lib().orc_run(self._h, lim_id(limiter), int(sc), float(dt), self._S(th), int(nsteps),
                           _ptr(th), _ptr(u))
        if rc != 0:
            raise ValueError("bad scheme")
        return th

    def run_scaled(self, limiter, scheme, dt, theta0, u, scales) -> np.ndarray:
        th = _f64(theta0).copy()
        self._check_S(th)
        u = _f64(u)
        sc = {"euler": EULER, "ssprk3": SSPRK3}.get(scheme, scheme)
        scales = _f64(scales)
        ns = 1 if sc == EULER else 3
        if scales.size % ns:
            raise ValueError("scales must hold stages * n_steps values")
        rc = lib().orc_run_scaled(self._h, lim_id(limiter), int(sc), float(dt), self._S(th),
                                  scales.size // ns, _ptr(th), _ptr(u), _ptr(scales))
        if rc != 0:
            raise ValueError("bad scheme")
        return th

    def rhs_jvp(self, limiter, theta, u, dtheta, du=None) -> np.ndarray:
        self._check_S(theta)
        theta, u, dtheta = _f64(theta), _f64(u), _f64(dtheta)
        out = np.empty_like(theta)
        dup = _ptr(_f64(du)) if du is not None else None
        duk = _f64(du) if du is not None else None
        lib().orc_rhs_jvp(self._h, lim_id(limiter), self._S(theta), _ptr(theta), _ptr(u),
                          _ptr(dtheta), _ptr(duk) if duk is not None else None, _ptr(out))
        del dup
        return out

    def rhs_vjp(self, limiter, theta, u, lam):
        self._check_S(theta)
        theta, u, lam = _f64(theta), _f64(u), _f64(lam)
        tb = np.empty_like(theta)
        ub = np.empty(self.n_faces)
        lib().orc_rhs_vjp(self._h, lim_id(limiter), self._S(theta), _ptr(theta), _ptr(u),
                          _ptr(lam), _ptr(tb), _ptr(ub))
        return tb, ub

    def run_tangent(self, limiter, scheme, dt, theta0, u, nsteps, dtheta0, du=None):
        self._check_S(theta0)
        th = _f64(theta0).copy()
        dth = _f64(dtheta0).copy()
        u = _f64(u)
        duk = _f64(du) if du is not None else np.zeros(self.n_faces)
        sc = {"euler": EULER, "ssprk3": SSPRK3}.get(scheme, scheme)
        rc = lib().orc_run_tangent(self._h, lim_id(limiter), int(sc), float(dt), self._S(th),
                                   int(nsteps), _ptr(th), _ptr(dth), _ptr(u), _ptr(duk))
        if rc != 0:
            raise ValueError("bad scheme")
        return th, dth

    def run_adjoint(self, limiter, scheme, dt, theta0, u, nsteps, theta_bar_final):
        self._check_S(theta0)
        th0 = _f64(theta0)
        u = _f64(u)
        tbf = _f64(theta_bar_final)
        tb0 = np.empty_like(th0)
        ub = np.empty(self.n_faces)
        sc = {"euler": EULER, "ssprk3": SSPRK3}.get(scheme, scheme)
        rc = lib().orc_run_adjoint(self._h, lim_id(limiter), int(sc), float(dt), self._S(th0),
                                   int(nsteps), _ptr(th0), _ptr(u), _ptr(tbf), _ptr(tb0), _ptr(ub))
        if rc != 0:
            raise ValueError(f"orc_run_adjoint failed ({rc})")
        return tb0, ub
