"""Python API of the flux-limited convective operator (thin layer over the C ABI).

PyTorch provides device memory and streams; every arithmetic step of the operator runs in the
HIP kernels of libfluxlim.so.  Tensors are float64, contiguous and on the mesh's device.
Cell fields are [n_cells] or [n_cells, S] (S <= 8 scalars, scalar index fastest).
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import call, lib

LIMITERS = {"upwind": 0, "minmod": 1, "vanleer": 2, "vanalbada": 3, "superbee": 4, "smart": 5,
            "central": 6}
SCHEMES = {"euler": 1, "ssprk3": 3}
MAX_SCALARS = 8


def limiter_id(lim) -> int:
    if isinstance(lim, str):
        return LIMITERS[lim]
    lim = int(lim)
    if not 0 <= lim < len(LIMITERS):
        raise ValueError(f"unknown limiter {lim}")
    return lim


def scheme_id(s) -> int:
    return SCHEMES[s] if isinstance(s, str) else int(s)


OPTIONS = {"xcd_remap": 1, "slot_velocity": 2, "lds_stage": 3, "check_finite": 4,
           "fwd_rates": 5, "face_share": 6}


def set_option(name: str, value: int) -> None:
    """Process-wide launch option (fl_set_option): "xcd_remap" (default 32), "slot_velocity"
    (default 1: multi-step calls read per-call slot tables with the signed face rates),
    "lds_stage" (default 1: those calls stage each tile's theta and halo in LDS) or
    "check_finite" (default 0: 1 makes the compute calls reject non-finite inputs with
    FL_E_NONFINITE, at the cost of a scan and a stream synchronisation per call) or
    "fwd_rates" (default 1: on lattice meshes those multi-step stages read the rates of each
    cell's forward faces only) or "face_share" (default 1: there the reverse stages of
    rk_steps_adjoint evaluate each face once per tile and share its terms; same bits)."""
    call("fl_set_option", OPTIONS[name], int(value))


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device: torch.device, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


class Mesh:
    """A mesh on one GPU, built from its face-to-cell incidence (see include/fluxlim.h)."""

    def __init__(self, face_cells, face_normal, face_area=None, cell_volume=None, n_cells=None,
                 device=0, reorder=False, face_path: bool = False, face_dist=None):
        fc = np.ascontiguousarray(face_cells, dtype=np.int32)
        nrm = np.ascontiguousarray(face_normal, dtype=np.float64)
        if fc.ndim != 2 or fc.shape[1] != 2 or nrm.shape != (fc.shape[0], 3):
            raise ValueError("face_cells must be [F, 2] and face_normal [F, 3]")
        C = int(n_cells) if n_cells is not None else int(fc.max()) + 1
        area = None if face_area is None else np.ascontiguousarray(face_area, dtype=np.float64)
        vol = None if cell_volume is None else np.ascontiguousarray(cell_volume, dtype=np.float64)
        if isinstance(device, torch.device):
            device = device.index if device.index is not None else 0
        if reorder not in (False, True, "curve", "bfs"):
            raise ValueError("reorder must be False, True/'curve' or 'bfs'")
        flags = ((_lib.FL_MESH_REORDER_BFS if reorder == "bfs" else _lib.FL_MESH_REORDER if reorder else 0)
                 | (_lib.FL_MESH_FACE_PATH if face_path else 0))
        dist = None if face_dist is None else np.ascontiguousarray(face_dist, dtype=np.float64)
        if dist is not None and dist.shape != (fc.shape[0],):
            raise ValueError("face_dist must hold one distance per face")
        h = ctypes.c_void_p()
        call("fl_mesh_create_dist", C, fc.shape[0], _np_ptr(fc), _np_ptr(nrm),
             _np_ptr(area) if area is not None else None, _np_ptr(vol) if vol is not None else None,
             _np_ptr(dist) if dist is not None else None, int(device), flags, ctypes.byref(h))
        self._h = h
        info = _lib.MeshInfo()
        call("fl_mesh_info", self._h, ctypes.byref(info))
        self.info = info
        self.n_cells = int(info.n_cells)
        self.n_faces = int(info.n_faces)
        self.device_index = int(info.device)
        self.device = torch.device("cuda", self.device_index) if self.device_index >= 0 else None
        self.path = "fused" if info.path == _lib.FL_PATH_FUSED else "face"
        self.reordered = bool(info.reordered)
        self.n_boundary = int(info.n_boundary)
        self._inflow = None

    def set_inflow(self, values: Optional[torch.Tensor]) -> None:
        """Inflow values of the boundary faces (fl_mesh_set_inflow): a contiguous float64
        [F] or [F, S] tensor on the mesh's device in mesh order (rows of the other faces are not
        read), or None to clear.  The mesh keeps a reference until cleared or closed."""
        if values is None:
            call("fl_mesh_set_inflow", self.handle, None, 0)
            self._inflow = None
            return
        if values.dtype != torch.float64 or values.device != self.device or \
                not values.is_contiguous() or values.shape[0] != self.n_faces or \
                values.dim() not in (1, 2):
            raise ValueError(f"inflow values must be a contiguous float64 [{self.n_faces}] or "
                             f"[{self.n_faces}, S] tensor on the mesh's device")
        call("fl_mesh_set_inflow", self.handle, _tptr(values), _S(values))
        self._inflow = values

    @classmethod
    def from_arrays(cls, m, **kw) -> "Mesh":
        """From a workloads.MeshArrays (with its face distances, if it has any, unless
        face_dist is given)."""
        kw.setdefault("face_dist", getattr(m, "face_dist", None))
        return cls(m.face_cells, m.face_normal, m.face_area, m.cell_volume, n_cells=m.n_cells, **kw)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("mesh was closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fl_mesh_destroy(self._h)
            self._h = None
        self._inflow = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- numbering ------------------------------------------------------------------------------
    def permutation(self):
        cp = np.empty(self.n_cells, dtype=np.int32)
        fp = np.empty(self.n_faces, dtype=np.int32)
        call("fl_mesh_permutation", self.handle, _np_ptr(cp), _np_ptr(fp))
        return cp, fp

    def export_tables(self):
        far = np.empty((self.n_faces, 2), dtype=np.int32)
        ptr = np.empty(self.n_cells + 1, dtype=np.int32)
        call("fl_mesh_export_tables", self.handle, _np_ptr(far), _np_ptr(ptr), None)
        idx = np.empty(int(ptr[-1]), dtype=np.int32)
        call("fl_mesh_export_tables", self.handle, None, None, _np_ptr(idx))
        return far, ptr, idx

    def cells_to_mesh(self, x: torch.Tensor) -> torch.Tensor:
        return self._permute_cells(x, 1)

    def cells_from_mesh(self, x: torch.Tensor) -> torch.Tensor:
        return self._permute_cells(x, 0)

    def faces_to_mesh(self, u: torch.Tensor) -> torch.Tensor:
        return self._permute_faces(u, 1)

    def faces_from_mesh(self, u: torch.Tensor) -> torch.Tensor:
        return self._permute_faces(u, 0)

    def _permute_cells(self, x, to_mesh):
        x = self._cells(x)
        out = torch.empty_like(x)
        call("fl_permute_cells", self.handle, to_mesh, _S(x), _tptr(x), _tptr(out),
             _stream(self.device))
        return out

    def _permute_faces(self, u, to_mesh):
        u = self._faces(u)
        out = torch.empty_like(u)
        call("fl_permute_faces", self.handle, to_mesh, _tptr(u), _tptr(out), _stream(self.device))
        return out

    # -- argument checks ------------------------------------------------------------------------
    def _cells(self, x: torch.Tensor) -> torch.Tensor:
        if x.dtype != torch.float64 or x.device != self.device or not x.is_contiguous():
            raise ValueError("cell fields must be contiguous float64 tensors on the mesh's device")
        if x.shape[0] != self.n_cells or x.dim() not in (1, 2) or _S(x) > MAX_SCALARS:
            raise ValueError(f"cell field must be [{self.n_cells}] or [{self.n_cells}, S<=8]")
        return x

    def _faces(self, u: torch.Tensor) -> torch.Tensor:
        if u.dtype != torch.float64 or u.device != self.device or not u.is_contiguous():
            raise ValueError("face fields must be contiguous float64 tensors on the mesh's device")
        if u.shape != (self.n_faces,):
            raise ValueError(f"face field must be [{self.n_faces}]")
        return u

    def debug_select(self, u: torch.Tensor) -> np.ndarray:
        out = np.empty((self.n_faces, 3), dtype=np.int32)
        call("fl_debug_select", self.handle, _tptr(self._faces(u)), _np_ptr(out),
             _stream(self.device))
        return out


def _S(x: torch.Tensor) -> int:
    return 1 if x.dim() == 1 else int(x.shape[1])


def _workspace(nbytes: int, device) -> Optional[torch.Tensor]:
    if nbytes == 0:
        return None
    w = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-w.data_ptr()) % 256
    return w[off:off + nbytes]


def apply_workspace(mesh: Mesh, S: int) -> Optional[torch.Tensor]:
    return _workspace(int(lib().fl_apply_workspace_bytes(mesh.handle, S)), mesh.device)


def rk_workspace(mesh: Mesh, scheme, S: int) -> torch.Tensor:
    return _workspace(int(lib().fl_rk_workspace_bytes(mesh.handle, scheme_id(scheme), S)),
                      mesh.device)


def convect_apply(mesh: Mesh, limiter, theta: torch.Tensor, u: torch.Tensor,
                  out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """rhs = L(theta): the divergence of the limited face fluxes (Algorithm 4's operator)."""
    theta = mesh._cells(theta)
    u = mesh._faces(u)
    S = _S(theta)
    if out is None:
        out = torch.empty_like(theta)
    if work is None:
        work = apply_workspace(mesh, S)
    call("fl_convect_apply", mesh.handle, limiter_id(limiter), S, _tptr(theta), _tptr(u),
         _tptr(out), _tptr(work), _stream(mesh.device, stream))
    return out


def rk_steps(mesh: Mesh, limiter, scheme, dt: float, theta: torch.Tensor, u: torch.Tensor,
             n_steps: int = 1, work: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Advances theta in place by n_steps explicit steps (forward Euler or SSP-RK3)."""
    theta = mesh._cells(theta)
    u = mesh._faces(u)
    S = _S(theta)
    if work is None:
        work = rk_workspace(mesh, scheme, S)
    call("fl_rk_steps", mesh.handle, limiter_id(limiter), scheme_id(scheme), float(dt), S,
         int(n_steps), _tptr(theta), _tptr(u), _tptr(work), _stream(mesh.device, stream))
    return theta


def rk_steps_scaled(mesh: Mesh, limiter, scheme, dt: float, theta: torch.Tensor,
                    u: torch.Tensor, scales, work: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    """Advances theta in place with the time-dependent velocity s(t) u; scales holds s at every
    stage (stages x steps values, e.g. workloads.deformation_scales)."""
    theta = mesh._cells(theta)
    u = mesh._faces(u)
    S = _S(theta)
    sc = np.ascontiguousarray(scales, dtype=np.float64)
    ns = n_stages(scheme)
    if sc.ndim != 1 or sc.size % ns:
        raise ValueError("scales must hold stages * n_steps values")
    if work is None:
        work = rk_workspace(mesh, scheme, S)
    call("fl_rk_steps_scaled", mesh.handle, limiter_id(limiter), scheme_id(scheme), float(dt), S,
         sc.size // ns, _tptr(theta), _tptr(u), _np_ptr(sc), _tptr(work),
         _stream(mesh.device, stream))
    return theta


# ---------------------------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------------------------

def n_stages(scheme) -> int:
    return 1 if scheme_id(scheme) == SCHEMES["euler"] else 3


def convect_adjoint(mesh: Mesh, limiter, theta: torch.Tensor, u: torch.Tensor,
                    rhs_bar: torch.Tensor, theta_bar: Optional[torch.Tensor] = None,
                    u_bar: Optional[torch.Tensor] = None, stream=None):
    """theta_bar += (dL/dtheta)^T rhs_bar and u_bar += (dL/du)^T rhs_bar (fresh zeros if None)."""
    theta = mesh._cells(theta)
    u = mesh._faces(u)
    rhs_bar = mesh._cells(rhs_bar)
    if theta_bar is None:
        theta_bar = torch.zeros_like(theta)
    if u_bar is None:
        u_bar = torch.zeros_like(u)
    work = _workspace(int(lib().fl_adjoint_workspace_bytes(mesh.handle, _S(theta))), mesh.device)
    call("fl_convect_adjoint", mesh.handle, limiter_id(limiter), _S(theta), _tptr(theta), _tptr(u),
         _tptr(rhs_bar), _tptr(mesh._cells(theta_bar)), _tptr(mesh._faces(u_bar)), _tptr(work),
         _stream(mesh.device, stream))
    return theta_bar, u_bar


def stage_buffer(mesh: Mesh, scheme, S: int, n_steps: int = 1) -> torch.Tensor:
    """Storage for the stage inputs of n_steps steps: [n_steps, stages, n_cells(, S)]."""
    shape = (n_steps, n_stages(scheme), mesh.n_cells) + ((S,) if S > 1 else ())
    return torch.empty(shape, dtype=torch.float64, device=mesh.device)


def rk_adjoint_workspace(mesh: Mesh, scheme, S: int) -> torch.Tensor:
    return _workspace(int(lib().fl_rk_adjoint_workspace_bytes(mesh.handle, scheme_id(scheme), S)),
                      mesh.device)


def rk_step_store(mesh: Mesh, limiter, scheme, dt, theta, u, stages, work=None, stream=None):
    """One step in place on theta, storing its stage inputs in stages ([stages, C(, S)])."""
    theta = mesh._cells(theta)
    S = _S(theta)
    if work is None:
        work = rk_workspace(mesh, scheme, S)
    if not stages.is_contiguous() or stages.numel() != n_stages(scheme) * theta.numel():
        raise ValueError("stages must be a contiguous [stages, n_cells(, S)] float64 buffer")
    call("fl_rk_step_store", mesh.handle, limiter_id(limiter), scheme_id(scheme), float(dt), S,
         _tptr(theta), _tptr(mesh._faces(u)), _tptr(stages), _tptr(work),
         _stream(mesh.device, stream))
    return theta


def rk_step_adjoint(mesh: Mesh, limiter, scheme, dt, stages, u, lam, u_bar=None, work=None,
                    stream=None):
    """Reverse of one step: lam (cotangent of theta^{n+1}) becomes that of theta^n in place;
    u_bar += the step's contribution to d/du."""
    lam = mesh._cells(lam)
    S = _S(lam)
    if work is None:
        work = rk_adjoint_workspace(mesh, scheme, S)
    if not stages.is_contiguous() or stages.numel() != n_stages(scheme) * lam.numel():
        raise ValueError("stages must be a contiguous [stages, n_cells(, S)] float64 buffer")
    call("fl_rk_step_adjoint", mesh.handle, limiter_id(limiter), scheme_id(scheme), float(dt), S,
         _tptr(stages), _tptr(mesh._faces(u)), _tptr(lam),
         _tptr(mesh._faces(u_bar)) if u_bar is not None else None, _tptr(work),
         _stream(mesh.device, stream))
    return lam


def adjoint_rates(mesh: Mesh, u, stream=None) -> torch.Tensor:
    """The face velocities as the signed-rate table that rk_steps_adjoint reads."""
    n = int(lib().fl_adjoint_rates_bytes(mesh.handle)) // 8
    rates = torch.empty(n, dtype=torch.float64, device=mesh.device)
    call("fl_adjoint_rates", mesh.handle, _tptr(mesh._faces(u)), _tptr(rates),
         _stream(mesh.device, stream))
    return rates


def rk_steps_adjoint(mesh: Mesh, limiter, scheme, dt, stages, rates, lam, n_steps: int,
                     u_acc: Optional[torch.Tensor] = None, work=None, stream=None):
    """Reverse of n_steps stored steps (stages[i] = step i's stage inputs; rates from
    adjoint_rates): lam becomes the cotangent of theta before step 0, in place; u_acc (see
    uacc_buffer) accumulates the face-velocity cotangent in the mesh's cell-slot layout (None:
    skipped)."""
    lam = mesh._cells(lam)
    S = _S(lam)
    if work is None:
        work = _workspace(int(lib().fl_rk_steps_adjoint_workspace_bytes(
            mesh.handle, scheme_id(scheme), S)), mesh.device)
    per = n_stages(scheme) * lam.numel()
    if not stages.is_contiguous() or stages.dtype != torch.float64 or \
            stages.numel() < n_steps * per or stages.device != lam.device:
        raise ValueError("stages must be a contiguous float64 [n_steps, stages, n_cells(, S)] buffer")
    call("fl_rk_steps_adjoint", mesh.handle, limiter_id(limiter), scheme_id(scheme), float(dt), S,
         int(n_steps), _tptr(stages), _tptr(rates), _tptr(lam), _tptr(u_acc),
         _tptr(work), _stream(mesh.device, stream))
    return lam


def uacc_buffer(mesh: Mesh) -> Optional[torch.Tensor]:
    """A zeroed face-velocity cotangent accumulator in the mesh's cell-slot layout (None where the
    mesh has none: not on the fused path)."""
    n = int(lib().fl_adjoint_uacc_bytes(mesh.handle)) // 8
    return torch.zeros(n, dtype=torch.float64, device=mesh.device) if n else None


def uacc_scatter(mesh: Mesh, u_acc: torch.Tensor, u_bar: torch.Tensor, stream=None):
    """u_bar += the accumulated face-velocity cotangent (face order)."""
    call("fl_adjoint_uacc_scatter", mesh.handle, _tptr(u_acc), _tptr(mesh._faces(u_bar)),
         _stream(mesh.device, stream))
    return u_bar


def checkpoint_interval(n_steps: int) -> int:
    """ceil(sqrt(n_steps)): sqrt(N) checkpoints, each segment recomputed once in the backward."""
    import math
    return max(1, math.isqrt(max(n_steps - 1, 0)) + 1) if n_steps > 0 else 1


def rk_steps_store(mesh: Mesh, limiter, scheme, dt, theta, u, stages, n_steps: int,
                   work=None, stream=None):
    """n_steps steps in place on theta, storing step i's stage inputs in stages[i]
    (stages: [>= n_steps, stages per step, C(, S)])."""
    theta = mesh._cells(theta)
    S = _S(theta)
    if work is None:
        work = rk_workspace(mesh, scheme, S)
    per = n_stages(scheme) * theta.numel()
    if not stages.is_contiguous() or stages.dtype != torch.float64 or stages.numel() < n_steps * per \
            or stages.device != theta.device:
        raise ValueError("stages must be a contiguous float64 [n_steps, stages, n_cells(, S)] buffer")
    call("fl_rk_steps_store", mesh.handle, limiter_id(limiter), scheme_id(scheme), float(dt), S,
         int(n_steps), _tptr(theta), _tptr(mesh._faces(u)), _tptr(stages), _tptr(work),
         _stream(mesh.device, stream))
    return theta


class _Advect(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta0, u, mesh, limiter, scheme, dt, n_steps, every):
        theta = mesh._cells(theta0.detach()).clone()
        u_d = mesh._faces(u.detach())
        S = _S(theta)
        work = rk_workspace(mesh, scheme, S)
        ckpts = []
        stages = stage_buffer(mesh, scheme, S, min(every, max(n_steps, 1)))
        for start in range(0, n_steps, every):
            ckpts.append(theta.clone())
            count = min(every, n_steps - start)
            if start + count < n_steps:
                rk_steps(mesh, limiter, scheme, dt, theta, u_d, count, work=work)
            else:  # the last segment keeps its stage inputs: the backward starts there
                rk_steps_store(mesh, limiter, scheme, dt, theta, u_d, stages, count, work=work)
        ctx.mesh, ctx.limiter, ctx.scheme, ctx.dt = mesh, limiter, scheme, dt
        ctx.n_steps, ctx.every, ctx.ckpts, ctx.stages = n_steps, every, ckpts, stages
        ctx.save_for_backward(u_d)
        return theta

    @staticmethod
    def backward(ctx, grad):
        (u_d,) = ctx.saved_tensors
        mesh, lim, scheme, dt = ctx.mesh, ctx.limiter, ctx.scheme, ctx.dt
        lam = grad.detach().to(torch.float64).contiguous().clone()
        S = _S(lam)
        u_bar = torch.zeros_like(u_d)
        want_u = ctx.needs_input_grad[1]
        work = rk_workspace(mesh, scheme, S)
        # the multi-step reverse sweep (one call per segment, u cotangent in cell-slot order,
        # scattered once at the end) where the mesh has it, else one call per step
        u_acc = uacc_buffer(mesh)
        multi = u_acc is not None
        if multi:
            awork = _workspace(int(lib().fl_rk_steps_adjoint_workspace_bytes(
                mesh.handle, scheme_id(scheme), S)), mesh.device)
            rates = adjoint_rates(mesh, u_d)  # once: u is the same in every segment
        else:
            awork = rk_adjoint_workspace(mesh, scheme, S)
        stages = ctx.stages
        last = len(ctx.ckpts) - 1
        for seg in reversed(range(len(ctx.ckpts))):
            start = seg * ctx.every
            count = min(ctx.every, ctx.n_steps - start)
            if seg != last:  # recompute the segment, storing every stage input (the checkpoint
                # is not needed again: it is advanced in place)
                th = ctx.ckpts[seg]
                ctx.ckpts[seg] = None
                rk_steps_store(mesh, lim, scheme, dt, th, u_d, stages, count, work=work)
                del th
            if multi:
                rk_steps_adjoint(mesh, lim, scheme, dt, stages, rates, lam, count,
                                 u_acc if want_u else None, work=awork)
            else:
                for j in reversed(range(count)):
                    rk_step_adjoint(mesh, lim, scheme, dt, stages[j], u_d, lam,
                                    u_bar if want_u else None, work=awork)
        if multi and want_u:
            uacc_scatter(mesh, u_acc, u_bar)
        ctx.ckpts = None
        ctx.stages = None
        return lam, (u_bar if want_u else None), None, None, None, None, None, None


def checkpoint_interval_for_budget(mesh: Mesh, scheme, S: int, n_steps: int,
                                   budget_bytes: int) -> int:
    """The longest checkpoint interval whose stored stage inputs ([every, stages, C, S] doubles)
    fit in budget_bytes, never shorter than ceil(sqrt(n_steps)); n_steps (nothing recomputed) when
    the whole run fits."""
    per_step = n_stages(scheme) * mesh.n_cells * S * 8
    fit = int(budget_bytes) // max(per_step, 1)
    return max(checkpoint_interval(n_steps), min(max(n_steps, 1), fit))


def advect(mesh: Mesh, limiter, scheme, dt: float, theta0: torch.Tensor, u: torch.Tensor,
           n_steps: int, checkpoint_every: Optional[int] = None,
           memory_budget: Optional[int] = None) -> torch.Tensor:
    """theta after n_steps explicit steps, differentiable w.r.t. theta0 and u (hand-written
    discrete adjoint).  The forward keeps theta every `checkpoint_every` steps (default
    ceil(sqrt(n_steps)), or the longest interval whose stage storage fits in memory_budget bytes)
    and the stage inputs of the last segment; the backward recomputes each other segment once,
    storing its stage inputs, and runs the reverse steps."""
    if checkpoint_every is None:
        if memory_budget is not None:
            checkpoint_every = checkpoint_interval_for_budget(mesh, scheme, _S(theta0), n_steps,
                                                              memory_budget)
        else:
            checkpoint_every = checkpoint_interval(n_steps)
    return _Advect.apply(theta0, u, mesh, limiter, scheme, float(dt), int(n_steps),
                         int(checkpoint_every))


# ---------------------------------------------------------------------------------------------
# The paper's algebraic form (SpMV + pointwise kernels), for comparison with the fused path
# ---------------------------------------------------------------------------------------------

ALG_MATRICES = ("D", "UUD", "OUD", "Pi", "M")


class Algebraic:
    """The matrices of Algorithms 3 and 4 (ELLPACK, on the mesh's device) and the literal
    SpMV/kbin chain over them (one scalar).  The mesh must stay open while this object is used."""

    def __init__(self, mesh: Mesh):
        h = ctypes.c_void_p()
        call("fl_algebraic_create", mesh.handle, ctypes.byref(h))
        self._h = h
        self.mesh = mesh
        info = _lib.AlgebraicInfo()
        call("fl_algebraic_info", h, ctypes.byref(info))
        self.rows = {k: int(info.rows[i]) for i, k in enumerate(ALG_MATRICES)}
        self.width = {k: int(info.width[i]) for i, k in enumerate(ALG_MATRICES)}
        self.device_bytes = int(info.device_bytes)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fl_algebraic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self, name: str):
        """(val, col) of one matrix, each [width, rows]."""
        i = ALG_MATRICES.index(name)
        val = np.empty((self.width[name], self.rows[name]), dtype=np.float64)
        col = np.empty((self.width[name], self.rows[name]), dtype=np.int32)
        call("fl_algebraic_export", self._h, i, _np_ptr(val), _np_ptr(col))
        return val, col

    def workspace(self) -> torch.Tensor:
        return _workspace(int(lib().fl_algebraic_workspace_bytes(self._h)), self.mesh.device)

    def face_values(self, limiter, theta, u, out=None, work=None, stream=None) -> torch.Tensor:
        theta = self.mesh._cells(theta)
        if _S(theta) != 1:
            raise ValueError("the algebraic chain takes one scalar field")
        u = self.mesh._faces(u)
        out = torch.empty_like(u) if out is None else self.mesh._faces(out)
        work = self.workspace() if work is None else work
        call("fl_algebraic_face_values", self._h, limiter_id(limiter), _tptr(theta), _tptr(u),
             _tptr(out), _tptr(work), _stream(self.mesh.device, stream))
        return out

    def rk_steps(self, limiter, scheme, dt, theta, u, n_steps=1, work=None, stream=None):
        theta = self.mesh._cells(theta)
        if _S(theta) != 1:
            raise ValueError("the algebraic chain takes one scalar field")
        work = self.workspace() if work is None else work
        call("fl_algebraic_rk_steps", self._h, limiter_id(limiter), scheme_id(scheme), float(dt),
             int(n_steps), _tptr(theta), _tptr(self.mesh._faces(u)), _tptr(work),
             _stream(self.mesh.device, stream))
        return theta


# ---------------------------------------------------------------------------------------------
# Batched problems
# ---------------------------------------------------------------------------------------------

class Batch:
    """Independent problems (mesh, limiter, theta, u, dt) advanced together: one kernel launch per
    Runge-Kutta stage for all the fused-path problems and two for all the face-path ones (general
    cells, boundary faces, face distances), recorded once in a HIP graph and replayed.

    problems: sequence of (mesh, limiter, theta, u, dt); theta is updated in place.  Meshes may
    be shared.  tile_cells = 0 lets the library pick the tile size at creation (timing the
    candidates, or from its on-disk tuning cache); creation also records the step's graph, so
    step() only replays it."""

    def __init__(self, problems, scheme="ssprk3", tile_cells: int = 0):
        n = len(problems)
        if n == 0:
            raise ValueError("empty batch")
        meshes = [p[0] for p in problems]
        dev = meshes[0].device_index
        self._keep = []
        mh = (ctypes.c_void_p * n)(*[m.handle.value for m in meshes])
        lim = (ctypes.c_int * n)(*[limiter_id(p[1]) for p in problems])
        ns = (ctypes.c_int * n)()
        th = (ctypes.c_void_p * n)()
        uu = (ctypes.c_void_p * n)()
        dts = (ctypes.c_double * n)()
        for i, (m, _, theta, u, dt) in enumerate(problems):
            m._cells(theta)
            m._faces(u)
            ns[i] = _S(theta)
            th[i] = theta.data_ptr()
            uu[i] = u.data_ptr()
            dts[i] = float(dt)
            self._keep += [theta, u]
        self.meshes = meshes
        self.n = n
        h = ctypes.c_void_p()
        call("fl_batch_create", n, mh, lim, ns, dts, scheme_id(scheme), th, uu, int(tile_cells),
             dev, ctypes.byref(h))
        self._h = h
        self.device = meshes[0].device

    def step(self, n_steps: int = 1, stream=None):
        call("fl_batch_step", self._h, int(n_steps), _stream(self.device, stream))

    def step_unbatched(self, n_steps: int = 1, stream=None):
        call("fl_batch_step_unbatched", self._h, int(n_steps), _stream(self.device, stream))

    @property
    def tile_cells(self) -> int:
        t = ctypes.c_int()
        call("fl_batch_tile", self._h, ctypes.byref(t))
        return t.value

    @property
    def lds_staged(self) -> bool:
        t = ctypes.c_int()
        call("fl_batch_lds", self._h, ctypes.byref(t))
        return bool(t.value)

    @property
    def tuned_from_cache(self) -> bool:
        t = ctypes.c_int()
        call("fl_batch_tuned_from_cache", self._h, ctypes.byref(t))
        return bool(t.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().fl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
