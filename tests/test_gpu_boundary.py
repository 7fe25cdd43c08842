"""GPU parity of meshes with boundary faces (inflow values, zero-gradient exterior) and of
distance-weighted meshes against the CPU oracle.

The boundary reading (a boundary face borders an exterior cell holding the inflow value where
the flow enters, the interior cell's value otherwise) is pinned on the oracle in
test_oracle_boundary.py.  Here the library runs it on the face path with the general kernel:
one operator application is compared at 1e-13 of max|rhs| and whole runs at the 1e-10 max
norm-relative error of the cell values, as for closed meshes.  The inflow arrays hold NaN on the
rows the rule never reads (interior faces and outflow faces), so a stray read shows.  The
distance weighting (Algorithm 1D / UNS ratios) is pinned in test_oracle_distances.py, and the
oracle's derivatives on such meshes in test_oracle_open_derivatives.py; the adjoint tests at the
end compare the library's with them (1e-12 of the largest cotangent for one application, 1e-10
for reverse sweeps, as on closed meshes).
"""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2110_03044_amd import _lib, fluxlim as FL, workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
LIMS = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart", "central"]
RUN_TOL = 1e-10


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def nrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rows_to_mesh(x, perm):
    out = np.empty_like(x)
    out[perm] = x
    return out


def library(m, inflow, **kw):
    mesh = FL.Mesh.from_arrays(m, device=0, **kw)
    cp, fp = mesh.permutation()
    assert mesh.path == "face" and mesh.n_boundary == int((m.face_cells[:, 1] < 0).sum())
    assert mesh.info.dist_weighted == (m.face_dist is not None)
    if inflow is not None:
        mesh.set_inflow(dev(rows_to_mesh(inflow, fp)))
    return mesh, cp, fp


@pytest.mark.parametrize("with_inflow", [True, False])
@pytest.mark.parametrize("reorder", [False, True, "bfs"])
@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("lim", LIMS)
def test_apply_open_box(lim, S, reorder, with_inflow):
    wl = W.workload_open_box(9, renumbered=True, S=S)
    m = wl.mesh
    inflow = wl.inflow if with_inflow else None
    mesh, cp, fp = library(m, inflow, reorder=reorder)
    om = O.OracleMesh.from_arrays(m)
    om.set_inflow(inflow)
    rng = np.random.default_rng(11)
    th = wl.theta0 + 0.05 * rng.standard_normal(wl.theta0.shape)
    want = om.rhs(lim, th, wl.u)
    got = host(FL.convect_apply(mesh, lim, dev(rows_to_mesh(th, cp)), dev(rows_to_mesh(wl.u, fp))))
    assert np.abs(got[cp] - want).max() <= 1e-13 * np.abs(want).max()
    mesh.close()


@pytest.mark.parametrize("scheme,steps", [("ssprk3", 12), ("euler", 20)])
@pytest.mark.parametrize("lim", LIMS)
def test_runs_open_box(lim, scheme, steps):
    wl = W.workload_open_box(12, renumbered=True)
    m = wl.mesh
    mesh, cp, fp = library(m, wl.inflow, reorder=True)
    om = O.OracleMesh.from_arrays(m)
    om.set_inflow(wl.inflow)
    want = om.run(lim, scheme, wl.dt, wl.theta0, wl.u, steps)
    th = dev(rows_to_mesh(wl.theta0, cp))
    FL.rk_steps(mesh, lim, scheme, wl.dt, th, dev(rows_to_mesh(wl.u, fp)), steps)
    assert nrel(host(th)[cp], want) <= RUN_TOL
    mesh.close()


@pytest.mark.parametrize("lim", ["upwind", "minmod", "vanleer", "superbee", "smart"])
def test_open_line_with_inflow_long_run(lim):
    """1-D line, flow to the right, a square wave entering through the left end: 150 Euler
    steps at CFL 0.5 against the oracle."""
    n = 80
    m = W.open_box(n, 1, (0,))
    u = m.face_normal[:, 0].copy()
    x = (np.arange(n) + 0.5) / n
    th0 = np.where((x > 0.2) & (x < 0.4), 1.0, 0.0)
    inflow = np.full(m.n_faces, np.nan)
    inflow[n] = 0.8
    om = O.OracleMesh.from_arrays(m)
    om.set_inflow(inflow)
    dt = 0.5 / n
    want = om.run(lim, "euler", dt, th0, u, 150)
    mesh, cp, fp = library(m, inflow)
    th = dev(rows_to_mesh(th0, cp))
    FL.rk_steps(mesh, lim, "euler", dt, th, dev(rows_to_mesh(u, fp)), 150)
    assert nrel(host(th)[cp], want) <= RUN_TOL
    mesh.close()


@pytest.mark.parametrize("lim", ["vanleer", "vanalbada"])
def test_time_dependent_velocity_swaps_inflow_and_outflow(lim):
    """u(t) = cos(pi t / T) u with T shorter than the run: the boundary faces change from outflow
    to inflow and back, so every boundary face needs its inflow value at some stage."""
    wl = W.workload_open_box(10, renumbered=True)
    m = wl.mesh
    inflow = W.inflow_values(W.open_box(10, 3, (0,)))  # every boundary face, natural order
    inflow = m.face_field_from_natural(inflow)
    steps = 16
    scales = W.deformation_scales(steps, wl.dt, 8 * wl.dt, "ssprk3")
    assert scales.min() < 0 < scales.max()
    om = O.OracleMesh.from_arrays(m)
    om.set_inflow(inflow)
    want = om.run_scaled(lim, "ssprk3", wl.dt, wl.theta0, wl.u, scales)
    mesh, cp, fp = library(m, inflow, reorder=True)
    th = dev(rows_to_mesh(wl.theta0, cp))
    FL.rk_steps_scaled(mesh, lim, "ssprk3", wl.dt, th, dev(rows_to_mesh(wl.u, fp)), scales)
    assert nrel(host(th)[cp], want) <= RUN_TOL
    mesh.close()


def test_inflow_scalar_count_must_match():
    wl = W.workload_open_box(6, S=2)
    mesh, cp, fp = library(wl.mesh, wl.inflow)
    th = dev(rows_to_mesh(wl.theta0, cp))
    u = dev(rows_to_mesh(wl.u, fp))
    FL.convect_apply(mesh, "vanleer", th, u)  # S = 2 matches
    with pytest.raises(_lib.FluxLimError) as e:
        FL.convect_apply(mesh, "vanleer", th[:, 0].contiguous(), u)
    assert e.value.status == -1
    mesh.set_inflow(None)
    FL.convect_apply(mesh, "vanleer", th[:, 0].contiguous(), u)
    mesh.close()


def test_algebraic_refuses_boundary_meshes():
    wl = W.workload_open_box(6)
    mesh, cp, fp = library(wl.mesh, None)
    with pytest.raises(_lib.FluxLimError) as e:
        FL.Algebraic(mesh)
    assert e.value.status == -3  # unsupported
    mesh.close()


@pytest.mark.parametrize("case", ["periodic", "open"])
@pytest.mark.parametrize("S", [1, 2])
@pytest.mark.parametrize("lim", LIMS)
def test_distance_weighted_apply_and_run(lim, S, case):
    """A box stretched along x (cell widths 1 +- 0.5 sin), periodic or cut open along x with
    inflow values: one application at 1e-13 and 10 SSP-RK3 steps at 1e-10 against the oracle
    with the same face distances."""
    open_axes = (0,) if case == "open" else ()
    nat = W.stretched_box(10, 3, amp=0.5, open_axes=open_axes)
    u_nat = W.velocity_open_box(nat)
    th_nat = W.field_blob_step(10)
    if S > 1:
        th_nat = W.multi_scalar([th_nat + 0.2 * k for k in range(S)])
    inflow_nat = W.inflow_values(nat, u_nat, S) if open_axes else None
    m = W.renumber(nat, seed=12)
    u = m.face_velocity_from_natural(u_nat)
    th0 = m.cell_field_from_natural(th_nat)
    inflow = None if inflow_nat is None else m.face_field_from_natural(inflow_nat)
    dt = W.cfl_dt(m, u, 0.4)
    mesh, cp, fp = library(m, inflow, reorder=True)
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(m.face_dist)
    om.set_inflow(inflow)
    want = om.rhs(lim, th0, u)
    ud = dev(rows_to_mesh(u, fp))
    got = host(FL.convect_apply(mesh, lim, dev(rows_to_mesh(th0, cp)), ud))
    assert np.abs(got[cp] - want).max() <= 1e-13 * np.abs(want).max()
    want = om.run(lim, "ssprk3", dt, th0, u, 10)
    th = dev(rows_to_mesh(th0, cp))
    FL.rk_steps(mesh, lim, "ssprk3", dt, th, ud, 10)
    assert nrel(host(th)[cp], want) <= RUN_TOL
    mesh.close()


def _adjoint_case(case, S):
    """(mesh arrays, theta, u, inflow or None): an open box with or without inflow values, or a
    stretched box (face distances), periodic or open with inflow values."""
    rng = np.random.default_rng(21 + S)
    if case.startswith("open_box"):
        wl = W.workload_open_box(7, renumbered=True, S=S)
        th = wl.theta0 + 0.05 * rng.standard_normal(wl.theta0.shape)
        th[::5] = np.round(th[::5], 1)  # plateaus next to the boundary too
        return wl.mesh, th, wl.u, (wl.inflow if case == "open_box_inflow" else None)
    open_axes = (0,) if case == "stretched_open" else ()
    nat = W.stretched_box(8, 3, amp=0.5, open_axes=open_axes)
    u_nat = W.velocity_open_box(nat)
    th_nat = W.field_blob_step(8)
    if S > 1:
        th_nat = W.multi_scalar([th_nat + 0.2 * k for k in range(S)])
    m = W.renumber(nat, seed=23)
    inflow = m.face_field_from_natural(W.inflow_values(nat, u_nat, S)) if open_axes else None
    th = m.cell_field_from_natural(th_nat) + 0.01 * rng.standard_normal((m.n_cells,) + th_nat.shape[1:])
    return m, th, m.face_velocity_from_natural(u_nat), inflow


ADJ_CASES = ["open_box_inflow", "open_box", "stretched", "stretched_open"]


@pytest.mark.parametrize("S", [1, 2])
@pytest.mark.parametrize("case", ADJ_CASES)
def test_adjoint_matches_oracle_on_boundary_and_distance_meshes(case, S):
    m, th, u, inflow = _adjoint_case(case, S)
    mesh, cp, fp = library(m, inflow, reorder=True)
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(m.face_dist)
    om.set_inflow(inflow)
    rng = np.random.default_rng(31)
    lam = rng.standard_normal(th.shape)
    thd, ud, lamd = dev(rows_to_mesh(th, cp)), dev(rows_to_mesh(u, fp)), dev(rows_to_mesh(lam, cp))
    for lim in LIMS:
        tb, ub = FL.convect_adjoint(mesh, lim, thd, ud, lamd)
        tb_o, ub_o = om.rhs_vjp(lim, th, u, lam)
        assert np.abs(host(tb)[cp] - tb_o).max() <= 1e-12 * np.abs(tb_o).max(), lim
        assert np.abs(host(ub)[fp] - ub_o).max() <= 1e-12 * np.abs(ub_o).max(), lim
    mesh.close()


@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee", "smart", "minmod"])
@pytest.mark.parametrize("case", ADJ_CASES)
def test_run_adjoint_matches_oracle_on_boundary_and_distance_meshes(case, lim, scheme):
    """advect's backward (per-step reverse, checkpointed) against the oracle's stored sweep."""
    m, th, u, inflow = _adjoint_case(case, 1)
    mesh, cp, fp = library(m, inflow, reorder=True)
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(m.face_dist)
    om.set_inflow(inflow)
    dt = W.cfl_dt(m, u, 0.4)
    steps = 6
    lam_N = np.random.default_rng(33).standard_normal(th.shape)
    t0 = dev(rows_to_mesh(th, cp)).requires_grad_(True)
    ud = dev(rows_to_mesh(u, fp)).requires_grad_(True)
    out = FL.advect(mesh, lim, scheme, dt, t0, ud, steps, checkpoint_every=4)
    out.backward(dev(rows_to_mesh(lam_N, cp)))
    tb_o, ub_o = om.run_adjoint(lim, scheme, dt, th, u, steps, lam_N)
    assert np.abs(host(t0.grad)[cp] - tb_o).max() <= 1e-10 * np.abs(tb_o).max()
    assert np.abs(host(ud.grad)[fp] - ub_o).max() <= 1e-10 * np.abs(ub_o).max()
    want = om.run(lim, scheme, dt, th, u, steps)
    assert nrel(host(out)[cp], want) <= RUN_TOL
    mesh.close()
