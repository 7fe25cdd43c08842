"""Pins of the oracle's boundary faces (no GPU).

Reading: a boundary face (one cell, nbr = -1, normal pointing out) borders an exterior cell with
no other faces.  That cell holds the caller's inflow value where the flow enters and inflow
values were given, and repeats the interior cell's value otherwise (Section 2's cell-to-face
shift copies the single cell of such a face).  The rules of the closed mesh then apply as they
are.  The tests below check that against closed forms written out here: the textbook
first-order upwind update with a Dirichlet inflow, the face values the rule gives at both kinds
of boundary face and next to them, conservation counted with the boundary fluxes, the TVD and
min/max properties with an inflow, and the periodic line seen as an open one.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_03044_amd import workloads as W

LIMS = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart", "central"]
# psi(0) = 0: an inflow face with d_U = 0 takes the exterior value itself
PSI0_ZERO = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart"]
TVD_LIMS = ["upwind", "minmod", "vanleer", "superbee"]


def psi_text(lim, r):
    """Sweby's limiters written out (minmod, van Leer, van Albada, superbee, SMART)."""
    if lim == "upwind":
        return 0.0
    if lim == "central":
        return 1.0
    if lim == "minmod":
        return max(0.0, min(1.0, r))
    if lim == "vanleer":
        return (r + abs(r)) / (1.0 + abs(r))
    if lim == "vanalbada":
        return (r * r + r) / (r * r + 1.0)
    if lim == "superbee":
        return max(0.0, min(1.0, 2.0 * r), min(r, 2.0))
    if lim == "smart":
        return max(0.0, min(2.0 * r, 0.25 + 0.75 * r, 4.0))
    raise ValueError(lim)


def open_line(n, speed):
    """n cells on [0, 1], boundary faces at both ends; faces 0..n-2 interior (+x normal), face
    n-1 the right end (+x), face n the left end (-x)."""
    m = W.open_box(n, 1, (0,))
    fc = m.face_cells
    assert fc[n - 1, 1] == -1 and fc[n, 0] == 0 and fc[n, 1] == -1
    u = speed * m.face_normal[:, 0]
    return m, u


@pytest.mark.parametrize("speed", [1.0, -0.7])
@pytest.mark.parametrize("with_inflow", [True, False])
def test_open_line_upwind_euler_is_the_textbook_scheme(speed, with_inflow):
    """Upwind, Euler: theta_i' = theta_i - nu (theta_i - theta_{i-1}) (flow to the right) with
    theta_{-1} the inflow value (or theta_0 itself without inflow values), and the mirror image
    for a flow to the left."""
    n = 17
    m, u = open_line(n, speed)
    rng = np.random.default_rng(3)
    th = rng.random(n)
    t_in = 0.625
    om = O.OracleMesh.from_arrays(m)
    assert om.n_boundary == 2
    inflow = np.full(m.n_faces, np.nan)
    inflow[n if speed > 0 else n - 1] = t_in
    if with_inflow:
        om.set_inflow(inflow)
    dt = 0.4 / n
    got = om.run("upwind", "euler", dt, th, u, 1)
    nu = abs(speed) * dt * n
    if speed > 0:
        left = np.concatenate([[t_in if with_inflow else th[0]], th[:-1]])
    else:
        left = np.concatenate([th[1:], [t_in if with_inflow else th[-1]]])
    want = th - nu * (th - left)
    assert np.allclose(got, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lim", LIMS)
def test_boundary_face_values(lim):
    """Outflow face: the interior value (d_u = 0).  Inflow face: the inflow value where
    psi(0) = 0, (inflow + interior)/2 for central differencing (d_U = 0 upwind of it), the
    interior value without inflow values.  The interior face next to the inflow face takes the
    inflow value as its far-upwind value: r = (theta_0 - theta_in) / (theta_1 - theta_0)."""
    n = 9
    m, u = open_line(n, 1.0)
    th = np.array([0.3, 0.5, 0.45, 0.9, 0.1, 0.2, 0.7, 0.65, 0.4])
    t_in = 0.15
    om = O.OracleMesh.from_arrays(m)
    tf0 = om.face_values(lim, th, u)
    assert tf0[n - 1] == th[-1]  # outflow
    assert tf0[n] == th[0]       # inflow, no inflow values
    inflow = np.full(m.n_faces, np.nan)
    inflow[n] = t_in
    om.set_inflow(inflow)
    tf = om.face_values(lim, th, u)
    assert tf[n - 1] == th[-1]
    if lim == "central":
        assert tf[n] == pytest.approx(0.5 * (t_in + th[0]), abs=1e-16)
    else:
        assert tf[n] == t_in
    r = (th[0] - t_in) / (th[1] - th[0])
    want = th[0] + 0.5 * psi_text(lim, r) * (th[1] - th[0])
    assert tf[0] == pytest.approx(want, rel=1e-15, abs=1e-16)
    # without inflow values the far-upwind value of face 0 repeats theta_0: r = 0
    om.set_inflow(None)
    want0 = th[0] + 0.5 * psi_text(lim, 0.0) * (th[1] - th[0])
    assert om.face_values(lim, th, u)[0] == pytest.approx(want0, rel=1e-15, abs=1e-16)


@pytest.mark.parametrize("lim", LIMS)
@pytest.mark.parametrize("S", [1, 3])
def test_open_box_conserves_with_boundary_fluxes(lim, S):
    """sum_c V_c (theta' - theta)_c = -dt sum over boundary faces of a_f u_f theta_f (Euler),
    with the boundary face values of the rule written out for the upwind case and taken from
    the oracle's face values otherwise."""
    wl = W.workload_open_box(7, renumbered=True, S=S)
    m = wl.mesh
    om = O.OracleMesh.from_arrays(m)
    om.set_inflow(wl.inflow)
    th1 = om.run(lim, "euler", wl.dt, wl.theta0, wl.u, 1)
    vol = m.cell_volume[:, None] if S > 1 else m.cell_volume
    lhs = (vol * (th1 - wl.theta0)).sum(axis=0)
    b = m.face_cells[:, 1] < 0
    own = m.face_cells[b, 0]
    tf = om.face_values(lim, wl.theta0, wl.u)[b]
    if lim == "upwind":
        inflow_face = ~(wl.u[b] > 0)
        ext = wl.inflow[b]
        want_tf = np.where(inflow_face[:, None] if S > 1 else inflow_face, ext, wl.theta0[own])
        assert np.array_equal(tf, want_tf)
    au = (m.face_area * wl.u)[b]
    rhs = -wl.dt * ((au[:, None] if S > 1 else au) * tf).sum(axis=0)
    scale = (vol * np.abs(wl.theta0)).sum(axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale)


@pytest.mark.parametrize("lim", TVD_LIMS)
def test_open_line_with_inflow_is_tvd_and_bounded(lim):
    """Euler at CFL 0.5, flow to the right, a square wave entering through the left end: the
    total variation of (theta_in, theta_0, ..., theta_{n-1}) never grows and every value stays
    within the initial range joined with the inflow value."""
    n = 60
    m, u = open_line(n, 1.0)
    x = (np.arange(n) + 0.5) / n
    th = np.where((x > 0.2) & (x < 0.4), 1.0, 0.0) + 0.3 * np.exp(-((x - 0.7) / 0.05) ** 2)
    t_in = 0.8
    inflow = np.full(m.n_faces, np.nan)
    inflow[n] = t_in
    om = O.OracleMesh.from_arrays(m)
    om.set_inflow(inflow)
    lo, hi = min(th.min(), t_in), max(th.max(), t_in)

    def tv(v):
        return np.abs(np.diff(np.concatenate([[t_in], v]))).sum()

    dt = 0.5 / n
    for _ in range(150):
        nxt = om.run(lim, "euler", dt, th, u, 1)
        assert tv(nxt) <= tv(th) + 1e-12
        assert nxt.min() >= lo - 1e-12 and nxt.max() <= hi + 1e-12
        th = nxt


@pytest.mark.parametrize("lim", LIMS)
def test_uniform_field_is_steady_without_inflow_values(lim):
    """A constant field under a constant velocity on the open box: every flux through a cell
    cancels (interior faces carry the constant, boundary faces repeat it), so rhs = 0."""
    m = W.renumber(W.open_box(5, 3, (0, 2)), seed=4)
    u = W.velocity_uniform(m, (1.0, 0.3, -0.2))
    th = np.full(m.n_cells, 0.37)
    om = O.OracleMesh.from_arrays(m)
    assert np.abs(om.rhs(lim, th, u)).max() <= 1e-14
    # an inflow value equal to the constant changes nothing
    om.set_inflow(np.full(m.n_faces, 0.37))
    assert np.abs(om.rhs(lim, th, u)).max() <= 1e-14


def test_periodic_line_is_an_open_line_with_its_wrap_value():
    """Upwind, Euler: the periodic line's step equals the open line's step when the inflow value
    of the left end is the last cell's value (the wrap face's upwind value)."""
    n = 13
    rng = np.random.default_rng(5)
    th = rng.random(n)
    dt = 0.45 / n
    per = W.periodic_box(n, 1)
    want = O.OracleMesh.from_arrays(per).run("upwind", "euler", dt, th, W.velocity_1d(per), 1)
    m, u = open_line(n, 1.0)
    om = O.OracleMesh.from_arrays(m)
    inflow = np.full(m.n_faces, np.nan)
    inflow[n] = th[-1]
    om.set_inflow(inflow)
    got = om.run("upwind", "euler", dt, th, u, 1)
    assert np.array_equal(got, want)


def test_mesh_checks():
    """nbr = -1 marks a boundary face; own = -1 is not a face."""
    fc = np.array([[0, 1], [1, -1], [-1, 0]], dtype=np.int32)
    nrm = np.array([[1.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0]])
    with pytest.raises(ValueError):
        O.OracleMesh(fc, nrm, n_cells=2)
    fc[2] = [0, -1]
    assert O.OracleMesh(fc, nrm, n_cells=2).n_boundary == 2
