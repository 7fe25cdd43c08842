"""Pins of the oracle's derivatives on meshes with boundary faces and face distances (no GPU).

The tangent and the reverse sweep take an inflow value as a constant and an exterior that
repeats its face's own cell as that cell (the boundary reading pinned in
test_oracle_boundary.py).  They are fixed here against:
* the Jacobian of the textbook first-order upwind scheme on an open line, written out as a
  matrix (both flow directions, with and without inflow values);
* central differences of the oracle's own operator, whose boundary faces and distance ratios
  are pinned in test_oracle_boundary.py and test_oracle_distances.py: an open box with inflow
  values and a stretched box (periodic and open), for the smooth van Albada and van Leer;
* the identity <J v, w> = <v, J^T w> between tangent and reverse sweep, for one operator
  application and for whole runs, every limiter.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_03044_amd import workloads as W

LIMS = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart", "central"]


def open_line(n, speed):
    """n cells on [0, 1]; faces 0..n-2 interior (+x normal), n-1 the right end (+x), n the left
    end (-x)."""
    m = W.open_box(n, 1, (0,))
    assert m.face_cells[n - 1, 1] == -1 and m.face_cells[n, 0] == 0
    return m, speed * m.face_normal[:, 0]


def upwind_line_jacobian(n, speed, dx, inflow):
    """d rhs / d theta of theta_i' = (|u| / dx) (theta_up(i) - theta_i), theta_up the upwind
    neighbour; beyond the inflow end the exterior holds the inflow value (a constant) or repeats
    the end cell."""
    c = abs(speed) / dx
    J = -c * np.eye(n)
    if speed > 0:
        J += c * np.eye(n, k=-1)  # theta_{i-1}
        if not inflow:
            J[0, 0] += c
    else:
        J += c * np.eye(n, k=1)  # theta_{i+1}
        if not inflow:
            J[n - 1, n - 1] += c
    return J


@pytest.mark.parametrize("with_inflow", [True, False])
@pytest.mark.parametrize("speed", [1.0, -0.7])
def test_upwind_open_line_jacobian(speed, with_inflow):
    n = 9
    m, u = open_line(n, speed)
    om = O.OracleMesh.from_arrays(m)
    if with_inflow:
        inflow = np.full(m.n_faces, np.nan)
        inflow[n if speed > 0 else n - 1] = 0.3
        om.set_inflow(inflow)
    rng = np.random.default_rng(1)
    th = rng.random(n)
    J = upwind_line_jacobian(n, speed, 1.0 / n, with_inflow)
    lam = rng.standard_normal(n)
    tb, _ = om.rhs_vjp("upwind", th, u, lam)
    assert np.allclose(tb, J.T @ lam, rtol=1e-13, atol=1e-12)
    v = rng.standard_normal(n)
    assert np.allclose(om.rhs_jvp("upwind", th, u, v), J @ v, rtol=1e-13, atol=1e-12)


def _open_box_case(S):
    wl = W.workload_open_box(6, renumbered=True, S=S)
    rng = np.random.default_rng(3)
    th = wl.theta0 + 0.05 * rng.standard_normal(wl.theta0.shape)
    return wl.mesh, th, wl.u, wl.inflow, None


def _stretched_case(open_):
    nat = W.stretched_box(7, 3, amp=0.5, open_axes=(0,) if open_ else ())
    m = W.renumber(nat, seed=5)
    u = m.face_velocity_from_natural(W.velocity_open_box(nat))
    th = m.cell_field_from_natural(W.field_smooth_random(7, 3, seed=4)) + 1.0
    inflow = m.face_field_from_natural(W.inflow_values(nat, W.velocity_open_box(nat))) \
        if open_ else None
    return m, th, u, inflow, m.face_dist


CASES = {"open_box_S1": lambda: _open_box_case(1), "open_box_S2": lambda: _open_box_case(2),
         "stretched": lambda: _stretched_case(False),
         "stretched_open": lambda: _stretched_case(True)}


def oracle_for(m, inflow, dist):
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(dist)
    om.set_inflow(inflow)
    return om


@pytest.mark.parametrize("lim", ["vanalbada", "vanleer"])
@pytest.mark.parametrize("case", list(CASES))
def test_tangent_matches_central_differences(case, lim):
    """J v + (dL/du) du against (L(theta + eps v, u + eps du) - L(theta - eps v, u - eps du)) /
    (2 eps); du is scaled so that no face velocity changes sign."""
    m, th, u, inflow, dist = CASES[case]()
    om = oracle_for(m, inflow, dist)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(th.shape)
    du = rng.standard_normal(u.shape)
    eps = 1e-6
    du *= 0.5 * np.abs(u).min() / (eps * np.abs(du).max())
    du = np.clip(du, -1.0, 1.0)
    jv = om.rhs_jvp(lim, th, u, v, du)
    fd = (om.rhs(lim, th + eps * v, u + eps * du) - om.rhs(lim, th - eps * v, u - eps * du)) / (2 * eps)
    assert np.abs(jv - fd).max() <= 2e-6 * np.abs(fd).max(), (case, lim)


@pytest.mark.parametrize("lim", LIMS)
@pytest.mark.parametrize("case", list(CASES))
def test_reverse_sweep_is_the_transpose_of_the_tangent(case, lim):
    m, th, u, inflow, dist = CASES[case]()
    om = oracle_for(m, inflow, dist)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(th.shape)
    du = rng.standard_normal(u.shape)
    w = rng.standard_normal(th.shape)
    lhs = float(np.sum(om.rhs_jvp(lim, th, u, v, du) * w))
    tb, ub = om.rhs_vjp(lim, th, u, w)
    rhs = float(np.sum(v * tb) + du @ ub)
    scale = float(np.sum(np.abs(om.rhs_jvp(lim, th, u, np.abs(v), np.abs(du)) * w))) + abs(lhs)
    assert abs(lhs - rhs) <= 1e-13 * scale, (case, lim, lhs, rhs)


@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee", "smart", "minmod"])
@pytest.mark.parametrize("case", ["open_box_S2", "stretched_open"])
def test_run_adjoint_against_run_tangent(case, lim, scheme):
    m, th, u, inflow, dist = CASES[case]()
    om = oracle_for(m, inflow, dist)
    dt = W.cfl_dt(m, u, 0.4)
    rng = np.random.default_rng(13)
    v = rng.standard_normal(th.shape)
    du = rng.standard_normal(u.shape)
    w = rng.standard_normal(th.shape)
    steps = 4
    _, jv = om.run_tangent(lim, scheme, dt, th, u, steps, v, du)
    tb, ub = om.run_adjoint(lim, scheme, dt, th, u, steps, w)
    lhs = float(np.sum(jv * w))
    rhs = float(np.sum(v * tb) + du @ ub)
    assert abs(lhs - rhs) <= 1e-12 * (np.sum(np.abs(jv * w)) + abs(lhs)), (lhs, rhs)
