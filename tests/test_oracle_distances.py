"""Pins of the oracle's distance-weighted upstream difference (no GPU).

Algorithm 1D forms the gradient ratio of a non-uniform line as r = (d_i / d_U)(theta_C -
theta_U) / (theta_D - theta_C), with d_i the distance across the face and d_U the distance
across the face upwind of C; Algorithm UNS divides every projected difference by the distance
across its face and the face difference by d_i.  The tests write Algorithm 1D's ratio out on
stretched lines (both flow directions, periodic and with an inflow end) and check the ratio's
invariances on a stretched box.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_03044_amd import workloads as W

LIMS = ["minmod", "vanleer", "vanalbada", "superbee", "smart", "central", "upwind"]


def psi_text(lim, r):
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


def line_1d(th, d, speed, lim, t_left=None):
    """Algorithm 1D on a line of n cells: face i joins cells i and i + 1 (periodic when
    t_left is None; else faces 0 .. n-2 are interior and the left end's exterior holds t_left,
    its distance d[n]), d[i] the distance across face i.  Returns theta_f of the interior faces
    (all n faces when periodic)."""
    n = th.shape[0]
    nf = n if t_left is None else n - 1
    out = np.empty(nf)
    for i in range(nf):
        if speed > 0:
            C, D, U, dU = i, (i + 1) % n, i - 1, i - 1
        else:
            C, D, U, dU = (i + 1) % n, i, (i + 2) % n, (i + 1) % n
        if t_left is None:
            tU, dist_U = th[U % n], d[dU % n]
        elif speed > 0 and U < 0:
            tU, dist_U = t_left, d[n]
        elif speed < 0 and U >= n:
            raise AssertionError("flow to the left leaves through the left end")
        else:
            tU, dist_U = th[U], d[dU]
        du = th[D] - th[C]
        r = (d[i] / dist_U) * (th[C] - tU) / du
        out[i] = th[C] + 0.5 * psi_text(lim, r) * du
    return out


@pytest.mark.parametrize("speed", [1.0, -1.0])
@pytest.mark.parametrize("lim", LIMS)
def test_stretched_periodic_line_is_algorithm_1d(lim, speed):
    n = 23
    m = W.stretched_box(n, 1, amp=0.6)
    rng = np.random.default_rng(7)
    th = rng.random(n)
    u = speed * m.face_normal[:, 0]
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(m.face_dist)
    got = om.face_values(lim, th, u)
    want = line_1d(th, m.face_dist, speed, lim)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-15)
    # the distance ratio matters: the unweighted ratio differs somewhere
    if lim not in ("upwind", "central"):
        om.set_distances(None)
        assert np.abs(om.face_values(lim, th, u) - want).max() > 1e-6


@pytest.mark.parametrize("lim", LIMS)
def test_stretched_open_line_uses_the_boundary_distance(lim):
    """Flow to the right: the first interior face's far-upwind value is the inflow value, at the
    distance the caller gives for the left boundary face."""
    n = 15
    m = W.stretched_box(n, 1, amp=0.5, open_axes=(0,))
    th = np.linspace(0.1, 0.9, n) ** 2
    u = m.face_normal[:, 0].copy()
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(m.face_dist)
    inflow = np.full(m.n_faces, np.nan)
    inflow[n] = 0.45
    om.set_inflow(inflow)
    got = om.face_values(lim, th, u)[: n - 1]
    want = line_1d(th, m.face_dist, 1.0, lim, t_left=0.45)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("lim", ["vanleer", "superbee", "vanalbada"])
def test_distance_scale_and_uniform_distances(lim):
    """Only the ratios of distances enter: scaling all of them changes nothing beyond rounding,
    and equal distances give the unweighted operator."""
    m = W.renumber(W.stretched_box(7, 3, amp=0.5), seed=9)
    wl = W.workload_box(7)
    th = m.cell_field_from_natural(wl.theta0)
    u = m.face_velocity_from_natural(wl.u)
    om = O.OracleMesh.from_arrays(m)
    om.set_distances(m.face_dist)
    a = om.rhs(lim, th, u)
    om.set_distances(7.3 * m.face_dist)
    b = om.rhs(lim, th, u)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    om.set_distances(np.full(m.n_faces, 0.3))
    c = om.rhs(lim, th, u)
    om.set_distances(None)
    d = om.rhs(lim, th, u)
    assert np.abs(c - d).max() <= 1e-12 * np.abs(d).max()
    assert np.abs(a - d).max() > 1e-8 * np.abs(d).max()
