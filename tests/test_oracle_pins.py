"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test ties the oracle to something other than itself: values printed in the paper, closed
forms of linear special cases, the one-dimensional stencil algorithm of the paper evaluated in
exact rational arithmetic, lattice geometry, conservation/TVD invariants, an independent sparse
matrix evaluation of the paper's algebraic chain, and finite differences for the derivatives.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from oracle.mini_oracle import AlgebraicMesh, psi_np
from paper_2110_03044_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LIMS = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart", "central"]
TVD_LIMS = ["upwind", "minmod", "vanleer", "superbee"]


def read_matrices(path):
    mats, cur, rows = {}, None, []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("matrix"):
            if cur:
                mats[cur] = np.array(rows, dtype=float)
            cur, rows = line.split()[1], []
        else:
            rows.append([float(x) for x in line.split()])
    mats[cur] = np.array(rows, dtype=float)
    return mats


# ------------------------------------------------------------------------------------------
# Limiters
# ------------------------------------------------------------------------------------------

def test_superbee_matches_table1():
    """Table 1, superbeexty: F(r) = (psi(r) - 1)/2 at hand-evaluated points."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "superbee_table1.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for r, p, F in rows:
        r, p, F = float(r), float(p), float(F)
        assert O.psi("superbee", r) == p
        assert 0.5 * (O.psi("superbee", r) - 1.0) == F


@pytest.mark.parametrize("lim,points", [
    ("minmod", [(-1, 0), (0.5, 0.5), (1, 1), (4, 1)]),
    ("vanleer", [(-1, 0), (1, 1), (3, 1.5), (0.5, 2 / 3)]),
    ("vanalbada", [(1, 1), (-0.5, -0.2), (0, 0), (2, 1.2), (-1, 0)]),
    ("smart", [(-1, 0), (0.1, 0.2), (1, 1), (3, 2.5), (5, 4), (10, 4)]),
    ("upwind", [(-1, 0), (1, 0), (5, 0)]),
    ("central", [(-1, 1), (1, 1), (5, 1)]),
])
def test_limiter_textbook_points(lim, points):
    for r, v in points:
        assert O.psi(lim, r) == pytest.approx(v, abs=1e-15)


@pytest.mark.parametrize("lim", ["minmod", "vanleer", "vanalbada", "superbee"])
def test_limiter_symmetry(lim):
    """Symmetric limiters satisfy psi(r)/r = psi(1/r) (Sweby)."""
    for r in [0.1, 0.3, 0.7, 1.3, 2.5, 7.0]:
        assert O.psi(lim, r) / r == pytest.approx(O.psi(lim, 1.0 / r), rel=1e-14)


def test_limiters_in_second_order_tvd_region():
    """Sweby's region: psi(1) = 1 and 0 <= psi <= min(2r, 2) for r > 0; SMART leaves it."""
    rs = np.linspace(1e-3, 10, 2001)
    for lim in ["minmod", "vanleer", "superbee"]:
        assert O.psi(lim, 1.0) == 1.0
        v = np.array([O.psi(lim, r) for r in rs])
        assert (v >= 0).all() and (v <= np.minimum(2 * rs, 2.0) + 1e-15).all()
    v = np.array([O.psi("smart", r) for r in rs])
    assert v.max() == 4.0  # beyond Sweby's bound 2


def test_limiter_infinity_limits():
    for lim in LIMS:
        assert O.psi(lim, 1e30) == pytest.approx(O.psi(lim, 1e17), abs=1e-15)
        assert O.psi(lim, -1e30) == pytest.approx(O.psi(lim, -1e17), abs=1e-15)
        assert O.psi(lim, math.inf) == O.psi(lim, 1e30)


@pytest.mark.parametrize("lim", LIMS)
def test_dpsi_matches_finite_difference(lim):
    for r in [-2.3, -0.4, 0.13, 0.37, 0.8, 1.4, 2.7, 4.1, 6.3]:
        h = 1e-7
        fd = (O.psi(lim, r + h) - O.psi(lim, r - h)) / (2 * h)
        assert O.dpsi(lim, r) == pytest.approx(fd, abs=1e-6)


def test_mini_oracle_limiters_agree_with_oracle():
    rs = np.concatenate([np.linspace(-5, 8, 1301), [1e20, -1e20, 0.0]])
    for lim in LIMS:
        a = psi_np(lim, rs)
        b = np.array([O.psi(lim, r) for r in rs])
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


# ------------------------------------------------------------------------------------------
# The paper's printed example (Section 2 and Section 3.1)
# ------------------------------------------------------------------------------------------

def test_printed_adjacency_matrices():
    """A_FF = B B^T - W reproduces the printed face adjacency exactly; A^D = offdiag(E B^T)
    reproduces the printed directed adjacency once E is oriented +1 on the cell the normal
    enters (the printed E_{C->F} carries the opposite sign)."""
    M = read_matrices(os.path.join(GOLDEN, "paper_example_2d.txt"))
    E_printed = M["E_CF"]
    am = AlgebraicMesh.from_incidence(-E_printed)
    np.testing.assert_array_equal(am.A.toarray(), M["A_FF"])
    np.testing.assert_array_equal(am.AD.toarray(), M["AD_FF"])
    # A_FF is non-negative and symmetric, A^D has A_FF's pattern (text of Section 3.1)
    assert (M["A_FF"] >= 0).all() and (M["A_FF"] == M["A_FF"].T).all()
    np.testing.assert_array_equal(np.abs(M["AD_FF"]), M["A_FF"])
    # with the printed sign the formula gives the negated matrix: the reading is recorded here
    am2 = AlgebraicMesh.from_incidence(E_printed)
    np.testing.assert_array_equal(am2.AD.toarray(), -M["AD_FF"])


def test_printed_exact_sequence_has_one_typo():
    """E_{F->V} E_{C->F} should vanish (Section 2); the printed pair leaves one entry."""
    M = read_matrices(os.path.join(GOLDEN, "paper_example_2d.txt"))
    P = M["E_FV"] @ M["E_CF"]
    nz = np.argwhere(P != 0)
    assert nz.tolist() == [[3, 2]] and P[3, 2] == -2


def test_exact_sequence_of_generated_velocity():
    """Discrete curl => zero discrete divergence in every cell, exactly (Section 2): the face
    areas are uniform, so the signed sum of the normal velocities of each cell vanishes."""
    for n in (4, 7, 16):
        m = W.periodic_box(n, 3)
        u = W.velocity_curl(n, seed=5)
        div = np.zeros(m.n_cells)
        np.add.at(div, m.face_cells[:, 0], u)
        np.add.at(div, m.face_cells[:, 1], -u)
        assert np.abs(div).max() == 0.0
        assert 0.99 < np.abs(u).max() < 1.01


# ------------------------------------------------------------------------------------------
# Face selection against lattice geometry
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("renum", [False, True])
def test_far_upwind_is_the_lattice_cell_behind(renum):
    n = 5
    nat = W.periodic_box(n, 3)
    m = W.renumber(nat, seed=11) if renum else nat
    u_nat = W.velocity_curl(n, seed=3)
    u = m.face_velocity_from_natural(u_nat)
    cdu = O.OracleMesh.from_arrays(m).select(u)
    # back to natural numbering
    cnew = m.cell_new_of_old if renum else np.arange(nat.n_cells)
    old_of_new = np.empty_like(cnew)
    old_of_new[cnew] = np.arange(cnew.size)
    fnew = m.face_new_of_old if renum else np.arange(nat.n_faces)
    ijk = lambda c: np.array([c % n, (c // n) % n, c // (n * n)])
    lin = lambda v: int(v[0] % n + n * (v[1] % n) + n * n * (v[2] % n))
    for f_old in range(nat.n_faces):
        C, D, U = (old_of_new[x] for x in cdu[fnew[f_old]])
        a, c_own = divmod(f_old, nat.n_cells)
        own, nbr = nat.face_cells[f_old]
        if u_nat[f_old] > 0:
            assert (C, D) == (own, nbr)
        else:
            assert (C, D) == (nbr, own)
        assert U == lin(2 * ijk(C) - ijk(D)), f_old
        assert U not in (C, D)


def test_zero_velocity_takes_the_negative_sign():
    """Table 1, signxty: x > 0 ? +1 : -1, so u_f = 0 (and -0.0) selects C = nbr."""
    m = W.periodic_box(6, 2)
    u = np.zeros(m.n_faces)
    u[::3] = -0.0
    u[1::3] = 1.0
    cdu = O.OracleMesh.from_arrays(m).select(u)
    pos = u > 0
    np.testing.assert_array_equal(cdu[pos, 0], m.face_cells[pos, 0])
    np.testing.assert_array_equal(cdu[~pos, 0], m.face_cells[~pos, 1])
    np.testing.assert_array_equal(cdu[~pos, 1], m.face_cells[~pos, 0])


def test_hex_weights_are_zero_or_one():
    m = W.renumber(W.periodic_box(4, 3), seed=2)
    om = O.OracleMesh.from_arrays(m)
    for f in range(0, m.n_faces, 7):
        for side in (False, True):
            faces, w = om.side_weights(f, side)
            assert len(w) == 6
            assert sorted(w.tolist()) == [0.0] * 5 + [1.0]


# ------------------------------------------------------------------------------------------
# Algorithm 1D in exact arithmetic
# ------------------------------------------------------------------------------------------

def _psi_exact(lim, r):
    if lim == "minmod":
        return max(Fraction(0), min(Fraction(1), r))
    if lim == "superbee":
        return max(Fraction(0), max(min(Fraction(1), 2 * r), min(r, Fraction(2))))
    if lim == "smart":
        return max(Fraction(0), min(2 * r, Fraction(1, 4) + Fraction(3, 4) * r, Fraction(4)))
    if lim == "vanleer":
        return (r + abs(r)) / (1 + abs(r))
    if lim == "vanalbada":
        return (r * r + r) / (r * r + 1)
    raise ValueError(lim)


@pytest.mark.parametrize("lim", ["minmod", "superbee", "smart", "vanleer", "vanalbada"])
def test_face_values_follow_algorithm_1d(lim):
    """Algorithm 1D (Section 3.3) on a uniform periodic line, evaluated in rationals."""
    th = [0, 1, 3, 4, 2, 2, -1, 5, 5, 6, 2, 0]
    n = len(th)
    m = W.periodic_box(n, 1)
    rng = np.random.default_rng(4)
    u = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    got = O.OracleMesh.from_arrays(m).face_values(lim, np.array(th, float), u)
    T = [Fraction(x) for x in th]
    for i in range(n):
        if u[i] > 0:
            tC, tU, tD = T[i], T[i - 1], T[(i + 1) % n]
        else:
            tC, tU, tD = T[(i + 1) % n], T[(i + 2) % n], T[i]
        if tD == tC:
            want = tC
        else:
            r = (tC - tU) / (tD - tC)
            want = (tC + tD) / 2 + (_psi_exact(lim, r) - 1) * (tD - tC) / 2
        assert abs(float(want) - got[i]) <= 1e-15 * max(1.0, abs(float(want))), (i, want, got[i])


# ------------------------------------------------------------------------------------------
# Literal algebraic chain (Algorithm 3) vs the gather oracle
# ------------------------------------------------------------------------------------------

def _tiny_meshes():
    out = []
    for n, d in [(7, 1), (5, 2), (4, 3), (5, 3)]:
        nat = W.periodic_box(n, d)
        out.append((f"{d}d{n}", nat))
        out.append((f"{d}d{n}r", W.renumber(nat, seed=n + d)))
    # general cells: triangles (one or two projected faces per side, weights +-1/sqrt 2) and a
    # sheared hexahedral lattice (five projected faces per side)
    for name, nat in [("tri5", W.periodic_triangles(5)), ("skew4", W.periodic_skewed_box(4))]:
        out.append((name, nat))
        out.append((name + "r", W.renumber(nat, seed=11)))
    return out


@pytest.mark.parametrize("name,mesh", _tiny_meshes(), ids=lambda x: x if isinstance(x, str) else "")
def test_algebraic_chain_matches_gather_oracle(name, mesh):
    rng = np.random.default_rng(7)
    th = rng.standard_normal(mesh.n_cells)
    u = rng.standard_normal(mesh.n_faces)
    am = AlgebraicMesh.from_arrays(mesh)
    om = O.OracleMesh.from_arrays(mesh)
    # the unsimplified and precomputed forms of d_U coincide
    np.testing.assert_allclose(am.upstream_difference(th, u),
                               am.upstream_difference_unsimplified(th, u), rtol=0, atol=1e-14)
    for lim in LIMS:
        tf_a = am.face_values(lim, th, u)
        tf_o = om.face_values(lim, th, u)
        np.testing.assert_allclose(tf_a, tf_o, rtol=0, atol=2e-14)
        np.testing.assert_allclose(am.rhs(lim, th, u), om.rhs(lim, th, u), rtol=0,
                                   atol=2e-13 * np.abs(om.rhs(lim, th, u)).max())


def test_algebraic_chain_euler_run_matches_oracle():
    wl = W.workload_line(n=50, steps=40)
    am = AlgebraicMesh.from_arrays(wl.mesh)
    om = O.OracleMesh.from_arrays(wl.mesh)
    for lim in LIMS[:6]:
        a = am.euler_run(lim, wl.dt, wl.theta0, wl.u, wl.steps)
        b = om.run(lim, "euler", wl.dt, wl.theta0, wl.u, wl.steps)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


def test_printed_simplified_form_picks_downstream_faces():
    """The printed d_U = (Q S + T) theta equals theta_{D'} - theta_D (the faces beyond D) on a
    uniform line, which is why the corrected (Q T - S) form is used."""
    n = 9
    m = W.periodic_box(n, 1)
    am = AlgebraicMesh.from_arrays(m)
    th = np.arange(n, dtype=float) ** 2
    u = np.ones(n)
    printed = u * (am.S @ th) + am.T @ th
    want_down = np.array([th[(i + 2) % n] - th[(i + 1) % n] for i in range(n)])
    np.testing.assert_array_equal(printed, want_down)
    want_up = np.array([th[i] - th[i - 1] for i in range(n)])
    np.testing.assert_array_equal(am.upstream_difference(th, u), want_up)


# ------------------------------------------------------------------------------------------
# Closed forms of the linear special cases
# ------------------------------------------------------------------------------------------

def test_upwind_line_is_binomial_convolution():
    """psi = 0 (paper's F = -1/2) at CFL 1/2: theta^N_i = sum_k C(N,k) 2^-N theta^0_{i-k}."""
    wl = W.workload_line()
    th = O.OracleMesh.from_arrays(wl.mesh).run("upwind", "euler", wl.dt, wl.theta0, wl.u, wl.steps)
    N, n = wl.steps, wl.mesh.n_cells
    wts = np.array([math.comb(N, k) for k in range(N + 1)], dtype=float) * 2.0**-N
    want = np.zeros(n)
    for k in range(N + 1):
        want += wts[k] * np.roll(wl.theta0, k)
    np.testing.assert_allclose(th, want, rtol=0, atol=2e-15)


def _fft_closed_form(n, vel, lim, scheme, dt, steps, th0):
    """Linear schemes with constant velocity on a periodic box are circulant: evolve in Fourier."""
    h = 1.0 / n
    k = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / n  # kappa = 2 pi m / n
    K = np.meshgrid(k, k, k, indexing="ij")
    sym = np.zeros((n, n, n), dtype=complex)
    for d in range(3):
        v = vel[d]
        e = np.exp(1j * K[d])  # shift +e_d
        if lim == "upwind":
            # v>0: -v/h (theta_c - theta_{c-e}); v<0: -v/h (theta_{c+e} - theta_c)
            sym += -(v / h) * (1 - 1 / e) if v > 0 else -(v / h) * (e - 1)
        else:  # central
            sym += -(v / h) * (e - 1 / e) / 2
    z = dt * sym
    amp = 1 + z if scheme == "euler" else 1 + z + z * z / 2 + z**3 / 6
    T = np.fft.fftn(th0.reshape((n, n, n), order="F"))
    return np.real(np.fft.ifftn(T * amp**steps)).ravel(order="F")


@pytest.mark.parametrize("lim", ["upwind", "central"])
@pytest.mark.parametrize("scheme", ["euler", "ssprk3"])
def test_linear_schemes_match_fourier_closed_form(lim, scheme):
    n = 8
    m = W.periodic_box(n, 3)
    vel = (0.7, -0.4, 0.25)
    u = W.velocity_uniform(m, vel)
    th0 = W.field_smooth_random(n, 3, seed=9) + W.field_blob_step(n)
    dt = 0.2 / n
    got = O.OracleMesh.from_arrays(m).run(lim, scheme, dt, th0, u, 12)
    want = _fft_closed_form(n, vel, lim, scheme, dt, 12, th0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("lim", ["upwind", "central"])
@pytest.mark.parametrize("scheme", ["euler", "ssprk3"])
def test_time_dependent_velocity_matches_fourier_closed_form(lim, scheme):
    """u(t) = s(t) u0 with constant u0: every stage multiplies each Fourier mode by its own
    symbol scaled by s; SSP-RK3 composes its three stages with those factors."""
    n, steps = 8, 9
    m = W.periodic_box(n, 3)
    vel = (0.6, 0.35, -0.5)
    u = W.velocity_uniform(m, vel)
    th0 = W.field_smooth_random(n, 3, seed=4) + W.field_blob_step(n)
    dt = 0.15 / n
    sc = W.deformation_scales(steps, dt, 0.05, scheme)  # crosses zero: the flow reverses
    assert sc.min() < 0 < sc.max()
    got = O.OracleMesh.from_arrays(m).run_scaled(lim, scheme, dt, th0, u, sc)
    h = 1.0 / n
    kk = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / n
    K = np.meshgrid(kk, kk, kk, indexing="ij")
    T = np.fft.fftn(th0.reshape((n, n, n), order="F"))

    def symbol(s):
        out = np.zeros((n, n, n), dtype=complex)
        for d in range(3):
            v = s * vel[d]
            e = np.exp(1j * K[d])
            if lim == "upwind":
                out += -(v / h) * (1 - 1 / e) if v > 0 else -(v / h) * (e - 1)
            else:
                out += -(v / h) * (e - 1 / e) / 2
        return dt * out

    ns = 1 if scheme == "euler" else 3
    for i in range(steps):
        z = [symbol(sc[i * ns + j]) for j in range(ns)]
        if scheme == "euler":
            T = T * (1 + z[0])
        else:
            t1 = T * (1 + z[0])
            t2 = 0.75 * T + 0.25 * (t1 * (1 + z[1]))
            T = T / 3 + 2.0 / 3.0 * (t2 * (1 + z[2]))
    want = np.real(np.fft.ifftn(T)).ravel(order="F")
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_deformation_flow_conserves_and_returns():
    """Section 4.1: the reversed deformation flow returns the sphere towards its initial shape
    (the error at t = T is well below the error at t = T/2) and conserves mass exactly.  A short
    period (T = 0.5) keeps the deformation resolvable on a 20^3 mesh; at T = 3 the sphere (three
    cells in radius) is smeared into a sheet before the reversal."""
    wl = W.workload_deformation(20, period=0.5)
    om = O.OracleMesh.from_arrays(wl.mesh)
    sc = W.deformation_scales(wl.steps, wl.dt, 0.5, wl.scheme)
    half = wl.steps // 2
    mid = om.run_scaled("superbee", wl.scheme, wl.dt, wl.theta0, wl.u, sc[: 3 * half])
    end = om.run_scaled("superbee", wl.scheme, wl.dt, mid, wl.u, sc[3 * half:])
    V = wl.mesh.cell_volume
    l1 = lambda x: float((V * np.abs(x - wl.theta0)).sum())
    assert l1(end) < 0.5 * l1(mid)
    assert abs((V * end).sum() - (V * wl.theta0).sum()) <= 1e-14
    # the normal velocity on the planes x, y, z in {0, 1} vanishes: the wrap carries no flux
    assert np.abs(wl.u[: wl.mesh.n_cells][np.arange(wl.mesh.n_cells) % 20 == 19]).max() < 1e-28


@pytest.mark.parametrize("lim", LIMS)
def test_3d_with_axis_flow_reduces_to_1d(lim):
    """Orthogonal meshes recover the one-dimensional formulation (Section 3.1, Conclusions)."""
    n = 16
    m3 = W.periodic_box(n, 3)
    m1 = W.periodic_box(n, 1)
    line = W.field_square_gauss_1d(n) + 0.1 * W.field_smooth_random(n, 1, 3)
    th3 = np.tile(line, n * n)  # theta depends on x only
    u3 = W.velocity_uniform(m3, (1.0, 0, 0))
    u1 = W.velocity_uniform(m1, (1.0, 0, 0))
    dt = 0.4 / n
    a = O.OracleMesh.from_arrays(m3).run(lim, "ssprk3", dt, th3, u3, 20)
    b = O.OracleMesh.from_arrays(m1).run(lim, "ssprk3", dt, line, u1, 20)
    np.testing.assert_array_equal(a.reshape(n * n, n), np.tile(b, (n * n, 1)))


# ------------------------------------------------------------------------------------------
# Invariants
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("lim", LIMS[:6])
def test_renumbering_and_orientation_invariance(lim):
    n = 8
    nat = W.periodic_box(n, 3)
    rn = W.renumber(nat, seed=21)
    u = W.velocity_curl(n, seed=1)
    th = W.field_blob_step(n)
    dt = W.cfl_dt(nat, u, 0.4)
    a = O.OracleMesh.from_arrays(nat).run(lim, "ssprk3", dt, th, u, 10)
    b = O.OracleMesh.from_arrays(rn).run(lim, "ssprk3", dt, rn.cell_field_from_natural(th),
                                          rn.face_velocity_from_natural(u), 10)
    np.testing.assert_allclose(rn.cell_field_to_natural(b), a, rtol=0, atol=1e-13)


@pytest.mark.parametrize("lim", LIMS[:6])
def test_conservation_on_periodic_mesh(lim):
    wl = W.workload_box(12, renumbered=True, steps=30)
    om = O.OracleMesh.from_arrays(wl.mesh)
    th = om.run(lim, "ssprk3", wl.dt, wl.theta0, wl.u, wl.steps)
    V = wl.mesh.cell_volume
    m0 = (V * wl.theta0).sum()
    assert abs((V * th).sum() - m0) <= 1e-13 * (V * np.abs(wl.theta0)).sum()


def test_conservation_multi_scalar_matches_single():
    wl = W.workload_box(6, renumbered=True, steps=5)
    om = O.OracleMesh.from_arrays(wl.mesh)
    th2 = W.multi_scalar([wl.theta0, 1.0 - 2.0 * wl.theta0, wl.theta0**2])
    out = om.run("vanleer", "ssprk3", wl.dt, th2, wl.u, 5)
    for s in range(3):
        np.testing.assert_array_equal(out[:, s], om.run("vanleer", "ssprk3", wl.dt, th2[:, s], wl.u, 5))


def _tv(x):
    return np.abs(np.diff(np.append(x, x[0]))).sum()


@pytest.mark.parametrize("lim", TVD_LIMS)
def test_tvd_and_bounded_in_1d(lim):
    """Harten/Sweby: 0 <= psi <= 2, 0 <= psi/r <= 2 and CFL <= 1/2 give a TVD forward-Euler step."""
    wl = W.workload_line()
    om = O.OracleMesh.from_arrays(wl.mesh)
    th = wl.theta0.copy()
    tv0, lo, hi = _tv(th), th.min(), th.max()
    for _ in range(wl.steps):
        nxt = om.run(lim, "euler", wl.dt, th, wl.u, 1)
        assert _tv(nxt) <= _tv(th) + 1e-12 * tv0
        assert nxt.min() >= lo - 1e-12 * (hi - lo) and nxt.max() <= hi + 1e-12 * (hi - lo)
        th = nxt


def test_smart_is_not_tvd_with_euler():
    """SMART (psi up to 4) lies outside Sweby's region: the forward-Euler run overshoots."""
    wl = W.workload_line()
    th = O.OracleMesh.from_arrays(wl.mesh).run("smart", "euler", wl.dt, wl.theta0, wl.u, wl.steps)
    assert th.max() > wl.theta0.max() + 0.1


def test_free_stream_preservation():
    wl = W.workload_box(10, renumbered=True, steps=20)
    om = O.OracleMesh.from_arrays(wl.mesh)
    th = np.full(wl.mesh.n_cells, 0.75)
    for lim in ["vanleer", "superbee", "smart"]:
        out = om.run(lim, "ssprk3", wl.dt, th, wl.u, 20)
        assert np.abs(out - 0.75).max() <= 1e-13


def test_sampled_rhs_equals_full_rhs():
    wl = W.workload_box(7, renumbered=True)
    om = O.OracleMesh.from_arrays(wl.mesh)
    full = om.rhs("superbee", wl.theta0, wl.u)
    cells = np.array([0, 5, 17, 100, wl.mesh.n_cells - 1])
    np.testing.assert_array_equal(om.rhs_cells("superbee", wl.theta0, wl.u, cells), full[cells])


# ------------------------------------------------------------------------------------------
# Derivatives
# ------------------------------------------------------------------------------------------

def _fd_setup(n=5, seed=0):
    wl = W.workload_box(n, renumbered=True)
    rng = np.random.default_rng(seed)
    th = wl.theta0 + 1e-2 * rng.standard_normal(wl.mesh.n_cells)  # no flat neighbours
    return wl, th, rng


@pytest.mark.parametrize("lim", ["vanalbada", "upwind", "central", "vanleer"])
def test_rhs_jvp_matches_finite_difference(lim):
    wl, th, rng = _fd_setup()
    om = O.OracleMesh.from_arrays(wl.mesh)
    v = rng.standard_normal(th.size)
    du = rng.standard_normal(wl.u.size)
    eps = 1e-7  # truncation ~1e-8 relative, rounding ~1e-8
    umin = np.abs(wl.u).min()
    du *= min(1.0, 0.5 * umin / eps) / np.abs(du).max()  # unit size, no face changes sign
    jv = om.rhs_jvp(lim, th, wl.u, v, du)
    fd = (om.rhs(lim, th + eps * v, wl.u + eps * du) - om.rhs(lim, th - eps * v, wl.u - eps * du)) / (2 * eps)
    np.testing.assert_allclose(jv, fd, rtol=0, atol=1e-6 * np.abs(jv).max())


@pytest.mark.parametrize("lim", LIMS)
def test_rhs_vjp_is_transpose_of_jvp(lim):
    wl, th, rng = _fd_setup(seed=1)
    om = O.OracleMesh.from_arrays(wl.mesh)
    v = rng.standard_normal(th.size)
    du = rng.standard_normal(wl.u.size)
    w = rng.standard_normal(th.size)
    jv = om.rhs_jvp(lim, th, wl.u, v, du)
    tb, ub = om.rhs_vjp(lim, th, wl.u, w)
    lhs = jv @ w
    rhs = v @ tb + du @ ub
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(jv).max() * np.abs(w).sum())


@pytest.mark.parametrize("scheme", ["euler", "ssprk3"])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee", "smart"])
def test_run_adjoint_is_transpose_of_run_tangent(lim, scheme):
    wl, th, rng = _fd_setup(seed=2)
    om = O.OracleMesh.from_arrays(wl.mesh)
    v = rng.standard_normal(th.size)
    du = rng.standard_normal(wl.u.size)
    w = rng.standard_normal(th.size)
    _, jv = om.run_tangent(lim, scheme, wl.dt, th, wl.u, 4, v, du)
    tb, ub = om.run_adjoint(lim, scheme, wl.dt, th, wl.u, 4, w)
    lhs, rhs = jv @ w, v @ tb + du @ ub
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(jv) @ np.abs(w))


def test_run_adjoint_matches_finite_difference_of_loss():
    """d/d(theta0) and d/du of J = |theta_N - target|^2 / 2 for the smooth van Albada limiter."""
    wl, th, rng = _fd_setup(seed=3)
    om = O.OracleMesh.from_arrays(wl.mesh)
    target = wl.theta0 * 0.5
    steps = 6

    def J(t0, u):
        tn = om.run("vanalbada", "ssprk3", wl.dt, t0, u, steps)
        return 0.5 * ((tn - target) ** 2).sum()

    tn = om.run("vanalbada", "ssprk3", wl.dt, th, wl.u, steps)
    tb, ub = om.run_adjoint("vanalbada", "ssprk3", wl.dt, th, wl.u, steps, tn - target)
    for k in range(3):
        v = rng.standard_normal(th.size)
        du = rng.standard_normal(wl.u.size)
        eps = 1e-6
        du *= min(1.0, 0.5 * np.abs(wl.u).min() / eps) / np.abs(du).max()  # no sign flips
        fd = (J(th + eps * v, wl.u + eps * du) - J(th - eps * v, wl.u - eps * du)) / (2 * eps)
        ad = v @ tb + du @ ub
        assert ad == pytest.approx(fd, rel=1e-6)


def test_general_cells_conservation_and_free_stream():
    """On triangles with the exactly solenoidal stream-function velocity: a constant field is
    steady (d_u = d_U = 0, so theta_f = theta_C and rhs = theta div u = 0 up to rounding), and
    every run conserves sum V theta."""
    n = 12
    m = W.periodic_triangles(n)
    u = W.velocity_stream_triangles(n, seed=4)
    om = O.OracleMesh.from_arrays(m)
    const = np.full(m.n_cells, 2.5)
    assert np.abs(om.rhs("superbee", const, u)).max() <= 1e-12
    xy = W.triangle_centroids(n)
    th = np.exp(-((xy[:, 0] - 0.4) ** 2 + (xy[:, 1] - 0.6) ** 2) / 0.02)
    dt = W.cfl_dt(m, u, 0.4)
    out = om.run("vanleer", "ssprk3", dt, th, u, 30)
    V = m.cell_volume
    assert abs((V * out).sum() - (V * th).sum()) <= 1e-14 * (V * th).sum()
    assert out.min() >= -1e-12 and out.max() <= 1.0 + 1e-12  # van Leer keeps the bounds here


def test_general_cell_weights_by_hand():
    """Triangle faces: the horizontal face of the upper triangle below it projects only on that
    triangle's diagonal, with weight 1/sqrt 2; a diagonal face projects on two faces."""
    m = W.periodic_triangles(4)
    om = O.OracleMesh.from_arrays(m)
    C2 = 16
    f = 0  # horizontal edge of square (0, 0): own = upper(0, -1) = cell 2*(0 + 4*3) + 1 = 25
    faces, w = om.side_weights(f, side_nbr=False)
    nz = [(int(j), float(x)) for j, x in zip(faces, w) if x != 0.0]
    assert m.face_cells[f, 0] == 25
    # the diagonal of square (0, 3) is face 2*C2 + 12; t_j points into the upper triangle (its nbr)
    assert len(nz) == 1 and nz[0][0] == 2 * C2 + 12
    assert nz[0][1] == pytest.approx(1.0 / np.sqrt(2.0), abs=1e-15)
    faces, w = om.side_weights(2 * C2 + 5, side_nbr=False)
    assert sum(1 for x in w if x != 0.0) == 2


# ------------------------------------------------------------------------------------------
# Derivatives at the special points of the gradient ratio (Section 3's Sweby form and ratio):
# theta_f = theta_C + g(d_U, d_u), g(a, b) = psi(a / b) b / 2.  Where d_u = 0, g vanishes for
# every d_U, and its derivative along d_u > 0 is the limit of g(a, b) / b = psi(a / b) / 2 as
# b -> 0+, i.e. psi(+-inf) / 2 with the sign of d_U (psi(0) / 2 where d_U = 0 too).  Where
# |r| is evaluated as infinite, psi is constant.  The pins below take one-sided difference
# quotients of the oracle's own face values, on the side where d_u > 0, at steps small enough
# that the quotient is exactly psi(+-inf) / 2 in binary arithmetic, and compare them with the
# tangent that the jvp / vjp use.
# ------------------------------------------------------------------------------------------

def _line(n=5):
    fc = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.int32)
    nrm = np.tile([1.0, 0.0, 0.0], (n, 1))
    return O.OracleMesh(fc, nrm, n_cells=n)


LINE_F, LINE_U, LINE_C, LINE_D = 2, 1, 2, 3  # with u > 0: face 2 joins C = 2 to D = 3, U = 1


def _tangent_of_face(om, lim, th, cell, f=LINE_F):
    u = np.ones(om.n_faces)
    e = np.zeros_like(th)
    e[cell] = 1.0
    _, dtf = om.face_values_jvp(lim, th, u, e)
    return dtf[f]


def _quotient(om, lim, th, cell, step, f=LINE_F):
    """(theta_f(theta + step e_cell) - theta_f(theta)) / step, exactly as the oracle rounds."""
    u = np.ones(om.n_faces)
    t1 = th.copy()
    t1[cell] += step
    return (om.face_values(lim, t1, u)[f] - om.face_values(lim, th, u)[f]) / step


@pytest.mark.parametrize("dU_sign", [1.0, -1.0])
@pytest.mark.parametrize("lim", LIMS)
def test_derivative_where_face_difference_vanishes(lim, dU_sign):
    om = _line()
    th = np.array([0.37, -dU_sign, 0.0, 0.0, 0.61])  # d_u = 0, d_U = dU_sign
    half_inf = 0.5 * O.lib().orc_psi_inf(O.lim_id(lim), int(dU_sign))
    tiny = 2.0 ** -70  # d_U / tiny = 2^70 > 1e18: the ratio is evaluated as infinite
    # theta_D up (d_u > 0): the quotient is exactly psi(+-inf) / 2 ...
    q = _quotient(om, lim, th, LINE_D, tiny)
    assert q == half_inf
    assert _tangent_of_face(om, lim, th, LINE_D) == q
    # ... and at a step in the finite range it tends to it (van Leer / van Albada: 1/r terms)
    assert abs(_quotient(om, lim, th, LINE_D, 1e-7) - q) <= 1e-6
    # theta_C down is also d_u > 0: theta_f = theta_C + g, so the quotient is 1 - psi(+-inf)/2
    q = _quotient(om, lim, th, LINE_C, -tiny)
    assert q == 1.0 - half_inf
    assert _tangent_of_face(om, lim, th, LINE_C) == q
    # theta_U moves d_U only, and g(., 0) = 0
    assert _quotient(om, lim, th, LINE_U, 1e-3) == 0.0
    assert _tangent_of_face(om, lim, th, LINE_U) == 0.0


@pytest.mark.parametrize("lim", LIMS)
def test_derivative_where_both_differences_vanish(lim):
    """d_u = d_U = 0: along d_u with d_U = 0 held, g(0, b) = psi(0) b / 2 (central: b / 2)."""
    om = _line()
    th = np.array([0.37, 0.0, 0.0, 0.0, 0.61])
    for step in (2.0 ** -70, 1e-3):
        q = _quotient(om, lim, th, LINE_D, step)
        assert q == 0.5 * O.psi(lim, 0.0)
        assert _tangent_of_face(om, lim, th, LINE_D) == q
    assert _tangent_of_face(om, lim, th, LINE_U) == 0.0


@pytest.mark.parametrize("lim", LIMS)
def test_derivative_where_ratio_is_infinite(lim):
    """0 < d_u with |r| > 1e18: psi is its value at infinity, constant in d_U and d_u."""
    om = _line()
    for sgn in (1.0, -1.0):
        th = np.array([0.37, -sgn, 0.0, 2.0 ** -70, 0.61])  # r = sgn 2^70
        half_inf = 0.5 * O.lib().orc_psi_inf(O.lim_id(lim), int(sgn))
        for step in (2.0 ** -72, -(2.0 ** -72)):  # r stays beyond 1e18 either way
            assert _quotient(om, lim, th, LINE_D, step) == half_inf
        assert _tangent_of_face(om, lim, th, LINE_D) == half_inf
        assert _quotient(om, lim, th, LINE_U, 1e-3) == 0.0
        assert _tangent_of_face(om, lim, th, LINE_U) == 0.0


def test_vjp_uses_the_same_special_point_derivatives():
    """The reverse sweep's partials at d_u = 0 and in the infinite-ratio band equal the one-sided
    quotients above: <vjp(e_c), e_D> over the cells of face 2's two neighbours."""
    om = _line()
    u = np.ones(om.n_faces)
    for lim in LIMS:
        for th in (np.array([0.37, -1.0, 0.0, 0.0, 0.61]),
                   np.array([0.37, -1.0, 0.0, 2.0 ** -70, 0.61])):
            jv = om.rhs_jvp(lim, th, u, np.eye(5)[LINE_D])
            for c in range(5):
                tb, _ = om.rhs_vjp(lim, th, u, np.eye(5)[c])
                assert tb[LINE_D] == pytest.approx(jv[c], abs=1e-15)
            # rhs_3 - rhs_2 picks up face 2's flux twice (own 2, nbr 3): its tangent is the
            # quotient of the face value, plus those of faces 1 and 3 through theta_3
            _, dtf = om.face_values_jvp(lim, th, u, np.eye(5)[LINE_D])
            assert dtf[LINE_F] == 0.5 * O.lib().orc_psi_inf(O.lim_id(lim), 1)
            assert jv[3] - jv[2] == pytest.approx(2 * dtf[2] - dtf[1] - dtf[3], abs=1e-15)


@pytest.mark.parametrize("a,b", [(0.3, 0.7), (-1.1, 0.4), (2.5, -0.2), (1e-9, 1.0), (1.0, 1e-12),
                                 (-3.0, -1e-5), (0.5, 0.5), (1.0, -1.0)])
def test_van_albada_partials_match_symbolic(a, b):
    """psi_vA(a/b) b / 2 = a b (a + b) / (2 (a^2 + b^2)); its partials in exact rationals.  The
    oracle forms g_b = (psi - r psi') / 2, which cancels for small |r|: compared at 1e-15
    absolute (the partials are O(1) quantities) or 1e-13 relative."""
    om = _line()
    th = np.array([0.37, -a, 0.0, b, 0.61])  # d_U = 0 - (-a) = a, d_u = b
    A, B = Fraction(a), Fraction(b)
    D = (A * A + B * B) ** 2
    ga = B * B * (B * B + 2 * A * B - A * A) / D / 2
    gb = A * A * (A * A + 2 * A * B - B * B) / D / 2
    assert _tangent_of_face(om, "vanalbada", th, LINE_U) == pytest.approx(-float(ga), rel=1e-13, abs=1e-15)
    assert _tangent_of_face(om, "vanalbada", th, LINE_D) == pytest.approx(float(gb), rel=1e-13, abs=1e-15)
    # the limits at b -> 0 are psi_vA(+-inf) / 2 = 1/2 and 0
    th0 = np.array([0.37, -a, 0.0, 0.0, 0.61])
    assert _tangent_of_face(om, "vanalbada", th0, LINE_D) == 0.5
    assert _tangent_of_face(om, "vanalbada", th0, LINE_U) == 0.0
