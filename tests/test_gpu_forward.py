"""GPU parity of the forward operator and time steps against the CPU oracle.

Tolerances: per face the kernels and the oracle evaluate the same FP64 expressions, except that
the kernels may contract a*b+c into one fused multiply-add and sum a cell's faces in another
order; each stage therefore differs by a few units in the last place of the cell values.  One
operator application is compared at 1e-13 of max|rhs|; whole runs (hundreds of stages) at the
1e-10 max norm-relative error of the cell values that the method's accuracy target fixes.
Connectivity and the upwind selection are compared bit for bit.
"""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2110_03044_amd import fluxlim as FL, workloads as W

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


def mesh_pair(m, **kw):
    """Library mesh plus the user -> mesh maps."""
    mesh = FL.Mesh.from_arrays(m, device=0, **kw)
    cp, fp = mesh.permutation()
    return mesh, cp, fp


def to_mesh_cells(x, cp):
    out = np.empty_like(x)
    out[cp] = x
    return out


def to_mesh_faces(u, fp):
    out = np.empty_like(u)
    out[fp] = u
    return out


CASES = [
    ("line7", lambda: W.periodic_box(7, 1)),
    ("quad9r", lambda: W.renumber(W.periodic_box(9, 2), seed=4)),
    ("hex11r", lambda: W.renumber(W.periodic_box(11, 3), seed=5)),
    ("hex24r", lambda: W.renumber(W.periodic_box(24, 3), seed=6)),
]


@pytest.mark.parametrize("path", ["fused", "face"])
@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_selection_bit_exact(name, make, reorder, path):
    m = make()
    mesh, cp, fp = mesh_pair(m, reorder=reorder, face_path=(path == "face"))
    rng = np.random.default_rng(2)
    u = rng.standard_normal(m.n_faces)
    u[::7] = 0.0
    u[3::7] = -0.0
    got = mesh.debug_select(dev(to_mesh_faces(u, fp)))
    want = O.OracleMesh.from_arrays(m).select(u)
    assert np.array_equal(got[fp], cp[want])


@pytest.mark.parametrize("path", ["fused", "face"])
@pytest.mark.parametrize("S", [1, 3, 8])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_apply_matches_oracle(name, make, S, path):
    m = make()
    mesh, cp, fp = mesh_pair(m, reorder=True, face_path=(path == "face"))
    assert mesh.path == path
    rng = np.random.default_rng(S)
    th = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
    th[::3] = np.round(th[::3])  # repeated values: d_u == 0 and infinite-ratio cases
    u = rng.standard_normal(m.n_faces)
    om = O.OracleMesh.from_arrays(m)
    thd, ud = dev(to_mesh_cells(th, cp)), dev(to_mesh_faces(u, fp))
    for lim in LIMS:
        want = om.rhs(lim, th, u)
        got = host(FL.convect_apply(mesh, lim, thd, ud))[cp]
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), lim


def test_apply_plateaus_and_infinite_ratio():
    """Integer-valued steps: many faces with d_u == 0 and r = +-inf."""
    m = W.renumber(W.periodic_box(13, 3), seed=9)
    mesh, cp, fp = mesh_pair(m)
    rng = np.random.default_rng(5)
    th = rng.integers(0, 3, m.n_cells).astype(np.float64)
    u = rng.standard_normal(m.n_faces)
    om = O.OracleMesh.from_arrays(m)
    for lim in LIMS:
        want = om.rhs(lim, th, u)
        got = host(FL.convect_apply(mesh, lim, dev(to_mesh_cells(th, cp)), dev(to_mesh_faces(u, fp))))[cp]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("lim", LIMS[:6])
def test_line_config_euler_400_steps(lim):
    """1-D line, 200 cells, square wave + Gaussian, u = 1, Euler at CFL 1/2, one period."""
    wl = W.workload_line()
    mesh, cp, fp = mesh_pair(wl.mesh)
    th = dev(wl.theta0)
    FL.rk_steps(mesh, lim, "euler", wl.dt, th, dev(wl.u), wl.steps)
    want = O.OracleMesh.from_arrays(wl.mesh).run(lim, "euler", wl.dt, wl.theta0, wl.u, wl.steps)
    got = host(th)
    assert nrel(got, want) <= RUN_TOL
    # conservation and (for TVD limiters) boundedness on the GPU result itself
    assert abs(got.sum() - wl.theta0.sum()) <= 1e-13 * np.abs(wl.theta0).sum()
    if lim in ("upwind", "minmod", "vanleer", "superbee"):
        lo, hi = wl.theta0.min(), wl.theta0.max()
        assert got.min() >= lo - 1e-12 and got.max() <= hi + 1e-12


@pytest.mark.parametrize("path", ["fused", "face"])
@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("lim", ["minmod", "vanleer", "superbee", "smart"])
def test_box_ssprk3_run(lim, reorder, path):
    wl = W.workload_box(20, renumbered=True, steps=40)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=reorder, face_path=(path == "face"))
    th = dev(to_mesh_cells(wl.theta0, cp))
    FL.rk_steps(mesh, lim, "ssprk3", wl.dt, th, dev(to_mesh_faces(wl.u, fp)), wl.steps)
    want = O.OracleMesh.from_arrays(wl.mesh).run(lim, "ssprk3", wl.dt, wl.theta0, wl.u, wl.steps)
    got = host(th)[cp]
    assert nrel(got, want) <= RUN_TOL
    V = wl.mesh.cell_volume
    assert abs((V * got).sum() - (V * wl.theta0).sum()) <= 1e-13 * (V * np.abs(wl.theta0)).sum()


@pytest.mark.parametrize("path", ["fused", "face"])
def test_euler_multi_scalar_and_ragged(path):
    m = W.renumber(W.periodic_box(7, 3), seed=2)  # 343 cells: a ragged last block
    wl_u = m.face_velocity_from_natural(W.velocity_curl(7, seed=4))
    th = W.multi_scalar([m.cell_field_from_natural(W.field_blob_step(7)),
                         m.cell_field_from_natural(W.field_smooth_random(7, 3, 1)),
                         m.cell_field_from_natural(W.field_sphere(7))])
    dt = W.cfl_dt(m, wl_u, 0.3)
    mesh, cp, fp = mesh_pair(m, reorder=True, face_path=(path == "face"))
    t = dev(to_mesh_cells(th, cp))
    FL.rk_steps(mesh, "superbee", "euler", dt, t, dev(to_mesh_faces(wl_u, fp)), 25)
    want = O.OracleMesh.from_arrays(m).run("superbee", "euler", dt, th, wl_u, 25)
    assert nrel(host(t)[cp], want) <= RUN_TOL


def test_zero_steps_and_zero_velocity_and_determinism():
    wl = W.workload_box(9, renumbered=True)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    th0 = dev(to_mesh_cells(wl.theta0, cp))
    u = dev(to_mesh_faces(wl.u, fp))
    t = th0.clone()
    FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, t, u, 0)
    assert torch.equal(t, th0)
    FL.rk_steps(mesh, "vanleer", "euler", wl.dt, t, torch.zeros_like(u), 3)
    assert torch.equal(t, th0)  # zero flux: theta + dt * 0 is theta
    FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, t, torch.zeros_like(u), 3)
    assert (t - th0).abs().max().item() <= 4e-16 * th0.abs().max().item()
    a, b = th0.clone(), th0.clone()
    FL.rk_steps(mesh, "smart", "ssprk3", wl.dt, a, u, 7)
    FL.rk_steps(mesh, "smart", "ssprk3", wl.dt, b, u, 7)
    assert torch.equal(a, b)


def test_permute_roundtrip():
    wl = W.workload_box(10, renumbered=True)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    th = dev(wl.theta0)
    tm = mesh.cells_to_mesh(th)
    assert np.array_equal(host(tm), to_mesh_cells(wl.theta0, cp))
    assert torch.equal(mesh.cells_from_mesh(tm), th)
    u = dev(wl.u)
    um = mesh.faces_to_mesh(u)
    assert np.array_equal(host(um), to_mesh_faces(wl.u, fp))
    assert torch.equal(mesh.faces_from_mesh(um), u)


def test_box128_config_van_leer():
    """3-D periodic hex box 128^3 in generic incidence, curl velocity, blob + step, van Leer,
    SSP-RK3 at CFL 0.4, all 100 steps (library reorder, one multi-step call)."""
    wl = W.workload_box(128, steps=100)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    th = dev(to_mesh_cells(wl.theta0, cp))
    FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, th, dev(to_mesh_faces(wl.u, fp)), wl.steps)
    want = O.OracleMesh.from_arrays(wl.mesh).run("vanleer", "ssprk3", wl.dt, wl.theta0, wl.u, wl.steps)
    assert nrel(host(th)[cp], want) <= RUN_TOL


@pytest.mark.parametrize("path", ["fused", "face"])
@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
def test_deformation_time_dependent_velocity(scheme, path):
    """Section 4.1's deformation flow, reversed by cos(pi t / T): the stage velocity s(t) u is
    formed in the kernel; compared with the oracle forming it on the host."""
    wl = W.workload_deformation(18, period=0.5, scheme=scheme, cfl=0.3)
    sc = W.deformation_scales(wl.steps, wl.dt, 0.5, scheme)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True, face_path=(path == "face"))
    th = dev(to_mesh_cells(wl.theta0, cp))
    FL.rk_steps_scaled(mesh, "superbee", scheme, wl.dt, th, dev(to_mesh_faces(wl.u, fp)), sc)
    want = O.OracleMesh.from_arrays(wl.mesh).run_scaled("superbee", scheme, wl.dt, wl.theta0,
                                                         wl.u, sc)
    got = host(th)[cp]
    assert nrel(got, want) <= RUN_TOL
    V = wl.mesh.cell_volume
    assert abs((V * got).sum() - (V * wl.theta0).sum()) <= 1e-14


def test_scaled_steps_with_unit_scale_equal_plain_steps():
    wl = W.workload_box(10, renumbered=True, steps=6)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    a = dev(to_mesh_cells(wl.theta0, cp))
    b = a.clone()
    u = dev(to_mesh_faces(wl.u, fp))
    FL.rk_steps(mesh, "smart", "ssprk3", wl.dt, a, u, wl.steps)
    FL.rk_steps_scaled(mesh, "smart", "ssprk3", wl.dt, b, u, np.ones(3 * wl.steps))
    assert torch.equal(a, b)


@pytest.mark.parametrize("S", [1, 3, 8])
@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("areas", [False, True])
def test_slot_rate_table_gives_the_same_bits(areas, scheme, S):
    """Multi-step calls read the signed face rates E a_f u_f from per-call slot tables, staging
    each 256-cell tile's theta and halo in LDS where it fits (FL_OPT_LDS_STAGE; here S <= 3 on
    this 2197-cell mesh with ragged last tile) and reading 16-byte slot records otherwise; single
    steps and FL_OPT_SLOT_VELOCITY = 0 gather u through the face index.  All must give the same
    bits, with uniform or per-face areas and volumes, and match the oracle."""
    import dataclasses

    m = W.renumber(W.periodic_box(13, 3), seed=8)  # 2197 cells: ragged last block
    if areas:
        rng = np.random.default_rng(9)
        m = dataclasses.replace(m, face_area=m.face_area * rng.uniform(0.5, 1.5, m.n_faces),
                                cell_volume=m.cell_volume * rng.uniform(0.5, 1.5, m.n_cells))
    u = m.face_velocity_from_natural(W.velocity_curl(13, seed=3))
    th = W.multi_scalar([m.cell_field_from_natural(W.field_blob_step(13)),
                         m.cell_field_from_natural(W.field_smooth_random(13, 3, 2)),
                         m.cell_field_from_natural(W.field_sphere(13))] * 3)[:, :S]
    th = np.ascontiguousarray(th if S > 1 else th[:, 0])
    dt = W.cfl_dt(m, u, 0.3)
    mesh, cp, fp = mesh_pair(m, reorder=True)
    ud = dev(to_mesh_faces(u, fp))
    t0 = dev(to_mesh_cells(th, cp))
    steps = 9
    assert mesh.info.tile_cells == 256 and mesh.info.max_halo > 0
    try:
        runs = {}
        for opt, lds in ((1, 1), (1, 0), (0, 1)):
            FL.set_option("slot_velocity", opt)
            FL.set_option("lds_stage", lds)
            t = t0.clone()
            FL.rk_steps(mesh, "vanleer", scheme, dt, t, ud, steps)
            runs[opt, lds] = t
        one = t0.clone()
        for _ in range(steps):
            FL.rk_steps(mesh, "vanleer", scheme, dt, one, ud, 1)
    finally:
        FL.set_option("slot_velocity", 1)
        FL.set_option("lds_stage", 1)
    assert torch.equal(runs[1, 1], runs[1, 0])
    assert torch.equal(runs[1, 1], runs[0, 1])
    assert torch.equal(runs[1, 1], one)
    runs = {1: runs[1, 1]}
    want = O.OracleMesh.from_arrays(m).run("vanleer", scheme, dt, th, u, steps)
    assert nrel(host(runs[1])[cp], want) <= RUN_TOL


@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("name", ["hex6r", "line200"])
def test_lds_stage_single_tile_with_empty_halo(name, S):
    """A mesh of at most 256 cells is one tile whose halo is empty: the LDS stage then reads the
    halo array's padding entry and stores every lane's halo value to the spare LDS entry.  The
    multi-step run (LDS-staged forward) and the reverse step (LDS-staged adjoint) must equal the
    global-gather kernels bit for bit, and the run must match the oracle."""
    m = W.renumber(W.periodic_box(6, 3), seed=3) if name == "hex6r" else W.periodic_box(200, 1)
    rng = np.random.default_rng(4)
    th = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
    u = rng.standard_normal(m.n_faces)
    dt = W.cfl_dt(m, u, 0.3)
    mesh, cp, fp = mesh_pair(m, reorder=True)
    assert mesh.info.tile_cells == 256 and mesh.info.max_halo == 0
    ud = dev(to_mesh_faces(u, fp))
    t0 = dev(to_mesh_cells(th, cp))
    lam0 = dev(to_mesh_cells(rng.standard_normal(th.shape), cp))
    res = {}
    try:
        for lds in (1, 0):
            FL.set_option("lds_stage", lds)
            t = t0.clone()
            FL.rk_steps(mesh, "superbee", "ssprk3", dt, t, ud, 7)
            st = FL.stage_buffer(mesh, "ssprk3", S, 1)
            FL.rk_step_store(mesh, "vanalbada", "ssprk3", dt, t0.clone(), ud, st[0])
            lam = lam0.clone()
            ubar = torch.zeros_like(ud)
            FL.rk_step_adjoint(mesh, "vanalbada", "ssprk3", dt, st[0], ud, lam, ubar)
            res[lds] = (t, lam, ubar)
    finally:
        FL.set_option("lds_stage", 1)
    for x, y in zip(res[1], res[0]):
        assert torch.equal(x, y)
    want = O.OracleMesh.from_arrays(m).run("superbee", "ssprk3", dt, th, u, 7)
    assert nrel(host(res[1][0])[cp], want) <= RUN_TOL


@pytest.mark.parametrize("slot_velocity", [1, 0])
def test_scaled_steps_with_face_areas(slot_velocity):
    import dataclasses

    wl = W.workload_deformation(12, period=0.5, cfl=0.3)
    rng = np.random.default_rng(10)
    m = dataclasses.replace(wl.mesh,
                            face_area=wl.mesh.face_area * rng.uniform(0.5, 1.5, wl.mesh.n_faces),
                            cell_volume=wl.mesh.cell_volume * rng.uniform(0.5, 1.5, wl.mesh.n_cells))
    dt = W.cfl_dt(m, wl.u, 0.3)
    steps = 30
    sc = W.deformation_scales(steps, dt, 0.5, "ssprk3")
    mesh, cp, fp = mesh_pair(m, reorder=True)
    th = dev(to_mesh_cells(wl.theta0, cp))
    try:
        FL.set_option("slot_velocity", slot_velocity)
        FL.rk_steps_scaled(mesh, "superbee", "ssprk3", dt, th, dev(to_mesh_faces(wl.u, fp)), sc)
    finally:
        FL.set_option("slot_velocity", 1)
    want = O.OracleMesh.from_arrays(m).run_scaled("superbee", "ssprk3", dt, wl.theta0, wl.u, sc)
    assert nrel(host(th)[cp], want) <= RUN_TOL


@pytest.mark.parametrize("remap", [1, 2, 5, 8, 32, 64])
def test_xcd_launch_orders_give_the_same_bits(remap):
    """FL_OPT_XCD_REMAP only changes which workgroup takes which 256-cell tile (a bijection over
    the padded grid; padding workgroups exit): 26^3 = 17576 cells is 69 tiles, enough to engage
    it.  Forward runs and the LDS-staged reverse step must give the same bits as launch order."""
    wl = W.workload_box(26, renumbered=True, steps=3)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    t0 = dev(to_mesh_cells(wl.theta0, cp))
    u = dev(to_mesh_faces(wl.u, fp))
    lam0 = dev(to_mesh_cells(np.random.default_rng(3).standard_normal(wl.mesh.n_cells), cp))
    runs = []
    try:
        for r in (0, remap):
            FL.set_option("xcd_remap", r)
            t = t0.clone()
            FL.rk_steps(mesh, "smart", "ssprk3", wl.dt, t, u, wl.steps)
            st = FL.stage_buffer(mesh, "ssprk3", 1, 1)
            FL.rk_step_store(mesh, "vanalbada", "ssprk3", wl.dt, t0.clone(), u, st[0])
            lam = lam0.clone()
            ubar = torch.zeros_like(u)
            FL.rk_step_adjoint(mesh, "vanalbada", "ssprk3", wl.dt, st[0], u, lam, ubar)
            runs.append((t, lam, ubar))
    finally:
        FL.set_option("xcd_remap", 32)
    for x, y in zip(runs[0], runs[1]):
        assert torch.equal(x, y)


GENERAL = [
    ("tri9r", lambda: W.renumber(W.periodic_triangles(9), seed=13)),
    ("skew6r", lambda: W.renumber(W.periodic_skewed_box(6), seed=14)),
]


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("name,make", GENERAL, ids=[c[0] for c in GENERAL])
def test_general_cells_selection(name, make, reorder):
    """(C, D, U) per face on general cells: U is the one projected face's far cell, or -2 where
    the upwind side projects on several faces (the oracle's convention)."""
    m = make()
    mesh, cp, fp = mesh_pair(m, reorder=reorder)
    assert mesh.info.general == 1 and mesh.path == "face"
    rng = np.random.default_rng(3)
    u = rng.standard_normal(m.n_faces)
    u[::5] = 0.0
    got = mesh.debug_select(dev(to_mesh_faces(u, fp)))
    want = O.OracleMesh.from_arrays(m).select(u)
    cpm = np.append(cp, [-2, -2])  # maps -2 (and -1) to themselves
    assert np.array_equal(got[fp], cpm[want])


@pytest.mark.parametrize("S", [1, 3, 8])
@pytest.mark.parametrize("name,make", GENERAL, ids=[c[0] for c in GENERAL])
def test_general_cells_apply_matches_oracle(name, make, S):
    m = make()
    mesh, cp, fp = mesh_pair(m, reorder=True)
    rng = np.random.default_rng(S + 20)
    th = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
    th[::3] = np.round(th[::3])
    u = rng.standard_normal(m.n_faces)
    om = O.OracleMesh.from_arrays(m)
    thd, ud = dev(to_mesh_cells(th, cp)), dev(to_mesh_faces(u, fp))
    for lim in LIMS:
        want = om.rhs(lim, th, u)
        got = host(FL.convect_apply(mesh, lim, thd, ud))[cp]
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), lim


@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("lim", ["minmod", "vanleer", "superbee", "smart"])
def test_general_cells_runs(lim, scheme):
    """Triangles with the stream-function velocity and the sheared hexahedral lattice with a
    uniform velocity, 30 steps, against the oracle; conservation."""
    n = 16
    tri = W.renumber(W.periodic_triangles(n), seed=15)
    xy = W.triangle_centroids(n)
    th_tri = tri.cell_field_from_natural(
        np.exp(-((xy[:, 0] - 0.4) ** 2 + (xy[:, 1] - 0.6) ** 2) / 0.02) + (xy[:, 0] > 0.5))
    u_tri = tri.face_velocity_from_natural(W.velocity_stream_triangles(n, seed=4))
    sk = W.periodic_skewed_box(8)
    th_sk = W.field_blob_step(8)
    u_sk = W.velocity_uniform(sk, (0.6, -0.3, 0.8), 1.0)
    for m, th, u in ((tri, th_tri, u_tri), (sk, th_sk, u_sk)):
        dt = W.cfl_dt(m, u, 0.3)
        mesh, cp, fp = mesh_pair(m, reorder=True)
        t = dev(to_mesh_cells(th, cp))
        FL.rk_steps(mesh, lim, scheme, dt, t, dev(to_mesh_faces(u, fp)), 30)
        want = O.OracleMesh.from_arrays(m).run(lim, scheme, dt, th, u, 30)
        got = host(t)[cp]
        assert nrel(got, want) <= RUN_TOL
        V = m.cell_volume
        assert abs((V * got).sum() - (V * th).sum()) <= 1e-13 * (V * np.abs(th)).sum()


def test_general_cells_in_a_batch():
    """General cells join a batch through the face-path kernels: the same bits as the
    single-problem call (more cases in test_gpu_batch.py)."""
    m = W.periodic_triangles(6)
    mesh = FL.Mesh.from_arrays(m, device=0)
    th = dev(np.cos(np.arange(m.n_cells) * 0.3))
    u = dev(W.velocity_stream_triangles(6))
    dt = W.cfl_dt(m, W.velocity_stream_triangles(6), 0.3)
    a, c = th.clone(), th.clone()
    b = FL.Batch([(mesh, "vanleer", a, u, dt)])
    b.step(3)
    FL.rk_steps(mesh, "vanleer", "ssprk3", dt, c, u, 3)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    b.close()


def test_full_size_box256_sampled_first_stage_and_conservation():
    """The 256^3 random mesh of the benchmark, library reorder, in the launch configuration the
    benchmark times (multi-step call: per-call rates, LDS-staged stages).  The first stage output
    t1 = theta0 + dt rhs(theta0), stored by the two-step store call, is compared with the oracle's
    rhs at 20000 sampled cells (computed from theta0 alone); the two-step result conserves
    sum V theta and equals the plain two-step call bit for bit."""
    wl = W.workload_box(256, renumbered=True)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    assert mesh.info.tile_cells > 0
    t0 = dev(to_mesh_cells(wl.theta0, cp))
    u = dev(to_mesh_faces(wl.u, fp))
    stages = FL.stage_buffer(mesh, "ssprk3", 1, 2)
    a = t0.clone()
    FL.rk_steps_store(mesh, "vanleer", "ssprk3", wl.dt, a, u, stages, 2)
    b = t0.clone()
    FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, b, u, 2)
    assert torch.equal(a, b)
    rng = np.random.default_rng(17)
    cells = np.sort(rng.choice(wl.mesh.n_cells, 20000, replace=False))
    rhs = O.OracleMesh.from_arrays(wl.mesh).rhs_cells("vanleer", wl.theta0, wl.u, cells)
    want = wl.theta0[cells] + wl.dt * rhs
    got = host(stages[0, 1])[cp[cells]]
    assert np.abs(got - want).max() <= 1e-13 * np.abs(wl.theta0).max()
    V = wl.mesh.cell_volume[0]
    total0 = float(t0.sum()) * V
    assert abs(float(a.sum()) * V - total0) <= 1e-12 * abs(total0)


@pytest.fixture(scope="module")
def box256():
    """The 256^3 random mesh of the benchmark with its oracle view and the library mesh in the
    benchmark's launch configuration (library reorder, fused LDS-staged path)."""
    wl = W.workload_box(256, renumbered=True)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    assert mesh.path == "fused" and mesh.info.tile_cells > 0
    om = O.OracleMesh.from_arrays(wl.mesh)
    yield wl, mesh, cp, fp, om
    mesh.close()


@pytest.mark.parametrize("lim", ["minmod", "vanleer", "superbee", "smart"])
def test_full_size_box256_all_cells_two_steps(box256, lim):
    """Every one of the 16.8 M cells after a two-step SSP-RK3 call (per-call rate table, six
    LDS-staged stage launches) against the oracle's two steps, for each limiter the benchmark
    times at this size."""
    wl, mesh, cp, fp, om = box256
    th = dev(to_mesh_cells(wl.theta0, cp))
    FL.rk_steps(mesh, lim, "ssprk3", wl.dt, th, dev(to_mesh_faces(wl.u, fp)), 2)
    got = host(th)[cp]
    want = om.run(lim, "ssprk3", wl.dt, wl.theta0, wl.u, 2)
    err = nrel(got, want)
    print(f"256^3 {lim}: max norm-relative error {err:.2e}")
    assert err <= RUN_TOL


def _rotated_box(n, angle, seed):
    """Periodic box with each face normal turned by `angle` about a random axis (renormalised)."""
    import dataclasses

    m = W.periodic_box(n, 3)
    rng = np.random.default_rng(seed)
    nrm = m.face_normal.copy()
    ax = rng.standard_normal(nrm.shape)
    ax -= (ax * nrm).sum(1, keepdims=True) * nrm
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    nrm = nrm * np.cos(angle) + ax * np.sin(angle)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return dataclasses.replace(m, face_normal=nrm)


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("lim", ["vanleer", "superbee", "smart"])
def test_nearly_orthogonal_mesh_keeps_every_weight(lim, reorder):
    """Normals off the axes by ~1e-10 rad: every nonzero projection weight is kept (general cells
    on the face path), as in the oracle; one application at 1e-13 of max|rhs| and a 20-step run
    at the run tolerance."""
    n = 12
    m = _rotated_box(n, 1e-10, seed=3)
    mesh, cp, fp = mesh_pair(m, reorder=reorder)
    assert mesh.info.general == 1 and mesh.path == "face"
    u = W.velocity_curl(n)
    th0 = W.field_blob_step(n) + 1e-3 * np.random.default_rng(1).standard_normal(m.n_cells)
    om = O.OracleMesh.from_arrays(m)
    rhs = FL.convect_apply(mesh, lim, dev(to_mesh_cells(th0, cp)), dev(to_mesh_faces(u, fp)))
    want = om.rhs(lim, th0, u)
    assert np.abs(host(rhs)[cp] - want).max() <= 1e-13 * np.abs(want).max()
    dt = W.cfl_dt(m, u, 0.4)
    th = dev(to_mesh_cells(th0, cp))
    FL.rk_steps(mesh, lim, "ssprk3", dt, th, dev(to_mesh_faces(u, fp)), 20)
    assert nrel(host(th)[cp], om.run(lim, "ssprk3", dt, th0, u, 20)) <= RUN_TOL
    mesh.close()


def test_opt_in_finite_check():
    """FL_OPT_CHECK_FINITE: a NaN or an infinity in theta, u_f or dt gives FL_E_NONFINITE with
    nothing enqueued (theta unchanged); finite inputs run as without the check, bit for bit."""
    from paper_2110_03044_amd import _lib

    wl = W.workload_box(10, renumbered=True, steps=3)
    mesh, cp, fp = mesh_pair(wl.mesh, reorder=True)
    u = dev(to_mesh_faces(wl.u, fp))
    t0 = dev(to_mesh_cells(wl.theta0, cp))
    ref = t0.clone()
    FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, ref, u, 3)
    FL.set_option("check_finite", 1)
    try:
        t = t0.clone()
        FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, t, u, 3)
        assert torch.equal(t, ref)
        for bad_cell, bad_face, bad_dt in [(5, None, None), (None, 7, None), (None, None, np.inf)]:
            t = t0.clone()
            uu = u.clone()
            if bad_cell is not None:
                t[bad_cell] = float("nan")
            if bad_face is not None:
                uu[bad_face] = float("inf")
            before = t.clone()
            with pytest.raises(_lib.FluxLimError) as e:
                FL.rk_steps(mesh, "vanleer", "ssprk3", bad_dt if bad_dt else wl.dt, t, uu, 3)
            assert e.value.status == -6
            assert torch.equal(t.isnan(), before.isnan()) and torch.equal(
                torch.nan_to_num(t), torch.nan_to_num(before))
        t = t0.clone()
        t[3] = float("-inf")
        with pytest.raises(_lib.FluxLimError) as e:
            FL.convect_apply(mesh, "vanleer", t, u)
        assert e.value.status == -6
    finally:
        FL.set_option("check_finite", 0)
    t = t0.clone()
    t[5] = float("nan")
    FL.rk_steps(mesh, "vanleer", "ssprk3", wl.dt, t, u, 1)  # unchecked: runs
    torch.cuda.synchronize()
    mesh.close()


@pytest.mark.parametrize("S", [1, 2, 3, 5])
@pytest.mark.parametrize("case", ["line", "quad", "hex", "hex_varied", "hex_scaled"])
def test_forward_rates_give_the_same_bits(case, S):
    """On lattice meshes (aligned slots) the multi-step LDS stages read only each cell's forward
    face rates and take the backward ones from the neighbours (FL_OPT_FWD_RATES); the results
    must equal the per-slot rate tables' bit for bit, also with face areas, volumes and a
    time-dependent velocity scale, and for a tile count with a ragged end."""
    import dataclasses

    rng = np.random.default_rng(len(case) * 10 + S)
    if case == "line":
        m = W.renumber(W.periodic_box(700, 1), seed=3)
        u = W.velocity_uniform(m, (1.0, 0.0, 0.0))
    elif case == "quad":
        m = W.renumber(W.periodic_box(37, 2), seed=4)
        u = W.velocity_uniform(m, (0.6, -0.8, 0.0))
    else:
        n = 19
        m = W.renumber(W.periodic_box(n, 3), seed=5)
        u = m.face_velocity_from_natural(W.velocity_curl(n, seed=2))
        if case == "hex_varied":
            m = dataclasses.replace(m, cell_volume=m.cell_volume * rng.uniform(0.7, 1.3, m.n_cells),
                                    face_area=m.face_area * rng.uniform(0.7, 1.3, m.n_faces))
    th0 = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
    dt = W.cfl_dt(m, u, 0.3)
    mesh, cp, fp = mesh_pair(m, reorder=True)
    assert mesh.info.tile_cells == 256
    uu = dev(to_mesh_faces(u, fp))
    res = []
    try:
        for on in (1, 0):
            FL.set_option("fwd_rates", on)
            t = dev(to_mesh_cells(th0, cp))
            if case == "hex_scaled":
                sc = 0.5 + rng.random(3 * 6) if on == 1 else sc
                FL.rk_steps_scaled(mesh, "superbee", "ssprk3", dt, t, uu, sc)
            else:
                FL.rk_steps(mesh, "vanleer", "ssprk3", dt, t, uu, 6)
            torch.cuda.synchronize()
            res.append(t)
    finally:
        FL.set_option("fwd_rates", 1)
    assert torch.equal(res[0], res[1])
    om = O.OracleMesh.from_arrays(m)
    if case != "hex_scaled":
        want = om.run("vanleer", "ssprk3", dt, th0, u, 6)
        assert nrel(host(res[0])[cp], want) <= RUN_TOL
    mesh.close()
