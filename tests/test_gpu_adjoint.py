"""GPU parity of the discrete adjoint against the CPU oracle's reverse sweep, tangent and finite
differences.

Tolerances: the adjoint kernels sum a cell's contributions in another order than the oracle's
serial scatter, so one reverse application agrees to a few ulps of the largest contribution
(compared at 1e-12 of max|grad|); reverse sweeps over many steps at 1e-10 norm-relative, as the
forward runs.  Finite differences use a smooth (van Albada) run whose field has no two equal
neighbours (no d_u = 0 kinks) and whose velocity perturbation flips no face's sign.  Near-flat
regions (differences of ~1e-3 from the seeded noise) make the central difference's truncation
error grow fast with the step (1.8e-4 relative at eps = 1e-5 and 1e-6 at eps = 1e-6 on the 16^3
case, measured with the oracle alone), so the 16^3 check uses eps = 3e-8 (1.5e-7 relative error for the oracle itself;
the velocity direction curves more than theta), against a 1e-6 relative bar.
"""

import dataclasses
import zlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2110_03044_amd import fluxlim as FL, workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
LIMS = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart", "central"]


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def maps(mesh):
    cp, fp = mesh.permutation()
    return cp, fp


def cells_in(x, cp):
    out = np.empty_like(x)
    out[cp] = x
    return out


def noisy_box(n, seed=0, renumbered=True):
    wl = W.workload_box(n, renumbered=renumbered)
    rng = np.random.default_rng(seed)
    th = wl.theta0 + 1e-3 * rng.standard_normal(wl.mesh.n_cells)
    return wl, th, rng


@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("lim", LIMS)
def test_operator_adjoint_matches_oracle(lim, reorder, S):
    wl, th1, rng = noisy_box(9, seed=S)
    m = wl.mesh
    th = np.stack([th1] + [rng.standard_normal(m.n_cells) for _ in range(S - 1)], 1) if S > 1 else th1
    th[::4] = np.round(th[::4])  # plateaus: d_u == 0 and infinite ratios
    lam = rng.standard_normal(th.shape)
    u = wl.u.copy()
    u[::9] = 0.0
    mesh = FL.Mesh.from_arrays(m, device=0, reorder=reorder)
    cp, fp = maps(mesh)
    uf = np.empty_like(u)
    uf[fp] = u
    tb, ub = FL.convect_adjoint(mesh, lim, dev(cells_in(th, cp)), dev(uf), dev(cells_in(lam, cp)))
    tb_o, ub_o = O.OracleMesh.from_arrays(m).rhs_vjp(lim, th, u, lam)
    got_t, got_u = host(tb)[cp], host(ub)[fp]
    assert np.abs(got_t - tb_o).max() <= 1e-12 * np.abs(tb_o).max()
    assert np.abs(got_u - ub_o).max() <= 1e-12 * np.abs(ub_o).max()


def test_operator_adjoint_accumulates_and_skips_null_u_bar():
    wl, th, rng = noisy_box(6)
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0)
    lam = dev(rng.standard_normal(th.shape))
    t, u = dev(th), dev(wl.u)
    tb1, ub1 = FL.convect_adjoint(mesh, "vanalbada", t, u, lam)
    tb2 = tb1.clone()
    ub2 = ub1.clone()
    FL.convect_adjoint(mesh, "vanalbada", t, u, lam, tb2, ub2)
    assert torch.allclose(tb2, 2 * tb1, rtol=1e-15, atol=0) and torch.allclose(ub2, 2 * ub1, rtol=1e-15, atol=0)
    from paper_2110_03044_amd._lib import lib
    import ctypes
    tb3 = torch.zeros_like(t)
    st = lib().fl_convect_adjoint(mesh.handle, 3, 1, ctypes.c_void_p(t.data_ptr()),
                                  ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                  ctypes.c_void_p(tb3.data_ptr()), None, None, None)
    torch.cuda.synchronize()
    assert st == 0 and torch.equal(tb3, tb1)


@pytest.mark.parametrize("scheme", ["euler", "ssprk3"])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee", "minmod", "smart"])
def test_run_adjoint_matches_oracle_reverse_sweep(lim, scheme):
    wl, th, rng = noisy_box(10, seed=4)
    steps = 8
    lam_N = rng.standard_normal(th.shape)
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    cp, fp = maps(mesh)
    uf = np.empty_like(wl.u)
    uf[fp] = wl.u
    t0 = dev(cells_in(th, cp)).requires_grad_(True)
    u = dev(uf).requires_grad_(True)
    out = FL.advect(mesh, lim, scheme, wl.dt, t0, u, steps)
    out.backward(dev(cells_in(lam_N, cp)))
    tb_o, ub_o = O.OracleMesh.from_arrays(wl.mesh).run_adjoint(lim, scheme, wl.dt, th, wl.u, steps, lam_N)
    g_t, g_u = host(t0.grad)[cp], host(u.grad)[fp]
    assert np.abs(g_t - tb_o).max() <= 1e-10 * np.abs(tb_o).max()
    assert np.abs(g_u - ub_o).max() <= 1e-10 * np.abs(ub_o).max()
    # forward value also matches the oracle
    want = O.OracleMesh.from_arrays(wl.mesh).run(lim, scheme, wl.dt, th, wl.u, steps)
    assert np.abs(host(out)[cp] - want).max() <= 1e-10 * np.abs(want).max()


def test_dot_product_against_oracle_tangent():
    """<J v, w> from the oracle's forward-mode tangent equals <v, J^T w> from the GPU reverse."""
    wl, th, rng = noisy_box(8, seed=5)
    steps = 6
    v = rng.standard_normal(th.shape)
    du = rng.standard_normal(wl.u.shape)
    w = rng.standard_normal(th.shape)
    _, jv = O.OracleMesh.from_arrays(wl.mesh).run_tangent("vanalbada", "ssprk3", wl.dt, th, wl.u,
                                                           steps, v, du)
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0)
    t0 = dev(th).requires_grad_(True)
    u = dev(wl.u).requires_grad_(True)
    FL.advect(mesh, "vanalbada", "ssprk3", wl.dt, t0, u, steps).backward(dev(w))
    lhs = float(jv @ w)
    rhs = float(v @ host(t0.grad) + du @ host(u.grad))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(jv) @ np.abs(w))


def test_finite_difference_16cubed():
    """The adjoint configuration's FD check on a 16^3 copy: van Albada, SSP-RK3, misfit loss."""
    wl, th, rng = noisy_box(16, seed=6, renumbered=False)
    steps = 40
    target = 0.5 * W.field_smooth_random(16, 3, seed=W.SEED_TARGET) + 0.5
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    cp, fp = maps(mesh)
    uf = np.empty_like(wl.u)
    uf[fp] = wl.u
    tgt = dev(cells_in(target, cp))
    t0 = dev(cells_in(th, cp)).requires_grad_(True)
    u = dev(uf).requires_grad_(True)
    loss = 0.5 * ((FL.advect(mesh, "vanalbada", "ssprk3", wl.dt, t0, u, steps) - tgt) ** 2).sum()
    loss.backward()

    def J(tt, uu):
        x = tt.clone()
        FL.rk_steps(mesh, "vanalbada", "ssprk3", wl.dt, x, uu, steps)
        return float(0.5 * ((x - tgt) ** 2).sum())

    eps = 3e-8
    umin = float(u.detach().abs().min())
    for k in range(3):
        v = dev(rng.standard_normal(th.shape))
        dv = dev(rng.standard_normal(wl.u.shape))
        # unit-size direction, shrunk further if needed so that no face changes sign
        dv *= min(1.0, 0.5 * umin / eps) / float(dv.abs().max())
        fd = (J(t0.detach() + eps * v, u.detach() + eps * dv)
              - J(t0.detach() - eps * v, u.detach() - eps * dv)) / (2 * eps)
        ad = float((t0.grad * v).sum() + (u.grad * dv).sum())
        assert ad == pytest.approx(fd, rel=1e-6), (k, ad, fd)


@pytest.mark.parametrize("every", [1, 3, 7])
def test_checkpointing_matches_full_storage(every):
    """sqrt(N) checkpoint-and-recompute gives the gradient of full stage storage, bit for bit."""
    wl, th, rng = noisy_box(12, seed=7)
    steps = 20
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    w = dev(rng.standard_normal(th.shape))
    grads = []
    for e in (every, steps):
        t0 = dev(th).requires_grad_(True)
        u = dev(wl.u).requires_grad_(True)
        FL.advect(mesh, "vanalbada", "ssprk3", wl.dt, t0, u, steps, checkpoint_every=e).backward(w)
        grads.append((t0.grad.clone(), u.grad.clone()))
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])


def test_adjoint_config_128_consistency():
    """128^3, van Albada, SSP-RK3 with sqrt(N) checkpoints: the reverse-mode directional
    derivative of the misfit matches a central difference of the GPU forward (the forward is
    itself checked against the oracle elsewhere).  60 of the configuration's 400 steps keep the
    test short; the benchmark times the full 400.  The field is a smooth seeded one: van Albada's
    face value is smooth except where both differences vanish, and plateaus or tiny noise put
    thousands of faces at or next to that point, where no finite difference is accurate."""
    n, steps = 128, 60
    wl = W.workload_box(n, renumbered=False)
    rng = np.random.default_rng(8)
    th = W.field_smooth_random(n, 3, seed=11) + 1.0
    target = 0.5 * W.field_smooth_random(n, 3, seed=W.SEED_TARGET) + 0.5
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    cp, fp = maps(mesh)
    uf = np.empty_like(wl.u)
    uf[fp] = wl.u
    tgt = dev(cells_in(target, cp))
    t0 = dev(cells_in(th, cp)).requires_grad_(True)
    u = dev(uf)
    loss = 0.5 * ((FL.advect(mesh, "vanalbada", "ssprk3", wl.dt, t0, u, steps) - tgt) ** 2).sum()
    loss.backward()
    v = dev(rng.standard_normal(th.shape))

    def run(tt):
        x = tt.clone()
        FL.rk_steps(mesh, "vanalbada", "ssprk3", wl.dt, x, u, steps)
        return x

    # dJ/d(eps) = sum (x - target) dx/d(eps): difference the final states (a difference of the
    # two losses would cancel catastrophically over 2M cells)
    eps = 1e-7
    dx = (run(t0.detach() + eps * v) - run(t0.detach() - eps * v)) / (2 * eps)
    fd = float(((run(t0.detach()) - tgt) * dx).sum())
    ad = float((t0.grad * v).sum())
    assert ad == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("scheme", ["euler", "ssprk3"])
def test_multi_step_store_equals_single_step_stores(scheme, S):
    """fl_rk_steps_store (one call per checkpoint segment, slot-rate table) stores the same stage
    inputs and leaves the same theta, bit for bit, as one fl_rk_step_store call per step."""
    wl, th, rng = noisy_box(11, seed=12)
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    cp, fp = maps(mesh)
    th = np.stack([th + 0.1 * s for s in range(S)], axis=1) if S > 1 else th
    u = mesh.faces_to_mesh(dev(wl.u))
    steps = 7
    a = mesh.cells_to_mesh(dev(th))
    b = a.clone()
    sa = FL.stage_buffer(mesh, scheme, S, steps)
    sb = torch.full_like(sa, float("nan"))
    for j in range(steps):
        FL.rk_step_store(mesh, "superbee", scheme, wl.dt, a, u, sa[j])
    FL.rk_steps_store(mesh, "superbee", scheme, wl.dt, b, u, sb, steps)
    assert torch.equal(a, b)
    assert torch.equal(sa, sb)
    c = mesh.cells_to_mesh(dev(th))
    FL.rk_steps(mesh, "superbee", scheme, wl.dt, c, u, steps)
    assert torch.equal(c, b)


@pytest.mark.parametrize("varied", [False, True], ids=["uniform", "varied_volumes"])
@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee"])
def test_lds_staged_adjoint_gives_the_same_bits(lim, S, varied):
    """With tile tables, the reverse stages stage theta and lambda of each tile and its halo in
    LDS (FL_OPT_LDS_STAGE), and the cell volumes beside them where they differ; the results must
    equal the global-gather kernel's bit for bit, for the operator adjoint and every mode of the
    reverse SSP-RK3 / Euler steps.  2197 cells: ragged last tile.  The varied case scales every
    cell volume and face area by a seeded factor in [0.7, 1.3] (the operator is defined for any
    positive V_c and a_f) and also checks the operator adjoint against the oracle."""
    wl, th, rng = noisy_box(13, seed=21)
    if varied:
        m = wl.mesh
        wl.mesh = dataclasses.replace(
            m, cell_volume=m.cell_volume * rng.uniform(0.7, 1.3, m.n_cells),
            face_area=m.face_area * rng.uniform(0.7, 1.3, m.n_faces))
    mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True)
    assert mesh.info.tile_cells == 256
    th = np.stack([th + 0.1 * s for s in range(S)], axis=1) if S > 1 else th
    t = mesh.cells_to_mesh(dev(th))
    u = mesh.faces_to_mesh(dev(wl.u))
    lam0 = mesh.cells_to_mesh(dev(rng.standard_normal(th.shape)))
    res = {}
    try:
        for lds in (1, 0):
            FL.set_option("lds_stage", lds)
            tb, ub = FL.convect_adjoint(mesh, lim, t, u, lam0)
            outs = [tb, ub]
            for scheme in ("ssprk3", "euler"):
                st = FL.stage_buffer(mesh, scheme, S, 1)
                FL.rk_step_store(mesh, lim, scheme, wl.dt, t.clone(), u, st[0])
                lam = lam0.clone()
                ubar = torch.zeros_like(u)
                FL.rk_step_adjoint(mesh, lim, scheme, wl.dt, st[0], u, lam, ubar)
                outs += [lam, ubar]
            res[lds] = outs
    finally:
        FL.set_option("lds_stage", 1)
    for x, y in zip(res[1], res[0]):
        assert torch.equal(x, y)
    if varied:
        lam_n = host(mesh.cells_from_mesh(lam0))
        tb_o, ub_o = O.OracleMesh.from_arrays(wl.mesh).rhs_vjp(lim, th, wl.u, lam_n)
        got_t = host(mesh.cells_from_mesh(res[1][0]))
        got_u = host(mesh.faces_from_mesh(res[1][1]))
        assert np.abs(got_t - tb_o).max() <= 1e-12 * np.abs(tb_o).max()
        assert np.abs(got_u - ub_o).max() <= 1e-12 * np.abs(ub_o).max()


@pytest.mark.parametrize("lds", [1, 0])
@pytest.mark.parametrize("lim", LIMS)
def test_operator_adjoint_on_flat_fields(lim, lds):
    """Flat regions put faces at d_u = d_U = 0 (every face of a constant field) and at d_u = 0
    with d_U != 0 (the edges of a plateau).  The reverse stage must use the same derivative there
    as the oracle: the derivative along d_u > 0 (psi(0)/2 where d_U = 0 too: 1/2 for central
    differencing, whose face value is linear)."""
    wl = W.workload_box(9, renumbered=True)
    rng = np.random.default_rng(31)
    m = wl.mesh
    mesh = FL.Mesh.from_arrays(m, device=0, reorder=True)
    cp, fp = maps(mesh)
    uf = np.empty_like(wl.u)
    uf[fp] = wl.u
    om = O.OracleMesh.from_arrays(m)
    try:
        FL.set_option("lds_stage", lds)
        for th in (np.full(m.n_cells, 0.25), np.where(rng.random(m.n_cells) < 0.3, 1.0, 0.0)):
            lam = rng.standard_normal(m.n_cells)
            tb, ub = FL.convect_adjoint(mesh, lim, dev(cells_in(th, cp)), dev(uf), dev(cells_in(lam, cp)))
            tb_o, ub_o = om.rhs_vjp(lim, th, wl.u, lam)
            scale = max(np.abs(tb_o).max(), 1e-300)
            assert np.abs(host(tb)[cp] - tb_o).max() <= 1e-12 * scale
            assert np.abs(host(ub)[fp] - ub_o).max() <= 1e-12 * max(np.abs(ub_o).max(), 1e-300)
    finally:
        FL.set_option("lds_stage", 1)
    mesh.close()


def _zigzag_line(n):
    """A periodic line along z whose face normals lean by +-1e-300 in x, alternately: opposite
    faces still project with weight exactly 1, but both outward normals of a cell point to the
    same side of the plane x = 0, so the forward faces come from the chain walk."""
    fc = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.int32)
    nrm = np.zeros((n, 3))
    nrm[:, 2] = 1.0
    nrm[:, 0] = np.where(np.arange(n) % 2 == 0, 1e-300, -1e-300)
    return W.MeshArrays(fc, nrm, np.ones(n), np.ones(n), n, 1)


@pytest.mark.parametrize("case", ["box", "box_varied", "zigzag"])
@pytest.mark.parametrize("S", [1, 2, 3])
@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("lds", [3, 7, 2, 1, 0],
                         ids=["fwd-lds", "fwd-lds-cellwise", "fwd-global", "planes-lds", "planes-global"])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee", "smart", "central"])
def test_multi_step_reverse_sweep_equals_per_step(lim, lds, scheme, S, case):
    """fl_rk_steps_adjoint over a segment (per-call slot rates, u cotangent accumulated in
    cell-slot order and scattered at the end) gives the same bits as one fl_rk_step_adjoint per
    step: lambda, and u_bar starting from zero.  The varied case scales volumes and areas; the
    zigzag line needs the chain walk for its forward faces.  fwd-lds shares each face's terms
    through LDS for S <= 2 (one evaluation per face and tile); fwd-lds-cellwise does not."""
    rng = np.random.default_rng(zlib.crc32(f"{lim}-{scheme}-{S}-{case}".encode()))
    if case == "zigzag":
        m = _zigzag_line(40)
        u0 = np.where(rng.random(m.n_faces) < 0.5, 1.0, -0.7)
        dt = 0.2
    else:
        wl, _, _ = noisy_box(11, seed=S)
        m, u0, dt = wl.mesh, wl.u, wl.dt
        if case == "box_varied":
            m = dataclasses.replace(
                m, cell_volume=m.cell_volume * rng.uniform(0.7, 1.3, m.n_cells),
                face_area=m.face_area * rng.uniform(0.7, 1.3, m.n_faces))
    th0 = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
    th0[::5] = np.round(th0[::5])
    steps = 5
    mesh = FL.Mesh.from_arrays(m, device=0, reorder=(case != "zigzag"))
    assert mesh.info.aligned == 1
    u = mesh.faces_to_mesh(dev(u0))
    t = mesh.cells_to_mesh(dev(th0))
    stages = FL.stage_buffer(mesh, scheme, S, steps)
    try:
        FL.set_option("lds_stage", lds & 1)
        FL.set_option("fwd_rates", (lds >> 1) & 1)
        FL.set_option("face_share", 0 if lds & 4 else 1)
        FL.rk_steps_store(mesh, lim, scheme, dt, t.clone(), u, stages, steps)
        lam0 = mesh.cells_to_mesh(dev(rng.standard_normal(th0.shape)))
        a = lam0.clone()
        ua = torch.zeros_like(u)
        for j in reversed(range(steps)):
            FL.rk_step_adjoint(mesh, lim, scheme, dt, stages[j], u, a, ua)
        b = lam0.clone()
        acc = FL.uacc_buffer(mesh)
        assert acc is not None and acc.numel() == mesh.info.pairs * mesh.n_cells
        # two calls, as a checkpointed backward makes them: the later steps first
        rates = FL.adjoint_rates(mesh, u)
        FL.rk_steps_adjoint(mesh, lim, scheme, dt, stages[2:], rates, b, steps - 2, acc)
        FL.rk_steps_adjoint(mesh, lim, scheme, dt, stages, rates, b, 2, acc)
        ub = FL.uacc_scatter(mesh, acc, torch.zeros_like(u))
        torch.cuda.synchronize()
        c = lam0.clone()
        FL.rk_steps_adjoint(mesh, lim, scheme, dt, stages, rates, c, steps, None)
        torch.cuda.synchronize()
    finally:
        FL.set_option("lds_stage", 1)
        FL.set_option("fwd_rates", 1)
        FL.set_option("face_share", 1)

    def diff(x, y):
        d = (x - y).abs()
        return f"{int((d > 0).sum())} of {d.numel()} differ, max {float(d.max()):.3e}"

    assert torch.equal(a, b), diff(a, b)
    assert torch.equal(ua, ub), diff(ua, ub)
    # and the lambda of a call without the u cotangent
    assert torch.equal(a, c), diff(a, c)
    mesh.close()


# ---------------------------------------------------------------------------------------------
# General cells (triangles; sheared hexahedra): the face-term kernel and the cell gather through
# the transposed projection lists.  The oracle's reverse sweep walks every face of C with the
# projection weights (zero weight for a face that does not project), so it shares no structure
# with the side lists the library builds.
# ---------------------------------------------------------------------------------------------

GENERAL = [
    ("tri8r", lambda: W.renumber(W.periodic_triangles(8), seed=21)),
    ("skew6r", lambda: W.renumber(W.periodic_skewed_box(6), seed=22)),
]


def _general_case(name, make, S, seed):
    m = make()
    rng = np.random.default_rng(seed)
    th = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
    th[::4] = np.round(th[::4])  # plateaus: d_u == 0 and infinite ratios
    if name.startswith("tri"):
        u = m.face_velocity_from_natural(W.velocity_stream_triangles(8, seed=seed))
    else:
        u = W.velocity_uniform(m, (0.6, -0.3, 0.8), 1.0) + 0.3 * rng.standard_normal(m.n_faces)
    u[::9] = 0.0
    return m, th, u, rng


@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("name,make", GENERAL, ids=[c[0] for c in GENERAL])
def test_general_cells_operator_adjoint_matches_oracle(name, make, reorder, S):
    m, th, u, rng = _general_case(name, make, S, seed=30 + S)
    lam = rng.standard_normal(th.shape)
    mesh = FL.Mesh.from_arrays(m, device=0, reorder=reorder)
    assert mesh.info.general == 1 and mesh.path == "face"
    cp, fp = maps(mesh)
    uf = np.empty_like(u)
    uf[fp] = u
    om = O.OracleMesh.from_arrays(m)
    for lim in LIMS:
        tb, ub = FL.convect_adjoint(mesh, lim, dev(cells_in(th, cp)), dev(uf),
                                    dev(cells_in(lam, cp)))
        tb_o, ub_o = om.rhs_vjp(lim, th, u, lam)
        got_t, got_u = host(tb)[cp], host(ub)[fp]
        assert np.abs(got_t - tb_o).max() <= 1e-12 * np.abs(tb_o).max(), lim
        assert np.abs(got_u - ub_o).max() <= 1e-12 * np.abs(ub_o).max(), lim
    mesh.close()


@pytest.mark.parametrize("name,make", GENERAL, ids=[c[0] for c in GENERAL])
def test_general_cells_operator_adjoint_accumulates_and_repeats(name, make):
    """theta_bar and u_bar accumulate; two calls give the same bits (no atomics)."""
    m, th, u, rng = _general_case(name, make, 2, seed=40)
    mesh = FL.Mesh.from_arrays(m, device=0, reorder=True)
    t = mesh.cells_to_mesh(dev(th))
    ud = mesh.faces_to_mesh(dev(u))
    lam = mesh.cells_to_mesh(dev(rng.standard_normal(th.shape)))
    tb1, ub1 = FL.convect_adjoint(mesh, "superbee", t, ud, lam)
    tb2, ub2 = FL.convect_adjoint(mesh, "superbee", t, ud, lam)
    assert torch.equal(tb1, tb2) and torch.equal(ub1, ub2)
    FL.convect_adjoint(mesh, "superbee", t, ud, lam, tb2, ub2)
    assert torch.equal(tb2, 2 * tb1) and torch.equal(ub2, 2 * ub1)
    mesh.close()


@pytest.mark.parametrize("scheme", ["euler", "ssprk3"])
@pytest.mark.parametrize("lim", ["vanalbada", "superbee", "minmod", "smart"])
@pytest.mark.parametrize("name,make", GENERAL, ids=[c[0] for c in GENERAL])
def test_general_cells_run_adjoint_matches_oracle(name, make, lim, scheme):
    """advect's backward on general cells (one reverse step per stored step, checkpointed)
    against the oracle's stored reverse sweep."""
    m, th, u, rng = _general_case(name, make, 1, seed=50)
    u[::9] = 0.1  # the run needs no stagnant faces; keep them small instead
    dt = W.cfl_dt(m, u, 0.3)
    steps = 7
    lam_N = rng.standard_normal(th.shape)
    mesh = FL.Mesh.from_arrays(m, device=0, reorder=True)
    cp, fp = maps(mesh)
    uf = np.empty_like(u)
    uf[fp] = u
    t0 = dev(cells_in(th, cp)).requires_grad_(True)
    ud = dev(uf).requires_grad_(True)
    out = FL.advect(mesh, lim, scheme, dt, t0, ud, steps, checkpoint_every=3)
    out.backward(dev(cells_in(lam_N, cp)))
    om = O.OracleMesh.from_arrays(m)
    tb_o, ub_o = om.run_adjoint(lim, scheme, dt, th, u, steps, lam_N)
    g_t, g_u = host(t0.grad)[cp], host(ud.grad)[fp]
    assert np.abs(g_t - tb_o).max() <= 1e-10 * np.abs(tb_o).max()
    assert np.abs(g_u - ub_o).max() <= 1e-10 * np.abs(ub_o).max()
    want = om.run(lim, scheme, dt, th, u, steps)
    assert np.abs(host(out)[cp] - want).max() <= 1e-10 * np.abs(want).max()
    mesh.close()


def test_general_cells_dot_product_against_oracle_tangent():
    """<J v, w> from the oracle's tangent on the triangles equals <v, J^T w> from the GPU."""
    name, make = GENERAL[0]
    m, th, u, rng = _general_case(name, make, 1, seed=60)
    u[::9] = 0.1
    dt = W.cfl_dt(m, u, 0.3)
    steps = 5
    v = rng.standard_normal(th.shape)
    du = rng.standard_normal(u.shape)
    w = rng.standard_normal(th.shape)
    _, jv = O.OracleMesh.from_arrays(m).run_tangent("vanalbada", "ssprk3", dt, th, u, steps, v, du)
    mesh = FL.Mesh.from_arrays(m, device=0)
    t0 = dev(th).requires_grad_(True)
    ud = dev(u).requires_grad_(True)
    FL.advect(mesh, "vanalbada", "ssprk3", dt, t0, ud, steps).backward(dev(w))
    lhs = float(jv @ w)
    rhs = float(v @ host(t0.grad) + du @ host(ud.grad))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(jv) @ np.abs(w))
    mesh.close()
