"""Batched problems on the GPU: each problem of a batch equals its single-problem run bit for
bit (same arithmetic in the same order), on every replay of the recorded graph, for autotuned
and fixed tile sizes, and matches the CPU oracle."""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2110_03044_amd import _lib, fluxlim as FL, workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
LIMS = ["upwind", "minmod", "vanleer", "vanalbada", "superbee", "smart", "central"]


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def make_problems(count=14, seed=5, dims=(1, 2, 3)):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(count):
        d = int(dims[i % len(dims)])
        n = int(rng.integers(5, 15)) if d == 3 else int(rng.integers(7, 40))
        S = int(rng.integers(1, 9))
        lim = LIMS[i % len(LIMS)]
        nat = W.periodic_box(n, d)
        m = W.renumber(nat, seed=100 + i) if i % 2 else nat
        if d == 3:
            u = m.face_velocity_from_natural(W.velocity_curl(n, seed=i))
        else:
            u = W.velocity_uniform(m, (0.8, -0.6, 0.0))
        th = rng.standard_normal((m.n_cells, S)) if S > 1 else rng.standard_normal(m.n_cells)
        dt = W.cfl_dt(m, u, float(rng.uniform(0.2, 0.45)))
        probs.append(dict(mesh=m, u=u, th=th, dt=dt, lim=lim))
    return probs


def to_dev(p, reorder=True):
    mesh = FL.Mesh.from_arrays(p["mesh"], device=0, reorder=reorder)
    th = mesh.cells_to_mesh(torch.from_numpy(p["th"]).to(DEV))
    u = mesh.faces_to_mesh(torch.from_numpy(p["u"]).to(DEV))
    return mesh, th, u


@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("tile", [0, 64, 256, 1024])
def test_batch_equals_single_runs_on_every_replay(scheme, tile):
    probs = make_problems()
    dev_probs = [to_dev(p) for p in probs]
    batch_th = [th.clone() for _, th, _ in dev_probs]
    single_th = [th.clone() for _, th, _ in dev_probs]
    b = FL.Batch([(m, p["lim"], bt, u, p["dt"]) for (m, _, u), bt, p in zip(dev_probs, batch_th, probs)],
                 scheme=scheme, tile_cells=tile)
    for replay in range(3):
        b.step(2)
        torch.cuda.synchronize()
        for (m, _, u), st, p in zip(dev_probs, single_th, probs):  # eager work between replays
            FL.rk_steps(m, p["lim"], scheme, p["dt"], st, u, 2)
        torch.cuda.synchronize()
        for i, (bt, st) in enumerate(zip(batch_th, single_th)):
            assert torch.equal(bt, st), (replay, i, probs[i]["lim"])
    assert b.tile_cells > 0 and (tile == 0 or b.tile_cells == tile)
    assert b.lds_staged == (tile == 256 or (tile == 0 and b.tile_cells == 256 and b.lds_staged))
    b.close()


@pytest.mark.parametrize("S", [1, 4, 8])
def test_lds_staged_batch_and_per_problem_launches(S):
    """Tiles of 256 cells run staged in LDS (two scalars at a time, so any S fits); the batch,
    its per-problem launches and the gather kernel give the same bits."""
    probs = make_problems(count=6, seed=31)
    for p in probs:
        rng = np.random.default_rng(p["mesh"].n_cells)
        p["th"] = rng.standard_normal((p["mesh"].n_cells, S)) if S > 1 else \
            rng.standard_normal(p["mesh"].n_cells)
    dev_probs = [to_dev(p) for p in probs]
    outs = {}
    try:
        for lds in (1, 0):
            FL.set_option("lds_stage", lds)
            for kind in ("batch", "unbatched"):
                ths = [th.clone() for _, th, _ in dev_probs]
                b = FL.Batch([(m, p["lim"], t, u, p["dt"])
                              for (m, _, u), t, p in zip(dev_probs, ths, probs)], tile_cells=256)
                assert b.lds_staged == bool(lds)
                (b.step if kind == "batch" else b.step_unbatched)(3)
                torch.cuda.synchronize()
                outs[lds, kind] = ths
                b.close()
    finally:
        FL.set_option("lds_stage", 1)
    ref = outs[0, "batch"]
    for key, ths in outs.items():
        for i, (x, y) in enumerate(zip(ths, ref)):
            assert torch.equal(x, y), (key, i)


def test_batch_matches_oracle_and_unbatched():
    probs = make_problems(count=8, seed=9)
    dev_probs = [to_dev(p) for p in probs]
    a = [th.clone() for _, th, _ in dev_probs]
    c = [th.clone() for _, th, _ in dev_probs]
    b1 = FL.Batch([(m, p["lim"], t, u, p["dt"]) for (m, _, u), t, p in zip(dev_probs, a, probs)])
    b2 = FL.Batch([(m, p["lim"], t, u, p["dt"]) for (m, _, u), t, p in zip(dev_probs, c, probs)],
                  tile_cells=256)
    b1.step(4)
    b2.step_unbatched(4)
    torch.cuda.synchronize()
    for i, ((m, _, _), p) in enumerate(zip(dev_probs, probs)):
        assert torch.equal(a[i], c[i]), i
        want = O.OracleMesh.from_arrays(p["mesh"]).run(p["lim"], "ssprk3", p["dt"], p["th"], p["u"], 4)
        got = m.cells_from_mesh(a[i]).cpu().numpy()
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max(), (i, p["lim"])


def test_batch_shared_mesh_and_rejections():
    p = make_problems(count=1, seed=2, dims=(3,))[0]
    mesh, th, u = to_dev(p)
    t1, t2 = th.clone(), (2.0 * th).clone()
    b = FL.Batch([(mesh, "superbee", t1, u, p["dt"]), (mesh, "vanleer", t2, u, 0.5 * p["dt"])])
    b.step(3)
    r1, r2 = th.clone(), (2.0 * th).clone()
    FL.rk_steps(mesh, "superbee", "ssprk3", p["dt"], r1, u, 3)
    FL.rk_steps(mesh, "vanleer", "ssprk3", 0.5 * p["dt"], r2, u, 3)
    torch.cuda.synchronize()
    assert torch.equal(t1, r1) and torch.equal(t2, r2)
    with pytest.raises(_lib.FluxLimError):
        FL.Batch([(mesh, "minmod", t1, u, p["dt"])], tile_cells=100)


def test_full_size_batch_of_512_problems():
    """The benchmark's batch in the launch configuration it times (512 periodic boxes, sides
    12-96, 1-8 scalars, per-problem limiter and CFL, SSP-RK3; autotuned tile, LDS staging, the
    default XCD order): two batched steps equal two steps of per-problem launches bit for bit on
    every problem, and the three smallest problems match the oracle."""
    recipe = W.batch_recipe(count=512)
    smallest = sorted(range(len(recipe)), key=lambda i: recipe[i].n)[:3]
    meshes, nat = {}, {}
    batched, single, start = [], [], {}
    try:
        for p in recipe:
            if p.n not in meshes:
                m = W.box_shared_cache(p.n)
                meshes[p.n] = FL.Mesh.from_arrays(m, device=0, reorder=True)
                nat[p.n] = (m, W.velocity_curl(p.n, seed=p.n))
            mesh = meshes[p.n]
            m, u = nat[p.n]
            th0 = W.batch_fields(p)
            t = mesh.cells_to_mesh(torch.from_numpy(th0).to(DEV))
            ud = mesh.faces_to_mesh(torch.from_numpy(u).to(DEV))
            dt = W.cfl_dt(m, u, p.cfl)
            batched.append((mesh, p.limiter, t, ud, dt))
            single.append((mesh, p.limiter, t.clone(), ud, dt))
            if len(batched) - 1 in smallest:
                start[len(batched) - 1] = th0
    finally:
        W._BOX_CACHE.clear()
    b1 = FL.Batch(batched)
    b2 = FL.Batch(single)
    try:
        b1.step(2)
        b2.step_unbatched(2)
        torch.cuda.synchronize()
        assert b1.lds_staged
    finally:
        b1.close()
        b2.close()
    for x, y in zip(batched, single):
        assert torch.equal(x[2], y[2])
    for i in smallest:
        p = recipe[i]
        m, u = nat[p.n]
        mesh, lim, t, _, dt = batched[i]
        got = mesh.cells_from_mesh(t).cpu().numpy()
        want = O.OracleMesh.from_arrays(m).run(LIMS[lim], "ssprk3", dt, start[i], u, 2)
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_tuning_at_creation_and_on_disk_cache(tmp_path, monkeypatch):
    """With tile_cells = 0 the tile is chosen when the batch is created (fl_batch_step only
    replays the graph); the choice is written to the tuning cache, a second batch of the same
    shape reads it instead of timing, and both give the same bits.  "0" disables the cache."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("FL_TUNE_CACHE", str(path))
    probs = make_problems(count=6, seed=9)
    runs = []
    for k in range(2):
        dev_probs = [to_dev(p) for p in probs]
        ths = [th.clone() for _, th, _ in dev_probs]
        b = FL.Batch([(m, p["lim"], t, u, p["dt"]) for (m, _, u), t, p in zip(dev_probs, ths, probs)])
        assert b.tile_cells > 0  # chosen before any step
        assert b.tuned_from_cache == (k == 1)
        lines = path.read_text().split("\n")
        assert len([x for x in lines if x.strip()]) == 1
        b.step(3)
        torch.cuda.synchronize()
        runs.append((b.tile_cells, b.lds_staged, [t.clone() for t in ths]))
        b.close()
    assert runs[0][:2] == runs[1][:2]
    for x, y in zip(runs[0][2], runs[1][2]):
        assert torch.equal(x, y)
    monkeypatch.setenv("FL_TUNE_CACHE", "0")
    dev_probs = [to_dev(p) for p in probs]
    b = FL.Batch([(m, p["lim"], th, u, p["dt"]) for (m, th, u), p in zip(dev_probs, probs)])
    assert not b.tuned_from_cache
    b.close()


def rows_to_mesh(x, perm):
    out = np.empty_like(x)
    out[perm] = x
    return out


def face_path_problems():
    """Problems on the face path: triangles and a sheared box (general cells), an open box with
    inflow values, a stretched box with face distances, and a box forced onto the face path."""
    out = []
    tri = W.renumber(W.periodic_triangles(10), seed=41)
    rng = np.random.default_rng(42)
    u = tri.face_velocity_from_natural(W.velocity_stream_triangles(10, seed=3))
    out.append(dict(mesh=tri, u=u, th=rng.standard_normal((tri.n_cells, 2)), lim="superbee",
                    dt=W.cfl_dt(tri, u, 0.3)))
    sk = W.renumber(W.periodic_skewed_box(6), seed=43)
    u = W.velocity_uniform(sk, (0.6, -0.3, 0.8), 1.0)
    out.append(dict(mesh=sk, u=u, th=rng.standard_normal(sk.n_cells), lim="vanleer",
                    dt=W.cfl_dt(sk, u, 0.3)))
    wl = W.workload_open_box(8, renumbered=True, S=3)
    out.append(dict(mesh=wl.mesh, u=wl.u, th=wl.theta0, lim="vanalbada", dt=wl.dt,
                    inflow=wl.inflow))
    nat = W.stretched_box(9, 3, amp=0.5)
    st = W.renumber(nat, seed=44)
    u = st.face_velocity_from_natural(W.velocity_open_box(nat))
    out.append(dict(mesh=st, u=u, th=st.cell_field_from_natural(W.field_blob_step(9)),
                    lim="smart", dt=W.cfl_dt(st, u, 0.4)))
    box = make_problems(count=1, seed=45, dims=(3,))[0]
    box.update(lim="minmod", face_path=True)
    out.append(box)
    return out


def to_dev_face(p):
    mesh = FL.Mesh.from_arrays(p["mesh"], device=0, reorder=True,
                               **({"face_path": True} if p.get("face_path") else {}))
    cp, fp = mesh.permutation()
    assert mesh.path == "face"
    if p.get("inflow") is not None:
        mesh.set_inflow(torch.from_numpy(rows_to_mesh(p["inflow"], fp)).to(DEV))
    th = torch.from_numpy(rows_to_mesh(p["th"], cp)).to(DEV)
    u = torch.from_numpy(rows_to_mesh(p["u"], fp)).to(DEV)
    return mesh, th, u


@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
@pytest.mark.parametrize("with_fused", [True, False])
def test_batch_with_face_path_problems(scheme, with_fused):
    """Face-path problems (general cells, boundary faces with inflow, face distances) join a
    batch: two more launches per stage for all of them.  Each equals its single-problem run bit
    for bit on every replay, the per-problem launches give the same bits, and the oracle agrees."""
    fprobs = face_path_problems()
    dev_probs = [to_dev_face(p) for p in fprobs]
    probs = list(fprobs)
    if with_fused:
        extra = make_problems(count=3, seed=46)
        probs += extra
        dev_probs += [to_dev(p) for p in extra]
    batch_th = [th.clone() for _, th, _ in dev_probs]
    single_th = [th.clone() for _, th, _ in dev_probs]
    unb_th = [th.clone() for _, th, _ in dev_probs]
    items = [(m, p["lim"], bt, u, p["dt"]) for (m, _, u), bt, p in zip(dev_probs, batch_th, probs)]
    b = FL.Batch(items, scheme=scheme)
    bu = FL.Batch([(m, p["lim"], t, u, p["dt"]) for (m, _, u), t, p in zip(dev_probs, unb_th, probs)],
                  scheme=scheme, tile_cells=256)
    steps = 0
    for replay in range(3):
        b.step(2)
        bu.step_unbatched(2)
        steps += 2
        torch.cuda.synchronize()
        for (m, _, u), st, p in zip(dev_probs, single_th, probs):
            FL.rk_steps(m, p["lim"], scheme, p["dt"], st, u, 2)
        torch.cuda.synchronize()
        for i, (bt, st, ut) in enumerate(zip(batch_th, single_th, unb_th)):
            assert torch.equal(bt, st), (replay, i, probs[i]["lim"])
            assert torch.equal(ut, st), (replay, i, probs[i]["lim"])
    for i, p in enumerate(fprobs):
        m = dev_probs[i][0]
        om = O.OracleMesh.from_arrays(p["mesh"])
        if p["mesh"].face_dist is not None:
            om.set_distances(p["mesh"].face_dist)
        om.set_inflow(p.get("inflow"))
        want = om.run(p["lim"], scheme, p["dt"], p["th"], p["u"], steps)
        cp, _ = m.permutation()
        got = batch_th[i].cpu().numpy()[cp]
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max(), (i, p["lim"])
    b.close()
    bu.close()
