"""Host-side checks of the HIP library (no GPU): exported symbols, mesh validation and the
tables the kernels read, compared bit for bit with the oracle's face selection."""

import ctypes
import dataclasses
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_03044_amd import _lib, fluxlim as FL, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\**(fl_[a-z0-9_]+)\s*\(",
                                text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 25
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing
    assert set(names) == set(_lib.SIGNATURES)


def test_status_strings():
    L = _lib.lib()
    assert L.fl_status_str(0) == b"FL_OK"
    assert L.fl_status_str(-3) == b"FL_E_UNSUPPORTED"
    assert L.fl_status_str(-6) == b"FL_E_NONFINITE"
    assert L.fl_status_str(-7) == b"FL_E_NODEVICE"
    for code, name in _lib.STATUS.items():
        assert L.fl_status_str(code).decode() == name


def test_finite_check_option():
    L = _lib.lib()
    assert L.fl_set_option(4, 1) == 0  # FL_OPT_CHECK_FINITE on
    assert L.fl_set_option(4, 0) == 0
    assert L.fl_set_option(4, 2) == -1


def test_batch_rejects_host_only_meshes_before_allocating():
    """A host-only mesh has no device tables: fl_batch_create must refuse it (FL_E_NODEVICE)
    before any allocation or launch, whatever device the batch names."""
    m = W.periodic_box(6, 3)
    mesh = FL.Mesh.from_arrays(m, device=-1)
    L = _lib.lib()
    mh = (ctypes.c_void_p * 1)(mesh.handle.value)
    lim = (ctypes.c_int * 1)(2)
    ns = (ctypes.c_int * 1)(1)
    dts = (ctypes.c_double * 1)(1e-3)
    th = (ctypes.c_void_p * 1)(256)
    uu = (ctypes.c_void_p * 1)(512)
    for device in (-1, 0):
        out = ctypes.c_void_p(1)
        st = L.fl_batch_create(1, mh, lim, ns, dts, 3, th, uu, 0, device, ctypes.byref(out))
        assert st == -7, (device, st)
        assert out.value is None
    mesh.close()


def _rotated_box(n, angle, seed):
    """A periodic box whose face normals are each turned by `angle` radians about a random axis
    and renormalised: geometrically a hexahedral mesh, but the projection weights are no longer
    exactly 0 and 1."""
    m = W.periodic_box(n, 3)
    rng = np.random.default_rng(seed)
    nrm = m.face_normal.copy()
    ax = rng.standard_normal(nrm.shape)
    ax -= (ax * nrm).sum(1, keepdims=True) * nrm  # axis orthogonal to the normal
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    nrm = nrm * np.cos(angle) + ax * np.sin(angle)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return dataclasses.replace(m, face_normal=nrm)


def test_nearly_orthogonal_normals_keep_every_weight():
    """No tolerance in the far-upwind selection: normals off the axes by 1e-10 rad give weights
    like 1e-10 on the side faces, which the upstream difference sums (the oracle does), so the
    mesh is built as general cells with the oracle's exact weights, not as hexahedra."""
    m = _rotated_box(5, 1e-10, seed=1)
    mesh = FL.Mesh.from_arrays(m, device=-1)
    assert mesh.info.general == 1 and mesh.path == "face" and mesh.info.pairs == 0
    far, _, _ = mesh.export_tables()
    assert (far == -1).all()
    om = O.OracleMesh.from_arrays(m)
    f = 7
    faces, w = om.side_weights(f, side_nbr=False)
    nz = w[w != 0.0]
    assert len(nz) >= 3 and np.abs(nz).min() < 1e-9 and np.abs(nz).max() == pytest.approx(1.0, abs=1e-15)
    mesh.close()
    # the exact box stays on the fused path
    exact = FL.Mesh.from_arrays(W.periodic_box(5, 3), device=-1)
    assert exact.info.general == 0 and exact.path == "fused"
    exact.close()


def _meshes():
    out = []
    for n, d in [(7, 1), (6, 2), (5, 3), (7, 3)]:
        nat = W.periodic_box(n, d)
        out.append((f"{d}d{n}", nat))
        out.append((f"{d}d{n}r", W.renumber(nat, seed=3 * n + d)))
    return out


@pytest.mark.parametrize("reorder", [False, True])
@pytest.mark.parametrize("name,m", _meshes(), ids=lambda x: x if isinstance(x, str) else "")
def test_tables_match_oracle_selection(name, m, reorder):
    mesh = FL.Mesh.from_arrays(m, device=-1, reorder=reorder)
    assert mesh.path == "fused" and mesh.info.pairs == max(m.dim, 1)
    far, ptr, idx = mesh.export_tables()
    cp, fp = mesh.permutation()
    assert np.array_equal(np.sort(cp), np.arange(m.n_cells))
    assert np.array_equal(np.sort(fp), np.arange(m.n_faces))
    if not reorder:
        assert np.array_equal(cp, np.arange(m.n_cells)) and np.array_equal(fp, np.arange(m.n_faces))
    om = O.OracleMesh.from_arrays(m)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(m.n_faces)
    u[::11] = 0.0
    cdu = om.select(u)  # user numbering
    # library tables are in mesh numbering: map the oracle's cells through cell_perm
    pos = u > 0
    mf = fp  # mesh face of each user face
    U_lib = np.where(pos, far[mf, 0], far[mf, 1])
    assert np.array_equal(U_lib, cp[cdu[:, 2]])
    # cell -> face lists: same sets, ascending in mesh order, orientation in the sign
    fc_mesh = np.empty_like(m.face_cells)
    fc_mesh[fp] = cp[m.face_cells]
    for c in range(0, m.n_cells, max(1, m.n_cells // 50)):
        ent = idx[ptr[c]:ptr[c + 1]]
        faces = np.where(ent >= 0, ent, ~ent)
        assert np.all(np.diff(faces) > 0)
        for e, f in zip(ent, faces):
            assert (fc_mesh[f, 1] == c) if e >= 0 else (fc_mesh[f, 0] == c)
        assert len(faces) == 2 * max(m.dim, 1)


def test_reorder_improves_index_locality():
    m = W.renumber(W.periodic_box(16, 3), seed=1)
    rnd = FL.Mesh.from_arrays(m, device=-1)
    ro = FL.Mesh.from_arrays(m, device=-1, reorder=True)

    def spread(mesh):
        far, ptr, idx = mesh.export_tables()
        faces = np.where(idx >= 0, idx, ~idx).reshape(-1, 6)
        return np.abs(faces - faces.mean(axis=1, keepdims=True)).mean()

    assert spread(ro) < 0.2 * spread(rnd)


def _err(fc, nrm, n_cells):
    L = _lib.lib()
    fc = np.ascontiguousarray(fc, dtype=np.int32)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    st = L.fl_mesh_validate(n_cells, fc.shape[0], fc.ctypes.data_as(ctypes.c_void_p),
                            nrm.ctypes.data_as(ctypes.c_void_p))
    return st, L.fl_last_error().decode()


def test_validate_accepts_periodic_hex():
    m = W.renumber(W.periodic_box(4, 3), seed=2)
    assert _err(m.face_cells, m.face_normal, m.n_cells)[0] == 0


def test_validate_rejections():
    m = W.periodic_box(4, 3)
    fc, nrm, C = m.face_cells.copy(), m.face_normal.copy(), m.n_cells
    bad = fc.copy(); bad[5, 1] = -1
    assert _err(bad, nrm, C)[0] == 0  # a boundary face (one cell)
    bad = fc.copy(); bad[5] = [-1, bad[5, 0]]
    st, msg = _err(bad, nrm, C)
    assert st == -2 and "own" in msg  # a boundary face lists its cell first
    bad = fc.copy(); bad[5, 1] = C
    assert _err(bad, nrm, C)[0] == -2  # out of range
    bad = fc.copy(); bad[5, 1] = bad[5, 0]
    assert _err(bad, nrm, C)[0] == -2  # own == nbr
    badn = nrm.copy(); badn[3] *= 1.1
    assert _err(fc, badn, C)[0] == -1  # not unit
    badn = nrm.copy(); badn[3, 0] = np.nan
    assert _err(fc, badn, C)[0] == -1
    # periodic side of 2 cells: two faces join the same pair of cells
    m2 = W.periodic_box(2, 3)
    st, msg = _err(m2.face_cells, m2.face_normal, m2.n_cells)
    assert st == -2 and "both join" in msg
    # a tilted normal makes the upstream difference project on several faces: a general mesh,
    # accepted (face/cell path with per-side weight lists)
    badn = nrm.copy(); badn[0] = [np.sqrt(0.5), np.sqrt(0.5), 0.0]
    st, msg = _err(fc, badn, C)
    assert st == 0
    mesh = FL.Mesh(fc, badn, n_cells=C, device=-1)
    assert mesh.info.general == 1 and mesh.info.max_side >= 2 and mesh.path == "face"
    mesh.close()


@pytest.mark.parametrize("reorder", [False, True, "bfs"])
def test_boundary_mesh_tables(reorder):
    """An open box builds on the face path with the general tables: the boundary faces are in
    their one cell's face list (as ~f: the cell is own), the permutation keeps each boundary
    face's cell, and the exterior side of a boundary face has no projected faces."""
    m = W.renumber(W.open_box(6, 3, (0, 1)), seed=3)
    nb = int((m.face_cells[:, 1] < 0).sum())
    assert nb == 2 * 2 * 36
    mesh = FL.Mesh.from_arrays(m, device=-1, reorder=reorder)
    assert mesh.path == "face" and mesh.info.general == 1 and mesh.n_boundary == nb
    assert mesh.info.pairs == 0 and mesh.info.max_halo == -1
    far, ptr, idx = mesh.export_tables()
    assert np.all(far == -1)
    assert ptr[-1] == 2 * m.n_faces - nb
    cp, fp = mesh.permutation()
    assert sorted(cp) == list(range(m.n_cells)) and sorted(fp) == list(range(m.n_faces))
    bmesh = fp[m.face_cells[:, 1] < 0]  # the boundary faces in mesh numbering
    owner = cp[m.face_cells[m.face_cells[:, 1] < 0, 0]]
    cell_of = np.repeat(np.arange(m.n_cells), np.diff(ptr))
    for f, c in zip(bmesh, owner):
        hits = np.nonzero((idx == ~f) | (idx == f))[0]
        assert len(hits) == 1 and idx[hits[0]] == ~f and cell_of[hits[0]] == c
    # every cell keeps its six faces
    assert np.all(np.diff(ptr) == 6)
    # the oracle's projected faces: none on the exterior side of a boundary face
    om = O.OracleMesh.from_arrays(m)
    f0 = int(np.nonzero(m.face_cells[:, 1] < 0)[0][0])
    assert om.side_weights(f0, True)[0].size == 0
    assert om.side_weights(f0, False)[0].size == 6
    L = _lib.lib()
    assert L.fl_mesh_set_inflow(mesh.handle, ctypes.c_void_p(8), 1) == -7  # host-only
    assert L.fl_mesh_set_inflow(mesh.handle, None, 0) == 0
    mesh.close()


def test_distance_weighted_tables():
    """Unequal face distances scale each side weight by d_f / d_j (the general path); equal
    distances build the unweighted tables (the fused path on a hex box); bad distances are
    refused."""
    m = W.stretched_box(6, 3, amp=0.5)
    mesh = FL.Mesh.from_arrays(m, device=-1, reorder=True)
    assert mesh.info.dist_weighted == 1 and mesh.path == "face" and mesh.info.general == 1
    mesh.close()
    same = FL.Mesh.from_arrays(W.periodic_box(6, 3), device=-1,
                               face_dist=np.full(3 * 216, 1.0 / 6))
    assert same.info.dist_weighted == 0 and same.path == "fused"
    same.close()
    for bad in (0.0, -1.0, np.nan, np.inf):
        d = m.face_dist.copy()
        d[4] = bad
        with pytest.raises(_lib.FluxLimError) as e:
            FL.Mesh.from_arrays(m, device=-1, face_dist=d)
        assert e.value.status == -1
    weighted = FL.Mesh.from_arrays(m, device=-1)
    with pytest.raises(_lib.FluxLimError) as e:
        FL.Algebraic(weighted)
    assert e.value.status == -3
    weighted.close()


def test_compact_forward_tables_on_lattice_meshes():
    """A Morton-ordered periodic box gets the compact forward-stage tables: every tile is an
    8x8x4 brick, so 128 leading halo entries carry a rate (the neighbours across backward slots)
    and 384 a next index (also the neighbours across forward slots and the far cells beyond the
    backward ones)."""
    m = W.renumber(W.periodic_box(16, 3), seed=6)
    mesh = FL.Mesh.from_arrays(m, device=-1, reorder=True)
    i = mesh.info
    assert i.compact == 1 and i.aligned == 1 and i.max_halo == 512
    assert i.max_rated == 128 and i.max_nexts == 384
    assert i.halo_nexts == 384 * (m.n_cells // 256)
    mesh.close()
    line = FL.Mesh.from_arrays(W.periodic_box(40, 1), device=-1, reorder=True)
    assert line.info.compact == 1
    line.close()


def test_algebraic_chain_refuses_boundary_meshes():
    mesh = FL.Mesh.from_arrays(W.open_box(5, 3, (2,)), device=-1)
    with pytest.raises(_lib.FluxLimError) as e:
        FL.Algebraic(mesh)
    assert e.value.status == -3
    mesh.close()


def test_create_rejects_bad_arguments_and_host_only_compute():
    m = W.periodic_box(4, 3)
    with pytest.raises(_lib.FluxLimError) as e:
        FL.Mesh(m.face_cells[:, ::-1].copy() * 0, m.face_normal, device=-1, n_cells=m.n_cells)
    assert e.value.status == -2
    mesh = FL.Mesh.from_arrays(m, device=-1)
    L = _lib.lib()
    st = L.fl_convect_apply(mesh.handle, 2, 1, ctypes.c_void_p(8), ctypes.c_void_p(8),
                            ctypes.c_void_p(16), None, None)
    assert st == -7  # FL_E_NODEVICE
    st = L.fl_rk_steps(mesh.handle, 9, 3, 0.1, 1, 1, ctypes.c_void_p(8), ctypes.c_void_p(8),
                       ctypes.c_void_p(256), None)
    assert st in (-1, -7)
    def a256(x):
        return (x + 255) // 256 * 256

    # two stage buffers + the 16-byte slot records (6 slots per hex cell) of the fused path
    assert L.fl_rk_workspace_bytes(mesh.handle, 3, 1) == (2 * a256(m.n_cells * 8)
                                                          + a256(6 * m.n_cells * 16))
    assert L.fl_rk_workspace_bytes(mesh.handle, 2, 1) == 0
    face = FL.Mesh.from_arrays(m, device=-1, face_path=True)
    assert face.path == "face"
    assert L.fl_apply_workspace_bytes(face.handle, 2) >= m.n_faces * 16


def test_nonuniform_area_and_volume_kept():
    m = W.periodic_box(5, 3)
    area = m.face_area * (1 + 0.1 * np.arange(m.n_faces) / m.n_faces)
    mesh = FL.Mesh(m.face_cells, m.face_normal, area, m.cell_volume, device=-1)
    assert mesh.info.uniform_area == 0 and mesh.info.uniform_volume == 1


def _ell_dense(val, col, n_cols):
    width, rows = val.shape
    A = np.zeros((rows, n_cols))
    for k in range(width):
        np.add.at(A, (np.arange(rows), col[k]), val[k])
    return A


@pytest.mark.parametrize("name,m,k", [
    ("line7", W.periodic_box(7, 1), 2),
    ("quad6r", W.renumber(W.periodic_box(6, 2), seed=3), 4),
    ("hex5r", W.renumber(W.periodic_box(5, 3), seed=4), 6),
])
def test_algebraic_matrices_match_the_literal_construction(name, m, k):
    """The library's ELLPACK matrices of Algorithms 3/4 equal the oracle's sparse-matrix
    construction of Section 2 (D = E, UUD = T, OUD = -S, Pi, M), with 2k stored entries per row
    of UUD and OUD (zero coefficients of the pattern included, as the paper counts them)."""
    from oracle.mini_oracle import AlgebraicMesh

    import dataclasses

    rng = np.random.default_rng(1)
    m = dataclasses.replace(m, face_area=m.face_area * rng.uniform(0.5, 1.5, m.n_faces),
                            cell_volume=m.cell_volume * rng.uniform(0.5, 1.5, m.n_cells))
    mesh = FL.Mesh.from_arrays(m, device=-1)
    alg = FL.Algebraic(mesh)
    ref = AlgebraicMesh.from_arrays(m)
    C, F = m.n_cells, m.n_faces
    assert alg.rows == {"D": F, "UUD": F, "OUD": F, "Pi": F, "M": C}
    assert alg.width == {"D": 2, "UUD": 2 * k, "OUD": 2 * k, "Pi": 2, "M": k}
    want = {"D": ref.E, "UUD": ref.T, "OUD": -ref.S, "Pi": ref.Pi, "M": ref.M}
    for key, A in want.items():
        val, col = alg.export(key)
        got = _ell_dense(val, col, F if key == "M" else C)
        np.testing.assert_allclose(got, A.toarray(), rtol=0, atol=1e-14, err_msg=key)
    # every structural column of a UUD row is a distinct cell
    _, col = alg.export("UUD")
    assert all(len(set(col[:, f])) == 2 * k for f in range(F))
    alg.close()
    mesh.close()


def test_checkpoint_interval_for_memory_budget():
    m = W.periodic_box(10, 3)  # 1000 cells: one SSP-RK3 step stores 3 * 1000 * 8 = 24000 bytes
    mesh = FL.Mesh.from_arrays(m, device=-1)
    f = FL.checkpoint_interval_for_budget
    assert f(mesh, "ssprk3", 1, 400, 0) == 20  # never below ceil(sqrt(N))
    assert f(mesh, "ssprk3", 1, 400, 24000 * 57) == 57
    assert f(mesh, "ssprk3", 1, 400, 10**12) == 400  # everything stored: nothing recomputed
    assert f(mesh, "euler", 2, 400, 16000 * 100) == 100
    assert [FL.checkpoint_interval(n) for n in (1, 2, 4, 5, 400, 401)] == [1, 2, 2, 3, 20, 21]
    mesh.close()


def test_empty_and_oversized_meshes_are_rejected_before_reading():
    """n_cells or n_faces of 0, and sizes beyond the 32-bit index range, are FL_E_INVALID; the
    size check comes before any array is read (the arrays passed here are one face long)."""
    L = _lib.lib()
    fc = np.zeros((1, 2), dtype=np.int32)
    nrm = np.zeros((1, 3))
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for nc, nf in [(0, 1), (1, 0), (0, 0), (2**31, 1), (4, 2**30)]:
        assert L.fl_mesh_validate(nc, nf, P(fc), P(nrm)) == -1, (nc, nf)


_TABLES_SCRIPT = r"""
import hashlib, sys
import numpy as np
sys.path.insert(0, {root!r})
from paper_2110_03044_amd import fluxlim as FL, workloads as W
meshes = [W.renumber(W.periodic_box(24, 3), seed=11), W.renumber(W.periodic_box(40, 2), seed=12),
          W.renumber(W.periodic_box(300, 1), seed=13), W.renumber(W.periodic_triangles(20), seed=14),
          W.periodic_box(17, 3)]
for m in meshes:
    for reorder in (False, True):
        mesh = FL.Mesh.from_arrays(m, device=-1, reorder=reorder)
        h = hashlib.sha256()
        for a in mesh.permutation() + mesh.export_tables():
            h.update(np.ascontiguousarray(a).tobytes())
        i = mesh.info
        print(h.hexdigest(), i.pairs, i.tile_cells, i.max_halo, i.halo_total, i.general)
        mesh.close()
"""


def test_tables_do_not_depend_on_thread_count():
    """The mesh builder's loops run on OpenMP threads; the numbering, the exported tables and
    the tile halo figures must be the same for any thread count (1 and 4 here, each in a fresh
    process so the runtime reads OMP_NUM_THREADS)."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = _TABLES_SCRIPT.format(root=root)
    outs = []
    for threads in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr
        outs.append(r.stdout)
    assert outs[0] == outs[1]
    assert len(outs[0].splitlines()) == 10


def test_mesh_progress_report():
    """With FL_MESH_PROGRESS set, fl_mesh_create reports each preprocessing phase on stderr;
    without it, nothing."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2110_03044_amd import fluxlim as FL, workloads as W\n"
            "FL.Mesh.from_arrays(W.periodic_box(10, 3), device=-1, reorder=True).close()\n" % root)
    phases = ["validated", "cells renumbered", "faces renumbered", "far-upwind cells",
              "slot tables", "tile tables"]
    for on in (True, False):
        env = dict(os.environ)
        env.pop("FL_MESH_PROGRESS", None)
        if on:
            env["FL_MESH_PROGRESS"] = "1"
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        lines = [l for l in r.stderr.splitlines() if l.startswith("fl_mesh_create:")]
        if on:
            assert [l.split(": ", 1)[1].split(" (")[0] for l in lines] == phases
            assert all("(1000 cells)" in l for l in lines)
        else:
            assert lines == []


def test_periodic_lattice_tiles_are_whole_bricks_whatever_the_input_order():
    """On a periodic box whose sides are multiples of the 8x8x4 brick, the Morton numbering gives
    every 256-cell tile the 512-cell halo of a whole brick, also when cells and faces come in
    random order with random orientations (the walk's cut plane is folded back)."""
    for n in (16, 32):
        for m in (W.periodic_box(n, 3), W.renumber(W.periodic_box(n, 3), seed=7)):
            mesh = FL.Mesh.from_arrays(m, device=-1, reorder=True)
            info = mesh.info
            tiles = (mesh.n_cells + 255) // 256
            assert info.tile_cells == 256
            assert info.max_halo == 512 and info.halo_total == 512 * tiles
            mesh.close()


def test_adjoint_workspace_sizes():
    """General cells' adjoint keeps four face terms per face and scalar in its workspace; the
    paired kernels need none.  The per-step reverse workspace adds them after its cell buffers."""
    L = _lib.lib()
    tri = FL.Mesh.from_arrays(W.periodic_triangles(6), device=-1)
    box = FL.Mesh.from_arrays(W.periodic_box(6, 3), device=-1)

    def a256(x):
        return (x + 255) // 256 * 256

    for S in (1, 3, 8):
        assert L.fl_adjoint_workspace_bytes(tri.handle, S) == a256(tri.n_faces * 4 * S * 8)
        assert L.fl_adjoint_workspace_bytes(box.handle, S) == 0
        for scheme, k in ((1, 1), (3, 3)):
            slab = a256(tri.n_cells * S * 8)
            assert L.fl_rk_adjoint_workspace_bytes(tri.handle, scheme, S) == \
                k * slab + a256(tri.n_faces * 4 * S * 8)
    assert L.fl_adjoint_workspace_bytes(tri.handle, 0) == 0
    assert L.fl_adjoint_workspace_bytes(tri.handle, 9) == 0
    tri.close()
    box.close()
