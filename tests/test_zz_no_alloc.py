"""fl_rk_steps_noalloc: the allocation-free variant of fl_rk_steps (workspace in the library's
fixed device array) gives the same bits as fl_rk_steps with a caller workspace, on two calls in
a row (the second on a smaller mesh, so the array holds the first call's contents), and rejects
a mesh whose workspace exceeds the array without enqueuing anything."""

import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2110_03044_amd import _lib, fluxlim as FL, workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _noalloc(mesh, lim, scheme, dt, theta, u, n_steps):
    S = 1 if theta.dim() == 1 else theta.shape[1]
    st = _lib.lib().fl_rk_steps_noalloc(mesh.handle, FL.limiter_id(lim), FL.scheme_id(scheme),
                                        float(dt), S, int(n_steps),
                                        ctypes.c_void_p(theta.data_ptr()),
                                        ctypes.c_void_p(u.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("scheme", ["ssprk3", "euler"])
def test_noalloc_equals_workspace_call_twice(scheme):
    print(f"no-alloc: {scheme}", flush=True)
    for n, S, lim, steps, path in [(40, 2, "vanleer", 5, False), (14, 1, "superbee", 3, True)]:
        wl = W.workload_box(n, renumbered=True, steps=steps)
        mesh = FL.Mesh.from_arrays(wl.mesh, device=0, reorder=True, face_path=path)
        th0 = W.multi_scalar([wl.theta0 + 0.1 * s for s in range(S)]) if S > 1 else wl.theta0
        t0 = mesh.cells_to_mesh(torch.from_numpy(np.ascontiguousarray(th0)).to(DEV))
        u = mesh.faces_to_mesh(torch.from_numpy(wl.u).to(DEV))
        a = t0.clone()
        FL.rk_steps(mesh, lim, scheme, wl.dt, a, u, steps)
        b = t0.clone()
        assert _noalloc(mesh, lim, scheme, wl.dt, b, u, steps) == 0
        torch.cuda.synchronize()
        assert torch.equal(a, b), (n, S, lim)
        if n == 14:  # the smaller call also against the oracle
            want = O.OracleMesh.from_arrays(wl.mesh).run(lim, scheme, wl.dt, th0, wl.u, steps)
            got = mesh.cells_from_mesh(b).cpu().numpy()
            assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
        mesh.close()


def test_noalloc_rejects_oversized_workspace():
    print("no-alloc: oversized", flush=True)
    n, S = 96, 8
    m = W.periodic_box(n, 3)
    mesh = FL.Mesh.from_arrays(m, device=0)
    need = _lib.lib().fl_rk_workspace_bytes(mesh.handle, 3, S)
    assert need > (128 << 20)
    th = torch.zeros((m.n_cells, S), dtype=torch.float64, device=DEV)
    u = torch.zeros(m.n_faces, dtype=torch.float64, device=DEV)
    assert _noalloc(mesh, "vanleer", "ssprk3", 1e-3, th, u, 1) == -1
    assert b"128" in _lib.lib().fl_last_error() or b"134217728" in _lib.lib().fl_last_error()
    assert _noalloc(mesh, "vanleer", "ssprk3", 1e-3, th[:, :1].contiguous(), u, 1) == 0
    torch.cuda.synchronize()
    mesh.close()
