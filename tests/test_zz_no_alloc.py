"""gdg_solve_noalloc, the entry point for callers that cannot allocate device
memory: the whole solve in the library's static device workspace.  Its result
must equal that of the same solve through gdg_create (caller workspace),
gdg_upload_state, gdg_run_to and gdg_download_state, on two calls in a row
(the second on a smaller mesh, in the same static array), from host and from
device buffers; a mesh whose workspace exceeds the array is refused."""
import numpy as np
import pytest
import torch

from paper_2402_04514_amd import gdg
from paper_2402_04514_amd import workloads as W

from test_gpu_parity import quadrant_on

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-noalloc] " + msg, flush=True)


def solve_noalloc(ms, prm, U0, t_final, max_steps, out, stream_ptr):
    mesh = gdg.mesh_desc(ms.dim, ms.degree, ms.cells, ms.lo, ms.hi, ms.bc, ms.bstate)
    return gdg.gdg_solve_noalloc(mesh, prm, U0, out, t_final, max_steps, stream_ptr)


def reference(ms, prm, U0, t_final, max_steps):
    S = gdg.Solver.from_spec(ms, prm)
    S.upload(U0)
    st = S.run_to(t_final, max_steps)
    out = S.download()
    S.close()
    return out, st


CASES = [
    # (mesh and state, final time, step limit)
    (lambda: quadrant_on(2, 2, (40, 36), (2, 2, 1, 1), seed=3), 0.02, 1000),
    (lambda: quadrant_on(2, 1, (12, 10), (1,) * 4, seed=5), 1e30, 13),
]


def test_noalloc_matches_workspace_path_twice():
    stream = torch.cuda.current_stream().cuda_stream
    for k, (make, tf, nmax) in enumerate(CASES):
        ms, U = make()
        prm = gdg.gdg_default_params(ms.degree)
        _say("call %d: %s cells, degree %d" % (k + 1, ms.cells, ms.degree))
        ref, rst = reference(ms, prm, U, tf, nmax)
        out = np.zeros_like(U)
        st = solve_noalloc(ms, prm, np.ascontiguousarray(U), tf, nmax, out, stream)
        assert st.steps == rst.steps and st.t == rst.t
        scale = np.abs(ref).max(axis=1, keepdims=True)
        err = float((np.abs(out - ref) / scale).max())
        _say("  %d steps, t %.6g, max relative difference %.2e" % (st.steps, st.t, err))
        assert err <= 1e-11
        assert st.bound_violations == rst.bound_violations == 0
        assert st.min_rho == rst.min_rho


def test_noalloc_device_buffers():
    ms, U = quadrant_on(2, 2, (16, 16), (2,) * 4, seed=7)
    prm = gdg.gdg_default_params(2)
    ref, rst = reference(ms, prm, U, 1e30, 9)
    Ud = torch.tensor(U, device="cuda:0")
    out = torch.zeros_like(Ud)
    stream = torch.cuda.current_stream().cuda_stream
    st = solve_noalloc(ms, prm, Ud, 1e30, 9, out, stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert st.steps == 9
    assert float((np.abs(got - ref) / scale).max()) <= 1e-11


def test_noalloc_refuses_a_mesh_beyond_its_array():
    ms = W.MeshSpec(2, 2, (512, 512), (0, 0), (1, 1), (1,) * 4)
    prm = gdg.gdg_default_params(2)
    U = np.zeros((4, ms.ndofs))
    out = np.zeros_like(U)
    with pytest.raises(gdg.GdgError) as ei:
        solve_noalloc(ms, prm, U, 1.0, 1, out, torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == gdg.GDG_E_NOMEM
    assert "at most" in str(ei.value)
