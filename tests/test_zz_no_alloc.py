"""wd_solve_noalloc (no device allocation: workspace and line-operator
tables in the library's static scratch) against wd_solve through the C ABI:
two calls in a row, the second on a smaller grid, each compared with the
plain solve of the same input at FP64 1e-12 relative (the same kernels run,
so the fields agree bit for bit in practice), plus the rejection of a grid
too large for the scratch."""
import ctypes as C

import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_09859_amd import api
    s = api.Solver(0)
    yield s
    s.close()


def run_both(solver, spec, scheme, precision, n_iter, **kw):
    import torch
    from paper_2111_09859_amd import _lib as L, api
    prep = solver.prepare(spec, scheme, precision)
    m = api.make_method(scheme=scheme, precision=precision, tol=0.0, max_iter=n_iter, **kw)
    ref = solver.solve(prep, m)
    phi = torch.zeros(spec.shape, dtype=prep.dtype, device=solver.device)
    hist = (C.c_double * (2 * n_iter))()
    torch.cuda.synchronize()
    rc, it = L.wd_solve_noalloc(solver.ctx, prep.desc, m, C.c_void_p(phi.data_ptr()), None,
                                hist, n_iter, stream=solver.stream())
    torch.cuda.synchronize()
    assert it == ref["iters"] == n_iter
    got = phi.double().cpu().numpy()
    want = ref["phi"].double().cpu().numpy()
    e = float(np.abs(got - want).max() / np.abs(want).max())
    h = np.frombuffer(hist, dtype=np.float64).reshape(n_iter, 2)
    print(f"[no-alloc] {spec.name} {spec.n[:spec.ndim]} {scheme} {precision}: rel {e:.2e}, "
          f"history max diff {np.abs(h[:, 0] - ref['hist'][:, 0]).max():.2e}", flush=True)
    return e, h, ref["hist"]


def test_noalloc_matches_solve_twice(solver):
    # first call: a curvilinear O-grid (general passes, reduction-level
    # tables, LAD + curvature), FP64
    e1, h1, r1 = run_both(solver, G.cylinder(64, 48, rout=6.0, dr1=1e-2, ratio=1.12), "C6",
                          "fp64", 30, equation="HJ", gamma="LAD", curvature=True)
    assert e1 <= 1e-12
    assert np.allclose(h1[:, 0], r1[:, 0], rtol=1e-12, atol=0)
    # second call, smaller grid: Cartesian (segmented passes), Poisson with
    # its FP64 conversion tables
    e2, h2, r2 = run_both(solver, G.channel(40, 33), "E6", "fp64", 25, equation="POISSON")
    assert e2 <= 1e-12
    assert np.allclose(h2[:, 0], r2[:, 0], rtol=1e-12, atol=0)


def test_noalloc_fp32_cartesian(solver):
    e, _, _ = run_both(solver, G.duct(40, nx=48), "C6", "fp32", 10, equation="HJ", gamma="LAD",
                       alpha_f=0.48)
    assert e <= 1e-6


def test_noalloc_rejects_a_grid_beyond_the_scratch(solver):
    import torch
    from paper_2111_09859_amd import _lib as L, api
    spec = G.duct(160)
    prep = solver.prepare(spec, "C6", "fp32")
    m = api.make_method(scheme="C6", precision="fp32", tol=0.0, max_iter=2)
    phi = torch.zeros(spec.shape, dtype=prep.dtype, device=solver.device)
    rc, _ = L.wd_solve_noalloc(solver.ctx, prep.desc, m, C.c_void_p(phi.data_ptr()), None, None,
                               0, stream=solver.stream(), check=False)
    assert rc == L.WD_ERR_NO_MEMORY
    # a later call still works
    e, _, _ = run_both(solver, G.box2d(33), "E4", "fp64", 12, equation="HJ", gamma="LINEAR")
    assert e <= 1e-12
