"""CPU tests of the library's host side: exported symbols, descriptor
validation paths that need no device, and the line-system reduction tables
the kernels use (checked against dense solves built here from the scheme
definitions)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2111_09859_amd import _lib
    _lib.lib()
    return _lib


def test_exports_every_declared_symbol(L):
    text = open(os.path.join(ROOT, "include", "wd.h")).read()
    names = set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(wd_\w+)\s*\(", text, re.M))
    assert len(names) >= 20
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: --gpus above 1 ends with a message
    and a non-zero status before anything touches a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_version_and_defaults(L):
    assert "gfx950" in L.wd_version()
    m = L.wd_method_default()
    assert m.equation == L.WD_EQ_HJ and m.scheme == L.WD_C6 and m.alpha_f == 0.48


def dense_deriv(n, periodic, scheme):
    al = {"C4": 0.25, "C6": 1 / 3}[scheme]
    A = np.eye(n)
    for i in range(n):
        for o in (-1, 1):
            j = i + o
            if periodic:
                A[i, j % n] += al
            elif 0 <= j < n:
                A[i, j] = al
    if not periodic:
        A[0, :] = 0
        A[0, 0], A[0, 1] = 1, 3
        A[-1, :] = 0
        A[-1, -1], A[-1, -2] = 1, 3
        if scheme == "C6":
            A[1, :3] = [0.25, 1, 0.25]
            A[-2, -3:] = [0.25, 1, 0.25]
    return A


def dense_filter(n, periodic, a):
    A = np.eye(n)
    for i in range(n):
        for o in (-1, 1):
            j = i + o
            if periodic:
                A[i, j % n] += a
            elif 0 < i < n - 1:
                A[i, j] = a
    return A


@pytest.mark.parametrize("n", [8, 33, 129, 256, 512, 1025, 2049])
@pytest.mark.parametrize("periodic", [0, 1])
def test_line_reduction_matches_dense(L, n, periodic):
    rng = np.random.default_rng(n + periodic)
    r = rng.standard_normal(n)
    for scheme in ("C4", "C6"):
        A = dense_deriv(n, periodic, scheme)
        want = np.linalg.solve(A, r)
        x, lev = L.wd_line_solve_host(0, r, periodic, scheme, 0.495, True)
        assert np.abs(x - want).max() < 1e-13 * max(1, np.abs(want).max()), (scheme, lev)
        x32, _ = L.wd_line_solve_host(0, r, periodic, scheme, 0.495, False)
        assert np.abs(x32 - want).max() < 2e-6 * max(1, np.abs(want).max())
    for a in (0.48, 0.495):
        A = dense_filter(n, periodic, a)
        rr = r.copy()
        if not periodic:
            rr[0] = rr[-1] = 0.0
        want = np.linalg.solve(A, rr)
        x, lev = L.wd_line_solve_host(1, rr, periodic, "C6", a, True)
        assert np.abs(x - want).max() < 1e-12 * max(1, np.abs(want).max()), (a, lev)
        assert lev <= 14


def test_line_reduction_rejects_bad_sizes(L):
    with pytest.raises(L.WDError):
        L.wd_line_solve_host(0, np.zeros(4), 0, "C6", 0.495, True)


def test_tile_quotient_by_reciprocal_is_exact():
    """The line kernels split an in-tile index a < 2^13 by a line length or
    band width b <= 4096 as int((a + 1/2) * fl(1/b)) in float32; check that
    this equals floor(a / b) for every such pair."""
    a = np.arange(0, 8192, dtype=np.float32)
    ai = np.arange(0, 8192)
    for b in range(1, 4097):
        rb = np.float32(1.0) / np.float32(b)
        q = ((a + np.float32(0.5)) * rb).astype(np.int64)
        assert np.array_equal(q, ai // b), b


def seg_plan(n):
    """(segments, segment length) the segmented passes use for a line of n
    points (None when no segmentation fits): segments of 32, 24 or 16,
    at most 16, the one shorter segment holding >= 2 positions (>= 5 when
    it is the first of two), a single segment full."""
    for M in (32, 24, 16):
        S = -(-n // M)
        r = n - (S - 1) * M
        if S > 16:
            continue
        if r == M or (S == 2 and r >= 5) or (S >= 3 and r >= 2):
            return S, M
    return None


@pytest.mark.parametrize("n", [16, 32, 33, 40, 48, 65, 96, 100, 129, 256, 257, 500])
@pytest.mark.parametrize("periodic", [0, 1])
def test_segmented_solve_matches_dense(L, n, periodic):
    """The segmented line solve (segments factored on their own, joined by
    the host-inverted reduced system) reproduces the dense solution of the
    compact-derivative and filter systems, with the segmentation the
    kernels use."""
    plan = seg_plan(n)
    rng = np.random.default_rng(7 * n + periodic)
    r = rng.standard_normal(n)
    for scheme in ("C4", "C6"):
        want = np.linalg.solve(dense_deriv(n, periodic, scheme), r)
        x, su = L.wd_seg_solve_host(0, r, periodic, scheme, 0.48)
        assert su == plan
        assert np.abs(x - want).max() < 1e-13 * max(1, np.abs(want).max()), (scheme, su)
    for a in (0.48, 0.495):
        rr = r.copy()
        if not periodic:
            rr[0] = rr[-1] = 0.0
        want = np.linalg.solve(dense_filter(n, periodic, a), rr)
        x, su = L.wd_seg_solve_host(1, rr, periodic, "C6", a)
        assert np.abs(x - want).max() < 1e-12 * max(1, np.abs(want).max()), (a, su)


def test_segmentation_choices(L):
    """Lines the segmented passes take, and lines they leave to the
    reduction-level passes (no segmentation fits)."""
    for n, want in ((256, (8, 32)), (129, (6, 24)), (65, (3, 24)), (16, (1, 16)), (100, (4, 32)),
                    (40, (2, 32)), (512, (16, 32)), (96, (3, 32))):
        assert seg_plan(n) == want
        _, su = L.wd_seg_solve_host(0, np.ones(n), 0, "C6", 0.48)
        assert su == want, (n, su)
    for n in (17, 20, 600, 4096):
        assert seg_plan(n) is None
        with pytest.raises(L.WDError):
            L.wd_seg_solve_host(0, np.ones(n), 0, "C6", 0.48)
