"""Writes the stored expected values under tests/golden/ from the FP64
oracle alone (plus the seeded grid generator).  Run from the repository
root:  python tests/golden/make_golden.py  (about 15 minutes on one core,
a few on eight: the oracle shares its line and point loops among threads,
with results independent of the thread count).

cyl512x256_lad_curv_fp64.json: the 2D cylinder O-grid 512 x 256 (wall
R = 0.5, far field r = 20, outflow faces, radial spacing 1e-3 * 1.03^j
capped), C6 derivatives, 10th-order filter (alpha_f 0.495), LAD pseudo-HJ
(eps 0.2, C 0.1) with curvature correction, RK4, sigma 1, solved from
phi = 0 until the max change is <= 1e-10 (Sec. 3.3-3.5): iteration count,
L-inf error against r - R, the field on 8 theta-lines at every 4th radial
node, and how far that field still is from the discrete fixed point
(2000 further iterations).
cyl512x256_lad_curv_fp64.f64.gz: that converged field at all 131,072
points, float64 little-endian, r-major (index j * 512 + i), gzip.
"""
import gzip
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2111_09859_amd import grids as G  # noqa: E402


def cylinder_config():
    spec = G.cylinder(512, 256)
    kw = dict(equation=O.HJ, gamma=O.GAMMA_LAD, curvature=1, eps=0.2, C_lad=0.1,
              scheme="C6", filter=1, alpha_f=0.495, rk=O.RK4, sigma=1.0)
    t0 = time.time()
    phi, st, it, hist = O.solve(spec, O.make_method(tol=1e-10, max_iter=20000, **kw))
    t1 = time.time()
    more = 2000
    phi2, _, it2, _ = O.solve(spec, O.make_method(fixed_iters=it + more, **kw))
    ti = np.arange(0, 512, 64)
    rj = np.arange(0, 256, 4)
    samples = [[int(i), int(j), float(phi[j, i])] for i in ti for j in rj]
    rec = {
        "grid": "cylinder 512x256, R=0.5, r_out=20, dr1=1e-3, ratio=1.03, outflow far field",
        "method": "HJ, LAD eps=0.2 C=0.1, curvature, C6, F10 alpha_f=0.495, RK4, sigma=1",
        "stop": "max change <= 1e-10",
        "status": int(st), "iters": int(it),
        "linf_err_vs_exact": float(np.abs(phi - spec.exact).max()),
        "hist_last": [float(hist[it - 1, 0]), float(hist[it - 1, 1])],
        "extra_iters": more,
        "max_change_over_extra_iters": float(np.abs(phi2 - phi).max()),
        "samples_i_j_phi": samples,
        "oracle_seconds": round(t1 - t0, 1),
    }
    with gzip.GzipFile(os.path.join(HERE, "cyl512x256_lad_curv_fp64.f64.gz"), "wb", mtime=0) as f:
        f.write(np.ascontiguousarray(phi, dtype="<f8").tobytes())
    with open(os.path.join(HERE, "cyl512x256_lad_curv_fp64.json"), "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    print("cylinder:", {k: v for k, v in rec.items() if k != "samples_i_j_phi"}, flush=True)


if __name__ == "__main__":
    cylinder_config()
