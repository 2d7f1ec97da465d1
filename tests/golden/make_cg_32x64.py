"""Write the stored oracle solution of the 32^3 x 64 even/odd system used by the benchmark.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators: links
smooth_links((64, 32, 32, 32), seed 3000, width 0.3), right-hand side gaussian_spinor(Vh, 3003),
kappa = 0.1575.  Solves M_oo^dag M_oo x = b (Sec. 2.2; CG as in Sec. 1) with the oracle's
textbook CG until the true relative residual is at most 1e-14, then stores

  cg_32x64_kappa0.1575.npz   sites  int64 [4096]          odd-site checkerboard indices (seed 3099)
                             x      complex128 [4096,4,3] the solution at those sites
  cg_32x64_kappa0.1575.json  |x|, |b|, iterations, true residual, the command and the inputs

The solve takes about an hour on one host core (the oracle's numpy kernels are single threaded):

    python tests/golden/make_cg_32x64.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dirac  # noqa: E402
from oracle.lattice import Lattice  # noqa: E402
from oracle.solve import cg, norm2  # noqa: E402
from paper_1805_03560_amd import synth  # noqa: E402

DIMS = (64, 32, 32, 32)
KAPPA = 0.1575
TOL = 1e-14
NSITES = 4096
NAME = "cg_32x64_kappa0.1575"


def main():
    t0 = time.time()
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, 3000, width=0.3, threads=min(16, os.cpu_count() or 1))
    b = synth.gaussian_spinor(lat.Vh, 3003)
    print(f"inputs ready in {time.time() - t0:.0f} s", flush=True)
    count = [0]

    def A(v):
        count[0] += 1
        if count[0] % 5 == 0:
            print(f"  {count[0]} applications of M_oo^dag M_oo, {time.time() - t0:.0f} s", flush=True)
        return dirac.apply_MooDagMoo(lat, U, v, KAPPA)

    x, iters, res = cg(A, b, tol=TOL, maxiter=1000)
    sites = np.sort(np.random.default_rng(3099).choice(lat.Vh, NSITES, replace=False)).astype(np.int64)
    np.savez(os.path.join(HERE, NAME + ".npz"), sites=sites, x=x[sites])
    meta = {
        "about": "oracle solution of M_oo^dag M_oo x = b (Sec. 2.2) on 32^3 x 64, written by "
                 "tests/golden/make_cg_32x64.py (oracle only)",
        "lattice_t_z_y_x": list(DIMS), "kappa": KAPPA,
        "links": "synth.smooth_links(dims, 3000, width=0.3)", "rhs": "synth.gaussian_spinor(Vh, 3003), odd sites",
        "cg_tol": TOL, "iterations": int(iters), "true_residual": float(res),
        "norm_x": float(np.sqrt(norm2(x))), "norm_b": float(np.sqrt(norm2(b))),
        "max_abs_x": float(np.max(np.abs(x))), "sites": f"{NSITES} odd-site cb indices, default_rng(3099)",
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, NAME + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
