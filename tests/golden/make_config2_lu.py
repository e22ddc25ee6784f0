"""Write the FP64 oracle's exact discrete solution of the 10,242-vertex sphere.

Sphere of 10,242 vertices / 20,480 triangles, k0 = 10, k1 = 10.5, density
ratio 1.05, unit plane wave along +z (the solve workload of the apply
benchmark).  The oracle assembles the dense PMCHWT matrix in FP64 (6-point far
rule, Sauter-Schwab order 6; 20,484 unknowns, 6.7 GB) and solves it by dense LU
(numpy/LAPACK), the exact discrete solution below the 25k-unknown bound of
dense solves.  Only ``oracle`` and ``bem_inputs`` are used.

Output: ``config2_lu_planewave_z.npy`` (complex128 [20484], unknowns in domain
order [u_D; u_N]) and ``config2_lu_planewave_z.json`` (the workload, the LU
solution's own residual and the time taken).  Needs about 27 GB of host memory
and a quarter of an hour on 8 cores.

    python tests/golden/make_config2_lu.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from bem_inputs import configs  # noqa: E402


def main():
    prob = configs.config2()
    t0 = time.perf_counter()
    A = oracle.pmchwt_matrix(prob)
    p, dp = oracle.plane_wave(prob.k0)
    b = oracle.rhs(prob, p, dp)
    t1 = time.perf_counter()
    print(f"assembled {A.shape} in {t1 - t0:.0f} s", flush=True)
    u = oracle.solve_lu(A, b)
    t2 = time.perf_counter()
    res = float(np.linalg.norm(b - A @ u) / np.linalg.norm(b))
    print(f"LU in {t2 - t1:.0f} s, relative residual {res:.2e}", flush=True)
    np.save(os.path.join(HERE, "config2_lu_planewave_z.npy"), u)
    meta = {"workload": "icosphere level 5 (10,242 v / 20,480 t), unit radius, k0 = 10, k1 = 10.5, rho1/rho0 = 1.05, "
                        "unit plane wave along +z; FP64 oracle, 6-point far rule, Sauter-Schwab order 6, dense LU",
            "unknowns": int(u.shape[0]), "lu_rel_residual": res, "assembly_s": t1 - t0, "lu_s": t2 - t1,
            "norm_uD": float(np.linalg.norm(u[:prob.domains[0].n_vertices])),
            "norm_uN": float(np.linalg.norm(u[prob.domains[0].n_vertices:]))}
    with open(os.path.join(HERE, "config2_lu_planewave_z.json"), "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
