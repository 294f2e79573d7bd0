"""Writes the oracle's solution of the 2D L-shape workload (1024^2 grid, 67k vertices).

Calls only the oracle and the seeded input generators.  For each order s of
the workload: T by Filon's rule with Richardson extrapolation at the paper's
levels M = 2^14 and 2^13 (Section 2.3), b = h^{2s} I_J^T f_FD and
K = I_J^T A_FD I_J (eq. GoFD-2 on the interior block), solved by the oracle's
conjugate gradients (FFT product of eq. AU-1) to a relative residual of 1e-13.
The stored solution u (all N_v vertices, zero on Dirichlet vertices) is the
truth the GPU solves of this workload are compared with; the file also keeps
the true relative residual ||b - K u|| / ||b|| of that solution and a hash of
the inputs, so that a test can tell when the generators have changed.

Run from the repository root:  python tests/golden/make_c2_oracle_solution.py
(about ten minutes on eight cores).
"""

from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fdweights as fw, operator, solve, transfer   # noqa: E402
from workloads import config_inputs                            # noqa: E402

OUT = os.path.join(HERE, "c2_oracle_solution.npz")
M_FINE = 2 ** 14
TOL = 1e-13


def input_hash(mesh, grid, f) -> str:
    h = hashlib.sha256()
    for a in (mesh.X, mesh.elems, f):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr((grid.d, grid.N, grid.R, tuple(grid.center))).encode())
    return h.hexdigest()[:16]


def main():
    c = config_inputs("c2")
    mesh, g, f = c["mesh"], c["grid"], c["f"][0]
    tr = transfer.Transfer(mesh.X, mesh.elems, 2, g.N, g.R, g.center)
    out = {"input_hash": np.array(input_hash(mesh, g, f)), "s": np.array(c["s"]),
           "M": np.array(M_FINE), "tol": np.array(TOL)}
    for s in c["s"]:
        t0 = time.time()
        T = fw.filon_richardson(s, 2, 2 * g.N, M_FINE)
        b = operator.rhs_grid(tr, s, f)
        Kop = lambda v: operator.apply_K(tr, T, v, "fft")          # noqa: E731
        uJ, it, hist = solve.pcg(Kop, b, tol=TOL, maxiter=20000)
        res = float(np.linalg.norm(b - Kop(uJ)) / np.linalg.norm(b))
        u = np.zeros(mesh.nv)
        u[tr.J] = uJ
        key = f"{s:g}"
        out[f"u_{key}"] = u
        out[f"iterations_{key}"] = np.array(it)
        out[f"true_residual_{key}"] = np.array(res)
        print(f"s={s}: {it} iterations, true relative residual {res:.3e}, {time.time() - t0:.0f} s", flush=True)
    np.savez(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
