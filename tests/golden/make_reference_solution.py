"""Write the oracle's own GMRES solution of a rigid sphere under a plane wave.

Calls only the FP64 oracle (``oracle/``) and the input generators
(``workloads``): the stored solution never depends on the GPU library.

Problem (Section 2, eq. (eq_bm) with zero Neumann data; Section 5): rigid
sphere of radius 0.5 meshed as an icosphere of ``--subdiv`` midpoint
subdivisions, wavenumber ``--k``, unit plane wave along +z, Burton-Miller
coupling of the oracle's default.  The dense operator is applied matrix-free
(every entry by the oracle's quadrature, OpenMP over rows) inside the
oracle's restarted MGS-GMRES, x0 = 0, stopping on the true relative residual
``--tol``.

A full product at 81,920 triangles takes several minutes on a few cores, so
``--cache-dir`` (optional) keeps every product on disk, keyed by a hash of
its input: a run that is stopped and started again replays the same
iterations from the cache.

Output: an ``.npz`` with the solution in the caller's element order
(``u``, complex128), the right-hand side's norm, the iteration count, the
final true relative residual, the wall time, the thread count and the
SHA-256 of the oracle sources and of the mesh arrays.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402


def _sha(*paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def mesh_sha(V, T):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(V, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(T, dtype=np.int32).tobytes())
    return h.hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--subdiv", type=int, default=6)
    ap.add_argument("--k", type=float, default=100.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--maxit", type=int, default=400)
    ap.add_argument("--out", default=None)
    ap.add_argument("--cache-dir", default=None)
    a = ap.parse_args(argv)

    V, T = W.icosphere(a.subdiv, 0.5)
    n = len(T)
    out = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                f"sphere{n}_k{a.k:g}_solution.npz")
    O.build(force=False)
    b = O.rhs_planewave(V, T, a.k, np.array([0.0, 0.0, 1.0]))
    if a.cache_dir:
        os.makedirs(a.cache_dir, exist_ok=True)
    count = [0]
    t0 = time.time()

    def A(x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        key = hashlib.sha256(x.tobytes()).hexdigest()[:32]
        path = os.path.join(a.cache_dir, f"{n}_{a.k:g}_{key}.npy") if a.cache_dir else None
        if path and os.path.exists(path):
            y = np.load(path)
            tag = "cached"
        else:
            y = O.matvec(V, T, a.k, x)
            if path:
                np.save(path + ".tmp.npy", y)
                os.replace(path + ".tmp.npy", path)
            tag = "computed"
        count[0] += 1
        print(f"product {count[0]} {tag} at {time.time() - t0:.0f} s", flush=True)
        return y

    u, info = O.gmres(A, b, tol=a.tol, restart=a.restart, maxit=a.maxit)
    r = b - A(u)
    relres = float(np.linalg.norm(r) / np.linalg.norm(b))
    print(f"iterations {info['iters']} relres {relres:.3e} converged {info['converged']}", flush=True)
    src = [os.path.join(ROOT, "oracle", "bem_oracle.c"), os.path.join(ROOT, "oracle", "oracle.py")]
    np.savez(out, u=u, b_norm=np.linalg.norm(b), iterations=info["iters"], rel_residual=relres,
             tol=a.tol, restart=a.restart, k=a.k, subdiv=a.subdiv, radius=0.5,
             direction=np.array([0.0, 0.0, 1.0]), seconds=time.time() - t0,
             threads=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
             oracle_sha256=_sha(*src), mesh_sha256=mesh_sha(V, T))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
