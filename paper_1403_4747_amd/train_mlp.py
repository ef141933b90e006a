"""Offline training of the learned per-leaf preconditioner (FDA_PRECOND_MLP).

Training data come from the method's own GMRES solves on seeded rigid
ellipsoids: for every case the surface is meshed (icosphere scaled along the
axes), a plan is built, the plane-wave right-hand side b is solved tightly
(x*), and the GMRES(50) iterates x_m after m = 0, 1, 2, 4, 8, 16 products give
pairs (r_m = b - A x_m, e_m = x* - x_m) with A e_m = r_m; a few
complex-normal residuals r with e = A^-1 r are added.  fda_mlp_samples turns
every pair into one row per leaf (features of r and the target
(e - z)/s on top of the block-Jacobi correction z, s the row scale).  The network is
then trained on the device (fda_mlp_train) and evaluated on held-out seeds by
GMRES iterations and time to the tolerance, against block Jacobi.

Every step runs in libfda; this module only draws the seeded cases and moves
tensors.  Usage:

    python -m paper_1403_4747_amd.train_mlp --train 64 --eval 16 --out weights.npz
    python -m paper_1403_4747_amd.train_mlp --eval-only weights.npz --eval 100
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Sequence, Tuple

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

SNAPSHOTS = (0, 1, 2, 4, 8, 16)


def ellipsoid_case(seed: int, subdiv: int = 5, axes=(0.3, 0.7), kD=(20.0, 60.0)):
    """One seeded case: (V, T, k, direction, info).  Semi-axes uniform in
    `axes`, kD (D = largest diameter) uniform in `kD`, incidence direction
    uniform on the sphere."""
    import workloads as W

    rng = np.random.default_rng(1_000_003 * (seed + 1))
    a = rng.uniform(axes[0], axes[1], size=3)
    V, T = W.ellipsoid(subdiv, tuple(a))
    D = 2.0 * float(a.max())
    kd = float(rng.uniform(kD[0], kD[1]))
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    return V, T, kd / D, d, dict(seed=seed, semi_axes=a.tolist(), kD=kd, n=len(T))


def case_samples(plan, direction, tol_star: float = 1e-6, snapshots: Sequence[int] = SNAPSHOTS, n_random: int = 4,
                 seed: int = 0, maxit_star: int = 400):
    """(X, T, M) rows of one case: the GMRES iterates of the plane-wave
    solve, plus `n_random` complex-normal residuals r with e = A^-1 r (their
    leaf components are independent, so the rows also carry the local part
    of A^-1 that GMRES residuals, dominated by a few global modes, hide).

    x* and A^-1 r are solved to `tol_star`: GMRES over the FP32 plan's
    products stalls near a relative residual of 2e-7 (the products' own
    rounding), so a tighter tolerance only spends iterations; the targets
    e_m = x* - x_m stay accurate to tol_star / |r_m|, at most 1e-3 relative
    for the iterates kept."""
    import torch

    import workloads as W

    b = plan.rhs_planewave(direction)
    xs, info = plan.solve(b, tol=tol_star, restart=50, maxit=maxit_star)
    rs, es = [], []
    for m in snapshots:
        if m == 0:
            xm = torch.zeros_like(b)
        else:
            xm, _ = plan.solve(b, tol=1e-300, restart=50, maxit=m)
        rs.append(b - plan.matvec(xm))
        es.append(xs - xm)
    if n_random > 0:
        R = torch.from_numpy(np.ascontiguousarray(W.complex_normal(plan.n, n_random, seed=seed).T)).to(b.device)
        E, _ = plan.solve(R, tol=tol_star, restart=50, maxit=maxit_star)
        rs.extend(R)
        es.extend(E)
    return plan.mlp_samples(torch.stack(rs), torch.stack(es)), info


def generate(seeds: Sequence[int], eps: float = 1e-4, prec: str = "fp32", log=print, n_random: int = 4,
             max_seconds: float = None, **case_kw):
    """Concatenated training rows of the given seeds (device tensors); with
    `max_seconds`, generation stops after the case that crosses it."""
    import torch

    from .fda import Plan

    t_all = time.perf_counter()
    Xs, Ts, Ms, meta = [], [], [], []
    for s in seeds:
        t0 = time.perf_counter()
        V, T, k, d, info = ellipsoid_case(s, **case_kw)
        with Plan(V, T, k, eps, prec=prec) as p:
            tb = time.perf_counter() - t0
            phases = [round(v, 2) for v in p.stats()["build_phase_seconds"][:7]]
            (X, Tg, M), sinfo = case_samples(p, d, n_random=n_random, seed=s)
        Xs.append(X)
        Ts.append(Tg)
        Ms.append(M)
        info.update(rows=int(X.shape[0]), its_star=sinfo["iterations"], res_star=sinfo["rel_residual"],
                    build_seconds=round(tb, 2), build_phase_seconds=phases,
                    seconds=round(time.perf_counter() - t0, 2))
        meta.append(info)
        log(f"[train_mlp] case {s}: N={info['n']} kD={info['kD']:.1f} rows={info['rows']} x* in "
            f"{info['its_star']} its ({info['seconds']} s, build {info['build_seconds']} s {phases})")
        if max_seconds is not None and time.perf_counter() - t_all > max_seconds:
            log(f"[train_mlp] generation stopped after {len(meta)} solves ({max_seconds} s budget)")
            break
    return torch.cat(Xs), torch.cat(Ts), torch.cat(Ms), meta


def evaluate(net, seeds: Sequence[int], eps: float = 1e-4, prec: str = "fp32", tol: float = 1e-5, log=print,
             **case_kw) -> List[Dict]:
    """GMRES(50) iterations and solve time to `tol` with block Jacobi and
    with the network, on held-out seeds."""
    import torch

    from .fda import Plan

    out = []
    for s in seeds:
        V, T, k, d, info = ellipsoid_case(s, **case_kw)
        with Plan(V, T, k, eps, prec=prec) as p:
            p.set_mlp(net)
            b = p.rhs_planewave(d)
            row = dict(info)
            sols = {}
            for pc in ("none", "block_jacobi", "mlp"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, st = p.solve(b, tol=tol, restart=50, maxit=2000, precond=pc)
                torch.cuda.synchronize()
                row[pc] = dict(iterations=st["iterations"], seconds=round(time.perf_counter() - t0, 4),
                               converged=st["converged"], mlp_fallbacks=st["mlp_fallbacks"],
                               mlp_rejected=st["mlp_rejected"])
                sols[pc] = x
            row["mlp_vs_none_rel_diff"] = float(torch.linalg.norm(sols["mlp"] - sols["none"]) /
                                                torch.linalg.norm(sols["none"]))
            p.set_mlp(None)
        log(f"[train_mlp] eval {s}: kD={info['kD']:.1f} its none/bj/mlp = {row['none']['iterations']}/"
            f"{row['block_jacobi']['iterations']}/{row['mlp']['iterations']} (judge rejected: "
            f"{row['mlp']['mlp_rejected']})")
        out.append(row)
    return out


def save(net, path: str, meta: Dict):
    np.savez(path, params=net.get_params(), hidden=np.int32(net.hidden),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load(path: str, device: int = 0):
    """A network from weights written by save() (no pickled objects)."""
    from .fda import Mlp

    z = np.load(path, allow_pickle=False)
    net = Mlp(hidden=int(z["hidden"]), seed=0, device=device)
    net.set_params(z["params"])
    return net


def summarize(ev: List[Dict]) -> Dict:
    """Means over held-out cases: iterations and seconds per preconditioner,
    how often the network needed fewer iterations than block Jacobi, and how
    often the solver's judge rejected it."""
    pcs = ("none", "block_jacobi", "mlp")
    return dict(
        eval_solves=len(ev),
        mean_iterations={pc: float(np.mean([r[pc]["iterations"] for r in ev])) for pc in pcs},
        mean_seconds={pc: float(np.mean([r[pc]["seconds"] for r in ev])) for pc in pcs},
        mlp_fewer_iterations_than_bj=int(sum(r["mlp"]["iterations"] < r["block_jacobi"]["iterations"] for r in ev)),
        judge_rejected=int(sum(r["mlp"]["mlp_rejected"] for r in ev)),
        all_converged=bool(all(r[pc]["converged"] for r in ev for pc in pcs)),
    )


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=64, help="training solves (seeds 0 ..)")
    ap.add_argument("--eval", type=int, default=16, help="held-out solves (seeds 100000 ..)")
    ap.add_argument("--subdiv", type=int, default=5)
    ap.add_argument("--hidden", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--prec", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--out", default="mlp_weights.npz")
    ap.add_argument("--random", type=int, default=4, help="random residuals per training solve")
    ap.add_argument("--report", default=None, help="write a JSON report here")
    ap.add_argument("--max-generate-seconds", type=float, default=None,
                    help="stop drawing training solves after this many seconds")
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="skip training: evaluate the network stored in WEIGHTS on the held-out seeds")
    args = ap.parse_args(argv)

    import torch

    from .fda import Mlp

    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    held_out = range(100000, 100000 + args.eval)
    if args.eval_only:
        net = load(args.eval_only)
        ev = evaluate(net, held_out, prec=args.prec, log=log, subdiv=args.subdiv)
        summary = dict(weights=os.path.basename(args.eval_only), subdiv=args.subdiv, prec=args.prec, **summarize(ev))
        if args.report:
            with open(args.report, "w") as f:
                json.dump(dict(summary=summary, eval=ev), f, indent=1)
        print(json.dumps(summary), flush=True)
        return
    t0 = time.perf_counter()
    X, Tg, M, meta = generate(range(args.train), prec=args.prec, log=log, n_random=args.random, subdiv=args.subdiv,
                              max_seconds=args.max_generate_seconds)
    gen_s = time.perf_counter() - t0
    log(f"[train_mlp] {X.shape[0]} rows from {args.train} solves in {gen_s:.1f} s")
    net = Mlp(hidden=args.hidden, seed=args.seed)
    t0 = time.perf_counter()
    losses = net.train(X, Tg, M, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=args.seed)
    train_s = time.perf_counter() - t0
    log(f"[train_mlp] trained {args.epochs} epochs in {train_s:.1f} s; loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    rows = int(X.shape[0])
    del X, Tg, M
    summary = dict(
        train_solves=len(meta), train_rows=rows, subdiv=args.subdiv, hidden=args.hidden, epochs=args.epochs,
        batch=args.batch, lr=args.lr, prec=args.prec, generate_seconds=round(gen_s, 2),
        train_seconds=round(train_s, 2), loss_first=float(losses[0]), loss_last=float(losses[-1]))
    save(net, args.out, dict(summary=summary, losses=[float(v) for v in losses]))
    ev = []
    if args.eval > 0:
        ev = evaluate(net, held_out, prec=args.prec, log=log, subdiv=args.subdiv)
        summary.update(summarize(ev))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(dict(summary=summary, losses=[float(v) for v in losses], train_cases=meta, eval=ev), f, indent=1)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
