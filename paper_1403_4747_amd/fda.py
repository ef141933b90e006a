"""Python binding of libfda (include/fda.h): argument marshalling only.

Every step of the build, matvec and solve runs in the HIP/C++ library; this
module converts numpy meshes and torch device tensors into pointers and
sizes.  It raises if the library is missing: there is no fallback path.

Vectors are torch.complex128 device tensors of shape (N,) for one
right-hand side or (nrhs, N) for several (each row is one column of the
N x nrhs column-major matrix the C ABI sees), in the caller's element order.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

__all__ = ["Plan", "Mlp", "Batch", "inspect", "library", "default_options", "FDAError", "PRECOND", "PREC", "MLP_IN",
           "MLP_OUT"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDA_LIBRARY may name another build of the same library (e.g. a variant
# compiled with different kernel options); the default is the in-tree build.
_SO = os.environ.get("FDA_LIBRARY") or os.path.join(_HERE, "libfda.so")

PREC = {"fp64": 0, "fp32": 1}
PRECOND = {"none": 0, "block_jacobi": 1, "mlp": 2}
MLP_IN, MLP_OUT = 272, 128

FDA_NOTCONV = 1


class FDAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfda error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("max_leaf", ctypes.c_int32), ("p_min", ctypes.c_int32), ("p0", ctypes.c_int32),
        ("svd_eps", ctypes.c_double), ("alpha_re", ctypes.c_double), ("alpha_im", ctypes.c_double),
        ("hf_wavelengths", ctypes.c_double), ("rho_c", ctypes.c_double), ("leaf_min_h", ctypes.c_double),
        ("prec", ctypes.c_int32), ("nrhs_max", ctypes.c_int32), ("device", ctypes.c_int32),
        ("verbose", ctypes.c_int32), ("svd_method", ctypes.c_int32), ("m2l_svd_eps", ctypes.c_double),
        ("neumann_rhs", ctypes.c_int32), ("adaptive", ctypes.c_int32), ("p_fixed", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("depth", ctypes.c_int32), ("top_level", ctypes.c_int32),
        ("nleaf", ctypes.c_int64), ("max_leaf_count", ctypes.c_int32), ("near_nnz", ctypes.c_int64),
        ("boxes", ctypes.c_int64 * 24), ("m2l_pairs", ctypes.c_int64 * 24), ("m2l_offsets", ctypes.c_int64 * 24),
        ("hf", ctypes.c_int32 * 24), ("ndir", ctypes.c_int32 * 24), ("active_dirs", ctypes.c_int32 * 24),
        ("p", ctypes.c_int32 * 24), ("rank_up", ctypes.c_int32 * 24), ("rank_dn", ctypes.c_int32 * 24),
        ("m2l_rank_max", ctypes.c_int32 * 24), ("m2l_rank_mean", ctypes.c_double * 24),
        ("m2l_level_flops", ctypes.c_double * 24), ("m2l_flops", ctypes.c_int64), ("m2l_bytes", ctypes.c_int64), ("h_max", ctypes.c_double),
        ("root_width", ctypes.c_double), ("build_seconds", ctypes.c_double), ("device_bytes", ctypes.c_int64),
        ("m2m_flops", ctypes.c_double), ("l2l_flops", ctypes.c_double), ("mlp_rows", ctypes.c_int64),
        ("build_phase_seconds", ctypes.c_double * 8), ("leaves", ctypes.c_int64 * 24),
        ("u_pairs", ctypes.c_int64), ("w_pairs", ctypes.c_int64), ("x_pairs", ctypes.c_int64),
        ("far_elem_pairs", ctypes.c_int64), ("max_near_cols", ctypes.c_int64),
        ("wx_elem_pairs", ctypes.c_int64), ("m2l_factor_bytes", ctypes.c_int64), ("m2l_state_bytes", ctypes.c_int64),
    ]

    def to_dict(self) -> Dict:
        d = {}
        L = self.depth
        for name, _ in self._fields_:
            v = getattr(self, name)
            if isinstance(v, ctypes.Array):
                v = list(v) if name == "build_phase_seconds" else list(v)[: L + 1]
            d[name] = v
        return d


class ProfileResult(ctypes.Structure):
    _fields_ = [
        ("near_ms", ctypes.c_double), ("s2m_ms", ctypes.c_double), ("m2m_ms", ctypes.c_double),
        ("m2l_ms", ctypes.c_double), ("l2l_ms", ctypes.c_double), ("l2t_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double), ("m2l_gemm_ms", ctypes.c_double * 24), ("perm_ms", ctypes.c_double),
        ("m2l_lowrank_ms", ctypes.c_double),
    ]


class M2LConfig(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("xcd_order", ctypes.c_int32), ("width", ctypes.c_int32 * 24)]

    def to_dict(self) -> Dict:
        return dict(variant=self.variant, xcd_order=self.xcd_order,
                    width={l: w for l, w in enumerate(self.width) if w})


class TuneResult(ctypes.Structure):
    _fields_ = [("best", M2LConfig), ("ms_before", ctypes.c_double), ("ms_after", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("nlevels", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("rel_residual", ctypes.c_double),
        ("seconds", ctypes.c_double), ("col_iterations", ctypes.c_int32 * 64), ("mlp_fallbacks", ctypes.c_int32),
        ("mlp_rejected", ctypes.c_int32),
    ]


_lib = None


def library():
    """Load libfda.so (built by paper_1403_4747_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise FDAError(-100, f"{_SO} is not built; run `python -m paper_1403_4747_amd.build`")
        L = ctypes.CDLL(_SO)
        vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.fda_default_options.argtypes = [ctypes.POINTER(Options)]
        L.fda_build.argtypes = [vp, i64, vp, i64, dbl, dbl, ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.fda_build.restype = ctypes.c_int
        L.fda_inspect.argtypes = [vp, i64, vp, i64, dbl, dbl, ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        L.fda_inspect.restype = ctypes.c_int
        L.fda_matvec.argtypes = [vp, vp, vp, i64, i64, vp]
        L.fda_matvec.restype = ctypes.c_int
        L.bm_rhs_planewave.argtypes = [vp, vp, i64, vp, i64, vp]
        L.bm_rhs_planewave.restype = ctypes.c_int
        L.bm_solve.argtypes = [vp, vp, vp, i64, i64, dbl, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.POINTER(SolveStats), vp]
        L.bm_solve.restype = ctypes.c_int
        L.fda_plan_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.fda_plan_stats.restype = ctypes.c_int
        L.fda_profile_matvec.argtypes = [vp, vp, vp, i64, i64, ctypes.c_int32, vp, ctypes.POINTER(ProfileResult)]
        L.fda_profile_matvec.restype = ctypes.c_int
        L.fda_free.argtypes = [vp]
        L.fda_mlp_create.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(vp)]
        L.fda_mlp_create.restype = ctypes.c_int
        L.fda_mlp_free.argtypes = [vp]
        L.fda_mlp_num_params.argtypes = [vp]
        L.fda_mlp_num_params.restype = i64
        L.fda_mlp_hidden.argtypes = [vp]
        L.fda_mlp_hidden.restype = ctypes.c_int32
        L.fda_mlp_get_params.argtypes = [vp, vp, i64]
        L.fda_mlp_get_params.restype = ctypes.c_int
        L.fda_mlp_set_params.argtypes = [vp, vp, i64]
        L.fda_mlp_set_params.restype = ctypes.c_int
        L.fda_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.fda_mlp_forward.restype = ctypes.c_int
        L.fda_mlp_forward_noalloc.argtypes = [vp, vp, i64, vp, vp]
        L.fda_mlp_forward_noalloc.restype = ctypes.c_int
        L.fda_mlp_gradient.argtypes = [vp, vp, vp, vp, i64, vp, ctypes.POINTER(dbl), vp]
        L.fda_mlp_gradient.restype = ctypes.c_int
        L.fda_mlp_train.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                    ctypes.c_uint64, vp, vp]
        L.fda_mlp_train.restype = ctypes.c_int
        L.fda_mlp_samples.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp, vp]
        L.fda_mlp_samples.restype = ctypes.c_int
        L.fda_plan_leaves.argtypes = [vp, vp, i64, vp, i64]
        L.fda_plan_leaves.restype = ctypes.c_int
        L.bm_rhs_neumann.argtypes = [vp, vp, vp, i64, i64, vp]
        L.bm_rhs_neumann.restype = ctypes.c_int
        L.fda_m2l_get_config.argtypes = [vp, ctypes.POINTER(M2LConfig)]
        L.fda_m2l_get_config.restype = ctypes.c_int
        L.fda_m2l_set_config.argtypes = [vp, ctypes.POINTER(M2LConfig)]
        L.fda_m2l_set_config.restype = ctypes.c_int
        L.fda_autotune.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(TuneResult)]
        L.fda_autotune.restype = ctypes.c_int
        L.fda_batch_create.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.POINTER(vp)]
        L.fda_batch_create.restype = ctypes.c_int
        L.fda_batch_launch.argtypes = [vp, vp]
        L.fda_batch_launch.restype = ctypes.c_int
        L.fda_batch_free.argtypes = [vp]
        L.fda_plan_set_mlp.argtypes = [vp, vp]
        L.fda_plan_set_mlp.restype = ctypes.c_int
        L.fda_last_error.restype = ctypes.c_char_p
        L.fda_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _err(rc: int):
    if rc < 0:
        raise FDAError(rc, library().fda_last_error().decode())


def default_options(**kw) -> Options:
    o = Options()
    library().fda_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _mesh(V, T):
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    if V.ndim != 2 or V.shape[1] != 3 or T.ndim != 2 or T.shape[1] != 3:
        raise ValueError("V must be (nv, 3) float64 and T (nt, 3) int32")
    return V, T


def inspect(V, T, k: float, eps: float = 1e-4, **opts) -> Dict:
    """Host-only dry run of the build's tree / list phase (no GPU)."""
    V, T = _mesh(V, T)
    o = default_options(**opts)
    st = Stats()
    rc = library().fda_inspect(V.ctypes.data, len(V), T.ctypes.data, len(T), float(k), float(eps),
                               ctypes.byref(o), ctypes.byref(st))
    _err(rc)
    return st.to_dict()


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A built fast-directional plan on the current GPU (fda_build)."""

    def __init__(self, V, T, k: float, eps: float = 1e-4, **opts):
        V, T = _mesh(V, T)
        self.n = len(T)
        self.k = float(k)
        o = default_options(**opts)
        h = ctypes.c_void_p()
        rc = library().fda_build(V.ctypes.data, len(V), T.ctypes.data, len(T), float(k), float(eps),
                                 ctypes.byref(o), ctypes.byref(h))
        _err(rc)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            library().fda_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @staticmethod
    def _check_vec(t, n):
        import torch

        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
            raise TypeError("expected a complex128 CUDA tensor")
        if not t.is_contiguous() or t.shape[-1] != n or t.dim() not in (1, 2):
            raise ValueError(f"expected a contiguous (N,) or (nrhs, N) tensor with N = {n}")
        return 1 if t.dim() == 1 else t.shape[0]

    def _check_out(self, out, x):
        """out (when given) must have x's shape and device: the library
        writes nrhs x N values into it."""
        import torch

        if out is None:
            return torch.empty_like(x)
        self._check_vec(out, self.n)
        if tuple(out.shape) != tuple(x.shape) or out.device != x.device:
            raise ValueError(f"out has shape {tuple(out.shape)} on {out.device}; expected {tuple(x.shape)} on "
                             f"{x.device}")
        if out.data_ptr() == x.data_ptr():
            raise ValueError("out must not be the input tensor")
        return out

    def matvec(self, x, out=None):
        """y = A x (fda_matvec).  x: (N,) or (nrhs, N) complex128 on the
        device; columns of a product of many columns (from 8 in FP64 plans,
        16 in FP32 ones) equal the single-column products to rounding."""
        nrhs = self._check_vec(x, self.n)
        y = self._check_out(out, x)
        rc = library().fda_matvec(self._h, x.data_ptr(), y.data_ptr(), nrhs, self.n, _stream())
        _err(rc)
        return y

    def rhs_neumann(self, g, out=None):
        """b = B g, the right-hand side for Neumann data du/dn = g
        (bm_rhs_neumann; the plan must be built with neumann_rhs=1)."""
        nrhs = self._check_vec(g, self.n)
        b = self._check_out(out, g)
        _err(library().bm_rhs_neumann(self._h, g.data_ptr(), b.data_ptr(), nrhs, self.n, _stream()))
        return b

    def rhs_planewave(self, directions: Sequence) -> "torch.Tensor":
        """b = u_inc + alpha du_inc/dn for unit plane waves (bm_rhs_planewave)."""
        import torch

        d = np.ascontiguousarray(np.atleast_2d(np.asarray(directions, dtype=np.float64)))
        nrhs = d.shape[0]
        b = torch.empty((nrhs, self.n) if np.ndim(directions) == 2 else (self.n,), dtype=torch.complex128,
                        device="cuda")
        rc = library().bm_rhs_planewave(self._h, d.ctypes.data, nrhs, b.data_ptr(), self.n, _stream())
        _err(rc)
        return b

    def solve(self, b, tol: float = 1e-5, restart: int = 50, maxit: int = 1000, precond: str = "none", out=None):
        """GMRES solve of A x = b (bm_solve).  Returns (x, stats dict)."""
        nrhs = self._check_vec(b, self.n)
        x = self._check_out(out, b)
        st = SolveStats()
        rc = library().bm_solve(self._h, b.data_ptr(), x.data_ptr(), nrhs, self.n, float(tol), int(restart),
                                int(maxit), PRECOND[precond], ctypes.byref(st), _stream())
        _err(rc)
        info = dict(iterations=st.iterations, restarts=st.restarts, rel_residual=st.rel_residual,
                    seconds=st.seconds, col_iterations=list(st.col_iterations)[:nrhs],
                    mlp_fallbacks=st.mlp_fallbacks, mlp_rejected=st.mlp_rejected, converged=(rc == 0))
        return x, info

    def leaves(self):
        """(perm, leaf_off): the caller's element index of each tree position
        and the tree-position range of each leaf (fda_plan_leaves)."""
        nl = self.stats()["nleaf"]
        perm = np.empty(self.n, dtype=np.int32)
        off = np.empty(nl + 1, dtype=np.int64)
        _err(library().fda_plan_leaves(self._h, perm.ctypes.data, self.n, off.ctypes.data, nl))
        return perm, off

    def set_mlp(self, mlp: Optional["Mlp"]):
        """Attach a learned preconditioner for precond="mlp" (fda_plan_set_mlp)."""
        _err(library().fda_plan_set_mlp(self._h, mlp._h if mlp is not None else None))
        self._mlp = mlp  # keep it alive while attached

    def mlp_samples(self, r, e=None):
        """Feature rows (and targets / masks when e = A^-1 r is given) of
        every row (a leaf, or a 64-element chunk of a larger leaf) for each
        residual column (fda_mlp_samples).  Returns float32 device tensors X
        (nrhs*mlp_rows, 272) and, with e, T and M (.., 128)."""
        import torch

        nrhs = self._check_vec(r, self.n)
        if e is not None and (self._check_vec(e, self.n) != nrhs):
            raise ValueError("r and e differ in shape")
        nl = self.stats()["mlp_rows"]
        X = torch.empty((nrhs * nl, MLP_IN), dtype=torch.float32, device=r.device)
        T = M = None
        if e is not None:
            T = torch.empty((nrhs * nl, MLP_OUT), dtype=torch.float32, device=r.device)
            M = torch.empty_like(T)
        rc = library().fda_mlp_samples(self._h, r.data_ptr(), e.data_ptr() if e is not None else None, nrhs, self.n,
                                       X.data_ptr(), T.data_ptr() if T is not None else None,
                                       M.data_ptr() if M is not None else None, _stream())
        _err(rc)
        return (X, T, M) if e is not None else X

    def stats(self) -> Dict:
        st = Stats()
        _err(library().fda_plan_stats(self._h, ctypes.byref(st)))
        return st.to_dict()

    def m2l_config(self) -> Dict:
        """The merged M2L launch configuration (fda_m2l_get_config):
        kernel variant, item order and pairs per work item per level."""
        c = M2LConfig()
        _err(library().fda_m2l_get_config(self._h, ctypes.byref(c)))
        return c.to_dict()

    def set_m2l_config(self, variant: Optional[int] = None, xcd_order: Optional[int] = None,
                       width: Optional[Dict[int, int]] = None) -> Dict:
        """Change the merged M2L launch configuration (fda_m2l_set_config);
        unnamed fields keep their current value."""
        c = M2LConfig()
        _err(library().fda_m2l_get_config(self._h, ctypes.byref(c)))
        if variant is not None:
            c.variant = int(variant)
        if xcd_order is not None:
            c.xcd_order = int(xcd_order)
        for l, w in (width or {}).items():
            c.width[int(l)] = int(w)
        _err(library().fda_m2l_set_config(self._h, ctypes.byref(c)))
        return self.m2l_config()

    def autotune(self, reps: int = 20) -> Dict:
        """Time the merged M2L launch configurations and keep the fastest
        (fda_autotune); returns the chosen configuration and the times."""
        r = TuneResult()
        _err(library().fda_autotune(self._h, int(reps), _stream(), ctypes.byref(r)))
        return dict(best=r.best.to_dict(), ms_before=r.ms_before, ms_after=r.ms_after, candidates=r.candidates,
                    nlevels=r.nlevels)

    def profile(self, x, reps: int = 10, out=None) -> Dict:
        """Per-stage HIP-event timings (ms) of fda_matvec, plus the merged
        low-rank M2L product kernel ("m2l_lowrank") and the full-rank M2L
        product kernel of every other level ("m2l_gemm", a list per level)."""
        nrhs = self._check_vec(x, self.n)
        y = self._check_out(out, x)
        res = ProfileResult()
        rc = library().fda_profile_matvec(self._h, x.data_ptr(), y.data_ptr(), nrhs, self.n, int(reps), _stream(),
                                          ctypes.byref(res))
        _err(rc)
        d = {q: getattr(res, q + "_ms") for q in ("near", "s2m", "m2m", "m2l", "l2l", "l2t", "perm", "total",
                                                  "m2l_lowrank")}
        d["m2l_gemm"] = list(res.m2l_gemm_ms)
        return d


def _f32_dev(t, width, name):
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if t.dim() != 2 or t.shape[1] != width:
        raise ValueError(f"{name} must have shape (rows, {width})")
    return t.shape[0]


class Mlp:
    """The learned per-leaf preconditioner network (fda_mlp_*)."""

    def __init__(self, hidden: int = 256, seed: int = 0, device: int = 0):
        h = ctypes.c_void_p()
        _err(library().fda_mlp_create(int(hidden), int(seed), int(device), ctypes.byref(h)))
        self._h = h
        self.hidden = int(hidden)

    def close(self):
        if getattr(self, "_h", None):
            library().fda_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(library().fda_mlp_num_params(self._h))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.num_params, dtype=np.float32)
        _err(library().fda_mlp_get_params(self._h, p.ctypes.data, p.size))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _err(library().fda_mlp_set_params(self._h, p.ctypes.data, p.size))

    def split(self, p=None) -> Dict[str, np.ndarray]:
        """The flat parameter array as W1, b1, W2, b2, W3, b3."""
        p = self.get_params() if p is None else p
        h, out = self.hidden, {}
        shapes = [("W1", (MLP_IN, h)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)), ("W3", (h, MLP_OUT)),
                  ("b3", (MLP_OUT,))]
        o = 0
        for name, shp in shapes:
            n = int(np.prod(shp))
            out[name] = p[o:o + n].reshape(shp)
            o += n
        return out

    def forward(self, X):
        import torch

        rows = _f32_dev(X, MLP_IN, "X")
        Y = torch.empty((rows, MLP_OUT), dtype=torch.float32, device=X.device)
        _err(library().fda_mlp_forward(self._h, X.data_ptr(), rows, Y.data_ptr(), _stream()))
        return Y

    def forward_noalloc(self, X, out):
        """forward() into the caller's `out` (rows x 128 float32) through the
        allocation-free entry point: the library allocates nothing."""
        rows = _f32_dev(X, MLP_IN, "X")
        if _f32_dev(out, MLP_OUT, "out") != rows:
            raise ValueError("X and out differ in rows")
        _err(library().fda_mlp_forward_noalloc(self._h, X.data_ptr(), rows, out.data_ptr(), _stream()))
        return out

    def gradient(self, X, T, M):
        """(loss, flat gradient as a float32 device tensor)."""
        import torch

        rows = _f32_dev(X, MLP_IN, "X")
        if _f32_dev(T, MLP_OUT, "T") != rows or _f32_dev(M, MLP_OUT, "M") != rows:
            raise ValueError("X, T and M differ in rows")
        g = torch.empty(self.num_params, dtype=torch.float32, device=X.device)
        loss = ctypes.c_double()
        _err(library().fda_mlp_gradient(self._h, X.data_ptr(), T.data_ptr(), M.data_ptr(), rows, g.data_ptr(),
                                        ctypes.byref(loss), _stream()))
        return loss.value, g

    def train(self, X, T, M, epochs: int = 10, batch: int = 1024, lr: float = 1e-3, seed: int = 0):
        """Adam training; returns the per-epoch mean losses."""
        rows = _f32_dev(X, MLP_IN, "X")
        if _f32_dev(T, MLP_OUT, "T") != rows or _f32_dev(M, MLP_OUT, "M") != rows:
            raise ValueError("X, T and M differ in rows")
        losses = np.zeros(int(epochs), dtype=np.float64)
        _err(library().fda_mlp_train(self._h, X.data_ptr(), T.data_ptr(), M.data_ptr(), rows, int(epochs), int(batch),
                                     float(lr), int(seed), losses.ctypes.data, _stream()))
        return losses


class Batch:
    """Products of several plans (different meshes and wavenumbers) captured
    in one HIP graph (fda_batch_*).  xs[i], ys[i]: complex128 device tensors
    of shape (N_i,) or (nrhs_i, N_i), fixed for the life of the batch."""

    def __init__(self, plans: Sequence[Plan], xs, ys):
        if not (len(plans) == len(xs) == len(ys)) or not plans:
            raise ValueError("plans, xs and ys must have the same nonzero length")
        nr = []
        for p, x, y in zip(plans, xs, ys):
            a = p._check_vec(x, p.n)
            if p._check_vec(y, p.n) != a:
                raise ValueError("x and y differ in columns")
            nr.append(a)
        n = len(plans)
        self._keep = (list(plans), list(xs), list(ys))
        ph = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
        xh = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        yh = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        nh = (ctypes.c_int64 * n)(*nr)
        h = ctypes.c_void_p()
        _err(library().fda_batch_create(ph, n, xh, yh, nh, ctypes.byref(h)))
        self._h = h

    def launch(self):
        _err(library().fda_batch_launch(self._h, _stream()))

    def close(self):
        if getattr(self, "_h", None):
            library().fda_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
