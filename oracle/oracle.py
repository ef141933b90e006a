"""FP64 CPU oracle: dense collocation Burton-Miller operator, right-hand
sides, solvers and the analytic solutions that pin them.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.

Paper map
---------
* Operators A (left-hand side) and B (right-hand side for Neumann data):
  Section 2, eqs. (cbie), (eq_bm), (eq_sum); collocation at centroids with
  piecewise-constant elements, Section 5.  The element integrals live in
  ``bem_oracle.c`` (see its header for the quadrature and self terms).
* Plane-wave right-hand side for a rigid body: eq. (eq_bm) with zero Neumann
  data, b = u_inc + alpha du_inc/dn.
* GMRES: Section 5 (tolerance, no preconditioner).
* Pulsating sphere: Section 5.1 (the printed closed form is the complex
  conjugate of what G = exp(ikr)/(4 pi r) gives; see ``pulsating_sphere``).
* Mie series of a rigid sphere and the n = 0 sphere eigenvalues of the four
  layer operators: textbook closed forms used to pin the operators.

Normal convention: the paper's n points out of the fluid into the body; the
mesh triangles are wound counter-clockwise seen from the fluid, so n is the
negated right-hand normal.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Callable, Dict, Optional

import numpy as np

__all__ = [
    "build", "lib", "geometry", "kernels", "self_integrals", "element_integrals",
    "r7_rule", "gl_rule", "rows", "assemble", "apply", "matvec",
    "rhs_planewave", "neumann_rhs", "gmres", "solve_dense",
    "mie_rigid_sphere", "mie_rigid_sphere_series", "sphere_n0_eigenvalues",
    "pulsating_sphere", "point_source_data", "OPS", "default_alpha",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

OPS = {"S": 0, "K": 1, "Kp": 2, "T": 3, "A": 4, "B": 5}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        L.or_geometry.argtypes = [dp, i64, ip, i64, dp, dp, dp, dp]
        L.or_geometry.restype = ctypes.c_int
        L.or_kernels.argtypes = [i64, dp, dp, dp, dp, ctypes.c_double, dp]
        L.or_rows.argtypes = [dp, i64, ip, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, lp, i64, dp]
        L.or_rows.restype = ctypes.c_int
        L.or_apply.argtypes = [dp, i64, ip, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, lp, i64, dp, i64, dp]
        L.or_apply.restype = ctypes.c_int
        L.or_r7_rule.argtypes = [dp, dp]
        L.or_gl_rule.argtypes = [dp, dp]
        L.or_self.argtypes = [dp, dp, dp, dp, ctypes.c_double, dp]
        L.or_element.argtypes = [dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(V, T):
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    return V, T


def geometry(V, T):
    """Centroids, paper normals (into the body), areas, largest edge."""
    V, T = _prep(V, T)
    nt = len(T)
    cen = np.empty((nt, 3))
    nrm = np.empty((nt, 3))
    area = np.empty(nt)
    h = np.empty(1)
    rc = lib().or_geometry(_d(V), len(V), T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nt,
                           _d(cen), _d(nrm), _d(area), _d(h))
    if rc != 0:
        raise ValueError("degenerate triangle or vertex index out of range")
    return cen, nrm, area, float(h[0])


def kernels(x, y, nx, ny, k):
    """[G, dG/dn_y, dG/dn_x, d2G/dn_x dn_y] at point pairs; shape (n, 4)."""
    x, y, nx, ny = (np.ascontiguousarray(np.atleast_2d(a), dtype=np.float64) for a in (x, y, nx, ny))
    n = len(x)
    out = np.empty((n, 4), dtype=np.complex128)
    lib().or_kernels(n, _d(x), _d(y), _d(nx), _d(ny), float(k), _d(out.view(np.float64)))
    return out


def self_integrals(a, b, c, x, k):
    """[int G, 0, 0, f.p. int d2G] over triangle abc at collocation point x."""
    a, b, c, x = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, x))
    out = np.empty(4, dtype=np.complex128)
    lib().or_self(_d(a), _d(b), _d(c), _d(x), float(k), _d(out.view(np.float64)))
    return out


def element_integrals(a, b, c, x, nx, k, level=0):
    """[int G, int dG/dn_y, int dG/dn_x, int d2G] over triangle abc by the
    7-point rule on 4**level midpoint sub-triangles (triangle normal = the
    negated right-hand normal of abc)."""
    a, b, c, x, nx = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, x, nx))
    out = np.empty(4, dtype=np.complex128)
    lib().or_element(_d(a), _d(b), _d(c), _d(x), _d(nx), float(k), int(level), _d(out.view(np.float64)))
    return out


def r7_rule():
    bary = np.empty((7, 3))
    w = np.empty(7)
    lib().or_r7_rule(_d(bary), _d(w))
    return bary, w


def gl_rule():
    x = np.empty(32)
    w = np.empty(32)
    lib().or_gl_rule(_d(x), _d(w))
    return x, w


def default_alpha(k):
    """Burton-Miller coupling.  The paper takes alpha = i/k (Section 2, after
    eq. (eq_bm)), the choice of the cited analysis, which is stated for the
    normal pointing into the fluid.  The paper's n points into the body, so
    the same coupling is alpha = -i/k here.  (With +i/k in this convention
    part of the spectrum moves to the left half-plane: GMRES(50) needs 77
    instead of 15 iterations on the 5,120-triangle sphere at kD = 40.)"""
    return -1j / k


def _alpha(k, alpha):
    return default_alpha(k) if alpha is None else complex(alpha)


def rows(V, T, k, row_idx, op="A", alpha=None):
    """Dense rows of an operator: M[row_idx, :] (complex128)."""
    V, T = _prep(V, T)
    r = np.ascontiguousarray(row_idx, dtype=np.int64)
    a = _alpha(k, alpha)
    out = np.empty((len(r), len(T)), dtype=np.complex128)
    rc = lib().or_rows(_d(V), len(V), T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(T),
                       float(k), a.real, a.imag, OPS[op], r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                       len(r), _d(out.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle: bad mesh")
    return out


def assemble(V, T, k, op="A", alpha=None):
    """Full dense operator (small meshes only)."""
    return rows(V, T, k, np.arange(len(T)), op, alpha)


def apply(V, T, k, x, op="A", alpha=None, row_idx=None):
    """Matrix-free product (M x)[row_idx]; x of shape (N,) or (N, nrhs)."""
    V, T = _prep(V, T)
    x = np.asarray(x, dtype=np.complex128)
    vec = x.ndim == 1
    X = np.ascontiguousarray(x.reshape(len(T), -1))
    nrhs = X.shape[1]
    r = np.arange(len(T), dtype=np.int64) if row_idx is None else np.ascontiguousarray(row_idx, dtype=np.int64)
    a = _alpha(k, alpha)
    Y = np.empty((len(r), nrhs), dtype=np.complex128)
    rc = lib().or_apply(_d(V), len(V), T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(T),
                        float(k), a.real, a.imag, OPS[op], r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        len(r), _d(X.view(np.float64)), nrhs, _d(Y.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle: bad mesh")
    return Y[:, 0] if vec else Y


def matvec(V, T, k, x, alpha=None, row_idx=None):
    """y = A x for the Burton-Miller left-hand operator."""
    return apply(V, T, k, x, "A", alpha, row_idx)


def rhs_planewave(V, T, k, direction, alpha=None):
    """Rigid (sound-hard) body under u_inc = exp(ik d.x): du/dn = 0 in
    eq. (eq_bm), so b_i = u_inc(c_i) + alpha du_inc/dn(c_i)
    = exp(ik d.c_i) (1 + alpha i k d.n_i).  direction: (3,) or (nrhs, 3)."""
    cen, nrm, _, _ = geometry(V, T)
    a = _alpha(k, alpha)
    D = np.atleast_2d(np.asarray(direction, dtype=np.float64))
    ph = np.exp(1j * k * (cen @ D.T))
    b = ph * (1.0 + a * 1j * k * (nrm @ D.T))
    return b[:, 0] if np.ndim(direction) == 1 else b


def neumann_rhs(V, T, k, g, alpha=None, row_idx=None):
    """Right-hand side of eq. (eq_bm) for Neumann data g (no incident wave):
    b = (-alpha/2 I + S + alpha K') g."""
    return apply(V, T, k, g, "B", alpha, row_idx)


def gmres(matvec_fn: Callable[[np.ndarray], np.ndarray], b, tol=1e-5, restart=50, maxit=1000,
          x0=None):
    """Restarted GMRES with modified Gram-Schmidt and Givens rotations.
    Stops when the true relative residual ||b - A x|| / ||b|| <= tol.
    Returns (x, info) with info = dict(iters, relres, converged)."""
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, dict(iters=0, relres=0.0, converged=True)
    iters = 0
    r = b - matvec_fn(x) if x0 is not None else b.copy()
    beta = np.linalg.norm(r)
    while iters < maxit:
        if beta / bnorm <= tol:
            return x, dict(iters=iters, relres=beta / bnorm, converged=True)
        m = restart
        Vb = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        Vb[0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec_fn(Vb[j])
            iters += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                Vb[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            hjj, hj1 = H[j, j], H[j + 1, j]
            den = math.sqrt(abs(hjj) ** 2 + abs(hj1) ** 2)
            cs[j] = hjj / den if den else 1.0
            sn[j] = hj1 / den if den else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            j_done = j + 1
            if abs(g[j + 1]) / bnorm <= tol or iters >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Vb[:j_done].T @ y
        r = b - matvec_fn(x)
        beta = np.linalg.norm(r)
    return x, dict(iters=iters, relres=beta / bnorm, converged=beta / bnorm <= tol)


def solve_dense(A, b):
    """Direct LU solve (SciPy)."""
    import scipy.linalg as sla

    return sla.lu_solve(sla.lu_factor(A), b)


# ------------------------------------------------------------ closed forms

def _sph(n, x):
    from scipy.special import spherical_jn, spherical_yn

    return (spherical_jn(n, x), spherical_jn(n, x, derivative=True),
            spherical_yn(n, x), spherical_yn(n, x, derivative=True))


def mie_rigid_sphere(a, k, cos_theta, nmax=None):
    """Total surface field of a rigid sphere of radius a under exp(ik d.x),
    cos_theta = d . x_hat.  Uses the Wronskian j_n y_n' - j_n' y_n = x^-2:
        u(a, theta) = i/(ka)^2 sum_n (2n+1) i^n P_n(cos theta) / h_n'(ka)."""
    from scipy.special import eval_legendre

    x = k * a
    if nmax is None:
        nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 10)
    ct = np.asarray(cos_theta, dtype=np.float64)
    u = np.zeros(ct.shape, dtype=np.complex128)
    for n in range(nmax + 1):
        j, jp, y, yp = _sph(n, x)
        hp = jp + 1j * yp
        u += (2 * n + 1) * (1j ** n) * eval_legendre(n, ct) / hp
    return 1j / x ** 2 * u


def mie_rigid_sphere_series(a, k, cos_theta, nmax=None):
    """The same field summed as incident + scattered partial waves,
    u = sum_n (2n+1) i^n [j_n(ka) + c_n h_n(ka)] P_n, c_n = -j_n'(ka)/h_n'(ka)
    (zero normal derivative on r = a), without the Wronskian shortcut."""
    from scipy.special import eval_legendre

    x = k * a
    if nmax is None:
        nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 10)
    ct = np.asarray(cos_theta, dtype=np.float64)
    u = np.zeros(ct.shape, dtype=np.complex128)
    for n in range(nmax + 1):
        j, jp, y, yp = _sph(n, x)
        h, hp = j + 1j * y, jp + 1j * yp
        u += (2 * n + 1) * (1j ** n) * (j - jp / hp * h) * eval_legendre(n, ct)
    return u


def sphere_n0_eigenvalues(a, k, alpha=None) -> Dict[str, complex]:
    """Action of the four layer operators on a constant density over a
    sphere of radius a (paper normal pointing into the sphere), from the
    addition theorem G = ik sum j_n(kr<) h_n(kr>) ...; only n = 0 survives:
        S 1  = ik a^2 j0(ka) h0(ka)
        K 1  = 1/2 - i k^2 a^2 j0'(ka) h0(ka)    (direct value, dG/dn_y)
        K' 1 = -1/2 - i k^2 a^2 j0(ka) h0'(ka)   (direct value, dG/dn_x)
        T 1  = i k^3 a^2 j0'(ka) h0'(ka)         (hypersingular)
    and A 1 = 1/2 + K 1 + alpha T 1 (alpha defaults to default_alpha(k))."""
    j, jp, y, yp = _sph(0, k * a)
    h, hp = j + 1j * y, jp + 1j * yp
    S1 = 1j * k * a * a * j * h
    K1 = 0.5 - 1j * k * k * a * a * jp * h
    Kp1 = -0.5 - 1j * k * k * a * a * j * hp
    T1 = 1j * k ** 3 * a * a * jp * hp
    al = _alpha(k, alpha)
    return dict(S=S1, K=K1, Kp=Kp1, T=T1, A=0.5 + K1 + al * T1)


def pulsating_sphere(a, k, vn=1.0):
    """Surface potential of a sphere of radius a pulsating with du/dn = vn
    (paper normal, into the sphere), exterior radiating field C h0(kr):
        u(a) = a vn / (1 - i k a).
    The paper prints 1/(1 + ik) for a = 1: the complex conjugate, i.e. the
    exp(-ikr) time convention; |u| agrees."""
    return a * vn / (1.0 - 1j * k * a)


def point_source_data(V, T, k, x0):
    """Exterior radiating field v = G(x, x0) of a point source x0 inside the
    body: returns (v(c_i), dv/dn(c_i)) at the centroids (paper normal)."""
    cen, nrm, _, _ = geometry(V, T)
    r = cen - np.asarray(x0, dtype=np.float64)[None, :]
    R = np.linalg.norm(r, axis=1)
    g = np.exp(1j * k * R) / (4 * np.pi * R)
    gp = g * (1j * k * R - 1.0) / R
    dn = gp * np.einsum("ij,ij->i", r, nrm) / R
    return g, dn
