"""Parity checks shared by the GPU tests: the HIP product against the
oracle's, element by element."""
import numpy as np

# Matvec bound of the method's specification (relative 2-norm), and the
# per-entry bound that catches a wrong leaf or block, which a 2-norm over many
# rows can hide: every entry within 1e-3 of the largest oracle entry.
MATVEC_TOL = 1e-4
ROW_TOL = 1e-3
# Regression bounds: a few times the measured error, so that a loss of
# accuracy well inside the specification still fails.  Default plans (SVD
# truncation at eps / 10): 2e-6 to 5e-6 on the 1,280- to 81,920-triangle
# spheres; plans truncated at the paper's eps (eqs. (eq_epsg), (eq_epsk)),
# the benchmark's headline configuration: 1.6e-5 to 2.8e-5.
REGRESS = 2e-5
REGRESS_EPS = 6e-5


def rel_err(y, yr):
    return float(np.linalg.norm(y - yr) / np.linalg.norm(yr))


def row_err(y, yr):
    """Largest entry error as a fraction of the largest oracle entry."""
    return float(np.max(np.abs(y - yr)) / np.max(np.abs(yr)))


def check(y, yr, tol=MATVEC_TOL, row_tol=ROW_TOL, regress=None):
    """Assert the relative 2-norm error <= tol, the per-entry error <=
    row_tol * max|yr| and, when given, the 2-norm error <= regress (a bound a
    few times above the measured error of the configuration, so that a loss of
    accuracy well inside the specification still fails).  Returns both
    errors."""
    e, r = rel_err(y, yr), row_err(y, yr)
    assert e <= tol, f"relative 2-norm error {e:.3e} > {tol:.1e}"
    assert r <= row_tol, f"largest entry error {r:.3e} of max|y| > {row_tol:.1e}"
    if regress is not None:
        assert e <= regress, f"relative 2-norm error {e:.3e} above the regression bound {regress:.1e}"
    return e, r
