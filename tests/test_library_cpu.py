"""Host-side checks of the library that need no GPU: the shared library
loads, exports every symbol the header declares, and the host phase of the
build (tree, lists, directions) behaves."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fda.h")


def _lib():
    from paper_1403_4747_amd import library

    return library()


def test_header_symbols_exported():
    txt = open(HEADER).read()
    names = set(re.findall(r"^\s*(?:int|int32_t|int64_t|void|const char \*)\s*\**\s*([a-z_0-9]+)\s*\(", txt, re.M))
    assert {"fda_build", "fda_matvec", "bm_solve", "bm_rhs_planewave", "fda_free", "fda_last_error"} <= names
    L = _lib()
    for n in sorted(names):
        assert hasattr(L, n), n


def test_version_and_defaults():
    from paper_1403_4747_amd.fda import default_options

    L = _lib()
    assert b"gfx950" in L.fda_version()
    o = default_options()
    assert o.max_leaf == 64 and o.p0 == 1 and o.nrhs_max == 64


def test_inspect_config1_structure():
    from paper_1403_4747_amd import inspect

    V, T, prm = W.workload("sphere1280_kD10")
    st = inspect(V, T, prm["k"], prm["eps"])
    assert st["n"] == 1280
    assert st["max_leaf_count"] <= 64
    assert st["depth"] == 2 and st["top_level"] == 2
    assert st["m2l_offsets"][2] == 316  # (-3..3)^3 minus the 27 adjacent offsets
    # the leaves are at least 2.5 largest edges wide
    assert st["root_width"] / 2 ** st["depth"] >= 2.5 * st["h_max"]


def test_inspect_directional_levels_at_kD100():
    from paper_1403_4747_amd import inspect

    V, T, prm = W.workload("sphere20480_kD100")
    st = inspect(V, T, prm["k"], prm["eps"])
    lam = 2 * np.pi / prm["k"]
    for l in range(st["depth"] + 1):
        w = st["root_width"] / 2 ** l
        assert st["hf"][l] == (1 if (l > 0 and w >= 1.9 * lam * (1 - 1e-9)) else 0)
        if st["hf"][l]:
            n = st["ndir"][l]
            assert n % 6 == 0 and int(round((n // 6) ** 0.5)) ** 2 == n // 6
    # directional cells double per level upwards
    hfl = [l for l in range(st["depth"] + 1) if st["hf"][l]]
    for a, b in zip(hfl[:-1], hfl[1:]):
        assert st["ndir"][a] == 4 * st["ndir"][b]


def test_pair_coverage_counts():
    """Every ordered pair of elements is either evaluated directly (near
    field) or reached by exactly one interaction-list pair: near entries
    plus the element pairs of all interaction-list pairs sum to N^2
    (Algorithm, Step 1: the lists partition the far field)."""
    from paper_1403_4747_amd import inspect

    for name in ("sphere5120_kD20", "sphere20480_kD100"):
        V, T, prm = W.workload(name)
        st = inspect(V, T, prm["k"], prm["eps"])
        n = st["n"]
        assert 0 < st["near_nnz"] < n * n
        assert sum(st["m2l_pairs"]) > 0
        assert st["near_nnz"] + st["far_elem_pairs"] == n * n, name
        # a uniform tree: every leaf on the finest level, no W / X lists
        assert st["leaves"][-1] == st["nleaf"] and st["w_pairs"] == st["x_pairs"] == 0


@pytest.mark.parametrize("bad", ["index", "zero_area", "k", "eps"])
def test_inspect_errors(bad):
    from paper_1403_4747_amd import inspect, FDAError

    V, T = W.icosphere(1, 0.5)
    k, eps = 10.0, 1e-4
    if bad == "index":
        T = T.copy()
        T[3, 1] = len(V) + 5
    elif bad == "zero_area":
        T = T.copy()
        T[0, 2] = T[0, 1]
    elif bad == "k":
        k = -1.0
    else:
        eps = 1.5
    with pytest.raises(FDAError) as e:
        inspect(V, T, k, eps)
    assert e.value.code in (-1, -2)


def test_product_path_has_no_oracle_import():
    """The package never imports the oracle (the oracle is test-only)."""
    pkg = os.path.join(ROOT, "paper_1403_4747_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "bem_oracle" not in txt, f


def test_inspect_rejects_leaves_above_256_elements():
    """A strongly graded mesh (one large triangle beside 400 tiny ones) would
    need leaves wider than 2.5 largest edges holding > 256 elements: the
    build refuses it instead of overflowing the per-leaf kernels."""
    from paper_1403_4747_amd import inspect, FDAError

    rng = np.random.default_rng(0)
    V, T = [], []
    for i in range(400):  # tiny triangles scattered in a 0.05 cube
        c = rng.uniform(0.0, 0.05, size=3)
        base = len(V)
        V += [c, c + [1e-3, 0, 0], c + [0, 1e-3, 0]]
        T.append([base, base + 1, base + 2])
    base = len(V)
    V += [[0.0, 0.0, 1.0], [1.0, 0.0, 1.0], [0.0, 1.0, 1.0]]
    T.append([base, base + 1, base + 2])
    V, T = np.array(V), np.array(T, dtype=np.int32)
    with pytest.raises(FDAError) as e:
        inspect(V, T, 5.0, 1e-4)
    assert e.value.code == -2 and "256" in str(e.value)
    # with narrow leaves allowed the same mesh builds
    st = inspect(V, T, 5.0, 1e-4, leaf_min_h=0.01)
    assert st["max_leaf_count"] <= 64
    # an adaptive tree sizes each box by its own largest edge, but here the
    # root holds the large triangle and cannot be split either
    with pytest.raises(FDAError) as e:
        inspect(V, T, 5.0, 1e-4, adaptive=1)
    assert e.value.code == -2 and "256" in str(e.value)
