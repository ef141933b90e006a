"""Adaptive trees (Section 3.2: leaves on any level) on the host: the tree
and list phase through fda_inspect.  The U, V, W and X lists together must
reach every ordered element pair exactly once; leaves sit on several
levels of a graded mesh that a uniform tree refuses; a uniform mesh built
adaptively is still covered exactly."""
import math

import numpy as np
import pytest

import workloads as W


def _inspect(V, T, k, **kw):
    from paper_1403_4747_amd import inspect

    return inspect(V, T, k, 1e-4, **kw)


def test_graded_sphere_mesh():
    V, T = W.graded_sphere(3)
    assert len(T) == 4952
    assert np.allclose(np.linalg.norm(V, axis=1), 0.5, atol=1e-12)
    p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    c = (p0 + p1 + p2) / 3.0
    assert np.all(np.einsum("ij,ij->i", nrm, c) > 0)  # outward
    el = np.linalg.norm(np.stack([p1 - p0, p2 - p1, p0 - p2]), axis=2)
    assert el.max() / el.min() > 4.0  # graded: 4:1 in edge length
    # refined towards +z: the finest triangles lie in the top cap
    small = el.max(axis=0) < 1.5 * el.min()
    assert np.all(c[small, 2] > 0.3 * 0.5)
    # area converges to the sphere's (flat triangles inside the sphere)
    area = 0.5 * np.linalg.norm(nrm, axis=1).sum()
    assert 0.97 * math.pi < area < math.pi


@pytest.mark.parametrize("s,k", [(3, 10.0), (4, 20.0)])
def test_adaptive_tree_covers_every_pair_once(s, k):
    V, T = W.graded_sphere(s)
    n = len(T)
    st = _inspect(V, T, k, adaptive=1)
    assert st["near_nnz"] + st["far_elem_pairs"] == n * n
    nz = [l for l, c in enumerate(st["leaves"]) if c > 0]
    assert len(nz) >= 3, st["leaves"]  # leaves on several levels
    assert sum(st["leaves"]) == st["nleaf"]
    # W and X lists are duals: a (target leaf, source box) W pair is an X
    # entry seen from the source side
    assert st["w_pairs"] == st["x_pairs"] > 0
    assert st["max_leaf_count"] <= 256
    assert sum(st["m2l_pairs"]) > 0


def test_uniform_tree_refuses_the_graded_mesh():
    from paper_1403_4747_amd import FDAError

    V, T = W.graded_sphere(3)
    with pytest.raises(FDAError) as e:
        _inspect(V, T, 10.0)
    assert e.value.code == -2 and "256" in str(e.value)


@pytest.mark.parametrize("name", ["sphere5120_kD20", "sphere20480_kD100"])
def test_adaptive_build_of_a_uniform_mesh(name):
    """On a quasi-uniform sphere the adaptive tree stops some boxes early;
    coverage stays exact and directional levels keep no leaves."""
    V, T, prm = W.workload(name)
    n = len(T)
    u = _inspect(V, T, prm["k"])
    a = _inspect(V, T, prm["k"], adaptive=1)
    assert a["near_nnz"] + a["far_elem_pairs"] == n * n
    assert a["depth"] == u["depth"] and a["nleaf"] <= u["nleaf"]
    for l, h in enumerate(a["hf"]):
        if h:
            assert a["leaves"][l] == 0


def test_adaptive_option_is_validated():
    from paper_1403_4747_amd import FDAError

    V, T, prm = W.workload("sphere1280_kD10")
    with pytest.raises(FDAError) as e:
        _inspect(V, T, prm["k"], adaptive=2)
    assert e.value.code == -1


# ---------------------------------------------------------------------------
# An independent model of the adaptive tree and of which leaf pairs are
# evaluated directly, written from the definitions (Section 3.2 and the
# separation rules of Section 3), against the library's host phase.

def _model_tree(V, T, k, max_leaf=64, leaf_min_h=2.5, hf_wavelengths=1.9, adaptive=True):
    """Leaves of the adaptive (or uniform) tree as (level, integer key,
    element count).  Uniform: every leaf on the first level whose boxes all
    hold <= max_leaf elements or whose children would be narrower than
    leaf_min_h largest edges of the whole mesh."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cen = (a + b + c) / 3.0
    emax = np.maximum(np.linalg.norm(b - a, axis=1),
                      np.maximum(np.linalg.norm(c - a, axis=1), np.linalg.norm(c - b, axis=1)))
    lo, hi = V.min(axis=0), V.max(axis=0)
    side = (hi - lo).max() * (1.0 + 1e-9)
    origin = 0.5 * (lo + hi) - 0.5 * side
    lam = 2.0 * math.pi / k
    active = np.ones(len(T), dtype=bool)
    leaves = []
    boxes = _model_tree.boxes = []  # integer keys of every box, per level
    Lu = None
    if not adaptive:
        Lu = 0
        while Lu < 20 and side / 2.0**Lu * 0.5 >= leaf_min_h * emax.max():
            key = np.clip(np.floor((cen - origin) / (side / 2.0**Lu)).astype(np.int64), 0, 2**Lu - 1)
            if np.unique(key, axis=0, return_counts=True)[1].max() <= max_leaf:
                break
            Lu += 1
    for l in range(21):
        w = side / 2.0**l
        hf = l > 0 and w >= hf_wavelengths * lam * (1.0 - 1e-9)
        idx = np.nonzero(active)[0]
        if len(idx) == 0:
            break
        key = np.clip(np.floor((cen[idx] - origin) / w).astype(np.int64), 0, 2**l - 1)
        ukey, inv = np.unique(key, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        cnt = np.bincount(inv, minlength=len(ukey))
        hbox = np.zeros(len(ukey))
        np.maximum.at(hbox, inv, emax[idx])
        cannot = (w * 0.5 < leaf_min_h * hbox) | (l >= 20)
        if adaptive:
            # a directional box is subdivided unless its children would be
            # too narrow (then it is a directional leaf)
            leaf = ((cnt <= max_leaf) & (not hf)) | cannot
        else:
            leaf = np.full(len(ukey), l == Lu)
        for j in np.nonzero(leaf)[0]:
            leaves.append((l, ukey[j], int(cnt[j])))
        boxes.append(ukey)
        active[idx[leaf[inv]]] = False
    return leaves, side, lam


def _separated(d, l, side, lam, hf_wavelengths=1.9, rho_c=1.0):
    """Well separated on level l for integer offsets d (rows): not touching,
    and on a directional level at least rho apart (Section 3)."""
    sep = np.abs(d).max(axis=1) >= 2
    w = side / 2.0**l
    if l > 0 and w >= hf_wavelengths * lam * (1.0 - 1e-9):
        rho = max(2.0 * w, rho_c * w * w / lam)
        sep &= np.sqrt((d.astype(np.float64) ** 2).sum(axis=1)) * w >= rho * (1.0 - 1e-12)
    return sep


def _model_v_pairs(boxes, side, lam):
    """Interaction-list pairs per level: ordered pairs of boxes of the same
    level that are well separated there and on no coarser level (their
    ancestors were all near each other)."""
    out = []
    for l, keys in enumerate(boxes):
        i, j = np.meshgrid(np.arange(len(keys)), np.arange(len(keys)), indexing="ij")
        i, j = i.ravel(), j.ravel()
        far = _separated(keys[i] - keys[j], l, side, lam)
        for m in range(l):
            far &= ~_separated((keys[i] >> (l - m)) - (keys[j] >> (l - m)), m, side, lam)
        out.append(int(far.sum()))
    return out


def _model_near_entries(leaves, side, lam, hf_wavelengths=1.9, rho_c=1.0):
    """Near-field entries: sum of n_t n_s over leaf pairs (t, s) none of whose
    same-level ancestor pairs is well separated (not touching, and on a
    directional level at least rho apart)."""
    lev = np.array([t[0] for t in leaves])
    key = np.array([t[1] for t in leaves])
    n = np.array([t[2] for t in leaves], dtype=np.int64)
    T_, S_ = np.meshgrid(np.arange(len(leaves)), np.arange(len(leaves)), indexing="ij")
    T_, S_ = T_.ravel(), S_.ravel()
    m = np.minimum(lev[T_], lev[S_])
    separated = np.zeros(len(T_), dtype=bool)
    for l in range(int(lev.max()) + 1):
        sel = m >= l
        kt = key[T_[sel]] >> (lev[T_[sel]] - l)[:, None]
        ks = key[S_[sel]] >> (lev[S_[sel]] - l)[:, None]
        d = kt - ks
        sep = np.abs(d).max(axis=1) >= 2
        w = side / 2.0**l
        if l > 0 and w >= hf_wavelengths * lam * (1.0 - 1e-9):
            rho = max(2.0 * w, rho_c * w * w / lam)
            sep &= np.sqrt((d.astype(np.float64) ** 2).sum(axis=1)) * w >= rho * (1.0 - 1e-12)
        separated[np.nonzero(sel)[0][sep]] = True
    direct = ~separated
    # classify the direct pairs: U (the two leaves touch), W (they do not
    # and the source is finer), X (they do not and the source is coarser)
    lt, ls = lev[T_[direct]], lev[S_[direct]]
    coarse_k = np.where((lt <= ls)[:, None], key[T_[direct]], key[S_[direct]])
    fine_k = np.where((lt <= ls)[:, None], key[S_[direct]], key[T_[direct]])
    sh = np.abs(lt - ls)[:, None]  # closed boxes meet: compare on the finer level
    touch = np.all((fine_k + 1 >= coarse_k << sh) & (fine_k <= (coarse_k + 1) << sh), axis=1)
    _model_near_entries.uwx = (int(touch.sum()), int((~touch & (ls > lt)).sum()), int((~touch & (ls < lt)).sum()))
    return int((n[T_[direct]] * n[S_[direct]]).sum())


def _coarse_ellipsoid(i):
    """Meshes of the seeded uneven batch whose leaves must sit on a
    directional level: 5,120 triangles at kD 90 (i = 20) and 97 (i = 25),
    about two elements per wavelength."""
    V, T, k, info = W.uneven_batch(32)[i]
    assert info["n"] == 5120 and info["kD"] > 90
    return V, T, k


@pytest.mark.parametrize("case,adaptive", [("graded3_kD10", 1), ("graded4_kD60", 1), ("sphere20480_kD50", 1),
                                           ("sphere20480_kD50", 0), ("sphere20480_kD100", 0),
                                           ("batch25", 0), ("batch25", 1), ("batch20", 1)])
def test_tree_and_direct_pairs_match_an_independent_model(case, adaptive):
    if case.startswith("graded"):
        s, k = (3, 10.0) if case == "graded3_kD10" else (4, 60.0)
        V, T = W.graded_sphere(s)
    elif case.startswith("batch"):
        V, T, k = _coarse_ellipsoid(int(case[5:]))
    else:
        V, T, prm = W.workload(case)
        k = prm["k"]
    st = _inspect(V, T, k, adaptive=adaptive)
    leaves, side, lam = _model_tree(V, T, k, adaptive=bool(adaptive))
    per_level = [0] * (st["depth"] + 1)
    for l, _, _ in leaves:
        per_level[l] += 1
    assert per_level == list(st["leaves"]), (per_level, st["leaves"])
    assert max(c for _, _, c in leaves) == st["max_leaf_count"]
    assert _model_near_entries(leaves, side, lam) == st["near_nnz"]
    assert _model_near_entries.uwx == (st["u_pairs"], st["w_pairs"], st["x_pairs"])
    assert _model_v_pairs(_model_tree.boxes, side, lam) == list(st["m2l_pairs"])
    if case != "graded3_kD10":
        assert any(st["hf"])  # directional levels above the leaves


def test_long_near_rows_are_planned():
    """A graded sphere with leaves of up to 256 elements has near-field rows
    longer than 4,096 columns; the plan accepts them (the long-row kernel
    needs no LDS) and still covers every ordered element pair once."""
    V, T = W.graded_sphere(3)
    st = _inspect(V, T, 10.0, max_leaf=256, adaptive=1)
    assert st["max_near_cols"] > 4096
    assert st["near_nnz"] + st["far_elem_pairs"] == len(T) ** 2


@pytest.mark.parametrize("i,adaptive", [(25, 0), (25, 1)])
def test_directional_leaves_are_planned(i, adaptive):
    """Coarse meshes at high frequency (Section 3.2): leaves on a
    directional level, which keep one state per direction slot; every
    ordered element pair is still reached exactly once."""
    V, T, k = _coarse_ellipsoid(i)
    st = _inspect(V, T, k, adaptive=adaptive)
    hf_leaves = [l for l in range(st["depth"] + 1) if st["hf"][l] and st["leaves"][l] > 0]
    assert hf_leaves, (st["hf"], st["leaves"])
    assert all(st["active_dirs"][l] > 1 for l in hf_leaves)
    assert st["near_nnz"] + st["far_elem_pairs"] == len(T) ** 2
