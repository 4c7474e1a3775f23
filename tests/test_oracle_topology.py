"""Pins of the oracle's topological control (ranked acceptance of simple-point
moves; Introduction, "The Region Competition (RC) algorithm").

The local simple-point test is held against definitions that do not use it:
in 2D, the global component counts of the region and of its complement
before and after toggling the pixel (exact equivalence for 8/4 connectivity);
in 3D, contractibility of the attachment of the voxel's closed cube to the
closed cubes of its neighbours (Alexander duality on the cube's boundary
sphere), plus the global invariants (components, complement components,
Euler characteristic) that every simple toggle must preserve.  Ranked
acceptance is pinned by its order independence (the paper's stated property),
by reducing to the simultaneous rule without control, and by preserving every
foreground region's topology.  None of these tests needs a GPU.
"""
import itertools

import numpy as np
import pytest

from paper_1403_0240_amd import workloads as W
from topo_invariants import topo as _topo


# ------------------------------------------------------------------ helpers

def _attachment_contractible(nb):
    """nb: 3x3x3 bool membership of the neighbours (centre ignored).  Is the
    intersection A of the centre's closed cube with the neighbours' closed
    cubes contractible?  On the boundary sphere S of the cube, A (a closed
    subcomplex) is contractible iff it is non-empty, connected, and S \\ A is
    non-empty and connected."""
    # boundary cells of [0,1]^3: per axis {0}, {1} or [0,1] (code 0, 1, 2); not all 2
    cells = [c for c in itertools.product((0, 1, 2), repeat=3) if c != (2, 2, 2)]

    def inside(c, o):
        for ci, oi in zip(c, o):
            if ci == 0 and oi not in (-1, 0):
                return False
            if ci == 1 and oi not in (0, 1):
                return False
            if ci == 2 and oi != 0:
                return False
        return True

    offs = [o for o in itertools.product((-1, 0, 1), repeat=3) if o != (0, 0, 0)]
    inA = {c: any(nb[o[0] + 1, o[1] + 1, o[2] + 1] and inside(c, o) for o in offs) for c in cells}

    def face_of(c, d):  # c is a face of d (c != d)
        return c != d and all(ci == di or di == 2 for ci, di in zip(c, d))

    def n_comp(sel):
        sel = list(sel)
        parent = {c: c for c in sel}

        def find(c):
            while parent[c] != c:
                parent[c] = parent[parent[c]]
                c = parent[c]
            return c
        for c, d in itertools.combinations(sel, 2):
            if face_of(c, d) or face_of(d, c):
                parent[find(c)] = find(d)
        return len({find(c) for c in sel})

    A = [c for c in cells if inA[c]]
    B = [c for c in cells if not inA[c]]
    return len(A) > 0 and len(B) > 0 and n_comp(A) == 1 and n_comp(B) == 1


def _params(ora, shape, topo=0):
    return ora.make_params(shape, 4.0, 0.1, topo=topo)


# ------------------------------------------------------------- simple points

@pytest.mark.parametrize("seed", range(6))
def test_simple_2d_equals_global_component_counts(ora, seed):
    """2D (8/4): toggling a pixel keeps the number of 8-components of the
    region and of 4-components of its complement iff the pixel is simple."""
    rng = np.random.default_rng(seed)
    shape = (9, 11)
    L = (rng.random(shape) < 0.3 + 0.08 * seed).astype(np.int32)
    P = _params(ora, shape)
    for i in range(L.size):
        X0 = (L == 1).copy()
        X0.flat[i] = False
        X1 = X0.copy()
        X1.flat[i] = True
        same = _topo(X0, True) == _topo(X1, True)
        assert ora.simple(P, L, i, 1) == same, (seed, i)


def test_simple_3d_equals_attachment_contractible(ora):
    """3D (26/6): the local test agrees with contractibility of the closed
    cube's attachment, on random neighbourhoods of every density."""
    rng = np.random.default_rng(7)
    P = _params(ora, (3, 3, 3))
    n_simple = 0
    for k in range(2500):
        p = (k % 25 + 0.5) / 25.0
        nb = rng.random((3, 3, 3)) < p
        L = nb.astype(np.int32)
        got = ora.simple(P, L, 13, 1)
        want = _attachment_contractible(nb)
        assert got == want, (k, nb.astype(int).tolist())
        n_simple += got
    assert 200 < n_simple < 2300  # both outcomes well represented


def test_simple_3d_at_the_border_equals_attachment(ora):
    """Voxels on the image border: missing neighbours belong to no region."""
    rng = np.random.default_rng(8)
    P = _params(ora, (3, 3, 3))
    for k in range(600):
        L = (rng.random((3, 3, 3)) < 0.2 + 0.6 * (k % 7) / 6).astype(np.int32)
        corner = tuple(rng.integers(0, 3, 3))
        i = int(np.ravel_multi_index(corner, L.shape))
        nb = np.zeros((3, 3, 3), bool)
        for o in itertools.product((-1, 0, 1), repeat=3):
            q = tuple(c + d for c, d in zip(corner, o))
            if o != (0, 0, 0) and all(0 <= v < 3 for v in q):
                nb[o[0] + 1, o[1] + 1, o[2] + 1] = L[q] == 1
        assert ora.simple(P, L, i, 1) == _attachment_contractible(nb), (k, corner)


@pytest.mark.parametrize("seed", range(3))
def test_simple_3d_toggle_preserves_global_topology(ora, seed):
    """Every simple toggle keeps components, complement components and the
    Euler characteristic of the region."""
    rng = np.random.default_rng(20 + seed)
    shape = (5, 6, 5)
    L = (rng.random(shape) < 0.35 + 0.1 * seed).astype(np.int32)
    P = _params(ora, shape)
    checked = 0
    for i in range(L.size):
        if not ora.simple(P, L, i, 1):
            continue
        X0 = (L == 1).copy()
        X0.flat[i] = False
        X1 = X0.copy()
        X1.flat[i] = True
        assert _topo(X0, True) == _topo(X1, True), (seed, i)
        checked += 1
    assert checked > 10


def test_simple_hand_cases(ora):
    P2 = _params(ora, (5, 5))
    L = np.zeros((5, 5), np.int32)
    L[2, 2] = 1
    assert not ora.simple(P2, L, 12, 1)          # removing an isolated pixel
    assert ora.simple(P2, L, 11, 1)              # growing it by one
    L[1:4, 1:4] = 1
    assert not ora.simple(P2, L, 12, 1)          # interior: removal makes a hole
    assert ora.simple(P2, L, 6, 1)               # corner of the square
    L = np.zeros((5, 5), np.int32)
    L[2, :] = 1
    assert not ora.simple(P2, L, 12, 1)          # middle of a line: split
    assert ora.simple(P2, L, 10, 1)              # its end
    L = np.zeros((5, 5), np.int32)
    L[2, 0:2] = 1
    L[2, 3:5] = 1
    assert not ora.simple(P2, L, 12, 1)          # adding the gap merges two pieces
    P3 = _params(ora, (3, 3, 3))
    L = np.ones((3, 3, 3), np.int32)
    assert not ora.simple(P3, L, 13, 1)          # removal makes a cavity
    L = np.zeros((3, 3, 3), np.int32)
    L[1, 1, :] = 1
    assert not ora.simple(P3, L, 13, 1)          # middle of a rod
    L[1, :, :] = 1
    L[1, 1, 1] = 0
    assert not ora.simple(P3, L, 13, 1)          # plate with a hole: filling it kills a tunnel


# ------------------------------------------------------------ ranked acceptance

def _state(ora, w, mode):
    P = ora.params_of(w)
    L1, d = ora.step(P, w.image, w.labels, mode)
    g = d["dE_h1"] if mode == ora.MODE_SOBOLEV else d["dE_l2"]
    return P, L1, d["lin"], d["a"], d["b"], g


@pytest.mark.parametrize("shape,blobs", [((23, 29), True), ((19, 17), False), ((9, 11, 10), True)])
def test_ranked_without_control_is_simultaneous(ora, shape, blobs):
    w = W.random_multilabel(3, shape, n_labels=4, blobs=blobs)
    for mode in (ora.MODE_L2, ora.MODE_SOBOLEV):
        P, L1, lin, a, b, g = _state(ora, w, mode)
        L2, done, m = ora.accept_ranked(P, w.labels, lin, a, b, g, ora.TOPO_OFF)
        assert np.array_equal(L1, L2)
        assert m == int((L1 != w.labels).sum())


@pytest.mark.parametrize("shape", [(23, 29), (9, 11, 10)])
def test_ranked_result_is_order_independent(ora, shape):
    """Ranking makes the result independent of the particles' indexing order."""
    w = W.random_multilabel(5, shape, n_labels=3, blobs=True)
    P, _, lin, a, b, g = _state(ora, w, ora.MODE_SOBOLEV)
    ref, done, _ = ora.accept_ranked(P, w.labels, lin, a, b, g, ora.TOPO_SIMPLE)
    rng = np.random.default_rng(1)
    for _ in range(3):
        p = rng.permutation(len(lin))
        L2, done2, _ = ora.accept_ranked(P, w.labels, lin[p], a[p], b[p], g[p], ora.TOPO_SIMPLE)
        assert np.array_equal(ref, L2)
        assert np.array_equal(done[p], done2)


@pytest.mark.parametrize("shape,n_labels", [((40, 48), 3), ((12, 13, 14), 3)])
def test_controlled_run_preserves_every_region(ora, shape, n_labels):
    """Several controlled iterations: no foreground region changes its
    component count, its complement's, or its Euler characteristic."""
    w = W.random_multilabel(11, shape, n_labels=n_labels, blobs=True, lam=0.05)
    P = ora.params_of(w)
    P.topo = ora.TOPO_SIMPLE
    L = w.labels.copy()
    before = {l: _topo(L == l, True) for l in range(1, n_labels)}
    moved = 0
    for _ in range(6):
        L_next, d = ora.step(P, w.image, L, ora.MODE_L2, want_arrays=False)
        moved += d["flips"]
        L = L_next
        for l in range(1, n_labels):
            assert _topo(L == l, True) == before[l], l
    assert moved > 0


def test_controlled_step_refuses_a_merge(ora):
    """Two label-1 bars one pixel apart: the gap pixel's move 0 -> 1 ranks
    first but would merge them, so it is refused; a free run takes it."""
    L = np.zeros((7, 9), np.int32)
    L[3, 1:4] = 1
    L[3, 5:8] = 1
    P = _params(ora, L.shape)
    gap = int(np.ravel_multi_index((3, 4), L.shape))
    tip = int(np.ravel_multi_index((2, 2), L.shape))
    lin = np.array([gap, tip], np.int64)
    a = np.array([0, 0], np.int32)
    b = np.array([1, 1], np.int32)
    g = np.array([-2.0, -1.0])
    Lc, done, m = ora.accept_ranked(P, L, lin, a, b, g, ora.TOPO_SIMPLE)
    assert done.tolist() == [False, True] and m == 1
    Lf, done, m = ora.accept_ranked(P, L, lin, a, b, g, ora.TOPO_OFF)
    assert done.tolist() == [True, True] and m == 2


def test_rank_decides_between_neighbours(ora):
    """Two moves that each keep the region intact alone but split it together:
    the better-ranked one runs, the other is refused; swapping the gradients
    swaps the outcome."""
    L = np.zeros((5, 6), np.int32)
    L[1:3, 1:5] = 1            # a 2 x 4 bar; emptying column 2 splits it
    P = _params(ora, L.shape)
    p1 = int(np.ravel_multi_index((1, 2), L.shape))
    p2 = int(np.ravel_multi_index((2, 2), L.shape))
    lin = np.array([p1, p2], np.int64)
    a = np.array([1, 1], np.int32)
    b = np.array([0, 0], np.int32)
    _, d1, _ = ora.accept_ranked(P, L, lin, a, b, np.array([-3.0, -1.0]), ora.TOPO_SIMPLE)
    _, d2, _ = ora.accept_ranked(P, L, lin, a, b, np.array([-1.0, -3.0]), ora.TOPO_SIMPLE)
    assert d1.tolist() == [True, False] and d2.tolist() == [False, True]
    # equal gradients: the smaller pixel index ranks first
    _, d3, _ = ora.accept_ranked(P, L, lin, a, b, np.array([-2.0, -2.0]), ora.TOPO_SIMPLE)
    assert d3.tolist() == [True, False]
    # a ring: removing a pixel opens the hole to the outside (not simple)
    R = np.zeros((5, 5), np.int32)
    R[1:4, 1:4] = 1
    R[2, 2] = 0
    q1 = int(np.ravel_multi_index((1, 2), R.shape))
    q2 = int(np.ravel_multi_index((3, 2), R.shape))
    lin = np.array([q1, q2], np.int64)
    PR = _params(ora, R.shape)
    _, d, m = ora.accept_ranked(PR, R, lin, a, b, np.array([-3.0, -1.0]), ora.TOPO_SIMPLE)
    assert m == 0
    _, d, m = ora.accept_ranked(PR, R, lin, a, b, np.array([-3.0, -1.0]), ora.TOPO_OFF)
    assert m == 2
