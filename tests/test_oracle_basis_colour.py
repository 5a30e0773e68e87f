"""Pins of the oracle's perturbation basis and greedy colouring."""
import numpy as np
import pytest
import scipy.sparse.csgraph as csg
import scipy.sparse as sp

from ccscenes import stretch2d, tet_bar, twist_beam, batch_bars
from oracle.basis import exact_basis, patch_basis, patch_supports, rest_hessian
from oracle.colour import greedy_colour, is_valid_colouring, layout
from oracle.fem import Problem


def _small_problems():
    s2 = stretch2d(n=7)
    s3 = tet_bar(6, 3, 3, E=1e5)
    return [Problem.from_scene(s2), Problem.from_scene(s3)]


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("deformed", [False, True])
def test_exact_basis_definition(k, deformed):
    """H_CC U_i + H_Ci = 0 and U_i = -H_CC^{-1} H_Ci by a direct dense solve,
    with H at rest or at a deformed state (the restarted basis)."""
    p = _small_problems()[k]
    d = p.d
    x = None
    if deformed:
        x = p.X + 0.05 * np.random.default_rng(k).normal(size=p.X.shape)
        x[p.fixed] = p.X[p.fixed]
    ptr, idx, U = exact_basis(p, x)
    H = (p.hessian(p.X if x is None else x)).toarray()
    for i in p.free:
        fi = p.fidx[i]
        C = [j for j in range(p.free.size) if j != fi]
        cd = np.concatenate([np.arange(j * d, j * d + d) for j in C])
        idd = np.arange(fi * d, fi * d + d)
        Ui = U[ptr[i]:ptr[i + 1]].reshape(-1, d)
        assert list(idx[ptr[i]:ptr[i + 1]]) == list(p.free[C])
        res = H[np.ix_(cd, cd)] @ Ui + H[np.ix_(cd, idd)]
        assert np.max(np.abs(res)) <= 1e-10 * np.max(np.abs(H))
        Ud = -np.linalg.solve(H[np.ix_(cd, cd)], H[np.ix_(cd, idd)])
        assert np.max(np.abs(Ud - Ui)) <= 1e-9 * max(1.0, np.max(np.abs(Ud)))


@pytest.mark.parametrize("k", [0, 1])
def test_patch_basis_equals_exact_for_large_radius(k):
    p = _small_problems()[k]
    e = exact_basis(p)
    q = patch_basis(p, R=50)
    np.testing.assert_array_equal(e[0], q[0])
    np.testing.assert_array_equal(e[1], q[1])
    assert np.max(np.abs(e[2] - q[2])) <= 1e-9 * np.max(np.abs(e[2]))


@pytest.mark.parametrize("R", [1, 2])
def test_patch_supports_are_hop_balls(R):
    p = Problem.from_scene(tet_bar(6, 4, 3))
    supp = patch_supports(p, R)
    # hop distances on the free-vertex graph by a library shortest-path routine
    adj = p.adjacency()
    rows = [i for i in range(p.n) for _ in adj[i]]
    cols = [j for i in range(p.n) for j in adj[i]]
    G = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(p.n, p.n))
    D = csg.shortest_path(G, unweighted=True)
    for i in p.free:
        want = sorted(int(j) for j in np.flatnonzero(D[i] <= R) if j != i and not p.fixed[j])
        assert supp[i] == want
    for i in np.flatnonzero(p.fixed):
        assert supp[i] == []


def test_patch_basis_equilibrium():
    p = Problem.from_scene(tet_bar(6, 4, 3, E=1e6))
    d = p.d
    ptr, idx, U = patch_basis(p, R=1)
    H = rest_hessian(p).toarray()
    for i in p.free[::5]:
        C = p.fidx[idx[ptr[i]:ptr[i + 1]]]
        assert np.all(C >= 0)
        cd = (C[:, None] * d + np.arange(d)).ravel()
        idd = p.fidx[i] * d + np.arange(d)
        Ui = U[ptr[i]:ptr[i + 1]].reshape(-1, d)
        res = H[np.ix_(cd, cd)] @ Ui + H[np.ix_(cd, idd)]
        assert np.max(np.abs(res)) <= 1e-10 * np.max(np.abs(H))


def _jones_plassmann(n, elems, fixed):
    """Round-based colouring: an uncoloured vertex whose uncoloured neighbours
    all have larger ids takes the smallest colour unused by its neighbours."""
    nbr = [set() for _ in range(n)]
    for e in elems:
        for a in e:
            for b in e:
                if a != b and not fixed[a] and not fixed[b]:
                    nbr[a].add(int(b))
    col = -np.ones(n, dtype=np.int64)
    todo = {i for i in range(n) if not fixed[i]}
    while todo:
        ready = [i for i in todo if all(j > i or j not in todo for j in nbr[i])]
        for i in ready:
            used = {col[j] for j in nbr[i] if col[j] >= 0}
            c = 0
            while c in used:
                c += 1
            col[i] = c
        todo -= set(ready)
    return col


@pytest.mark.parametrize("scene", [stretch2d(), tet_bar(), tet_bar(9, 7, 6, clamp_face=3)])
def test_greedy_matches_jones_plassmann(scene):
    col = greedy_colour(scene.n, scene.elems, scene.fixed)
    jp = _jones_plassmann(scene.n, scene.elems, scene.fixed.astype(bool))
    np.testing.assert_array_equal(col, jp)
    assert is_valid_colouring(scene.elems, col)
    assert np.all((col < 0) == scene.fixed.astype(bool))


def test_colouring_valid_on_batch():
    for s in batch_bars(count=6):
        col = greedy_colour(s.n, s.elems, s.fixed)
        assert is_valid_colouring(s.elems, col)
        assert col.max() < 16


def test_layout_orderings():
    s = tet_bar(8, 4, 4)
    col = greedy_colour(s.n, s.elems, s.fixed)
    vperm, eperm = layout(col, s.elems)
    assert sorted(vperm) == list(range(s.n)) and sorted(eperm) == list(range(s.m))
    key = [(col[v] if col[v] >= 0 else 10 ** 9, v) for v in vperm]
    assert key == sorted(key)
    ekey = []
    for e in eperm:
        fr = [int(a) for a in s.elems[e] if col[a] >= 0]
        ekey.append((min(fr) if fr else 10 ** 12, e))
    assert ekey == sorted(ekey)


def test_state_basis_at_rest_is_rest_basis():
    p = _small_problems()[1]
    a, b = exact_basis(p), exact_basis(p, p.X.copy())
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    x = p.X + 0.05 * np.random.default_rng(3).normal(size=p.X.shape)
    x[p.fixed] = p.X[p.fixed]
    c = exact_basis(p, x)
    assert np.max(np.abs(c[2] - a[2])) > 1e-3 * np.max(np.abs(a[2]))


def test_exact_basis_rows_subset():
    """Rows computed for a subset of vertices equal the full basis's rows;
    the other rows are empty."""
    p = _small_problems()[1]
    full = exact_basis(p)
    sub = [int(p.free[0]), int(p.free[5]), int(p.free[-1])]
    part = exact_basis(p, verts=sub)
    for i in range(p.n):
        a0, a1 = full[0][i], full[0][i + 1]
        b0, b1 = part[0][i], part[0][i + 1]
        if i in sub:
            np.testing.assert_array_equal(part[1][b0:b1], full[1][a0:a1])
            np.testing.assert_array_equal(part[2][b0:b1], full[2][a0:a1])
        else:
            assert b1 == b0
