"""Structured-grid counts of the colouring and of the R = 1 supports, and the
paper's normalised residual on a hand-worked case.

The colour counts follow from the greedy rule (free vertices in increasing
id, smallest colour unused by a neighbour sharing an element) applied to the
Kuhn-split grids; the R = 1 support sizes are the free 1-ring sizes.  Both
are counted here by the oracle and compared with totals computed
independently of it when the workloads were sized (a per-vertex walk of the
structured lattice).  A dropped Dirichlet face, a wrong tet split or a
colouring that ignores the element-sharing rule changes these numbers.
"""
import numpy as np
import pytest

from ccscenes import stretch2d, tet_bar, twist_beam
from oracle.basis import patch_supports
from oracle.colour import greedy_colour, is_valid_colouring
from oracle.fem import Problem
from oracle.solvers import paper_measure

# (scene, colour class sizes in colour order, total R = 1 support entries)
CASES = {
    "square17": (stretch2d, [72, 64, 56, 63], 1404),
    "bar21x6x6": (tet_bar, [90, 118, 128, 118, 81, 79, 60, 46], 7998),
    "beam81x21x21": (twist_beam, [4840, 5389, 4581, 5027, 4070, 3792, 3570, 3570], 458156),
}


@pytest.mark.parametrize("name", list(CASES))
def test_colour_class_sizes(name):
    make, sizes, _ = CASES[name]
    s = make()
    col = greedy_colour(s.n, s.elems, s.fixed)
    assert is_valid_colouring(s.elems, col)
    counts = np.bincount(col[col >= 0])
    assert counts.tolist() == sizes
    assert int((col < 0).sum()) == int(s.fixed.sum())


@pytest.mark.parametrize("name", list(CASES))
def test_r1_support_totals(name):
    make, _, total = CASES[name]
    p = Problem.from_scene(make())
    supp = patch_supports(p, 1)
    assert sum(len(supp[i]) for i in p.free) == total
    assert all(len(supp[i]) == 0 for i in np.flatnonzero(p.fixed))


def test_beam_sizes():
    """C3's vertex, element and free counts, and its largest 1-ring."""
    s = twist_beam()
    p = Problem.from_scene(s)
    assert (s.n, s.m, p.free.size) == (35721, 192000, 34839)
    supp = patch_supports(p, 1)
    assert max(len(supp[i]) for i in p.free) == 14


def test_paper_measure_hand_case():
    """|g| / (V n E), divided by h when dynamic (Results, Termination criteria),
    on one unit right tetrahedron: V = 1/6, n = 4."""
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    el = np.array([[0, 1, 2, 3]])
    g = np.zeros(12)
    g[0], g[4] = 3.0, 4.0                              # |g| = 5
    dyn = Problem(X, el, np.zeros(4, bool), 1000.0, 0.3, 1.0, np.zeros(3), 0.1, False)
    qs = Problem(X, el, np.zeros(4, bool), 1000.0, 0.3, 1.0, np.zeros(3), 0.1, True)
    # 5 / (1/6 * 4 * 1000) = 0.0075; dynamic: / h = 0.075
    assert paper_measure(qs, g) == pytest.approx(0.0075, rel=1e-14)
    assert paper_measure(dyn, g) == pytest.approx(0.075, rel=1e-14)
