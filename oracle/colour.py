"""Greedy graph colouring and colour-sorted orderings (exact integer work).

The paper notes that Gauss-Seidel-style sweeps use the most recent values
(Background, Coordinate Descent); a parallel Gauss-Seidel sweep needs a
colouring in which no two vertices of one colour share an element.  The paper
does not specify one; this package's reading:

* graph: free vertices, edge iff the two share an element; Dirichlet vertices
  get colour -1 and impose no constraint;
* visit free vertices in increasing id and give each the smallest colour not
  used by an already-coloured neighbour;
* vertex order: sorted by (colour, id), Dirichlet vertices last by id;
* element order: sorted by (smallest caller id among the element's free
  vertices, id); elements with no free vertex last by id (the elements of
  neighbouring vertices then sit together in memory).

Pins: tests/test_oracle_basis_colour.py -- validity on every scene, the colour
counts and class sizes of the structured grids, and agreement with a
brute-force "sequential greedy" restated as Jones-Plassmann rounds with
vertex-id priority.
"""
import numpy as np


def greedy_colour(n, elems, fixed):
    fixed = np.asarray(fixed).astype(bool)
    nbr = [set() for _ in range(n)]
    for e in np.asarray(elems):
        fe = [int(a) for a in e if not fixed[a]]
        for a in fe:
            for b in fe:
                if a != b:
                    nbr[a].add(b)
    col = -np.ones(n, dtype=np.int32)
    for i in range(n):
        if fixed[i]:
            continue
        used = {int(col[j]) for j in nbr[i] if col[j] >= 0}
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def is_valid_colouring(elems, colours):
    for e in np.asarray(elems):
        c = [int(colours[a]) for a in e if colours[a] >= 0]
        if len(c) != len(set(c)):
            return False
    return True


def layout(colours, elems):
    """Return (vperm, eperm): vperm[new] = old vertex id, eperm[new] = old element id."""
    colours = np.asarray(colours)
    n = colours.size
    free = colours >= 0
    key_c = np.where(free, colours, np.iinfo(np.int32).max)
    vperm = np.lexsort((np.arange(n), key_c)).astype(np.int32)
    big = np.iinfo(np.int64).max
    ne = np.where(free[elems], np.asarray(elems, dtype=np.int64), big)
    first = ne.min(axis=1)
    m = elems.shape[0]
    eperm = np.lexsort((np.arange(m), first)).astype(np.int32)
    return vperm, eperm
