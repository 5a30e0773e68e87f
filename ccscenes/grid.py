"""Structured simplicial grids.

Vertex numbering is lexicographic with x fastest: id = i + nx*(j + ny*k).
2D cells split into two counter-clockwise triangles; 3D cells split into the
six Kuhn tetrahedra, one per permutation of the axes, each following the
monotone lattice path 000 -> e_a -> e_a+e_b -> 111.  Tetrahedra of odd
permutations have their last two vertices swapped so that every element has a
positive signed volume.  Element id = 2*cell + t (2D) or 6*cell + p (3D) with
cell = i + (nx-1)*(j + (ny-1)*k).
"""
import itertools

import numpy as np


def grid2d(nx, ny, lx=1.0, ly=1.0):
    """Return (X (n,2) float64, tris (m,3) int32) for an nx-by-ny vertex grid."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    X = np.stack([i.ravel() * (lx / (nx - 1)), j.ravel() * (ly / (ny - 1))], axis=1)
    tris = []
    for cj in range(ny - 1):
        for ci in range(nx - 1):
            c00 = ci + nx * cj
            c10 = ci + 1 + nx * cj
            c11 = ci + 1 + nx * (cj + 1)
            c01 = ci + nx * (cj + 1)
            tris.append((c00, c10, c11))
            tris.append((c00, c11, c01))
    return X.astype(np.float64), np.asarray(tris, dtype=np.int32)


_PERMS = list(itertools.permutations((0, 1, 2)))


def _perm_parity(p):
    inv = sum(1 for a in range(3) for b in range(a + 1, 3) if p[a] > p[b])
    return inv % 2


def grid3d(nx, ny, nz, lx, ly, lz):
    """Return (X (n,3) float64, tets (m,4) int32) for an nx*ny*nz vertex grid."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([i.ravel() * (lx / (nx - 1)),
                  j.ravel() * (ly / (ny - 1)),
                  k.ravel() * (lz / (nz - 1))], axis=1)

    def vid(a, b, c):
        return a + nx * (b + ny * c)

    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1),
                             indexing="ij")
    # cell id = i + (nx-1)*(j + (ny-1)*k): order cells with i fastest
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    ncell = ci.size
    tets = np.empty((ncell, 6, 4), dtype=np.int32)
    for pi, p in enumerate(_PERMS):
        off = [0, 0, 0]
        path = [tuple(off)]
        for ax in p:
            off[ax] += 1
            path.append(tuple(off))
        ids = [vid(ci + o[0], cj + o[1], ck + o[2]) for o in path]
        if _perm_parity(p):
            ids[2], ids[3] = ids[3], ids[2]
        tets[:, pi, :] = np.stack(ids, axis=1)
    return X.astype(np.float64), tets.reshape(-1, 4)
