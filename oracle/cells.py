"""Cell binning of electrolyte sites: the integer reference.

The paper's timings list neighbour-list building as one of the four costs
of an MD step (Computational Efficiency subsection, Fig. 10).  The real-space
sums only need, for every site, the sites and electrode atoms within rcut;
binning the sites into cells provides that, the partners of a site lying in
the cells within reach(d) cells of its own along every axis.  The grid is a
property of the neighbour list, not of the method: any grid whose reach
covers rcut gives the same sums.

Definition used here (and required bit for bit of the GPU binning):

* n_d = max(1, floor(L_d / rcut)) cells along x and y (reach 1); along z
  the same, unless floor(L_z / rcut) >= 3: then n_z = floor(2 L_z / rcut),
  cells at least rcut/2 thick, reach 2;
* fractional coordinate f = x/L - floor(x/L), computed in double precision
  in exactly that order, cell index c_d = min(floor(f * n_d), n_d - 1);
* linear cell id (c_z * n_y + c_y) * n_x + c_x;
* cell_start[c] = number of sites in cells < c (length n_cells + 1);
* the sites of each cell are listed in increasing original index.
"""

from __future__ import annotations

import math

import numpy as np


def cell_grid(box, rcut):
    n = [max(1, int(math.floor(L / rcut))) for L in box]
    if n[2] >= 3:
        n[2] = int(math.floor(2.0 * box[2] / rcut))
    return tuple(n)


def cell_reach(box, rcut):
    """Cells searched on either side along each axis."""
    return (1, 1, 2 if int(math.floor(box[2] / rcut)) >= 3 else 1)


def cell_of(xyz, box, ncell):
    box = np.asarray(box, dtype=np.float64)
    c = []
    for d in range(3):
        t = xyz[d] / box[d]
        f = t - np.floor(t)
        c.append(np.minimum(np.floor(f * ncell[d]).astype(np.int64), ncell[d] - 1))
    return (c[2] * ncell[1] + c[1]) * ncell[0] + c[0]


def bin_sites(xyz, box, rcut):
    """Returns (cell_of_site, cell_start, order): order lists site indices cell by cell."""
    ncell = cell_grid(box, rcut)
    cid = cell_of(xyz, box, ncell)
    n_cells = ncell[0] * ncell[1] * ncell[2]
    counts = np.bincount(cid, minlength=n_cells)
    start = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    order = np.argsort(cid, kind="stable")
    return cid, start, order
