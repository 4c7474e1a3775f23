"""Global topological invariants of a binary region, for tests: components
of the region (full adjacency), components of its complement (face adjacency,
the outside of the image counted as complement) and the Euler characteristic
of the union of the closed unit squares / cubes."""
import itertools

import numpy as np
from scipy import ndimage


def n_fg(X):
    """Components of X under full (8 / 26) adjacency."""
    return ndimage.label(X, structure=np.ones((3,) * X.ndim, bool))[1]


def n_bg(X):
    """Components of the complement under face (4 / 6) adjacency, the outside
    of the image included as background (one layer of padding)."""
    Y = np.pad(~X, 1, constant_values=True)
    return ndimage.label(Y, structure=ndimage.generate_binary_structure(X.ndim, 1))[1]


def euler(X):
    """Euler characteristic of the union of the closed unit squares / cubes of X."""
    X = np.pad(X, 1).astype(bool)
    nd = X.ndim
    chi = 0
    # a k-cell of the grid complex is present when any pixel containing it is;
    # enumerate cells by which axes they extend along
    for ext in itertools.product((0, 1), repeat=nd):
        dim = sum(ext)
        # cell at lattice point v extending along axes with ext=1: contained in
        # pixels v - s for s in {0,1} on non-extended axes, s = 0 on extended axes
        shape = X.shape
        present = np.zeros(tuple(n + 1 for n in shape), bool)
        for s in itertools.product(*[(0, 1) if e == 0 else (0,) for e in ext]):
            sl_dst = tuple(slice(si, si + n) for si, n in zip(s, shape))
            present[sl_dst] |= X
        chi += (-1) ** dim * int(present.sum())
    return chi


def topo(X, with_euler=True):
    t = (n_fg(X), n_bg(X))
    return t + ((euler(X),) if with_euler else ())
