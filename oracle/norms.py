"""Error norms of Section 5: volume-weighted L1 and L2 over the non-empty
cells normalised by the domain area, and the maximum over non-empty cells."""
import numpy as np


def norms(values, volumes):
    """(L1, L2, Linf) of cell values; ``volumes`` are the cut-cell volumes
    (any common scale), zero on empty cells."""
    v = np.asarray(values, dtype=float).ravel()
    w = np.asarray(volumes, dtype=float).ravel()
    ne = w > 0
    tot = w[ne].sum()
    e = np.abs(v[ne])
    return float(np.sum(w[ne] * e) / tot), float(np.sqrt(np.sum(w[ne] * e * e) / tot)), float(e.max())
