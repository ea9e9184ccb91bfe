"""Oracle: explicit 4x4 Dirac matrices and traces with contracted indices.

TEST INFRASTRUCTURE (see oracle/graphs.py).

A trace of a product of gamma matrices in which every Lorentz index occurs
exactly twice is evaluated by its definition: an explicit sum over the four
values of each index, with g = diag(1,-1,-1,-1) (Sec. II gives the metric and
the Clifford relation).  Products are formed left to right; an index axis is
summed as soon as its second occurrence has been multiplied in.  No 4D
contraction identity is used here, so this route is independent of any
symbolic reduction.
"""
from __future__ import annotations

import numpy as np

I4 = np.eye(4, dtype=complex)
_s = [np.array([[0, 1], [1, 0]], dtype=complex),
      np.array([[0, -1j], [1j, 0]], dtype=complex),
      np.array([[1, 0], [0, -1]], dtype=complex)]
Z2 = np.zeros((2, 2), dtype=complex)
GAMMA_UP = np.zeros((4, 4, 4), dtype=complex)
GAMMA_UP[0] = np.block([[np.eye(2), Z2], [Z2, -np.eye(2)]])
for k in range(3):
    GAMMA_UP[k + 1] = np.block([[Z2, _s[k]], [-_s[k], Z2]])
METRIC = np.array([1.0, -1.0, -1.0, -1.0])
GAMMA_LO = GAMMA_UP * METRIC[:, None, None]


def slash(vec_upper):
    """a-slash = a^mu gamma_mu for a contravariant 4-vector."""
    return np.einsum('m,mij->ij', np.asarray(vec_upper, dtype=complex), GAMMA_LO)


P_VEC = np.array([1.0, 0.0, 0.0, 0.0])      # external momentum, rest frame, m = 1
PSLASH = slash(P_VEC)
Q_DIRS = [np.eye(4)[i] for i in (1, 2, 3)]   # unit spacelike q, q^2 = -1


def trace_chain(factors):
    """Trace of a product.  factors: list of 4x4 arrays or ('idx', label).

    Each label must occur exactly twice.  Returns a complex number."""
    open_labels = []          # axis order of the leading tensor axes
    T = I4.copy()             # shape (4,)*len(open) + (4, 4)
    counts = {}
    for f in factors:
        if isinstance(f, tuple):
            lab = f[1]
            counts[lab] = counts.get(lab, 0) + 1
    for lab, c in counts.items():
        if c != 2:
            raise ValueError(f"index {lab} occurs {c} times")
    for f in factors:
        if not isinstance(f, tuple):
            T = T @ f
            continue
        lab = f[1]
        if lab not in open_labels:
            # new axis: T[..., nu, :, :] = T @ gamma^nu
            T = np.einsum('...ij,njk->...nik', T, GAMMA_UP)
            open_labels.append(lab)
        else:
            ax = open_labels.index(lab)
            nd = len(open_labels)
            # contract: sum_nu T[.., nu(ax), ..] @ gamma_nu
            Tm = np.moveaxis(T, ax, nd - 1)     # put label axis last before matrix dims
            T = np.einsum('...nij,njk->...ik', Tm, GAMMA_LO)
            open_labels.pop(ax)
    assert not open_labels
    return np.trace(T)


def exact_int(x, tol=1e-7):
    """Traces of integer-entry matrices are exact integers; check and round."""
    r = round(x.real)
    if abs(x.real - r) > tol or abs(x.imag) > tol:
        raise ValueError(f"non-integer trace {x}")
    return int(r)
