"""Dense, definition-level helpers for tests (not the oracle, not the HIP path).

Everything here is written straight from the paper's definitions with dense
numpy/scipy calls, so that tests can pin the oracle against something other
than itself.
"""
import numpy as np


def incidence(n, tail, head):
    """A[i, l] = +1 if edge l enters i, -1 if it leaves i (Section 1.1, "Network")."""
    m = len(tail)
    A = np.zeros((n, m))
    A[np.asarray(head), np.arange(m)] = 1.0
    A[np.asarray(tail), np.arange(m)] = -1.0
    return A


def weights_matrix(inst):
    """(n, n) matrix with entry (i, j) = weight of the traffic from j to i."""
    return np.asarray(inst.w).reshape(inst.n, inst.n).T


def util(inst, s, w):
    """u(s): w log s, w s^gamma, or the alpha-fair w s^(1-alpha)/(1-alpha) (alpha in inst.gamma)."""
    if inst.utility == 0:
        return w * np.log(s)
    if inst.utility == 1:
        return w * s ** inst.gamma
    a = inst.gamma
    return w * s ** (1.0 - a) / (1.0 - a)


def dutil(inst, s, w):
    if inst.utility == 0:
        return w / s
    if inst.utility == 1:
        return w * inst.gamma * s ** (inst.gamma - 1.0)
    return w * s ** (-inst.gamma)


def offdiag_mask(n):
    return ~np.eye(n, dtype=bool)
