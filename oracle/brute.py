"""Brute-force point-tuple counts that pin the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see oracle/conker.py).

The estimator of Eq. ksin_delta sums, over every grid cell x taken as vertex 0,
the signed tracer content of x times the content of each shell around x.  With
the cell content F(x) = sum of signed weights u_p of the tracers in x, that is a
sum over tuples of tracers (p_0, p_1, ..., p_{n-1}):

    W_n(a_1..a_{n-1}) = sum u_{p_0} u_{p_1} ... u_{p_{n-1}}
                        [cell(p_i) - cell(p_0) lies on shell a_i for every i].

These routines evaluate that tuple sum by explicit enumeration over the tracers
themselves, with no grid, FFT or map: the shell test is done on the integer
separation of the two cells, as "nearest integer of |d| equals m" (integer
radii only, where the shell r - 1/2 <= |d| < r + 1/2 has no ties).
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence

import numpy as np


def _cells(pos, origin, cell, dims):
    """NGP cells (float64 floor) and inside mask, written independently of the oracle."""
    out = []
    inside = []
    o = [float(v) for v in origin]
    for p in np.asarray(pos, dtype=np.float32):
        c = [int(math.floor((float(p[k]) - o[k]) / float(cell))) for k in range(3)]
        ok = all(0 <= c[k] < int(dims[k]) for k in range(3))
        out.append(c)
        inside.append(ok)
    return np.array(out, dtype=np.int64).reshape(-1, 3), np.array(inside, dtype=bool)


def shell_of(d: Sequence[int]) -> int:
    """Nearest integer to |d| for an integer separation vector (no ties occur)."""
    d2 = int(d[0]) ** 2 + int(d[1]) ** 2 + int(d[2]) ** 2
    return int(math.floor(math.sqrt(d2) + 0.5))


def separation(ci, cj, dims, periodic: bool):
    d = [int(cj[k]) - int(ci[k]) for k in range(3)]
    if periodic:
        for k in range(3):
            n = int(dims[k])
            d[k] = (d[k] + n // 2) % n - n // 2
    return d


def signed_tracers(data_pos, rand_pos, origin, cell, dims, data_w=None, rand_w=None):
    """In-grid tracers with signed weights u = +w (data) and -alpha w (randoms).

    Returns (cells [M, 3], u [M], alpha, cells_rand, w_rand)."""
    cd, ind = _cells(data_pos, origin, cell, dims)
    cr, inr = _cells(rand_pos, origin, cell, dims)
    wd = np.ones(len(cd)) if data_w is None else np.asarray(data_w, np.float32).astype(np.float64)
    wr = np.ones(len(cr)) if rand_w is None else np.asarray(rand_w, np.float32).astype(np.float64)
    cd, wd = cd[ind], wd[ind]
    cr, wr = cr[inr], wr[inr]
    alpha = float(wd.sum()) / float(wr.sum())
    cells = np.concatenate([cd, cr])
    u = np.concatenate([wd, -alpha * wr])
    return cells, u, alpha, cr, wr


def tuple_sum(cells, u, shells: Sequence[int], dims, periodic: bool) -> float:
    """Explicit sum over all tracer tuples (p_0, ..., p_{n-1}) for one radius tuple.

    O(M^n): only for a few dozen tracers.
    """
    M = len(u)
    total = 0.0
    for p0 in range(M):
        for rest in itertools.product(range(M), repeat=len(shells)):
            ok = True
            for a, pi in zip(shells, rest):
                if shell_of(separation(cells[p0], cells[pi], dims, periodic)) != a:
                    ok = False
                    break
            if ok:
                prod = u[p0]
                for pi in rest:
                    prod *= u[pi]
                total += prod
    return total


def shell_counts(cells, u, dims, periodic: bool, m_max: int) -> np.ndarray:
    """g[p, m] = sum of u_q over tracers q whose cell lies on shell m around p's cell.

    O(M^2) pair loop written with NumPy broadcasting; used for larger tracer sets.
    """
    cells = np.asarray(cells, dtype=np.int64)
    d = cells[None, :, :] - cells[:, None, :]
    if periodic:
        n = np.asarray(dims, dtype=np.int64)
        d = (d + n // 2) % n - n // 2
    dist = np.sqrt((d.astype(np.float64) ** 2).sum(axis=-1))
    m = np.floor(dist + 0.5).astype(np.int64)
    g = np.zeros((len(u), m_max + 1))
    for k in range(m_max + 1):
        g[:, k] = ((m == k) * u[None, :]).sum(axis=1)
    return g


def pair_factorised_sum(cells, u, shells: Sequence[int], dims, periodic: bool) -> float:
    """Same tuple sum, factorised over p_1..p_{n-1} given p_0 (exact rearrangement)."""
    g = shell_counts(cells, u, dims, periodic, max(shells))
    prod = np.asarray(u, dtype=np.float64).copy()
    for a in shells:
        prod = prod * g[:, a]
    return float(prod.sum())


def cross_shell_counts(cells0, cells1, v1, dims, periodic: bool, m_max: int) -> np.ndarray:
    """g[p, m] = sum of v_q over tracers q of set 1 on shell m around tracer p of set 0."""
    c0 = np.asarray(cells0, dtype=np.int64)
    c1 = np.asarray(cells1, dtype=np.int64)
    d = c1[None, :, :] - c0[:, None, :]
    if periodic:
        n = np.asarray(dims, dtype=np.int64)
        d = (d + n // 2) % n - n // 2
    m = np.floor(np.sqrt((d.astype(np.float64) ** 2).sum(axis=-1)) + 0.5).astype(np.int64)
    g = np.zeros((len(c0), m_max + 1))
    for k in range(m_max + 1):
        g[:, k] = ((m == k) * np.asarray(v1)[None, :]).sum(axis=1)
    return g


def cross_tuple_sum(cells0, u0, cells1, v1, shells: Sequence[int], dims, periodic: bool) -> float:
    """sum over tracer tuples (p_0 from set 0; p_1 .. p_{n-1} from set 1) of
    u_{p_0} v_{p_1} ... v_{p_{n-1}} [cell(p_i) - cell(p_0) on shell a_i]."""
    g = cross_shell_counts(cells0, cells1, v1, dims, periodic, max(shells))
    prod = np.asarray(u0, dtype=np.float64).copy()
    for a in shells:
        prod = prod * g[:, a]
    return float(prod.sum())
