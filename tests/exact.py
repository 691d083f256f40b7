"""Exact-rational geometry used to pin the oracle (brute force, no rounding).

Every double converts exactly to a Fraction, so these predicates decide
containment with no rounding at all.  They are a textbook orientation test,
evaluated independently of the oracle's floating-point expressions.
"""
from fractions import Fraction

import numpy as np


def orient(a, b, c):
    """Exact twice-signed-area of (a, b, c): > 0 for a left turn."""
    ax, ay = Fraction(float(a[0])), Fraction(float(a[1]))
    bx, by = Fraction(float(b[0])), Fraction(float(b[1]))
    cx, cy = Fraction(float(c[0])), Fraction(float(c[1]))
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def contains_closed(xy, tri_row, p):
    """Exact: does the closed triangle (any orientation) contain p?"""
    a, b, c = xy[tri_row[0]], xy[tri_row[1]], xy[tri_row[2]]
    s = orient(a, b, c)
    o1, o2, o3 = orient(a, b, p), orient(b, c, p), orient(c, a, p)
    if s > 0:
        return o1 >= 0 and o2 >= 0 and o3 >= 0
    return o1 <= 0 and o2 <= 0 and o3 <= 0


def containing_sets(xy, tri, pts):
    """For each point, the sorted list of triangles whose closed region holds it."""
    xy = np.asarray(xy)
    P = xy[tri]  # [nt, 3, 2]
    lo = P.min(axis=1)
    hi = P.max(axis=1)
    out = []
    for p in np.asarray(pts):
        cand = np.nonzero((lo[:, 0] <= p[0]) & (hi[:, 0] >= p[0]) & (lo[:, 1] <= p[1]) & (hi[:, 1] >= p[1]))[0]
        out.append([int(t) for t in cand if contains_closed(xy, tri[t], p)])
    return out


def edge_distance(xy, tri_row, p):
    """Euclidean distance (FP64) from p to the nearest of the triangle's edge segments."""
    best = np.inf
    for k in range(3):
        a = np.asarray(xy[tri_row[k]], dtype=np.float64)
        b = np.asarray(xy[tri_row[(k + 1) % 3]], dtype=np.float64)
        d = b - a
        t = np.clip(np.dot(np.asarray(p) - a, d) / np.dot(d, d), 0.0, 1.0)
        best = min(best, float(np.hypot(*(a + t * d - p))))
    return best


def edge_distances(xy, tri, hosts, pts):
    """Vectorised edge_distance over many (host, point) pairs."""
    xy = np.asarray(xy)
    pts = np.asarray(pts, dtype=np.float64)
    V = xy[tri[hosts]]  # [n, 3, 2]
    best = np.full(len(pts), np.inf)
    for k in range(3):
        a = V[:, k]
        b = V[:, (k + 1) % 3]
        d = b - a
        t = np.clip(np.einsum("ij,ij->i", pts - a, d) / np.einsum("ij,ij->i", d, d), 0.0, 1.0)
        q = a + t[:, None] * d
        best = np.minimum(best, np.hypot(*(q - pts).T))
    return best
