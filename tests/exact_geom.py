"""Exact rational plane geometry (fractions.Fraction) used to pin the oracle.

Nothing here imports the oracle or the GPU library: these are independent
textbook routines on the exact binary values of the fp32 inputs.
"""
from fractions import Fraction

import numpy as np


def fpoly(xy, n=None):
    xy = np.asarray(xy)
    n = xy.shape[0] if n is None else n
    return [(Fraction(float(xy[k, 0])), Fraction(float(xy[k, 1]))) for k in range(n)]


def orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def meet(a, b, c, d):
    """Meeting point of line ab and line cd (not parallel), exact."""
    e = (b[0] - a[0], b[1] - a[1])
    f = (d[0] - c[0], d[1] - c[1])
    den = e[0] * f[1] - e[1] * f[0]
    t = ((c[0] - a[0]) * f[1] - (c[1] - a[1]) * f[0]) / den
    return (a[0] + t * e[0], a[1] + t * e[1])


def clip(P, Q):
    """Sutherland-Hodgman: P clipped by the closed left half-planes of Q's edges."""
    out = list(P)
    n2 = len(Q)
    for j in range(n2):
        a, b = Q[j], Q[(j + 1) % n2]
        if not out:
            break
        cur, out = out, []
        for k in range(len(cur)):
            s, e = cur[k], cur[(k + 1) % len(cur)]
            ds, de = orient(a, b, s), orient(a, b, e)
            if ds >= 0:
                out.append(s)
            if (ds >= 0) != (de >= 0):
                t = ds / (ds - de)
                out.append((s[0] + t * (e[0] - s[0]), s[1] + t * (e[1] - s[1])))
    # drop repeated points
    res = []
    for p in out:
        if not res or res[-1] != p:
            res.append(p)
    while len(res) > 1 and res[0] == res[-1]:
        res.pop()
    return res


def area(poly):
    s = Fraction(0)
    n = len(poly)
    for k in range(n):
        a, b = poly[k], poly[(k + 1) % n]
        s += a[0] * b[1] - a[1] * b[0]
    return s / 2


def vertex_from_code(P, Q, code):
    """The exact point a provenance code names (P vertex, Q vertex or the
    crossing of P edge i with Q edge j)."""
    n1, n2 = len(P), len(Q)
    if code < 0x10:
        return P[code]
    if code < 0x40:
        return Q[code & 0x0F]
    i, j = (code >> 3) & 7, code & 7
    return meet(P[i], P[(i + 1) % n1], Q[j], Q[(j + 1) % n2])


def classify(P, Q, v):
    """Set of codes that could name the exact point v (used on generic inputs,
    where exactly one applies)."""
    n1, n2 = len(P), len(Q)
    codes = set()
    for i in range(n1):
        if P[i] == v:
            codes.add(i)
    for j in range(n2):
        if Q[j] == v:
            codes.add(0x10 | j)
    for i in range(n1):
        for j in range(n2):
            a, b = P[i], P[(i + 1) % n1]
            c, d = Q[j], Q[(j + 1) % n2]
            if orient(a, b, v) == 0 and orient(c, d, v) == 0:
                # on both edges' segments
                if (min(a[0], b[0]) <= v[0] <= max(a[0], b[0]) and
                        min(a[1], b[1]) <= v[1] <= max(a[1], b[1]) and
                        min(c[0], d[0]) <= v[0] <= max(c[0], d[0]) and
                        min(c[1], d[1]) <= v[1] <= max(c[1], d[1])):
                    codes.add(0x40 | (i << 3) | j)
    return codes
