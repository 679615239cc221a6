"""Exact rational brute-force coverage for tiny images (test infrastructure only).

Independent of tko.c: no orientation swap, no bias trick.  A pixel centre is
inside a triangle when, for every edge, it lies strictly on the side of the
opposite vertex, or exactly on the edge line of an edge that is a "top" edge
(horizontal, triangle below it in the y-down image) or a "left" edge (the
triangle lies to the right of it).  This is the usual top-left fill rule stated
geometrically; degenerate triangles cover nothing.
"""
from __future__ import annotations

from fractions import Fraction


def _cross(ax, ay, bx, by):
    return ax * by - ay * bx


def _edge_ok(v0, v1, w, p) -> bool:
    ex, ey = v1[0] - v0[0], v1[1] - v0[1]
    s_w = _cross(ex, ey, w[0] - v0[0], w[1] - v0[1])
    s_p = _cross(ex, ey, p[0] - v0[0], p[1] - v0[1])
    if s_p != 0:
        return (s_p > 0) == (s_w > 0)
    if ey == 0:                      # horizontal: top edge iff the triangle is below
        return w[1] > v0[1]
    # left edge iff the opposite vertex is to the right of the edge line at its height
    x_line = Fraction(v0[0]) + Fraction(w[1] - v0[1]) * Fraction(ex, ey)
    return w[0] > x_line


def covers(tri, p) -> bool:
    a, b, c = tri
    if _cross(b[0] - a[0], b[1] - a[1], c[0] - a[0], c[1] - a[1]) == 0:
        return False
    return _edge_ok(a, b, c, p) and _edge_ok(b, c, a, p) and _edge_ok(c, a, b, p)


def coverage_counts(snapped, flags, triangles, width, height):
    """Per-pixel number of covering triangles, [H][W] list of ints.
    snapped: Q8 integer vertex coordinates (pixel centre of (x, y) is
    (256x+128, 256y+128))."""
    out = [[0] * width for _ in range(height)]
    tris = []
    for t in triangles:
        i0, i1, i2 = (int(v) for v in t)
        if flags[i0] or flags[i1] or flags[i2]:
            continue
        tris.append(tuple((int(snapped[i][0]), int(snapped[i][1])) for i in (i0, i1, i2)))
    for y in range(height):
        for x in range(width):
            p = (256 * x + 128, 256 * y + 128)
            out[y][x] = sum(1 for tri in tris if covers(tri, p))
    return out
