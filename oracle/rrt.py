"""Plain-Python RRT in the plane -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The planner's main thread of Sec. 3.3 in its simplest form, written out loop by loop
so that a run of the library's RRT can be replayed on the same sequence of samples:
each iteration takes the next sample, finds the nearest tree node (squared distance,
ties to the lowest index), steers at most `step` toward the sample, and adds the new
node if the edge misses every (closed) disc; the run stops once a new node within
`goal_tol` of the goal connects to the goal by a free edge (the goal is then added as
the last node), or when the samples run out.  Distances and the steering step are
evaluated in double precision from the single-precision values and the new node is
stored in single precision.
"""
from __future__ import annotations

import math

import numpy as np


def f32(v: float) -> float:
    """Round a Python float to the nearest single-precision value."""
    return float(np.float32(v))


def segment_hits_disc(ax, ay, bx, by, cx, cy, r) -> bool:
    """True iff the closed disc (c, r) meets the segment [a, b]: the closest point of
    the segment to c is a + t (b - a), t the clamped projection parameter."""
    dx, dy = bx - ax, by - ay
    len2 = dx * dx + dy * dy
    t = 0.0
    if len2 > 0.0:
        t = ((cx - ax) * dx + (cy - ay) * dy) / len2
        t = min(max(t, 0.0), 1.0)
    px, py = ax + t * dx, ay + t * dy
    ex, ey = cx - px, cy - py
    return ex * ex + ey * ey <= r * r


def segment_free(discs, ax, ay, bx, by) -> bool:
    cx, cy, rr = discs
    for k in range(len(rr)):
        if segment_hits_disc(ax, ay, bx, by, float(cx[k]), float(cy[k]), float(rr[k])):
            return False
    return True


def rrt_replay(samples, start, goal, step, goal_tol, discs):
    """Run the RRT on the given [k][2] samples; returns (nodes [m][2] float32,
    parents [m], solved, iterations used)."""
    step, goal_tol = f32(step), f32(goal_tol)
    nodes = [(f32(start[0]), f32(start[1]))]
    parents = [-1]
    gx0, gy0 = f32(goal[0]), f32(goal[1])
    solved, it = False, 0
    for it in range(1, len(samples) + 1):
        qx, qy = f32(samples[it - 1][0]), f32(samples[it - 1][1])
        best, bd = 0, 0.0
        for j, (nx, ny) in enumerate(nodes):
            dx, dy = qx - nx, qy - ny
            d2 = dx * dx + dy * dy
            if j == 0 or d2 < bd:
                best, bd = j, d2
        px, py = nodes[best]
        newx, newy = qx, qy
        dist = math.sqrt(bd)
        if dist > step:
            newx = px + step * ((qx - px) / dist)
            newy = py + step * ((qy - py) / dist)
        fx, fy = f32(newx), f32(newy)
        if not segment_free(discs, px, py, fx, fy):
            continue
        nodes.append((fx, fy))
        parents.append(best)
        added = len(nodes) - 1
        ex, ey = gx0 - fx, gy0 - fy
        if goal_tol >= 0 and ex * ex + ey * ey <= goal_tol * goal_tol and \
                segment_free(discs, fx, fy, gx0, gy0):
            nodes.append((gx0, gy0))
            parents.append(added)
            solved = True
            break
    return np.array(nodes, dtype=np.float32), np.array(parents, dtype=np.int32), solved, it
