"""Pins of the oracle's plane RRT (the planner's main thread of Sec. 3.3, simplest
form): segment-disc geometry by closed forms, straight-line growth, a blocking wall."""
import math

import numpy as np

from oracle import rrt as R


def test_segment_disc_closed_forms():
    # horizontal segment y = 0 from x = 0 to 10; a disc at (5, d) of radius 1
    assert R.segment_hits_disc(0, 0, 10, 0, 5, 0.999, 1.0)
    assert R.segment_hits_disc(0, 0, 10, 0, 5, 1.0, 1.0)          # tangent: closed disc
    assert not R.segment_hits_disc(0, 0, 10, 0, 5, 1.001, 1.0)
    # beyond the end: distance to the endpoint (10, 0) is the nearest
    assert R.segment_hits_disc(0, 0, 10, 0, 10.6, 0.8, 1.0)      # |(0.6, 0.8)| = 1
    assert not R.segment_hits_disc(0, 0, 10, 0, 10.61, 0.8, 1.0)
    # a degenerate segment is a point
    assert R.segment_hits_disc(2, 2, 2, 2, 2.5, 2, 0.5)
    assert not R.segment_hits_disc(2, 2, 2, 2, 2.6, 2, 0.5)


def test_straight_line_growth_without_obstacles():
    no = (np.zeros(0), np.zeros(0), np.zeros(0))
    samples = np.tile([[10.0, 0.0]], (20, 1))
    nodes, parents, solved, it = R.rrt_replay(samples, (0, 0), (10, 0), 1.0, 0.5, no)
    # each sample adds one node a step further along the axis until the goal is in reach
    assert solved and it == 10
    assert np.allclose(nodes[:, 0], np.r_[np.arange(0, 11, 1.0), 10.0][:nodes.shape[0]])
    assert list(parents) == [-1] + list(range(len(parents) - 1))


def test_wall_blocks_edges():
    # a wall of discs on x = 5 between y = -10 and 10
    ys = np.arange(-10, 10.5, 0.5)
    discs = (np.full(ys.size, 5.0), ys, np.full(ys.size, 0.3))
    samples = np.tile([[9.0, 0.0]], (30, 1))
    nodes, _, solved, it = R.rrt_replay(samples, (0, 0), (9, 0), 1.0, 0.5, discs)
    assert not solved and it == 30
    assert nodes[:, 0].max() < 5.0 - 0.3
    # the same run without the wall reaches the goal
    no = (np.zeros(0), np.zeros(0), np.zeros(0))
    _, _, solved2, _ = R.rrt_replay(samples, (0, 0), (9, 0), 1.0, 0.5, no)
    assert solved2


def test_steer_length_is_the_step():
    no = (np.zeros(0), np.zeros(0), np.zeros(0))
    nodes, _, _, _ = R.rrt_replay([[3.0, 4.0]], (0, 0), (100, 100), 2.0, 0.1, no)
    assert math.isclose(math.hypot(*nodes[1]), 2.0, rel_tol=1e-7)
    assert math.isclose(nodes[1][1] / nodes[1][0], 4.0 / 3.0, rel_tol=1e-6)
