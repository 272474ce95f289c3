"""Pins of the oracle's Koch snowflake rule (sec. 4.4).

Checked against the closed-form area of the level-L snowflake, the paper's
triangle count for level 13, the outline's shoelace area, an independent
method on an independent rule (the edge integral of eq. nsli over the
outline polygon), and the six-fold symmetry of the domain (for L >= 1), which
the rule itself (built from the three-fold Omega_0) does not have.
"""
import math

import numpy as np
import pytest

import oracle

A0 = 3 * math.sqrt(3) / 4  # the equilateral triangle of side sqrt 3


def koch_area(L):
    return A0 * (1 + sum(3 * 4 ** (k - 1) / 9 ** k for k in range(1, L + 1)))


@pytest.mark.parametrize("L,p", [(0, [5]), (1, [7, 3]), (3, [9, 4, 2, 1]), (6, [4, 3, 3, 2, 2, 1, 1])])
def test_koch_area_and_symmetry_of_rule(L, p):
    x, y, w = oracle.quad_koch(L, p)
    assert len(x) == oracle.koch_size(L, p)
    assert abs(w.sum() - koch_area(L)) < 1e-14
    assert abs((w * x).sum()) < 1e-15 and abs((w * y).sum()) < 1e-15
    assert np.hypot(x, y).max() <= 1.0 + 1e-15
    vx, vy = oracle.koch_outline(L)
    assert len(vx) == 3 * 4 ** L
    shoelace = 0.5 * np.sum(vx * np.roll(vy, -1) - np.roll(vx, -1) * vy)
    assert abs(shoelace - koch_area(L)) < 1e-14
    # the limit area is 8/5 of the first triangle
    assert koch_area(40) == pytest.approx(1.6 * A0, rel=1e-13)


def test_koch_paper_triangle_count():
    # sec. 4.4: reaching level 13 takes 1 + 3 sum_{k<13} 4^k = 67,108,864 triangles
    assert oracle.koch_size(13, [1] * 14) == 67108864


def test_koch_direct_sum_vs_edge_integral_and_sixfold_symmetry():
    # level 3 at lambda z = 0.1 (Fresnel number 10): the areal sum over a
    # converged rule against the edge integral over the outline polygon
    L, lz = 3, 0.1
    x, y, w = oracle.quad_koch(L, [80, 40, 24, 14])
    vx, vy = oracle.koch_outline(L)
    B = oracle.boundary_polygon(vx, vy, 16)
    g = np.random.Generator(np.random.PCG64(9))
    xi = np.concatenate([g.uniform(-1.2, 1.2, 40), vx[:5]]); eta = np.concatenate([g.uniform(-1.2, 1.2, 40), vy[:5]])
    ua = oracle.fresnel_direct(x, y, w, 1.0, lz, xi, eta)
    ue = oracle.nsli(*B, 1.0, lz, xi, eta)
    assert np.abs(ua - ue).max() < 1e-11
    # the domain (L >= 1) is symmetric under rotation by 60 degrees
    c, s = math.cos(math.pi / 3), math.sin(math.pi / 3)
    ur = oracle.fresnel_direct(x, y, w, 1.0, lz, c * xi - s * eta, s * xi + c * eta)
    assert np.abs(ur - ua).max() < 1e-11
