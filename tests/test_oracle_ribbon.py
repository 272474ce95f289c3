"""Pins of the oracle's ribbon quadrature (sec. 5, third construction): the
perturbed starshade as the ideal rule plus signed ribbons along the petal
edges.  Checked against what the construction must satisfy independently of
its own code: the zero perturbation, the ribbons' exact signed area, the
field of the independently built deformed-petal rule (orc_starshade with the
same coefficients, pinned by its own area and finite-difference tests), and
the second-order error of the line-integral form (mr = 0) in the ribbon
width."""
import math

import numpy as np
import pytest

import oracle
import workloads

LAM, Z = 0.5e-6, 3.7e7


def geometry():
    return workloads.workload(5, reduced=True).shape


def targets(n=300, seed=5):
    g = np.random.Generator(np.random.PCG64(seed))
    return g.uniform(-12, 12, n), g.uniform(-12, 12, n)


def ribbon(s, coef, mr):
    return oracle.quad_starshade_ribbon(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md, coef, s.K, mr)


def test_zero_perturbation_is_the_ideal_rule():
    s = geometry()
    x, y, w = ribbon(s, np.zeros_like(s.coef), 3)
    xi_, yi_, wi_ = oracle.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md)
    n = len(xi_)
    assert len(x) == n + 2 * s.Np * s.m * 3
    assert np.array_equal(x[:n], xi_) and np.array_equal(y[:n], yi_) and np.array_equal(w[:n], wi_)
    assert np.all(w[n:] == 0.0)
    # zero-weight nodes add exact zeros; only the pairwise summation's
    # grouping differs
    xi, eta = targets(50)
    u = oracle.fresnel_direct(x, y, w, LAM, Z, xi, eta)
    ref = oracle.fresnel_direct(xi_, yi_, wi_, LAM, Z, xi, eta)
    assert np.abs(u - ref).max() <= 1e-14


@pytest.mark.parametrize("mr", [0, 1, 3])
def test_ribbon_area_closed_form(mr):
    # signed ribbon area = sum over petals and edges of int_a^R d(r) dr, with
    # int_a^R sin(s pi (r - a)/(R - a)) dr = (R - a)(1 - cos s pi)/(s pi)
    s = geometry()
    x, y, w = ribbon(s, s.coef, mr)
    n0 = s.nd * s.md + s.Np * s.np_ * s.m
    c = s.coef.reshape(s.Np, 2, s.K)
    ks = np.arange(1, s.K + 1)
    exact = float((c * ((s.R - s.a) * (1 - np.cos(ks * math.pi)) / (ks * math.pi))).sum())
    got = float(w[n0:].sum())
    assert abs(got - exact) <= 1e-14 * (s.R - s.a) * np.abs(c).sum()
    # and each edge's ribbon separately (the sign of the lower edge)
    per = s.m * max(mr, 1)
    wr = w[n0:].reshape(s.Np, 2, per)
    ex_edge = (c * ((s.R - s.a) * (1 - np.cos(ks * math.pi)) / (ks * math.pi))).sum(axis=2)
    assert np.abs(wr.sum(axis=2) - ex_edge).max() <= 1e-14 * (s.R - s.a) * np.abs(c).sum()


def test_ribbon_matches_deformed_petals():
    # two different rules of the same perturbed domain: fields agree to
    # quadrature accuracy once the ribbon has two or more nodes across
    s = geometry()
    xi, eta = targets()
    ref = oracle.fresnel_direct(*oracle.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md,
                                                       s.coef, s.K), LAM, Z, xi, eta)
    ideal = oracle.fresnel_direct(*oracle.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md),
                                  LAM, Z, xi, eta)
    assert np.abs(ideal - ref).max() > 1e-3  # the perturbation matters at these targets
    for mr, bar in ((2, 1e-12), (4, 1e-13)):
        u = oracle.fresnel_direct(*ribbon(s, s.coef, mr), LAM, Z, xi, eta)
        assert np.abs(u - ref).max() <= bar, mr


def test_line_integral_form_is_second_order_in_width():
    # mr = 0 puts one node on the ideal edge: its error against the exact
    # perturbed field falls by 4 when the displacements halve
    s = geometry()
    xi, eta = targets(200)
    errs = []
    for sc in (1.0, 0.5, 0.25):
        c = s.coef * sc
        ref = oracle.fresnel_direct(*oracle.quad_starshade(s.Np, s.a, s.R, s.b, s.p, s.m, s.np_, s.nd, s.md,
                                                           c, s.K), LAM, Z, xi, eta)
        u = oracle.fresnel_direct(*ribbon(s, c, 0), LAM, Z, xi, eta)
        errs.append(np.abs(u - ref).max())
    assert errs[0] < 1e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5
