"""Pins of the boundary labels (oracle step O2; eq. JanusBC and the smoothed-arc
label of the benchmark workloads).

The smoothed arc f(phi) = 1/2 [tanh((phi + h)/w) - tanh((phi - h)/w)] has values
that its definition fixes without evaluating the oracle's formula: f(0) =
tanh(h/w), f(+-h) = tanh(2h/w)/2, and its integral over a full turn is
w [ln cosh((pi + h)/w) - ln cosh((pi - h)/w)] (an antiderivative of tanh(x/w)
is w ln cosh(x/w)).  The default call must be the 90-degree arc with edge width
0.1 rad: a half-opening of pi/2 instead of pi/4, or an opening or width taken in
degrees, changes every one of these values.  The polar angle is tested through
points placed at known angles from the director of a rotated, shifted disk.
"""
import math
import types

import numpy as np
import pytest

import oracle


def _points_at(phis, center=(1.7, -0.4), angle=0.9, radius=0.8):
    """A fake discretisation whose nodes sit at polar angles phis from the director."""
    phis = np.asarray(phis, dtype=np.float64)
    a = angle + phis
    x = np.stack([center[0] + radius * np.cos(a), center[1] + radius * np.sin(a)], axis=1)
    return types.SimpleNamespace(x=x, particle=np.zeros(len(phis), dtype=int),
                                 center=np.array([center]), angle=np.array([angle]))


def _log_cosh(x):
    x = abs(x)
    return x + math.log1p(math.exp(-2.0 * x)) - math.log(2.0)


def test_arc_label_point_values_fixed_by_its_definition():
    h, w = math.pi / 4, 0.1
    f = oracle.arc_label(_points_at([0.0, h, -h, math.pi, math.pi / 2]))
    assert abs(f[0] - math.tanh(h / w)) < 1e-15
    assert abs(f[1] - 0.5 * math.tanh(2 * h / w)) < 1e-15
    assert abs(f[2] - 0.5 * math.tanh(2 * h / w)) < 1e-15
    # far from the arc the label vanishes: 1/2 [tanh((pi+h)/w) - tanh((pi-h)/w)]
    assert 0.0 <= f[3] < 1e-13
    # a quarter turn from the director lies pi/4 outside the arc's edge (7.85 edge widths)
    assert abs(f[4] - 0.5 * (math.tanh(0.75 * math.pi / w) - math.tanh(0.25 * math.pi / w))) < 1e-12
    assert f[4] < 2e-6


@pytest.mark.parametrize("h,w", [(math.pi / 4, 0.1), (math.pi / 3, 0.25), (1.0, 0.05)])
def test_arc_label_integral_over_a_turn(h, w):
    # trapezoid rule on a periodic function: exponentially accurate in the number of points
    n = 40000
    phis = -math.pi + 2 * math.pi * (np.arange(n) + 0.5) / n
    f = oracle.arc_label(_points_at(phis), half=h, width=w)
    integral = f.sum() * 2 * math.pi / n
    exact = w * (_log_cosh((math.pi + h) / w) - _log_cosh((math.pi - h) / w))
    assert abs(integral - exact) < 1e-10
    # the arc's opening: the integral is 2h up to the edges' exponentially small tails
    assert abs(exact - 2 * h) < 1e-6


def test_arc_label_default_is_the_90_degree_arc():
    phis = np.linspace(-math.pi, math.pi, 721)
    f_default = oracle.arc_label(_points_at(phis))
    f_explicit = 0.5 * (np.tanh((phis + math.pi / 4) / 0.1) - np.tanh((phis - math.pi / 4) / 0.1))
    assert np.abs(f_default - f_explicit).max() < 1e-14
    # half of the maximum is reached at +-45 degrees (the edge centres)
    inside = phis[f_default > 0.5 * f_default.max()]
    assert abs(inside.max() - math.pi / 4) < 0.01 and abs(inside.min() + math.pi / 4) < 0.01


def test_polar_angle_is_measured_from_the_director():
    # a point on the director's side has phi = 0, on the opposite side phi = pi,
    # counter-clockwise quarter turn phi = pi/2 (for any centre and director)
    for angle in (0.0, 0.9, -2.5):
        d = _points_at([0.0, math.pi, math.pi / 2, -math.pi / 2], center=(-3.0, 2.0),
                       angle=angle, radius=1.3)
        phi = oracle.labels.polar_angle(d)
        assert abs(phi[0]) < 1e-14
        assert abs(abs(phi[1]) - math.pi) < 1e-14
        assert abs(phi[2] - math.pi / 2) < 1e-14 and abs(phi[3] + math.pi / 2) < 1e-14


def test_janus_label_values_fixed_by_its_reading():
    # f = 1 - sin^p(phi/2): 1 at the director (head), 0 opposite (tail), 1/2 at a
    # quarter turn for p = 2; for p = 2 it equals 1/2 (1 + cos phi), the data of the
    # single-disk solution (eq. true_soln)
    d = _points_at([0.0, math.pi, math.pi / 2, -math.pi / 2, 1.1])
    f2 = oracle.janus_label(d, p=2)
    assert abs(f2[0] - 1.0) < 1e-15 and abs(f2[1]) < 1e-15
    assert abs(f2[2] - 0.5) < 1e-15 and abs(f2[3] - 0.5) < 1e-15
    assert abs(f2[4] - 0.5 * (1 + math.cos(1.1))) < 1e-15
    f4 = oracle.janus_label(d, p=4)
    assert abs(f4[2] - 0.75) < 1e-15
