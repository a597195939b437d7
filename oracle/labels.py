"""Boundary data f on the particles (oracle step O2).

The hydrophobicity label has range [0, 1] (section 1).  Two forms:

* arc_label: a smoothed arc, f = 1/2 [tanh((phi + h)/w) - tanh((phi - h)/w)],
  phi in (-pi, pi] the polar angle of x - a_i measured from the director d_i,
  h the half-opening of the hydrophobic arc (pi/4 for a 90 degree arc) and w
  the edge width in radians.
* janus_label: eq. JanusBC reads f = 1 - sin^p(theta).  As printed it is even
  under theta -> pi - theta, so head and tail would both be hydrophobic; the
  single-disk solution eq. true_soln corresponds to f = 1/2 (1 + cos theta) =
  1 - sin^2(theta/2).  Reading used: f = 1 - sin^p(phi/2), p even.
"""
from __future__ import annotations

import numpy as np


def polar_angle(disc):
    """phi in (-pi, pi]: angle of x - a_i measured from the director d_i."""
    a = disc.center[disc.particle]
    th = disc.angle[disc.particle]
    dx = disc.x[:, 0] - a[:, 0]
    dy = disc.x[:, 1] - a[:, 1]
    c, s = np.cos(th), np.sin(th)
    return np.arctan2(c * dy - s * dx, c * dx + s * dy)


def arc_label(disc, half=np.pi / 4, width=0.1):
    phi = polar_angle(disc)
    return 0.5 * (np.tanh((phi + half) / width) - np.tanh((phi - half) / width))


def janus_label(disc, p=2):
    phi = polar_angle(disc)
    return 1.0 - np.sin(phi / 2.0) ** p
