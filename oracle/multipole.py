"""Multipoles as sets of point forces, Sec. III (TEST INFRASTRUCTURE ONLY).

The paper builds the Stokes doublet from two monopoles of strength F a
distance apart along the force, and the rotlet from four point forces in a
pinwheel ("swastika-like") arrangement, which cancels the symmetric part.
Reading of the unstated geometry:
  type 0 Stokeslet : s p at R
  type 1 stresslet : +s p at R + (d/2) p,  -s p at R - (d/2) p
  type 2 rotlet    : with e2 = n x e1,
                     +s e2 at R + (d/2) e1,  -s e2 at R - (d/2) e1,
                     -s e1 at R + (d/2) e2,  +s e1 at R - (d/2) e2
                     (zero net force, zero symmetric first moment, torque 2 d s n)
``axis`` is p (types 0, 1) or n (type 2); ``e1`` is a unit vector normal to n.
"""
from __future__ import annotations

import numpy as np

STOKESLET, STRESSLET, ROTLET = 0, 1, 2


def expand(types, centers, axes, e1s, strengths, sep):
    pos, frc = [], []
    for t, R, ax, e1, s in zip(types, np.reshape(centers, (-1, 3)), np.reshape(axes, (-1, 3)),
                               np.reshape(e1s, (-1, 3)), strengths):
        R = np.asarray(R, dtype=np.float64)
        if t == STOKESLET:
            pos.append(R)
            frc.append(s * ax)
        elif t == STRESSLET:
            pos += [R + 0.5 * sep * ax, R - 0.5 * sep * ax]
            frc += [s * ax, -s * ax]
        elif t == ROTLET:
            e2 = np.cross(ax, e1)
            pos += [R + 0.5 * sep * e1, R - 0.5 * sep * e1, R + 0.5 * sep * e2, R - 0.5 * sep * e2]
            frc += [s * e2, -s * e2, -s * e1, s * e1]
        else:
            raise ValueError("unknown multipole type %r" % (t,))
    if not pos:
        return np.zeros((0, 3)), np.zeros((0, 3))
    return np.array(pos), np.array(frc)
