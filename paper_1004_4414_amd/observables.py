"""Contact angle of a sphere at a flat interface (Sec. V, Eq. (32)).

The interface is the (linearly interpolated) zero of the plane-averaged order
parameter phi = rho_r - rho_b along the axis normal to it, taken as the
crossing nearest the sphere's centre (periodic box).  With Delta h the signed
distance of the centre from that plane, positive on the side where phi < 0
(the blue fluid), cos(theta) = Delta h / r.  A sphere that prefers red
(positive colour) sits on the red side, Delta h < 0 and theta > 90 degrees,
the same sign convention as the colour-angle conversion of the library.
"""
import math

import numpy as np


def interface_crossings(profile):
    """positions z (plane units, periodic) where the profile changes sign,
    linearly interpolated, with the sign change (+1: phi decreases in +z)"""
    p = np.asarray(profile, dtype=np.float64)
    n = len(p)
    out = []
    for z in range(n):
        a, b = p[z], p[(z + 1) % n]
        if a == 0.0 and b == 0.0:
            continue
        if (a > 0.0) != (b > 0.0) or a == 0.0:
            t = a / (a - b) if a != b else 0.0
            out.append(((z + t) % n, 1 if a > b else -1))
    return out


def contact_angle_from_profile(profile, centre, radius):
    """theta in degrees of a sphere of the given radius whose centre is at
    `centre` (plane units) along the profile's axis"""
    n = len(profile)
    best = None
    for zi, direction in interface_crossings(profile):
        d = (centre - zi + n / 2.0) % n - n / 2.0  # centre minus interface, minimum image
        if best is None or abs(d) < abs(best[0]):
            best = (d, direction)
    if best is None:
        raise ValueError("the profile has no interface")
    d, direction = best
    dh = d if direction > 0 else -d  # positive on the blue (phi < 0) side
    return math.degrees(math.acos(max(-1.0, min(1.0, dh / radius))))


def contact_angle(lattice, particle=0, axis=2):
    """the contact angle of sphere `particle` of a Lattice at the interface
    normal to `axis` (Eq. (32))"""
    prof = lattice.order_parameter_profile(axis)
    P = lattice.particles()
    return contact_angle_from_profile(prof, float(P["R"][particle][axis]), float(lattice.radii[particle]))
