"""Helpers for building oracle states in tests (no arithmetic of the method
beyond calling the oracle's own equilibrium for initial conditions)."""
import numpy as np

from oracle import oracle as O


def equilibrium_field(rho, u, order=3):
    """populations (2,19,nz,ny,nx) at equilibrium with densities rho (2,nz,ny,nx)
    and a common velocity u (nz,ny,nx,3)"""
    shape = rho.shape[1:]
    f = np.zeros((2, 19) + shape)
    for idx in np.ndindex(*shape):
        for c in range(2):
            f[(c, slice(None)) + idx] = O.equilibrium(rho[(c,) + idx], u[idx], order)
    return f


def mixture_velocity(orc):
    return orc.fields()["u"]


def total_momentum(orc):
    s = orc.sums()
    return s["fluid_momentum"] + s["particle_momentum"] + s["pending"]
