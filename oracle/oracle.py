"""ctypes wrapper of the plain FP64 CPU oracle in ``lbm_oracle.c``.

Test infrastructure: only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module.  It never imports the GPU
package and the GPU package never imports it.

Parameters come as a plain dict (keys listed in ``DEFAULTS``); particles as a
dict of numpy arrays (``pos`` (n,3), ``vel`` (n,3), ``omega`` (n,3),
``radius``, ``density``, ``color``, ``prescribed``).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

Q = 19

DEFAULTS = dict(
    nx=16, ny=16, nz=16,
    tau=(1.0, 1.0), g_br=0.08, rho0=1.0, w_face=4.0, w_edge=2.0,
    velocity_mode=1, eq_order=3,
    rho_init=(0.35, 0.35), noise_amp=0.01, seed=1,
    body_accel=(0.0, 0.0, 0.0), wall_axis=-1, wall_vel=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
    c0_mass_corr=0.0, k_hertz=100.0, lub_hc=2.0 / 3.0, lub_hmin=0.1, lub_mode=1,
    force_average=0, virtual_fluid=1,
)


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("tau", ctypes.c_double * 2), ("g_br", ctypes.c_double), ("rho0", ctypes.c_double),
        ("w_face", ctypes.c_double), ("w_edge", ctypes.c_double),
        ("velocity_mode", ctypes.c_int32), ("eq_order", ctypes.c_int32),
        ("rho_init", ctypes.c_double * 2), ("noise_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("body_accel", ctypes.c_double * 3), ("wall_axis", ctypes.c_int32),
        ("wall_vel", (ctypes.c_double * 3) * 2),
        ("c0_mass_corr", ctypes.c_double), ("k_hertz", ctypes.c_double),
        ("lub_hc", ctypes.c_double), ("lub_hmin", ctypes.c_double),
        ("virtual_fluid", ctypes.c_int32), ("lub_mode", ctypes.c_int32),
        ("force_average", ctypes.c_int32),
    ]


def build(force=False):
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ctypes.POINTER(_Params)]
        L.orc_destroy.argtypes = [vp]
        L.orc_add_particles.restype = ctypes.c_int
        L.orc_add_particles.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp, dp, dp, ip]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [vp, ctypes.c_int]
        L.orc_get_populations.argtypes = [vp, dp]
        L.orc_set_populations.argtypes = [vp, dp]
        L.orc_get_fields.argtypes = [vp, dp, dp, dp, dp]
        L.orc_get_virtual_density.argtypes = [vp, dp]
        L.orc_get_owner.argtypes = [vp, ip]
        L.orc_num_particles.restype = ctypes.c_int
        L.orc_num_particles.argtypes = [vp]
        L.orc_get_particles.argtypes = [vp, dp]
        L.orc_set_particle_state.argtypes = [vp, dp]
        L.orc_set_previous_fluid_force.argtypes = [vp, dp]
        L.orc_particle_counts.argtypes = [vp, ip, ip]
        L.orc_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_sums.argtypes = [vp, dp]
        L.orc_event_mass.argtypes = [vp, dp]
        L.orc_lattice.argtypes = [ip, dp, ip]
        L.orc_equilibrium.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, dp]
        L.orc_psi.restype = ctypes.c_double
        L.orc_psi.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_viscosity.restype = ctypes.c_double
        L.orc_viscosity.argtypes = [ctypes.c_double]
        L.orc_cs2.restype = ctypes.c_double
        L.orc_uniform01.restype = ctypes.c_double
        L.orc_uniform01.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def make_params(**kw):
    p = dict(DEFAULTS)
    for k in kw:
        if k not in DEFAULTS:
            raise KeyError(f"unknown oracle parameter {k!r}")
    p.update(kw)
    return p


class Oracle:
    """One oracle lattice.  All arrays returned are fresh numpy float64/int32."""

    def __init__(self, params):
        p = make_params(**params)
        self.params = p
        s = _Params()
        s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
        s.tau[0], s.tau[1] = p["tau"]
        s.g_br, s.rho0, s.w_face, s.w_edge = p["g_br"], p["rho0"], p["w_face"], p["w_edge"]
        s.velocity_mode, s.eq_order = int(p["velocity_mode"]), int(p["eq_order"])
        s.rho_init[0], s.rho_init[1] = p["rho_init"]
        s.noise_amp, s.seed = p["noise_amp"], int(p["seed"]) & (2 ** 64 - 1)
        for a in range(3):
            s.body_accel[a] = p["body_accel"][a]
            s.wall_vel[0][a] = p["wall_vel"][0][a]
            s.wall_vel[1][a] = p["wall_vel"][1][a]
        s.wall_axis = int(p["wall_axis"])
        s.c0_mass_corr, s.k_hertz = p["c0_mass_corr"], p["k_hertz"]
        s.lub_hc, s.lub_hmin = p["lub_hc"], p["lub_hmin"]
        s.virtual_fluid = int(p["virtual_fluid"])
        s.lub_mode = int(p["lub_mode"])
        s.force_average = int(p["force_average"])
        self.shape = (s.nz, s.ny, s.nx)
        self.N = s.nx * s.ny * s.nz
        self._h = lib().orc_create(ctypes.byref(s))
        if not self._h:
            raise MemoryError("oracle allocation failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- particles -----------------------------------------------------------
    def add_particles(self, parts):
        n = len(parts["radius"])
        f64 = lambda k, shape: np.ascontiguousarray(np.asarray(parts[k], dtype=np.float64).reshape(shape))
        pos, vel, om = f64("pos", (n, 3)), f64("vel", (n, 3)), f64("omega", (n, 3))
        rad, den, col = f64("radius", (n,)), f64("density", (n,)), f64("color", (n,))
        pre = np.ascontiguousarray(np.asarray(parts["prescribed"], dtype=np.int32).reshape(n))
        return lib().orc_add_particles(self._h, n, _dp(pos), _dp(vel), _dp(om), _dp(rad), _dp(den),
                                       _dp(col), _ip(pre))

    @property
    def num_particles(self):
        return lib().orc_num_particles(self._h)

    def particles(self):
        """dict of (np,3) arrays: R U W Ffluid Tfluid Ftotal Ttotal P PT"""
        n = self.num_particles
        out = np.zeros((max(n, 1), 27))
        if n:
            lib().orc_get_particles(self._h, _dp(out))
        out = out[:n]
        names = ["R", "U", "W", "Ffluid", "Tfluid", "Ftotal", "Ttotal", "P", "PT"]
        return {k: out[:, 3 * i:3 * i + 3].copy() for i, k in enumerate(names)}

    def set_particle_state(self, R, U, W, P=None, PT=None):
        n = self.num_particles
        z = np.zeros((n, 3))
        buf = np.ascontiguousarray(np.concatenate(
            [np.asarray(R, float), np.asarray(U, float), np.asarray(W, float),
             z if P is None else np.asarray(P, float), z if PT is None else np.asarray(PT, float)], axis=1))
        lib().orc_set_particle_state(self._h, _dp(buf))

    def set_previous_fluid_force(self, F, T):
        """the fluid force and torque (n,3) each sphere took in the step before,
        for force_average 1 (set after set_particle_state, which forgets them)"""
        buf = np.ascontiguousarray(np.concatenate([np.asarray(F, float), np.asarray(T, float)], axis=1))
        lib().orc_set_previous_fluid_force(self._h, _dp(buf))

    # -- stepping ------------------------------------------------------------
    def step(self, n=1):
        if lib().orc_step(self._h, int(n)) != 0:
            raise RuntimeError("a sphere moved a lattice unit or more in one step: outside the scheme")

    # -- state ---------------------------------------------------------------
    def populations(self):
        out = np.zeros((2, Q) + self.shape)
        lib().orc_get_populations(self._h, _dp(out))
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape((2, Q) + self.shape))
        lib().orc_set_populations(self._h, _dp(f))

    def fields(self):
        """rho (2,nz,ny,nx), j (2,nz,ny,nx,3), F (2,nz,ny,nx,3), u (nz,ny,nx,3)"""
        rho = np.zeros((2,) + self.shape)
        j = np.zeros((2,) + self.shape + (3,))
        F = np.zeros((2,) + self.shape + (3,))
        u = np.zeros(self.shape + (3,))
        lib().orc_get_fields(self._h, _dp(rho), _dp(j), _dp(F), _dp(u))
        return dict(rho=rho, j=j, F=F, u=u)

    def virtual_density(self):
        out = np.zeros((2,) + self.shape)
        lib().orc_get_virtual_density(self._h, _dp(out))
        return out

    def owner(self):
        out = np.zeros(self.shape, dtype=np.int32)
        lib().orc_get_owner(self._h, _ip(out))
        return out

    def particle_counts(self):
        n = max(self.num_particles, 1)
        links = np.zeros(n, dtype=np.int32)
        shell = np.zeros(n, dtype=np.int32)
        lib().orc_particle_counts(self._h, _ip(links), _ip(shell))
        return links[:self.num_particles], shell[:self.num_particles]

    def counts(self):
        out = np.zeros(6, dtype=np.int64)
        lib().orc_counts(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        keys = ["step", "covered_total", "uncovered_total", "refill_fallback", "covered_last", "uncovered_last"]
        return dict(zip(keys, (int(v) for v in out)))

    def event_mass(self):
        out = np.zeros(6)
        lib().orc_event_mass(self._h, _dp(out))
        return dict(covered=out[0:2].copy(), refilled=out[2:4].copy(), wall=out[4:6].copy())

    def sums(self):
        out = np.zeros(14)
        lib().orc_sums(self._h, _dp(out))
        return dict(mass=out[0:2].copy(), fluid_momentum=out[2:5].copy(),
                    particle_momentum=out[5:8].copy(), pending=out[8:11].copy(),
                    wall_force=out[11:14].copy())


# -- small pure functions used by the lattice and equilibrium pins ----------
def lattice():
    c = np.zeros((Q, 3), dtype=np.int32)
    zeta = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    lib().orc_lattice(_ip(c), _dp(zeta), _ip(opp))
    return c, zeta, opp


def equilibrium(rho, u, order=3):
    out = np.zeros(Q)
    lib().orc_equilibrium(float(rho), float(u[0]), float(u[1]), float(u[2]), int(order), _dp(out))
    return out


def psi(rho, rho0=1.0):
    return lib().orc_psi(float(rho), float(rho0))


def viscosity(tau):
    return lib().orc_viscosity(float(tau))


def cs2():
    return lib().orc_cs2()


def uniform01(seed, k):
    return lib().orc_uniform01(int(seed) & (2 ** 64 - 1), int(k))


# ---------------------------------------------------------------------------
# Analysis observables of the oracle state (Sec. V, Eq. (32); Sec. VI,
# Eqs. (33)-(35)), from the order parameter phi = rho_r - rho_b on fluid sites
# (0 on solid ones).  The structure function is taken from the full 3-D FFT
# of the fluctuations, as the equations define it.
# ---------------------------------------------------------------------------
def order_parameter(orc):
    """phi = rho_r - rho_b on fluid sites, 0 on solid ones; indexed [z, y, x]"""
    rho = orc.fields()["rho"]
    return np.where(orc.owner() == -1, rho[0] - rho[1], 0.0)


def domain_size(phi):
    """(L_x, L_y, L_z) = 2 pi / sqrt(<k_i^2>) with <k_i^2> the S(k)-weighted
    mean of k_i^2, S(k) = |phi'_k|^2 / N; phi indexed [z, y, x]"""
    phi = np.asarray(phi, dtype=np.float64)
    N = phi.size
    S = np.abs(np.fft.fftn(phi - phi.mean())) ** 2 / N
    nz, ny, nx = phi.shape
    k = [2.0 * np.pi * np.fft.fftfreq(n) for n in (nx, ny, nz)]  # |m| <= n/2 as 2 pi m / n
    kz, ky, kx = np.meshgrid(k[2], k[1], k[0], indexing="ij")
    tot = S.sum()
    out = []
    for ki in (kx, ky, kz):
        m2 = (ki ** 2 * S).sum() / tot if tot > 0 else 0.0
        out.append(2.0 * np.pi / np.sqrt(m2) if m2 > 0 else np.inf)
    return np.array(out)


def order_parameter_profile(phi, axis=2):
    """plane averages of phi along axis (0 = x, 1 = y, 2 = z); phi indexed [z, y, x]"""
    phi = np.asarray(phi, dtype=np.float64)
    other = {0: (0, 1), 1: (0, 2), 2: (1, 2)}[axis]  # array axes averaged over
    return phi.mean(axis=other)
