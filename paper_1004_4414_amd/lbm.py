"""Python binding of ``liblbm.so`` (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP library; PyTorch provides the device
memory (through the caching allocator) and the stream.  The binding refuses
to run without the built library.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# an alternative build of the same library (e.g. with other tuning macros) can
# be selected with LBM_LIBRARY
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")

Q = 19
LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EOVERLAP, LB_ESTATE, LB_EUNSTABLE, LB_ECAPACITY = 0, -1, -2, -3, -4, -5, -6, -7
LB_FP64, LB_FP32, LB_FP16, LB_BF16 = 0, 1, 2, 3
LB_KERNEL_AUTO, LB_KERNEL_FUSED, LB_KERNEL_TWOPASS = 0, 1, 2
PRECISIONS = {"fp64": LB_FP64, "fp32": LB_FP32, "fp16": LB_FP16, "bf16": LB_BF16}
KERNELS = {"auto": LB_KERNEL_AUTO, "fused": LB_KERNEL_FUSED, "twopass": LB_KERNEL_TWOPASS}

#: C-ABI entry points declared in include/lbm.h
ENTRY_POINTS = [
    "lb_default_params", "lb_create", "lb_destroy", "lb_last_error", "lb_add_particles", "lb_step",
    "lb_synchronize", "lb_observables", "lb_get_fields", "lb_get_populations", "lb_set_populations",
    "lb_get_owner", "lb_num_particles", "lb_get_particles", "lb_set_particle_state", "lb_particle_counts",
    "lb_get_state", "lb_set_state", "lb_contact_angle_to_color", "lb_footprint_bytes",
    "lb_enable_timing", "lb_kernel_timing",
    "lb_batch_create", "lb_batch_step", "lb_batch_steps_per_launch", "lb_batch_last_error", "lb_batch_destroy",
    "lb_autotune", "lb_domain_size", "lb_order_parameter_profile", "lb_order_parameter_profile_noalloc",
]


class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("tau", ctypes.c_double * 2), ("g_br", ctypes.c_double), ("rho0", ctypes.c_double),
        ("w_face", ctypes.c_double), ("w_edge", ctypes.c_double),
        ("velocity_mode", ctypes.c_int32), ("eq_order", ctypes.c_int32),
        ("rho_init", ctypes.c_double * 2), ("noise_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("body_accel", ctypes.c_double * 3), ("wall_axis", ctypes.c_int32),
        ("wall_vel", (ctypes.c_double * 3) * 2),
        ("c0_mass_corr", ctypes.c_double), ("k_hertz", ctypes.c_double),
        ("lub_hc", ctypes.c_double), ("lub_hmin", ctypes.c_double),
        ("kernel", ctypes.c_int32), ("tile", ctypes.c_int32 * 3),
        ("lub_mode", ctypes.c_int32),
        ("link_writes", ctypes.c_int32),
        ("force_average", ctypes.c_int32),
    ]


class Particle(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("vel", ctypes.c_double * 3), ("omega", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("density", ctypes.c_double), ("color", ctypes.c_double),
                ("prescribed", ctypes.c_int32)]


class ParticleState(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double * 3) for k in (
        "pos", "vel", "omega", "force_fluid", "torque_fluid", "force_total", "torque_total",
        "pending_impulse", "pending_angular")]


class Observables(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double * 2), ("fluid_momentum", ctypes.c_double * 3),
        ("particle_momentum", ctypes.c_double * 3), ("pending_impulse", ctypes.c_double * 3),
        ("n_links", ctypes.c_int64), ("n_shell", ctypes.c_int64),
        ("covered_total", ctypes.c_int64), ("uncovered_total", ctypes.c_int64), ("refill_fallback", ctypes.c_int64),
        ("n_particles", ctypes.c_int32), ("unstable", ctypes.c_int32),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_lib = None


def lib():
    """Load the HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so both share one runtime (and its view of the devices)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1004_4414_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
        sig = {
            "lb_default_params": (None, [ctypes.POINTER(Params)]),
            "lb_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(Allocator), vp, ctypes.POINTER(vp)]),
            "lb_destroy": (None, [vp]),
            "lb_last_error": (ctypes.c_char_p, [vp]),
            "lb_add_particles": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(Particle)]),
            "lb_step": (ctypes.c_int, [vp, ctypes.c_int32]),
            "lb_synchronize": (ctypes.c_int, [vp]),
            "lb_observables": (ctypes.c_int, [vp, ctypes.POINTER(Observables)]),
            "lb_get_fields": (ctypes.c_int, [vp, dp, dp, dp, dp]),
            "lb_get_populations": (ctypes.c_int, [vp, dp]),
            "lb_set_populations": (ctypes.c_int, [vp, dp]),
            "lb_get_owner": (ctypes.c_int, [vp, ip]),
            "lb_num_particles": (ctypes.c_int, [vp, ip]),
            "lb_get_particles": (ctypes.c_int, [vp, ctypes.POINTER(ParticleState)]),
            "lb_set_particle_state": (ctypes.c_int, [vp, dp]),
            "lb_particle_counts": (ctypes.c_int, [vp, ip, ip]),
            "lb_get_state": (ctypes.c_int, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
            "lb_set_state": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
            "lb_contact_angle_to_color": (ctypes.c_int, [ctypes.c_double, dp]),
            "lb_footprint_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_double,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
            "lb_enable_timing": (ctypes.c_int, [vp, ctypes.c_int32]),
            "lb_kernel_timing": (ctypes.c_int, [vp, ctypes.c_int32, dp, ctypes.POINTER(ctypes.c_int64)]),
            "lb_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, vp,
                                               ctypes.POINTER(vp)]),
            "lb_batch_step": (ctypes.c_int, [vp, ctypes.c_int32]),
            "lb_batch_steps_per_launch": (ctypes.c_int32, [vp]),
            "lb_batch_last_error": (ctypes.c_char_p, [vp]),
            "lb_batch_destroy": (None, [vp]),
            "lb_autotune": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(Particle),
                                           ctypes.c_int32, dp]),
            "lb_domain_size": (ctypes.c_int, [vp, dp]),
            "lb_order_parameter_profile": (ctypes.c_int, [vp, ctypes.c_int32, dp]),
            "lb_order_parameter_profile_noalloc": (ctypes.c_int, [vp, ctypes.c_int32, dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def make_params(p, precision="fp32", kernel="auto", tile=(0, 0, 0)):
    """lb_params from a plain parameter dict (keys of workloads.PARAM_DEFAULTS)."""
    s = Params()
    lib().lb_default_params(ctypes.byref(s))
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    s.precision = PRECISIONS[precision]
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
    s.lub_mode = int(p.get("lub_mode", 1))
    s.link_writes = int(p.get("link_writes", 1))
    s.force_average = int(p.get("force_average", 0))
    s.kernel = KERNELS[kernel]
    for a in range(3):
        s.tile[a] = int(tile[a])
    return s


class _TorchAllocator:
    """Device memory from torch's caching allocator, kept alive by reference."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.calls = 0  # allocations requested so far
        self._alloc = ALLOC_FN(self.alloc)
        self._free = FREE_FN(self.free)
        self.struct = Allocator(self._alloc, self._free, None)

    def alloc(self, nbytes, ctx):
        self.calls += 1
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except RuntimeError:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def free(self, ptr, ctx):
        self.live.pop(ptr, None)


def _particle_array(parts):
    n = len(parts["radius"])
    arr = (Particle * max(n, 1))()
    for k in range(n):
        q = arr[k]
        for a in range(3):
            q.pos[a] = float(parts["pos"][k][a])
            q.vel[a] = float(parts["vel"][k][a])
            q.omega[a] = float(parts["omega"][k][a])
        q.radius = float(parts["radius"][k])
        q.density = float(parts["density"][k])
        q.color = float(parts["color"][k])
        q.prescribed = int(parts["prescribed"][k])
    return n, arr


class Lattice:
    """One lattice on one GPU.  ``params`` is a plain dict (workloads.params)."""

    def __init__(self, params, precision="fp32", kernel="auto", tile=(0, 0, 0), device="cuda:0", stream=None):
        import torch
        self.params = dict(params)
        self.precision = precision
        self.shape = (int(params["nz"]), int(params["ny"]), int(params["nx"]))
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._allocator = _TorchAllocator(self.device)
        self._p = make_params(params, precision, kernel, tile)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().lb_create(ctypes.byref(self._p), ctypes.byref(self._allocator.struct),
                                 ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != LB_OK:
            raise LBError(rc, "lb_create failed: " + lib().lb_last_error(None).decode())
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().lb_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != LB_OK:
            raise LBError(rc, lib().lb_last_error(self._h).decode())
        return rc

    # -- particles -----------------------------------------------------------
    def add_particles(self, parts, check=True):
        n, arr = _particle_array(parts)
        rc = lib().lb_add_particles(self._h, n, arr)
        if rc == LB_OK:
            self.radii = np.concatenate([getattr(self, "radii", np.zeros(0)), np.asarray(parts["radius"], float)])
        if check:
            self._check(rc)
        return rc

    @property
    def num_particles(self):
        n = ctypes.c_int32()
        self._check(lib().lb_num_particles(self._h, ctypes.byref(n)))
        return n.value

    def particles(self):
        n = self.num_particles
        arr = (ParticleState * max(n, 1))()
        self._check(lib().lb_get_particles(self._h, arr))
        out = {}
        names = {"R": "pos", "U": "vel", "W": "omega", "Ffluid": "force_fluid", "Tfluid": "torque_fluid",
                 "Ftotal": "force_total", "Ttotal": "torque_total", "P": "pending_impulse", "PT": "pending_angular"}
        for k, f in names.items():
            out[k] = np.array([[getattr(arr[p], f)[a] for a in range(3)] for p in range(n)]).reshape(n, 3)
        return out

    def set_particle_state(self, R, U, W, P=None, PT=None):
        n = self.num_particles
        z = np.zeros((n, 3))
        buf = np.ascontiguousarray(np.concatenate(
            [np.asarray(R, float), np.asarray(U, float), np.asarray(W, float),
             z if P is None else np.asarray(P, float), z if PT is None else np.asarray(PT, float)], axis=1))
        self._check(lib().lb_set_particle_state(self._h, _dp(buf)))

    def particle_counts(self):
        n = max(self.num_particles, 1)
        links = np.zeros(n, dtype=np.int32)
        shell = np.zeros(n, dtype=np.int32)
        self._check(lib().lb_particle_counts(self._h, _ip(links), _ip(shell)))
        return links[:self.num_particles], shell[:self.num_particles]

    # -- stepping ------------------------------------------------------------
    def step(self, n=1):
        self._check(lib().lb_step(self._h, int(n)))

    def synchronize(self):
        self._check(lib().lb_synchronize(self._h))

    # -- state ---------------------------------------------------------------
    def observables(self):
        o = Observables()
        self._check(lib().lb_observables(self._h, ctypes.byref(o)))
        return dict(step=o.step, mass=np.array(o.mass[:]), fluid_momentum=np.array(o.fluid_momentum[:]),
                    particle_momentum=np.array(o.particle_momentum[:]), pending=np.array(o.pending_impulse[:]),
                    n_links=o.n_links, n_shell=o.n_shell, covered_total=o.covered_total,
                    uncovered_total=o.uncovered_total, refill_fallback=o.refill_fallback,
                    n_particles=o.n_particles, unstable=o.unstable)

    def fields(self):
        rho = np.zeros((2,) + self.shape)
        j = np.zeros((2,) + self.shape + (3,))
        F = np.zeros((2,) + self.shape + (3,))
        u = np.zeros(self.shape + (3,))
        self._check(lib().lb_get_fields(self._h, _dp(rho), _dp(j), _dp(F), _dp(u)))
        return dict(rho=rho, j=j, F=F, u=u)

    def populations(self):
        out = np.zeros((2, Q) + self.shape)
        self._check(lib().lb_get_populations(self._h, _dp(out)))
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape((2, Q) + self.shape))
        self._check(lib().lb_set_populations(self._h, _dp(f)))

    def owner(self):
        out = np.zeros(self.shape, dtype=np.int32)
        self._check(lib().lb_get_owner(self._h, _ip(out)))
        return out

    def get_state(self):
        n = ctypes.c_size_t(0)
        self._check(lib().lb_get_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().lb_get_state(self._h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(lib().lb_set_state(self._h, buf, len(blob)))


    # -- observables ---------------------------------------------------------
    def domain_size(self):
        """(L_x, L_y, L_z) of Sec. VI from the order-parameter structure function"""
        out = np.zeros(3)
        self._check(lib().lb_domain_size(self._h, _dp(out)))
        return out

    def order_parameter_profile(self, axis=2):
        """plane averages of phi = rho_r - rho_b along axis (0 = x, 1 = y, 2 = z)"""
        n = (self.shape[2], self.shape[1], self.shape[0])[axis]
        out = np.zeros(n)
        self._check(lib().lb_order_parameter_profile(self._h, int(axis), _dp(out)))
        return out

    def order_parameter_profile_noalloc(self, axis=2):
        """the same profile from lb_order_parameter_profile_noalloc (no device allocation)"""
        n = (self.shape[2], self.shape[1], self.shape[0])[axis]
        out = np.zeros(n)
        self._check(lib().lb_order_parameter_profile_noalloc(self._h, int(axis), _dp(out)))
        return out

    # -- measurement ---------------------------------------------------------
    def enable_timing(self, on=True):
        self._check(lib().lb_enable_timing(self._h, 1 if on else 0))

    def kernel_timing(self, which):
        """(milliseconds, launches) since timing was enabled; which = 0 the
        collide-and-stream sweep, 1 the density sweep, 2 whole steps"""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().lb_kernel_timing(self._h, int(which), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def contact_angle_to_color(theta_deg):
    c = ctypes.c_double()
    rc = lib().lb_contact_angle_to_color(float(theta_deg), ctypes.byref(c))
    if rc != LB_OK:
        raise LBError(rc, "contact angle out of range")
    return c.value


def footprint_bytes(params, n_particles=0, max_radius=0.0, precision="fp32"):
    p = make_params(params, precision)
    out = ctypes.c_size_t()
    rc = lib().lb_footprint_bytes(ctypes.byref(p), int(n_particles), float(max_radius), ctypes.byref(out))
    if rc != LB_OK:
        raise LBError(rc, "invalid parameters")
    return out.value


class Batch:
    """Lattices advanced together by one graph launch of ``steps_per_launch``
    steps each (lb_batch_*).  The members must be set up and outlive the batch."""

    def __init__(self, members, steps_per_launch=2, stream=None):
        import torch
        self.members = list(members)
        if stream is None:
            stream = torch.cuda.current_stream(self.members[0].device)
        self.stream = stream
        arr = (ctypes.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        b = ctypes.c_void_p()
        rc = lib().lb_batch_create(arr, len(self.members), int(steps_per_launch), ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(b))
        if rc != LB_OK:
            raise LBError(rc, "lb_batch_create failed: " + lib().lb_batch_last_error(None).decode())
        self._b = b
        self.steps_per_launch = lib().lb_batch_steps_per_launch(b)

    def step(self, nlaunches=1):
        rc = lib().lb_batch_step(self._b, int(nlaunches))
        if rc != LB_OK:
            raise LBError(rc, lib().lb_batch_last_error(self._b).decode())

    def close(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value:
            lib().lb_batch_destroy(b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(params, parts=None, precision="fp32", trial_steps=10):
    """(kernel name, tile, ms per step) of the fastest sweep variant for this box (lb_autotune)."""
    p = make_params(params, precision)
    n, arr = _particle_array(parts) if parts is not None else (0, (Particle * 1)())
    ms = ctypes.c_double()
    rc = lib().lb_autotune(ctypes.byref(p), n, arr, int(trial_steps), ctypes.byref(ms))
    if rc != LB_OK:
        raise LBError(rc, "autotune found no runnable variant")
    name = {v: k for k, v in KERNELS.items()}[p.kernel]
    return name, (p.tile[0], p.tile[1], p.tile[2]), ms.value
