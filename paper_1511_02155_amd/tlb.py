"""ctypes binding of libtlb (the C ABI in include/tlb.h).

The functions below carry the C names and only marshal arguments: every
step of the lattice Boltzmann update runs in the HIP kernels of libtlb.so.
Importing this module loads the library and raises ``ImportError`` when it
has not been built (``python -m paper_1511_02155_amd.build``); there is no
fallback implementation.

``Sim`` wraps one ``tlb_sim*`` for convenience; torch tensors on the GPU can
be passed to the ``*_dev`` calls through ``tensor.data_ptr()``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1511_02155_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

TLB_OK, TLB_EINVAL, TLB_ENOMEM, TLB_EHIP, TLB_ENAN, TLB_ESTATE = 0, -1, -2, -3, -4, -5
TLB_D2Q9, TLB_D3Q19 = 0, 1
TLB_F32, TLB_F64 = 0, 1
TLB_BGK, TLB_MRT = 0, 1
TLB_MAX_COMP = 5
FIELDS = ("C1", "C2", "C3", "rho", "phi", "psi", "ux", "uy", "uz", "mu_phi", "mu_psi")
FIELD_INDEX = {name: i for i, name in enumerate(FIELDS)}
FIELD_INDEX.update(C4=11, C5=12)  # simulations with more than three components

# Every symbol declared in include/tlb.h.
EXPORTS = (
    "tlb_status_str", "tlb_last_hip_error", "tlb_version", "tlb_create", "tlb_destroy",
    "tlb_get_params", "tlb_set_wetting", "tlb_init_equilibrium", "tlb_step", "tlb_set_check_every", "tlb_set_graph",
    "tlb_get_field", "tlb_get_populations", "tlb_set_populations", "tlb_diagnostics", "tlb_get_step",
    "tlb_synchronize", "tlb_get_stream", "tlb_init_equilibrium_dev", "tlb_get_field_dev",
    "tlb_get_populations_dev", "tlb_set_populations_dev", "tlb_set_wetting_dev", "tlb_set_launch",
    "tlb_get_launch", "tlb_set_adjoint_launch", "tlb_get_adjoint_launch", "tlb_bytes_per_node", "tlb_state_bytes",
    "tlb_save_state", "tlb_load_state",
    "tlb_save_state_dev", "tlb_load_state_dev", "tlb_device_copy",
    "tlb_batch_create", "tlb_batch_destroy", "tlb_batch_size", "tlb_batch_nodes", "tlb_batch_get_stream",
    "tlb_batch_synchronize", "tlb_batch_set_wetting", "tlb_batch_init_equilibrium", "tlb_batch_step",
    "tlb_batch_get_field", "tlb_batch_get_populations", "tlb_batch_diagnostics", "tlb_batch_set_launch",
    "tlb_batch_get_launch", "tlb_batch_autotune", "tlb_batch_set_graph",
    "tlb_set_kappa", "tlb_adjoint_seed_dev", "tlb_adjoint_step_dev", "tlb_checkpoint_slots",
    "tlb_forward_checkpointed", "tlb_adjoint_backward", "tlb_contact_angles", "tlb_wetting_from_angles",
    "tlb_wetting_outside_range", "tlb_batch_wetting_outside_range", "tlb_adjoint_step",
    "tlb_adjoint_step_noalloc", "tlb_adjoint_step_noalloc_scratch", "tlb_stream_only",
)
TLB_NOALLOC_SCRATCH_BYTES = 1 << 20


class tlb_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("walls_y", ctypes.c_int32),
        ("kappa", ctypes.c_double * 3), ("alpha", ctypes.c_double),
        ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double), ("tau_k", ctypes.c_double),
        ("gamma_phi", ctypes.c_double), ("gamma_psi", ctypes.c_double),
        ("no_advection", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("tau_bulk", ctypes.c_double),
        ("tau_ghost", ctypes.c_double),
        ("ncomp", ctypes.c_int32),
        ("kappa_hi", ctypes.c_double * 2),
    ]


class tlb_diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double * 3), ("momentum", ctypes.c_double * 3),
        ("max_speed", ctypes.c_double), ("nonfinite", ctypes.c_int64), ("step", ctypes.c_int64),
        ("interface", ctypes.c_double * 3),
        ("mass_hi", ctypes.c_double * 2), ("interface_hi", ctypes.c_double * 2),
    ]


class tlb_launch(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_P = ctypes.POINTER(tlb_params)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


tlb_status_str = _sig("tlb_status_str", ctypes.c_char_p, [ctypes.c_int])
tlb_last_hip_error = _sig("tlb_last_hip_error", ctypes.c_int, [])
tlb_version = _sig("tlb_version", ctypes.c_int, [])
tlb_create = _sig("tlb_create", ctypes.c_int, [_P, _vp, ctypes.POINTER(_vp)])
tlb_destroy = _sig("tlb_destroy", ctypes.c_int, [_vp])
tlb_get_params = _sig("tlb_get_params", ctypes.c_int, [_vp, _P])
tlb_set_wetting = _sig("tlb_set_wetting", ctypes.c_int, [_vp, ctypes.c_int, _dp])
tlb_init_equilibrium = _sig("tlb_init_equilibrium", ctypes.c_int, [_vp, _dp, _dp])
tlb_step = _sig("tlb_step", ctypes.c_int, [_vp, ctypes.c_int64])
tlb_set_check_every = _sig("tlb_set_check_every", ctypes.c_int, [_vp, ctypes.c_int64])
tlb_set_graph = _sig("tlb_set_graph", ctypes.c_int, [_vp, ctypes.c_int64])
tlb_get_field = _sig("tlb_get_field", ctypes.c_int, [_vp, ctypes.c_int, _dp])
tlb_get_populations = _sig("tlb_get_populations", ctypes.c_int, [_vp, ctypes.c_int, _dp])
tlb_set_populations = _sig("tlb_set_populations", ctypes.c_int, [_vp, ctypes.c_int, _dp])
tlb_diagnostics = _sig("tlb_diagnostics", ctypes.c_int, [_vp, ctypes.POINTER(tlb_diag)])
tlb_get_step = _sig("tlb_get_step", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)])
tlb_synchronize = _sig("tlb_synchronize", ctypes.c_int, [_vp])
tlb_get_stream = _sig("tlb_get_stream", _vp, [_vp])
tlb_init_equilibrium_dev = _sig("tlb_init_equilibrium_dev", ctypes.c_int, [_vp, _vp, _vp])
tlb_get_field_dev = _sig("tlb_get_field_dev", ctypes.c_int, [_vp, ctypes.c_int, _vp])
tlb_get_populations_dev = _sig("tlb_get_populations_dev", ctypes.c_int, [_vp, ctypes.c_int, _vp])
tlb_set_populations_dev = _sig("tlb_set_populations_dev", ctypes.c_int, [_vp, ctypes.c_int, _vp])
tlb_set_wetting_dev = _sig("tlb_set_wetting_dev", ctypes.c_int, [_vp, ctypes.c_int, _vp])
tlb_set_launch = _sig("tlb_set_launch", ctypes.c_int, [_vp, ctypes.POINTER(tlb_launch)])
tlb_get_launch = _sig("tlb_get_launch", ctypes.c_int, [_vp, ctypes.POINTER(tlb_launch)])
tlb_contact_angles = _sig("tlb_contact_angles", ctypes.c_int, [_dp, ctypes.c_double, _dp, _dp])
tlb_wetting_from_angles = _sig("tlb_wetting_from_angles", ctypes.c_int,
                               [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp])
tlb_set_adjoint_launch = _sig("tlb_set_adjoint_launch", ctypes.c_int, [_vp, ctypes.POINTER(tlb_launch)])
tlb_get_adjoint_launch = _sig("tlb_get_adjoint_launch", ctypes.c_int, [_vp, ctypes.POINTER(tlb_launch)])
tlb_bytes_per_node = _sig("tlb_bytes_per_node", ctypes.c_double, [_vp])
tlb_state_bytes = _sig("tlb_state_bytes", ctypes.c_int64, [_vp])
tlb_save_state = _sig("tlb_save_state", ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64)])
tlb_load_state = _sig("tlb_load_state", ctypes.c_int, [_vp, _vp, ctypes.c_int64])
tlb_save_state_dev = _sig("tlb_save_state_dev", ctypes.c_int, [_vp, _vp])
tlb_load_state_dev = _sig("tlb_load_state_dev", ctypes.c_int, [_vp, _vp, ctypes.c_int64])
tlb_stream_only = _sig("tlb_stream_only", ctypes.c_int, [_vp, ctypes.c_int64])
tlb_device_copy = _sig("tlb_device_copy", ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp])
tlb_batch_create = _sig("tlb_batch_create", ctypes.c_int, [_P, ctypes.c_int32, _vp, ctypes.POINTER(_vp)])
tlb_batch_destroy = _sig("tlb_batch_destroy", ctypes.c_int, [_vp])
tlb_batch_size = _sig("tlb_batch_size", ctypes.c_int32, [_vp])
tlb_batch_nodes = _sig("tlb_batch_nodes", ctypes.c_int64, [_vp])
tlb_batch_get_stream = _sig("tlb_batch_get_stream", _vp, [_vp])
tlb_batch_synchronize = _sig("tlb_batch_synchronize", ctypes.c_int, [_vp])
tlb_batch_set_wetting = _sig("tlb_batch_set_wetting", ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int, _dp])
tlb_batch_init_equilibrium = _sig("tlb_batch_init_equilibrium", ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp])
tlb_batch_step = _sig("tlb_batch_step", ctypes.c_int, [_vp, ctypes.c_int64])
tlb_batch_get_field = _sig("tlb_batch_get_field", ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int, _dp])
tlb_batch_get_populations = _sig("tlb_batch_get_populations", ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int, _dp])
tlb_batch_diagnostics = _sig("tlb_batch_diagnostics", ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(tlb_diag)])
tlb_batch_set_launch = _sig("tlb_batch_set_launch", ctypes.c_int, [_vp, ctypes.POINTER(tlb_launch)])
tlb_batch_get_launch = _sig("tlb_batch_get_launch", ctypes.c_int, [_vp, ctypes.POINTER(tlb_launch)])
tlb_batch_autotune = _sig("tlb_batch_autotune", ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(tlb_launch)])
tlb_batch_set_graph = _sig("tlb_batch_set_graph", ctypes.c_int, [_vp, ctypes.c_int32])
tlb_set_kappa = _sig("tlb_set_kappa", ctypes.c_int, [_vp, _dp])
tlb_adjoint_seed_dev = _sig("tlb_adjoint_seed_dev", ctypes.c_int, [_vp, _vp, _vp])
tlb_adjoint_step_dev = _sig("tlb_adjoint_step_dev", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp])
tlb_adjoint_step = _sig("tlb_adjoint_step", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp])
tlb_wetting_outside_range = _sig("tlb_wetting_outside_range", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)])
tlb_batch_wetting_outside_range = _sig("tlb_batch_wetting_outside_range", ctypes.c_int,
                                       [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)])
tlb_adjoint_step_noalloc = _sig("tlb_adjoint_step_noalloc", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp])
tlb_adjoint_step_noalloc_scratch = _sig("tlb_adjoint_step_noalloc_scratch", ctypes.c_int64, [_vp])
tlb_checkpoint_slots = _sig("tlb_checkpoint_slots", ctypes.c_int64, [ctypes.c_int64, ctypes.c_int64])
tlb_forward_checkpointed = _sig("tlb_forward_checkpointed", ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64, _vp])
tlb_adjoint_backward = _sig("tlb_adjoint_backward", ctypes.c_int,
                            [_vp, ctypes.c_int64, ctypes.c_int64, _vp, _vp, _vp, _vp])


class TLBError(RuntimeError):
    def __init__(self, code, what):
        msg = tlb_status_str(code).decode()
        if code == TLB_EHIP:
            msg += f" (hip error {tlb_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]")
        self.code = code


def check(code, what="tlb"):
    if code != TLB_OK:
        raise TLBError(code, what)
    return code


def _arr(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_params(lattice, nx, ny, nz=1, prec=TLB_F64, walls_y=0, kappa=(0.01, 0.01, 0.01), alpha=1.0,
                tau_f=1.0, tau_g=1.0, tau_k=1.0, gamma_phi=1.0, gamma_psi=1.0, no_advection=0, collision=0,
                tau_bulk=1.0, tau_ghost=1.0, **_ignored):
    """kappa has one coefficient per component: three for the ternary model, up to TLB_MAX_COMP
    (Sec. II.E; tlb_params.ncomp is set from its length)."""
    p = tlb_params()
    p.lattice, p.prec, p.nx, p.ny, p.nz, p.walls_y = lattice, prec, nx, ny, nz, walls_y
    kappa = [float(k) for k in kappa]
    if not 3 <= len(kappa) <= TLB_MAX_COMP:
        raise ValueError(f"expected 3 .. {TLB_MAX_COMP} kappa values, got {len(kappa)}")
    for m in range(3):
        p.kappa[m] = kappa[m]
    p.ncomp = len(kappa)
    for m in range(3, len(kappa)):
        p.kappa_hi[m - 3] = kappa[m]
    p.alpha, p.tau_f, p.tau_g, p.tau_k = alpha, tau_f, tau_g, tau_k
    p.gamma_phi, p.gamma_psi = gamma_phi, gamma_psi
    p.no_advection = int(no_advection)
    p.collision = int(collision)
    p.tau_bulk, p.tau_ghost = float(tau_bulk), float(tau_ghost)
    return p


def interface_measures(interface_sum, alpha, area):
    """From the diagnostics' sum of C_m^2 (1 - C_m)^2: the boundary length (area in 3D) of each
    component, 6 * sum / alpha (a flat interface of the tanh profile contributes alpha / 6 per unit
    length), and the typical domain size area / length (volume / area in 3D) of Sec. V.C."""
    length = [6.0 * s / alpha for s in interface_sum]
    return dict(length=length, domain_size=[area / l if l > 0 else float("inf") for l in length])


def contact_angles(kappa, alpha, h):
    """(theta_12, theta_23, theta_31) in degrees for wetting parameters h[3] (tlb_contact_angles)."""
    k, hh = _arr(kappa, 3), _arr(h, 3)
    out = np.zeros(3)
    check(tlb_contact_angles(k.ctypes.data_as(_dp), float(alpha), hh.ctypes.data_as(_dp), out.ctypes.data_as(_dp)),
          "tlb_contact_angles")
    return tuple(float(v) for v in out)


def wetting_from_angles(kappa, alpha, theta12, theta23):
    """h[3] giving theta_12, theta_23 with sum h_m / kappa_m = 0 (tlb_wetting_from_angles)."""
    k = _arr(kappa, 3)
    out = np.zeros(3)
    check(tlb_wetting_from_angles(k.ctypes.data_as(_dp), float(alpha), float(theta12), float(theta23),
                                  out.ctypes.data_as(_dp)), "tlb_wetting_from_angles")
    return tuple(float(v) for v in out)


class Sim:
    """One simulation (owns a tlb_sim*)."""

    def __init__(self, params: tlb_params, stream=None):
        self._h = _vp()
        check(tlb_create(ctypes.byref(params), stream, ctypes.byref(self._h)), "tlb_create")
        self.params = params
        self.Q = 9 if params.lattice == TLB_D2Q9 else 19
        self.D = 2 if params.lattice == TLB_D2Q9 else 3
        self.N = params.nx * params.ny * params.nz
        self.nc = params.ncomp if params.ncomp else 3

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            tlb_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_wetting(self, wall, h):
        h = _arr(h, self.nc * self.params.nx * self.params.nz)
        check(tlb_set_wetting(self._h, wall, h.ctypes.data_as(_dp)), "tlb_set_wetting")

    def set_wetting_both(self, h):
        """h: [2][ncomp][nx*nz] (wall 0 = below y=0, wall 1 = above y=ny-1)."""
        h = _arr(h).reshape(2, -1)
        self.set_wetting(0, h[0])
        self.set_wetting(1, h[1])

    def wetting_outside_range(self):
        """Wetting values of both walls with |4 h_m / (alpha kappa_m)| > 1 (-1: set from device memory)."""
        c = ctypes.c_int64()
        check(tlb_wetting_outside_range(self._h, ctypes.byref(c)), "tlb_wetting_outside_range")
        return c.value

    def init_equilibrium(self, C, u=None):
        C = _arr(C, self.nc * self.N)
        up = None
        if u is not None:
            u = _arr(u, self.D * self.N)
            up = u.ctypes.data_as(_dp)
        check(tlb_init_equilibrium(self._h, C.ctypes.data_as(_dp), up), "tlb_init_equilibrium")

    def step(self, n):
        check(tlb_step(self._h, int(n)), "tlb_step")

    def set_graph(self, steps_per_graph):
        """Replay steps from a captured hipGraph in chains of this many (even; 0 = direct launches)."""
        check(tlb_set_graph(self._h, int(steps_per_graph)), "tlb_set_graph")

    def set_check_every(self, every):
        check(tlb_set_check_every(self._h, int(every)), "tlb_set_check_every")

    def synchronize(self):
        check(tlb_synchronize(self._h), "tlb_synchronize")

    def stream_only(self, n):
        """Propagation alone (no collision) n times, in the step's pattern: a bandwidth reference."""
        check(tlb_stream_only(self._h, int(n)), "tlb_stream_only")

    def field(self, which):
        idx = FIELD_INDEX[which] if isinstance(which, str) else int(which)
        out = np.empty(self.N)
        check(tlb_get_field(self._h, idx, out.ctypes.data_as(_dp)), "tlb_get_field")
        return out

    def fields(self):
        out = {name: self.field(i) for i, name in enumerate(FIELDS)}
        for m in range(3, self.nc):
            out[f"C{m + 1}"] = self.field(f"C{m + 1}")
        return out

    def populations(self, species):
        out = np.empty((self.Q, self.N))
        check(tlb_get_populations(self._h, species, out.ctypes.data_as(_dp)), "tlb_get_populations")
        return out

    def all_populations(self):
        return np.stack([self.populations(s) for s in range(self.nc)])

    def set_populations(self, species, pop):
        pop = _arr(pop, self.Q * self.N)
        check(tlb_set_populations(self._h, species, pop.ctypes.data_as(_dp)), "tlb_set_populations")

    def diagnostics(self, allow_nan=False):
        d = tlb_diag()
        rc = tlb_diagnostics(self._h, ctypes.byref(d))
        if rc != TLB_OK and not (allow_nan and rc == TLB_ENAN):
            check(rc, "tlb_diagnostics")
        extra = self.nc - 3
        return dict(mass=list(d.mass) + list(d.mass_hi)[:extra], momentum=list(d.momentum), max_speed=d.max_speed,
                    nonfinite=d.nonfinite, step=d.step, interface=list(d.interface) + list(d.interface_hi)[:extra])

    def set_launch(self, width, height=1, chunk=0, variant=1):
        l = tlb_launch(width, height, chunk, variant)
        check(tlb_set_launch(self._h, ctypes.byref(l)), "tlb_set_launch")

    def set_adjoint_launch(self, width, chunk=0, variant=0, rows=1):
        l = tlb_launch(width, rows, chunk, variant)
        check(tlb_set_adjoint_launch(self._h, ctypes.byref(l)), "tlb_set_adjoint_launch")

    def adjoint_launch(self):
        l = tlb_launch()
        check(tlb_get_adjoint_launch(self._h, ctypes.byref(l)), "tlb_get_adjoint_launch")
        return dict(width=l.width, rows=l.height, chunk=l.chunk, variant=l.variant)

    def launch(self):
        l = tlb_launch()
        check(tlb_get_launch(self._h, ctypes.byref(l)), "tlb_get_launch")
        return dict(width=l.width, height=l.height, chunk=l.chunk, variant=l.variant)

    def save_state(self):
        """Raw state bytes and step count (bitwise resume with load_state)."""
        buf = np.empty(tlb_state_bytes(self._h), dtype=np.uint8)
        st = ctypes.c_int64()
        check(tlb_save_state(self._h, buf.ctypes.data_as(_vp), ctypes.byref(st)), "tlb_save_state")
        return buf, st.value

    def load_state(self, buf, step):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        if buf.size != tlb_state_bytes(self._h):
            raise ValueError("state size mismatch")
        check(tlb_load_state(self._h, buf.ctypes.data_as(_vp), int(step)), "tlb_load_state")

    def bytes_per_node(self):
        return tlb_bytes_per_node(self._h)

    def state_bytes(self):
        return tlb_state_bytes(self._h)

    def set_kappa(self, kappa):
        k = _arr(kappa, self.nc)
        check(tlb_set_kappa(self._h, k.ctypes.data_as(_dp)), "tlb_set_kappa")
        for m in range(self.nc):
            if m < 3:
                self.params.kappa[m] = float(k[m])
            else:
                self.params.kappa_hi[m - 3] = float(k[m])

    def stream(self):
        return tlb_get_stream(self._h)


class Batch:
    """Many independent D2Q9 lattices advanced together (owns a tlb_batch*)."""

    def __init__(self, params_list, stream=None):
        arr = (tlb_params * len(params_list))(*params_list)
        self._h = _vp()
        check(tlb_batch_create(arr, len(params_list), stream, ctypes.byref(self._h)), "tlb_batch_create")
        self.params = list(params_list)
        self.ndom = len(params_list)

    def close(self):
        if self._h:
            tlb_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def nodes(self):
        return tlb_batch_nodes(self._h)

    def _N(self, d):
        return self.params[d].nx * self.params[d].ny

    def set_wetting(self, d, wall, h):
        h = _arr(h, 3 * self.params[d].nx)
        check(tlb_batch_set_wetting(self._h, d, wall, h.ctypes.data_as(_dp)), "tlb_batch_set_wetting")

    def wetting_outside_range(self, d=-1):
        """Wetting values with |4 h_m / (alpha kappa_m)| > 1 of domain d (all domains for d = -1)."""
        c = ctypes.c_int64()
        check(tlb_batch_wetting_outside_range(self._h, int(d), ctypes.byref(c)), "tlb_batch_wetting_outside_range")
        return c.value

    def init_equilibrium(self, d, C, u=None):
        C = _arr(C, 3 * self._N(d))
        up = None
        if u is not None:
            u = _arr(u, 2 * self._N(d))
            up = u.ctypes.data_as(_dp)
        check(tlb_batch_init_equilibrium(self._h, d, C.ctypes.data_as(_dp), up), "tlb_batch_init_equilibrium")

    def step(self, n):
        check(tlb_batch_step(self._h, int(n)), "tlb_batch_step")

    def synchronize(self):
        check(tlb_batch_synchronize(self._h), "tlb_batch_synchronize")

    def field(self, d, which):
        idx = FIELD_INDEX[which] if isinstance(which, str) else int(which)
        out = np.empty(self._N(d))
        check(tlb_batch_get_field(self._h, d, idx, out.ctypes.data_as(_dp)), "tlb_batch_get_field")
        return out

    def populations(self, d, species):
        out = np.empty((9, self._N(d)))
        check(tlb_batch_get_populations(self._h, d, species, out.ctypes.data_as(_dp)), "tlb_batch_get_populations")
        return out

    def all_populations(self, d):
        return np.stack([self.populations(d, s) for s in range(3)])

    def diagnostics(self, d):
        dg = tlb_diag()
        check(tlb_batch_diagnostics(self._h, d, ctypes.byref(dg)), "tlb_batch_diagnostics")
        return dict(mass=list(dg.mass), momentum=list(dg.momentum), max_speed=dg.max_speed,
                    nonfinite=dg.nonfinite, step=dg.step, interface=list(dg.interface))

    def set_launch(self, width, chunk, variant=1, groups=1):
        l = tlb_launch(width, groups, chunk, variant)
        check(tlb_batch_set_launch(self._h, ctypes.byref(l)), "tlb_batch_set_launch")

    def launch(self):
        l = tlb_launch()
        check(tlb_batch_get_launch(self._h, ctypes.byref(l)), "tlb_batch_get_launch")
        return dict(width=l.width, chunk=l.chunk, variant=l.variant, groups=l.height)

    def autotune(self, trial_steps=10):
        l = tlb_launch()
        check(tlb_batch_autotune(self._h, int(trial_steps), ctypes.byref(l)), "tlb_batch_autotune")
        return dict(width=l.width, chunk=l.chunk, variant=l.variant, groups=l.height)

    def set_graph(self, steps_per_graph):
        check(tlb_batch_set_graph(self._h, int(steps_per_graph)), "tlb_batch_set_graph")

    def stream(self):
        return tlb_batch_get_stream(self._h)
