"""Plain FP64 CPU oracle of the ternary free-energy LB step (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and
shares no source with it.  ``tlb_oracle.c`` is the oracle itself; this module
marshals numpy arrays into it through ctypes.

Layouts match the C code: node index ``n = x + nx*(y + ny*z)``, populations
``[species (f, g, k)][q][n]``, concentration fields ``[3][n]``, wetting
parameters ``[wall (y-, y+)][component][x + nx*z]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tlb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")

FIELDS = ("C1", "C2", "C3", "rho", "phi", "psi", "ux", "uy", "uz", "mu_phi", "mu_psi")


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("walls_y", ctypes.c_int32),
        ("kappa", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
        ("tau_f", ctypes.c_double),
        ("tau_g", ctypes.c_double),
        ("tau_k", ctypes.c_double),
        ("gamma_phi", ctypes.c_double),
        ("gamma_psi", ctypes.c_double),
        ("no_advection", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("tau_bulk", ctypes.c_double),
        ("tau_ghost", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O3, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(OrcParams)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_check_params.argtypes = [P]
        L.orc_lattice_info.argtypes = [ctypes.c_int, ip, ip, dp, dp, ip]
        L.orc_node_thermo.argtypes = [P, ctypes.c_double, dp, dp, dp]
        L.orc_node_equilibria.argtypes = [P, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double,
                                          dp, dp, dp, dp, dp]
        L.orc_gradients.argtypes = [P, dp, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [P, dp, dp, dp, dp]
        L.orc_step.argtypes = [P, dp, dp, ctypes.c_long]
        L.orc_fields.argtypes = [P, dp, dp, dp]
        L.orc_mrt_basis.argtypes = [ctypes.c_int, dp, ip]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Params:
    """Physical and lattice parameters of one simulation (plain Python)."""

    def __init__(self, lattice, nx, ny, nz=1, walls_y=0, kappa=(0.01, 0.01, 0.01), alpha=1.0,
                 tau_f=1.0, tau_g=1.0, tau_k=1.0, gamma_phi=1.0, gamma_psi=1.0, no_advection=0, collision=0,
                 tau_bulk=1.0, tau_ghost=1.0):
        self.lattice = int(lattice)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.walls_y = int(walls_y)
        self.kappa = tuple(float(k) for k in kappa)
        self.alpha = float(alpha)
        self.tau_f, self.tau_g, self.tau_k = float(tau_f), float(tau_g), float(tau_k)
        self.gamma_phi, self.gamma_psi = float(gamma_phi), float(gamma_psi)
        self.no_advection = int(no_advection)
        self.collision = int(collision)
        self.tau_bulk, self.tau_ghost = float(tau_bulk), float(tau_ghost)

    @property
    def Q(self):
        return 9 if self.lattice == 0 else 19

    @property
    def D(self):
        return 2 if self.lattice == 0 else 3

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def c(self):
        p = OrcParams()
        p.lattice, p.nx, p.ny, p.nz, p.walls_y = self.lattice, self.nx, self.ny, self.nz, self.walls_y
        for m in range(3):
            p.kappa[m] = self.kappa[m]
        p.alpha, p.tau_f, p.tau_g, p.tau_k = self.alpha, self.tau_f, self.tau_g, self.tau_k
        p.gamma_phi, p.gamma_psi = self.gamma_phi, self.gamma_psi
        p.no_advection = self.no_advection
        p.collision, p.tau_bulk, p.tau_ghost = self.collision, self.tau_bulk, self.tau_ghost
        return p

    def replace(self, **kw):
        d = dict(lattice=self.lattice, nx=self.nx, ny=self.ny, nz=self.nz, walls_y=self.walls_y,
                 kappa=self.kappa, alpha=self.alpha, tau_f=self.tau_f, tau_g=self.tau_g,
                 tau_k=self.tau_k, gamma_phi=self.gamma_phi, gamma_psi=self.gamma_psi,
                 no_advection=self.no_advection, collision=self.collision, tau_bulk=self.tau_bulk,
                 tau_ghost=self.tau_ghost)
        d.update(kw)
        return Params(**d)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def lattice_info(lattice):
    Q = 9 if lattice == 0 else 19
    q = ctypes.c_int()
    e = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    wab = np.zeros((Q, 6))
    opp = np.zeros(Q, dtype=np.int32)
    lib().orc_lattice_info(lattice, ctypes.byref(q), e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           _dp(w), _dp(wab), opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return dict(Q=q.value, e=e, w=w, wab=wab, opp=opp)


def mrt_basis(lattice):
    """Moment basis of the multiple-relaxation-time collision: M[Q][Q] (row k = moment k over the
    velocities) and the class of each moment (0 conserved, 1 energy, 2 viscous stress, 3 other)."""
    Q = 9 if lattice == 0 else 19
    M = np.zeros((Q, Q))
    cls = (ctypes.c_int * Q)()
    q = lib().orc_mrt_basis(int(lattice), _dp(M), cls)
    if q != Q:
        raise ValueError("oracle mrt_basis failed")
    return M, np.array(cls[:], dtype=int)


def node_thermo(p: Params, rho, C, lapC):
    """(mu_phi, mu_psi, p_b, Lambda) at one node."""
    C, lapC = _f64(C), _f64(lapC)
    out = np.zeros(4)
    pc = p.c()
    _check(lib().orc_node_thermo(ctypes.byref(pc), float(rho), _dp(C), _dp(lapC), _dp(out)), "thermo")
    return out


def node_equilibria(p: Params, rho, v, phi, psi, gradC, lapC):
    """(f_eq, g_eq, k_eq) at one node; gradC is [3 components][3 axes]."""
    v = _f64(np.resize(np.asarray(v, dtype=np.float64), 3))
    g = _f64(np.asarray(gradC, dtype=np.float64).reshape(3, -1))
    g3 = np.zeros((3, 3))
    g3[:, : g.shape[1]] = g
    lapC = _f64(lapC)
    feq, geq, keq = np.zeros(p.Q), np.zeros(p.Q), np.zeros(p.Q)
    pc = p.c()
    _check(lib().orc_node_equilibria(ctypes.byref(pc), float(rho), _dp(v), float(phi), float(psi),
                                     _dp(g3), _dp(lapC), _dp(feq), _dp(geq), _dp(keq)), "equilibria")
    return feq, geq, keq


def _h_arr(p: Params, h):
    if h is None:
        return None
    h = _f64(h)
    assert h.size == 2 * 3 * p.nx * p.nz, "h must be [2][3][nx*nz]"
    return h


def gradients(p: Params, C, h=None):
    C = _f64(C).reshape(3, p.N)
    h = _h_arr(p, h)
    grad = np.zeros((3, 3, p.N))
    lap = np.zeros((3, p.N))
    pc = p.c()
    _check(lib().orc_gradients(ctypes.byref(pc), _dp(h), _dp(C), _dp(grad), _dp(lap)), "gradients")
    return grad, lap


def init_equilibrium(p: Params, C, u=None, h=None):
    """State s_0: populations [3][Q][N] equal to the equilibria of C (and u)."""
    C = _f64(C).reshape(3, p.N)
    u = None if u is None else _f64(u).reshape(p.D, p.N)
    h = _h_arr(p, h)
    pop = np.zeros((3, p.Q, p.N))
    pc = p.c()
    _check(lib().orc_init_equilibrium(ctypes.byref(pc), _dp(h), _dp(C), _dp(u), _dp(pop)), "init")
    return pop


def step(p: Params, pop, nsteps, h=None):
    """Advance the state in place by nsteps; returns pop."""
    assert pop.dtype == np.float64 and pop.flags.c_contiguous and pop.size == 3 * p.Q * p.N
    h = _h_arr(p, h)
    pc = p.c()
    _check(lib().orc_step(ctypes.byref(pc), _dp(h), _dp(pop), int(nsteps)), "step")
    return pop


def fields(p: Params, pop, h=None):
    """Dict of the macroscopic fields of the state (see FIELDS)."""
    h = _h_arr(p, h)
    out = np.zeros((11, p.N))
    pc = p.c()
    _check(lib().orc_fields(ctypes.byref(pc), _dp(h), _dp(_f64(pop)), _dp(out)), "fields")
    return {name: out[i] for i, name in enumerate(FIELDS)}
