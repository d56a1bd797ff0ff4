"""GPU (HIP, through the C ABI) against the FP64 CPU oracle on the same seeded inputs.

Tolerances: FP64 max |gpu - oracle| <= 1e-12 * max |oracle| per population
species and per concentration field; FP32 max |C_gpu - C_oracle| <= 1e-5
absolute on the concentrations after the stated step count.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_1511_02155_amd import inputs

pytestmark = pytest.mark.gpu

F64_REL = 1e-12
F32_ABS = 1e-5


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_1511_02155_amd import tlb as t

    return t


_PKEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi",
          "gamma_psi", "no_advection", "collision", "tau_bulk", "tau_ghost")


def _oparams(orc, w):
    return orc.Params(**{k: w[k] for k in _PKEYS if k in w})


def _gsim(tlb, w, prec, launch=None):
    p = tlb.make_params(prec=prec, **{k: v for k, v in w.items() if k in _PKEYS})
    s = tlb.Sim(p)
    if launch:
        s.set_launch(**launch)
    return s


def _run_both(tlb, orc, w, C, h, steps, prec, launch=None):
    _note(f"{w.get('name', 'case')} prec={prec} steps={steps} launch={launch}")
    p = _oparams(orc, w)
    pop = orc.init_equilibrium(p, C, None, h)
    orc.step(p, pop, steps, h)
    s = _gsim(tlb, w, prec, launch)
    if h is not None:
        s.set_wetting_both(h)
    s.init_equilibrium(C)
    s.step(steps)
    s.synchronize()
    return p, pop, s


def _compare_f64(orc, p, pop, h, s):
    for sp in range(3):
        g = s.populations(sp)
        o = pop[sp]
        err = np.abs(g - o).max()
        assert err <= F64_REL * np.abs(o).max(), (sp, err)
    Fo = orc.fields(p, pop, h)
    for name in ("C1", "C2", "C3", "rho", "phi", "psi"):
        err = np.abs(s.field(name) - Fo[name]).max()
        assert err <= F64_REL * max(np.abs(Fo[name]).max(), 1e-300), (name, err)
    vscale = np.abs(pop[0]).max()
    for name in ("ux", "uy", "uz"):
        assert np.abs(s.field(name) - Fo[name]).max() <= F64_REL * vscale, name
    for name in ("mu_phi", "mu_psi"):
        err = np.abs(s.field(name) - Fo[name]).max()
        assert err <= 1e-11 * max(np.abs(Fo[name]).max(), 1e-6), (name, err)


def _compare_f32(orc, p, pop, h, s, tol=F32_ABS):
    Fo = orc.fields(p, pop, h)
    for name in ("C1", "C2", "C3"):
        err = np.abs(s.field(name) - Fo[name]).max()
        assert err <= tol, (name, err)


def _wet_case(nx, ny, nz=1, lattice=0, seed=1, walls=1, kappa=(0.012, 0.02, 0.016), tau=(1.0, 0.9, 0.8)):
    M = 0.1
    gp, gk = inputs.mobility_to_gamma(M, tau[1], tau[2])
    w = dict(lattice=lattice, nx=nx, ny=ny, nz=nz, walls_y=walls, kappa=kappa, alpha=1.0, tau_f=tau[0],
             tau_g=tau[1], tau_k=tau[2], gamma_phi=gp, gamma_psi=gk, name=f"wet_{lattice}_{nx}x{ny}x{nz}")
    if lattice == 0:
        C = inputs.sessile_drop(nx, ny, 0.35 * min(nx, ny), top_layer=0.75 * ny)
    else:
        C = inputs.spinodal(nx, ny, nz, delta=0.25, seed=seed)
    h = inputs.random_h(nx, -0.004, 0.004, nz=nz, seed=seed + 100, bottom_only=False) if walls else None
    return w, C, h


# --------------------------------------------------------------------------
# FP64 parity: 1e-12 relative
# --------------------------------------------------------------------------

def test_double_emulsion_64_fp64_1000_steps(tlb, orc):
    """64x64 periodic double emulsion, FP64, 1000 steps (the small correctness workload)."""
    w = inputs.double_emulsion_64()
    C = w["C"]()
    p, pop, s = _run_both(tlb, orc, w, C, None, w["steps"], tlb.TLB_F64)
    _compare_f64(orc, p, pop, None, s)


@pytest.mark.parametrize("nx,ny,width,chunk", [(70, 37, 64, 8), (131, 20, 128, 7), (300, 9, 256, 3),
                                               (3, 3, 64, 1), (5, 64, 64, 64)])
def test_d2q9_walls_wetting_ragged_fp64(tlb, orc, nx, ny, width, chunk):
    """Walls with per-node wetting, ragged strips and chunks, minimum sizes."""
    w, C, h = _wet_case(nx, ny)
    for hold in (0, 1):
        p, pop, s = _run_both(tlb, orc, w, C, h, 150, tlb.TLB_F64, dict(width=width, chunk=chunk, variant=hold))
        _compare_f64(orc, p, pop, h, s)


@pytest.mark.parametrize("walls", [0, 1])
@pytest.mark.parametrize("dims,tile", [((37, 21, 13), (32, 8)), ((9, 70, 5), (64, 4)), ((3, 3, 3), (32, 8))])
def test_d3q19_ragged_fp64(tlb, orc, dims, tile, walls):
    nx, ny, nz = dims
    w, C, h = _wet_case(nx, ny, nz, lattice=1, walls=walls)
    for variant in (0, 1):
        p, pop, s = _run_both(tlb, orc, w, C, h, 30, tlb.TLB_F64,
                              dict(width=tile[0], height=tile[1], chunk=4, variant=variant))
        _compare_f64(orc, p, pop, h, s)


# --------------------------------------------------------------------------
# FP32 parity: 1e-5 absolute on C_m
# --------------------------------------------------------------------------

def test_double_emulsion_64_fp32_1000_steps(tlb, orc):
    w = inputs.double_emulsion_64()
    C = w["C"]()
    p, pop, s = _run_both(tlb, orc, w, C, None, w["steps"], tlb.TLB_F32)
    _compare_f32(orc, p, pop, None, s)


@pytest.mark.parametrize("width,hold", [(64, 0), (128, 1), (256, 1)])
def test_d2q9_walls_fp32(tlb, orc, width, hold):
    w, C, h = _wet_case(150, 61)
    p, pop, s = _run_both(tlb, orc, w, C, h, 400, tlb.TLB_F32, dict(width=width, chunk=9, variant=hold))
    _compare_f32(orc, p, pop, h, s)


@pytest.mark.parametrize("tile", [(32, 8, 0), (64, 4, 0), (32, 8, 1), (64, 4, 1), (32, 8, 2), (64, 4, 2)])
def test_d3q19_fp32(tlb, orc, tile):
    w, C, h = _wet_case(40, 34, 12, lattice=1, walls=1)
    p, pop, s = _run_both(tlb, orc, w, C, h, 60, tlb.TLB_F32,
                          dict(width=tile[0], height=tile[1], chunk=5, variant=tile[2]))
    _compare_f32(orc, p, pop, h, s)


# --------------------------------------------------------------------------
# Launch shapes give bitwise identical results; determinism
# --------------------------------------------------------------------------

def test_launch_shapes_bitwise_identical(tlb):
    w, C, h = _wet_case(200, 50)
    ref = None
    for width in (64, 128, 256):
        for chunk in (1, 5, 50):
            for hold in (0, 1):
                _note(f"shape width={width} chunk={chunk} variant={hold}")
                s = _gsim(tlb, w, tlb.TLB_F64, dict(width=width, chunk=chunk, variant=hold))
                s.set_wetting_both(h)
                s.init_equilibrium(C)
                s.step(40)
                got = np.stack([s.populations(k) for k in range(3)])
                if ref is None:
                    ref = got
                else:
                    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_d3q19_launch_shapes_bitwise_identical(tlb, prec):
    """For each variant (plane z pulled again, held from the previous plane, or held with the loads of
    plane z+2 in flight; the last for FP32 storage) both tiles and every chunk give the same bits.  The variants are separate kernels in which the compiler may fuse a
    different set of multiply-adds, so across variants the results agree to rounding."""
    w, C, h = _wet_case(70, 19, 11, lattice=1, walls=1)
    P = tlb.TLB_F64 if prec == "f64" else tlb.TLB_F32
    per_variant = {}
    for variant in ((0, 1, 2) if prec == "f32" else (0, 1)):
        for tile in ((32, 8), (64, 4)):
            for chunk in (1, 4, 11):
                _note(f"d3q19 {prec} tile {tile} chunk {chunk} variant {variant}")
                s = _gsim(tlb, w, P, dict(width=tile[0], height=tile[1], chunk=chunk, variant=variant))
                s.set_wetting_both(h)
                s.init_equilibrium(C)
                s.step(12)
                got = s.all_populations()
                s.close()
                if variant not in per_variant:
                    per_variant[variant] = got
                else:
                    assert np.array_equal(got, per_variant[variant]), (tile, chunk, variant)
    ref = per_variant[0]
    tol = 1e-13 * np.abs(ref).max() if prec == "f64" else 1e-6
    for variant in per_variant:
        assert np.abs(per_variant[variant] - ref).max() <= tol, variant


def test_launch_validation(tlb):
    w2, _, _ = _wet_case(40, 20)
    w3, _, _ = _wet_case(20, 12, 8, lattice=1)
    s2 = _gsim(tlb, w2, tlb.TLB_F64)
    s3 = _gsim(tlb, w3, tlb.TLB_F32)
    s3d = _gsim(tlb, w3, tlb.TLB_F64)
    for s, bad in ((s2, dict(width=96, chunk=4, variant=0)), (s2, dict(width=64, chunk=-1, variant=0)),
                   (s2, dict(width=64, chunk=4, variant=2)),  # the pipelined sweep is a D3Q19 variant
                   (s3, dict(width=64, height=8, chunk=4, variant=0)), (s3, dict(width=32, height=8, chunk=4, variant=3)),
                   (s3d, dict(width=32, height=8, chunk=4, variant=2))):  # pipelined sweep: FP32 storage only
        with pytest.raises(tlb.TLBError):
            s.set_launch(**bad)
    s3.set_launch(width=32, height=8, chunk=4, variant=2)
    s2.close()
    s3.close()
    s3d.close()


def test_run_twice_is_deterministic_and_restart_continues(tlb):
    w, C, h = _wet_case(96, 40)
    runs = []
    for _ in range(2):
        s = _gsim(tlb, w, tlb.TLB_F32)
        s.set_wetting_both(h)
        s.init_equilibrium(C)
        s.step(100)
        runs.append(s.all_populations())
    assert np.array_equal(runs[0], runs[1])
    # checkpoint / restart: 50 steps, save, load into a new sim, 50 more == 100 steps, bit for bit
    a = _gsim(tlb, w, tlb.TLB_F64)
    a.set_wetting_both(h)
    a.init_equilibrium(C)
    a.step(50)
    raw, step = a.save_state()
    pops50 = a.all_populations()
    a.step(50)
    b = _gsim(tlb, w, tlb.TLB_F64)
    b.set_wetting_both(h)
    b.load_state(raw, step)
    b.step(50)
    assert np.array_equal(a.all_populations(), b.all_populations())
    assert b.diagnostics()["step"] == 100
    # restart from exported populations (s_t in absolute terms): equal to rounding
    c = _gsim(tlb, w, tlb.TLB_F64)
    c.set_wetting_both(h)
    for sp in range(3):
        c.set_populations(sp, pops50[sp])
    c.step(50)
    assert np.abs(c.all_populations() - a.all_populations()).max() < 1e-14


# --------------------------------------------------------------------------
# Invariants on the GPU
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lattice", [0, 1])
def test_gpu_conservation_and_fixed_point(tlb, lattice):
    if lattice == 0:
        w, C, h = _wet_case(120, 50)
    else:
        w, C, h = _wet_case(24, 20, 16, lattice=1)
    s = _gsim(tlb, w, tlb.TLB_F64)
    s.set_wetting_both(h)
    s.init_equilibrium(C)
    d0 = s.diagnostics()
    s.step(200)
    d1 = s.diagnostics()
    for m in range(3):
        assert abs(d1["mass"][m] - d0["mass"][m]) <= 1e-12 * max(1.0, abs(d0["mass"][m]))
    assert d1["nonfinite"] == 0 and d1["step"] == 200
    # uniform state at rest between neutral walls: fixed point
    U = np.zeros_like(C)
    U[0], U[1], U[2] = 0.25, 0.45, 0.30
    s2 = _gsim(tlb, w, tlb.TLB_F64)
    s2.init_equilibrium(U)
    a = s2.all_populations()
    s2.step(20)
    assert np.abs(s2.all_populations() - a).max() < 1e-14


def test_nan_is_detected(tlb):
    w, C, _ = _wet_case(64, 32, walls=0)
    s = _gsim(tlb, w, tlb.TLB_F64)
    s.init_equilibrium(C)
    pop = s.populations(1)
    pop[3, 100] = np.nan
    s.set_populations(1, pop)
    d = s.diagnostics(allow_nan=True)
    assert d["nonfinite"] >= 1
    rc = tlb.tlb_set_check_every(s.handle, 1)
    assert rc == 0
    assert tlb.tlb_step(s.handle, 1) == tlb.TLB_ENAN


# --------------------------------------------------------------------------
# Full-size workloads in the benchmark's launch configuration
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spinodal_1024_full_size_few_steps(tlb, orc, prec):
    """1024x1024 spinodal at full size, default launch shape: every node after 3 steps."""
    w = inputs.spinodal_2d(1024, 3)
    C = w["C"]()
    P = tlb.TLB_F64 if prec == "f64" else tlb.TLB_F32
    p, pop, s = _run_both(tlb, orc, w, C, None, 3, P)
    if prec == "f64":
        _compare_f64(orc, p, pop, None, s)
    else:
        _compare_f32(orc, p, pop, None, s, tol=1e-6)


def _window(C, dims, centre, W):
    nx, ny, nz = dims
    xs = (np.arange(W) + centre[0] - W // 2) % nx
    ys = (np.arange(W) + centre[1] - W // 2) % ny
    zs = (np.arange(W) + centre[2] - W // 2) % nz
    Cg = C.reshape(3, nz, ny, nx)
    sub = Cg[:, zs][:, :, ys][:, :, :, xs]
    return sub.reshape(3, -1)


def test_spinodal_256cube_full_size_sampled(tlb, orc):
    """256^3 D3Q19 FP32 at full size: sampled nodes after 2 steps, each recomputed by the oracle on a
    periodic 16^3 window around it (the update reaches 2 nodes per step plus 1 for the initial stencil,
    so the window's own wrap-around cannot reach the centre)."""
    steps = 2
    w = inputs.spinodal_3d(256, steps)
    C = w["C"]()
    _note("256^3 fp32 full size")
    s = _gsim(tlb, w, tlb.TLB_F32)
    s.init_equilibrium(C)
    s.step(steps)
    gpu_pops = [s.populations(k) for k in range(3)]
    rng = np.random.default_rng(77)
    W = 16
    pw = _oparams(orc, w).replace(nx=W, ny=W, nz=W)
    for _ in range(6):
        c = rng.integers(0, 256, 3)
        sub = _window(C, (256, 256, 256), c, W)
        pop = orc.init_equilibrium(pw, sub)
        orc.step(pw, pop, steps)
        ic = W // 2 + W * (W // 2 + W * (W // 2))
        n = c[0] + 256 * (c[1] + 256 * c[2])
        for sp in range(3):
            assert np.abs(gpu_pops[sp][:, n] - pop[sp][:, ic]).max() < 2e-7, (c, sp)


def _window2(C, nx, ny, centre, W):
    xs = (np.arange(W) + centre[0] - W // 2) % nx
    ys = (np.arange(W) + centre[1] - W // 2) % ny
    return C.reshape(3, ny, nx)[:, ys][:, :, xs].reshape(3, -1)


def test_d2q9_state_beyond_32bit_offsets_sampled(tlb, orc):
    """6144^2 D2Q9 FP64 (8.2 GB per state, past the 4 GiB one buffer descriptor can address): C_m at
    seeded nodes after 3 steps against the oracle on a periodic 24^2 window around each (the update
    reaches 2 nodes per step plus 1 for the initial stencil, less than the half-width 12)."""
    n, steps, W = 6144, 3, 24
    w = inputs.spinodal_2d(n, steps)
    C = w["C"]()
    _note("6144^2 fp64 beyond 32-bit offsets")
    s = _gsim(tlb, w, tlb.TLB_F64)
    assert s.state_bytes() > 2 ** 32
    s.init_equilibrium(C)
    s.step(steps)
    got = np.stack([s.field(f) for f in ("C1", "C2", "C3")])
    s.close()
    pw = _oparams(orc, w).replace(nx=W, ny=W)
    rng = np.random.default_rng(78)
    ic = W // 2 + W * (W // 2)
    for c in [(0, 0), (n - 1, n - 1)] + [tuple(rng.integers(0, n, 2)) for _ in range(6)]:
        pop = orc.init_equilibrium(pw, _window2(C, n, n, c, W))
        orc.step(pw, pop, steps)
        F = orc.fields(pw, pop)
        node = c[0] + n * c[1]
        for m, f in enumerate(("C1", "C2", "C3")):
            assert abs(got[m][node] - F[f][ic]) <= 1e-12, (c, f)


def test_d3q19_state_beyond_32bit_offsets_sampled(tlb, orc):
    """448^3 D3Q19 FP32 (20.5 GB per state; a species-major state stopped at 383^3): C_m at seeded nodes
    after 2 steps against the oracle on periodic 16^3 windows."""
    n, steps, W = 448, 2, 16
    w = inputs.spinodal_3d(n, steps)
    C = w["C"]()
    _note("448^3 fp32 beyond 32-bit offsets")
    s = _gsim(tlb, w, tlb.TLB_F32)
    s.init_equilibrium(C)
    s.step(steps)
    got = np.stack([s.field(f) for f in ("C1", "C2", "C3")])
    s.close()
    pw = _oparams(orc, w).replace(nx=W, ny=W, nz=W)
    rng = np.random.default_rng(79)
    ic = W // 2 + W * (W // 2 + W * (W // 2))
    for c in [(0, 0, 0), (n - 1, n - 1, n - 1)] + [tuple(rng.integers(0, n, 3)) for _ in range(4)]:
        pop = orc.init_equilibrium(pw, _window(C, (n, n, n), c, W))
        orc.step(pw, pop, steps)
        F = orc.fields(pw, pop)
        node = c[0] + n * (c[1] + n * c[2])
        for m, f in enumerate(("C1", "C2", "C3")):
            assert abs(got[m][node] - F[f][ic]) <= 1e-6, (c, f)


def _pull_np(pop, lattice, dims, walls):
    """Propagation of s [NC][Q][N] with half-way bounce-back in y, in numpy: s'_i(r) = s_i(r - e_i), or
    s_opp(i)(r) where r - e_i is beyond a wall."""
    from oracle import torch_ref

    nx, ny, nz = dims
    E = torch_ref.E3 if lattice == 1 else [(e[0], e[1], 0) for e in torch_ref.E]
    opp = torch_ref.OPP3 if lattice == 1 else torch_ref.OPP
    a = pop.reshape(pop.shape[0], len(E), nz, ny, nx)
    out = np.empty_like(a)
    for i, (ex, ey, ez) in enumerate(E):
        out[:, i] = np.roll(a[:, i], shift=(ez, ey, ex), axis=(1, 2, 3))
        if walls and ey == 1:
            out[:, i, :, 0, :] = a[:, opp[i], :, 0, :]
        if walls and ey == -1:
            out[:, i, :, ny - 1, :] = a[:, opp[i], :, ny - 1, :]
    return out.reshape(pop.shape)


@pytest.mark.parametrize("lattice,dims,walls,launch", [
    (0, (70, 23, 1), 1, dict(width=64, chunk=5)), (0, (300, 9, 1), 0, dict(width=256, chunk=4)),
    (1, (37, 21, 13), 1, dict(width=32, height=8, chunk=4)), (1, (9, 70, 5), 0, dict(width=64, height=4, chunk=3))])
def test_stream_only_is_propagation(tlb, lattice, dims, walls, launch):
    """tlb_stream_only moves the populations exactly as propagation with half-way bounce-back does
    (bit for bit), without touching the step counter."""
    w, C, h = _wet_case(*dims, lattice=lattice, walls=walls, seed=4)
    s = _gsim(tlb, w, tlb.TLB_F64, dict(launch, variant=0))
    if h is not None:
        s.set_wetting_both(h)
    s.init_equilibrium(C)
    s.step(3)
    before = s.all_populations()
    s.stream_only(2)
    after = s.all_populations()
    want = _pull_np(_pull_np(before, lattice, dims, walls), lattice, dims, walls)
    assert np.array_equal(after, want)
    assert s.diagnostics()["step"] == 3
    s.close()


# --------------------------------------------------------------------------
# Diffusive Cahn-Hilliard (no advection) and the interface diagnostics
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,walls", [(0, 1), (0, 0), (1, 1)])
def test_no_advection_fp64(tlb, orc, lattice, walls):
    """g^eq and k^eq without velocity terms (tlb_params.no_advection), against the oracle, with a
    non-zero initial flow so that the dropped terms matter."""
    dims = (40, 27, 1) if lattice == 0 else (20, 17, 9)
    w, C, h = _wet_case(*dims, lattice=lattice, walls=walls, seed=7)
    w["no_advection"] = 1
    _note(f"no advection lattice={lattice} walls={walls}")
    p = _oparams(orc, w)
    N = p.N
    rng = np.random.default_rng(8)
    u = rng.uniform(-0.02, 0.02, size=(p.D, N))
    pop = orc.init_equilibrium(p, C, u, h)
    orc.step(p, pop, 40, h)
    s = _gsim(tlb, w, tlb.TLB_F64)
    if h is not None:
        s.set_wetting_both(h)
    s.init_equilibrium(C, u)
    s.step(40)
    _compare_f64(orc, p, pop, h, s)


@pytest.mark.parametrize("lattice", [0, 1])
def test_interface_diagnostics_match_oracle_fields(tlb, orc, lattice):
    """tlb_diag.interface[m] = sum over nodes of C_m^2 (1 - C_m)^2 of the current state."""
    dims = (50, 31, 1) if lattice == 0 else (18, 14, 11)
    w, C, h = _wet_case(*dims, lattice=lattice, walls=1, seed=9)
    p, pop, s = _run_both(tlb, orc, w, C, h, 25, tlb.TLB_F64)
    F = orc.fields(p, pop, h)
    d = s.diagnostics()
    for m, name in enumerate(("C1", "C2", "C3")):
        want = float(np.sum(F[name] ** 2 * (1 - F[name]) ** 2))
        assert d["interface"][m] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("lattice,walls", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_mass_momentum_and_max_speed_match_oracle_fields(tlb, orc, lattice, walls):
    """tlb_diag.mass, momentum and max_speed of the current state against sums of the oracle's moment
    fields (Sec. IV, eq. lbconstraint): sum rho, sum phi, sum psi, sum rho v_a and max |v|, FP64, from a
    state with a seeded velocity field so that every momentum component is non-trivial."""
    dims = (50, 31, 1) if lattice == 0 else (18, 14, 11)
    w, C, h = _wet_case(*dims, lattice=lattice, walls=walls, seed=13)
    D = 2 if lattice == 0 else 3
    N = dims[0] * dims[1] * dims[2]
    u = 0.03 * np.random.default_rng(14).uniform(-1.0, 1.0, size=(D, N))
    _note(f"diagnostics vs oracle lattice={lattice} walls={walls}")
    p = _oparams(orc, w)
    pop = orc.init_equilibrium(p, C, u, h)
    orc.step(p, pop, 15, h)
    s = _gsim(tlb, w, tlb.TLB_F64)
    if h is not None:
        s.set_wetting_both(h)
    s.init_equilibrium(C, u)
    s.step(15)
    d = s.diagnostics()
    F = orc.fields(p, pop, h)
    for m, name in enumerate(("rho", "phi", "psi")):
        want = float(F[name].sum())
        assert abs(d["mass"][m] - want) <= 1e-12 * float(np.abs(F[name]).sum()), (name, d["mass"][m], want)
    for a, name in enumerate(("ux", "uy", "uz")[:D]):
        j = F["rho"] * F[name]
        want = float(j.sum())
        assert abs(d["momentum"][a] - want) <= 1e-12 * float(np.abs(j).sum()), (name, d["momentum"][a], want)
    if D == 2:
        assert d["momentum"][2] == 0.0
    speed = np.sqrt(sum(F[name] ** 2 for name in ("ux", "uy", "uz")[:D]))
    assert d["max_speed"] == pytest.approx(float(speed.max()), rel=1e-12)
    assert d["nonfinite"] == 0


# --------------------------------------------------------------------------
# Multiple relaxation times for f (tlb_params.collision = TLB_MRT)
# --------------------------------------------------------------------------
_MRT_LAUNCH = {0: [dict(width=64, chunk=5, variant=0), dict(width=128, chunk=7, variant=1),
                   dict(width=256, chunk=3, variant=0)],
               1: [dict(width=32, height=8, chunk=4, variant=0), dict(width=64, height=4, chunk=3, variant=1)]}


@pytest.mark.parametrize("lattice,walls,li", [(0, 1, 0), (0, 1, 1), (0, 0, 2), (1, 1, 0), (1, 0, 1)])
def test_mrt_fp64(tlb, orc, lattice, walls, li):
    """Distinct stress, bulk and ghost rates against the oracle's M^-1 S M collision, with an initial flow
    (ragged strips and tiles, walls with wetting)."""
    dims = (70, 23, 1) if lattice == 0 else (37, 21, 9)
    w, C, h = _wet_case(*dims, lattice=lattice, walls=walls, seed=9, tau=(0.8, 0.9, 0.8))
    w.update(collision=1, tau_bulk=0.65, tau_ghost=1.3)
    launch = _MRT_LAUNCH[lattice][li]
    _note(f"mrt fp64 lattice={lattice} walls={walls} launch={launch}")
    p = _oparams(orc, w)
    u = np.random.default_rng(10).uniform(-0.02, 0.02, size=(p.D, p.N))
    pop = orc.init_equilibrium(p, C, u, h)
    orc.step(p, pop, 30, h)
    s = _gsim(tlb, w, tlb.TLB_F64, launch)
    if h is not None:
        s.set_wetting_both(h)
    s.init_equilibrium(C, u)
    s.step(30)
    _compare_f64(orc, p, pop, h, s)


@pytest.mark.parametrize("lattice", [0, 1])
def test_mrt_fp32(tlb, orc, lattice):
    dims = (64, 40, 1) if lattice == 0 else (24, 20, 12)
    w, C, h = _wet_case(*dims, lattice=lattice, walls=1, seed=11, tau=(0.8, 0.9, 0.8))
    w.update(collision=1, tau_bulk=1.2, tau_ghost=0.7)
    p, pop, s = _run_both(tlb, orc, w, C, h, 200, tlb.TLB_F32)
    _compare_f32(orc, p, pop, h, s)


@pytest.mark.parametrize("lattice", [0, 1])
def test_mrt_with_equal_rates_is_bgk_on_the_gpu(tlb, lattice):
    dims = (40, 19, 1) if lattice == 0 else (20, 13, 7)
    w, C, h = _wet_case(*dims, lattice=lattice, walls=1, seed=12, tau=(0.85, 0.9, 0.8))
    out = []
    for col in (0, 1):
        w2 = dict(w, collision=col, tau_bulk=0.85, tau_ghost=0.85)
        s = _gsim(tlb, w2, tlb.TLB_F64)
        s.set_wetting_both(h)
        s.init_equilibrium(C)
        s.step(25)
        out.append(s.all_populations())
        s.close()
    assert np.abs(out[0] - out[1]).max() <= 1e-13 * np.abs(out[0]).max()


def test_mrt_is_rejected_by_the_batch_and_the_reverse_step(tlb):
    import ctypes

    w, C, h = _wet_case(24, 16, walls=1, seed=13)
    w.update(collision=1, tau_bulk=0.7, tau_ghost=1.1)
    p = tlb.make_params(prec=tlb.TLB_F64, **{k: v for k, v in w.items() if k in _PKEYS})
    ps = (tlb.tlb_params * 1)(p)
    hb = ctypes.c_void_p()
    assert tlb.tlb_batch_create(ps, 1, None, ctypes.byref(hb)) == tlb.TLB_EINVAL
    s = tlb.Sim(p)
    s.init_equilibrium(C)
    n = s.state_bytes()
    import torch

    u = torch.zeros(n // 8, dtype=torch.float64, device="cuda")
    l0, l1 = torch.zeros_like(u), torch.zeros_like(u)
    assert tlb.tlb_adjoint_step_dev(s.handle, u.data_ptr(), l0.data_ptr(), l1.data_ptr(), None, None) == \
        tlb.TLB_EINVAL
    s.close()
