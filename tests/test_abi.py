"""The C ABI library loads and exports every symbol include/tlb.h declares.

No test here launches a kernel: argument validation happens before any HIP
call, so the invalid-argument paths run without a GPU.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlb.h")


def _has_gpu():
    """A valid create would reach the device; without one it fails there (not at validation)."""
    return os.path.exists("/dev/kfd")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tlb_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for must in ("tlb_create", "tlb_destroy", "tlb_step", "tlb_init_equilibrium", "tlb_get_field",
                 "tlb_set_wetting", "tlb_diagnostics", "tlb_get_populations", "tlb_set_populations"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1511_02155_amd import tlb

    lib = ctypes.CDLL(tlb.LIB_PATH)
    declared = _declared()
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(tlb.EXPORTS) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", tlb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(tlb_[a-z0-9_]+)\b", out))
    assert set(declared) <= exported


def test_library_is_built_for_gfx950():
    from paper_1511_02155_amd import tlb

    blob = open(tlb.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_status_strings():
    from paper_1511_02155_amd import tlb

    assert tlb.tlb_status_str(0) == b"ok"
    assert tlb.tlb_status_str(-1) == b"invalid argument"
    assert tlb.tlb_version() >= 100


@pytest.mark.parametrize("bad", [
    dict(tau_f=0.5), dict(tau_g=0.4), dict(tau_k=-1.0), dict(kappa=(0.01, 0.0, 0.01)),
    dict(kappa=(0.01, 0.01, -0.1)), dict(alpha=0.0), dict(nx=2), dict(ny=2), dict(nz=2),
    dict(prec=7), dict(lattice=5), dict(walls_y=2), dict(alpha=float("nan")), dict(no_advection=2),
    dict(collision=2), dict(collision=1, tau_bulk=0.5), dict(collision=1, tau_ghost=0.3),
    dict(collision=1, tau_bulk=float("inf")),
])
def test_create_rejects_invalid_parameters(bad):
    from paper_1511_02155_amd import tlb

    kw = dict(lattice=tlb.TLB_D2Q9, nx=8, ny=8, nz=1)
    kw.update(bad)
    if "nz" in bad:
        kw["lattice"] = tlb.TLB_D3Q19
    p = tlb.make_params(**kw)
    h = ctypes.c_void_p()
    assert tlb.tlb_create(ctypes.byref(p), None, ctypes.byref(h)) == tlb.TLB_EINVAL
    assert not h.value


def test_create_rejects_lattices_beyond_32bit_offsets():
    """Every buffer descriptor covers at most 4 GiB - 256 B: one population array on D2Q9, one z plane of
    all populations on D3Q19.  Shapes beyond that are rejected before any device call; shapes within it
    pass validation (on a machine without a GPU the call then fails at the device, not with EINVAL)."""
    from paper_1511_02155_amd import tlb

    def rc(*a, **k):
        p = tlb.make_params(*a, **k)
        h = ctypes.c_void_p()
        return tlb.tlb_create(ctypes.byref(p), None, ctypes.byref(h))

    # one D2Q9 FP64 array of 32768 x 16385 nodes is 4 GiB + 256 KiB; 23170^2 is the largest square
    assert rc(tlb.TLB_D2Q9, 32768, 16385, prec=tlb.TLB_F64) == tlb.TLB_EINVAL
    assert rc(tlb.TLB_D2Q9, 32768, 32768, prec=tlb.TLB_F32) == tlb.TLB_EINVAL
    # one D3Q19 FP32 plane of 8192 x 4096 nodes holds 57 x 2^25 values = 7.1 GiB
    assert rc(tlb.TLB_D3Q19, 8192, 4096, 3, prec=tlb.TLB_F32) == tlb.TLB_EINVAL
    assert rc(tlb.TLB_D3Q19, 4096, 4096, 3, prec=tlb.TLB_F64) == tlb.TLB_EINVAL
    if not _has_gpu():
        # beyond the former whole-state limit of 4 GiB, within the per-array / per-plane one
        assert rc(tlb.TLB_D2Q9, 6144, 6144, prec=tlb.TLB_F64) != tlb.TLB_EINVAL
        assert rc(tlb.TLB_D3Q19, 448, 448, 448, prec=tlb.TLB_F32) != tlb.TLB_EINVAL


def test_null_handles_are_rejected():
    from paper_1511_02155_amd import tlb

    assert tlb.tlb_step(None, 1) == tlb.TLB_EINVAL
    assert tlb.tlb_destroy(None) == tlb.TLB_EINVAL
    assert tlb.tlb_get_field(None, 0, None) == tlb.TLB_EINVAL
    assert tlb.tlb_bytes_per_node(None) == 0.0


def test_create_rejects_invalid_component_counts():
    """ncomp in 3 .. TLB_MAX_COMP (0 = 3) on either lattice, every kappa_m > 0."""
    from paper_1511_02155_amd import tlb

    def rc(p):
        h = ctypes.c_void_p()
        r = tlb.tlb_create(ctypes.byref(p), None, ctypes.byref(h))
        assert r != tlb.TLB_OK or h.value  # a successful create would need a GPU; only errors are expected here
        return r

    for lat, nz in ((tlb.TLB_D2Q9, 1), (tlb.TLB_D3Q19, 8)):
        for n, bad in ((6, None), (2, None), (4, 0.0), (5, float("nan"))):
            p = tlb.make_params(lattice=lat, nx=8, ny=8, nz=nz, kappa=(0.01,) * 5)
            p.ncomp = n
            if bad is not None:
                p.kappa_hi[n - 4] = bad
            assert rc(p) == tlb.TLB_EINVAL, (lat, n, bad)
        if not _has_gpu():
            p = tlb.make_params(lattice=lat, nx=8, ny=8, nz=nz, kappa=(0.01,) * 4)
            assert rc(p) != tlb.TLB_EINVAL
    with pytest.raises(ValueError):
        tlb.make_params(lattice=tlb.TLB_D2Q9, nx=8, ny=8, kappa=(0.01,) * 6)
