"""C-ABI checks that need no GPU: the library loads, exports exactly the
entry points include/lbm.h declares, and validates descriptions."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"LBM_API\s+[\w\s\*]*?\b(lbm_\w+)\s*\(", txt)))


def _lbm():
    from paper_2302_04120_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        pytest.skip("liblbm.so not built")
    return lbm


def test_header_declares_the_binding_exports():
    lbm = _lbm()
    assert _declared() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol():
    lbm = _lbm()
    out = subprocess.check_output(["nm", "-D", "--defined-only", lbm.LIB_PATH], text=True)
    exported = sorted(l.split()[-1] for l in out.splitlines() if l.split()[-1].startswith("lbm_"))
    assert exported == _declared()
    L = lbm.lib()
    for name in _declared():
        assert getattr(L, name) is not None


def _desc(lbm, **kw):
    d = lbm.Desc()
    d.lattice = kw.get("lattice", lbm.LBM_D2Q9_PHASE)
    d.nx, d.ny, d.batch = kw.get("nx", 64), kw.get("ny", 64), kw.get("batch", 1)
    d.prec = kw.get("prec", lbm.LBM_FP32_DEV)
    for i, v in enumerate(kw.get("bc", (0, 0, 0, 0))):
        d.bc[i] = v
    d.flags = kw.get("flags", 1)
    return d


def test_query_bytes_layout_and_validation():
    lbm = _lbm()
    L = lbm.lib()
    n = C.c_size_t()
    d = _desc(lbm)
    assert L.lbm_query_bytes(C.byref(d), C.byref(n)) == lbm.LBM_OK
    N = 64 * 64
    # two buffers of 19 FP32 planes + (phi u) + 7 FP64 staging planes at least
    assert n.value >= (2 * 19 + 2) * N * 4 + 7 * N * 8
    d64 = _desc(lbm, prec=lbm.LBM_FP64)
    n64 = C.c_size_t()
    assert L.lbm_query_bytes(C.byref(d64), C.byref(n64)) == lbm.LBM_OK
    assert n64.value > n.value
    bad = [
        _desc(lbm, nx=0),
        _desc(lbm, prec=7),
        _desc(lbm, lattice=99),
        _desc(lbm, bc=(2, 3, 0, 0)),  # inlet/outlet not supported for the phase lattice
        _desc(lbm, lattice=lbm.LBM_D2Q9_D2Q5, bc=(2, 0, 0, 0)),
        _desc(lbm, lattice=lbm.LBM_D2Q9_D2Q5, flags=0),
        _desc(lbm, lattice=lbm.LBM_D1Q2, nx=101, ny=1, prec=lbm.LBM_FP32_DEV, bc=(4, 4, 0, 0)),
        _desc(lbm, lattice=lbm.LBM_D1Q2, nx=2000, ny=1, prec=lbm.LBM_FP64, bc=(4, 4, 0, 0)),
    ]
    for d in bad:
        assert L.lbm_query_bytes(C.byref(d), C.byref(n)) in (lbm.LBM_E_ARG, lbm.LBM_E_UNSUPPORTED)
    ok = _desc(lbm, lattice=lbm.LBM_D1Q3, nx=101, ny=1, prec=lbm.LBM_FP64, bc=(4, 4, 0, 0))
    assert L.lbm_query_bytes(C.byref(ok), C.byref(n)) == lbm.LBM_OK
    assert L.lbm_create(None, None) == lbm.LBM_E_ARG
    assert L.lbm_query_bytes(C.byref(ok), None) == lbm.LBM_E_ARG


def test_fp64_arithmetic_mode_layout_and_validation():
    """FP32 storage with FP64 step arithmetic: the FP32 layout, two-phase D2Q9 only."""
    lbm = _lbm()
    L = lbm.lib()
    n32, na = C.c_size_t(), C.c_size_t()
    assert L.lbm_query_bytes(C.byref(_desc(lbm)), C.byref(n32)) == lbm.LBM_OK
    d = _desc(lbm, prec=lbm.LBM_FP32_DEV_ARITH64)
    assert L.lbm_query_bytes(C.byref(d), C.byref(na)) == lbm.LBM_OK
    assert na.value == n32.value
    for lat in (lbm.LBM_D2Q9_D2Q5, lbm.LBM_D3Q19, lbm.LBM_D3Q19_PHASE):
        d = _desc(lbm, lattice=lat, nx=32, ny=16, prec=lbm.LBM_FP32_DEV_ARITH64)
        d.nz = 8
        assert L.lbm_query_bytes(C.byref(d), C.byref(na)) == lbm.LBM_E_UNSUPPORTED
    assert lbm.PRECISIONS["fp32_arith64"] == lbm.LBM_FP32_DEV_ARITH64


def test_create_rejects_small_or_misaligned_buffer():
    lbm = _lbm()
    L = lbm.lib()
    d = _desc(lbm)
    h = C.c_void_p()
    d.dev_buf = C.c_void_p(0x100000)
    d.dev_buf_bytes = 16
    assert L.lbm_create(C.byref(d), C.byref(h)) == lbm.LBM_E_ARG
    n = C.c_size_t()
    L.lbm_query_bytes(C.byref(d), C.byref(n))
    d.dev_buf_bytes = n.value
    d.dev_buf = C.c_void_p(0x100004)
    assert L.lbm_create(C.byref(d), C.byref(h)) == lbm.LBM_E_ARG
    assert not h.value


def test_product_binding_refuses_without_gpu():
    lbm = _lbm()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        lbm.Lattice("phase", 16, 16)


def test_channel_description_validation():
    """D2Q9_D2Q5 descriptions: the D2Q9 thermal flag needs THERMAL, the
    symmetry plane only sits at y+ above a wall, fixed-temperature side walls
    need the thermal field."""
    lbm = _lbm()
    L = lbm.lib()
    n = C.c_size_t()
    cases = [((1 | 2 | 4), (2, 3, 1, 1), lbm.LBM_OK),
             ((1 | 2), (2, 3, 1, 5), lbm.LBM_OK),
             ((1 | 2 | 4), (2, 3, 1, 5), lbm.LBM_OK),
             ((1 | 2), (4, 4, 1, 1), lbm.LBM_OK),
             ((1 | 4), (2, 3, 1, 1), lbm.LBM_E_ARG),
             ((1 | 2), (0, 0, 5, 1), lbm.LBM_E_UNSUPPORTED),
             ((1 | 2), (0, 0, 5, 5), lbm.LBM_E_UNSUPPORTED),
             (1, (4, 4, 1, 1), lbm.LBM_E_ARG),
             ((1 | 2), (0, 0, 1, 6), lbm.LBM_E_ARG)]
    for flags, bc, want in cases:
        d = _desc(lbm, lattice=lbm.LBM_D2Q9_D2Q5, nx=64, ny=12, bc=bc, flags=flags)
        assert L.lbm_query_bytes(C.byref(d), C.byref(n)) == want, (flags, bc)
    # D2Q9 thermal planes: 9 + 9 per buffer instead of 9 + 5
    d5 = _desc(lbm, lattice=lbm.LBM_D2Q9_D2Q5, nx=64, ny=12, bc=(2, 3, 1, 1), flags=3)
    d9 = _desc(lbm, lattice=lbm.LBM_D2Q9_D2Q5, nx=64, ny=12, bc=(2, 3, 1, 1), flags=7)
    n5, n9 = C.c_size_t(), C.c_size_t()
    L.lbm_query_bytes(C.byref(d5), C.byref(n5))
    L.lbm_query_bytes(C.byref(d9), C.byref(n9))
    # (each plane also carries the layout's inter-plane padding, under 64 Ki elements)
    assert 2 * 4 * 64 * 12 * 4 <= n9.value - n5.value < 2 * 4 * (64 * 12 + 65536) * 4


def test_d3q19_description_validation():
    """D3Q19: nz >= 1, each axis periodic or walls on both sides, no flags but
    FLOW; the 2D lattices refuse nz > 1 and z boundaries.  The buffer holds
    two states of 19 planes over nx ny nz batch nodes."""
    lbm = _lbm()
    L = lbm.lib()
    n = C.c_size_t()

    def d3(nz=8, bc=(0, 0, 1, 1), bcz=(1, 1), flags=0, prec=lbm.LBM_FP32_DEV, batch=1):
        d = _desc(lbm, lattice=lbm.LBM_D3Q19, nx=32, ny=16, bc=bc, flags=flags, prec=prec,
                  batch=batch)
        d.nz = nz
        d.bc_z[0], d.bc_z[1] = bcz
        return d

    for d, want in [(d3(), lbm.LBM_OK), (d3(bc=(1, 1, 1, 1)), lbm.LBM_OK),
                    (d3(flags=1), lbm.LBM_OK), (d3(nz=1, bcz=(0, 0)), lbm.LBM_OK),
                    (d3(nz=0), lbm.LBM_E_ARG), (d3(flags=2), lbm.LBM_E_ARG),
                    (d3(bc=(2, 3, 1, 1)), lbm.LBM_E_UNSUPPORTED),
                    (d3(bc=(1, 0, 1, 1)), lbm.LBM_E_UNSUPPORTED),
                    (d3(bcz=(1, 0)), lbm.LBM_E_UNSUPPORTED),
                    (d3(bcz=(5, 5)), lbm.LBM_E_UNSUPPORTED)]:
        assert L.lbm_query_bytes(C.byref(d), C.byref(n)) == want, (d.nz, list(d.bc), list(d.bc_z))
    N = 32 * 16 * 8
    assert L.lbm_query_bytes(C.byref(d3()), C.byref(n)) == lbm.LBM_OK
    assert n.value >= 2 * 19 * N * 4 + 8 * N * 8
    n2 = C.c_size_t()
    assert L.lbm_query_bytes(C.byref(d3(batch=3)), C.byref(n2)) == lbm.LBM_OK
    assert n2.value >= 3 * 2 * 19 * N * 4
    twod = _desc(lbm)
    twod.nz = 4
    assert L.lbm_query_bytes(C.byref(twod), C.byref(n)) == lbm.LBM_E_ARG
    twod.nz, twod.bc_z[0] = 1, 1
    assert L.lbm_query_bytes(C.byref(twod), C.byref(n)) == lbm.LBM_E_ARG
    # a grid whose 64 x 4 tiles do not fit the 32-bit launch grid
    big = d3(nz=1 << 14)
    big.nx, big.ny = 4096, 4096
    assert L.lbm_query_bytes(C.byref(big), C.byref(n)) == lbm.LBM_E_ARG


def test_d3q19_phase_description_validation():
    """D3Q19_PHASE: each axis periodic or walls, no flags; its buffer holds two
    states of h 19 + z 19 (+ the low part of h_0 in FP32) + (phi u) 3 planes
    and one phi plane."""
    lbm = _lbm()
    L = lbm.lib()
    n = C.c_size_t()

    def p3(nz=6, bc=(0, 0, 1, 1), bcz=(0, 0), flags=0, prec=lbm.LBM_FP32_DEV):
        d = _desc(lbm, lattice=lbm.LBM_D3Q19_PHASE, nx=32, ny=8, bc=bc, flags=flags, prec=prec)
        d.nz = nz
        d.bc_z[0], d.bc_z[1] = bcz
        return d

    for d, want in [(p3(), lbm.LBM_OK), (p3(bc=(1, 1, 1, 1), bcz=(1, 1)), lbm.LBM_OK),
                    (p3(flags=1), lbm.LBM_E_ARG), (p3(nz=0), lbm.LBM_E_ARG),
                    (p3(bc=(2, 3, 0, 0)), lbm.LBM_E_UNSUPPORTED),
                    (p3(bcz=(0, 1)), lbm.LBM_E_UNSUPPORTED)]:
        assert L.lbm_query_bytes(C.byref(d), C.byref(n)) == want, (list(d.bc), list(d.bc_z), d.flags)
    N = 32 * 8 * 6
    assert L.lbm_query_bytes(C.byref(p3()), C.byref(n)) == lbm.LBM_OK
    assert n.value >= 2 * (39 + 3) * N * 4 + N * 4 + 8 * N * 8
    n64 = C.c_size_t()
    assert L.lbm_query_bytes(C.byref(p3(prec=lbm.LBM_FP64)), C.byref(n64)) == lbm.LBM_OK
    assert n64.value >= 2 * (38 + 3) * N * 8 + N * 8 + 8 * N * 8
