"""Host-only tests of the C ABI: the library loads, exports every function
that include/sph.h declares, and validates arguments on the host (these calls
return before any device work, so no GPU is needed)."""
import ctypes
import os
import re

import pytest
import torch

import paper_1909_04504_amd as sph
import sph_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(sph_[a-z_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for need in ("sph_bin_sort", "sph_neighbors", "sph_density", "sph_eos", "sph_momentum",
                 "sph_step", "sph_step_backward"):
        assert need in names
    assert set(names) == set(sph.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = sph.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_sizes_match_header_layout():
    # 8 int32 + 6 double + 9 double + 4 int32 (scheme, integrator, pair_tiles, cell_order)
    assert ctypes.sizeof(sph.Params) == 8 * 4 + 15 * 8 + 4 * 4
    # n, x/u/a (3 pointers each), rho, p, m, type, id, arho
    assert ctypes.sizeof(sph.Particles) == 8 + 9 * 8 + 6 * 8


def _params(**kw):
    p, _ = W.taylor_green(32)
    p = p.replace(**kw) if kw else p
    return sph.make_params(p, sph.FP64)


def test_grid_and_workspace_queries():
    prm = _params()
    nc, ncells = sph.grid(prm)
    # 32x32 lattice, h = 1.3/32: R = 2.6/32, floor(32/2.6) = 12 cells per axis
    assert nc == (12, 12, 1) and ncells == 144
    b1 = sph.workspace_bytes(prm, 1024)
    b2 = sph.workspace_bytes(prm, 2048)
    assert 0 < b1 < b2 and b1 % 256 == 0
    prm2 = _params(cell_div=2)
    assert sph.grid(prm2)[0] == (24, 24, 1)


def test_workspace_holds_the_neighbour_lists():
    """Lists take 4 bytes per entry, capacity (rounded up to a multiple of 4)
    entries per particle in tiles of 64 particles; nbr_cap < 0 (cell walks
    only) drops them."""
    p, _ = W.taylor_green(32)
    n = 1000  # 16 tiles of 64
    walk = sph.workspace_bytes(sph.make_params(p, sph.FP64, -1), n)
    for cap, rounded in ((8, 8), (62, 64), (100, 100), (1, 4)):
        b = sph.workspace_bytes(sph.make_params(p, sph.FP64, cap), n)
        assert 4 * rounded * 16 * 64 <= b - walk < 4 * rounded * 16 * 64 + 512  # + alignment
    assert (sph.workspace_bytes(sph.make_params(p, sph.FP64, 0), n)
            == sph.workspace_bytes(sph.make_params(p, sph.FP64, 64), n))


@pytest.mark.parametrize("field,value", [("dim", 4), ("kernel", 7), ("precision", 3),
                                         ("cell_div", 3), ("h", 0.0), ("h", -1.0),
                                         ("rho0", 0.0), ("c0", 0.0), ("nu", -1.0),
                                         ("eta", -0.5), ("nbr_cap", 5000),
                                         ("scheme", 2), ("scheme", -1), ("integrator", 2),
                                         ("integrator", 1), ("cell_order", 2),
                                         ("cell_order", -1)])
def test_invalid_params_rejected(field, value):
    prm = _params()
    setattr(prm, field, value)
    assert sph.lib().sph_workspace_bytes(ctypes.byref(prm), 100, 0) == 0
    assert sph.lib().sph_last_error()


def test_short_periodic_axis_rejected():
    prm = _params(h=0.2)  # floor(1/0.4) = 2 < 3 cells
    with pytest.raises(sph.SphError) as ei:
        sph.grid(prm)
    assert ei.value.code == sph.SPH_EINVAL
    assert b"stencil" in sph.lib().sph_last_error()


def _fake_particles(n, dim=2):
    s = sph.Particles()
    s.n = n
    for k in range(dim):
        s.x[k] = 4096
        s.u[k] = 4096
        s.a[k] = 4096
    s.rho = s.p = s.m = s.type = s.id = 4096
    return s


def test_entry_points_validate_before_launch():
    L = sph.lib()
    prm = _params()
    cs = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(4096 * 1024)
    # NULL params / particles
    assert L.sph_bin_sort(None, None, ws, 1 << 30, cs, cs, None) == sph.SPH_EINVAL
    # n = 0 and NULL arrays
    s = _fake_particles(0)
    assert L.sph_step(ctypes.byref(prm), ctypes.byref(s), 1, 1, ws, 1 << 30, None,
                      None) == sph.SPH_EINVAL
    s = _fake_particles(100)
    s.m = None
    assert L.sph_density(ctypes.byref(prm), ctypes.byref(s), cs, cs, ws, 1 << 30,
                         None) == sph.SPH_EINVAL
    # workspace too small
    s = _fake_particles(100)
    assert L.sph_step(ctypes.byref(prm), ctypes.byref(s), 1, 1, ws, 256, None,
                      None) == sph.SPH_EWORKSPACE
    assert b"workspace" in L.sph_last_error()
    # misaligned workspace
    assert L.sph_step(ctypes.byref(prm), ctypes.byref(s), 1, 1, ctypes.c_void_p(4096 + 8),
                      1 << 30, None, None) == sph.SPH_EINVAL
    # negative steps, bad prime flag, dt <= 0
    assert L.sph_step(ctypes.byref(prm), ctypes.byref(s), -1, 1, ws, 1 << 30, None,
                      None) == sph.SPH_EINVAL
    assert L.sph_step(ctypes.byref(prm), ctypes.byref(s), 1, 2, ws, 1 << 30, None,
                      None) == sph.SPH_EINVAL
    prm0 = _params(dt=0.0)
    assert L.sph_step(ctypes.byref(prm0), ctypes.byref(s), 1, 1, ws, 1 << 30, None,
                      None) == sph.SPH_EINVAL
    # negative neighbour capacity
    tot = ctypes.c_int64()
    assert L.sph_neighbors(ctypes.byref(prm), ctypes.byref(s), cs, cs, -1, cs, cs,
                           ctypes.byref(tot), ws, 1 << 30, None) == sph.SPH_EINVAL
    # NULL workspace in sph_check
    assert L.sph_check(None, 0, None) == sph.SPH_EINVAL


def test_particle_arrays_are_checked_against_the_parameters():
    """rho is FP64 under the continuity scheme (an integrated state) and of
    the pair type otherwise; the binding refuses arrays of the other type
    before anything reaches the library."""
    p, s = W.dam_break_2d()
    for prec in (sph.FP64, sph.FP32_MIXED):
        prm_c = sph.make_params(p, prec)
        prm_s = sph.make_params(p.replace(scheme=W.SUMMATION), prec)
        dc = sph.DeviceParticles.from_state(s, prec, device="cpu", scheme=sph.CONTINUITY)
        ds = sph.DeviceParticles.from_state(s, prec, device="cpu")
        assert dc.rho.dtype == torch.float64
        dc.struct(prm_c)
        ds.struct(prm_s)
        if prec == sph.FP32_MIXED:
            with pytest.raises(ValueError):
                ds.struct(prm_c)
            with pytest.raises(ValueError):
                dc.struct(prm_s)
    with pytest.raises(ValueError):
        sph.DeviceParticles.from_state(s, sph.FP64, device="cpu").struct(
            sph.make_params(p, sph.FP32_MIXED))
    assert (s.rho == p.rho0).all()


def test_continuity_needs_arho():
    """Under the continuity scheme the particle set must carry drho/dt; a
    NULL arho is refused on the host before any launch."""
    p, s = W.dam_break_2d()
    prm = sph.make_params(p, sph.FP64)
    dp = sph.DeviceParticles.from_state(s, sph.FP64, device="cpu", scheme=sph.CONTINUITY)
    c = dp.struct(prm)
    c.arho = None
    cs = torch.zeros(4, dtype=torch.int32)
    ws = torch.zeros(256, dtype=torch.uint8)
    rc = sph.lib().sph_bin_sort(ctypes.byref(prm), ctypes.byref(c), ws.data_ptr(), ws.numel(),
                                cs.data_ptr(), cs.data_ptr(), None)
    assert rc == sph.SPH_EINVAL
    assert b"arho" in sph.lib().sph_last_error()


def test_binding_layout_matches_the_c_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what a
    C compiler makes of include/sph.h (compiled here with gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = {"sph_params": sph.Params, "sph_particles": sph.Particles}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sph.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'    printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.split("\n"):
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, cls in fields.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_noalloc_scratch_size_mirrors_header():
    """The binding's NOALLOC_SCRATCH_BYTES is the header's
    SPH_NOALLOC_SCRATCH_BYTES (64 MiB)."""
    import re
    hdr = open(os.path.join(ROOT, "include", "sph.h")).read()
    m = re.search(r"#define SPH_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m
    assert sph.NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
