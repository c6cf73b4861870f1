"""The C-ABI library loads and exports every function include/sph.h declares
(no GPU needed: symbols only, no compute call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")
LIB = os.path.join(ROOT, "paper_2110_02621_amd", "libsph.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(sph_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("sph_build_cells", "sph_density", "sph_wall_bc", "sph_forces", "sph_step"):
        assert required in names
    assert len(names) >= 12


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libsph.so is not built: run `python -m paper_2110_02621_amd.build`")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_header():
    from paper_2110_02621_amd import abi
    assert sorted(abi.EXPORTED) == declared()
    text = open(HEADER).read()
    for name, val in [("SPH_OK", abi.SPH_OK), ("SPH_ERR_ARG", abi.SPH_ERR_ARG),
                      ("SPH_ERR_CONFIG", abi.SPH_ERR_CONFIG), ("SPH_ERR_LAUNCH", abi.SPH_ERR_LAUNCH),
                      ("SPH_ERR_CAPACITY", abi.SPH_ERR_CAPACITY), ("SPH_F64", abi.SPH_F64),
                      ("SPH_CONTINUITY", abi.SPH_CONTINUITY), ("SPH_MOMENTUM", abi.SPH_MOMENTUM),
                      ("SPH_NO_KICK", abi.SPH_NO_KICK), ("SPH_DIAG_LEN", abi.SPH_DIAG_LEN),
                      ("SPH_DIAG_PROBE", abi.SPH_DIAG_PROBE), ("SPH_STATUS_LEN", abi.SPH_STATUS_LEN)]:
        m = re.search(rf"#define {name} (\d+)", text)
        assert m and int(m.group(1)) == val, name
    assert re.search(r"#define SPH_DIAG_NOALLOC_BYTES \(4u << 20\)", text) and abi.SPH_DIAG_NOALLOC_BYTES == 4 << 20
    assert re.search(r"#define SPH_DIAG_NOALLOC_MAX_FLUID \(\(int64_t\)1 << 24\)", text)
    assert abi.SPH_DIAG_NOALLOC_MAX_FLUID == 1 << 24
    # the partials of the largest accepted input fill the workspace exactly:
    # one block of 256 particles leaves 8 doubles
    assert abi.SPH_DIAG_NOALLOC_MAX_FLUID // 256 * 8 * 8 == abi.SPH_DIAG_NOALLOC_BYTES


def test_host_configuration_checks():
    # sph_configure is host-only: it validates and derives the grid without a GPU.
    from paper_2110_02621_amd import abi, scenes
    from paper_2110_02621_amd.solver import make_desc
    sc = scenes.dam_break_3d(dx=0.02)
    d = make_desc(sc, "f32")
    assert d.cell >= 2 * sc.h and abs(d.cell - 2 * sc.h) < 1e-6 * sc.h
    assert d.n_cells == d.grid[0] * d.grid[1] * d.grid[2]
    import oracle
    assert d.sigma0 == pytest.approx(oracle.sigma0_lattice(3, sc.dx, sc.h), rel=1e-12)
    with pytest.raises(abi.SPHError):
        make_desc(sc.with_params(dt=sc.dt * 1.02), "f32")   # above the CFL bound
    make_desc(sc.with_params(dt=sc.dt * 1.005), "f32")      # within the 1 % slack
    with pytest.raises(abi.SPHError):
        make_desc(sc.with_params(dim=4), "f32")


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sph.h"', 'int main(void) {',
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("cname,pyname", [("sph_desc", "Desc"), ("sph_buffers", "Buffers"),
                                          ("sph_frame", "Frame"), ("sph_adjoint", "Adjoint")])
def test_ctypes_structs_match_header_layout(cname, pyname, tmp_path):
    from paper_2110_02621_amd import abi, adjoint
    cls = getattr(abi, pyname, None) or getattr(adjoint, pyname)
    fields = [f[0] for f in cls._fields_]
    size, offs = _c_layout(cname, fields, tmp_path)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs


def test_particle_count_limits():
    # gathers use 32-bit byte offsets: record arrays must stay below 4 GiB,
    # 2^28 - 1 particles per set in FP32 (16-byte records), 2^27 - 1 in FP64
    from paper_2110_02621_amd import abi, scenes
    from paper_2110_02621_amd.solver import make_desc
    lib = ctypes.CDLL(LIB)
    lib.sph_scratch_bytes.argtypes = [ctypes.POINTER(abi.Desc), ctypes.c_int64, ctypes.c_int64]
    lib.sph_scratch_bytes.restype = ctypes.c_size_t
    lib.sph_adjoint_work_bytes.argtypes = lib.sph_scratch_bytes.argtypes
    lib.sph_adjoint_work_bytes.restype = ctypes.c_size_t
    sc = scenes.dam_break_3d(dx=0.02)
    for prec, top in (("f32", 2 ** 28 - 1), ("f64", 2 ** 27 - 1)):
        d = make_desc(sc, prec)
        for fn in (lib.sph_scratch_bytes, lib.sph_adjoint_work_bytes):
            assert fn(ctypes.byref(d), top, 1000) > 0, prec
            assert fn(ctypes.byref(d), 1000, top) > 0, prec
            assert fn(ctypes.byref(d), top + 1, 1000) == 0, prec
            assert fn(ctypes.byref(d), 1000, top + 1) == 0, prec


def test_diag_noalloc_refuses_inputs_beyond_its_workspace():
    # Host-side checks run before any HIP call: a state larger than the fixed
    # workspace is refused with SPH_ERR_CAPACITY, a missing buffer with
    # SPH_ERR_ARG.  The pointers are never dereferenced on these paths.
    from paper_2110_02621_amd import abi, scenes
    from paper_2110_02621_amd.solver import make_desc
    lib = abi.load()
    d = make_desc(scenes.dam_break_3d(dx=0.02), "f32")
    b = abi.Buffers()
    fake = 1 << 20
    for c in range(2):
        b.key[c] = b.pid[c] = b.off[c] = b.vel[c] = b.rho[c] = fake
    b.acc = b.wkey = b.wpid = b.woff = b.pw = b.nrm = b.fstart = b.wstart = fake
    b.status = b.diag = fake
    b.n_wall = 10
    b.n_fluid = abi.SPH_DIAG_NOALLOC_MAX_FLUID + 1
    assert lib.sph_diag_noalloc(ctypes.byref(d), ctypes.byref(b), None) == abi.SPH_ERR_CAPACITY
    assert b"workspace" in lib.sph_strerror(abi.SPH_ERR_CAPACITY)
    b.n_fluid = 1000
    b.diag = None
    assert lib.sph_diag_noalloc(ctypes.byref(d), ctypes.byref(b), None) == abi.SPH_ERR_ARG
