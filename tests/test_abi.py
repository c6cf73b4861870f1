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
                      ("SPH_ERR_CONFIG", abi.SPH_ERR_CONFIG), ("SPH_F64", abi.SPH_F64),
                      ("SPH_CONTINUITY", abi.SPH_CONTINUITY), ("SPH_MOMENTUM", abi.SPH_MOMENTUM),
                      ("SPH_NO_KICK", abi.SPH_NO_KICK), ("SPH_DIAG_LEN", abi.SPH_DIAG_LEN),
                      ("SPH_DIAG_PROBE", abi.SPH_DIAG_PROBE), ("SPH_STATUS_LEN", abi.SPH_STATUS_LEN)]:
        m = re.search(rf"#define {name} (\d+)", text)
        assert m and int(m.group(1)) == val, name


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
        make_desc(sc.with_params(dt=sc.dt * 1.01), "f32")   # above the CFL bound
    with pytest.raises(abi.SPHError):
        make_desc(sc.with_params(dim=4), "f32")
