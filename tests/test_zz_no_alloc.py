"""sph_diag_noalloc (fixed device workspace, no allocation) against sph_diag
(caller's scratch) through the C ABI: the same kernels in the same order, so
every diagnostic must agree bit for bit.  Two calls in a row on one GPU, the
second on a smaller state, so the second reads only partials it wrote
itself; then the first state again, after the smaller call."""
import ctypes as C

import numpy as np
import pytest

from paper_2110_02621_amd import abi, scenes

pytestmark = pytest.mark.gpu


def _noalloc(S):
    # the caller's buffers minus the scratch: the entry point must not need it
    b = abi.Buffers.from_buffer_copy(S.buf)
    b.scratch = None
    b.scratch_bytes = 0
    S.t["diag"].zero_()
    rc = S.lib.sph_diag_noalloc(C.byref(S.desc), C.byref(b), S._stream())
    abi.check(rc, "sph_diag_noalloc")
    S.synchronize()
    return S.t["diag"].cpu().numpy().copy(), S.status()


def _reference(S):
    S.t["diag"].zero_()
    S._call("sph_diag", S.lib.sph_diag)
    S.synchronize()
    return S.t["diag"].cpu().numpy().copy(), S.status()


def test_diag_noalloc_matches_diag_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2110_02621_amd.solver import Solver
    big = Solver(scenes.dam_break_3d(dx=0.01), "f32")     # 108,000 fluid: 422 blocks of partials
    big.step(5)
    small = Solver(scenes.dam_break_2d(dx=0.04), "f64")   # 1,250 fluid: 5 blocks
    small.step(3)
    print(f"[noalloc] big nf={big.scene.n_fluid} small nf={small.scene.n_fluid}", flush=True)
    for S in (big, small, big):
        ref, st_ref = _reference(S)
        got, st_got = _noalloc(S)
        print(f"  nf={S.scene.n_fluid}: M={got[abi.SPH_DIAG_MASS]:.9e} Ek={got[abi.SPH_DIAG_EKIN]:.9e}",
              flush=True)
        assert np.array_equal(got[:abi.SPH_DIAG_VMAX + 1], ref[:abi.SPH_DIAG_VMAX + 1]), (got, ref)
        assert got[abi.SPH_DIAG_MASS] > 0 and got[abi.SPH_DIAG_EKIN] > 0
        assert st_got == st_ref == dict(out_of_grid=0, fast=0, nonfinite=0, list_overflow=0)
