"""The allocation-free sweep entry point against the allocating one, through
the C ABI: same arguments, same update kernels, so the links and the
exhausted-draw count must be bitwise equal; its plaquette history comes from
the standalone plaquette kernel instead of the last overrelaxation pass and
must agree to rounding (1e-13 fp64, 1e-7 fp32).  Two calls in a row share
the device scratch array, the second on a smaller lattice, so a state left
over from the first call would show."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1510_04675_amd as msmc
    msmc.lib()
    return msmc


def _pair(m, dims, prec, seed, lid):
    a, b = m.Field(dims, prec), m.Field(dims, prec)
    m.su3_init_hot(a, seed, lid)
    m.su3_init_hot(b, seed, lid)
    return a, b


@pytest.mark.parametrize("prec", ["fp64", "fp32_r12"])
def test_noalloc_sweeps_equal_allocating_sweeps(m, prec):
    cases = [([8, 8, 8, 8], 6.0, m.hb_params(n_or=2, reunit_every=2), 10, 5),
             ([4, 6, 4, 2], 1.0, m.hb_params(n_or=1, hb_max_tries=1, reunit_every=0), 3, 4)]
    for dims, beta, params, first, n in cases:
        a, b = _pair(m, dims, prec, 17, 3)
        ha = m.su3_sweep_hb_or(a, beta, 17, 3, first, n, params)
        hb = m.su3_sweep_hb_or_noalloc(b, beta, 17, 3, first, n, params)
        assert np.max(np.abs(ha - hb)) < (1e-13 if prec == "fp64" else 1e-7), (dims, ha, hb)
        assert np.array_equal(m.su3_field_to_host(a), m.su3_field_to_host(b)), dims
        assert m.su3_last_exhausted(a) == m.su3_last_exhausted(b)
        if beta == 1.0:
            assert m.su3_last_exhausted(b) > 0
        # without a history the field evolves the same way
        m.su3_sweep_hb_or(a, beta, 17, 3, first + n, 2, params, record=False)
        m.su3_sweep_hb_or_noalloc(b, beta, 17, 3, first + n, 2, params, record=False)
        assert np.array_equal(m.su3_field_to_host(a), m.su3_field_to_host(b)), dims
        a.close()
        b.close()


def test_noalloc_rejects_sizes_beyond_its_limits(m):
    from paper_1510_04675_amd import capi
    L = capi.lib()
    # a lattice of 2^25 sites, never touched: validation comes first
    dims = (C.c_int32 * 4)(64, 64, 64, 128)
    nbytes = capi.su3_field_bytes(list(dims), capi.SU3_FP32_R12)
    h = C.c_void_p()
    assert L.su3_field_wrap(dims, capi.SU3_FP32_R12, C.c_void_p(1 << 20), nbytes, None, C.byref(h)) == 0
    try:
        assert L.su3_sweep_hb_or_noalloc(h, C.c_double(6.0), 1, 0, 0, 1, None, None) == 6
        assert "2^24" in capi.su3_last_error()
    finally:
        L.su3_field_destroy(h)
    f = m.Field([4, 4, 4, 4], "fp32")
    hist = np.zeros(4097)
    assert L.su3_sweep_hb_or_noalloc(f.handle, C.c_double(6.0), 1, 0, 0, 4097, None,
                                     hist.ctypes.data_as(C.c_void_p)) == 1
    f.close()
