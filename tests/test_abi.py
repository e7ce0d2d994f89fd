"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and validates arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msmc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(su3_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1510_04675_amd import capi
    L = capi.lib()
    names = _declared()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(capi.SIGNATURES), set(names) ^ set(capi.SIGNATURES)


def test_field_bytes_and_shape_validation():
    from paper_1510_04675_amd import capi
    # 18 reals per link record, component stride padded to an odd number of 128 B lines
    b64 = capi.su3_field_bytes([4, 4, 4, 4], capi.SU3_FP64)
    assert b64 >= 1024 * 144 and b64 % 128 == 0
    b32 = capi.su3_field_bytes([32, 32, 32, 32], capi.SU3_FP32)
    r12 = capi.su3_field_bytes([32, 32, 32, 32], capi.SU3_FP32_R12)
    assert b32 >= 4 * 32**4 * 72 and r12 >= 4 * 32**4 * 48 and r12 < b32
    for bad in ([3, 4, 4, 4], [4, 4, 0, 4], [4, 4, 4, 1], [1024, 1024, 1024, 2]):
        with pytest.raises(capi.SU3Error) as e:
            capi.su3_field_bytes(bad, capi.SU3_FP64)
        assert e.value.code == 2
    with pytest.raises(capi.SU3Error) as e:
        capi.su3_field_bytes([4, 4, 4, 4], 7)
    assert e.value.code == 1


def test_null_handles_are_rejected():
    from paper_1510_04675_amd import capi
    L = capi.lib()
    assert L.su3_init_cold(None) == 1
    assert L.su3_plaquette(None, None) == 1
    assert "NULL" in capi.su3_last_error()
    assert L.su3_field_destroy(None) == 0
    assert L.su3_set_launch(100, 1) == 1
    assert L.su3_profile_read(3, None, None) == 1
    assert L.su3_batch_sweep_hb_or(None, 0, None, None, None, 0, 1, None, None) == 1


def test_host_only_entry_points_validate_and_compute():
    """Calls that do no device work run without a GPU: t0 interpolation
    against the oracle's, its error cases, and the setters' argument checks."""
    import numpy as np
    import oracle as orc
    from paper_1510_04675_amd import capi
    tt = np.linspace(0.1, 2.0, 20)
    EE = (0.05 + 0.2 * tt) / tt**2  # t^2 E = 0.05 + 0.2 t crosses 0.3 at t = 1.25
    t0 = capi.su3_flow_t0(tt, EE, 0.3)
    assert abs(t0 - orc.flow_t0(tt, EE, 0.3)) < 1e-15
    assert abs(t0 - 1.25) < 1e-12  # t^2 E is linear in t here, so the interpolation is exact
    with pytest.raises(capi.SU3Error) as e:
        capi.su3_flow_t0(tt, EE, 5.0)  # never reached
    assert e.value.code == 5
    L = capi.lib()
    assert L.su3_set_tile(-1, 2, 2) == 1
    assert L.su3_set_tile(0, 0, 0) == 0
    assert L.su3_set_launch(0, 2) == 1
    assert L.su3_set_launch(0, 1) == 0
    assert L.su3_set_group_bytes(224 << 20) == 0


# Entry points that implement a step or a measurement of the method; each
# must name the passage of the paper it follows in the comment above its
# declaration.  (Field plumbing, launch tuning and diagnostics have none.)
METHOD_CALLS = ["su3_init_cold", "su3_init_hot", "su3_restrict", "su3_prolongate", "su3_sweep_hb_or",
                "su3_batch_sweep_hb_or", "su3_hmc_trajectory", "su3_plaquette", "su3_action", "su3_wilson_flow",
                "su3_wilson_flow_adaptive", "su3_flow_t0", "su3_max_plaquette_action", "su3_topological_charge",
                "su3_clover_energy", "su3_wilson_loop", "su3_partial_plaquettes", "su3_displaced_loops",
                "su3_gauge_transform", "su3_last_exhausted"]


def _comment_before(txt, name):
    """The comment block that documents `name`: the last /* ... */ ending
    before its declaration (declarations of a group share one comment)."""
    i = re.search(r"\bint32_t\s+" + name + r"\s*\(", txt).start()
    j = txt.rfind("*/", 0, i)
    k = txt.rfind("/*", 0, j)
    return txt[k:j]


def test_method_entry_points_cite_the_paper():
    txt = open(HEADER).read()
    for n in METHOD_CALLS:
        c = _comment_before(txt, n)
        assert re.search(r"Sec\. [IV]+|App\. [A-D]", c), n


def test_last_exhausted_validates():
    from paper_1510_04675_amd import capi
    L = capi.lib()
    c = C.c_int64(7)
    assert L.su3_last_exhausted(None, C.byref(c)) == 1
    assert c.value == 7


def test_noalloc_sweep_validates_sizes_before_device_work():
    """The allocation-free sweep rejects a lattice beyond its 2^24-site
    scratch before any device call (the wrapped pointer is never touched)."""
    from paper_1510_04675_amd import capi
    L = capi.lib()
    dims = (C.c_int32 * 4)(64, 64, 64, 128)
    nbytes = capi.su3_field_bytes(list(dims), capi.SU3_FP32_R12)
    h = C.c_void_p()
    assert L.su3_field_wrap(dims, capi.SU3_FP32_R12, C.c_void_p(1 << 20), nbytes, None, C.byref(h)) == 0
    try:
        assert L.su3_sweep_hb_or_noalloc(h, C.c_double(6.0), 1, 0, 0, 1, None, None) == 6
        assert "2^24" in capi.su3_last_error()
        assert L.su3_sweep_hb_or_noalloc(h, C.c_double(-1.0), 1, 0, 0, 1, None, None) == 1
        assert L.su3_sweep_hb_or_noalloc(None, C.c_double(6.0), 1, 0, 0, 1, None, None) == 1
    finally:
        L.su3_field_destroy(h)
