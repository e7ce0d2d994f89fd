"""Thin ctypes binding of the C ABI in include/msmc.h.

Each function has the name of the C call it wraps and only marshals
arguments: field handles come from :class:`Field`, host outputs are returned
as Python / numpy values, and a non-zero status raises :class:`SU3Error`
with the library's message.  Every computation runs in the HIP library; if
it is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmsmc.so")

SU3_FP64, SU3_FP32, SU3_FP32_R12 = 0, 1, 2
PRECISIONS = {"fp64": SU3_FP64, "fp32": SU3_FP32, "fp32_r12": SU3_FP32_R12}
SU3_SAMPLER_KP, SU3_SAMPLER_CREUTZ = 0, 1
STATUS = {0: "SU3_OK", 1: "SU3_ERR_ARG", 2: "SU3_ERR_SHAPE", 3: "SU3_ERR_NOMEM", 4: "SU3_ERR_HIP",
          5: "SU3_ERR_NUMERIC", 6: "SU3_ERR_UNSUPPORTED"}

# every symbol the header declares, with (restype, argtypes)
_i32, _u32, _u64, _i64, _d = C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double
_p, _sz = C.c_void_p, C.c_size_t


class HbParams(C.Structure):
    _fields_ = [("n_or", C.c_int32), ("n_hb_hits", C.c_int32), ("hb_max_tries", C.c_int32),
                ("reunit_every", C.c_int32), ("sampler", C.c_int32)]


SIGNATURES = {
    "su3_field_bytes": (_i32, [_p, _i32, C.POINTER(_sz)]),
    "su3_field_create": (_i32, [_p, _i32, _p, C.POINTER(_p)]),
    "su3_field_wrap": (_i32, [_p, _i32, _p, _sz, _p, C.POINTER(_p)]),
    "su3_field_destroy": (_i32, [_p]),
    "su3_field_set_stream": (_i32, [_p, _p]),
    "su3_field_info": (_i32, [_p, _p, C.POINTER(_i32), C.POINTER(_sz)]),
    "su3_init_cold": (_i32, [_p]),
    "su3_init_hot": (_i32, [_p, _u32, _u32]),
    "su3_field_to_host": (_i32, [_p, _p]),
    "su3_field_from_host": (_i32, [_p, _p]),
    "su3_field_copy": (_i32, [_p, _p]),
    "su3_restrict": (_i32, [_p, _p]),
    "su3_prolongate": (_i32, [_p, _p, _d, _d, _i32, _p]),
    "su3_sweep_hb_or": (_i32, [_p, _d, _u32, _u32, _u64, _i32, C.POINTER(HbParams), _p]),
    "su3_sweep_hb_or_noalloc": (_i32, [_p, _d, _u32, _u32, _u64, _i32, C.POINTER(HbParams), _p]),
    "su3_batch_sweep_hb_or": (_i32, [_p, _i32, _p, _p, _p, _u64, _i32, C.POINTER(HbParams), _p]),
    "su3_hmc_trajectory": (_i32, [_p, _d, _d, _i32, _u32, _u32, _u64, _i32, C.POINTER(_d), C.POINTER(_i32)]),
    "su3_plaquette": (_i32, [_p, C.POINTER(_d)]),
    "su3_action": (_i32, [_p, _d, C.POINTER(_d)]),
    "su3_wilson_flow": (_i32, [_p, _d, _i32]),
    "su3_topological_charge": (_i32, [_p, C.POINTER(_d)]),
    "su3_clover_energy": (_i32, [_p, C.POINTER(_d)]),
    "su3_reunitarize": (_i32, [_p]),
    "su3_gauge_transform": (_i32, [_p, _u32]),
    "su3_check_field": (_i32, [_p, _d, C.POINTER(_d), C.POINTER(_i64)]),
    "su3_last_exhausted": (_i32, [_p, C.POINTER(_i64)]),
    "su3_set_launch": (_i32, [_i32, _i32]),
    "su3_autotune": (_i32, [_i32]),
    "su3_get_launch": (_i32, [C.POINTER(_i32), C.POINTER(_i32)]),
    "su3_set_tile": (_i32, [_i32, _i32, _i32]),
    "su3_get_config": (_i32, [_p, _i32, _p]),
    "su3_profile_enable": (_i32, [_i32]),
    "su3_profile_read": (_i32, [_i32, C.POINTER(_d), C.POINTER(_i64)]),
    "su3_set_group_bytes": (_i32, [C.c_uint64]),
    "su3_wilson_loop": (_i32, [_p, _i32, _i32, C.POINTER(_d)]),
    "su3_partial_plaquettes": (_i32, [_p, C.c_void_p]),
    "su3_displaced_loops": (_i32, [_p, C.c_void_p]),
    "su3_wilson_flow_adaptive": (_i32, [_p, _d, _d, _d, _d, _p, _i32, _p, _p, C.POINTER(_i32), C.POINTER(_i32)]),
    "su3_flow_t0": (_i32, [_p, _p, _i32, _d, C.POINTER(_d)]),
    "su3_max_plaquette_action": (_i32, [_p, C.POINTER(_d)]),
    "su3_last_error": (C.c_char_p, []),
}


class SU3Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libmsmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1510_04675_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ck(rc: int):
    if rc != 0:
        raise SU3Error(rc, lib().su3_last_error().decode())


def _dims(dims):
    a = (C.c_int32 * 4)(*[int(x) for x in dims])
    return a


def hb_params(n_or=4, n_hb_hits=1, hb_max_tries=64, reunit_every=10, sampler=SU3_SAMPLER_KP) -> HbParams:
    return HbParams(n_or, n_hb_hits, hb_max_tries, reunit_every, sampler)


def su3_field_bytes(dims, prec: int) -> int:
    out = C.c_size_t()
    _ck(lib().su3_field_bytes(_dims(dims), prec, C.byref(out)))
    return out.value


class Field:
    """A link field whose device memory is a torch tensor, wrapped by the
    library (su3_field_wrap).  ``stream`` defaults to torch's current
    stream on the device."""

    def __init__(self, dims, prec="fp64", device="cuda", stream=None):
        import torch
        self.dims = [int(x) for x in dims]
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        nbytes = su3_field_bytes(self.dims, self.prec)
        self.storage = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.storage.data_ptr()
        ptr = (base + 255) // 256 * 256
        if stream is None:
            stream = torch.cuda.current_stream(self.storage.device).cuda_stream
        self.stream = stream
        h = C.c_void_p()
        _ck(lib().su3_field_wrap(_dims(self.dims), self.prec, C.c_void_p(ptr), nbytes, C.c_void_p(stream),
                                 C.byref(h)))
        self.handle = h
        self.nbytes = nbytes

    @property
    def volume(self) -> int:
        return int(np.prod(self.dims))

    def close(self):
        if getattr(self, "handle", None):
            lib().su3_field_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def su3_field_destroy(f: Field):
    f.close()


def su3_field_set_stream(f: Field, stream: int):
    _ck(lib().su3_field_set_stream(f.handle, C.c_void_p(stream)))
    f.stream = stream


def su3_field_info(f: Field):
    d = (C.c_int32 * 4)()
    p = C.c_int32()
    b = C.c_size_t()
    _ck(lib().su3_field_info(f.handle, d, C.byref(p), C.byref(b)))
    return list(d), p.value, b.value


def su3_init_cold(f: Field):
    _ck(lib().su3_init_cold(f.handle))


def su3_init_hot(f: Field, seed: int, lattice_id: int = 0):
    _ck(lib().su3_init_hot(f.handle, seed, lattice_id))


def su3_field_to_host(f: Field) -> np.ndarray:
    out = np.empty((f.volume, 4, 3, 3, 2), dtype=np.float64)
    _ck(lib().su3_field_to_host(f.handle, out.ctypes.data_as(C.c_void_p)))
    return out


def su3_field_from_host(f: Field, U: np.ndarray):
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.size != f.volume * 72:
        raise ValueError("host field has the wrong size")
    _ck(lib().su3_field_from_host(f.handle, U.ctypes.data_as(C.c_void_p)))


def su3_field_copy(dst: Field, src: Field):
    _ck(lib().su3_field_copy(dst.handle, src.handle))


def su3_restrict(fine: Field, coarse: Field):
    _ck(lib().su3_restrict(fine.handle, coarse.handle))


def su3_prolongate(coarse: Field, fine: Field, c=0.05, rel_tol=1e-5, max_iter=10000):
    it = (C.c_int32 * 3)()
    _ck(lib().su3_prolongate(coarse.handle, fine.handle, c, rel_tol, max_iter, it))
    return list(it)


def su3_sweep_hb_or(f: Field, beta, seed, lattice_id=0, first_sweep=0, n_sweeps=1, params: HbParams = None,
                    record=True):
    hist = np.zeros(max(n_sweeps, 1))
    pp = C.byref(params) if params is not None else None
    _ck(lib().su3_sweep_hb_or(f.handle, beta, seed, lattice_id, first_sweep, n_sweeps, pp,
                              hist.ctypes.data_as(C.c_void_p) if record else None))
    return hist[:n_sweeps] if record else None


def su3_sweep_hb_or_noalloc(f: Field, beta, seed, lattice_id=0, first_sweep=0, n_sweeps=1, params: HbParams = None,
                            record=True):
    hist = np.zeros(max(n_sweeps, 1))
    pp = C.byref(params) if params is not None else None
    _ck(lib().su3_sweep_hb_or_noalloc(f.handle, beta, seed, lattice_id, first_sweep, n_sweeps, pp,
                                      hist.ctypes.data_as(C.c_void_p) if record else None))
    return hist[:n_sweeps] if record else None


def su3_batch_sweep_hb_or(fields, betas, seeds, lattice_ids, first_sweep=0, n_sweeps=1, params: HbParams = None,
                          record=True):
    n = len(fields)
    hs = (C.c_void_p * n)(*[f.handle.value for f in fields])
    b = np.ascontiguousarray(betas, dtype=np.float64)
    s = np.ascontiguousarray(seeds, dtype=np.uint32)
    l = np.ascontiguousarray(lattice_ids, dtype=np.uint32)
    out = np.zeros((max(n_sweeps, 1), n))
    pp = C.byref(params) if params is not None else None
    _ck(lib().su3_batch_sweep_hb_or(hs, n, b.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p),
                                    l.ctypes.data_as(C.c_void_p), first_sweep, n_sweeps, pp,
                                    out.ctypes.data_as(C.c_void_p) if record else None))
    return out[:n_sweeps] if record else None


def su3_hmc_trajectory(f: Field, beta, tau, n_steps, seed, lattice_id=0, traj=0, metropolis=1):
    dH = C.c_double()
    acc = C.c_int32()
    _ck(lib().su3_hmc_trajectory(f.handle, beta, tau, n_steps, seed, lattice_id, traj, metropolis, C.byref(dH),
                                 C.byref(acc)))
    return bool(acc.value), dH.value


def su3_plaquette(f: Field) -> float:
    out = C.c_double()
    _ck(lib().su3_plaquette(f.handle, C.byref(out)))
    return out.value


def su3_action(f: Field, beta) -> float:
    out = C.c_double()
    _ck(lib().su3_action(f.handle, beta, C.byref(out)))
    return out.value


def su3_wilson_flow(f: Field, eps, n_steps):
    _ck(lib().su3_wilson_flow(f.handle, eps, n_steps))


def su3_wilson_flow_adaptive(f: Field, t_end, tol=0.01, max_step=0.2, eps0=0.01, t_meas=()):
    """Returns (E, Q, n_accepted, n_rejected) at the measurement times."""
    tm = np.ascontiguousarray(t_meas, dtype=np.float64)
    E = np.zeros(tm.size)
    Q = np.zeros(tm.size)
    na, nr = C.c_int32(), C.c_int32()
    _ck(lib().su3_wilson_flow_adaptive(f.handle, t_end, tol, max_step, eps0, tm.ctypes.data_as(C.c_void_p),
                                       int(tm.size), E.ctypes.data_as(C.c_void_p), Q.ctypes.data_as(C.c_void_p),
                                       C.byref(na), C.byref(nr)))
    return E, Q, na.value, nr.value


def su3_flow_t0(t, E, target=0.3) -> float:
    t = np.ascontiguousarray(t, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    out = C.c_double()
    _ck(lib().su3_flow_t0(t.ctypes.data_as(C.c_void_p), E.ctypes.data_as(C.c_void_p), int(t.size), target,
                          C.byref(out)))
    return out.value


def su3_max_plaquette_action(f: Field) -> float:
    out = C.c_double()
    _ck(lib().su3_max_plaquette_action(f.handle, C.byref(out)))
    return out.value


def su3_topological_charge(f: Field) -> float:
    out = C.c_double()
    _ck(lib().su3_topological_charge(f.handle, C.byref(out)))
    return out.value


def su3_clover_energy(f: Field) -> float:
    out = C.c_double()
    _ck(lib().su3_clover_energy(f.handle, C.byref(out)))
    return out.value


def su3_wilson_loop(f: Field, m: int, n: int) -> float:
    out = C.c_double()
    _ck(lib().su3_wilson_loop(f.handle, m, n, C.byref(out)))
    return out.value


def su3_partial_plaquettes(f: Field) -> np.ndarray:
    out = np.zeros(3)
    _ck(lib().su3_partial_plaquettes(f.handle, out.ctypes.data_as(C.c_void_p)))
    return out


def su3_displaced_loops(f: Field) -> np.ndarray:
    out = np.zeros(5)
    _ck(lib().su3_displaced_loops(f.handle, out.ctypes.data_as(C.c_void_p)))
    return out


def su3_reunitarize(f: Field):
    _ck(lib().su3_reunitarize(f.handle))


def su3_gauge_transform(f: Field, seed: int):
    _ck(lib().su3_gauge_transform(f.handle, seed))


def su3_check_field(f: Field, tol: float):
    """Returns (ok, max_dev, worst_index); ok is False on SU3_ERR_NUMERIC."""
    md = C.c_double()
    w = C.c_int64()
    rc = lib().su3_check_field(f.handle, tol, C.byref(md), C.byref(w))
    if rc not in (0, 5):
        _ck(rc)
    return rc == 0, md.value, w.value


def su3_last_exhausted(f: Field) -> int:
    c = C.c_int64()
    _ck(lib().su3_last_exhausted(f.handle, C.byref(c)))
    return c.value


def su3_set_launch(block: int, xcd_remap: int = 1):
    _ck(lib().su3_set_launch(block, xcd_remap))


def su3_get_launch():
    b, r = C.c_int32(), C.c_int32()
    _ck(lib().su3_get_launch(C.byref(b), C.byref(r)))
    return b.value, r.value


def su3_set_group_bytes(nbytes: int):
    _ck(lib().su3_set_group_bytes(int(nbytes)))


def su3_set_tile(ty: int, tz: int, tt: int):
    _ck(lib().su3_set_tile(ty, tz, tt))


def su3_get_config(fields):
    """{block, xcd_remap, ty, tz, tt} the next sweep on these fields uses."""
    n = len(fields)
    hs = (C.c_void_p * n)(*[f.handle.value for f in fields])
    out = (C.c_int32 * 5)()
    _ck(lib().su3_get_config(hs, n, out))
    return dict(zip(("block", "xcd_remap", "ty", "tz", "tt"), list(out)))


def su3_autotune(enable: bool):
    _ck(lib().su3_autotune(1 if enable else 0))


def su3_profile_enable(enable: bool):
    _ck(lib().su3_profile_enable(1 if enable else 0))


def su3_profile_read(kind: int):
    ms = C.c_double()
    n = C.c_int64()
    _ck(lib().su3_profile_read(kind, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def su3_last_error() -> str:
    return lib().su3_last_error().decode()
