"""FP64 CPU oracle for the SU(3) rethermalization path (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``su3_oracle.c`` (plain C99,
complex arithmetic, sequential loops) through ctypes and shares no code with
the HIP library.

Field arrays use the host exchange layout: float64 ``[V, 4, 3, 3, 2]`` with
the site index ``n0 + L0*(n1 + L1*(n2 + L2*n3))`` (n0 fastest), direction,
row-major 3x3 matrix, (re, im).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "su3_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

KP, CREUTZ = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        d, i32, u32, u64, i64 = C.c_double, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64
        P = C.c_void_p
        sig = {
            "orc_philox": (None, [P, P, P]),
            "orc_u01": (d, [u32]),
            "orc_ln": (d, [d]),
            "orc_exp": (d, [d]),
            "orc_cossin_2pi": (None, [d, P, P]),
            "orc_init_cold": (None, [P, P]),
            "orc_init_hot": (None, [P, P, u32, u32]),
            "orc_reunitarize": (None, [P, P]),
            "orc_gauge_transform": (None, [P, P, u32]),
            "orc_plaquette": (d, [P, P]),
            "orc_action": (d, [P, P, d]),
            "orc_staple": (None, [P, P, i64, C.c_int, P]),
            "orc_sample_g0": (i64, [d, i32, i32, u32, i64, P]),
            "orc_hb_pass": (i64, [P, P, d, u32, u32, u64, i32, i32, i32]),
            "orc_or_pass": (None, [P, P]),
            "orc_or_pass_reversed": (None, [P, P]),
            "orc_sweep_hb_or": (i64, [P, P, d, u32, u32, u64, i32, i32, i32, i32, i32, i32, P]),
            "orc_hmc_momenta": (None, [P, P, u32, u32, u64]),
            "orc_hmc_force": (None, [P, P, d, P]),
            "orc_hmc_kinetic": (d, [P, P]),
            "orc_md_leapfrog": (None, [P, P, P, d, d, i32]),
            "orc_hmc_trajectory": (i32, [P, P, d, d, i32, u32, u32, u64, i32, P]),
            "orc_restrict": (None, [P, P, P]),
            "orc_prolong_transfer": (None, [P, P, P]),
            "orc_partial_action": (d, [P, P, i32, d]),
            "orc_project_su3": (None, [P, P]),
            "orc_ape_step": (None, [P, P, i32, d]),
            "orc_prolongate": (i32, [P, P, P, d, d, i32, P]),
            "orc_wilson_loop": (d, [P, P, i32, i32]),
            "orc_partial_plaquette": (d, [P, P, i32]),
            "orc_displaced_2x2": (d, [P, P, i32]),
            "orc_displaced_loop": (d, [P, P, i32, i32, i32]),
            "orc_hb_link": (i64, [P, P, i64, i32, i32, d, u32, u32, u64, i32, i32, i32, P]),
            "orc_wilson_flow": (None, [P, P, d, i32]),
            "orc_topological_charge": (d, [P, P]),
            "orc_clover_energy": (d, [P, P]),
            "orc_wilson_flow_adaptive": (i32, [P, P, d, d, d, d, P, i32, P, P, P, P]),
            "orc_flow_t0": (i32, [P, P, i32, d, P]),
            "orc_max_splaq": (d, [P, P]),
            "orc_flow_step_distance": (d, [P, P, d]),
            "orc_max_su3_dev": (d, [P, P]),
            "orc_set_threads": (None, [i32]),
            "orc_max_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dims(dims):
    a = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert a.shape == (4,)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def empty_field(dims) -> np.ndarray:
    return np.zeros((volume(dims), 4, 3, 3, 2), dtype=np.float64)


def _chk(U, dims):
    assert U.dtype == np.float64 and U.flags.c_contiguous
    assert U.shape == (volume(dims), 4, 3, 3, 2)


def as_complex(U: np.ndarray) -> np.ndarray:
    """[V,4,3,3,2] float64 -> [V,4,3,3] complex128 view/copy."""
    return U[..., 0] + 1j * U[..., 1]


def from_complex(M: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.stack([M.real, M.imag], axis=-1).astype(np.float64))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


def u01(x: int) -> float:
    return lib().orc_u01(int(x) & 0xFFFFFFFF)


def det_ln(x: float) -> float:
    """The oracle's fixed-sequence natural logarithm."""
    return lib().orc_ln(float(x))


def det_exp(x: float) -> float:
    """The oracle's fixed-sequence exponential."""
    return lib().orc_exp(float(x))


def det_cossin_2pi(u: float):
    """The oracle's fixed-sequence (cos 2 pi u, sin 2 pi u)."""
    c, s = C.c_double(), C.c_double()
    lib().orc_cossin_2pi(float(u), C.byref(c), C.byref(s))
    return c.value, s.value


def init_cold(dims) -> np.ndarray:
    U = empty_field(dims)
    lib().orc_init_cold(_ptr(_dims(dims)), _ptr(U))
    return U


def init_hot(dims, seed: int, lattice_id: int = 0) -> np.ndarray:
    U = empty_field(dims)
    lib().orc_init_hot(_ptr(_dims(dims)), _ptr(U), seed, lattice_id)
    return U


def reunitarize(dims, U):
    _chk(U, dims)
    lib().orc_reunitarize(_ptr(_dims(dims)), _ptr(U))


def gauge_transform(dims, U, seed: int):
    _chk(U, dims)
    lib().orc_gauge_transform(_ptr(_dims(dims)), _ptr(U), seed)


def plaquette(dims, U) -> float:
    _chk(U, dims)
    return lib().orc_plaquette(_ptr(_dims(dims)), _ptr(U))


def action(dims, U, beta: float) -> float:
    _chk(U, dims)
    return lib().orc_action(_ptr(_dims(dims)), _ptr(U), beta)


def staple(dims, U, site: int, mu: int) -> np.ndarray:
    _chk(U, dims)
    out = np.zeros((3, 3, 2))
    lib().orc_staple(_ptr(_dims(dims)), _ptr(U), site, mu, _ptr(out))
    return out


def sample_g0(alpha: float, n: int, seed: int = 1, sampler: int = KP, max_tries: int = 64):
    out = np.zeros(n)
    fails = lib().orc_sample_g0(alpha, sampler, max_tries, seed, n, _ptr(out))
    return out, fails


def hb_pass(dims, U, beta, seed, lattice_id, sweep, n_hits=1, max_tries=64, sampler=KP) -> int:
    _chk(U, dims)
    return lib().orc_hb_pass(_ptr(_dims(dims)), _ptr(U), beta, seed, lattice_id, sweep, n_hits, max_tries, sampler)


def hb_link(dims, U, site, mu, beta, seed, lattice_id, sweep, kind=0, n_hits=1, max_tries=64, sampler=KP,
            record=False):
    """Full update of the one link (site, mu) in place, every other link
    unchanged; kind 0 = heat bath, 1 = overrelaxation.  Returns the number
    of exhausted draws, and with record=True also an array [n_hits*3, 11]:
    per (hit, subgroup) step k, outcome (1 applied, 0 exhausted, -1 k = 0),
    alpha and the applied SU(2) factor r (re, im of r00, r01, r10, r11)."""
    _chk(U, dims)
    nh = n_hits if kind == 0 else 1
    rec = np.zeros((3 * nh, 11)) if record else None
    ex = lib().orc_hb_link(_ptr(_dims(dims)), _ptr(U), site, mu, kind, beta, seed, lattice_id, sweep, n_hits,
                           max_tries, sampler, _ptr(rec) if record else None)
    return (ex, rec) if record else ex


def or_pass(dims, U):
    _chk(U, dims)
    lib().orc_or_pass(_ptr(_dims(dims)), _ptr(U))


def or_pass_reversed(dims, U):
    _chk(U, dims)
    lib().orc_or_pass_reversed(_ptr(_dims(dims)), _ptr(U))


def sweep_hb_or(dims, U, beta, seed, lattice_id=0, first_sweep=0, n_sweeps=1, n_or=4, n_hb_hits=1,
                hb_max_tries=64, reunit_every=0, sampler=KP):
    """Returns (plaquette history, number of exhausted subgroup draws)."""
    _chk(U, dims)
    hist = np.zeros(max(n_sweeps, 1))
    ex = lib().orc_sweep_hb_or(_ptr(_dims(dims)), _ptr(U), beta, seed, lattice_id, first_sweep, n_sweeps,
                               n_or, n_hb_hits, hb_max_tries, reunit_every, sampler, _ptr(hist))
    return hist[:n_sweeps], ex


def hmc_momenta(dims, seed, lattice_id, traj) -> np.ndarray:
    p = np.zeros((volume(dims), 4, 8))
    lib().orc_hmc_momenta(_ptr(_dims(dims)), _ptr(p), seed, lattice_id, traj)
    return p


def hmc_force(dims, U, beta) -> np.ndarray:
    _chk(U, dims)
    F = np.zeros((volume(dims), 4, 8))
    lib().orc_hmc_force(_ptr(_dims(dims)), _ptr(U), beta, _ptr(F))
    return F


def hmc_kinetic(dims, p) -> float:
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_hmc_kinetic(_ptr(_dims(dims)), _ptr(p))


def md_leapfrog(dims, U, p, beta, eps, n_steps):
    _chk(U, dims)
    assert p.dtype == np.float64 and p.flags.c_contiguous
    lib().orc_md_leapfrog(_ptr(_dims(dims)), _ptr(U), _ptr(p), beta, eps, n_steps)


def hmc_trajectory(dims, U, beta, tau, n_steps, seed, lattice_id=0, traj=0, metropolis=1):
    """Returns (accepted, dH)."""
    _chk(U, dims)
    dH = np.zeros(1)
    acc = lib().orc_hmc_trajectory(_ptr(_dims(dims)), _ptr(U), beta, tau, n_steps, seed, lattice_id, traj,
                                   metropolis, _ptr(dH))
    return bool(acc), float(dH[0])


def restrict(dims_fine, Uf) -> np.ndarray:
    _chk(Uf, dims_fine)
    dc = [d // 2 for d in dims_fine]
    Uc = empty_field(dc)
    lib().orc_restrict(_ptr(_dims(dims_fine)), _ptr(Uf), _ptr(Uc))
    return Uc


def prolong_transfer(dims_coarse, Uc) -> np.ndarray:
    _chk(Uc, dims_coarse)
    Uf = empty_field([2 * d for d in dims_coarse])
    lib().orc_prolong_transfer(_ptr(_dims(dims_coarse)), _ptr(Uc), _ptr(Uf))
    return Uf


def partial_action(dims, U, d, beta=1.0) -> float:
    _chk(U, dims)
    return lib().orc_partial_action(_ptr(_dims(dims)), _ptr(U), d, beta)


def project_su3(M: np.ndarray) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float64).reshape(3, 3, 2)
    X = np.zeros((3, 3, 2))
    lib().orc_project_su3(_ptr(M), _ptr(X))
    return X


def ape_step(dims, U, d, c=0.05):
    _chk(U, dims)
    lib().orc_ape_step(_ptr(_dims(dims)), _ptr(U), d, c)


def prolongate(dims_coarse, Uc, c=0.05, rel_tol=1e-5, max_iter=10000):
    """Returns (fine field, iterations per stage)."""
    _chk(Uc, dims_coarse)
    Uf = empty_field([2 * d for d in dims_coarse])
    it = np.zeros(3, dtype=np.int32)
    lib().orc_prolongate(_ptr(_dims(dims_coarse)), _ptr(Uc), _ptr(Uf), c, rel_tol, max_iter, _ptr(it))
    return Uf, [int(x) for x in it]


def wilson_loop(dims, U, m, n) -> float:
    _chk(U, dims)
    return lib().orc_wilson_loop(_ptr(_dims(dims)), _ptr(U), m, n)


def partial_plaquette(dims, U, d) -> float:
    _chk(U, dims)
    return lib().orc_partial_plaquette(_ptr(_dims(dims)), _ptr(U), d)


def displaced_loop(dims, U, d, m, n) -> float:
    _chk(U, dims)
    return lib().orc_displaced_loop(_ptr(_dims(dims)), _ptr(U), d, m, n)


def displaced_2x2(dims, U, d) -> float:
    _chk(U, dims)
    return lib().orc_displaced_2x2(_ptr(_dims(dims)), _ptr(U), d)


def wilson_flow(dims, U, eps, n_steps):
    _chk(U, dims)
    lib().orc_wilson_flow(_ptr(_dims(dims)), _ptr(U), eps, n_steps)


def topological_charge(dims, U) -> float:
    _chk(U, dims)
    return lib().orc_topological_charge(_ptr(_dims(dims)), _ptr(U))


def clover_energy(dims, U) -> float:
    _chk(U, dims)
    return lib().orc_clover_energy(_ptr(_dims(dims)), _ptr(U))


def wilson_flow_adaptive(dims, U, t_end, tol=0.01, max_step=0.2, eps0=0.01, t_meas=()):
    """Adaptive-step RK3 flow of U (in place) to t_end; returns (E, Q, n_accepted,
    n_rejected) with E, Q measured at the ascending times t_meas (<= t_end)."""
    _chk(U, dims)
    tm = np.ascontiguousarray(t_meas, dtype=np.float64)
    if tm.size and (np.any(np.diff(tm) <= 0) or tm[-1] > t_end):
        raise ValueError("measurement times must ascend and not exceed t_end")
    E = np.full(tm.size, np.nan)
    Q = np.full(tm.size, np.nan)
    na, nr = C.c_int32(), C.c_int32()
    rc = lib().orc_wilson_flow_adaptive(_ptr(_dims(dims)), _ptr(U), t_end, tol, max_step, eps0, _ptr(tm),
                                        int(tm.size), _ptr(E), _ptr(Q), C.byref(na), C.byref(nr))
    if rc != 0:
        raise RuntimeError("adaptive flow did not converge")
    return E, Q, na.value, nr.value


def flow_step_distance(dims, U, h) -> float:
    """One RK3 flow step of size h in place; returns the embedded error distance."""
    _chk(U, dims)
    return lib().orc_flow_step_distance(_ptr(_dims(dims)), _ptr(U), h)


def flow_t0(t, E, target=0.3) -> float:
    """The t where t^2 E(t) crosses target, linearly interpolated (NaN if not bracketed)."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    out = C.c_double()
    rc = lib().orc_flow_t0(_ptr(t), _ptr(E), int(t.size), target, C.byref(out))
    return out.value if rc == 0 else float("nan")


def max_splaq(dims, U) -> float:
    _chk(U, dims)
    return lib().orc_max_splaq(_ptr(_dims(dims)), _ptr(U))


def max_su3_dev(dims, U) -> float:
    _chk(U, dims)
    return lib().orc_max_su3_dev(_ptr(_dims(dims)), _ptr(U))


def set_threads(n: int):
    lib().orc_set_threads(n)


def max_threads() -> int:
    return lib().orc_max_threads()
