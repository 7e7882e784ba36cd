"""FP64 CPU oracle for the twisted Wilson flow -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
oracle shares no code with it.  ``build()`` compiles ``tgf_oracle.c`` (SU(3),
Monte Carlo) and ``sun_oracle.c`` (SU(N), 2 <= N <= 8) with gcc (+OpenMP); the
functions below are ctypes wrappers over numpy arrays in the canonical layout
``complex128 [d3, d2, d1, d0, 4, N, N]``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tgf_oracle.c")
SRC_SUN = os.path.join(HERE, "sun_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force=True):
    """Compile the oracle (always, when force=True)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, SRC, SRC_SUN, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                  os.path.getmtime(SRC_SUN)):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        I4 = ctypes.POINTER(ctypes.c_int)
        lib.oracle_measure.argtypes = [P, I4, I4, I4, P]
        lib.oracle_force.argtypes = [P, I4, I4, I4, P]
        lib.oracle_expm.argtypes = [P, P]
        lib.oracle_densities.argtypes = [P, I4, I4, I4, P, P]
        lib.oracle_rk3_step.argtypes = [P, I4, I4, I4, ctypes.c_double]
        lib.oracle_flow.argtypes = [P, I4, I4, I4, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, P, ctypes.c_int]
        lib.oracle_mc.argtypes = [P, I4, I4, I4, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_ulonglong, ctypes.c_uint, ctypes.c_uint]
        lib.oracle_or_sweeps.argtypes = [P, I4, I4, I4, ctypes.c_int]
        lib.oracle_su2_samples.argtypes = [ctypes.c_double, ctypes.c_ulonglong, ctypes.c_int, P]
        lib.oracle_philox.argtypes = [P, ctypes.c_uint, ctypes.c_uint, P]
        C = ctypes.c_int
        lib.oracle_sun_measure.argtypes = [P, C, I4, I4, I4, P]
        lib.oracle_sun_densities.argtypes = [P, C, I4, I4, I4, P, P]
        lib.oracle_sun_force.argtypes = [P, C, I4, I4, I4, P]
        lib.oracle_sun_expm.argtypes = [C, P, P]
        lib.oracle_sun_rk3_step.argtypes = [P, C, I4, I4, I4, ctypes.c_double]
        lib.oracle_sun_flow.argtypes = [P, C, I4, I4, I4, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, P, C]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_get_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ivec(vals, n):
    vals = [0] * n if vals is None else list(vals)
    assert len(vals) == n
    return (ctypes.c_int * n)(*[int(v) for v in vals])


def _check_links(links, dims):
    d0, d1, d2, d3 = dims
    if not (isinstance(links, np.ndarray) and links.dtype == np.complex128
            and links.flags.c_contiguous and links.shape == (d3, d2, d1, d0, 4, 3, 3)):
        raise ValueError("links must be C-contiguous complex128 [d3,d2,d1,d0,4,3,3]")


PAPER_TWIST = (1, 0, 0, 0, 0, 0)   # n_01 = 1: the paper's (1,2)-plane twist, k = 1


def set_threads(n):
    _load().oracle_set_threads(int(n))


def get_threads():
    return int(_load().oracle_get_threads())


def measure(links, dims, twist=PAPER_TWIST, base=None):
    """-> dict(E, plaq, Q, action) at the current links."""
    _check_links(links, dims)
    out = np.zeros(4)
    rc = _load().oracle_measure(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6),
                                _ivec(base, 4), out.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_measure failed ({rc})")
    return dict(E=out[0], plaq=out[1], Q=out[2], action=out[3])


def densities(links, dims, twist=PAPER_TWIST, base=None):
    _check_links(links, dims)
    V = int(np.prod(dims))
    e = np.zeros(V)
    q = np.zeros(V)
    rc = _load().oracle_densities(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6),
                                  _ivec(base, 4), e.ctypes.data, q.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_densities failed ({rc})")
    return e, q


def force(links, dims, twist=PAPER_TWIST, base=None):
    _check_links(links, dims)
    F = np.zeros_like(links)
    rc = _load().oracle_force(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6),
                              _ivec(base, 4), F.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_force failed ({rc})")
    return F


def expm(A):
    A = np.ascontiguousarray(A, dtype=np.complex128).reshape(3, 3)
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().oracle_expm(A.ctypes.data, out.ctypes.data)
    return out


def rk3_step(links, dims, eps, twist=PAPER_TWIST, base=None):
    """One RK3 step in place."""
    _check_links(links, dims)
    rc = _load().oracle_rk3_step(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6),
                                 _ivec(base, 4), float(eps))
    if rc:
        raise RuntimeError(f"oracle_rk3_step failed ({rc})")


ROW_FIELDS = ("t", "E", "t2E", "plaq", "Q", "action")


def flow(links, dims, eps, t_end, meas_dt=0.0, t0=0.0, twist=PAPER_TWIST, base=None,
         max_rows=100000):
    """Flow ``links`` in place from t0 to t_end; returns rows [n, 6] with the
    columns ROW_FIELDS."""
    _check_links(links, dims)
    rows = np.zeros((max_rows, 6))
    n = _load().oracle_flow(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6),
                            _ivec(base, 4), float(eps), float(t0), float(t_end),
                            float(meas_dt), rows.ctypes.data, int(max_rows))
    if n < 0:
        raise RuntimeError(f"oracle_flow failed ({n})")
    return rows[:n].copy()


def mc(links, dims, b, n_hybrid, n_or, seed, sweep0=0, cfg=0, twist=PAPER_TWIST, base=None):
    """Hybrid over-relaxation in place: n_hybrid x (1 heat-bath + n_or OR sweeps),
    beta = 18 b (b = 1/lambda_0, sec. 3.1)."""
    _check_links(links, dims)
    rc = _load().oracle_mc(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6), _ivec(base, 4),
                           18.0 * float(b), int(n_hybrid), int(n_or), int(seed), int(sweep0),
                           int(cfg))
    if rc:
        raise RuntimeError(f"oracle_mc failed ({rc})")


def or_sweeps(links, dims, n, twist=PAPER_TWIST, base=None):
    _check_links(links, dims)
    rc = _load().oracle_or_sweeps(links.ctypes.data, _ivec(dims, 4), _ivec(twist, 6),
                                  _ivec(base, 4), int(n))
    if rc:
        raise RuntimeError(f"oracle_or_sweeps failed ({rc})")


def su2_samples(alpha, seed, n):
    out = np.zeros((n, 4))
    _load().oracle_su2_samples(float(alpha), int(seed), int(n), out.ctypes.data)
    return out


def philox(ctr, k0, k1):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox(c.ctypes.data, int(k0), int(k1), out.ctypes.data)
    return out


# ---------------------------------------------------------------- SU(N)
# Canonical layout complex128 [d3, d2, d1, d0, 4, N, N]; twist entries mod N.

def _check_links_n(links, dims):
    d0, d1, d2, d3 = dims
    if not (isinstance(links, np.ndarray) and links.dtype == np.complex128
            and links.flags.c_contiguous and links.ndim == 7
            and links.shape[:5] == (d3, d2, d1, d0, 4) and links.shape[5] == links.shape[6]):
        raise ValueError("links must be C-contiguous complex128 [d3,d2,d1,d0,4,N,N]")
    return links.shape[-1]


def sun_measure(links, dims, twist=PAPER_TWIST, base=None):
    """SU(N) observables -> dict(E, plaq, Q, action); N from the link shape."""
    n = _check_links_n(links, dims)
    out = np.zeros(4)
    rc = _load().oracle_sun_measure(links.ctypes.data, n, _ivec(dims, 4), _ivec(twist, 6),
                                    _ivec(base, 4), out.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_sun_measure failed ({rc})")
    return dict(E=out[0], plaq=out[1], Q=out[2], action=out[3])


def sun_densities(links, dims, twist=PAPER_TWIST, base=None):
    n = _check_links_n(links, dims)
    V = int(np.prod(dims))
    e = np.zeros(V)
    q = np.zeros(V)
    rc = _load().oracle_sun_densities(links.ctypes.data, n, _ivec(dims, 4), _ivec(twist, 6),
                                      _ivec(base, 4), e.ctypes.data, q.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_sun_densities failed ({rc})")
    return e, q


def sun_force(links, dims, twist=PAPER_TWIST, base=None):
    n = _check_links_n(links, dims)
    F = np.zeros_like(links)
    rc = _load().oracle_sun_force(links.ctypes.data, n, _ivec(dims, 4), _ivec(twist, 6),
                                  _ivec(base, 4), F.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_sun_force failed ({rc})")
    return F


def sun_expm(A):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    if _load().oracle_sun_expm(n, A.ctypes.data, out.ctypes.data):
        raise RuntimeError("oracle_sun_expm failed")
    return out


def sun_rk3_step(links, dims, eps, twist=PAPER_TWIST, base=None):
    n = _check_links_n(links, dims)
    rc = _load().oracle_sun_rk3_step(links.ctypes.data, n, _ivec(dims, 4), _ivec(twist, 6),
                                     _ivec(base, 4), float(eps))
    if rc:
        raise RuntimeError(f"oracle_sun_rk3_step failed ({rc})")


def sun_flow(links, dims, eps, t_end, meas_dt=0.0, t0=0.0, twist=PAPER_TWIST, base=None,
             max_rows=100000):
    """SU(N) flow in place; rows [n, 6] with the columns ROW_FIELDS."""
    n = _check_links_n(links, dims)
    rows = np.zeros((max_rows, 6))
    nr = _load().oracle_sun_flow(links.ctypes.data, n, _ivec(dims, 4), _ivec(twist, 6),
                                 _ivec(base, 4), float(eps), float(t0), float(t_end),
                                 float(meas_dt), rows.ctypes.data, int(max_rows))
    if nr < 0:
        raise RuntimeError(f"oracle_sun_flow failed ({nr})")
    return rows[:nr].copy()
