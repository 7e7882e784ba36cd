"""FP64 CPU oracle for the twisted Wilson flow -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
oracle shares no code with it.  ``build()`` compiles ``tgf_oracle.c`` with gcc
(+OpenMP); the functions below are ctypes wrappers over numpy arrays in the
canonical layout ``complex128 [d3, d2, d1, d0, 4, 3, 3]``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tgf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force=True):
    """Compile the oracle (always, when force=True)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
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
