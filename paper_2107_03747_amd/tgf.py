"""ctypes binding of libtgf.so (include/tgf.h), argument marshalling only.

Every function of the C ABI is exposed under its own name; ``Flow`` wraps a
context together with its workspace (a torch uint8 device tensor) and a HIP
stream.  All arithmetic runs in the library's kernels; torch only provides
device memory and streams.  Importing this module raises if libtgf.so has not
been built (``python -m paper_2107_03747_amd.build``) -- there is no CPU path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtgf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2107_03747_amd.build` (hipcc, gfx950)")

# torch ships its own HIP runtime with the same SONAME (libamdhip64.so.7) as
# the ROCm one libtgf.so links against.  Loading torch first makes libtgf.so
# bind to that same runtime, so device pointers and streams from torch are
# valid in the library; the other order would map two runtimes.
try:
    import torch as _torch  # noqa: F401
except ImportError:       # the library itself does not need torch
    _torch = None

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes():
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                p = line.split()[-1]
                if "libamdhip64" in os.path.basename(p):
                    paths.add(os.path.realpath(p))
    except OSError:
        pass
    return paths


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are mapped in this process "
                      f"({sorted(_hip_runtimes())}); import torch before loading libtgf.so")

# --- status / enums -----------------------------------------------------------
TGF_OK = 0
TGF_E_INVAL = -1
TGF_E_SIZE = -2
TGF_E_HIP = -3
TGF_E_NOT_SU3 = -4
TGF_E_NONFINITE = -5
TGF_E_STATE = -6
TGF_E_UNSUPPORTED = -7
STATUS_NAMES = {0: "TGF_OK", -1: "TGF_E_INVAL", -2: "TGF_E_SIZE", -3: "TGF_E_HIP",
                -4: "TGF_E_NOT_SU3", -5: "TGF_E_NONFINITE", -6: "TGF_E_STATE",
                -7: "TGF_E_UNSUPPORTED"}

TGF_F64_FULL = 0
TGF_F32_FULL = 1
TGF_F32_C12 = 2
STORAGES = {"f64": TGF_F64_FULL, "f32": TGF_F32_FULL, "f32c12": TGF_F32_C12}

TGF_NO_GRAPH = 1
TGF_TIMING = 2
TGF_MAX_ROWS = 4096
TGF_NOALLOC_MAX_SITES = 12582912

PAPER_TWIST = (1, 0, 0, 0, 0, 0)


class tgf_geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("twist", ctypes.c_int32 * 6)]


class tgf_obs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("t", "E", "t2E", "plaq", "Q", "action")]


class tgf_flow_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("t_end", ctypes.POINTER(ctypes.c_double)),
                ("meas_dt", ctypes.c_double), ("reunit_every", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class tgf_timing(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double), ("stage_launches", ctypes.c_int64),
                ("stage_bytes", ctypes.c_double), ("stage_site_updates", ctypes.c_double),
                ("measure_ms", ctypes.c_double), ("measure_launches", ctypes.c_int64)]


OBS_FIELDS = ("t", "E", "t2E", "plaq", "Q", "action")

_P = ctypes.c_void_p
_I = ctypes.c_int32
_st = ctypes.c_int
_sig = {
    "tgf_workspace_bytes": (ctypes.c_size_t, [_I, ctypes.POINTER(tgf_geom), _st]),
    "tgf_create": (_st, [ctypes.POINTER(_P), _I, ctypes.POINTER(tgf_geom), _st, _P,
                         ctypes.c_size_t, _P]),
    "tgf_workspace_bytes_sun": (ctypes.c_size_t, [_I, _I, ctypes.POINTER(tgf_geom), _st]),
    "tgf_create_sun": (_st, [ctypes.POINTER(_P), _I, _I, ctypes.POINTER(tgf_geom), _st, _P,
                             ctypes.c_size_t, _P]),
    "tgf_sun_variant_count": (_I, [_I]),
    "tgf_sun_rows_per_lane": (_I, [_I, _I]),
    "tgf_sun_variant_lds": (_I, [_I, _I]),
    "tgf_load_links": (_st, [_P, _I, _P, ctypes.c_double]),
    "tgf_load_links_all": (_st, [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_double)]),
    "tgf_store_links": (_st, [_P, _I, _P]),
    "tgf_get_time": (_st, [_P, _I, ctypes.POINTER(ctypes.c_double)]),
    "tgf_densities": (_st, [_P, _I, _P, _P]),
    "tgf_link_buffer": (_st, [_P, _I, ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(ctypes.c_size_t)]),
    "tgf_measure": (_st, [_P, ctypes.POINTER(tgf_obs)]),
    "tgf_flow": (_st, [_P, ctypes.POINTER(tgf_flow_params), ctypes.POINTER(tgf_obs), _I,
                       ctypes.POINTER(_I)]),
    "tgf_get_timing": (_st, [_P, ctypes.POINTER(tgf_timing)]),
    "tgf_unitarity": (_st, [_P, _I, ctypes.POINTER(ctypes.c_double)]),
    "tgf_autotune": (_st, [_P, ctypes.c_char_p]),
    "tgf_get_block": (_st, [_P, _I, ctypes.POINTER(_I)]),
    "tgf_set_block": (_st, [_P, _I, _I]),
    "tgf_set_variant": (_st, [_P, _I]),
    "tgf_get_variant": (_I, [_P]),
    "tgf_variant_count": (_I, []),
    "tgf_variant_name": (ctypes.c_char_p, [_I]),
    "tgf_stream_copy": (_st, [_P, _P, ctypes.c_size_t, _P]),
    "tgf_slice_charge": (_st, [_P, _I, ctypes.POINTER(ctypes.c_double), _I]),
    "tgf_mc": (_st, [_P, ctypes.c_double, _I, _I, ctypes.c_uint64, ctypes.c_uint32]),
    "tgf_latt_norm": (_st, [ctypes.c_double, _I, _I, ctypes.POINTER(ctypes.c_double)]),
    "tgf_coupling": (_st, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _I,
                           ctypes.c_double, _I, _I, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double)]),
    "tgf_charge_correlator": (_st, [ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), _I, _I, _I,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    "tgf_susceptibility": (_st, [ctypes.POINTER(ctypes.c_double), _I, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]),
    "tgf_measure_noalloc": (_st, [ctypes.POINTER(tgf_geom), _P, ctypes.c_double, _P, _P]),
    "tgf_stats_last_error": (ctypes.c_char_p, []),
    "tgf_last_error": (ctypes.c_char_p, []),
    "tgf_destroy": (None, [_P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_sig)


class TGFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status != TGF_OK:
        raise TGFError(status, tgf_last_error().decode())
    return status


def make_geoms(geoms):
    """geoms: list of (dims, twist) or of dims (paper twist)."""
    arr = (tgf_geom * len(geoms))()
    for k, g in enumerate(geoms):
        if len(g) == 2 and hasattr(g[0], "__len__"):
            dims, tw = g
        else:
            dims, tw = g, PAPER_TWIST
        arr[k].dims[:] = [int(x) for x in dims]
        arr[k].twist[:] = [int(x) for x in tw]
    return arr


def workspace_bytes(geoms, storage="f32c12"):
    g = make_geoms(geoms)
    return int(tgf_workspace_bytes(len(geoms), g, STORAGES[storage]))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Flow:
    """A flow context over one batch of configurations.

    geoms:   list of dims (d0, d1, d2, d3) or (dims, twist) pairs.
    storage: "f64" (plain FP64), "f32" (FP32 full), "f32c12" (FP32 rows 0, 1).
    nc:      None for the SU(3)-specialised kernels; 2..8 for the general SU(N)
             kernels (FP64 storage, links [d3,d2,d1,d0,4,nc,nc], twist mod nc).
    """

    def __init__(self, geoms, storage="f32c12", device="cuda", stream=None, nc=None):
        import torch
        self.torch = torch
        self.geoms = list(geoms)
        self.n = len(self.geoms)
        self.dims = [tuple(int(x) for x in (g[0] if hasattr(g[0], "__len__") else g))
                     for g in self.geoms]
        self.storage = storage
        self.nc = 3 if nc is None else int(nc)
        self.general = nc is not None
        self.device = torch.device(device)
        self._g = make_geoms(self.geoms)
        if self.general:
            nbytes = int(tgf_workspace_bytes_sun(self.nc, self.n, self._g, STORAGES[storage]))
        else:
            nbytes = int(tgf_workspace_bytes(self.n, self._g, STORAGES[storage]))
        if nbytes == 0:
            raise TGFError(TGF_E_INVAL, "invalid geometries, storage or nc: " +
                           tgf_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._ctx = ctypes.c_void_p()
        if self.general:
            check(tgf_create_sun(ctypes.byref(self._ctx), self.nc, self.n, self._g,
                                 STORAGES[storage], _ptr(self.workspace), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)))
        else:
            check(tgf_create(ctypes.byref(self._ctx), self.n, self._g, STORAGES[storage],
                             _ptr(self.workspace), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream)))

    def close(self):
        if self._ctx:
            tgf_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _links_ok(self, cfg, links):
        t = self.torch
        d0, d1, d2, d3 = self.dims[cfg]
        n = self.nc
        if not (links.is_cuda and links.dtype == t.complex128 and links.is_contiguous()
                and tuple(links.shape) == (d3, d2, d1, d0, 4, n, n)):
            raise ValueError("links must be a contiguous complex128 CUDA tensor "
                             f"[{d3},{d2},{d1},{d0},4,{n},{n}]")

    def _sync_in(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def load(self, cfg, links, t0=0.0):
        self._links_ok(cfg, links)
        self._sync_in()
        check(tgf_load_links(self._ctx, int(cfg), _ptr(links), float(t0)))

    def load_all(self, links_list, t0=0.0):
        assert len(links_list) == self.n
        for k, l in enumerate(links_list):
            self._links_ok(k, l)
        self._sync_in()
        ptrs = (ctypes.c_void_p * self.n)(*[l.data_ptr() for l in links_list])
        t0s = (ctypes.c_double * self.n)(*([float(t0)] * self.n if np.isscalar(t0) else
                                           [float(x) for x in t0]))
        check(tgf_load_links_all(self._ctx, ptrs, t0s))

    def store(self, cfg, out=None):
        t = self.torch
        dims = self.dims[cfg]
        if out is None:
            out = t.empty((dims[3], dims[2], dims[1], dims[0], 4, self.nc, self.nc),
                          dtype=t.complex128, device=self.device)
        self._links_ok(cfg, out)
        self._sync_in()
        check(tgf_store_links(self._ctx, int(cfg), _ptr(out)))
        t.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def time(self, cfg):
        v = ctypes.c_double()
        check(tgf_get_time(self._ctx, int(cfg), ctypes.byref(v)))
        return v.value

    def densities(self, cfg):
        """Per-site e(n) and q(n) of cfg (FP64 device tensors [V], site order)."""
        t = self.torch
        V = int(np.prod(self.dims[cfg]))
        e = t.empty(V, dtype=t.float64, device=self.device)
        q = t.empty(V, dtype=t.float64, device=self.device)
        self._sync_in()
        check(tgf_densities(self._ctx, int(cfg), _ptr(e), _ptr(q)))
        t.cuda.current_stream(self.device).wait_stream(self.stream)
        return e, q

    def link_buffer(self, cfg):
        """(byte offset in the workspace, bytes) of cfg's stored links."""
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        check(tgf_link_buffer(self._ctx, int(cfg), ctypes.byref(off), ctypes.byref(nb)))
        return int(off.value), int(nb.value)

    def measure(self):
        """-> structured numpy array [n_cfg] with OBS_FIELDS."""
        out = (tgf_obs * self.n)()
        self._sync_in()
        check(tgf_measure(self._ctx, out))
        return _obs_to_numpy(out, (self.n,))

    def flow(self, eps, t_end, meas_dt=0.0, reunit_every=0, flags=0, max_rows=None):
        """Flow every config to t_end (scalar or per config).
        -> numpy array [n_rows, n_cfg, 6] with columns OBS_FIELDS."""
        te = [float(t_end)] * self.n if np.isscalar(t_end) else [float(x) for x in t_end]
        assert len(te) == self.n
        te_arr = (ctypes.c_double * self.n)(*te)
        p = tgf_flow_params(float(eps), te_arr, float(meas_dt), int(reunit_every), int(flags))
        if max_rows is None:
            span = max(te[k] - self.time(k) for k in range(self.n))
            est = 2 + (int(span / meas_dt + 1e-9) + 1 if meas_dt > 0 else 0)
            max_rows = min(TGF_MAX_ROWS, max(2, est + 2))
        rows = (tgf_obs * (max_rows * self.n))()
        nr = ctypes.c_int32()
        self._sync_in()
        check(tgf_flow(self._ctx, ctypes.byref(p), rows, int(max_rows), ctypes.byref(nr)))
        a = np.ctypeslib.as_array(ctypes.cast(rows, ctypes.POINTER(ctypes.c_double)),
                                  shape=(max_rows * self.n * 6,))
        return a.reshape(max_rows, self.n, 6)[: nr.value].copy()

    def slice_charge(self, dir=3):
        """Topological charge per slice of direction dir -> [n_cfg, max extent]."""
        ms = max(d[dir] for d in self.dims)
        out = np.zeros((self.n, ms))
        self._sync_in()
        check(tgf_slice_charge(self._ctx, int(dir),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ms))
        return out

    def mc(self, b, n_hybrid=1, n_or=0, seed=0, sweep0=0):
        """Hybrid over-relaxation in place on every configuration: n_hybrid x
        (one heat-bath sweep + n_or over-relaxation sweeps), beta = 18 b; needs
        f64 storage and even extents.  Returns the next free sweep index."""
        self._sync_in()
        check(tgf_mc(self._ctx, float(b), int(n_hybrid), int(n_or), int(seed), int(sweep0)))
        return int(sweep0) + int(n_hybrid) * (1 + int(n_or))

    def timing(self):
        t = tgf_timing()
        check(tgf_get_timing(self._ctx, ctypes.byref(t)))
        return {n: getattr(t, n) for n, _ in tgf_timing._fields_}

    def unitarity(self, cfg):
        out = (ctypes.c_double * 2)()
        self._sync_in()
        check(tgf_unitarity(self._ctx, int(cfg), out))
        return out[0], out[1]

    def autotune(self, cache_path=None):
        check(tgf_autotune(self._ctx, cache_path.encode() if cache_path else None))
        return self.variant

    def set_variant(self, v):
        check(tgf_set_variant(self._ctx, int(v)))

    def block(self, cfg):
        """Sites per work-group of the LDS-staged variants for cfg."""
        v = ctypes.c_int32()
        check(tgf_get_block(self._ctx, int(cfg), ctypes.byref(v)))
        return int(v.value)

    def set_block(self, cfg, sites):
        """Pin cfg's LDS work-group shape (0 = the default whole-plane shape)."""
        check(tgf_set_block(self._ctx, int(cfg), int(sites)))

    @property
    def variant(self):
        return int(tgf_get_variant(self._ctx))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_stats(status):
    if status != TGF_OK:
        raise TGFError(status, tgf_stats_last_error().decode())


def latt_norm(c, Lt, N=3):
    """Lattice normalisation N(c, Lt) of the coupling (host FP64)."""
    out = ctypes.c_double()
    _check_stats(tgf_latt_norm(float(c), int(Lt), int(N), ctypes.byref(out)))
    return out.value


def coupling(t2E, Q, c, Lt, N=3):
    """(lambda_TGF, jackknife error) from per-configuration t^2 E and Q."""
    t2E = np.ascontiguousarray(t2E, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    lam, err = ctypes.c_double(), ctypes.c_double()
    _check_stats(tgf_coupling(_dptr(t2E), _dptr(Q), len(t2E), float(c), int(Lt), int(N),
                              ctypes.byref(lam), ctypes.byref(err)))
    return lam.value, err.value


def charge_correlator(q, Q):
    """C(x0) and its jackknife error from slice charges q[n_cfg, T] and Q[n_cfg]."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    n, T = q.shape
    C = np.zeros(T)
    E = np.zeros(T)
    _check_stats(tgf_charge_correlator(_dptr(q), _dptr(Q), n, T, T, _dptr(C), _dptr(E)))
    return C, E


def susceptibility(Q, V):
    """chi = <Q^2>/V and its jackknife error from total charges Q[n_cfg]."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    chi = ctypes.c_double()
    err = ctypes.c_double()
    _check_stats(tgf_susceptibility(_dptr(Q), len(Q), float(V), ctypes.byref(chi),
                                    ctypes.byref(err)))
    return chi.value, err.value


def variant_names():
    return [tgf_variant_name(v).decode() for v in range(tgf_variant_count())]


def _obs_to_numpy(arr, shape):
    a = np.ctypeslib.as_array(ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)),
                              shape=(int(np.prod(shape)) * 6,))
    return a.reshape(shape + (6,)).copy()


def stream_copy(dst, src, nbytes=None, stream=None):
    """Plain HBM copy kernel (counter calibration)."""
    import torch
    nbytes = nbytes if nbytes is not None else src.numel() * src.element_size()
    s = stream if stream is not None else torch.cuda.current_stream()
    check(tgf_stream_copy(_ptr(dst), _ptr(src), int(nbytes), ctypes.c_void_p(s.cuda_stream)))
