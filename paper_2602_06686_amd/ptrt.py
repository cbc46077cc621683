"""Python binding of libptrt (include/ptrt.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own; all lattice work runs in the HIP kernels of
``libptrt.so``.  Host arrays are NumPy float64 (uint8 for masks) in the C
layouts: rho [nz,ny,nx], u [3,nz,ny,nx], f [Q,nz,ny,nx].

``torch`` is imported before the library is loaded on purpose: the library
then binds to the HIP runtime that torch already loaded, so a
``torch.cuda.Stream`` can be handed to :func:`ptrt_set_stream` and timed with
``torch.cuda.Event``.  There is no CPU fallback: if ``libptrt.so`` is missing
the import of this module fails.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede loading libptrt.so, see above)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libptrt.so")

PTRT_D2Q9, PTRT_D3Q19, PTRT_D3Q27 = 0, 1, 2
PTRT_F64, PTRT_F32, PTRT_F16, PTRT_BF16, PTRT_F16_SR, PTRT_BF16_SR = 0, 1, 2, 3, 4, 5
PTRT_MODEL_PTRT, PTRT_MODEL_TRT_RLB, PTRT_MODEL_TRT, PTRT_MODEL_PTRT_EXACT = 0, 1, 2, 3
MODEL = {"ptrt": PTRT_MODEL_PTRT, "trt-rlb": PTRT_MODEL_TRT_RLB, "trt": PTRT_MODEL_TRT,
         "ptrt-exact": PTRT_MODEL_PTRT_EXACT}
STORAGE = {"f64": PTRT_F64, "f32": PTRT_F32, "f16": PTRT_F16, "bf16": PTRT_BF16,
           "f16sr": PTRT_F16_SR, "bf16sr": PTRT_BF16_SR}
PTRT_FORCING_SCHEME2, PTRT_FORCING_SCHEME2_G, PTRT_FORCING_GUO = 0, 1, 2
FORCING = {"scheme2": PTRT_FORCING_SCHEME2, "scheme2+g": PTRT_FORCING_SCHEME2_G,
           "guo": PTRT_FORCING_GUO}
Q_OF = {PTRT_D2Q9: 9, PTRT_D3Q19: 19, PTRT_D3Q27: 27}

STATUS = {0: "PTRT_OK", -1: "PTRT_EINVAL", -2: "PTRT_ETAU", -3: "PTRT_ENOMEM",
          -4: "PTRT_EDEVICE", -5: "PTRT_EDIVERGED", -6: "PTRT_ESTATE"}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p


class PtrtError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code


class ptrt_instance_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("tau_plus", ctypes.c_double), ("Lambda", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("solid_mask", _u8p)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2602_06686_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

_SIGS = {
    "ptrt_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double, _dp, _u8p,
                                   ctypes.POINTER(_vp)]),
    "ptrt_set_storage": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_set_model": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_set_forcing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_set_open_x": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
    "ptrt_set_steps_per_pass": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_last_pass": (ctypes.c_int, [_vp, _ip, _dp]),
    "ptrt_momentum_exchange": (ctypes.c_int, [_vp, _dp]),
    "ptrt_momentum_exchange_noalloc": (ctypes.c_int, [_vp, _dp]),
    "ptrt_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ptrt_init_equilibrium": (ctypes.c_int, [_vp, _dp, _dp]),
    "ptrt_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_moments": (ctypes.c_int, [_vp, _dp, _dp]),
    "ptrt_diagnostics": (ctypes.c_int, [_vp, _dp, _dp]),
    "ptrt_get_populations": (ctypes.c_int, [_vp, _dp]),
    "ptrt_set_populations": (ctypes.c_int, [_vp, _dp]),
    "ptrt_get_time": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_longlong)]),
    "ptrt_set_divergence_check": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_divergence_step": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_longlong)]),
    "ptrt_last_error": (ctypes.c_char_p, [_vp]),
    "ptrt_destroy": (ctypes.c_int, [_vp]),
    "ptrt_velocity_set": (ctypes.c_int, [ctypes.c_int, _ip, _dp]),
    "ptrt_bytes_per_node": (ctypes.c_double, [_vp]),
    "ptrt_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ptrt_instance_desc),
                                         ctypes.c_int, ctypes.POINTER(_vp)]),
    "ptrt_batch_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ptrt_batch_init_equilibrium": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "ptrt_batch_set_plan": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]),
    "ptrt_batch_autotune": (ctypes.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "ptrt_batch_set_plan2": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int]),
    "ptrt_batch_get_plan2": (ctypes.c_int, [_vp, _ip]),
    "ptrt_batch_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_batch_set_steps_per_pass": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_batch_last_pass": (ctypes.c_int, [_vp, _ip, _dp]),
    "ptrt_batch_step_separate": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ptrt_batch_moments": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "ptrt_batch_get_populations": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "ptrt_batch_diagnostics": (ctypes.c_int, [_vp, _dp, _dp]),
    "ptrt_batch_nodes": (ctypes.c_longlong, [_vp]),
    "ptrt_batch_bytes_per_step": (ctypes.c_double, [_vp]),
    "ptrt_batch_last_error": (ctypes.c_char_p, [_vp]),
    "ptrt_batch_destroy": (ctypes.c_int, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _check(rc, handle, batch=False):
    if rc != 0:
        msg = (_lib.ptrt_batch_last_error if batch else _lib.ptrt_last_error)(handle)
        raise PtrtError(rc, msg.decode() if msg else "")
    return rc


def _f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape} values, got array of shape {a.shape}")
    return a.reshape(shape)


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


# ------------------------------------------------------------ single lattice

class Handle:
    """An open ptrt_ctx with the sizes the marshalling needs."""

    def __init__(self, ptr, lattice, nx, ny, nz):
        self.ptr = ptr
        self.lattice = lattice
        self.Q = Q_OF[lattice]
        self.shape = (nz, ny, nx)

    @property
    def value(self):
        return self.ptr.value


def ptrt_create(lattice, nx, ny, nz, tau_plus, Lambda, force=None, solid_mask=None):
    f3 = None
    if force is not None:
        f3 = np.zeros(3)
        g = np.asarray(force, dtype=np.float64).ravel()
        f3[: g.size] = g
    m = None
    if solid_mask is not None:
        m = np.ascontiguousarray(np.asarray(solid_mask, dtype=np.uint8).reshape(nz, ny, nx))
    out = _vp()
    rc = _lib.ptrt_create(lattice, nx, ny, nz, tau_plus, Lambda, _ptr(f3), _ptr(m, _u8p),
                          ctypes.byref(out))
    _check(rc, None)
    return Handle(out, lattice, nx, ny, nz)


def ptrt_set_storage(h, storage):
    storage = STORAGE.get(storage, storage)
    return _check(_lib.ptrt_set_storage(h.ptr, storage), h.ptr)


def ptrt_set_model(h, model):
    model = MODEL.get(model, model)
    return _check(_lib.ptrt_set_model(h.ptr, model), h.ptr)


def ptrt_set_forcing(h, forcing):
    forcing = FORCING.get(forcing, forcing)
    return _check(_lib.ptrt_set_forcing(h.ptr, forcing), h.ptr)


def ptrt_set_steps_per_pass(h, steps):
    return _check(_lib.ptrt_set_steps_per_pass(h.ptr, int(steps)), h.ptr)


def ptrt_last_pass(h):
    """(steps covered, algorithmic HBM bytes) of the most recent kernel pass."""
    steps = ctypes.c_int()
    nbytes = ctypes.c_double()
    _check(_lib.ptrt_last_pass(h.ptr, ctypes.byref(steps), ctypes.byref(nbytes)), h.ptr)
    return steps.value, nbytes.value


def ptrt_set_open_x(h, u_in, rho_out):
    return _check(_lib.ptrt_set_open_x(h.ptr, float(u_in), float(rho_out)), h.ptr)


def ptrt_momentum_exchange(h):
    F = np.zeros(3)
    _check(_lib.ptrt_momentum_exchange(h.ptr, _ptr(F)), h.ptr)
    return F


def ptrt_momentum_exchange_noalloc(h):
    F = np.zeros(3)
    _check(_lib.ptrt_momentum_exchange_noalloc(h.ptr, _ptr(F)), h.ptr)
    return F


def ptrt_set_stream(h, stream):
    return _check(_lib.ptrt_set_stream(h.ptr, _stream_handle(stream)), h.ptr)


def ptrt_init_equilibrium(h, rho=None, u=None):
    r = None if rho is None else _f64(rho, h.shape)
    uu = None
    if u is not None:
        u = np.asarray(u, dtype=np.float64)
        uu = np.zeros((3,) + h.shape)
        uu[: u.shape[0]] = u.reshape((u.shape[0],) + h.shape)
    return _check(_lib.ptrt_init_equilibrium(h.ptr, _ptr(r), _ptr(uu)), h.ptr)


def ptrt_step(h, n=1):
    return _check(_lib.ptrt_step(h.ptr, int(n)), h.ptr)


def ptrt_moments(h):
    rho = np.empty(h.shape)
    u = np.empty((3,) + h.shape)
    _check(_lib.ptrt_moments(h.ptr, _ptr(rho), _ptr(u)), h.ptr)
    return rho, u


def ptrt_diagnostics(h, raise_on_divergence=True):
    m = ctypes.c_double()
    k = ctypes.c_double()
    rc = _lib.ptrt_diagnostics(h.ptr, ctypes.byref(m), ctypes.byref(k))
    if rc != -5 or raise_on_divergence:
        _check(rc, h.ptr)
    return m.value, k.value


def ptrt_get_populations(h):
    f = np.empty((h.Q,) + h.shape)
    _check(_lib.ptrt_get_populations(h.ptr, _ptr(f)), h.ptr)
    return f


def ptrt_set_populations(h, f):
    f = _f64(f, (h.Q,) + h.shape)
    return _check(_lib.ptrt_set_populations(h.ptr, _ptr(f)), h.ptr)


def ptrt_get_time(h):
    t = ctypes.c_longlong()
    _check(_lib.ptrt_get_time(h.ptr, ctypes.byref(t)), h.ptr)
    return t.value


def ptrt_set_divergence_check(h, every):
    return _check(_lib.ptrt_set_divergence_check(h.ptr, int(every)), h.ptr)


def ptrt_divergence_step(h):
    """Earliest checked step with a non-finite state, or -1."""
    t = ctypes.c_longlong()
    _check(_lib.ptrt_divergence_step(h.ptr, ctypes.byref(t)), h.ptr)
    return t.value


def ptrt_last_error(h=None):
    return _lib.ptrt_last_error(None if h is None else h.ptr).decode()


def ptrt_destroy(h):
    if h is not None and h.ptr:
        rc = _lib.ptrt_destroy(h.ptr)
        h.ptr = _vp()
        return rc
    return 0


def ptrt_velocity_set(lattice):
    if lattice not in Q_OF:
        raise PtrtError(-1, f"unknown lattice {lattice}")
    Q = Q_OF[lattice]
    e = np.zeros((Q, 3), dtype=np.intc)
    w = np.zeros(Q)
    rc = _lib.ptrt_velocity_set(lattice, _ptr(e, _ip), _ptr(w))
    if rc != Q:
        raise PtrtError(rc, "ptrt_velocity_set failed")
    return e.astype(np.int64), w


def ptrt_bytes_per_node(h):
    return _lib.ptrt_bytes_per_node(h.ptr)


class Lattice:
    """Convenience owner of one handle: create / init / step / read back."""

    def __init__(self, lattice, nx, ny, nz, tau_plus, Lambda, force=None, solid_mask=None,
                 storage="f32", stream=None, model="ptrt", forcing="scheme2", open_x=None,
                 steps_per_pass=2):
        self.h = ptrt_create(lattice, nx, ny, nz, tau_plus, Lambda, force, solid_mask)
        try:
            ptrt_set_storage(self.h, storage)
            if model != "ptrt":
                ptrt_set_model(self.h, model)
            if forcing != "scheme2":
                ptrt_set_forcing(self.h, forcing)
            if open_x is not None:
                ptrt_set_open_x(self.h, *open_x)
            if steps_per_pass != 2:
                ptrt_set_steps_per_pass(self.h, steps_per_pass)
            if stream is not None:
                ptrt_set_stream(self.h, stream)
        except Exception:
            ptrt_destroy(self.h)
            raise

    def init_equilibrium(self, rho=None, u=None):
        ptrt_init_equilibrium(self.h, rho, u)

    def step(self, n=1):
        ptrt_step(self.h, n)

    def moments(self):
        return ptrt_moments(self.h)

    def diagnostics(self, raise_on_divergence=True):
        return ptrt_diagnostics(self.h, raise_on_divergence)

    def populations(self):
        return ptrt_get_populations(self.h)

    def momentum_exchange(self):
        return ptrt_momentum_exchange(self.h)

    def last_pass(self):
        return ptrt_last_pass(self.h)

    def set_populations(self, f):
        ptrt_set_populations(self.h, f)

    def set_divergence_check(self, every):
        ptrt_set_divergence_check(self.h, every)

    def divergence_step(self):
        return ptrt_divergence_step(self.h)

    @property
    def t(self):
        return ptrt_get_time(self.h)

    @property
    def bytes_per_node(self):
        return ptrt_bytes_per_node(self.h)

    def close(self):
        ptrt_destroy(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ batching

class BatchHandle:
    def __init__(self, ptr, sizes):
        self.ptr = ptr
        self.sizes = sizes  # [(nx, ny)]


def ptrt_batch_create(specs, storage="f32"):
    """specs: iterable of dicts with nx, ny, tau_plus, Lambda, g (3), mask [1,ny,nx] or None."""
    specs = list(specs)
    arr = (ptrt_instance_desc * len(specs))()
    keep = []
    for k, s in enumerate(specs):
        d = arr[k]
        d.nx, d.ny = int(s["nx"]), int(s["ny"])
        d.tau_plus, d.Lambda = float(s["tau_plus"]), float(s["Lambda"])
        g = list(s.get("g", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
        for a in range(3):
            d.force[a] = float(g[a])
        m = s.get("mask")
        if m is not None:
            m = np.ascontiguousarray(np.asarray(m, dtype=np.uint8).reshape(d.ny, d.nx))
            keep.append(m)
            d.solid_mask = m.ctypes.data_as(_u8p)
        else:
            d.solid_mask = None
    out = _vp()
    rc = _lib.ptrt_batch_create(len(specs), arr, STORAGE.get(storage, storage), ctypes.byref(out))
    _check(rc, None, batch=True)
    return BatchHandle(out, [(int(s["nx"]), int(s["ny"])) for s in specs])


def ptrt_batch_set_stream(b, stream):
    return _check(_lib.ptrt_batch_set_stream(b.ptr, _stream_handle(stream)), b.ptr, True)


def ptrt_batch_init_equilibrium(b, k, rho=None, u=None):
    nx, ny = b.sizes[k]
    r = None if rho is None else _f64(rho, (1, ny, nx))
    uu = None
    if u is not None:
        u = np.asarray(u, dtype=np.float64)
        uu = np.zeros((3, 1, ny, nx))
        uu[: u.shape[0]] = u.reshape((u.shape[0], 1, ny, nx))
    return _check(_lib.ptrt_batch_init_equilibrium(b.ptr, k, _ptr(r), _ptr(uu)), b.ptr, True)


def ptrt_batch_set_plan(b, tile_x, tile_y, blocks=0, xcd_order=0):
    return _check(_lib.ptrt_batch_set_plan(b.ptr, tile_x, tile_y, blocks, xcd_order), b.ptr, True)


def ptrt_batch_autotune(b):
    v = [ctypes.c_int() for _ in range(4)]
    _check(_lib.ptrt_batch_autotune(b.ptr, *[ctypes.byref(x) for x in v]), b.ptr, True)
    return tuple(x.value for x in v)


def ptrt_batch_set_plan2(b, rows, masked_rows, waves=4, blocks=0, concurrent=0):
    return _check(_lib.ptrt_batch_set_plan2(b.ptr, int(rows), int(masked_rows), int(waves),
                                            int(blocks), int(concurrent)), b.ptr, True)


def ptrt_batch_get_plan2(b):
    """(rows, masked_rows, waves, blocks, concurrent) of the two-step plan."""
    v = (ctypes.c_int * 5)()
    _check(_lib.ptrt_batch_get_plan2(b.ptr, v), b.ptr, True)
    return tuple(v)


def ptrt_batch_step(b, n=1):
    return _check(_lib.ptrt_batch_step(b.ptr, int(n)), b.ptr, True)


def ptrt_batch_set_steps_per_pass(b, steps):
    return _check(_lib.ptrt_batch_set_steps_per_pass(b.ptr, int(steps)), b.ptr, True)


def ptrt_batch_last_pass(b):
    """(steps covered, algorithmic HBM bytes) of the most recent pass."""
    steps = ctypes.c_int()
    nbytes = ctypes.c_double()
    _check(_lib.ptrt_batch_last_pass(b.ptr, ctypes.byref(steps), ctypes.byref(nbytes)), b.ptr, True)
    return steps.value, nbytes.value


def ptrt_batch_step_separate(b, n=1):
    return _check(_lib.ptrt_batch_step_separate(b.ptr, int(n)), b.ptr, True)


def ptrt_batch_moments(b, k):
    nx, ny = b.sizes[k]
    rho = np.empty((1, ny, nx))
    u = np.empty((3, 1, ny, nx))
    _check(_lib.ptrt_batch_moments(b.ptr, k, _ptr(rho), _ptr(u)), b.ptr, True)
    return rho, u


def ptrt_batch_get_populations(b, k):
    nx, ny = b.sizes[k]
    f = np.empty((9, 1, ny, nx))
    _check(_lib.ptrt_batch_get_populations(b.ptr, k, _ptr(f)), b.ptr, True)
    return f


def ptrt_batch_diagnostics(b, raise_on_divergence=True):
    n = len(b.sizes)
    m = np.empty(n)
    k = np.empty(n)
    rc = _lib.ptrt_batch_diagnostics(b.ptr, _ptr(m), _ptr(k))
    if rc != -5 or raise_on_divergence:
        _check(rc, b.ptr, True)
    return m, k


def ptrt_batch_nodes(b):
    return _lib.ptrt_batch_nodes(b.ptr)


def ptrt_batch_bytes_per_step(b):
    return _lib.ptrt_batch_bytes_per_step(b.ptr)


def ptrt_batch_last_error(b=None):
    return _lib.ptrt_batch_last_error(None if b is None else b.ptr).decode()


def ptrt_batch_destroy(b):
    if b is not None and b.ptr:
        rc = _lib.ptrt_batch_destroy(b.ptr)
        b.ptr = _vp()
        return rc
    return 0
