"""ctypes front end of the C oracle (``ptrt_oracle.c``).  Test infrastructure.

Arrays cross the boundary in the layout the C-ABI of the GPU library also
uses for host data: populations ``[Q][nz][ny][nx]``, density ``[nz][ny][nx]``,
velocity ``[3][nz][ny][nx]`` (component-major), solid mask ``uint8
[nz][ny][nx]`` with 1 = solid.  Internally the oracle keeps ``[node][Q]``;
the transposes happen here.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptrt_oracle.so")

D2Q9, D3Q19, D3Q27 = 0, 1, 2
_Q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}

# collision models of the oracle
PTRT, TRT, PTRT_EXACT, PTRT_GHOST = 0, 2, 3, 4
# forcing schemes: Scheme II without G_i, Scheme II with G_i, Scheme I (Guo)
FORCING_II, FORCING_II_G, FORCING_GUO = 0, 1, 2

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_llp = ctypes.POINTER(ctypes.c_longlong)

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = bind(ctypes.CDLL(LIB_PATH))
    return _lib


def bind(lib):
    """Declare the argument types of the oracle's C functions on a loaded
    library (the oracle itself, or a copy built from altered source by the
    tests that check that the pins catch planted mistakes)."""
    lib.ptrt_oracle_lattice.argtypes = [ctypes.c_int, _ip, _dp, _ip]
    lib.ptrt_oracle_ghost_basis.argtypes = [ctypes.c_int, _dp, _dp]
    lib.ptrt_oracle_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
    lib.ptrt_oracle_collide.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp,
                                        ctypes.c_double, ctypes.c_double, _dp]
    lib.ptrt_oracle_collide_tau.argtypes = lib.ptrt_oracle_collide.argtypes
    lib.ptrt_oracle_moments.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.ptrt_oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    _dp, _u8p, _dp, ctypes.c_int, ctypes.c_int]
    lib.ptrt_oracle_run_model.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, _dp, _u8p, _dp, ctypes.c_int,
                                          ctypes.c_int]
    lib.ptrt_oracle_collide_trt.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp,
                                            ctypes.c_double, ctypes.c_double, _dp]
    lib.ptrt_oracle_step_sampled.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             _dp, _u8p, _dp, ctypes.c_int, _llp, _dp]
    lib.ptrt_oracle_diagnostics.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _u8p,
                                            _dp, _dp]
    lib.ptrt_oracle_collide_model.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                              _dp, ctypes.c_double, ctypes.c_double, _dp]
    lib.ptrt_oracle_fifth_modes.argtypes = [ctypes.c_int, _dp]
    lib.ptrt_oracle_run_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _dp, _u8p, _dp,
                                       ctypes.c_int, ctypes.c_int]
    lib.ptrt_oracle_run_open.argtypes = lib.ptrt_oracle_run_ex.argtypes + [_dp]
    lib.ptrt_oracle_apply_outlet.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, _u8p, _dp, ctypes.c_double]
    lib.ptrt_oracle_momentum_exchange.argtypes = [
        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _u8p, _dp, _dp, _dp]
    lib.ptrt_oracle_phi_gradient.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, _dp, _u8p, _dp, _dp]
    lib.ptrt_oracle_collide_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                           ctypes.c_double, _dp]
    lib.ptrt_oracle_max_threads.argtypes = []
    return lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _g3(g):
    out = np.zeros(3, dtype=np.float64)
    if g is not None:
        g = np.asarray(g, dtype=np.float64).ravel()
        out[: g.size] = g
    return out


def max_threads():
    return _load().ptrt_oracle_max_threads()


def lattice(lat):
    """Velocities e [Q,3] (int), weights w [Q], opposite index [Q]."""
    Q = _Q[lat]
    e = np.zeros((Q, 3), dtype=np.intc)
    w = np.zeros(Q, dtype=np.float64)
    opp = np.zeros(Q, dtype=np.intc)
    assert _load().ptrt_oracle_lattice(lat, _p(e, _ip), _p(w), _p(opp, _ip)) == Q
    return e.astype(np.int64), w, opp.astype(np.int64)


def ghost_basis(lat):
    """Orthogonal ghost basis phi [NG,Q] and its weighted norms [NG]."""
    Q = _Q[lat]
    phi = np.zeros((7, Q))
    nrm = np.zeros(7)
    ng = _load().ptrt_oracle_ghost_basis(lat, _p(phi), _p(nrm))
    return phi[:ng].copy(), nrm[:ng].copy()


def equilibrium(lat, rho, u):
    """f^eq for rho [n], u [n,D or 3] -> [n,Q]."""
    rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).ravel())
    n = rho.size
    u3 = np.zeros((n, 3))
    u = np.asarray(u, dtype=np.float64).reshape(n, -1)
    u3[:, : u.shape[1]] = u
    out = np.zeros((n, _Q[lat]))
    _load().ptrt_oracle_equilibrium(lat, n, _p(rho), _p(u3), _p(out))
    return out


def collide(lat, f, g, tau_plus, Lambda=None, tau_minus=None):
    """P-TRT post-collision state of independent nodes, f [n,Q] -> [n,Q]."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, _Q[lat]))
    out = np.zeros_like(f)
    g3 = _g3(g)
    if tau_minus is not None:
        _load().ptrt_oracle_collide_tau(lat, f.shape[0], _p(f), _p(g3), tau_plus, tau_minus, _p(out))
    else:
        _load().ptrt_oracle_collide(lat, f.shape[0], _p(f), _p(g3), tau_plus, Lambda, _p(out))
    return out


def collide_trt(lat, f, g, tau_plus, tau_minus):
    """Standard TRT (no ghost subtraction) of independent nodes, [n,Q] -> [n,Q]."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, _Q[lat]))
    out = np.zeros_like(f)
    _load().ptrt_oracle_collide_trt(lat, f.shape[0], _p(f), _p(_g3(g)), tau_plus, tau_minus,
                                    _p(out))
    return out


def collide_model(lat, model, f, g, tau_plus, tau_minus):
    """Collision of independent nodes with an oracle model (PTRT, TRT,
    PTRT_EXACT, PTRT_GHOST), [n,Q] -> [n,Q]."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, _Q[lat]))
    out = np.zeros_like(f)
    rc = _load().ptrt_oracle_collide_model(lat, int(model), f.shape[0], _p(f), _p(_g3(g)),
                                           tau_plus, tau_minus, _p(out))
    if rc != 0:
        raise ValueError(f"oracle collide_model failed ({rc})")
    return out


def collide_ex(lat, model, forcing, f, g, tau_plus, tau_minus, dphi=None):
    """Collision of independent nodes with a model and a forcing scheme;
    dphi [n,3] = d_a (rho u_a^3) per node (Scheme II with G_i)."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, _Q[lat]))
    out = np.zeros_like(f)
    dp = None
    if dphi is not None:
        dp = np.ascontiguousarray(np.asarray(dphi, dtype=np.float64).reshape(f.shape[0], 3))
    rc = _load().ptrt_oracle_collide_ex(lat, int(model), int(forcing), f.shape[0], _p(f),
                                        _p(_g3(g)), _p(dp) if dp is not None else None,
                                        tau_plus, tau_minus, _p(out))
    if rc != 0:
        raise ValueError(f"oracle collide_ex failed ({rc})")
    return out


def fifth_modes(lat=D3Q27):
    """psi^(5,k) of D3Q27 as rows [3,27] (App. A.3)."""
    psi = np.zeros((3, 27))
    assert _load().ptrt_oracle_fifth_modes(lat, _p(psi)) == 3
    return psi


def node_moments(lat, f, g=None):
    """rho [n], u [n,3] of independent nodes f [n,Q] (Eq. macro)."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1, _Q[lat]))
    n = f.shape[0]
    rho = np.zeros(n)
    u3 = np.zeros((n, 3))
    _load().ptrt_oracle_moments(lat, n, _p(f), _p(_g3(g)), _p(rho), _p(u3))
    return rho, u3


class Lattice:
    """A whole lattice advanced by the oracle.

    ``f`` holds the pre-collision populations at the current time, in the
    oracle's node-major layout ``[N][Q]``.  ``nthreads`` > 0 sets the
    OpenMP thread count for this and every later call in the process
    (OpenMP's setting is global); 0 keeps the current setting.
    """

    def __init__(self, lat, nx, ny, nz, tau_plus, Lambda, g=None, solid=None,
                 tau_minus=None, nthreads=0, model=0, forcing=0, open_x=None):
        self.lat = lat
        # open_x = (u_in, rho_out): velocity inlet at x = -1/2 and Zou-He
        # pressure outlet at x = nx - 1 instead of periodic x (D2Q9)
        self.open_x = None if open_x is None else np.array(open_x, dtype=np.float64)
        self.model = int(model)  # PTRT, TRT, PTRT_EXACT or PTRT_GHOST
        self.forcing = int(forcing)  # FORCING_II, FORCING_II_G or FORCING_GUO
        self.Q = _Q[lat]
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.tau_plus = float(tau_plus)
        self.Lambda = float(Lambda) if Lambda is not None else 0.0
        self.tau_minus = -1.0 if tau_minus is None else float(tau_minus)
        self.g = _g3(g)
        self.solid = None if solid is None else np.ascontiguousarray(
            np.asarray(solid, dtype=np.uint8).reshape(nz, ny, nx))
        self.nthreads = int(nthreads)
        self.f = np.zeros((self.N, self.Q))
        self.t = 0

    # ---- state in the ABI layout -------------------------------------
    def set_populations(self, f_qzyx):
        f_qzyx = np.asarray(f_qzyx, dtype=np.float64).reshape((self.Q,) + self.shape)
        self.f = np.ascontiguousarray(f_qzyx.reshape(self.Q, self.N).T)
        self._apply_outlet()

    def _apply_outlet(self):
        """With open x the outlet condition also holds for a state set from
        outside (its entering populations are computed, not stored)."""
        if self.open_x is None:
            return
        nz, ny, nx = self.shape
        solid = _p(self.solid, _u8p) if self.solid is not None else None
        assert _load().ptrt_oracle_apply_outlet(self.lat, nx, ny, nz, solid, _p(self.f),
                                                float(self.open_x[1])) == 0

    def populations(self):
        return np.ascontiguousarray(self.f.T).reshape((self.Q,) + self.shape)

    def init_equilibrium(self, rho=None, u=None):
        nz, ny, nx = self.shape
        rho = np.ones(self.shape) if rho is None else np.asarray(rho, dtype=np.float64).reshape(self.shape)
        u3 = np.zeros((3,) + self.shape)
        if u is not None:
            u = np.asarray(u, dtype=np.float64)
            u3[: u.shape[0]] = u.reshape((u.shape[0],) + self.shape)
        feq = equilibrium(self.lat, rho.ravel(), u3.reshape(3, -1).T)
        self.f = np.ascontiguousarray(feq)
        self._apply_outlet()
        self.t = 0

    # ---- dynamics ------------------------------------------------------
    def step(self, n=1):
        nz, ny, nx = self.shape
        solid = _p(self.solid, _u8p) if self.solid is not None else None
        args = (self.lat, self.model, self.forcing, nx, ny, nz, self.tau_plus, self.Lambda,
                self.tau_minus, _p(self.g), solid, _p(self.f), int(n), self.nthreads)
        if self.open_x is None:
            rc = _load().ptrt_oracle_run_ex(*args)
        else:
            rc = _load().ptrt_oracle_run_open(*args, _p(self.open_x))
        if rc != 0:
            raise RuntimeError(f"oracle run failed ({rc})")
        self.t += n

    def momentum_exchange(self):
        """Force on the solid nodes at the current time (Eq. Fx), [3]."""
        nz, ny, nx = self.shape
        F = np.zeros(3)
        solid = _p(self.solid, _u8p) if self.solid is not None else None
        rc = _load().ptrt_oracle_momentum_exchange(
            self.lat, self.model, self.forcing, nx, ny, nz, self.tau_plus, self.Lambda,
            self.tau_minus, _p(self.g), solid, _p(self.f),
            _p(self.open_x) if self.open_x is not None else None, _p(F))
        if rc != 0:
            raise RuntimeError(f"oracle momentum exchange failed ({rc})")
        return F

    def phi_gradient(self):
        """d_a (rho u_a^3) of the current state at every node, [N,3]."""
        nz, ny, nx = self.shape
        out = np.zeros((self.N, 3))
        solid = _p(self.solid, _u8p) if self.solid is not None else None
        _load().ptrt_oracle_phi_gradient(self.lat, nx, ny, nz, _p(self.g), solid, _p(self.f),
                                         _p(out))
        return out

    def step_sampled(self, nodes):
        """f(t+1) at the given flat node indices, [len(nodes), Q]; state unchanged."""
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64))
        out = np.zeros((nodes.size, self.Q))
        nz, ny, nx = self.shape
        solid = _p(self.solid, _u8p) if self.solid is not None else None
        _load().ptrt_oracle_step_sampled(self.lat, nx, ny, nz, self.tau_plus, self.Lambda,
                                         _p(self.g), solid, _p(self.f), int(nodes.size),
                                         _p(nodes, _llp), _p(out))
        return out

    # ---- observables ---------------------------------------------------
    def moments(self):
        """rho [nz,ny,nx], u [3,nz,ny,nx]; solid nodes report 0."""
        rho, u3 = node_moments(self.lat, self.f, self.g)
        if self.solid is not None:
            s = self.solid.ravel().astype(bool)
            rho[s] = 0.0
            u3[s] = 0.0
        return rho.reshape(self.shape), np.ascontiguousarray(u3.T).reshape((3,) + self.shape)

    def diagnostics(self):
        """(mass, kinetic energy) over fluid nodes."""
        m = ctypes.c_double()
        k = ctypes.c_double()
        solid = _p(self.solid, _u8p) if self.solid is not None else None
        _load().ptrt_oracle_diagnostics(self.lat, self.N, _p(self.f), _p(self.g), solid,
                                        ctypes.byref(m), ctypes.byref(k))
        return m.value, k.value


def steps_from_fields_sampled(lat, rho, u, tau_plus, Lambda, g, nodes, nsteps):
    """Pre-collision populations after `nsteps` steps at the flat node
    indices `nodes` of a periodic lattice without solid nodes that starts
    from f(0) = f^eq(rho, u) (equilibrium initialisation), [len(nodes), Q].

    rho [nz, ny, nx], u [D or 3, nz, ny, nx].  Each step is Eq. PTRT,
    collide then stream: f_i(x, s) = f*_i(x - e_i, s - 1), so f(x, nsteps)
    depends only on f(0) within nsteps nodes of x.  The equilibrium is
    formed on that neighbourhood (Eq. feq) and collided level by level with
    the oracle's collision, the neighbourhood shrinking by one node per
    step; no whole-lattice state is formed, so this reaches lattices of any
    size at a few thousand nodes.
    """
    e, _, _ = lattice(lat)
    Q = e.shape[0]
    rho = np.asarray(rho, dtype=np.float64)
    nz, ny, nx = rho.shape
    u = np.asarray(u, dtype=np.float64)
    D = 2 if lat == D2Q9 else 3
    nodes = np.asarray(nodes, dtype=np.int64).ravel()
    z, rem = np.divmod(nodes, nx * ny)
    y, x = np.divmod(rem, nx)

    def cube(r):
        """Offsets (dz, dy, dx) within r nodes, as an [m, 3] array, and the
        index of an offset in it."""
        rz = r if D == 3 else 0
        s = 2 * r + 1
        dz, dy, dx = np.meshgrid(np.arange(-rz, rz + 1), np.arange(-r, r + 1),
                                 np.arange(-r, r + 1), indexing="ij")
        off = np.stack([dz.ravel(), dy.ravel(), dx.ravel()], axis=1)

        def index(o):
            return ((o[..., 0] + rz) * s + (o[..., 1] + r)) * s + (o[..., 2] + r)
        return off, index

    # f(0) on the neighbourhood of radius nsteps
    off, _ = cube(nsteps)
    gz = (z[:, None] + off[None, :, 0]) % nz
    gy = (y[:, None] + off[None, :, 1]) % ny
    gx = (x[:, None] + off[None, :, 2]) % nx
    u3 = np.zeros((3,) + gz.shape)
    for a in range(min(D, u.shape[0])):
        u3[a] = u[a][gz, gy, gx]
    f = equilibrium(lat, rho[gz, gy, gx].ravel(),
                    np.moveaxis(u3, 0, -1).reshape(-1, 3)).reshape(gz.shape + (Q,))
    g3 = _g3(g)
    for level in range(1, nsteps + 1):
        r = nsteps - level
        post = collide(lat, f.reshape(-1, Q), g3, tau_plus, Lambda=Lambda).reshape(f.shape)
        _, index_prev = cube(r + 1)
        off_r, _ = cube(r)
        nxt = np.empty((len(nodes), off_r.shape[0], Q))
        for i in range(Q):
            src = off_r - np.array([e[i, 2], e[i, 1], e[i, 0]])[None, :]
            nxt[:, :, i] = post[:, index_prev(src), i]
        f = nxt
    return f[:, 0, :]
