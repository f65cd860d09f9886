"""TEST INFRASTRUCTURE: ctypes wrapper of the plain FP64 CPU oracle (hydro_oracle.c).

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this package.  It never touches the HIP library and shares no code with
it; the two are compared only through their outputs on the same seeded inputs.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

FIELDS = {"eps": 0, "ux": 1, "uy": 2, "ue": 3}
FIELDS.update({f"pi{m}": 4 + m for m in range(10)})
FIELDS.update({f"T{m}": 14 + m for m in range(4)})
FIELDS.update({"uprev_x": 18, "uprev_y": 19, "uprev_e": 20})
FIELDS.update({"Pi": 21, "nb": 22})  # bulk pressure, net-baryon density


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("ne", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("de", C.c_double),
                ("tau0", C.c_double), ("h", C.c_double), ("etas", C.c_double),
                ("viscous", C.c_int), ("cartesian", C.c_int),
                ("eps_cut", C.c_double), ("theta", C.c_double), ("newton_tol", C.c_double),
                ("newton_maxit", C.c_int), ("pi_reg", C.c_double),
                ("taupi_coef", C.c_double), ("lambda1_hat", C.c_double),
                ("zetas", C.c_double), ("taubulk_coef", C.c_double), ("baryon", C.c_int),
                ("cfl_limit", C.c_double)]


class _Diag(C.Structure):
    _fields_ = [("tau", C.c_double), ("step", C.c_long), ("eps_max", C.c_double),
                ("sum_Ttt", C.c_double), ("geo_src", C.c_double), ("max_cfl", C.c_double),
                ("newton_mean", C.c_double), ("newton_max", C.c_long), ("solves", C.c_long),
                ("fallbacks", C.c_long), ("nonconv", C.c_long), ("nans", C.c_long),
                ("vacuum", C.c_long), ("clamps", C.c_long), ("negative", C.c_long),
                ("errors", C.c_int)]


MUT_LIB_PATH = os.path.join(_HERE, "liboracle_mut.so")

_lib = None
_plain = None    # liboracle.so
_mutant = None   # liboracle_mut.so, loaded by set_mutant() only


def load():
    global _lib, _plain
    if _lib is not None:
        return _lib
    _plain = _open(LIB_PATH)
    _lib = _plain
    return _lib


def _open(path):
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = C.CDLL(path)
    P = C.POINTER(C.c_double)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [C.POINTER(_Params)]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_set_eos_conformal.argtypes = [C.c_void_p, C.c_double]
    lib.orc_set_eos_table.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, P, P, P]
    lib.orc_set_initial_primitive.argtypes = [C.c_void_p, P, P, P, P, P]
    lib.orc_set_initial_primitive_ext.argtypes = [C.c_void_p, P, P, P, P, P, P, P]
    lib.orc_set_initial_conserved.argtypes = [C.c_void_p, P, P]
    lib.orc_step.argtypes = [C.c_void_p, C.c_int]
    lib.orc_read.argtypes = [C.c_void_p, C.c_int, P]
    lib.orc_diag_get.argtypes = [C.c_void_p, C.POINTER(_Diag)]
    lib.orc_eos_eval.argtypes = [C.c_void_p, C.c_int, P, P, P, P, P]
    lib.orc_con2prim.argtypes = [C.c_void_p, C.c_int, P, P, P, P, C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)]
    lib.orc_con2prim_bulk.argtypes = [C.c_void_p, C.c_int, P, P, P, P, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
    lib.orc_prim2K.argtypes = [C.c_void_p, C.c_int, P, P, P]
    lib.orc_local_speed.argtypes = [C.c_int, P, C.c_int, P, P]
    lib.orc_regulate.argtypes = [C.c_void_p, C.c_double, P]
    lib.orc_shear_at.argtypes = [C.c_void_p, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int, P]
    lib.orc_mlp_nparam.restype = C.c_int
    lib.orc_mlp_forward.argtypes = [P, C.c_int, P, P, P]
    lib.orc_mlp_loss_grad.argtypes = [P, C.c_int, P, P, P, P, P]
    lib.orc_mlp_adam.argtypes = [P, P, P, P, C.c_int, C.c_double, C.c_double, C.c_double,
                                 C.c_double]
    lib.orc_surface.restype = C.c_long
    lib.orc_surface.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                P, C.c_double, P, C.c_double, C.c_int, C.c_double, C.c_int, P,
                                C.c_long]
    lib.orc_spectra.argtypes = [P, C.c_long, C.c_double, C.c_double, C.c_int, P, P,
                                C.POINTER(C.c_int), P, C.c_int, P, C.c_int, P, C.c_int, P, P]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_max_threads.restype = C.c_int
    return lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int):
    load().orc_set_threads(int(n))


def set_mutant(k: int):
    """Plant mistake k (0: none).  Used only by the pins' self-check: a nonzero k
    switches this module to the separate mutant build liboracle_mut.so, k = 0
    switches back to liboracle.so (which has no switches).  Oracle objects keep
    the library that was current when they were created."""
    global _lib, _mutant
    load()
    if k:
        if _mutant is None:
            _mutant = _open(MUT_LIB_PATH)
            _mutant.orc_set_mutant.argtypes = [C.c_int]
        _mutant.orc_set_mutant(int(k))
        _lib = _mutant
    else:
        if _mutant is not None:
            _mutant.orc_set_mutant(0)
        _lib = _plain


def max_threads() -> int:
    return int(load().orc_max_threads())


@dataclass
class Params:
    nx: int
    ny: int
    ne: int
    dx: float
    dy: float
    de: float
    tau0: float
    h: float
    etas: float = 0.0
    viscous: bool = False
    cartesian: bool = False
    eps_cut: float = 1e-7
    theta: float = 1.8
    newton_tol: float = 1e-12
    newton_maxit: int = 100
    pi_reg: float = 0.3
    taupi_coef: float = 5.0
    lambda1_hat: float = 0.0
    zetas: float = 0.0         # zeta/s of the bulk pressure (0: no bulk)
    taubulk_coef: float = 5.0  # tau_Pi = taubulk_coef (zeta/s) hbarc / T
    baryon: bool = False       # transport the net-baryon density
    cfl_limit: float = 0.5     # c h / Delta above which the CFL error bit is raised

    def c(self):
        return _Params(self.nx, self.ny, self.ne, self.dx, self.dy, self.de, self.tau0, self.h,
                       self.etas, int(self.viscous), int(self.cartesian), self.eps_cut,
                       self.theta, self.newton_tol, self.newton_maxit, self.pi_reg,
                       self.taupi_coef, self.lambda1_hat, self.zetas, self.taubulk_coef,
                       int(self.baryon), self.cfl_limit)


class Oracle:
    """One grid evolved by the CPU oracle."""

    def __init__(self, params: Params, eos=None):
        self.lib = load()
        self.params = params
        self._cp = params.c()
        self.h = self.lib.orc_create(C.byref(self._cp))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.shape = (params.nx, params.ny, params.ne)
        self.ncell = params.nx * params.ny * params.ne
        if eos is not None:
            self.set_eos(eos)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def set_eos(self, eos):
        """eos: None/'conformal' for P = e/3, or an EosTable."""
        if eos is None or (isinstance(eos, str) and eos == "conformal"):
            from hydro_inputs.eos import C_SB
            assert self.lib.orc_set_eos_conformal(self.h, C_SB) == 0
            return
        self._eos = (_c(eos.P), _c(eos.T), _c(eos.cs2))
        rc = self.lib.orc_set_eos_table(self.h, eos.eps0, eos.deps, eos.n, *[_p(a) for a in self._eos])
        assert rc == 0

    def set_initial(self, ic: dict):
        e, ux, uy, ue = (_c(ic[k]).reshape(-1) for k in ("eps", "ux", "uy", "ue"))
        pi = ic.get("pi")
        pi = None if pi is None else _c(pi).reshape(10, -1)
        Pi, nb = (None if ic.get(k) is None else _c(ic[k]).reshape(-1) for k in ("Pi", "nb"))
        rc = self.lib.orc_set_initial_primitive_ext(self.h, _p(e), _p(ux), _p(uy), _p(ue), _p(pi),
                                                    _p(Pi), _p(nb))
        assert rc == 0

    def set_initial_conserved(self, T4, pi=None):
        T4 = _c(T4).reshape(4, -1)
        pi = None if pi is None else _c(pi).reshape(10, -1)
        assert self.lib.orc_set_initial_conserved(self.h, _p(T4), _p(pi)) == 0

    def step(self, n: int = 1):
        assert self.lib.orc_step(self.h, int(n)) == 0

    def read(self, name):
        out = np.empty(self.shape, dtype=np.float64)
        fid = FIELDS[name] if isinstance(name, str) else int(name)
        assert self.lib.orc_read(self.h, fid, _p(out)) == 0
        return out

    def fields(self):
        return {k: self.read(k) for k in FIELDS}

    def diag(self) -> dict:
        d = _Diag()
        self.lib.orc_diag_get(self.h, C.byref(d))
        return {k: getattr(d, k) for k, _ in _Diag._fields_}

    # ---- point functions ----
    def eos_eval(self, e):
        e = _c(e).reshape(-1)
        outs = [np.empty_like(e) for _ in range(4)]
        self.lib.orc_eos_eval(self.h, e.size, _p(e), *[_p(o) for o in outs])
        return tuple(outs)  # P, T, cs2, dP/de

    def con2prim(self, K, guess=None):
        K = _c(K).reshape(-1, 4)
        n = K.shape[0]
        e = np.empty(n)
        u = np.empty((n, 3))
        it = np.empty(n, dtype=np.int32)
        fl = np.empty(n, dtype=np.int32)
        g = None if guess is None else _c(guess).reshape(-1)
        self.lib.orc_con2prim(self.h, n, _p(K), _p(g), _p(e), _p(u),
                              it.ctypes.data_as(C.POINTER(C.c_int)),
                              fl.ctypes.data_as(C.POINTER(C.c_int)))
        return e, u, it, fl

    def con2prim_bulk(self, K, Pi):
        """Root solve of K = (e+P+Pi) u~^tau u~ - (P+Pi) g~^{tau .} for (e, u~)."""
        K = _c(K).reshape(-1, 4)
        Pi = _c(Pi).reshape(-1)
        n = K.shape[0]
        e = np.empty(n)
        u = np.empty((n, 3))
        it = np.empty(n, dtype=np.int32)
        fl = np.empty(n, dtype=np.int32)
        self.lib.orc_con2prim_bulk(self.h, n, _p(K), _p(Pi), _p(e), _p(u),
                                   it.ctypes.data_as(C.POINTER(C.c_int)),
                                   fl.ctypes.data_as(C.POINTER(C.c_int)))
        return e, u, it, fl

    def shear_at(self, uE, uL, u, tau, i, j, k):
        """(sigma~[10], theta, a~[4]) at cell (i, j, k); u* arrays have shape (3, nx, ny, ne)."""
        arrs = [_c(a).reshape(3, -1) for a in (uE, uL, u)]
        out = np.empty(15)
        self.lib.orc_shear_at(self.h, *[_p(a) for a in arrs], float(tau), i, j, k, _p(out))
        return out[:10], out[10], out[11:]

    def regulate(self, e, q):
        """The shear regulator on one cell: q holds the transported components
        (10 pi~, plus Pi and n with bulk/baryon); returns the regulated copy."""
        q = _c(q).copy()
        self.lib.orc_regulate(self.h, float(e), _p(q))
        return q

    def prim2K(self, e, u):
        e = _c(e).reshape(-1)
        u = _c(u).reshape(-1, 3)
        K = np.empty((e.size, 4))
        self.lib.orc_prim2K(self.h, e.size, _p(e), _p(u), _p(K))
        return K


def local_speed(u3, axis, cs2):
    u3 = _c(u3).reshape(-1, 3)
    cs2 = _c(cs2).reshape(-1)
    out = np.empty(u3.shape[0])
    load().orc_local_speed(u3.shape[0], _p(u3), int(axis), _p(cs2), _p(out))
    return out


C2P_FALLBACK, C2P_NONCONV, C2P_NAN, C2P_VAC, C2P_CLAMP, C2P_NEG = 1, 2, 4, 8, 16, 32
ERR_NAN, ERR_NEG_EPS, ERR_NONCONV, ERR_CFL = 1, 2, 4, 8


# ---- learned root-solve guess (FP64 reference) ----
def mlp_nparam() -> int:
    return int(load().orc_mlp_nparam())


def mlp_forward(params, E, M):
    p, E, M = _c(params), _c(E).reshape(-1), _c(M).reshape(-1)
    out = np.empty(E.size)
    load().orc_mlp_forward(_p(p), E.size, _p(E), _p(M), _p(out))
    return out


def mlp_loss_grad(params, E, M, eps):
    p, E, M, e = _c(params), _c(E).reshape(-1), _c(M).reshape(-1), _c(eps).reshape(-1)
    loss = np.zeros(1)
    g = np.empty(p.size)
    load().orc_mlp_loss_grad(_p(p), E.size, _p(E), _p(M), _p(e), _p(loss), _p(g))
    return float(loss[0]), g


def mlp_adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, epsilon=1e-8):
    """In-place Adam step on float64 arrays params, m, v."""
    load().orc_mlp_adam(_p(params), _p(_c(grad)), _p(m), _p(v), int(t), lr, b1, b2, epsilon)


SURF_REC = 24


def surface(shape, spacing, A, tauA, B, tauB, eps_f, cartesian=False):
    """Freeze-out surface elements between slices A (tau_A) and B (tau_B) of shape
    (nf, nx, ny, ne), nf = 4 (e, u~x, u~y, u~eta) or 14 (+ pi~): an (n, 24) array in
    hypercube order (record layout in surface_oracle.c)."""
    lib = load()
    nx, ny, ne = shape
    A = _c(A)
    B = _c(B)
    nf = A.shape[0]
    assert A.shape == B.shape == (nf, nx, ny, ne)
    n = lib.orc_surface(nx, ny, ne, *spacing, _p(A), tauA, _p(B), tauB, nf, eps_f, int(cartesian),
                        None, 0)
    if n < 0:
        raise ValueError("orc_surface rejected its arguments")
    out = np.zeros((max(n, 1), SURF_REC))
    lib.orc_surface(nx, ny, ne, *spacing, _p(A), tauA, _p(B), tauB, nf, eps_f, int(cartesian),
                    _p(out), n)
    return out[:n]


def spectra(elements, T, eps_plus_P, species, Y, pt, phi):
    """Smooth Cooper-Frye spectra dN/(dY pT dpT dphi) (GeV^-2) of the surface elements
    (n, 24) for species = (mass, dof, stat, mu) arrays: shape (ns, nY, npt, nphi).
    eps_plus_P = 0 leaves out delta f (formulas in spectra_oracle.c)."""
    lib = load()
    el = _c(np.asarray(elements).reshape(-1, SURF_REC))
    mass, dof, stat, mu = species
    mass, dof, mu = _c(mass), _c(dof), _c(mu)
    stat = np.ascontiguousarray(stat, dtype=np.int32)
    Y, pt, phi = _c(Y), _c(pt), _c(phi)
    ns = mass.size
    out = np.zeros((ns, Y.size, pt.size, phi.size))
    rc = lib.orc_spectra(_p(el), el.shape[0], T, eps_plus_P, ns, _p(mass), _p(dof),
                         stat.ctypes.data_as(C.POINTER(C.c_int)), _p(mu), Y.size, _p(Y), pt.size,
                         _p(pt), phi.size, _p(phi), _p(out))
    if rc != 0:
        raise ValueError("orc_spectra rejected its arguments")
    return out
