"""Python binding of libktmi (include/ktmi.h): one RK2 step of the Kurganov-Tadmor
scheme for (3+1)D viscous hydrodynamics in Milne coordinates on MI355X.

The functions ktmi_* mirror the C ABI one to one and only marshal arguments.
PyTorch supplies device memory (the workspace and field tensors) and the HIP
stream.  Every step of the method runs in the HIP kernels of libktmi.so; there is
no CPU fallback: if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libktmi.so")

KTMI_OK, KTMI_EINVAL, KTMI_ESTATE, KTMI_EHIP = 0, -22, -5, -71
KTMI_FP64, KTMI_MIXED = 0, 1
KTMI_GUESS_PREV, KTMI_GUESS_COLD, KTMI_GUESS_MLP = 0, 1, 2
KTMI_MLP_FP32, KTMI_MLP_BF16 = 0, 1
KTMI_F_EPS, KTMI_F_UX, KTMI_F_PI, KTMI_F_T, KTMI_F_UPREV = 0, 1, 4, 14, 18

FIELDS = {"eps": 0, "ux": 1, "uy": 2, "ue": 3}
FIELDS.update({f"pi{m}": 4 + m for m in range(10)})
FIELDS.update({f"T{m}": 14 + m for m in range(4)})
FIELDS.update({"uprev_x": 18, "uprev_y": 19, "uprev_e": 20})
FIELDS.update({"Pi": 21, "nb": 22})  # bulk pressure, net-baryon density


class ktmi_desc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("ne", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("de", C.c_double),
                ("tau0", C.c_double), ("h", C.c_double), ("etas", C.c_double),
                ("viscous", C.c_int), ("cartesian", C.c_int),
                ("eps_cut", C.c_double), ("theta", C.c_double), ("newton_tol", C.c_double),
                ("newton_maxit", C.c_int), ("pi_reg", C.c_double), ("precision", C.c_int),
                ("guess", C.c_int), ("tile", C.c_int), ("taupi_coef", C.c_double),
                ("lambda1_hat", C.c_double), ("zetas", C.c_double),
                ("taubulk_coef", C.c_double), ("baryon", C.c_int), ("cfl_limit", C.c_double)]


class ktmi_diagnostics(C.Structure):
    _fields_ = [("tau", C.c_double), ("step", C.c_long), ("eps_max", C.c_double),
                ("sum_Ttt", C.c_double), ("geo_src", C.c_double), ("max_cfl", C.c_double),
                ("newton_mean", C.c_double), ("newton_max", C.c_long), ("solves", C.c_long),
                ("fallbacks", C.c_long), ("nonconv", C.c_long), ("nans", C.c_long),
                ("vacuum", C.c_long), ("clamps", C.c_long), ("negative", C.c_long),
                ("errors", C.c_int)]


def _load():
    # torch first: libktmi.so then binds to the HIP runtime torch already loaded, so
    # device memory from torch and the library's launches share one runtime
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -c "
                          "'import __graft_entry__ as g; g.build()' (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    vp, dp, sz, f = C.c_void_p, C.POINTER(C.c_double), C.c_size_t, C.c_float
    sig = {
        "ktmi_desc_default": (None, [C.POINTER(ktmi_desc)]),
        "ktmi_create": (C.c_int, [C.POINTER(ktmi_desc), C.POINTER(vp)]),
        "ktmi_workspace_bytes": (sz, [C.POINTER(ktmi_desc)]),
        "ktmi_bind": (C.c_int, [vp, vp, sz, vp]),
        "ktmi_set_eos_conformal": (C.c_int, [vp, C.c_double]),
        "ktmi_set_eos_table": (C.c_int, [vp, C.c_double, C.c_double, C.c_int, dp, dp, dp]),
        "ktmi_set_initial_primitive": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "ktmi_set_initial_primitive_ext": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "ktmi_set_initial_conserved": (C.c_int, [vp, vp, vp]),
        "ktmi_step": (C.c_int, [vp, C.c_int]),
        "ktmi_read": (C.c_int, [vp, C.c_int, vp]),
        "ktmi_diag": (C.c_int, [vp, C.POINTER(ktmi_diagnostics)]),
        "ktmi_set_timing": (C.c_int, [vp, C.c_int]),
        "ktmi_kernel_count": (C.c_int, []),
        "ktmi_kernel_name": (C.c_char_p, [C.c_int]),
        "ktmi_timing": (C.c_int, [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_long)]),
        "ktmi_tile_count": (C.c_int, []),
        "ktmi_tile_shape": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]),
        "ktmi_set_tile": (C.c_int, [vp, C.c_int]),
        "ktmi_get_tile": (C.c_int, [vp]),
        "ktmi_set_graph": (C.c_int, [vp, C.c_int]),
        "ktmi_group_workspace_bytes": (sz, [C.c_int]),
        "ktmi_group_create": (C.c_int, [C.POINTER(vp), C.c_int, vp, sz, C.POINTER(vp)]),
        "ktmi_group_step": (C.c_int, [vp, C.c_int]),
        "ktmi_group_set_graph": (C.c_int, [vp, C.c_int]),
        "ktmi_group_class_count": (C.c_int, [vp]),
        "ktmi_group_last_error": (C.c_char_p, [vp]),
        "ktmi_group_destroy": (None, [vp]),
        "ktmi_mlp_nparam": (C.c_int, []),
        "ktmi_set_mlp": (C.c_int, [vp, vp, C.c_int]),
        "ktmi_set_guess": (C.c_int, [vp, C.c_int]),
        "ktmi_set_quiet_skip": (C.c_int, [vp, C.c_int]),
        "ktmi_quiet_tiles": (C.c_int, [vp, C.POINTER(C.c_long), C.POINTER(C.c_long)]),
        "ktmi_harvest": (C.c_int, [vp, vp, vp, vp]),
        "ktmi_mlp_forward": (C.c_int, [vp, C.c_int, vp, vp, C.c_double, vp, C.c_int, vp]),
        "ktmi_mlp_grad_workspace_bytes": (sz, [C.c_int]),
        "ktmi_mlp_grad": (C.c_int, [vp, C.c_int, vp, vp, vp, C.c_double, C.c_int, vp, vp, sz,
                                    vp]),
        "ktmi_mlp_grad_noalloc": (C.c_int, [vp, C.c_int, vp, vp, vp, C.c_double, C.c_int, vp,
                                            vp]),
        "ktmi_mlp_adam": (C.c_int, [vp, vp, vp, vp, C.c_int, f, f, f, f, vp]),
        "ktmi_step_until": (C.c_int, [vp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int)]),
        "ktmi_snapshot_doubles": (sz, [vp, C.c_int]),
        "ktmi_snapshot": (C.c_int, [vp, vp, C.c_int]),
        "ktmi_surface": (C.c_int, [vp, vp, C.c_double, vp, C.c_double, C.c_int, C.c_double, vp,
                                   C.c_long, vp]),
        "ktmi_spectra_workspace_bytes": (sz, [C.c_long, C.c_int, C.c_int, C.c_int, C.c_int]),
        "ktmi_spectra": (C.c_int, [vp, C.c_long, C.c_double, C.c_double, C.c_int, dp, dp,
                                   C.POINTER(C.c_int), dp, C.c_int, dp, C.c_int, dp, C.c_int, dp,
                                   vp, vp, sz, vp]),
        "ktmi_last_error": (C.c_char_p, [vp]),
        "ktmi_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class KtmiError(RuntimeError):
    pass


def _check(rc, h=None):
    if rc != KTMI_OK:
        msg = lib.ktmi_last_error(h)
        raise KtmiError(f"ktmi error {rc}: {msg.decode() if msg else ''}")


# ---- one-to-one wrappers of the C ABI ------------------------------------
def ktmi_desc_default() -> ktmi_desc:
    d = ktmi_desc()
    lib.ktmi_desc_default(C.byref(d))
    return d


def ktmi_create(desc: ktmi_desc):
    h = C.c_void_p()
    _check(lib.ktmi_create(C.byref(desc), C.byref(h)))
    return h


def ktmi_workspace_bytes(desc: ktmi_desc) -> int:
    return int(lib.ktmi_workspace_bytes(C.byref(desc)))


def ktmi_bind(h, dev_ptr: int, nbytes: int, stream_ptr: int):
    _check(lib.ktmi_bind(h, C.c_void_p(dev_ptr), nbytes, C.c_void_p(stream_ptr)), h)


def ktmi_set_eos_conformal(h, c_sb: float):
    _check(lib.ktmi_set_eos_conformal(h, float(c_sb)), h)


def ktmi_set_eos_table(h, e0, de, P, T, cs2):
    """P, T, cs2: contiguous float64 host numpy arrays of equal length."""
    import numpy as np
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (P, T, cs2)]
    ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs]
    _check(lib.ktmi_set_eos_table(h, float(e0), float(de), int(arrs[0].size), *ptrs), h)


def ktmi_set_initial_primitive(h, e_ptr, ux_ptr, uy_ptr, ue_ptr, pi_ptr=None):
    _check(lib.ktmi_set_initial_primitive(h, C.c_void_p(e_ptr), C.c_void_p(ux_ptr),
                                          C.c_void_p(uy_ptr), C.c_void_p(ue_ptr),
                                          C.c_void_p(pi_ptr) if pi_ptr else None), h)


def ktmi_set_initial_primitive_ext(h, e_ptr, ux_ptr, uy_ptr, ue_ptr, pi_ptr=None, Pi_ptr=None,
                                   n_ptr=None):
    def vp(x):
        return C.c_void_p(x) if x else None
    _check(lib.ktmi_set_initial_primitive_ext(h, vp(e_ptr), vp(ux_ptr), vp(uy_ptr), vp(ue_ptr),
                                              vp(pi_ptr), vp(Pi_ptr), vp(n_ptr)), h)


def ktmi_set_initial_conserved(h, T_ptr, pi_ptr=None):
    _check(lib.ktmi_set_initial_conserved(h, C.c_void_p(T_ptr),
                                          C.c_void_p(pi_ptr) if pi_ptr else None), h)


def ktmi_step(h, n: int):
    _check(lib.ktmi_step(h, int(n)), h)


def ktmi_read(h, field: int, dst_ptr: int):
    _check(lib.ktmi_read(h, int(field), C.c_void_p(dst_ptr)), h)


def ktmi_diag(h) -> dict:
    d = ktmi_diagnostics()
    _check(lib.ktmi_diag(h, C.byref(d)), h)
    return {k: getattr(d, k) for k, _ in ktmi_diagnostics._fields_}


def ktmi_set_timing(h, on: bool):
    _check(lib.ktmi_set_timing(h, int(bool(on))), h)


def ktmi_kernel_names():
    return [lib.ktmi_kernel_name(k).decode() for k in range(lib.ktmi_kernel_count())]


def ktmi_timing(h, k: int):
    t = C.c_double()
    n = C.c_long()
    _check(lib.ktmi_timing(h, int(k), C.byref(t), C.byref(n)), h)
    return t.value, n.value


def ktmi_tile_count() -> int:
    return int(lib.ktmi_tile_count())


def ktmi_tile_shape(t: int):
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(lib.ktmi_tile_shape(int(t), C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def ktmi_set_tile(h, t: int):
    _check(lib.ktmi_set_tile(h, int(t)), h)


def ktmi_get_tile(h) -> int:
    return int(lib.ktmi_get_tile(h))


def ktmi_set_graph(h, on: bool):
    _check(lib.ktmi_set_graph(h, int(bool(on))), h)


def ktmi_group_workspace_bytes(nev: int) -> int:
    return int(lib.ktmi_group_workspace_bytes(int(nev)))


def _gcheck(rc, g):
    if rc != KTMI_OK:
        msg = lib.ktmi_group_last_error(g)
        raise KtmiError(f"ktmi group error {rc}: {msg.decode() if msg else ''}")


def ktmi_group_create(handles, dev_ptr: int, nbytes: int):
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    g = C.c_void_p()
    _check(lib.ktmi_group_create(arr, len(handles), C.c_void_p(dev_ptr), nbytes, C.byref(g)))
    return g


def ktmi_group_step(g, n: int):
    _gcheck(lib.ktmi_group_step(g, int(n)), g)


def ktmi_group_set_graph(g, on: bool):
    _gcheck(lib.ktmi_group_set_graph(g, int(bool(on))), g)


def ktmi_group_class_count(g) -> int:
    return int(lib.ktmi_group_class_count(g))


def ktmi_group_destroy(g):
    lib.ktmi_group_destroy(g)


def ktmi_mlp_nparam() -> int:
    return int(lib.ktmi_mlp_nparam())


def ktmi_set_mlp(h, params_ptr: int, mode: int):
    _check(lib.ktmi_set_mlp(h, C.c_void_p(params_ptr), int(mode)), h)


def ktmi_set_guess(h, guess: int):
    _check(lib.ktmi_set_guess(h, int(guess)), h)


def ktmi_set_quiet_skip(h, on: bool):
    _check(lib.ktmi_set_quiet_skip(h, int(bool(on))), h)


def ktmi_quiet_tiles(h):
    q, t = C.c_long(), C.c_long()
    _check(lib.ktmi_quiet_tiles(h, C.byref(q), C.byref(t)), h)
    return q.value, t.value


KTMI_SURF_REC = 24


def ktmi_step_until(h, eps_stop: float, max_steps: int, check_every: int = 1) -> int:
    taken = C.c_int()
    _check(lib.ktmi_step_until(h, float(eps_stop), int(max_steps), int(check_every),
                               C.byref(taken)), h)
    return taken.value


def ktmi_snapshot_doubles(h, with_pi: bool) -> int:
    return int(lib.ktmi_snapshot_doubles(h, int(bool(with_pi))))


def ktmi_snapshot(h, dst_ptr: int, with_pi: bool):
    _check(lib.ktmi_snapshot(h, C.c_void_p(dst_ptr), int(bool(with_pi))), h)


def ktmi_surface(h, A_ptr: int, tau_A: float, B_ptr: int, tau_B: float, with_pi: bool,
                 eps_f: float, out_ptr: int, capacity: int, count_ptr: int):
    _check(lib.ktmi_surface(h, C.c_void_p(A_ptr), float(tau_A), C.c_void_p(B_ptr), float(tau_B),
                            int(bool(with_pi)), float(eps_f), C.c_void_p(out_ptr), int(capacity),
                            C.c_void_p(count_ptr)), h)


def ktmi_spectra_workspace_bytes(n: int, ns: int, nY: int, npt: int, nphi: int) -> int:
    return int(lib.ktmi_spectra_workspace_bytes(int(n), int(ns), int(nY), int(npt), int(nphi)))


def ktmi_spectra(el_ptr: int, n: int, T: float, eps_plus_P: float, mass, dof, stat, mu, Y, pt, phi,
                 out_ptr: int, ws_ptr: int, ws_bytes: int, stream_ptr: int):
    """Pointer-level call: device records, output and workspace; host numpy arrays for
    the species (mass, dof, stat as int32, mu) and the bins (Y, pt, phi)."""
    import numpy as np
    mass, dof, mu, Y, pt, phi = (np.ascontiguousarray(x, dtype=np.float64)
                                 for x in (mass, dof, mu, Y, pt, phi))
    stat = np.ascontiguousarray(stat, dtype=np.int32)
    P = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    rc = lib.ktmi_spectra(C.c_void_p(el_ptr), int(n), float(T), float(eps_plus_P), mass.size,
                          P(mass), P(dof), stat.ctypes.data_as(C.POINTER(C.c_int)), P(mu), Y.size,
                          P(Y), pt.size, P(pt), phi.size, P(phi), C.c_void_p(out_ptr),
                          C.c_void_p(ws_ptr), int(ws_bytes), C.c_void_p(stream_ptr))
    if rc != 0:
        raise KtmiError(f"ktmi_spectra failed ({rc})")


def spectra(elements, T, eps_plus_P, species, Y, pt, phi, stream=None):
    """Smooth Cooper-Frye spectra of device surface records (torch tensor (n, 24)):
    a device tensor (ns, nY, npt, nphi) of dN/(dY pT dpT dphi) in GeV^-2.
    species = (mass, dof, stat, mu) sequences; Y, pt, phi sequences (host)."""
    import numpy as np
    import torch
    mass, dof, stat, mu = species
    ns, nY, npt, nphi = len(mass), len(Y), len(pt), len(phi)
    el = elements.contiguous()
    n = int(el.shape[0])
    dev = el.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    nb = ktmi_spectra_workspace_bytes(n, ns, nY, npt, nphi)
    ws = torch.empty(nb // 8 + 1, dtype=torch.float64, device=dev)
    out = torch.empty((ns, nY, npt, nphi), dtype=torch.float64, device=dev)
    ktmi_spectra(el.data_ptr() if n else 0, n, T, eps_plus_P, mass, dof, stat, mu, Y, pt, phi,
                 out.data_ptr(), ws.data_ptr(), nb, st.cuda_stream)
    return out


def ktmi_harvest(h, E_ptr: int, M_ptr: int, eps_ptr: int):
    _check(lib.ktmi_harvest(h, C.c_void_p(E_ptr), C.c_void_p(M_ptr), C.c_void_p(eps_ptr)), h)


def ktmi_mlp_forward(params_ptr, n, E_ptr, M_ptr, emin, guess_ptr, mode, stream_ptr):
    _check(lib.ktmi_mlp_forward(C.c_void_p(params_ptr), int(n), C.c_void_p(E_ptr),
                                C.c_void_p(M_ptr), float(emin), C.c_void_p(guess_ptr), int(mode),
                                C.c_void_p(stream_ptr)))


def ktmi_mlp_grad_workspace_bytes(n: int) -> int:
    return int(lib.ktmi_mlp_grad_workspace_bytes(int(n)))


def ktmi_mlp_grad(params_ptr, n, E_ptr, M_ptr, eps_ptr, emin, mode, out_ptr, ws_ptr, ws_bytes,
                  stream_ptr):
    _check(lib.ktmi_mlp_grad(C.c_void_p(params_ptr), int(n), C.c_void_p(E_ptr),
                             C.c_void_p(M_ptr), C.c_void_p(eps_ptr), float(emin), int(mode),
                             C.c_void_p(out_ptr), C.c_void_p(ws_ptr), int(ws_bytes),
                             C.c_void_p(stream_ptr)))


def ktmi_mlp_grad_noalloc(params_ptr, n, E_ptr, M_ptr, eps_ptr, emin, mode, out_ptr, stream_ptr):
    _check(lib.ktmi_mlp_grad_noalloc(C.c_void_p(params_ptr), int(n), C.c_void_p(E_ptr),
                                     C.c_void_p(M_ptr), C.c_void_p(eps_ptr), float(emin),
                                     int(mode), C.c_void_p(out_ptr), C.c_void_p(stream_ptr)))


def ktmi_mlp_adam(params_ptr, grad_ptr, m_ptr, v_ptr, t, lr, b1, b2, epsilon, stream_ptr):
    _check(lib.ktmi_mlp_adam(C.c_void_p(params_ptr), C.c_void_p(grad_ptr), C.c_void_p(m_ptr),
                             C.c_void_p(v_ptr), int(t), float(lr), float(b1), float(b2),
                             float(epsilon), C.c_void_p(stream_ptr)))


def ktmi_destroy(h):
    lib.ktmi_destroy(h)


# ---- convenience object: torch-owned memory around one handle -------------
class Hydro:
    """One grid on the GPU.  Owns a torch workspace tensor and a handle."""

    def __init__(self, device="cuda", stream=None, **desc_kw):
        import torch
        self.torch = torch
        d = ktmi_desc_default()
        for k, v in desc_kw.items():
            if not hasattr(d, k):
                raise KeyError(k)
            setattr(d, k, v)
        self.desc = d
        self.shape = (d.nx, d.ny, d.ne)
        self.ncell = d.nx * d.ny * d.ne
        self.h = ktmi_create(d)
        nbytes = ktmi_workspace_bytes(d)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=self.device)
        ptr = self.ws.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        ktmi_bind(self.h, aligned, nbytes, self.stream.cuda_stream)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                self.torch.cuda.synchronize(self.device)
            except Exception:
                pass
            ktmi_destroy(h)
            self.h = None

    def set_eos(self, eos):
        if eos is None or (isinstance(eos, str) and eos == "conformal"):
            from hydro_inputs.eos import C_SB
            ktmi_set_eos_conformal(self.h, C_SB)
        else:
            ktmi_set_eos_table(self.h, eos.eps0, eos.deps, eos.P, eos.T, eos.cs2)

    def _dev(self, a):
        t = self.torch.as_tensor(a, dtype=self.torch.float64)
        return t.to(self.device).contiguous()

    def set_initial(self, ic: dict):
        with self.torch.cuda.stream(self.stream):
            keep = [self._dev(ic[k]).reshape(-1) for k in ("eps", "ux", "uy", "ue")]
            pi = ic.get("pi")
            pit = None if pi is None else self._dev(pi).reshape(10, -1)
            Pi, nb = ((None if ic.get(k) is None else self._dev(ic[k]).reshape(-1))
                      for k in ("Pi", "nb"))
            if Pi is None and nb is None:
                ktmi_set_initial_primitive(self.h, *[t.data_ptr() for t in keep],
                                           pit.data_ptr() if pit is not None else None)
            else:
                ktmi_set_initial_primitive_ext(
                    self.h, *[t.data_ptr() for t in keep],
                    pit.data_ptr() if pit is not None else None,
                    Pi.data_ptr() if Pi is not None else None,
                    nb.data_ptr() if nb is not None else None)
            self.stream.synchronize()

    def set_initial_conserved(self, T4, pi=None):
        with self.torch.cuda.stream(self.stream):
            Tt = self._dev(T4).reshape(4, -1)
            pit = None if pi is None else self._dev(pi).reshape(10, -1)
            ktmi_set_initial_conserved(self.h, Tt.data_ptr(),
                                       pit.data_ptr() if pit is not None else None)
            self.stream.synchronize()

    def step(self, n=1):
        ktmi_step(self.h, n)

    def read(self, name, out=None):
        """Field as a device tensor of shape (nx, ny, ne) (stream-ordered)."""
        if out is None:
            out = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        fid = FIELDS[name] if isinstance(name, str) else int(name)
        ktmi_read(self.h, fid, out.data_ptr())
        return out

    def read_numpy(self, name):
        t = self.read(name)
        self.stream.synchronize()
        return t.cpu().numpy()

    def fields(self):
        return {k: self.read_numpy(k) for k in FIELDS}

    def diag(self):
        return ktmi_diag(self.h)

    def set_graph(self, on=True):
        ktmi_set_graph(self.h, on)

    def set_mlp(self, params, mode=KTMI_MLP_FP32):
        """Network parameters (device float32 tensor of ktmi_mlp_nparam() values)."""
        ktmi_set_mlp(self.h, params.data_ptr(), mode)

    def set_guess(self, guess):
        ktmi_set_guess(self.h, guess)

    def set_quiet_skip(self, on=True):
        ktmi_set_quiet_skip(self.h, on)

    def step_until(self, eps_stop, max_steps, check_every=1):
        """Steps until the maximum energy density falls below eps_stop (checked
        every check_every steps) or max_steps are taken; returns the steps taken."""
        return ktmi_step_until(self.h, eps_stop, max_steps, check_every)

    def snapshot(self, with_pi=False):
        """The current (e, u~[, pi~]) slice as a device tensor (nf, nx, ny, ne)."""
        t = self.torch
        nf = 14 if with_pi else 4
        out = t.empty((nf,) + self.shape, dtype=t.float64, device=self.device)
        ktmi_snapshot(self.h, out.data_ptr(), with_pi)
        return out

    def surface(self, A, tau_A, B, tau_B, eps_f, capacity=None):
        """Freeze-out elements between slices A (tau_A) and B (tau_B): a device
        tensor (n, KTMI_SURF_REC) in hypercube order (grown once if the first
        buffer was too small)."""
        t = self.torch
        with_pi = A.shape[0] == 14
        assert A.shape == B.shape and A.is_contiguous() and B.is_contiguous()
        cap = capacity if capacity is not None else max(1024, self.ncell // 8)
        count = t.zeros(1, dtype=t.int64, device=self.device)
        for _ in range(2):
            out = t.empty((cap, KTMI_SURF_REC), dtype=t.float64, device=self.device)
            ktmi_surface(self.h, A.data_ptr(), tau_A, B.data_ptr(), tau_B, with_pi, eps_f,
                         out.data_ptr(), cap, count.data_ptr())
            self.stream.synchronize()
            n = int(count.item())
            if n <= cap:
                return out[:n]
            cap = n
        raise KtmiError("surface element count changed between calls")

    def harvest(self):
        """(E, M, eps) of every cell of the current state, device tensors."""
        t = self.torch
        out = [t.empty(self.ncell, dtype=t.float64, device=self.device) for _ in range(3)]
        ktmi_harvest(self.h, *[o.data_ptr() for o in out])
        return out


class Group:
    """Several Hydro objects stepped together (one launch per class and stage).
    All members must use the same (non-default, for graphs) torch stream."""

    def __init__(self, members):
        import torch
        self.torch = torch
        self.members = list(members)
        nb = ktmi_group_workspace_bytes(len(self.members))
        dev = self.members[0].device
        self.ws = torch.empty(nb // 8 + 32, dtype=torch.float64, device=dev)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.g = ktmi_group_create([m.h for m in self.members], ptr, nb)

    def __del__(self):
        g = getattr(self, "g", None)
        if g:
            try:
                self.torch.cuda.synchronize()
            except Exception:
                pass
            ktmi_group_destroy(g)
            self.g = None

    def step(self, n=1):
        ktmi_group_step(self.g, n)

    def set_graph(self, on=True):
        ktmi_group_set_graph(self.g, on)

    @property
    def classes(self):
        return ktmi_group_class_count(self.g)
