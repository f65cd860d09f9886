"""Helpers for the GPU parity tests: run one workload on the HIP library and on
the CPU oracle from the same seeded inputs and compare them field by field."""
from __future__ import annotations

import numpy as np

import oracle as O

GROUPS = {
    "eps": ["eps"],
    "u": ["ux", "uy", "ue"],
    "pi": [f"pi{m}" for m in range(10)],
    "T": [f"T{m}" for m in range(4)],
    "uprev": ["uprev_x", "uprev_y", "uprev_e"],
    "Pi": ["Pi"],
    "nb": ["nb"],
}


def oracle_params(p: dict, **kw) -> O.Params:
    q = dict(p)
    q.update(kw)
    return O.Params(q["nx"], q["ny"], q["ne"], q["dx"], q["dy"], q["de"], tau0=q["tau0"],
                    h=q["h"], etas=q["etas"], viscous=bool(q["viscous"]),
                    cartesian=bool(q["cartesian"]), **{k: q[k] for k in
                                                      ("eps_cut", "theta", "newton_tol",
                                                       "newton_maxit", "pi_reg", "taupi_coef",
                                                       "lambda1_hat", "zetas", "taubulk_coef",
                                                       "cfl_limit")
                                                      if k in q},
                    baryon=bool(q.get("baryon", 0)))


def run_oracle(wl, steps, threads=None, **kw):
    if threads:
        O.set_threads(threads)
    o = O.Oracle(oracle_params(wl.params, **kw), eos=wl.eos)
    if wl.T4 is not None:
        o.set_initial_conserved(wl.T4, wl.ic.get("pi") if wl.ic else None)
    else:
        o.set_initial(wl.ic)
    o.step(steps)
    return o


def run_gpu(wl, steps, **kw):
    import paper_1802_04449_amd as K
    desc = dict(wl.params)
    desc.update(kw)
    g = K.Hydro(**desc)
    g.set_eos(wl.eos)
    if wl.T4 is not None:
        g.set_initial_conserved(wl.T4, wl.ic.get("pi") if wl.ic else None)
    else:
        g.set_initial(wl.ic)
    g.step(steps)
    return g


def compare(gpu_fields: dict, ref_fields: dict) -> dict:
    """rel = max|gpu - ref| / scale per field; the scale is shared by a tensor's
    components (max |ref| over the group; u~ components use max u~^tau)."""
    out = {}
    ux, uy, ue = (ref_fields[k] for k in ("ux", "uy", "ue"))
    ut_max = float(np.sqrt(1 + ux ** 2 + uy ** 2 + ue ** 2).max())
    for gname, names in GROUPS.items():
        if gname in ("u", "uprev"):
            scale = ut_max
        else:
            scale = max(float(np.abs(ref_fields[n]).max()) for n in names)
        scale = scale if scale > 0 else 1.0
        for n in names:
            d = np.abs(gpu_fields[n] - ref_fields[n])
            out[n] = float(d.max()) / scale
    return out


def assert_parity(gpu_fields, ref_fields, tol, label=""):
    rel = compare(gpu_fields, ref_fields)
    worst = max(rel, key=rel.get)
    assert rel[worst] <= tol, f"{label}: worst field {worst} rel {rel[worst]:.3e} > {tol:.1e}; {rel}"
    return rel


def perturbed(wl, rel=1e-15, seed=0):
    """Copy of wl whose initial arrays carry relative noise of size rel."""
    import copy
    rng = np.random.default_rng(seed)
    w2 = copy.copy(wl)
    if wl.T4 is not None:
        w2.T4 = wl.T4 * (1.0 + rel * rng.standard_normal(wl.T4.shape))
    if wl.ic is not None:
        w2.ic = {k: v * (1.0 + rel * rng.standard_normal(np.shape(v))) for k, v in wl.ic.items()}
    return w2


def conditioning(wl, steps, rel=1e-15):
    """Per-field response of the oracle itself to a relative input perturbation of
    size rel: the scale below which no implementation can be asked to agree."""
    a = run_oracle(wl, steps).fields()
    b = run_oracle(perturbed(wl, rel), steps).fields()
    return a, compare(b, a)


def dense_compare(gpu_fields, ref_fields, eps_min):
    """compare() restricted to cells whose reference e is at least eps_min."""
    m = ref_fields["eps"] >= eps_min
    sub_g = {k: v[m] for k, v in gpu_fields.items()}
    sub_r = {k: v[m] for k, v in ref_fields.items()}
    return compare(sub_g, sub_r)


def precision_errors(gpu_fields, ref_fields, eps_min=0.1):
    """Per-field errors of a reduced-precision run against an FP64 reference.
    'max' = max|d| / scale over all cells, 'max_hydro' the same over cells with
    e >= eps_min (0.1 GeV/fm^3, the typical freeze-out energy density below which
    hydrodynamics is no longer applied), 'l2' = ||d||_2 / ||scale field||_2.  The
    scale is shared by a tensor's components, as in compare(): max|ref| over the
    group (max u~^tau for velocities) for 'max', and the L2 norm of the whole
    tensor (of u~^tau for velocities) for 'l2'."""
    out = {}
    ux, uy, ue = ref_fields["ux"], ref_fields["uy"], ref_fields["ue"]
    ut = np.sqrt(1 + ux ** 2 + uy ** 2 + ue ** 2)
    m = ref_fields["eps"] >= eps_min
    for gname, names in GROUPS.items():
        if gname in ("u", "uprev"):
            scale, l2s = float(ut.max()), float(np.sqrt((ut ** 2).sum()))
        else:
            scale = max(float(np.abs(ref_fields[n]).max()) for n in names)
            l2s = float(np.sqrt(sum((ref_fields[n] ** 2).sum() for n in names)))
        scale = scale if scale > 0 else 1.0
        l2s = l2s if l2s > 0 else 1.0
        for n in names:
            d = np.abs(gpu_fields[n] - ref_fields[n])
            out[n] = {"max": float(d.max()) / scale,
                      "max_hydro": float(d[m].max()) / scale if m.any() else 0.0,
                      "l2": float(np.sqrt((d ** 2).sum())) / l2s}
    return out
