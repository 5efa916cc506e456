"""Thin ctypes binding of the rsfde C ABI (include/rsfde.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device buffers are torch tensors on a ROCm device (passed by data pointer);
the stream is torch's current stream unless one is given.  Importing this
module loads librsfde.so from this package directory and raises if it is
missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsfde.so")

RSFDE_OK = 0
RSFDE_W_NOT_CONVERGED = 1
RSFDE_E_INVALID_ARG = -1
RSFDE_E_WORKSPACE = -2
RSFDE_E_HIP = -3
RSFDE_E_NONFINITE = -4
RSFDE_E_UNSUPPORTED = -5
RSFDE_E_STATE = -6

RSFDE_FP64 = 0
RSFDE_MIXED = 1
RSFDE_OPGM, RSFDE_TPGM, RSFDE_SPGM = 0, 1, 2
PREC_BP_INV, PREC_PHALF_BINV, PREC_PHALF, PREC_STRANG = 0, 1, 2, 3

FIELD_KINDS = {
    "zero": 0, "const": 1, "sumsq_exp": 2, "poly_t": 3, "sinprod_cos": 4,
    "sine_field": 5, "manufactured": 6, "sine_modes": 7,
}
WHICH_E, WHICH_F, WHICH_PSI = 0, 1, 2

EXPORTED = (
    "rsfde_workspace_size", "rsfde_setup", "rsfde_set_ebar", "rsfde_step", "rsfde_solve",
    "rsfde_destroy", "rsfde_strerror", "rsfde_set_fields", "rsfde_eval_field",
    "rsfde_eval_field_batch", "rsfde_set_graph", "rsfde_apply_A",
    "rsfde_apply_prec", "rsfde_apply_prec_form", "rsfde_compute_F", "rsfde_rhs", "rsfde_get_tables", "rsfde_set_timing",
    "rsfde_get_timing", "rsfde_prescan_ebar", "rsfde_get_pass_shape", "rsfde_set_true_residual",
    "rsfde_apply_prec_noalloc", "rsfde_get_pass_plan", "rsfde_solve_range",
)

K_CLASSES = ("mv_first", "mv_mid", "mv_last", "dst", "dsd", "dots", "orth_dots", "orth_norm", "update")


class rsfde_params(C.Structure):
    _fields_ = [
        ("d", C.c_int), ("n", C.c_int64 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("alpha", C.c_double * 3), ("kappa", C.c_double * 3), ("dt", C.c_double),
        ("e_min", C.c_double), ("e_max", C.c_double), ("restart", C.c_int), ("rtol", C.c_double),
        ("max_cycles", C.c_int), ("precision", C.c_int), ("x0_mode", C.c_int),
        ("inner_rtol", C.c_double), ("max_outer", C.c_int), ("method", C.c_int),
        ("outer_rtol", C.c_double),
    ]


class rsfde_stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("cycles", C.c_int), ("outer_sweeps", C.c_int), ("converged", C.c_int),
        ("beta0", C.c_double), ("rel_pres", C.c_double), ("rel_true_res", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rsfde_field(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("c", C.c_double * 4), ("modes", C.c_int),
        ("amp", C.POINTER(C.c_double)), ("time_dependent", C.c_int),
    ]


SAMPLE_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_double),
                        C.POINTER(C.c_double), C.c_void_p)


class RsfdeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {strerror(status)}")


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librsfde.so (raises OSError when it is missing or unloadable)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    P, I, D, V = C.c_void_p, C.c_int, C.c_double, C.c_void_p
    lib.rsfde_workspace_size.argtypes = [C.POINTER(rsfde_params), I, C.POINTER(C.c_size_t)]
    lib.rsfde_setup.argtypes = [C.POINTER(rsfde_params), I, P, C.c_size_t, P, C.POINTER(P)]
    lib.rsfde_set_ebar.argtypes = [P, I, D, D]
    lib.rsfde_step.argtypes = [P, D, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(rsfde_stats)]
    lib.rsfde_solve.argtypes = [P, I, SAMPLE_FN, P, C.POINTER(P), C.POINTER(rsfde_stats)]
    lib.rsfde_solve_range.argtypes = [P, I, I, SAMPLE_FN, P, C.POINTER(P), C.POINTER(rsfde_stats)]
    lib.rsfde_destroy.argtypes = [P]
    lib.rsfde_strerror.argtypes = [I]
    lib.rsfde_strerror.restype = C.c_char_p
    lib.rsfde_set_fields.argtypes = [P, I, C.POINTER(rsfde_field), C.POINTER(rsfde_field), C.POINTER(rsfde_field)]
    lib.rsfde_eval_field.argtypes = [P, I, I, D, P]
    lib.rsfde_eval_field_batch.argtypes = [P, I, D, C.POINTER(P)]
    lib.rsfde_apply_A.argtypes = [P, I, P, P, P]
    lib.rsfde_apply_prec.argtypes = [P, I, P, P]
    lib.rsfde_apply_prec_noalloc.argtypes = [P, I, P, P]
    lib.rsfde_apply_prec_form.argtypes = [P, I, I, P, P]
    lib.rsfde_compute_F.argtypes = [P, I, P, P]
    lib.rsfde_rhs.argtypes = [P, I, P, P, P, P]
    lib.rsfde_get_tables.argtypes = [P, I, I, P, P, P]
    lib.rsfde_set_timing.argtypes = [P, C.c_uint, I]
    lib.rsfde_set_graph.argtypes = [P, I]
    lib.rsfde_set_true_residual.argtypes = [P, I]
    lib.rsfde_get_timing.argtypes = [P, I, C.POINTER(C.c_longlong), C.POINTER(D), C.POINTER(D)]
    lib.rsfde_prescan_ebar.argtypes = [P, I, I]
    lib.rsfde_get_pass_shape.argtypes = [P, I, I, I, I, C.POINTER(I), C.POINTER(I)]
    lib.rsfde_get_pass_plan.argtypes = [P, I, I, I, I, C.POINTER(I), C.POINTER(I), C.POINTER(I)]
    for name in EXPORTED:
        getattr(lib, name)
        if name != "rsfde_strerror":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load_library().rsfde_strerror(int(status)).decode()


def _check(status: int, where: str) -> int:
    if status < 0:
        raise RsfdeError(status, where)
    return status


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def make_params(d, n, alpha, kappa, dt, *, lo=None, hi=None, e_min=0.0, e_max=0.0, restart=20,
                rtol=1e-10, max_cycles=10, precision=RSFDE_FP64, x0_mode=0, inner_rtol=0.0,
                max_outer=0, method=0, outer_rtol=0.0) -> rsfde_params:
    p = rsfde_params()
    p.d = int(d)
    for i in range(3):
        p.n[i] = int(n[i]) if i < d else 1
        p.lo[i] = float(lo[i]) if (lo is not None and i < d) else 0.0
        p.hi[i] = float(hi[i]) if (hi is not None and i < d) else 1.0
        p.alpha[i] = float(alpha[i]) if i < d else 1.5
        p.kappa[i] = float(kappa[i]) if i < d else 0.0
    p.dt = float(dt)
    p.e_min, p.e_max = float(e_min), float(e_max)
    p.restart, p.rtol, p.max_cycles = int(restart), float(rtol), int(max_cycles)
    p.precision, p.x0_mode = int(precision), int(x0_mode)
    p.inner_rtol, p.max_outer = float(inner_rtol), int(max_outer)
    p.method = int(method)
    p.outer_rtol = float(outer_rtol)
    return p


def params_from_instance(inst, **over) -> rsfde_params:
    """rsfde_params for a rsfde_workloads.Instance (solver settings may be overridden)."""
    kw = dict(lo=inst.lo, hi=inst.hi, restart=inst.restart, rtol=inst.rtol, max_cycles=inst.max_cycles)
    kw.update(over)
    return make_params(inst.d, inst.n, inst.alpha, inst.kappa, inst.T / inst.M, **kw)


def make_field(spec) -> tuple:
    """rsfde_field for a rsfde_workloads.FieldSpec; returns (field, keepalive)."""
    f = rsfde_field()
    f.kind = FIELD_KINDS[spec.kind]
    for i, v in enumerate(spec.c[:4]):
        f.c[i] = float(v)
    f.modes = int(spec.modes)
    keep = None
    if spec.amp is not None:
        keep = (C.c_double * len(spec.amp))(*[float(v) for v in spec.amp])
        f.amp = C.cast(keep, C.POINTER(C.c_double))
    f.time_dependent = 1 if spec.time_dependent else 0
    return f, keep


# ---- entry points with the C names ------------------------------------------------

def rsfde_workspace_size(params: Sequence[rsfde_params]) -> int:
    arr = (rsfde_params * len(params))(*params)
    out = C.c_size_t(0)
    _check(load_library().rsfde_workspace_size(arr, len(params), C.byref(out)), "rsfde_workspace_size")
    return int(out.value)


def rsfde_setup(params: Sequence[rsfde_params], workspace, stream=None) -> C.c_void_p:
    arr = (rsfde_params * len(params))(*params)
    h = C.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(load_library().rsfde_setup(arr, len(params), _ptr(workspace), nbytes, _stream(stream),
                                      C.byref(h)), "rsfde_setup")
    return h


def rsfde_set_ebar(h, instance: int, e_min: float, e_max: float) -> None:
    _check(load_library().rsfde_set_ebar(h, instance, e_min, e_max), "rsfde_set_ebar")


def _ptr_array(ts) -> C.Array:
    return (C.c_void_p * len(ts))(*[_ptr(t) for t in ts])


def rsfde_step(h, t_m: float, e_half: Sequence, f_half: Sequence, u: Sequence) -> tuple:
    st = (rsfde_stats * len(u))()
    s = _check(load_library().rsfde_step(h, t_m, _ptr_array(e_half), _ptr_array(f_half), _ptr_array(u), st),
               "rsfde_step")
    return s, [x.as_dict() for x in st]


def rsfde_solve(h, M: int, u: Sequence, sample=None, ctx=None) -> tuple:
    st = (rsfde_stats * len(u))()
    fn = SAMPLE_FN(0) if sample is None else SAMPLE_FN(sample)
    s = _check(load_library().rsfde_solve(h, int(M), fn, ctx, _ptr_array(u), st), "rsfde_solve")
    return s, [x.as_dict() for x in st]


def rsfde_solve_range(h, m0: int, M: int, u: Sequence, sample=None, ctx=None) -> tuple:
    st = (rsfde_stats * len(u))()
    fn = SAMPLE_FN(0) if sample is None else SAMPLE_FN(sample)
    s = _check(load_library().rsfde_solve_range(h, int(m0), int(M), fn, ctx, _ptr_array(u), st),
               "rsfde_solve_range")
    return s, [x.as_dict() for x in st]


def rsfde_destroy(h) -> None:
    _check(load_library().rsfde_destroy(h), "rsfde_destroy")


def rsfde_strerror(status: int) -> str:
    return strerror(status)


def rsfde_set_fields(h, instance: int, e_spec, f_spec, psi_spec) -> None:
    fe, k1 = make_field(e_spec)
    ff, k2 = make_field(f_spec)
    fp, k3 = make_field(psi_spec)
    _check(load_library().rsfde_set_fields(h, instance, C.byref(fe), C.byref(ff), C.byref(fp)),
           "rsfde_set_fields")
    del k1, k2, k3


def rsfde_eval_field(h, instance: int, which: int, t: float, out) -> None:
    _check(load_library().rsfde_eval_field(h, instance, which, t, _ptr(out)), "rsfde_eval_field")


def rsfde_eval_field_batch(h, which: int, t: float, outs: Sequence) -> None:
    _check(load_library().rsfde_eval_field_batch(h, which, t, _ptr_array(outs)), "rsfde_eval_field_batch")


def rsfde_apply_A(h, instance: int, e, v, out) -> None:
    _check(load_library().rsfde_apply_A(h, instance, _ptr(e), _ptr(v), _ptr(out)), "rsfde_apply_A")


def rsfde_apply_prec(h, instance: int, r, out) -> None:
    _check(load_library().rsfde_apply_prec(h, instance, _ptr(r), _ptr(out)), "rsfde_apply_prec")


def rsfde_apply_prec_noalloc(h, instance: int, r, out) -> None:
    _check(load_library().rsfde_apply_prec_noalloc(h, instance, _ptr(r), _ptr(out)),
           "rsfde_apply_prec_noalloc")


def rsfde_apply_prec_form(h, instance: int, form: int, r, out) -> None:
    """form: PREC_BP_INV, PREC_PHALF_BINV, PREC_PHALF or (Strang-form instances) PREC_STRANG."""
    _check(load_library().rsfde_apply_prec_form(h, instance, form, _ptr(r), _ptr(out)),
           "rsfde_apply_prec_form")


def rsfde_compute_F(h, instance: int, f_closure, out) -> None:
    _check(load_library().rsfde_compute_F(h, instance, _ptr(f_closure), _ptr(out)), "rsfde_compute_F")


def rsfde_rhs(h, instance: int, e, F, u, out) -> None:
    _check(load_library().rsfde_rhs(h, instance, _ptr(e), _ptr(F), _ptr(u), _ptr(out)), "rsfde_rhs")


def rsfde_get_tables(h, instance: int, axis: int, N: int):
    import numpy as np
    s = np.zeros(N)
    q = np.zeros(N)
    lam = np.zeros(N)
    _check(load_library().rsfde_get_tables(h, instance, axis, s.ctypes.data, q.ctypes.data, lam.ctypes.data),
           "rsfde_get_tables")
    return s, q, lam


def rsfde_get_pass_shape(h, instance: int, axis: int, precision: int, transform: int):
    """(L, complex transforms per workgroup) of the autotuned pencil passes."""
    L, F = C.c_int(0), C.c_int(0)
    _check(load_library().rsfde_get_pass_shape(h, instance, axis, precision, transform,
                                               C.byref(L), C.byref(F)), "rsfde_get_pass_shape")
    return L.value, F.value


def rsfde_get_pass_plan(h, instance: int, axis: int, precision: int, transform: int):
    """(plan code, radices) of the radix plan the autotuner picked for a pencil pass."""
    code, n = C.c_int(0), C.c_int(0)
    rad = (C.c_int * 8)()
    _check(load_library().rsfde_get_pass_plan(h, instance, axis, precision, transform, C.byref(code),
                                              rad, C.byref(n)), "rsfde_get_pass_plan")
    return int(code.value), [int(rad[k]) for k in range(n.value)]


def rsfde_set_graph(h, enable: bool) -> None:
    _check(load_library().rsfde_set_graph(h, 1 if enable else 0), "rsfde_set_graph")


def rsfde_set_true_residual(h, enable: bool) -> None:
    _check(load_library().rsfde_set_true_residual(h, 1 if enable else 0), "rsfde_set_true_residual")


def rsfde_set_timing(h, mask: int, every: int = 1) -> None:
    """mask: bit i enables HIP-event timing of kernel class K_CLASSES[i] (one launch in
    `every`); 0 disables."""
    _check(load_library().rsfde_set_timing(h, int(mask), int(every)), "rsfde_set_timing")


def rsfde_get_timing(h, kclass: int) -> tuple:
    """(launches, total ms, total algorithmic bytes) of one kernel class."""
    n = C.c_longlong(0)
    ms = C.c_double(0)
    by = C.c_double(0)
    _check(load_library().rsfde_get_timing(h, int(kclass), C.byref(n), C.byref(ms), C.byref(by)),
           "rsfde_get_timing")
    return int(n.value), float(ms.value), float(by.value)


def rsfde_prescan_ebar(h, instance: int, M: int) -> None:
    _check(load_library().rsfde_prescan_ebar(h, instance, int(M)), "rsfde_prescan_ebar")


class Solver:
    """Owns a handle and its torch-allocated workspace for a list of instances."""

    def __init__(self, params: Sequence[rsfde_params], device="cuda", stream=None):
        import torch
        self.params = list(params)
        self.nbytes = rsfde_workspace_size(self.params)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.h = rsfde_setup(self.params, self.workspace, stream)

    def close(self):
        if self.h is not None and self.h.value:
            rsfde_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
