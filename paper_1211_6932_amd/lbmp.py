"""ctypes binding of liblbmp.so (include/lbmp.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The functions keep the C names; ``Sim`` is a small convenience
wrapper that lets torch supply device memory and the stream.

The library must have been built (``python -m paper_1211_6932_amd.build``);
importing this module raises if it is missing, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmp.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_EUNSTABLE, LB_ESTATE = 0, -1, -2, -3, -4, -5
LB_BC_PERIODIC, LB_BC_WALLS_Y = 0, 1
LB_STORE_F32, LB_STORE_F16_OFFSET, LB_STORE_BF16_OFFSET = 0, 1, 2
LB_STORE_F16_LOCAL, LB_STORE_BF16_LOCAL, LB_STORE_F16_DEST = 3, 4, 5
LB_PSI_CS, LB_PSI_SS = 0, 1
LB_STENCIL_NEAREST, LB_STENCIL_MULTIRANGE = 0, 1
STORE_NAMES = {"f32": LB_STORE_F32, "f16": LB_STORE_F16_OFFSET, "bf16": LB_STORE_BF16_OFFSET,
               "f16local": LB_STORE_F16_LOCAL, "bf16local": LB_STORE_BF16_LOCAL, "f16dest": LB_STORE_F16_DEST}
STATUS_NAMES = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EHIP", -4: "LB_EUNSTABLE",
                -5: "LB_ESTATE"}


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc", ctypes.c_int32), ("store", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("T", ctypes.c_double),
        ("G", ctypes.c_double), ("sigma", ctypes.c_double),
        ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double), ("s_zeta", ctypes.c_double),
        ("s_j", ctypes.c_double), ("s_q", ctypes.c_double),
        ("nu_l", ctypes.c_double), ("nu_g", ctypes.c_double), ("rho_switch", ctypes.c_double),
        ("rho_ref", ctypes.c_double),
        ("psi_form", ctypes.c_int32), ("stencil", ctypes.c_int32), ("psi_eps", ctypes.c_double),
    ]


class lb_region(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_double), ("cy", ctypes.c_double), ("r_min", ctypes.c_double),
                ("r_max", ctypes.c_double)]


class lb_diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("p_in", ctypes.c_double), ("p_out", ctypes.c_double), ("dp", ctypes.c_double),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("n_in", ctypes.c_double), ("n_out", ctypes.c_double), ("max_u", ctypes.c_double),
        ("unstable", ctypes.c_int32), ("reserved", ctypes.c_int32), ("step", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


EXPORTS = [
    "lb_validate_params", "lb_workspace_bytes", "lb_state_bytes", "lb_init", "lb_step", "lb_moments",
    "lb_diagnostics", "lb_check", "lb_time", "lb_get_state", "lb_set_state", "lb_set_launch",
    "lb_destroy", "lb_last_error", "lb_copy_probe",
    "lb_batch_workspace_bytes", "lb_batch_init", "lb_batch_step", "lb_batch_moments",
    "lb_batch_diagnostics", "lb_batch_get_state", "lb_batch_check", "lb_batch_times", "lb_batch_set_launch",
    "lb_batch_destroy", "lb_batch_diagnostics_all", "lb_batch_tune",
    "lbml_workspace_bytes", "lbml_init", "lbml_set_params", "lbml_get_params", "lbml_forward",
    "lbml_loss_grad", "lbml_adam", "lbml_train_step", "lbml_destroy", "lbml_profile_extract",
    "lbml_profile_to_rho0", "lbml_gemm_bf16", "lbml_profile_scratch_bytes", "lbml_profile_to_rho0_mass",
    "lbml_profile_extract_noalloc", "lbml_profile_levels", "lbml_profile_anchor", "lbml_level_fit",
    "lbml_level_eval", "lbml_train_steps",
]
LBML_IN, LBML_HIDDEN, LBML_OUT, LBML_PARAMS = 4, 256, 128, 165760
LBML_LEVEL_TERMS = 168


class lbml_level_model(ctypes.Structure):
    """Level model of include/lbml.h: feature ranges and Chebyshev coefficients."""
    _fields_ = [("lo", ctypes.c_double * LBML_IN), ("hi", ctypes.c_double * LBML_IN),
                ("coef", ctypes.c_double * LBML_LEVEL_TERMS)]

_lib = None


def load():
    """Load liblbmp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1211_6932_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(lb_params)
    vp = ctypes.c_void_p
    L.lb_validate_params.argtypes = [P]
    L.lb_validate_params.restype = ctypes.c_int
    L.lb_workspace_bytes.argtypes = [P]
    L.lb_workspace_bytes.restype = ctypes.c_size_t
    L.lb_state_bytes.argtypes = [P]
    L.lb_state_bytes.restype = ctypes.c_size_t
    L.lb_init.argtypes = [ctypes.POINTER(vp), P, vp, ctypes.c_size_t, vp, vp, vp, vp]
    L.lb_init.restype = ctypes.c_int
    L.lb_step.argtypes = [vp, ctypes.c_int64]
    L.lb_step.restype = ctypes.c_int
    L.lb_moments.argtypes = [vp, vp, vp, vp]
    L.lb_moments.restype = ctypes.c_int
    L.lb_diagnostics.argtypes = [vp, ctypes.POINTER(lb_region), ctypes.POINTER(lb_region),
                                 ctypes.POINTER(lb_diag)]
    L.lb_diagnostics.restype = ctypes.c_int
    L.lb_check.argtypes = [vp]
    L.lb_check.restype = ctypes.c_int
    L.lb_time.argtypes = [vp]
    L.lb_time.restype = ctypes.c_int64
    L.lb_get_state.argtypes = [vp, vp]
    L.lb_get_state.restype = ctypes.c_int
    L.lb_set_state.argtypes = [vp, vp, ctypes.c_int64]
    L.lb_set_state.restype = ctypes.c_int
    L.lb_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.lb_set_launch.restype = ctypes.c_int
    L.lb_destroy.argtypes = [vp]
    L.lb_destroy.restype = ctypes.c_int
    L.lb_last_error.argtypes = []
    L.lb_last_error.restype = ctypes.c_char_p
    L.lb_copy_probe.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.lb_copy_probe.restype = ctypes.c_int
    vpp = ctypes.POINTER(vp)
    L.lb_batch_workspace_bytes.argtypes = [P, ctypes.c_int32]
    L.lb_batch_workspace_bytes.restype = ctypes.c_size_t
    L.lb_batch_init.argtypes = [ctypes.POINTER(vp), P, ctypes.c_int32, vp, ctypes.c_size_t, vpp, vpp, vpp, vp]
    L.lb_batch_init.restype = ctypes.c_int
    L.lb_batch_step.argtypes = [vp, ctypes.c_int64]
    L.lb_batch_step.restype = ctypes.c_int
    L.lb_batch_moments.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    L.lb_batch_moments.restype = ctypes.c_int
    L.lb_batch_diagnostics.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(lb_region), ctypes.POINTER(lb_region),
                                       ctypes.POINTER(lb_diag)]
    L.lb_batch_diagnostics.restype = ctypes.c_int
    L.lb_batch_get_state.argtypes = [vp, ctypes.c_int32, vp]
    L.lb_batch_get_state.restype = ctypes.c_int
    L.lb_batch_check.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.lb_batch_check.restype = ctypes.c_int
    L.lb_batch_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.lb_batch_times.restype = ctypes.c_int
    L.lb_batch_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.lb_batch_set_launch.restype = ctypes.c_int
    L.lb_batch_tune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.lb_batch_tune.restype = ctypes.c_int
    L.lb_batch_destroy.argtypes = [vp]
    L.lb_batch_destroy.restype = ctypes.c_int
    L.lb_batch_diagnostics_all.argtypes = [vp, ctypes.POINTER(lb_region), ctypes.POINTER(lb_region),
                                           ctypes.POINTER(lb_diag)]
    L.lb_batch_diagnostics_all.restype = ctypes.c_int
    i32, i64, f32, f64, dp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.POINTER(
        ctypes.c_double)
    sigs = {
        "lbml_workspace_bytes": ([i32], ctypes.c_size_t),
        "lbml_init": ([ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, vp, dp, dp, vp], ctypes.c_int),
        "lbml_set_params": ([vp, vp], ctypes.c_int),
        "lbml_get_params": ([vp, vp], ctypes.c_int),
        "lbml_forward": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "lbml_loss_grad": ([vp, vp, vp, vp, i32, vp, vp], ctypes.c_int),
        "lbml_adam": ([vp, f32], ctypes.c_int),
        "lbml_train_step": ([vp, vp, vp, vp, i32, f32, vp], ctypes.c_int),
        "lbml_train_steps": ([vp, vp, vp, vp, i32, vp, vp, i32, i32, vp], ctypes.c_int),
        "lbml_destroy": ([vp], ctypes.c_int),
        "lbml_profile_scratch_bytes": ([i32], ctypes.c_size_t),
        "lbml_profile_extract": ([vp, i32, i32, f64, f64, f64, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
        "lbml_profile_extract_noalloc": ([vp, i32, i32, f64, f64, f64, vp, vp], ctypes.c_int),
        "lbml_profile_to_rho0": ([vp, f64, f64, f64, i32, i32, vp, vp], ctypes.c_int),
        "lbml_profile_to_rho0_mass": ([vp, f64, f64, f64, i32, i32, f64, vp, vp, vp], ctypes.c_int),
        "lbml_gemm_bf16": ([vp, i64, i64, vp, i64, i64, vp, i32, i32, i32, i32, vp], ctypes.c_int),
        "lbml_profile_levels": ([vp, vp, i32, vp, vp], ctypes.c_int),
        "lbml_profile_anchor": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "lbml_level_fit": ([dp, dp, i32, ctypes.POINTER(lbml_level_model)], ctypes.c_int),
        "lbml_level_eval": ([ctypes.POINTER(lbml_level_model), dp, i32, dp], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


class LbError(RuntimeError):
    def __init__(self, status, where):
        msg = load().lb_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({msg})")
        self.status = status


def _check(status, where):
    if status != LB_OK:
        raise LbError(status, where)
    return status


def make_params(d: dict, store="f32", rho_ref=0.0) -> lb_params:
    """lb_params from a parameter dictionary (keys as in the C struct)."""
    s = STORE_NAMES[store] if isinstance(store, str) else int(store)
    return lb_params(int(d["nx"]), int(d["ny"]), int(d.get("bc", 0)), s,
                     float(d["a"]), float(d["b"]), float(d["R"]), float(d["T"]), float(d["G"]),
                     float(d["sigma"]), float(d["s_rho"]), float(d["s_e"]), float(d["s_zeta"]),
                     float(d["s_j"]), float(d["s_q"]), float(d["nu_l"]), float(d["nu_g"]),
                     float(d["rho_switch"]), float(rho_ref), int(d.get("psi_form", 0)),
                     int(d.get("stencil", 0)), float(d.get("psi_eps", 0.0)))


# -------------------------------------------------------------- C names (marshalling only)

def lb_validate_params(p: lb_params) -> int:
    return load().lb_validate_params(ctypes.byref(p))


def lb_workspace_bytes(p: lb_params) -> int:
    return load().lb_workspace_bytes(ctypes.byref(p))


def lb_state_bytes(p: lb_params) -> int:
    return load().lb_state_bytes(ctypes.byref(p))


def lb_init(p: lb_params, workspace_ptr: int, workspace_bytes: int, rho0_ptr: int, ux0_ptr,
            uy0_ptr, stream: int):
    ctx = ctypes.c_void_p()
    st = load().lb_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(workspace_ptr),
                        workspace_bytes, ctypes.c_void_p(rho0_ptr), ctypes.c_void_p(ux0_ptr or None),
                        ctypes.c_void_p(uy0_ptr or None), ctypes.c_void_p(stream or None))
    _check(st, "lb_init")
    return ctx


def lb_step(ctx, n: int):
    return _check(load().lb_step(ctx, int(n)), "lb_step")


def lb_moments(ctx, rho_ptr, ux_ptr, uy_ptr):
    return _check(load().lb_moments(ctx, ctypes.c_void_p(rho_ptr or None), ctypes.c_void_p(ux_ptr or None),
                                    ctypes.c_void_p(uy_ptr or None)), "lb_moments")


def lb_diagnostics(ctx, region_in: lb_region, region_out: lb_region, raise_unstable=True) -> lb_diag:
    d = lb_diag()
    st = load().lb_diagnostics(ctx, ctypes.byref(region_in), ctypes.byref(region_out), ctypes.byref(d))
    if st != LB_OK and (raise_unstable or st != LB_EUNSTABLE):
        raise LbError(st, "lb_diagnostics")
    return d


def lb_check(ctx) -> int:
    return load().lb_check(ctx)


def lb_time(ctx) -> int:
    return load().lb_time(ctx)


def lb_get_state(ctx, dst_ptr: int):
    return _check(load().lb_get_state(ctx, ctypes.c_void_p(dst_ptr)), "lb_get_state")


def lb_set_state(ctx, src_ptr: int, t: int):
    return _check(load().lb_set_state(ctx, ctypes.c_void_p(src_ptr), int(t)), "lb_set_state")


def lb_set_launch(ctx, strip_rows: int = 0, band: int = 0, graph_chunk: int = 0):
    return _check(load().lb_set_launch(ctx, int(strip_rows), int(band), int(graph_chunk)), "lb_set_launch")


def lb_destroy(ctx):
    return load().lb_destroy(ctx)


def lb_last_error() -> str:
    return load().lb_last_error().decode(errors="replace")


def lb_copy_probe(src_ptr: int, dst_ptr: int, nbytes: int, stream: int):
    return _check(load().lb_copy_probe(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes),
                                       ctypes.c_void_p(stream or None)), "lb_copy_probe")


def lb_batch_workspace_bytes(params_array, n: int) -> int:
    return load().lb_batch_workspace_bytes(params_array, int(n))


def lb_batch_init(params_array, n, workspace_ptr, workspace_bytes, rho0_ptrs, ux0_ptrs, uy0_ptrs, stream):
    def arr(ptrs):
        if ptrs is None:
            return None
        return (ctypes.c_void_p * n)(*[p or None for p in ptrs])
    b = ctypes.c_void_p()
    st = load().lb_batch_init(ctypes.byref(b), params_array, int(n), ctypes.c_void_p(workspace_ptr),
                              workspace_bytes, arr(rho0_ptrs), arr(ux0_ptrs), arr(uy0_ptrs),
                              ctypes.c_void_p(stream or None))
    _check(st, "lb_batch_init")
    return b


def lb_batch_step(b, n: int):
    return _check(load().lb_batch_step(b, int(n)), "lb_batch_step")


def lb_batch_moments(b, i, rho_ptr, ux_ptr, uy_ptr):
    return _check(load().lb_batch_moments(b, int(i), ctypes.c_void_p(rho_ptr or None),
                                          ctypes.c_void_p(ux_ptr or None), ctypes.c_void_p(uy_ptr or None)),
                  "lb_batch_moments")


def lb_batch_diagnostics(b, i, region_in: lb_region, region_out: lb_region, raise_unstable=True) -> lb_diag:
    d = lb_diag()
    st = load().lb_batch_diagnostics(b, int(i), ctypes.byref(region_in), ctypes.byref(region_out), ctypes.byref(d))
    if st != LB_OK and (raise_unstable or st != LB_EUNSTABLE):
        raise LbError(st, "lb_batch_diagnostics")
    return d


def lb_batch_diagnostics_all(b, regions_in, regions_out):
    """Returns (status, list of lb_diag); status LB_EUNSTABLE still fills every entry."""
    n = len(regions_in)
    rin = (lb_region * n)(*regions_in)
    rout = (lb_region * n)(*regions_out)
    out = (lb_diag * n)()
    st = load().lb_batch_diagnostics_all(b, rin, rout, out)
    if st not in (LB_OK, LB_EUNSTABLE):
        raise LbError(st, "lb_batch_diagnostics_all")
    return st, list(out)


def lb_batch_get_state(b, i, dst_ptr):
    return _check(load().lb_batch_get_state(b, int(i), ctypes.c_void_p(dst_ptr)), "lb_batch_get_state")


def lb_batch_check(b):
    n = ctypes.c_int32(0)
    st = load().lb_batch_check(b, ctypes.byref(n))
    return st, n.value


def lb_batch_times(b, n):
    out = (ctypes.c_double * n)()
    _check(load().lb_batch_times(b, out), "lb_batch_times")
    return list(out)


LB_BATCH_STEPWISE, LB_BATCH_PERSISTENT = 0, 1


def lb_batch_set_launch(b, mode: int, strip_rows: int = 0):
    return _check(load().lb_batch_set_launch(b, int(mode), int(strip_rows)), "lb_batch_set_launch")


def lb_batch_tune(b, n: int, trial_steps: int = 8):
    """Autotune the stepwise strip heights; returns the height chosen for each lattice."""
    rows = (ctypes.c_int32 * n)()
    _check(load().lb_batch_tune(b, int(trial_steps), rows), "lb_batch_tune")
    return list(rows)


def lb_batch_destroy(b):
    return load().lb_batch_destroy(b)


def _vp(x):
    return ctypes.c_void_p(x or None)


def lbml_workspace_bytes(max_batch: int) -> int:
    return load().lbml_workspace_bytes(int(max_batch))


def lbml_init(max_batch, workspace_ptr, workspace_bytes, theta0_ptr, mu, sd, stream):
    net = ctypes.c_void_p()
    mu_a = (ctypes.c_double * 4)(*[float(v) for v in mu])
    sd_a = (ctypes.c_double * 4)(*[float(v) for v in sd])
    _check(load().lbml_init(ctypes.byref(net), int(max_batch), _vp(workspace_ptr), int(workspace_bytes),
                            _vp(theta0_ptr), mu_a, sd_a, _vp(stream)), "lbml_init")
    return net


def lbml_set_params(net, theta_ptr):
    return _check(load().lbml_set_params(net, _vp(theta_ptr)), "lbml_set_params")


def lbml_get_params(net, theta_ptr):
    return _check(load().lbml_get_params(net, _vp(theta_ptr)), "lbml_get_params")


def lbml_forward(net, x_ptr, base_ptr, B, y_ptr):
    return _check(load().lbml_forward(net, _vp(x_ptr), _vp(base_ptr), int(B), _vp(y_ptr)), "lbml_forward")


def lbml_loss_grad(net, x_ptr, base_ptr, target_ptr, B, loss_ptr, grad_ptr):
    return _check(load().lbml_loss_grad(net, _vp(x_ptr), _vp(base_ptr), _vp(target_ptr), int(B), _vp(loss_ptr),
                                        _vp(grad_ptr)), "lbml_loss_grad")


def lbml_adam(net, lr):
    return _check(load().lbml_adam(net, float(lr)), "lbml_adam")


def lbml_train_step(net, x_ptr, base_ptr, target_ptr, B, lr, loss_ptr):
    return _check(load().lbml_train_step(net, _vp(x_ptr), _vp(base_ptr), _vp(target_ptr), int(B), float(lr),
                                         _vp(loss_ptr)), "lbml_train_step")


def lbml_destroy(net):
    return load().lbml_destroy(net)


def lbml_profile_scratch_bytes(ny):
    return load().lbml_profile_scratch_bytes(int(ny))


def lbml_profile_extract_noalloc(rho_ptr, nx, ny, cx, cy, R, logrho_ptr, stream):
    return _check(load().lbml_profile_extract_noalloc(_vp(rho_ptr), int(nx), int(ny), float(cx), float(cy), float(R),
                                                      _vp(logrho_ptr), _vp(stream)), "lbml_profile_extract_noalloc")


def lbml_profile_extract(rho_ptr, nx, ny, cx, cy, R, scratch_ptr, scratch_bytes, logrho_ptr, stream):
    return _check(load().lbml_profile_extract(_vp(rho_ptr), int(nx), int(ny), float(cx), float(cy), float(R),
                                              _vp(scratch_ptr), int(scratch_bytes), _vp(logrho_ptr), _vp(stream)),
                  "lbml_profile_extract")


def lbml_profile_to_rho0(logrho_ptr, R, cx, cy, nx, ny, rho0_ptr, stream):
    return _check(load().lbml_profile_to_rho0(_vp(logrho_ptr), float(R), float(cx), float(cy), int(nx), int(ny),
                                              _vp(rho0_ptr), _vp(stream)), "lbml_profile_to_rho0")


def lbml_profile_to_rho0_mass(logrho_ptr, R, cx, cy, nx, ny, mass, shift_ptr, rho0_ptr, stream):
    return _check(load().lbml_profile_to_rho0_mass(_vp(logrho_ptr), float(R), float(cx), float(cy), int(nx), int(ny),
                                                   float(mass), _vp(shift_ptr), _vp(rho0_ptr), _vp(stream)),
                  "lbml_profile_to_rho0_mass")


def lbml_profile_levels(L_ptr, x_ptr, B, levels_ptr, stream):
    return _check(load().lbml_profile_levels(_vp(L_ptr), _vp(x_ptr), int(B), _vp(levels_ptr), _vp(stream)),
                  "lbml_profile_levels")


def lbml_profile_anchor(L_ptr, x_ptr, target_ptr, B, stream):
    return _check(load().lbml_profile_anchor(_vp(L_ptr), _vp(x_ptr), _vp(target_ptr), int(B), _vp(stream)),
                  "lbml_profile_anchor")


def _host_f64(a, cols=None):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    if cols is not None:
        a = a.reshape(-1, cols)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lbml_level_fit(x, y):
    """Level model fitted to targets y [n] at raw features x [n][4] (host arrays)."""
    x, xp = _host_f64(x, LBML_IN)
    y, yp = _host_f64(y)
    if y.size != x.shape[0]:
        raise ValueError("x and y disagree in length")
    m = lbml_level_model()
    _check(load().lbml_level_fit(xp, yp, int(x.shape[0]), ctypes.byref(m)), "lbml_level_fit")
    return m


def lbml_level_eval(model, x):
    """The level model at raw features x [n][4] (host); returns a float64 array [n]."""
    import numpy as np
    x, xp = _host_f64(x, LBML_IN)
    y = np.empty(x.shape[0], dtype=np.float64)
    _check(load().lbml_level_eval(ctypes.byref(model), xp, int(x.shape[0]),
                                  y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "lbml_level_eval")
    return y


def lbml_gemm_bf16(A_ptr, sam, sak, B_ptr, sbk, sbn, C_ptr, ldc, M, N, K, stream):
    return _check(load().lbml_gemm_bf16(_vp(A_ptr), int(sam), int(sak), _vp(B_ptr), int(sbk), int(sbn), _vp(C_ptr),
                                        int(ldc), int(M), int(N), int(K), _vp(stream)), "lbml_gemm_bf16")


# -------------------------------------------------------------- torch convenience wrapper

class Sim:
    """One lattice on the current ROCm device.  torch allocates the workspace,
    the input/output fields and (by default) a dedicated non-default stream."""

    def __init__(self, params: dict, rho0, ux0=None, uy0=None, store="f32", rho_ref=0.0,
                 stream=None, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbmp.Sim needs a ROCm GPU")
        self.torch = torch
        self.p = make_params(params, store, rho_ref)
        _check(lb_validate_params(self.p), "lb_validate_params")
        self.nx, self.ny = self.p.nx, self.p.ny
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.device = torch.device(device)
        shape = (self.ny, self.nx)

        def dev(t):
            if t is None:
                return None
            t = torch.as_tensor(t)
            if tuple(t.shape) != shape:
                raise ValueError(f"field shape {tuple(t.shape)} != {shape}")
            return t.to(device=self.device, dtype=torch.float32).contiguous()

        r, ux, uy = dev(rho0), dev(ux0), dev(uy0)
        nbytes = lb_workspace_bytes(self.p)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.stream(self.stream):
            # the inputs were produced on torch's current stream
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            self.ctx = lb_init(self.p, self.workspace.data_ptr(), nbytes, r.data_ptr(),
                               ux.data_ptr() if ux is not None else 0,
                               uy.data_ptr() if uy is not None else 0, self.stream.cuda_stream)

    def close(self):
        """Synchronise the stream and release the library context."""
        ctx = getattr(self, "ctx", None)
        if ctx is not None:
            self.ctx = None
            self.stream.synchronize()
            lb_destroy(ctx)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may already be gone
            pass

    @property
    def t(self):
        return lb_time(self.ctx)

    def step(self, n=1):
        lb_step(self.ctx, n)
        return self

    def set_launch(self, strip_rows=0, band=0, graph_chunk=0):
        lb_set_launch(self.ctx, strip_rows, band, graph_chunk)

    def moments(self):
        """(rho, ux, uy) FP32 device tensors [ny][nx] at the current time."""
        torch = self.torch
        out = [torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device) for _ in range(3)]
        lb_moments(self.ctx, *[o.data_ptr() for o in out])
        self.stream.synchronize()
        return tuple(out)

    def check(self):
        st = lb_check(self.ctx)
        if st != LB_OK:
            raise LbError(st, "lb_check")

    def diagnostics(self, cx, cy, r_in, r_out0, r_out1=math.inf, raise_unstable=True):
        """Reductions with region in = d < r_in and out = r_out0 <= d < r_out1 around (cx, cy)."""
        rin = lb_region(cx, cy, 0.0, r_in)
        rout = lb_region(cx, cy, r_out0, r_out1)
        return lb_diagnostics(self.ctx, rin, rout, raise_unstable).as_dict()

    def get_state(self):
        torch = self.torch
        buf = torch.empty(lb_state_bytes(self.p), dtype=torch.uint8, device=self.device)
        lb_get_state(self.ctx, buf.data_ptr())
        self.stream.synchronize()
        return buf

    def set_state(self, buf, t):
        lb_set_state(self.ctx, buf.data_ptr(), t)
        self.stream.synchronize()


class Batch:
    """Many independent lattices advanced together (one launch per step, or one
    persistent launch)."""

    def __init__(self, params_list, rho0_list, ux0_list=None, uy0_list=None, store="f32", stream=None,
                 device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbmp.Batch needs a ROCm GPU")
        self.torch = torch
        self.n = n = len(params_list)
        self.params = (lb_params * n)(*[make_params(d, store) for d in params_list])
        self.shapes = [(p.ny, p.nx) for p in self.params]
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)

        def dev(t, shape):
            if t is None:
                return None
            t = torch.as_tensor(t)
            if tuple(t.shape) != shape:
                raise ValueError(f"field shape {tuple(t.shape)} != {shape}")
            return t.to(device=self.device, dtype=torch.float32).contiguous()

        self._inputs = []
        ptrs = {"rho": [], "ux": [], "uy": []}
        for i in range(n):
            for key, lst in (("rho", rho0_list), ("ux", ux0_list), ("uy", uy0_list)):
                t = dev(None if lst is None else lst[i], self.shapes[i])
                self._inputs.append(t)
                ptrs[key].append(0 if t is None else t.data_ptr())
        nbytes = lb_batch_workspace_bytes(self.params, n)
        if nbytes == 0:
            raise LbError(LB_EINVAL, "lb_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.stream(self.stream):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            self.b = lb_batch_init(self.params, n, self.workspace.data_ptr(), nbytes, ptrs["rho"],
                                   None if ux0_list is None else ptrs["ux"],
                                   None if uy0_list is None else ptrs["uy"], self.stream.cuda_stream)
        self._inputs = None

    def close(self):
        b = getattr(self, "b", None)
        if b is not None:
            self.b = None
            self.stream.synchronize()
            lb_batch_destroy(b)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def step(self, n):
        lb_batch_step(self.b, n)
        return self

    def times(self):
        return lb_batch_times(self.b, self.n)

    def set_launch(self, mode=0, strip_rows=0):
        """mode: LB_BATCH_STEPWISE (0) or LB_BATCH_PERSISTENT (1)."""
        lb_batch_set_launch(self.b, mode, strip_rows)

    def tune(self, trial_steps=8):
        """Autotune the stepwise strip heights (state unchanged); per-lattice heights."""
        return lb_batch_tune(self.b, self.n, trial_steps)

    def check(self):
        return lb_batch_check(self.b)

    def diagnostics(self, i, cx, cy, r_in, r_out0, r_out1=math.inf, raise_unstable=True):
        """Reductions of lattice i (see Sim.diagnostics)."""
        return lb_batch_diagnostics(self.b, i, lb_region(cx, cy, 0.0, r_in), lb_region(cx, cy, r_out0, r_out1),
                                    raise_unstable).as_dict()

    def diagnostics_all(self, regions_in, regions_out):
        """Reductions of every lattice in one call: lists of (cx, cy, r_min, r_max).
        Returns a list of dicts (unstable lattices carry unstable = 1)."""
        _, ds = lb_batch_diagnostics_all(self.b, [lb_region(*r) for r in regions_in],
                                         [lb_region(*r) for r in regions_out])
        return [d.as_dict() for d in ds]

    def moments(self, i):
        torch = self.torch
        out = [torch.empty(self.shapes[i], dtype=torch.float32, device=self.device) for _ in range(3)]
        lb_batch_moments(self.b, i, *[o.data_ptr() for o in out])
        self.stream.synchronize()
        return tuple(out)

    def get_state(self, i, state_bytes):
        torch = self.torch
        buf = torch.empty(state_bytes, dtype=torch.uint8, device=self.device)
        lb_batch_get_state(self.b, i, buf.data_ptr())
        self.stream.synchronize()
        return buf


class Net:
    """The initialiser network on the current ROCm device (torch supplies the
    workspace, parameters and stream).  Features: [B][4] raw (a, T/T_c, R,
    nu_g/nu_l); outputs [B][128] log-density samples."""

    def __init__(self, theta0, mu, sd, max_batch=4096, stream=None, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbmp.Net needs a ROCm GPU")
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.max_batch = int(max_batch)
        theta0 = torch.as_tensor(theta0).to(device=self.device, dtype=torch.float32).contiguous()
        if theta0.numel() != LBML_PARAMS:
            raise ValueError(f"theta0 has {theta0.numel()} values, expected {LBML_PARAMS}")
        nbytes = lbml_workspace_bytes(self.max_batch)
        if nbytes == 0:
            raise ValueError("max_batch must be a positive multiple of 32")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)
        with torch.cuda.stream(self.stream):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            self.net = lbml_init(self.max_batch, self.workspace.data_ptr(), nbytes, theta0.data_ptr(), mu, sd,
                                 self.stream.cuda_stream)

    def close(self):
        net = getattr(self, "net", None)
        if net is not None:
            self.net = None
            self.stream.synchronize()
            lbml_destroy(net)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def _dev(self, t, cols):
        t = self.torch.as_tensor(t).to(device=self.device, dtype=self.torch.float32).contiguous()
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected [B][{cols}], got {tuple(t.shape)}")
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        return t

    def forward(self, x, base=None):
        """network(x) + base, [B][128] (base: [B][128] or None)."""
        x = self._dev(x, LBML_IN)
        base = None if base is None else self._dev(base, LBML_OUT)
        y = self.torch.empty((x.shape[0], LBML_OUT), dtype=self.torch.float32, device=self.device)
        lbml_forward(self.net, x.data_ptr(), 0 if base is None else base.data_ptr(), x.shape[0], y.data_ptr())
        self.stream.synchronize()
        return y

    def loss_grad(self, x, target, base=None):
        x, target = self._dev(x, LBML_IN), self._dev(target, LBML_OUT)
        base = None if base is None else self._dev(base, LBML_OUT)
        g = self.torch.empty(LBML_PARAMS, dtype=self.torch.float32, device=self.device)
        lbml_loss_grad(self.net, x.data_ptr(), 0 if base is None else base.data_ptr(), target.data_ptr(), x.shape[0],
                       self.loss_buf.data_ptr(), g.data_ptr())
        self.stream.synchronize()
        return float(self.loss_buf.item()), g

    def train_step(self, x, target, lr, base=None, sync=True):
        """x, target, base: device tensors already in place (no copies when they are)."""
        lbml_train_step(self.net, x.data_ptr(), 0 if base is None else base.data_ptr(), target.data_ptr(),
                        x.shape[0], lr, self.loss_buf.data_ptr())
        if sync:
            self.stream.synchronize()
            return float(self.loss_buf.item())
        return None

    def train_steps(self, x_all, target_all, idx, lr, base_all=None, loss=None):
        """len(lr) Adam steps replayed from a graph: step s on rows idx[s] of the device
        tensors x_all [rows][4], target_all [rows][128] and base_all [rows][128] (or
        None), learning rate lr[s]; idx: device int32 [steps][B], lr: device float32
        [steps]; loss: device float32 [steps] receiving each step's loss, or None."""
        steps, B = idx.shape
        for t, cols in ((x_all, LBML_IN), (target_all, LBML_OUT), (base_all, LBML_OUT)):
            if t is not None and (t.dim() != 2 or t.shape[1] != cols or t.dtype != self.torch.float32
                                  or not t.is_contiguous()):
                raise ValueError(f"expected a contiguous float32 [rows][{cols}] tensor")
        if (idx.dtype != self.torch.int32 or lr.dtype != self.torch.float32 or lr.numel() != steps
                or not idx.is_contiguous() or not lr.is_contiguous()):
            raise ValueError("idx must be a contiguous int32 [steps][B] tensor and lr a contiguous float32 [steps]")
        if loss is not None and (loss.dtype != self.torch.float32 or loss.numel() != steps
                                 or not loss.is_contiguous()):
            raise ValueError("loss must be a contiguous float32 [steps] tensor")
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        _check(load().lbml_train_steps(self.net, _vp(x_all.data_ptr()),
                                       _vp(0 if base_all is None else base_all.data_ptr()),
                                       _vp(target_all.data_ptr()), int(x_all.shape[0]), _vp(idx.data_ptr()),
                                       _vp(lr.data_ptr()), int(steps), int(B),
                                       _vp(0 if loss is None else loss.data_ptr())), "lbml_train_steps")

    def params(self):
        th = self.torch.empty(LBML_PARAMS, dtype=self.torch.float32, device=self.device)
        lbml_get_params(self.net, th.data_ptr())
        self.stream.synchronize()
        return th

    def set_params(self, theta):
        theta = self.torch.as_tensor(theta).to(device=self.device, dtype=self.torch.float32).contiguous()
        lbml_set_params(self.net, theta.data_ptr())
        self.stream.synchronize()


def profile_extract(rho, cx, cy, R, out=None, scratch=None, stream=0):
    """Least-squares profile [128] of a device density field [ny][nx] (torch tensor)."""
    import torch
    ny, nx = rho.shape
    if out is None:
        out = torch.empty(LBML_OUT, dtype=torch.float32, device=rho.device)
    need = lbml_profile_scratch_bytes(ny)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=rho.device)
    lbml_profile_extract(rho.data_ptr(), nx, ny, cx, cy, R, scratch.data_ptr(), need, out.data_ptr(), stream)
    return out


def profile_to_rho0(logrho, R, cx, cy, nx, ny, out=None, stream=0):
    """Device density field [ny][nx] of a profile (device tensor [128])."""
    import torch
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=logrho.device)
    lbml_profile_to_rho0(logrho.data_ptr(), R, cx, cy, nx, ny, out.data_ptr(), stream)
    return out


def profile_to_rho0_mass(logrho, R, cx, cy, nx, ny, mass, out=None, shift=None, stream=0):
    """Device density field [ny][nx] of a profile moved radially to carry `mass`;
    returns (field, shift tensor [2] = (delta, achieved mass))."""
    import torch
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=logrho.device)
    if shift is None:
        shift = torch.empty(2, dtype=torch.float64, device=logrho.device)
    lbml_profile_to_rho0_mass(logrho.data_ptr(), R, cx, cy, nx, ny, mass, shift.data_ptr(), out.data_ptr(), stream)
    return out, shift


def profile_levels(L, x, out=None, stream=0):
    """Inner and outer band means [B][2] (device float64) of device profiles L [B][128]
    around the radii x[:, 2] of device features x [B][4]."""
    import torch
    if out is None:
        out = torch.empty((L.shape[0], 2), dtype=torch.float64, device=L.device)
    lbml_profile_levels(L.data_ptr(), x.data_ptr(), L.shape[0], out.data_ptr(), stream)
    return out


def profile_anchor(L, x, target, stream=0):
    """Pin device profiles L [B][128] (in place) to the inner levels target [B]
    (device float64); radii from device features x [B][4]."""
    lbml_profile_anchor(L.data_ptr(), x.data_ptr(), target.data_ptr(), L.shape[0], stream)
    return L
