"""C ABI checks that need no GPU: the library loads, exports every function the
header declares, and the pure host functions validate and size correctly."""
import ctypes
import os
import re
import subprocess

import pytest

import workloads as W
from paper_1211_6932_amd import lbmp as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbmp.h", "lbml.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(lb\w*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lb_init", "lb_step", "lb_moments", "lb_diagnostics", "lb_destroy", "lb_batch_init",
                 "lb_batch_diagnostics_all", "lbml_init", "lbml_forward", "lbml_train_step",
                 "lbml_profile_to_rho0"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(B.EXPORTS) <= exported


def test_struct_layouts_match_header():
    # lb_params: 4 int32 + 15 doubles + 2 int32 + 1 double; lb_diag: 11 doubles + 2 int32 + int64
    assert ctypes.sizeof(B.lb_params) == 16 + 15 * 8 + 8 + 8
    assert ctypes.sizeof(B.lb_diag) == 11 * 8 + 8 + 8
    assert ctypes.sizeof(B.lb_region) == 32


def good():
    return B.make_params(W.stationary_droplet(n=128).params)


def test_validate_accepts_paper_parameters():
    assert B.lb_validate_params(good()) == B.LB_OK
    sp = W.splash(nx=64, ny=32).params
    assert B.lb_validate_params(B.make_params(sp)) == B.LB_OK
    for st in ("f16", "bf16"):
        assert B.lb_validate_params(B.make_params(sp, st, 0.47)) == B.LB_OK


@pytest.mark.parametrize("field,value", [
    ("nx", 2), ("ny", 0), ("nx", (1 << 20) + 1), ("bc", 2), ("store", 6), ("store", -1), ("b", 0.0), ("T", -1.0),
    ("G", 0.0), ("G", 1.0), ("sigma", -0.1), ("s_e", 0.0), ("s_e", 2.0), ("s_q", 2.5),
    ("s_rho", -1.0), ("s_j", 2.0), ("nu_l", 0.0), ("nu_g", -0.1), ("a", float("nan")),
    ("R", 0.0), ("T", float("inf")), ("psi_form", 2), ("psi_form", -1), ("psi_eps", float("nan")),
])
def test_validate_rejects(field, value):
    p = good()
    setattr(p, field, value)
    assert B.lb_validate_params(p) == B.LB_EINVAL
    assert B.lb_last_error() != ""
    assert B.lb_workspace_bytes(p) == 0
    assert B.lb_state_bytes(p) == 0


def test_validate_eq23_pseudopotential():
    """LB_PSI_SS (Eq. 23) needs G < 0 and psi_eps >= 0; the Carnahan-Starling constants
    are then unused and not checked."""
    p = B.make_params(W.ss_params(64, 64, -2.7, 1.0, sigma=0.023))
    assert p.psi_form == B.LB_PSI_SS
    assert B.lb_validate_params(p) == B.LB_OK
    p.b, p.T, p.R = 0.0, 0.0, 0.0
    assert B.lb_validate_params(p) == B.LB_OK
    for field, value in (("psi_eps", -0.5), ("G", 0.5)):
        q = B.make_params(W.ss_params(64, 64, -2.7, 1.0))
        setattr(q, field, value)
        assert B.lb_validate_params(q) == B.LB_EINVAL
    # lattices of one batch share the pseudopotential form
    a = B.make_params(W.stationary_droplet(n=64).params)
    b = B.make_params(W.ss_params(64, 64, -2.7, 1.0))
    assert B.lb_batch_workspace_bytes((B.lb_params * 2)(a, b), 2) == 0
    assert B.lb_batch_workspace_bytes((B.lb_params * 2)(b, b), 2) > 0


def test_sizes():
    p = good()
    assert B.lb_state_bytes(p) == 9 * 128 * 128 * 4
    ws = B.lb_workspace_bytes(p)
    assert ws >= 2 * 9 * 128 * 128 * 4 and ws % 256 == 0
    p.store = B.LB_STORE_F16_OFFSET
    assert B.lb_state_bytes(p) == 9 * 128 * 128 * 2
    p.store = B.LB_STORE_F16_LOCAL  # 16-bit offsets plus the FP32 site densities
    assert B.lb_state_bytes(p) == 9 * 128 * 128 * 2 + 128 * 128 * 4
    assert B.lb_workspace_bytes(p) >= 2 * 11 * 128 * 128 * 2
    # population rows are packed (pitch = nx): two buffers of 9 x 5 x 67 floats plus the
    # flag, result and diagnostics-partial blocks (< 2 KiB here), each 256-byte aligned
    p2 = good()
    p2.nx, p2.ny = 67, 5
    packed = 2 * 9 * 5 * 67 * 4
    assert packed <= B.lb_workspace_bytes(p2) <= packed + 2048 + 3 * 256
    # the local-density encodings round the pitch to even (4-byte aligned FP32 densities)
    p2.store = B.LB_STORE_F16_LOCAL
    assert B.lb_workspace_bytes(p2) >= 2 * 11 * 5 * 68 * 2


def test_host_side_errors_need_no_gpu():
    L = B.load()
    p = good()
    ctx = ctypes.c_void_p()
    # NULL out pointer, NULL workspace, bad params: rejected before any device work
    assert L.lb_init(None, ctypes.byref(p), None, 0, None, None, None, None) == B.LB_EINVAL
    assert L.lb_init(ctypes.byref(ctx), ctypes.byref(p), None, 0, None, None, None, None) == B.LB_EINVAL
    p.nx = 1
    assert L.lb_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(256), 1 << 30,
                     ctypes.c_void_p(256), None, None, None) == B.LB_EINVAL
    p = good()
    assert L.lb_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(256 + 8), 1 << 30,
                     ctypes.c_void_p(256), None, None, None) == B.LB_EINVAL  # misaligned
    assert L.lb_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(256), 16,
                     ctypes.c_void_p(256), None, None, None) == B.LB_ENOMEM
    assert L.lb_step(None, 1) == B.LB_EINVAL
    assert L.lb_moments(None, None, None, None) == B.LB_EINVAL
    assert L.lb_check(None) == B.LB_EINVAL
    assert L.lb_time(None) == -1
    assert L.lb_destroy(None) == B.LB_OK
    assert L.lb_copy_probe(None, None, 16, None) == B.LB_EINVAL


def test_batch_workspace_sizing_is_pure_host():
    a = B.make_params(W.stationary_droplet(n=64).params)
    b = B.make_params(W.stationary_droplet(n=100).params)
    arr = (B.lb_params * 2)(a, b)
    total = B.lb_batch_workspace_bytes(arr, 2)
    assert total >= B.lb_workspace_bytes(a) + B.lb_workspace_bytes(b)
    assert B.lb_batch_workspace_bytes(arr, 0) == 0
    b.bc = 1  # lattices of one batch share the boundary type
    assert B.lb_batch_workspace_bytes((B.lb_params * 2)(a, b), 2) == 0


def test_learned_initialiser_host_checks():
    L = B.load()
    vp = ctypes.c_void_p
    assert B.lbml_workspace_bytes(0) == 0 and B.lbml_workspace_bytes(48) == 0 and B.lbml_workspace_bytes(-32) == 0
    ws = B.lbml_workspace_bytes(64)
    assert ws > 4 * B.LBML_PARAMS * 4 and ws % 256 == 0
    assert B.lbml_workspace_bytes(128) > ws
    net = vp()
    mu = (ctypes.c_double * 4)(0, 0, 0, 0)
    sd = (ctypes.c_double * 4)(1, 1, 1, 1)
    bad_sd = (ctypes.c_double * 4)(1, 0, 1, 1)
    assert L.lbml_init(None, 64, vp(256), ws, vp(256), mu, sd, None) == B.LB_EINVAL
    assert L.lbml_init(ctypes.byref(net), 48, vp(256), ws, vp(256), mu, sd, None) == B.LB_EINVAL
    assert L.lbml_init(ctypes.byref(net), 64, vp(264), ws, vp(256), mu, sd, None) == B.LB_EINVAL
    assert L.lbml_init(ctypes.byref(net), 64, vp(256), ws - 256, vp(256), mu, sd, None) == B.LB_ENOMEM
    assert L.lbml_init(ctypes.byref(net), 64, vp(256), ws, vp(256), mu, bad_sd, None) == B.LB_EINVAL
    assert L.lbml_init(ctypes.byref(net), 64, vp(256), ws, None, mu, sd, None) == B.LB_EINVAL
    assert B.lb_last_error() != ""
    assert L.lbml_forward(None, vp(256), None, 16, vp(256)) == B.LB_EINVAL
    assert L.lbml_loss_grad(None, vp(256), None, vp(256), 32, None, None) == B.LB_EINVAL
    assert L.lbml_adam(None, 1e-3) == B.LB_EINVAL
    assert L.lbml_destroy(None) == B.LB_OK
    assert L.lbml_gemm_bf16(vp(256), 32, 1, vp(256), 16, 1, vp(256), 16, 16, 16, 48, None) == B.LB_EINVAL
    assert L.lbml_gemm_bf16(vp(256), 32, 1, vp(256), 16, 1, vp(256), 8, 16, 16, 32, None) == B.LB_EINVAL
    sb = B.lbml_profile_scratch_bytes(64)
    assert sb == 3 * 64 * 128 * 8 and B.lbml_profile_scratch_bytes(1) == 0
    assert L.lbml_profile_extract(vp(256), 1, 64, 0.0, 0.0, 10.0, vp(256), sb, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_extract(vp(256), 64, 64, float("nan"), 0.0, 10.0, vp(256), sb, vp(256),
                                  None) == B.LB_EINVAL
    assert L.lbml_profile_extract(vp(256), 64, 64, 0.0, 0.0, 10.0, vp(256), sb - 8, vp(256), None) == B.LB_ENOMEM
    assert L.lbml_profile_extract(vp(256), 64, 64, 0.0, 0.0, 10.0, None, sb, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_to_rho0(vp(256), -1.0, 0.0, 0.0, 64, 64, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_to_rho0(None, 10.0, 0.0, 0.0, 64, 64, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_to_rho0_mass(vp(256), 10.0, 0.0, 0.0, 64, 64, 100.0, None, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_to_rho0_mass(vp(256), 10.0, 0.0, 0.0, 64, 64, -1.0, vp(256), vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_to_rho0_mass(vp(256), 10.0, 0.0, 0.0, 64, 64, 100.0, vp(260), vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_levels(vp(256), vp(256), 0, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_levels(vp(256), vp(256), 4, vp(260), None) == B.LB_EINVAL
    assert L.lbml_profile_levels(None, vp(256), 4, vp(256), None) == B.LB_EINVAL
    assert L.lbml_profile_anchor(vp(256), vp(256), vp(256), (1 << 20) + 1, None) == B.LB_EINVAL
    assert L.lbml_profile_anchor(vp(256), vp(256), vp(252), 4, None) == B.LB_EINVAL
    assert L.lbml_profile_anchor(vp(256), None, vp(256), 4, None) == B.LB_EINVAL


def _level_features(n, seed, a_values=(0.25, 0.5, 1.0)):
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.c_[rng.choice(a_values, n), rng.uniform(0.5, 0.85, n), rng.uniform(25.0, 77.0, n),
                 rng.uniform(1.0, 15.0, n)]


@pytest.mark.parametrize("n, a_values", [(3000, (0.25, 0.5, 1.0)), (600, (0.5,)), (40, (0.25, 1.0))])
def test_level_fit_matches_the_oracle(n, a_values):
    """The library's host Householder fit against the oracle's least squares on the
    same stacked ridge system: full rank, a feature with one value, fewer rows than
    terms."""
    import numpy as np
    from oracle import level as OL
    x = _level_features(n, 11, a_values)
    y = 1e-3 * np.sin(5.0 * x[:, 1]) * (1.0 + x[:, 0]) + 0.03 / x[:, 2] + 1e-4 * x[:, 3]
    m = B.lbml_level_fit(x, y)
    lo, hi, coef = OL.fit(x, y)
    np.testing.assert_array_equal(np.array(m.lo), lo)
    np.testing.assert_array_equal(np.array(m.hi), hi)
    scale = np.max(np.abs(coef))
    np.testing.assert_allclose(np.array(m.coef), coef, rtol=0, atol=1e-8 * scale)
    xe = _level_features(200, 12, a_values)
    np.testing.assert_allclose(B.lbml_level_eval(m, xe), OL.evaluate((lo, hi, coef), xe), rtol=0, atol=1e-12)


def test_level_fit_and_eval_reject_bad_input():
    import numpy as np
    L = B.load()
    x = _level_features(50, 3)
    y = np.zeros(50)
    m = B.lbml_level_fit(x, y)
    bad = x.copy()
    bad[7, 2] = 0.0
    for xx, yy in ((bad, y), (x, np.full(50, np.nan))):
        with pytest.raises(B.LbError):
            B.lbml_level_fit(xx, yy)
    with pytest.raises(B.LbError):
        B.lbml_level_eval(m, bad)
    dp = ctypes.POINTER(ctypes.c_double)
    assert L.lbml_level_fit(None, None, 10, None) == B.LB_EINVAL
    assert L.lbml_level_fit(x.ctypes.data_as(dp), y.ctypes.data_as(dp), 0, ctypes.byref(m)) == B.LB_EINVAL
    assert L.lbml_level_fit(x.ctypes.data_as(dp), y.ctypes.data_as(dp), 262145, ctypes.byref(m)) == B.LB_EINVAL
    assert L.lbml_level_eval(ctypes.byref(m), None, 0, None) == B.LB_OK
    assert L.lbml_level_eval(ctypes.byref(m), x.ctypes.data_as(dp), -1, y.ctypes.data_as(dp)) == B.LB_EINVAL


def test_headers_are_plain_c(tmp_path):
    """include/*.h declare a C ABI: a C99 translation unit that includes both headers and
    links every declared function (by taking its address) compiles with -pedantic and no
    warnings, and the struct sizes seen by C equal those of the ctypes binding."""
    names = declared_functions()
    src = tmp_path / "abi.c"
    src.write_text(
        '#include <stdio.h>\n#include "lbmp.h"\n#include "lbml.h"\n'
        "int main(void) {\n"
        + "".join(f"    (void)&{n};\n" for n in names)
        + '    printf("%zu %zu %zu %zu\\n", sizeof(lb_params), sizeof(lb_diag), sizeof(lb_region),'
          " sizeof(lbml_level_model));\n"
        "    return 0;\n}\n")
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe), "-L", os.path.dirname(B.LIB_PATH), "-llbmp",
                    f"-Wl,-rpath,{os.path.dirname(B.LIB_PATH)}"], check=True, capture_output=True, text=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert sizes == [ctypes.sizeof(B.lb_params), ctypes.sizeof(B.lb_diag), ctypes.sizeof(B.lb_region),
                     ctypes.sizeof(B.lbml_level_model)]
