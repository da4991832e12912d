"""The interaction stencil of nearest and next-nearest neighbours (LB_STENCIL_MULTIRANGE,
24 sites, Sec. III.B) on the GPU, through the C ABI, against the FP64 oracle.

Bounds as for the nearest-neighbour stencil: one step from the same state at every site
|d f*| <= 2e-6 max|f|; 1000 steps of a droplet max|d rho|/rho_l <= 1e-5 and max|d u| <=
1e-3 max|u| + 1e-7; launch shapes bitwise; a flat interface with sigma = 0 reaches the
Eq. (21) densities at epsilon = 10/31 (and the oracle's to 1e-5)."""
import numpy as np
import pytest

import workloads as W
from oracle import eos
from oracle import lbref as O
from oracle import post

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_1211_6932_amd.lbmp")

MR = 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    B.load()
    yield


def f32(a):
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def sim(params, rho0, ux0=None, uy0=None, strip_rows=0, band=0):
    t = lambda a: None if a is None else torch.from_numpy(f32(a))
    s = B.Sim(params, t(rho0), t(ux0), t(uy0))
    if strip_rows or band:
        s.set_launch(strip_rows=strip_rows, band=band)
    return s


def oracle(params, rho0, ux0=None, uy0=None):
    d = lambda a: None if a is None else f32(a).astype(np.float64)
    return O.State(O.Params(**params), d(rho0), d(ux0), d(uy0))


def state(s):
    return s.get_state().view(torch.float32).cpu().numpy().astype(np.float64).reshape(9, s.ny, s.nx)


def droplet(n=96, R0=20.0, bc=0, nx=None, ny=None):
    nx, ny = nx or n, ny or n
    p = dict(W.base_params(nx, ny, bc=bc), stencil=MR)
    rl, rg = W.coexistence(0.6)
    return p, W.droplet_field(nx, ny, R0, rl, rg, periodic_y=(bc == 0)), rl


@pytest.mark.parametrize("bc", [0, 1])
def test_initial_state_matches_oracle(bc):
    """The FP64 init kernel with the 24-site force (7 x 7 psi block)."""
    p, rho0, _ = droplet(bc=bc)
    rng = np.random.default_rng(2)
    ux0, uy0 = 0.01 * rng.standard_normal((2, 96, 96))
    print(f"[gpu-case] multirange init bc={bc}", flush=True)
    s, o = sim(p, rho0, ux0, uy0), oracle(p, rho0, ux0, uy0)
    assert np.abs(O.stream(O.Params(**p), state(s)) - o.f).max() <= 2e-8
    rho, ux, uy = (t.cpu().numpy().astype(np.float64) for t in s.moments())
    ro, uxo, uyo, *_ = o.moments()
    assert np.abs(rho - ro).max() <= 1e-7 and np.abs(ux - uxo).max() <= 1e-7 and np.abs(uy - uyo).max() <= 1e-7


CASES = [((96, 96), 0), ((90, 130), 1), ((67, 67), 0), ((3, 3), 0), ((3, 5), 1), ((70, 3), 0), ((3, 64), 1),
         ((125, 63), 1), ((61, 4), 0), ((6, 121), 1)]


@pytest.mark.parametrize("shape,bc", CASES)
def test_one_step_every_site_matches_oracle(shape, bc):
    """Tiles of 60 columns (two halo lanes a side), ragged widths and heights, widths
    below the stencil's reach (3, 4), walls and periodic."""
    ny, nx = shape
    rng = np.random.default_rng(nx * 1000 + ny)
    p, rho0, _ = droplet(bc=bc, nx=nx, ny=ny, R0=max(1.0, 0.25 * min(nx, ny)))
    rho0 = rho0 * (1 + 0.01 * rng.random(rho0.shape))
    ux0, uy0 = 0.01 * rng.standard_normal((2, ny, nx))
    print(f"[gpu-case] multirange one step shape={shape} bc={bc}", flush=True)
    s = sim(p, rho0, ux0, uy0, strip_rows=7)
    s.step(5)
    S5 = state(s)
    s.step(1)
    S6 = state(s)
    P = O.Params(**p)
    ref = O.collide_at(P, O.stream(P, S5), np.arange(nx * ny)).T.reshape(9, ny, nx)
    err = np.abs(S6 - ref).max()
    assert err <= 2e-6 * np.abs(ref).max(), err


def test_droplet_1000_steps_parity():
    """96 x 96 periodic droplet (a = 0.5, T = 0.6 T_c, sigma = 0.11, R0 = 20), FP32 GPU
    against the FP64 oracle after 1000 steps: the gate of the nearest-neighbour stencil."""
    p, rho0, rl = droplet()
    print("[gpu-case] multirange parity 1000 steps", flush=True)
    s, o = sim(p, rho0), oracle(p, rho0)
    s.step(1000)
    s.check()
    o.step(1000)
    rho, ux, uy = (t.cpu().numpy().astype(np.float64) for t in s.moments())
    ro, uxo, uyo, *_ = o.moments()
    drho = np.abs(rho - ro).max() / rl
    du = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max())
    umax = np.sqrt(uxo ** 2 + uyo ** 2).max()
    print(f"multirange: max|drho|/rho_l = {drho:.3e}  max|du| = {du:.3e}  max|u| = {umax:.3e}")
    assert drho <= 1e-5
    assert du <= 1e-3 * umax + 1e-7


@pytest.mark.parametrize("bc", [0, 1])
def test_launch_shapes_are_bitwise_equal(bc):
    p, rho0, _ = droplet(bc=bc, nx=130, ny=77, R0=18.0)
    print(f"[gpu-case] multirange launch shapes bc={bc}", flush=True)
    ref = None
    for rows, band in ((0, 0), (1, 1), (2, 3), (5, 1), (9, 2), (40, 1)):
        s = sim(p, rho0, strip_rows=rows, band=band)
        s.step(37)
        st = state(s)
        s.close()
        if ref is None:
            ref = st
        assert np.array_equal(st, ref), (rows, band)


def test_flat_interface_follows_eq21_at_ten_over_thirty_one():
    """sigma = 0, T = 0.85 T_c, a = 0.5: the GPU's flat interface matches the oracle's bulk
    densities and the Eq. (21) solution at epsilon = 10/31."""
    nx, ny, tb = 4, 200, 0.85
    p = dict(W.base_params(nx, ny, a=0.5, t_over_tc=tb, sigma=0.0, nu_l=0.1, nu_g=0.1), stencil=MR)
    rl, rg = W.coexistence(tb)
    rho0 = W.slab_field(nx, ny, ny / 2, rl, rg)
    print("[gpu-case] multirange flat interface", flush=True)
    s, o = sim(p, rho0), oracle(p, rho0)
    s.step(30000)
    s.check()
    o.step(30000)
    r = s.moments()[0].cpu().numpy().astype(np.float64)[:, 0]
    ro = o.moments()[0][:, 0]
    tl, tg = eos.mechanical_stability(p["T"], 0.5, 10.0 / 31.0)
    print(f"GPU {r[ny // 2]:.7f} {r[0]:.7e}  oracle {ro[ny // 2]:.7f} {ro[0]:.7e}  Eq. (21) {tl:.7f} {tg:.7e}")
    assert abs(r[ny // 2] / ro[ny // 2] - 1) <= 1e-5 and abs(r[0] / ro[0] - 1) <= 1e-5
    assert r[ny // 2] == pytest.approx(tl, rel=1e-3) and r[0] == pytest.approx(tg, rel=1e-2)


def test_diagnostics_are_the_pressure_of_the_device_densities():
    """The diagnostics pass with the 24-site stencil: region pressures equal the host's FP64
    Eq. (30) of the device's own densities (1e-12), mass equals the oracle's."""
    p, rho0, _ = droplet()
    print("[gpu-case] multirange diagnostics", flush=True)
    s, o = sim(p, rho0), oracle(p, rho0)
    s.step(200)
    o.step(200)
    c = 47.5
    d = s.diagnostics(c, c, 10.0 + 1e-12, 35.0)
    rg = s.moments()[0].cpu().numpy().astype(np.float64)
    hp = post.laplace(rg, p, 20.0)
    assert d["p_in"] == pytest.approx(hp["p_in"], rel=1e-12)
    assert d["p_out"] == pytest.approx(hp["p_out"], rel=1e-12)
    assert d["mass"] == pytest.approx(o.f.sum(), rel=1e-6)


def test_unsupported_combinations_are_rejected():
    """The 24-site stencil runs with FP32 storage on single lattices."""
    p, rho0, _ = droplet()
    for store in ("f16", "f16local", "f16dest"):
        assert B.lb_validate_params(B.make_params(p, store, 0.4)) == B.LB_EINVAL
    q = B.make_params(p)
    assert B.lb_validate_params(q) == B.LB_OK
    assert B.lb_batch_workspace_bytes((B.lb_params * 1)(q), 1) == 0
    q.stencil = 2
    assert B.lb_validate_params(q) == B.LB_EINVAL
