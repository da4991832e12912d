"""The splash case at its own size (2048 x 1024, walls in y, x periodic, a = 0.25,
T = 0.45 T_c, R = 100, film 20, U = 0.05, nu_g = 15 nu_l), through the C ABI.

The full 20,000-step runs at Re = 40, 200 and 1000 are `bench.py --workload splash1k`;
here a shorter stretch of the impact checks what a run must keep: no unstable site, and
the FP64 sum of the stored FP32 densities constant to 1e-6 (storage rounding only:
Eqs. (5) and (6) conserve mass exactly, including the bounce-back walls)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_1211_6932_amd.lbmp")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    B.load()
    yield


@pytest.mark.parametrize("Re", [200, 1000])
def test_splash_2048x1024_stays_stable_and_keeps_its_mass(Re):
    w = W.splash(scale=1, Re=Re)
    print(f"[gpu-case] splash 2048x1024 Re={Re}, 4000 steps", flush=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32)))
    s = B.Sim(w.params, t(w.rho0), t(w.ux0), t(w.uy0))
    c = (w.params["nx"] / 2.0, w.info["film"] + w.info["R"] + 5.0)
    d0 = s.diagnostics(c[0], c[1], 1.0, 2.0)
    drift = []
    for _ in range(4):
        s.step(1000)
        d = s.diagnostics(c[0], c[1], 1.0, 2.0)  # raises on an unstable site
        drift.append(d["mass"] / d0["mass"] - 1.0)
    print(f"Re={Re}: mass drift {drift}, max|u| {d['max_u']:.4f}")
    assert np.abs(drift).max() <= 1e-6
    # the droplet has hit the film by step 4000 (gap 5 + the film's tanh width at U = 0.05)
    rho = s.moments()[0].cpu().numpy()
    assert rho[int(w.info["film"]) + 3, :].max() > 0.5 * w.info["rho_l"]
    s.close()
