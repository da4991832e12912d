"""The allocation-free entry point lbml_profile_extract_noalloc (static device scratch)
against lbml_profile_extract (caller's scratch), through the C ABI: bitwise equal on
two calls in a row, the second with a smaller lattice (the static array keeps the first
call's partials, which the second must not read); ny beyond the static limit is
rejected before any launch."""
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


def field(nx, ny, R, tb=0.6):
    rl, rg = W.coexistence(tb)
    rng = np.random.default_rng(nx + ny)
    rho = W.droplet_field(nx, ny, R, rl, rg) * (1.0 + 0.01 * rng.random((ny, nx)))
    return torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float32)).cuda()


def test_noalloc_profile_extract_equals_the_scratch_version():
    stream = torch.cuda.current_stream().cuda_stream
    for nx, ny, R in ((300, 256, 60.0), (90, 70, 21.5)):  # second call smaller
        print(f"[gpu-case] no-alloc profile extract {nx}x{ny}", flush=True)
        rho = field(nx, ny, R)
        cx, cy = (nx - 1) / 2.0 + 0.3, (ny - 1) / 2.0 - 0.2
        need = B.lbml_profile_scratch_bytes(ny)
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
        ref = torch.empty(B.LBML_OUT, dtype=torch.float32, device="cuda")
        got = torch.full((B.LBML_OUT,), float("nan"), dtype=torch.float32, device="cuda")
        B.lbml_profile_extract(rho.data_ptr(), nx, ny, cx, cy, R, scratch.data_ptr(), need, ref.data_ptr(), stream)
        B.lbml_profile_extract_noalloc(rho.data_ptr(), nx, ny, cx, cy, R, got.data_ptr(), stream)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(r))
        assert np.array_equal(r, g), np.abs(r - g).max()
    with pytest.raises(B.LbError) as e:
        B.lbml_profile_extract_noalloc(rho.data_ptr(), nx, 2049, cx, cy, R, got.data_ptr(), stream)
    assert e.value.status == B.LB_EINVAL and "2048" in B.lb_last_error()
