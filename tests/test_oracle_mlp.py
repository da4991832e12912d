"""Pins of the FP64 MLP oracle (oracle/mlp.py): finite differences for the backward
pass, library routines for GELU, bfloat16 rounding and Adam.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def test_parameter_count():
    # 4*256 + 256 + 2 * (256*256 + 256) + 256*128 + 128
    assert M.N_PARAMS == 165760


def test_gelu_matches_library_exact_gelu():
    z = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    assert np.abs(M.gelu(z) - ref).max() < 1e-15
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.abs(M.gelu_prime(z) - fd).max() < 1e-8


def test_bf16_rounding_matches_library():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 3.0e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


@pytest.mark.parametrize("bf16", [False, True])
def test_backward_matches_finite_differences(bf16):
    """Central differences of the FP64 loss (bf16=False).  With bf16=True the same
    backward is compared against the FP64 one: the roundings only perturb it."""
    rng = np.random.default_rng(1)
    theta = M.init_params(seed=3) * 0.5
    X = rng.standard_normal((8, 4))
    T = rng.standard_normal((8, 128)) * 0.1
    loss, g = M.loss_and_grad(theta, X, T, bf16=False)
    if bf16:
        _, gb = M.loss_and_grad(theta, X, T, bf16=True)
        assert np.linalg.norm(gb - g) / np.linalg.norm(g) < 2e-2
        return
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 6) for i in range(len(offs) - 1)])
    h = 1e-6
    for j in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (M.loss_and_grad(tp, X, T)[0] - M.loss_and_grad(tm, X, T)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(g).max()), (j, fd, g[j])


def test_adam_matches_library():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    opt = torch.optim.Adam([p], lr=1e-3)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        theta, m, v = M.adam_step(theta, m, v, g, t, 1e-3)
    assert np.abs(theta - p.detach().numpy()).max() < 1e-12


def test_base_profile_shifts_outputs_not_gradients():
    """A base added to the outputs is the same as a target shifted by it."""
    rng = np.random.default_rng(5)
    theta = M.init_params(seed=6)
    X = rng.standard_normal((8, 4))
    T = rng.standard_normal((8, 128))
    base = rng.standard_normal((8, 128))
    y0, _ = M.forward(theta, X)
    y1, _ = M.forward(theta, X, base=base)
    assert np.array_equal(y1, y0 + base)
    l1, g1 = M.loss_and_grad(theta, X, T, base=base)
    l2, g2 = M.loss_and_grad(theta, X, T - base)
    assert abs(l1 - l2) < 1e-12 * l2 and np.abs(g1 - g2).max() < 1e-12 * np.abs(g2).max()
