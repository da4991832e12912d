"""Learned-initialiser kernels through the C ABI against the FP64 oracles
(oracle/mlp.py with the same bf16 operand roundings, oracle/profile.py).

Tolerances:
  * matrix-core product on small integers: exact (every product and partial sum
    is an integer below 2^24, exact in bf16 inputs and FP32 accumulation);
  * forward outputs: relative Frobenius 2e-4 (FP32 accumulation over K <= 256 is
    about 1e-5; a bf16 rounding that lands on the other side of a tie moves one
    activation by 2^-8 relative, rarely);
  * gradients, per parameter block: relative Frobenius 1e-3;
  * Adam: FP32 arithmetic of the same update, 1e-6 lr absolute;
  * profile field: FP64 geometry on FP32 data, 1e-6 relative;
  * profile fit: FP64 normal equations summed in another order, FP32 result, 2e-6;
  * band levels: FP64 means of the same FP32 samples in another order, 1e-14;
  * anchoring: FP64 arithmetic rounded once to FP32 on both sides, 2 ulp (rtol
    2.5e-7); samples whose profile must stay unchanged, bitwise.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import level as OL
from oracle import mlp as M
from oracle import profile as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_1211_6932_amd.lbmp")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    B.load()
    yield


def bf16_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


@pytest.mark.parametrize("M_,N_,K_,a_t,b_t", [(16, 16, 32, False, False), (48, 80, 96, False, False),
                                              (48, 80, 96, True, False), (64, 32, 256, False, True),
                                              (32, 256, 64, True, True)])
def test_gemm_lane_layout_exact(M_, N_, K_, a_t, b_t):
    print(f"[gpu-case] gemm M={M_} N={N_} K={K_} a_t={a_t} b_t={b_t}", flush=True)
    rng = np.random.default_rng(M_ + N_ + K_)
    A = rng.integers(-8, 9, (M_, K_))
    Bm = rng.integers(-8, 9, (K_, N_))
    ref = (A @ Bm).astype(np.float64)
    # operand storage: A as [M][K] or transposed [K][M]; B as [K][N] or [N][K]
    a_dev = bf16_dev(A.T if a_t else A)
    b_dev = bf16_dev(Bm.T if b_t else Bm)
    sam, sak = (1, M_) if a_t else (K_, 1)
    sbk, sbn = (1, K_) if b_t else (N_, 1)
    ldc = N_ + 16
    C = torch.full((M_, ldc), -7.0, dtype=torch.float32, device="cuda")
    B.lbml_gemm_bf16(a_dev.data_ptr(), sam, sak, b_dev.data_ptr(), sbk, sbn, C.data_ptr(), ldc, M_, N_, K_, 0)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[:, :N_], ref)
    assert np.all(got[:, N_:] == -7.0)  # the padding columns of C are not touched


def features(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.choice([0.25, 0.5, 1.0], n), rng.uniform(0.5, 0.85, n), rng.uniform(10, 150, n),
                     rng.uniform(1, 15, n)], axis=1)


def standardise(X, mu, sd):
    return (X - mu) / sd


def theta32(seed):
    return M.init_params(seed).astype(np.float32).astype(np.float64)


def blocks(v):
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    return [v[offs[i]:offs[i + 1]] for i in range(len(offs) - 1)]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def make_net(theta, X, max_batch=256):
    mu, sd = X.mean(0), X.std(0) + 1e-3
    return B.Net(torch.from_numpy(theta.astype(np.float32)), mu, sd, max_batch=max_batch), mu, sd


@pytest.mark.parametrize("batch,with_base", [(16, False), (48, True), (256, False), (256, True), (512, True)])
def test_forward_matches_oracle(batch, with_base):
    print(f"[gpu-case] lbml forward B={batch} base={with_base}", flush=True)
    th = theta32(1)
    X = features(batch, 11)
    base = np.random.default_rng(21).normal(-3.0, 2.0, (batch, 128)).astype(np.float32) if with_base else None
    net, mu, sd = make_net(th, X, max_batch=max(256, batch))
    y = net.forward(torch.from_numpy(X.astype(np.float32)),
                    None if base is None else torch.from_numpy(base)).cpu().numpy().astype(np.float64)
    net.close()
    ref, _ = M.forward(th, standardise(X.astype(np.float32).astype(np.float64), mu, sd), bf16=True,
                       base=None if base is None else base.astype(np.float64))
    assert rel(y, ref) < 2e-4, rel(y, ref)


@pytest.mark.parametrize("batch,with_base", [(32, False), (96, True), (512, True)])
def test_gradients_match_oracle(batch, with_base):
    """Batch 512 with a base is the training minibatch of the full protocol."""
    print(f"[gpu-case] lbml gradients B={batch} base={with_base}", flush=True)
    th = theta32(2)
    X = features(batch, 12)
    T = np.random.default_rng(13).normal(-2.0, 1.0, (batch, 128)).astype(np.float32).astype(np.float64)
    base = np.random.default_rng(22).normal(-2.0, 1.0, (batch, 128)).astype(np.float32) if with_base else None
    net, mu, sd = make_net(th, X, max_batch=max(256, batch))
    loss, g = net.loss_grad(torch.from_numpy(X.astype(np.float32)), torch.from_numpy(T.astype(np.float32)),
                            None if base is None else torch.from_numpy(base))
    net.close()
    g = g.cpu().numpy().astype(np.float64)
    Xs = standardise(X.astype(np.float32).astype(np.float64), mu, sd)
    bb = None if base is None else base.astype(np.float64)
    loss_ref, g_ref = M.loss_and_grad(th, Xs, T, bf16=True, base=bb)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    for i, (gb, rb) in enumerate(zip(blocks(g), blocks(g_ref))):
        assert rel(gb, rb) < 1e-3, (M.SHAPES[i], rel(gb, rb))
    # the bf16 operand rounding itself stays a small perturbation of the FP64 gradient
    _, g64 = M.loss_and_grad(th, Xs, T, bf16=False, base=bb)
    assert rel(g, g64) < 3e-2


def test_adam_matches_oracle():
    print("[gpu-case] lbml adam", flush=True)
    th = theta32(3)
    X = features(64, 14)
    T = np.random.default_rng(15).normal(-2.0, 1.0, (64, 128))
    net, mu, sd = make_net(th, X)
    _, g = net.loss_grad(torch.from_numpy(X.astype(np.float32)), torch.from_numpy(T.astype(np.float32)))
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    p, m, v = th.copy(), np.zeros_like(th), np.zeros_like(th)
    for t in (1, 2, 3):  # the same stored gradient three times: exercises the bias corrections
        B.lbml_adam(net.net, lr)
        p, m, v = M.adam_step(p, m, v, g, t, lr)
    got = net.params().cpu().numpy().astype(np.float64)
    net.close()
    assert np.abs(got - p).max() < 1e-6 * lr + 2e-7 * np.abs(p).max()


def test_training_reduces_the_loss():
    """Fit tanh-profile targets (Eq. (31) shape, widths by a) with the device training step."""
    print("[gpu-case] lbml training", flush=True)
    X = features(256, 16)
    r = (np.arange(128) - 63.5) * 0.5
    T = np.empty((256, 128))
    for i, (a, tb, R, _) in enumerate(X):
        rl, rg = W.coexistence(tb)
        T[i] = np.log(W.tanh_profile(r, rl, rg, W=5.0 * math.sqrt(0.5 / a)))
    th = M.init_params(4)
    net, _, _ = make_net(th, X)
    x = torch.from_numpy(X.astype(np.float32)).cuda()
    t = torch.from_numpy(T.astype(np.float32)).cuda()
    first = net.train_step(x, t, 1e-3)
    for _ in range(400):
        net.train_step(x, t, 1e-3, sync=False)
    last = net.train_step(x, t, 1e-3)
    net.close()
    assert np.isfinite(last) and last < 0.02 * first, (first, last)


@pytest.mark.parametrize("with_base", [False, True])
def test_graph_replayed_training_equals_single_steps(with_base):
    """lbml_train_steps (one step captured into a HIP graph, replayed) against the same
    minibatches run one lbml_train_step at a time: parameters and every step's loss
    bitwise equal, over two consecutive calls (the schedule and Adam's bias correction
    carry over) with different learning rates per step."""
    print(f"[gpu-case] lbml graph-replayed training with_base={with_base}", flush=True)
    rows, B, steps = 200, 64, 37
    X = features(rows, 21)
    rng = np.random.default_rng(22)
    T = -1.0 + 0.3 * rng.standard_normal((rows, 128))
    base = 0.1 * rng.standard_normal((rows, 128)) if with_base else None
    idx = np.stack([rng.choice(rows, B, replace=False) for _ in range(2 * steps)]).astype(np.int32)
    lr = (1e-3 * (0.5 + rng.random(2 * steps))).astype(np.float32)
    th = M.init_params(7)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    x_all, t_all = dev(X), dev(T)
    b_all = None if base is None else dev(base)
    # one step at a time
    net1, _, _ = make_net(th, X, max_batch=B)
    loss1 = []
    for s in range(2 * steps):
        sel = torch.from_numpy(idx[s].astype(np.int64)).cuda()
        loss1.append(net1.train_step(x_all.index_select(0, sel), t_all.index_select(0, sel), float(lr[s]),
                                     base=None if b_all is None else b_all.index_select(0, sel)))
    p1 = net1.params().cpu().numpy()
    net1.close()
    # the same, graph-replayed, in two calls
    net2, _, _ = make_net(th, X, max_batch=B)
    idx_d = torch.from_numpy(idx).cuda()
    lr_d = torch.from_numpy(lr).cuda()
    loss2 = torch.full((2 * steps,), -1.0, dtype=torch.float32, device="cuda")
    net2.train_steps(x_all, t_all, idx_d[:steps], lr_d[:steps], base_all=b_all, loss=loss2[:steps])
    net2.train_steps(x_all, t_all, idx_d[steps:], lr_d[steps:], base_all=b_all, loss=loss2[steps:])
    p2 = net2.params().cpu().numpy()
    net2.close()
    np.testing.assert_array_equal(loss2.cpu().numpy(), np.array(loss1, dtype=np.float32))
    np.testing.assert_array_equal(p2, p1)


def test_graph_replayed_training_without_loss_output_and_with_no_steps():
    """loss=None leaves the loss-record kernel out of the captured graph: the parameters
    are bitwise those of the same steps with a loss output; steps = 0 changes nothing."""
    print("[gpu-case] lbml graph-replayed training, no loss output, zero steps", flush=True)
    rows, B, steps = 96, 32, 9
    X = features(rows, 31)
    T = -1.0 + 0.3 * np.random.default_rng(32).standard_normal((rows, 128))
    idx = np.stack([np.random.default_rng(33 + s).choice(rows, B, replace=False) for s in range(steps)])
    th = M.init_params(9)
    x_all = torch.from_numpy(X.astype(np.float32)).cuda()
    t_all = torch.from_numpy(T.astype(np.float32)).cuda()
    idx_d = torch.from_numpy(idx.astype(np.int32)).cuda()
    lr_d = torch.full((steps,), 1e-3, dtype=torch.float32, device="cuda")
    out = []
    for with_loss in (True, False):
        net, _, _ = make_net(th, X, max_batch=B)
        p0 = net.params().cpu().numpy()
        net.train_steps(x_all, t_all, idx_d[:0], lr_d[:0])
        assert np.array_equal(net.params().cpu().numpy(), p0)
        loss = torch.zeros(steps, dtype=torch.float32, device="cuda") if with_loss else None
        net.train_steps(x_all, t_all, idx_d, lr_d, loss=loss)
        out.append(net.params().cpu().numpy())
        net.close()
    np.testing.assert_array_equal(out[0], out[1])


def test_graph_replayed_training_rejects_bad_rows():
    print("[gpu-case] lbml graph-replayed training, out-of-range row", flush=True)
    X = features(64, 23)
    net, _, _ = make_net(M.init_params(8), X, max_batch=32)
    th0 = net.params().cpu().numpy()
    x_all = torch.from_numpy(X.astype(np.float32)).cuda()
    t_all = torch.zeros((64, 128), dtype=torch.float32, device="cuda")
    idx = torch.zeros((3, 32), dtype=torch.int32)
    idx[2, 5] = 64
    with pytest.raises(B.LbError):
        net.train_steps(x_all, t_all, idx.cuda(), torch.full((3,), 1e-3, device="cuda"))
    np.testing.assert_array_equal(net.params().cpu().numpy(), th0)
    net.close()


def test_profile_extract_matches_oracle():
    print("[gpu-case] lbml profile extract", flush=True)
    rl, rg = W.coexistence(0.6)
    rng = np.random.default_rng(5)
    # ragged sizes; centres off the lattice; small R (empty inner radii); wrap of the window
    for (nx, ny, cx, cy, R) in [(150, 124, 70.3, 60.8, 30.0), (97, 64, 10.0, 3.5, 12.0),
                                (256, 256, 127.5, 127.5, 70.0)]:
        rho = W.droplet_field(nx, ny, R, rl, rg, cx=cx, cy=cy) * np.exp(0.01 * rng.standard_normal((ny, nx)))
        rho = rho.astype(np.float32)
        r_dev = torch.from_numpy(rho).cuda()
        out = B.profile_extract(r_dev, cx, cy, R)
        again = B.profile_extract(r_dev, cx, cy, R)
        torch.cuda.synchronize()
        ref = P.extract(rho.astype(np.float64), cx, cy, R)
        got = out.cpu().numpy()
        # FP64 normal equations on both sides, different summation order; FP32 output
        assert np.abs(got - ref).max() <= 2e-6 * max(1.0, np.abs(ref).max()), (nx, ny)
        assert torch.equal(out, again)  # fixed reduction order: bitwise reproducible


def test_profile_to_rho0_matches_oracle():
    print("[gpu-case] lbml profile to rho0", flush=True)
    logrho = np.linspace(-0.7, -5.0, 128) + 0.05 * np.cos(np.arange(128))
    lr_dev = torch.from_numpy(logrho.astype(np.float32)).cuda()
    for (nx, ny, cx, cy, R) in [(256, 256, 127.5, 127.5, 50.0), (67, 301, 10.25, 290.0, 12.0)]:
        out = B.profile_to_rho0(lr_dev, R, cx, cy, nx, ny)
        torch.cuda.synchronize()
        ref = P.to_rho0(logrho.astype(np.float32).astype(np.float64), R, cx, cy, nx, ny)
        assert np.abs(out.cpu().numpy() / ref - 1).max() < 1e-6


def test_mass_matched_field_matches_oracle():
    print("[gpu-case] lbml profile to rho0 with mass", flush=True)
    R = 30.0
    r = R + (np.arange(128) - 63.5) * 0.5
    L = np.log(0.26 + 0.24 * np.tanh((R - r) / 2.5)).astype(np.float32)
    lr_dev = torch.from_numpy(L).cuda()
    for (nx, ny, cx, cy, dm) in [(128, 128, 63.5, 63.5, 40.0), (150, 97, 70.25, 40.5, -25.0)]:
        L64 = L.astype(np.float64)
        mass = P.to_rho0(L64, R, cx, cy, nx, ny).sum() + dm
        field, shift = B.profile_to_rho0_mass(lr_dev, R, cx, cy, nx, ny, mass)
        torch.cuda.synchronize()
        ref, delta = P.to_rho0_mass(L64, R, cx, cy, nx, ny, mass)
        got = shift.cpu().numpy()
        assert abs(got[0] - delta) < 1e-9, (got[0], delta)
        assert abs(got[1] / mass - 1.0) < 1e-12
        assert np.abs(field.cpu().numpy() / ref - 1).max() < 1e-6


def test_profile_round_trip_on_the_device():
    """extract(to_rho0(L)) = L for a profile in the model's span (up to the smoothness term)."""
    print("[gpu-case] lbml profile round trip", flush=True)
    R = 50.0
    r = R + (np.arange(128) - 63.5) * 0.5
    L = np.log(0.26 + 0.24 * np.tanh((R - r) / 3.0)).astype(np.float32)
    field = B.profile_to_rho0(torch.from_numpy(L).cuda(), R, 127.5, 127.5, 256, 256)
    back = B.profile_extract(field, 127.5, 127.5, R).cpu().numpy()
    assert np.abs(back - L).max() < 2e-5


def test_entry_points_reject_bad_batches():
    X = features(64, 17)
    net, _, _ = make_net(theta32(5), X, max_batch=64)
    x = torch.zeros((64, 4), dtype=torch.float32, device="cuda")
    y = torch.zeros((64, 128), dtype=torch.float32, device="cuda")
    L = B.load()
    assert L.lbml_forward(net.net, B._vp(x.data_ptr()), None, 8, B._vp(y.data_ptr())) == B.LB_EINVAL
    assert L.lbml_forward(net.net, B._vp(x.data_ptr()), None, 80, B._vp(y.data_ptr())) == B.LB_EINVAL
    assert L.lbml_loss_grad(net.net, B._vp(x.data_ptr()), None, B._vp(y.data_ptr()), 48, None, None) == B.LB_EINVAL
    assert L.lbml_adam(net.net, 1e-3) == B.LB_ESTATE  # no gradient yet
    net.close()


def _noisy_profiles(n, seed):
    """Droplet-like log profiles with per-sample noise of the network's size, at radii
    8..80 (small radii put part of the inner band at r_k < 0)."""
    rng = np.random.default_rng(seed)
    R = rng.uniform(8.0, 80.0, n)
    rl, rg = rng.uniform(0.3, 0.45, n), rng.uniform(0.002, 0.05, n)
    d = (np.arange(128) - 63.5) * 0.5
    s = 0.5 * (1.0 - np.tanh(2.0 * d[None, :] / rng.uniform(4.0, 8.0, (n, 1))))
    L = np.log(rg[:, None] + (rl - rg)[:, None] * s) + 1e-3 * rng.standard_normal((n, 128))
    x = np.c_[rng.choice([0.25, 0.5, 1.0], n), rng.uniform(0.5, 0.85, n), R, rng.uniform(1.0, 15.0, n)]
    return L.astype(np.float32), x.astype(np.float32)


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_profile_levels_match_oracle(n):
    print(f"[gpu-case] profile levels n={n}", flush=True)
    L, x = _noisy_profiles(n, 20 + n)
    got = B.profile_levels(torch.from_numpy(L).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    want = np.array([OL.levels(L[i].astype(np.float64), float(x[i, 2])) for i in range(n)])
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_profile_anchor_matches_oracle(n):
    print(f"[gpu-case] profile anchor n={n}", flush=True)
    L, x = _noisy_profiles(n, 40 + n)
    rng = np.random.default_rng(n)
    lev = np.array([OL.levels(L[i].astype(np.float64), float(x[i, 2]))[0] for i in range(n)])
    target = lev + rng.uniform(-3e-3, 3e-3, n)
    # unusable targets and a reversed map that would turn a sample negative: left alone
    if n > 4:
        target[1], target[2] = np.nan, np.inf
        L[3, 50] = np.log(0.6)
        target[3] = np.log(1e-5)
    Ld = torch.from_numpy(L).cuda()
    B.profile_anchor(Ld, torch.from_numpy(x).cuda(), torch.from_numpy(target).cuda())
    got = Ld.cpu().numpy()
    for i in range(n):
        want = OL.anchor(L[i].astype(np.float64), float(x[i, 2]), target[i]).astype(np.float32)
        if n > 4 and i in (1, 2, 3):
            np.testing.assert_array_equal(got[i], L[i])
            np.testing.assert_array_equal(want, L[i])
        else:
            np.testing.assert_allclose(got[i], want, rtol=2.5e-7, atol=0)
