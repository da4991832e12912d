"""Learned droplet initialiser: training profiles produced by the lattice itself,
training and inference of the profile network, and the comparison of
learned starts against the tanh start of Eq. (31).

Every device computation runs in liblbmp.so (lattice steps, diagnostics,
profile fit and field, network forward / backward / Adam).  This module
sequences those calls and keeps the host-side bookkeeping: feature statistics,
the tanh base profile (the same Eq. (31) recipe the lattice starts from),
convergence detection on the recorded diagnostics.

Features: (a, T/T_c, R0, nu_g/nu_l).  Outputs: L_k = log rho(r_k),
r_k = R + (k - 63.5) / 2, predicted as tanh base + network correction.  The
training profiles are sampled around the relaxed droplet's equimolar radius
R = sqrt((M - rho_out N) / (pi (rho_in - rho_out))), not around R0: mass is
conserved, so where the interface settles is fixed by the start's mass, and at
inference the predicted profile is moved radially until it carries the tanh
start's mass.  The network then learns only the shape of the profile; the
position, which jumps with the lattice as R0 varies (the tanh start's mass is a
lattice sum), comes from the mass of the droplet at hand.

Convergence of one run (checked every `every` steps), against the values a
tanh-started run of the same droplet reaches at the end of the window:
  * spurious-current convergence: the first check after which the maximum
    velocity stays within 5 % of the reference's;
  * strict convergence: the same, and the Laplace pressure jump within 1 %.
A run that is outside those bounds at the last check does not converge in the
window (None).

Liquid level.  The network's 128 outputs each carry an independent error of
about 1e-3 in log density (the matrix products take bf16 operands), and the
density inside the droplet sets how far the start's pressure jump lies from the
relaxed one: an interior 1e-3 too dense puts the jump tens of per cent off, and
that error then relaxes over thousands of steps.  The interior level is
therefore predicted separately, by an FP64 linear model on a Chebyshev basis of
the features fitted to the training profiles' inner band means (relative to the
tanh base's), and the network's profile is pinned to it (lbml_profile_anchor:
affine in density, interior band made flat, interface and vapour kept).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import lbmp

U_TOL = 0.05
DP_TOL = 0.01
N_OUT = lbmp.LBML_OUT


def radii(R):
    return R + (np.arange(N_OUT, dtype=np.float64) - 63.5) * 0.5


def features(ws):
    return np.array([w.info["features"] for w in ws], dtype=np.float64)


def tanh_base(ws, W=5.0):
    """log of the Eq. (31) tanh start at the sample radii (the fallback profile)."""
    out = np.empty((len(ws), N_OUT))
    for i, w in enumerate(ws):
        rl, rg, R = w.info["rho_l"], w.info["rho_g"], w.info["R0"]
        d = radii(R) - R
        out[i] = np.log(0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh(2.0 * d / W))
    return out


def regions(w):
    """Inner disc d < R0/2 and outer region d >= R0 + 15 around the droplet centre."""
    c = (w.info["cx"], w.info["cy"])
    R = w.info["R0"]
    return (c[0], c[1], 0.0, 0.5 * R), (c[0], c[1], R + 15.0, math.inf)


def record(batch, ws, steps, every, log=None, tag=""):
    """Advance `steps` in chunks of `every`, recording max|u|, dp, rho_in, rho_out of
    every lattice after each chunk (column 0 = the initial state)."""
    rin, rout = zip(*[regions(w) for w in ws])
    nc = steps // every + 1
    rec = {k: np.zeros((len(ws), nc)) for k in ("U", "DP", "RHO_IN", "RHO_OUT")}
    t0 = time.time()
    for c in range(nc):
        if c:
            batch.step(every)
        ds = batch.diagnostics_all(rin, rout)
        rec["U"][:, c] = [d["max_u"] for d in ds]
        rec["DP"][:, c] = [d["dp"] for d in ds]
        rec["RHO_IN"][:, c] = [d["rho_in"] for d in ds]
        rec["RHO_OUT"][:, c] = [d["rho_out"] for d in ds]
        if log and (c % max(1, nc // 10) == 0 or c == nc - 1):
            log(f"{tag} step {c * every}/{steps}  {time.time() - t0:.1f} s")
    rec["unstable"] = np.array([bool(d["unstable"]) for d in ds])
    return rec


def n_conv(U, DP, u_ref, dp_ref, every, strict=False):
    """Per run: first step after which |U - u_ref| <= 5 % u_ref (and, if strict,
    |DP - dp_ref| <= 1 % |dp_ref|) holds at every later check; None if the last
    check fails."""
    ok = np.abs(U - u_ref[:, None]) <= U_TOL * u_ref[:, None]
    if strict:
        ok &= np.abs(DP - dp_ref[:, None]) <= DP_TOL * np.abs(dp_ref[:, None])
    out = []
    for row in ok:
        bad = np.nonzero(~row)[0]
        if len(bad) == 0:
            out.append(0)
        elif bad[-1] == len(row) - 1:
            out.append(None)
        else:
            out.append(int((bad[-1] + 1) * every))
    return out


def equimolar_radius(mass, rho_in, rho_out, sites):
    """Radius of the disc of density rho_in in a background rho_out that holds `mass`."""
    return math.sqrt(max(mass - rho_out * sites, 0.0) / (math.pi * (rho_in - rho_out)))


def relaxed_profiles(batch, ws, members, centres=None):
    """Least-squares profile of the current density field of batch lattices `members`
    (descriptions `ws`), sampled around radius centres[i] (default R0), [n][128]
    device tensor.  The fits run on the batch's stream, ordered after the moments
    they read."""
    import torch
    out = torch.empty((len(ws), N_OUT), dtype=torch.float32, device=batch.device)
    scratch = torch.empty(max(lbmp.lbml_profile_scratch_bytes(w.params["ny"]) for w in ws), dtype=torch.uint8,
                          device=batch.device)
    s = batch.stream.cuda_stream
    for i, (m, w) in enumerate(zip(members, ws)):
        rho = batch.moments(int(m))[0]
        R = w.info["R0"] if centres is None else float(centres[i])
        lbmp.profile_extract(rho, w.info["cx"], w.info["cy"], R, out=out[i], scratch=scratch, stream=s)
        rho.record_stream(batch.stream)
    batch.stream.synchronize()
    return out


def generate(ws, steps, every=1000, log=None):
    """Run every tanh-started lattice for `steps` and fit its relaxed profile.
    Returns (features [n][4], base [n][128], target [n][128], kept mask); lattices
    that went unstable are dropped."""
    import torch
    batch = lbmp.Batch([w.params for w in ws], [torch.from_numpy(w.rho0.astype(np.float32)) for w in ws])
    t0 = time.time()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        batch.step(n)
        done += n
        batch.stream.synchronize()
        if log:
            log(f"training runs: step {done}/{steps}  {time.time() - t0:.1f} s")
    rin, rout = zip(*[regions(w) for w in ws])
    diag = batch.diagnostics_all(rin, rout)
    kept = np.array([not d["unstable"] for d in diag])
    members = np.nonzero(kept)[0]
    keep = [ws[i] for i in members]
    centres = [equimolar_radius(diag[i]["mass"], diag[i]["rho_in"], diag[i]["rho_out"],
                                ws[i].params["nx"] * ws[i].params["ny"]) for i in members]
    prof = relaxed_profiles(batch, keep, members, centres).cpu().numpy().astype(np.float64)
    batch.close()
    finite = np.all(np.isfinite(prof), axis=1)
    kept[members[~finite]] = False
    keep = [w for w, f in zip(keep, finite) if f]
    return features(keep), tanh_base(keep), prof[finite], kept


def init_params(seed=1211):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, in the parameter layout
    of include/lbml.h."""
    rng = np.random.default_rng(seed)
    sizes = [lbmp.LBML_IN, lbmp.LBML_HIDDEN, lbmp.LBML_HIDDEN, lbmp.LBML_HIDDEN, N_OUT]
    parts = []
    for i in range(4):
        parts.append(rng.standard_normal(sizes[i + 1] * sizes[i]) * math.sqrt(2.0 / sizes[i]))
        parts.append(np.zeros(sizes[i + 1]))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == lbmp.LBML_PARAMS
    return theta


def schedule(n, steps, minibatch, lr, lr_min, seed):
    """Minibatch rows (int32 [steps][mb], drawn without replacement within each pass
    over the n rows, a new permutation per pass) and the cosine learning-rate decay
    from lr to lr_min (float32 [steps])."""
    import torch
    mb = min(minibatch, n // 32 * 32)
    if mb < 32:
        raise ValueError("need at least 32 training profiles")
    gen = torch.Generator(device="cpu").manual_seed(seed)
    order, pos = torch.randperm(n, generator=gen), 0
    idx = torch.empty((steps, mb), dtype=torch.int32)
    rates = np.empty(steps, dtype=np.float32)
    for k in range(steps):
        if pos + mb > n:
            order, pos = torch.randperm(n, generator=gen), 0
        idx[k] = order[pos:pos + mb].to(torch.int32)
        pos += mb
        rates[k] = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * k / max(1, steps - 1)))
    return idx, rates


def train(X, base, T, steps=3000, lr=1e-3, lr_min=1e-5, minibatch=512, seed=1211, log=None, chunk=1000):
    """Adam on the mean squared error of (network + base) against T with a cosine
    learning-rate decay from lr to lr_min; minibatches drawn without replacement
    within each pass over the data.  The steps run on the device in graph-replayed
    chunks (lbml_train_steps).  Then the FP64 level model of the interior is fitted.
    Returns (Initialiser, losses) with losses [(step, loss)] every 100 steps."""
    import torch
    n = X.shape[0]
    idx, rates = schedule(n, steps, minibatch, lr, lr_min, seed)
    mb = idx.shape[1]
    mu, sd = X.mean(0), X.std(0)
    sd = np.where(sd > 0, sd, 1.0)
    net = lbmp.Net(init_params(seed), mu, sd, max_batch=max(mb, 32))
    dev = net.device
    x = torch.from_numpy(X.astype(np.float32)).to(dev)
    b = torch.from_numpy(base.astype(np.float32)).to(dev)
    t = torch.from_numpy(T.astype(np.float32)).to(dev)
    idx_d = idx.to(dev)
    lr_d = torch.from_numpy(rates).to(dev)
    loss_d = torch.zeros(steps, dtype=torch.float32, device=dev)
    t0 = time.time()
    for s in range(0, steps, chunk):
        e = min(steps, s + chunk)
        net.train_steps(x, t, idx_d[s:e], lr_d[s:e], base_all=b, loss=loss_d[s:e])
        if log:
            log(f"train step {e - 1}/{steps} loss {float(loss_d[e - 1]):.3e} lr {rates[e - 1]:.2e}  "
                f"{time.time() - t0:.1f} s")
    all_losses = loss_d.cpu().numpy()
    losses = [(k, float(all_losses[k])) for k in range(steps) if k % 100 == 0 or k == steps - 1]
    return Initialiser(net, fit_level(net.device, X, base, T)), losses


@dataclass
class Initialiser:
    """The trained network and the level model of the droplet interior."""
    net: "lbmp.Net"
    level: "lbmp.lbml_level_model | None" = None

    def close(self):
        self.net.close()


def inner_levels(device, X, P):
    """Inner band means of profiles P [n][128] around the radii of features X (host
    arrays), computed by the library on `device`; float64 [n]."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    p = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).to(device)
    lev = lbmp.profile_levels(p, x, stream=torch.cuda.current_stream(device).cuda_stream)
    return lev[:, 0].cpu().numpy()


def fit_level(device, X, base, T):
    """Level model of the training profiles' inner level relative to the tanh base's."""
    return lbmp.lbml_level_fit(X, inner_levels(device, X, T) - inner_levels(device, X, base))


def predict(model, ws, anchored=True):
    """Predicted profiles [n][128] (device) for droplets described by workloads:
    network + tanh base, pinned to the level model's interior level when `anchored`
    (and the model has one)."""
    import torch
    net = model.net
    n = len(ws)
    pad = (n + 15) // 16 * 16
    X = np.zeros((pad, lbmp.LBML_IN))
    base = np.zeros((pad, N_OUT))
    X[:n], base[:n] = features(ws), tanh_base(ws)
    X[n:] = X[0]
    base[n:] = base[0]
    out = torch.empty((pad, N_OUT), dtype=torch.float32, device=net.device)
    for s in range(0, pad, net.max_batch // 16 * 16):
        e = min(pad, s + net.max_batch // 16 * 16)
        out[s:e] = net.forward(torch.from_numpy(X[s:e].astype(np.float32)),
                               torch.from_numpy(base[s:e].astype(np.float32)))
    if anchored and model.level is not None:
        target = inner_levels(net.device, X, base) + lbmp.lbml_level_eval(model.level, X)
        x = torch.from_numpy(X.astype(np.float32)).to(net.device)
        t = torch.from_numpy(target).to(net.device)
        lbmp.profile_anchor(out, x, t, stream=torch.cuda.current_stream(net.device).cuda_stream)
    return out[:n]


def learned_rho0(model, ws, anchored=True):
    """Initial density fields from the predicted profiles (device tensors), each moved
    radially so that it carries the mass of the tanh start of the same droplet (both
    starts then relax towards the same equilibrium).  Returns (fields, shifts)."""
    import torch
    prof = predict(model, ws, anchored)
    fields, shifts = [], []
    for i, w in enumerate(ws):
        mass = float(w.rho0.astype(np.float32).sum(dtype=np.float64))
        f, sh = lbmp.profile_to_rho0_mass(prof[i], w.info["R0"], w.info["cx"], w.info["cy"], w.params["nx"],
                                          w.params["ny"], mass)
        fields.append(f)
        shifts.append(sh)
    torch.cuda.synchronize()
    return fields, [float(s[0]) for s in torch.stack(shifts).cpu()]


def evaluate(model, ws, steps=30000, every=50, log=None, ablation=False):
    """Tanh and learned starts of the same droplets, advanced together in one batch.
    Returns per-droplet n_conv of both arms, the final-state errors of the learned
    arm against the tanh arm and the inference wall time.  With `ablation`, a third
    arm starts from the network's profile without the level anchoring; its summary
    is res["network_only"]."""
    import torch
    n = len(ws)
    t0 = time.time()
    rho_l, shifts = learned_rho0(model, ws)
    t_infer = time.time() - t0
    rho_t = [torch.from_numpy(w.rho0.astype(np.float32)) for w in ws]
    arms = [rho_t, rho_l]
    if ablation:
        arms.append(learned_rho0(model, ws, anchored=False)[0])
    # fallback to the tanh start where a prediction is not a usable density
    fallback = [i for i, f in enumerate(rho_l) if not bool(torch.isfinite(f).all() and (f > 0).all())]
    for arm in arms[1:]:
        for i in range(n):
            if not bool(torch.isfinite(arm[i]).all() and (arm[i] > 0).all()):
                arm[i] = rho_t[i]
    batch = lbmp.Batch([w.params for w in ws] * len(arms), [f for arm in arms for f in arm])
    rec = record(batch, list(ws) * len(arms), steps, every, log=log, tag="evaluation")
    batch.close()
    parts = [{k: v[a * n:(a + 1) * n] for k, v in rec.items()} for a in range(len(arms))]
    tanh = parts[0]
    u_ref, dp_ref = tanh["U"][:, -1], tanh["DP"][:, -1]
    bad = np.zeros(n, dtype=bool)
    for p in parts:
        bad |= p["unstable"]

    def compare(lrn):
        res = dict(unstable=bad.tolist(), dp_err=(lrn["DP"][:, -1] / dp_ref - 1.0).tolist(),
                   rho_in_err=(lrn["RHO_IN"][:, -1] / tanh["RHO_IN"][:, -1] - 1.0).tolist(),
                   rho_out_err=(lrn["RHO_OUT"][:, -1] / tanh["RHO_OUT"][:, -1] - 1.0).tolist(),
                   dp_err_start=(lrn["DP"][:, 0] / dp_ref - 1.0).tolist(), steps=steps, every=every)
        for crit, strict in (("u", False), ("strict", True)):
            res[f"n_tanh_{crit}"] = n_conv(tanh["U"], tanh["DP"], u_ref, dp_ref, every, strict)
            res[f"n_learned_{crit}"] = n_conv(lrn["U"], lrn["DP"], u_ref, dp_ref, every, strict)
        res["summary"] = {crit: summarise(res, crit) for crit in ("u", "strict")}
        return res

    res = compare(parts[1])
    res.update(infer_seconds=t_infer, fallback=fallback, shifts=shifts)
    if ablation:
        res["network_only"] = compare(parts[2])["summary"]
    return res, rec


def summarise(res, crit="u"):
    """Median steps to convergence of both arms and the median per-droplet ratio
    (tanh / learned), over droplets whose tanh run converges inside the window; a
    learned run that does not converge counts as the full window.  Final-state
    errors of the learned arm against the tanh arm over the same droplets."""
    steps, every = res["steps"], res["every"]
    nt, nl, bad = res[f"n_tanh_{crit}"], res[f"n_learned_{crit}"], res["unstable"]
    idx = [i for i in range(len(nt)) if not bad[i] and nt[i] is not None and nt[i] < steps - every]
    if not idx:
        return dict(converged=0, total=len(nt))
    a = np.array([nt[i] for i in idx], dtype=np.float64)
    b = np.array([steps if nl[i] is None else max(nl[i], every) for i in idx], dtype=np.float64)

    def med(key):
        return float(np.median(np.abs([res[key][i] for i in idx])))

    return dict(converged=len(idx), total=len(nt), unstable=int(np.sum(bad)),
                median_steps_tanh=float(np.median(a)), median_steps_learned=float(np.median(b)),
                ratio_of_medians=float(np.median(a) / np.median(b)), median_ratio=float(np.median(a / b)),
                learned_not_converged=int(sum(1 for i in idx if nl[i] is None)),
                median_abs_dp_err=med("dp_err"), max_abs_dp_err=float(np.max(np.abs([res["dp_err"][i] for i in idx]))),
                median_abs_rho_in_err=med("rho_in_err"), median_abs_rho_out_err=med("rho_out_err"),
                median_abs_dp_err_start=med("dp_err_start"))
