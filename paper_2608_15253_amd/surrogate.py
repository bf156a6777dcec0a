"""Learned demag operator for 128 x 128 films: training data produced by the
method itself, training with the library's own network kernels, and the
measured gain of RK45 with learned stages over plain FP32 RK45.

Everything numeric runs in libmmx: trajectories (mmx_heun), labels (the exact
demag field from mmx_field), network forward/backward/Adam (mmx_fno_*) and the
integrations (mmx_rk45, mmx_rk45_surrogate).  Python only orders the calls,
slices device buffers and times them.

Data (an extension of the paper, which has no learned part): snapshots of
stochastic Heun trajectories of 4 nm-cell films (Ms 8e5 A/m, open boundaries)
in three styles -- thermal switching of a perpendicular film (from +z, field
against it, 300 K), Neel-skyrmion films with interfacial DMI (seeded skyrmion
states, 50 K) and relaxation of random states into domain patterns (0 K).
Initial-state seeds are 5e6 + k.  Targets are h = H_demag / Ms, learned as the
residual on the local thin-film part: t = h + (0, 0, m_z).

Run ``python -m paper_2608_15253_amd.surrogate --out <report.json>``.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

import paper_2608_15253_amd as mmx
from workloads import neel_skyrmions, random_unit, replica_seeds, uniform

MS = 8.0e5
CELL = (4e-9, 4e-9, 4e-9)
SEED0 = 5_000_000


@dataclass
class Style:
    name: str
    A: float = 1.3e-11
    alpha: float = 0.1
    Ku: float = 0.0
    D: float = 0.0
    B: tuple = (0.0, 0.0, 0.0)
    T: float = 0.0
    init: str = "uniform"
    dt: float = 2e-14
    extra: dict = field(default_factory=dict)


STYLES = [
    Style("switching", alpha=0.1, Ku=5e5, B=(0.0, 0.0, -0.15), T=300.0, init="uniform"),
    Style("skyrmions", alpha=0.3, Ku=6e5, D=3e-3, B=(0.0, 0.0, 0.1), T=50.0, init="skyrmions"),
    Style("domains", alpha=0.5, Ku=5e5, D=2e-3, T=0.0, init="random"),
]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def initial_states(style: Style, n, R, seed):
    nx, ny, _ = n
    if style.init == "uniform":
        return uniform(n, (0.0, 0.0, 1.0), replicas=R)
    if style.init == "random":
        return random_unit(n, seed=seed, replicas=R)
    out = np.empty((R, 3, 1, ny, nx))
    rng = np.random.default_rng(seed)
    for r in range(R):
        count = int(rng.integers(1, 7))
        m, _, _ = neel_skyrmions(n, CELL, count, 8e-9, 25e-9, seed=seed + 1 + r, width=4e-9,
                                 gap=12e-9, periodic=False)
        out[r] = m
    return out


def _film_ctx(n, R, style: Style, prec=mmx.MMX_F32, terms=None):
    ctx = mmx.mmx_create([mmx.make_group(n, CELL, replicas=R)], prec)
    mmx.mmx_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
    mmx.mmx_set_material(ctx, 0, Ms=MS, A=style.A, alpha=style.alpha, Ku=style.Ku, D=style.D)
    mmx.mmx_set_field(ctx, 0, style.B)
    if terms is not None:
        mmx.mmx_set_terms(ctx, terms)
    mmx.mmx_build_demag(ctx)
    return ctx


def generate(n=(128, 128, 1), snapshots=20000, replicas=256, every=500, seed0=SEED0,
             styles=STYLES, log=print):
    """Snapshots m (S, 3, H, W) and residual targets t (S, 3, H, W) on the GPU.
    Consecutive entries belong to different replicas (time-major order), so
    contiguous batches mix trajectories without a gather."""
    nx, ny, _ = n
    S_total = snapshots
    per_style = [S_total // len(styles) + (1 if i < S_total % len(styles) else 0)
                 for i in range(len(styles))]
    m_all = torch.empty((S_total, 3, ny, nx), dtype=torch.float32, device="cuda:0")
    t_all = torch.empty_like(m_all)
    label = _film_ctx(n, replicas, Style("label"), terms=mmx.MMX_DEMAG)
    Hbuf = torch.empty((replicas, 3, 1, ny, nx), dtype=torch.float32, device="cuda:0")
    pos = 0
    try:
        for si, (style, count) in enumerate(zip(styles, per_style)):
            seed = seed0 + 1000 * si
            ctx = _film_ctx(n, replicas, style)
            try:
                if style.T > 0:
                    mmx.mmx_set_thermal(ctx, 0, [style.T] * replicas,
                                        replica_seeds(seed, replicas))
                    mmx.mmx_set_terms(ctx, mmx.MMX_ALL_TERMS)
                m = _dev(initial_states(style, n, replicas, seed))
                step, taken = 0, 0
                t0 = time.time()
                while taken < count:
                    mmx.mmx_heun(ctx, m, style.dt, every, step0=step)
                    step += every
                    k = min(replicas, count - taken)
                    mmx.mmx_field(label, m, Hbuf)
                    m_all[pos:pos + k] = m[:k, :, 0]
                    t_all[pos:pos + k] = Hbuf[:k, :, 0] / MS
                    t_all[pos:pos + k, 2] += m[:k, 2, 0]
                    pos += k
                    taken += k
                torch.cuda.synchronize()
                log(f"  data {style.name}: {count} snapshots, {step} Heun steps, "
                    f"{time.time() - t0:.1f} s")
            finally:
                mmx.mmx_destroy(ctx)
    finally:
        mmx.mmx_destroy(label)
    return m_all, t_all


class Net:
    """Parameters, Adam moments and gradient buffer of one mmx_fno."""

    def __init__(self, H, W, C=32, M1=12, M2=12, L=4, Cp=128, batch=32, use_mfma=True, seed=1):
        self.shape = dict(H=H, W=W, C=C, M1=M1, M2=M2, L=L, Cp=Cp)
        self.batch = batch
        self.f = mmx.mmx_fno_create(H, W, C, M1, M2, L, Cp, batch, use_mfma)
        mmx.mmx_fno_set_stream(self.f, torch.cuda.current_stream().cuda_stream)
        self.n = mmx.mmx_fno_param_count(self.f)
        self.params = torch.empty(self.n, dtype=torch.float32, device="cuda:0")
        mmx.mmx_fno_init(self.f, self.params, seed)
        self.grads = torch.zeros_like(self.params)
        self.moments = torch.zeros(2 * self.n, dtype=torch.float32, device="cuda:0")
        self.h = torch.empty((batch, 3, H, W), dtype=torch.float32, device="cuda:0")
        self.t = 0

    def close(self):
        if self.f:
            mmx.mmx_fno_destroy(self.f)
            self.f = None

    def loss_on(self, m, target, B):
        mmx.mmx_fno_forward(self.f, self.params, m, self.h, B)
        return mmx.mmx_fno_backward(self.f, self.params, self.h, target, self.grads)

    def step(self, m, target, B, lr, want_loss=False):
        mmx.mmx_fno_forward(self.f, self.params, m, self.h, B)
        loss = mmx.mmx_fno_backward(self.f, self.params, self.h, target, self.grads, want_loss)
        self.t += 1
        mmx.mmx_fno_adam(self.f, self.params, self.grads, self.moments, lr, self.t)
        return loss


def _batch_ptrs(x, start, B):
    per = x[0].numel() * x.element_size()
    return x.data_ptr() + int(start) * per


def evaluate(net: Net, m_all, t_all, lo, hi):
    """Mean relative-L2 loss (on the residual target) and the per-snapshot
    relative error of the total field |Ms(h - t)| / |H_demag| over [lo, hi)."""
    B = net.batch
    losses, gate = [], []
    for s in range(lo, hi, B):
        b = min(B, hi - s)
        mmx.mmx_fno_forward(net.f, net.params, _batch_ptrs(m_all, s, b), net.h, b)
        h = net.h[:b]
        t = t_all[s:s + b]
        num = torch.linalg.vector_norm((h - t).reshape(b, -1), dim=1)
        full = t.clone()
        full[:, 2] -= m_all[s:s + b, 2]
        den_res = torch.linalg.vector_norm(t.reshape(b, -1), dim=1)
        den = torch.linalg.vector_norm(full.reshape(b, -1), dim=1)
        losses.append(((num / den_res) ** 2).cpu())
        gate.append((num / den).cpu())
    return float(torch.cat(losses).mean()), torch.cat(gate).numpy()


def train(net: Net, m_all, t_all, n_train, epochs, lr0=1e-3, log=print, seed=0):
    """Adam with cosine decay from lr0 over all iterations; batches are
    contiguous slices visited in a seeded random order each epoch."""
    B = net.batch
    nb = n_train // B
    total = epochs * nb
    rng = np.random.default_rng(seed)
    hist = []
    it = 0
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(nb)
        sampled = []
        for j, bi in enumerate(order):
            lr = 0.5 * lr0 * (1.0 + math.cos(math.pi * it / total))
            want = (j % 16 == 0)   # loss read back (a synchronisation) on every 16th batch
            loss = net.step(_batch_ptrs(m_all, bi * B, B), _batch_ptrs(t_all, bi * B, B), B, lr,
                            want_loss=want)
            if want:
                sampled.append(loss)
            it += 1
        torch.cuda.synchronize()
        hist.append(float(np.mean(sampled)) if sampled else None)
        log(f"  epoch {ep + 1}/{epochs}: mean sampled train loss {hist[-1]:.4e} "
            f"({time.time() - t0:.1f} s)")
    return hist, time.time() - t0


def speedup(net: Net, n=(128, 128, 1), R=8, t_end=5e-11, tol=1e-5, gates=(1e-3,),
            seed=SEED0 + 90_000, log=print):
    """Held-out skyrmion-film relaxations (0 K): plain FP32 RK45 versus RK45
    with learned stages at each gate threshold, all against an FP64 RK45
    reference at tol 1e-9; plus a per-kernel time split of one learned run."""
    style = Style("eval", alpha=0.3, Ku=6e5, D=3e-3, B=(0.0, 0.0, 0.1), init="skyrmions")
    m0 = initial_states(style, n, R, seed)
    ref_ctx = _film_ctx(n, R, style, prec=mmx.MMX_F64)
    try:
        mref = torch.as_tensor(m0, dtype=torch.float64, device="cuda:0").contiguous()
        mmx.mmx_rk45(ref_ctx, mref, 0.0, t_end, 1e-9)
        torch.cuda.synchronize()
    finally:
        mmx.mmx_destroy(ref_ctx)
    ctx = _film_ctx(n, R, style)
    out = dict(workload=f"skyrmion film relaxation {n[0]}x{n[1]}x1, {R} replicas, "
                        f"0..{t_end:g} s, tol {tol:g}, held-out seeds")
    try:
        def timed(fn):
            m = _dev(m0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn(m)
            torch.cuda.synchronize()
            return m, time.perf_counter() - t0, res

        def dm(m):
            return float((m.double() - mref).norm(dim=1).max())

        timed(lambda m: mmx.mmx_rk45(ctx, m, 0.0, t_end / 10, tol))  # warm-up (graph, buffers)
        m_plain, t_plain, st_plain = timed(lambda m: mmx.mmx_rk45(ctx, m, 0.0, t_end, tol))
        out["plain"] = dict(seconds=t_plain, dm=dm(m_plain), accepted=st_plain.accepted,
                            rejected=st_plain.rejected)
        log(f"  plain FP32 RK45: {t_plain:.3f} s, |dm| {dm(m_plain):.2e}, "
            f"{st_plain.accepted} steps")
        runs = []
        for g in gates:
            m_sur, t_sur, (st, gl) = timed(lambda m: mmx.mmx_rk45_surrogate(
                ctx, net.f, net.params, m, 0.0, t_end, tol, gate_tol=g, gate_cap=100000))
            gl = np.asarray(gl)
            run = dict(
                gate=g, seconds=t_sur, speedup=t_plain / t_sur, dm=dm(m_sur),
                accepted=st.accepted, surrogate_steps=st.surrogate_steps,
                exact_steps=st.exact_steps, gate_checks=st.gate_checks,
                gate_failures=st.gate_failures, surrogate_rejected=st.surrogate_rejected,
                fallback_rate=(st.gate_failures / st.gate_checks) if st.gate_checks else None,
                gate_error_quantiles=(dict(zip(["min", "p10", "p50", "p90", "max"],
                                               np.quantile(gl, [0, .1, .5, .9, 1]).tolist()))
                                      if gl.size else None),
                gate_histogram_log10=(np.histogram(np.log10(np.maximum(gl, 1e-12)),
                                                   bins=np.arange(-5, 1.01, 0.5))[0].tolist()
                                      if gl.size else None))
            runs.append(run)
            log(f"  learned, gate {g:g}: {t_sur:.3f} s (x{t_plain / t_sur:.3f}), "
                f"|dm| {run['dm']:.2e}, kept {st.surrogate_steps}/{st.accepted}, "
                f"gate failures {st.gate_failures}/{st.gate_checks}")
        out["learned"] = runs
        out["gate_histogram_bins"] = "log10 edges -5.0, -4.5, ..., 1.0"
        # where the time of a learned run goes (HIP events around each launch)
        mmx.mmx_profile_enable(ctx, 1)
        m = _dev(m0)
        mmx.mmx_rk45_surrogate(ctx, net.f, net.params, m, 0.0, t_end, tol, gate_tol=math.inf)
        prof = mmx.mmx_profile_get(ctx)
        mmx.mmx_profile_enable(ctx, 0)
        out["learned_time_split_ms"] = {k: dict(total=v[0], launches=v[1])
                                        for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    finally:
        mmx.mmx_destroy(ctx)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--snapshots", type=int, default=20000)
    ap.add_argument("--val", type=int, default=2000)
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--fp32-net", action="store_true", help="FP32 1x1 maps instead of BF16 MFMA")
    ap.add_argument("--eval-replicas", type=int, default=8)
    ap.add_argument("--t-end", type=float, default=5e-11)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--gate", type=float, nargs="+", default=[1e-3, 3e-2, math.inf],
                    help="gate thresholds to evaluate (the first is the method's)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--save-params", default=None)
    ap.add_argument("--load-params", default=None,
                    help="start from saved parameters (with --epochs 0: evaluation only)")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    n = (a.n, a.n, 1)
    gate = a.gate[0]
    net = Net(a.n, a.n, batch=a.batch, use_mfma=not a.fp32_net)
    try:
        if a.load_params:
            prm = np.fromfile(a.load_params, dtype=np.float32)
            if prm.size != net.n:
                raise SystemExit(f"{a.load_params}: {prm.size} floats, the network has {net.n}")
            net.params.copy_(torch.from_numpy(prm))
        report = dict(net=dict(net.shape, params=net.n, batch=a.batch,
                               bf16_mfma=not a.fp32_net, loaded=a.load_params))
        if a.snapshots > 0:
            log(f"generating {a.snapshots} snapshots of {a.n}x{a.n} films")
            t0 = time.time()
            m_all, t_all = generate(n, a.snapshots, a.replicas, a.every, log=log)
            t_data = time.time() - t0
            n_train = a.snapshots - a.val
            loss0, _ = evaluate(net, m_all, t_all, n_train, a.snapshots)
            log(f"initial validation loss {loss0:.4e}")
            hist, t_train = train(net, m_all, t_all, n_train, a.epochs, a.lr, log=log)
            vloss, vgate = evaluate(net, m_all, t_all, n_train, a.snapshots)
            log(f"validation loss {vloss:.4e}; total-field error median "
                f"{np.median(vgate):.3e}, fraction <= {gate:g}: {(vgate <= gate).mean():.3f}")
            report["data"] = dict(snapshots=a.snapshots, train=n_train, val=a.val,
                                  replicas=a.replicas, every=a.every,
                                  styles=[s.name for s in STYLES], seconds=t_data)
            report["train"] = dict(
                epochs=a.epochs, lr0=a.lr, schedule="cosine", seconds=t_train,
                loss_history=hist, val_loss_initial=loss0, val_loss=vloss,
                val_total_error_median=float(np.median(vgate)),
                val_total_error_p90=float(np.quantile(vgate, 0.9)),
                val_fraction_within_gate=float((vgate <= gate).mean()))
            del m_all, t_all
            torch.cuda.empty_cache()
        if a.save_params:
            net.params.cpu().numpy().tofile(a.save_params)
        report["rk45"] = speedup(net, n, a.eval_replicas, a.t_end, a.tol, a.gate, log=log)
        text = json.dumps(report, indent=1)
        log(text)
        if a.out:
            with open(a.out, "w") as fh:
                fh.write(text + "\n")
    finally:
        net.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
