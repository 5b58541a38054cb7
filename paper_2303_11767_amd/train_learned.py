"""Train and evaluate the learned r = 1 right-hand-side correction.

    python -m paper_2303_11767_amd.train_learned [--traj 200] [--out model.npz]

Data: seeded band-limited states on the 360 x 180 mesh, advanced with the
plain r = 4 solver; at snapshots of each trajectory the target is
    c* = P1 L4(q4) - L1(P1 q4),
P1 the cos-weighted projection onto r = 1 (dg_project), L_r the plain DG
right-hand side (dg_rhs): the correction that makes the r = 1 right-hand side
of the projected state equal the projection of the r = 4 one.  Features are
the 3 x 3 element stencil of P1 q4 (dg_features), standardised per feature;
targets are standardised per latitude row.  The network is trained with the
library's own forward/backward/Adam kernels (dg_mlp_train_step).

Evaluation: on held-out seeds, the truth is the plain r = 5 solver from the same
initial polynomial field; the error of a method is the RMS over the sphere of
P1 h_method - P1 h_truth at the horizon (held-out seeds 200-219, 30 s).
Compared: plain r = 1 .. 4, learned r = 1 (trained), learned r = 1 with an
untrained network; wall-clock of learned r = 1 against plain r = 4 for the
same simulated time, and against the lowest plain order that reaches the
learned error (equal-error comparison).

Device work runs in the library; torch provides buffers, random batch
indices and the mean/standard-deviation statistics of the training set.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_LON, N_LAT, L_MAX, CFL = 360, 180, 32, 0.1
MASK = [0.0] + [1.0] * 11          # (h, mode 00) is set by the mass correction


def log(*a):
    print("[learned]", *a, flush=True)


def h_rms(d_h, n_lon, n_lat):
    """RMS over the sphere of an order-1 height field given by its modal
    coefficients d_h[E][4]: sqrt(int d^2 cos / int cos), by Gauss-Legendre
    quadrature on each element."""
    x, w = np.polynomial.legendre.leggauss(4)
    P = np.stack([np.full_like(x, np.sqrt(0.5)), np.sqrt(1.5) * x], axis=1)   # [q, a]
    dth = math.pi / n_lat
    d = d_h.reshape(n_lat, n_lon, 2, 2)                                      # [j, i, b, a]
    vals = np.einsum("jiba,pa,sb->jisp", d, P, P)
    th = -0.5 * math.pi + (np.arange(n_lat)[:, None] + 0.5 * (1 + x[None, :])) * dth
    wt = (np.cos(th) * w[None, :])[:, None, :, None] * w[None, None, None, :]
    num = (vals ** 2 * wt).sum()
    den = (np.ones_like(vals) * wt).sum()
    return float(np.sqrt(num / den))


class Workbench:
    """Meshes and helpers on one GPU."""

    def __init__(self, dtype="f32"):
        import torch
        import paper_2303_11767_amd as dg
        self.dg, self.torch = dg, torch
        href = 1e4 if dtype == "f32" else 0.0
        self.dtype = dtype
        self.m1 = dg.Mesh(N_LON, N_LAT, 1, dtype=dtype, h_ref=href)
        self.m4 = dg.Mesh(N_LON, N_LAT, 4, dtype=dtype, h_ref=href)
        self.tdt = self.m1.dtype

    def initial(self, seed):
        from dg_inputs import band_limited_state
        q4, info = band_limited_state(N_LON, N_LAT, 4, L_MAX, seed)
        return q4, info


def build_dataset(args, wb):
    from paper_2303_11767_amd import learned
    torch = wb.torch
    gen = torch.Generator(device="cuda").manual_seed(1234)
    Xs, Ts, Js = [], [], []
    s_sum = torch.zeros((N_LAT, 12), dtype=torch.float64, device="cuda")
    s_sq = torch.zeros((N_LAT, 12), dtype=torch.float64, device="cuda")
    count = 0
    work = wb.m4.empty_work()
    t0 = time.time()
    for k in range(args.traj):
        q4h, info = wb.initial(args.seed0 + k)
        q4 = torch.from_numpy(q4h).to("cuda", wb.tdt)
        dt = wb.dg.cfl_time_step(wb.m4, info.cmax, CFL)
        nsnap = args.snapshots
        per = max(1, int(round(args.t_train / (nsnap - 1) / dt))) if nsnap > 1 else 0
        for sidx in range(nsnap):
            if sidx:
                wb.m4.rk_step(q4, work, dt, nsteps=per)
            q1 = learned.project(wb.m4, wb.m1, q4)
            L1 = wb.m1.rhs(q1)
            PL4 = learned.project(wb.m4, wb.m1, wb.m4.rhs(q4))
            c = (PL4 - L1).to(torch.float64).view(N_LAT, N_LON, 12)
            s_sum += c.sum(1)
            s_sq += (c * c).sum(1)
            count += N_LON
            X = learned.features(wb.m1, q1)
            idx = torch.randperm(wb.m1.E, generator=gen, device="cuda")[:args.rows_per_snapshot]
            Xs.append(X[idx].clone())
            Ts.append(c.view(-1, 12)[idx].to(torch.float32))
            Js.append((idx // N_LON).to(torch.int32))
        if k % 20 == 0 or k == args.traj - 1:
            torch.cuda.synchronize()
            log(f"trajectory {k + 1}/{args.traj}, {time.time() - t0:.0f} s")
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    J = torch.cat(Js).long()
    feat_mean = X.mean(0)
    feat_istd = 1.0 / (X.std(0) + 1e-12)
    out_mean = (s_sum / count).to(torch.float32)
    out_std = torch.sqrt(torch.clamp(s_sq / count - (s_sum / count) ** 2, min=0)).to(torch.float32)
    out_std = torch.where(out_std > 0, out_std, torch.ones_like(out_std))
    Xn = ((X - feat_mean) * feat_istd).contiguous()
    Tn = ((T - out_mean[J]) / out_std[J]).contiguous()
    return Xn, Tn, {"feat_mean": feat_mean.contiguous(), "feat_istd": feat_istd.contiguous(),
                    "out_mean": out_mean.contiguous(), "out_std": out_std.contiguous()}


def he_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((108, 256), (256, 256), (256, 12)):
        parts.append(rng.standard_normal(fan_in * fan_out) * math.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def fit(args, wb, X, T):
    from paper_2303_11767_amd import learned
    torch = wb.torch
    P = learned.param_count()
    params = torch.from_numpy(he_params(args.seed0 + 777)).cuda()
    m = torch.zeros(P, dtype=torch.float32, device="cuda")
    v = torch.zeros(P, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(99)
    n = X.shape[0]
    hist = []
    t0 = time.time()
    for step in range(1, args.steps + 1):
        idx = torch.randint(0, n, (args.batch,), generator=gen, device="cuda")
        learned.mlp_train_step(params, X[idx].contiguous(), T[idx].contiguous(), MASK, m, v, step,
                               args.lr, loss=loss)
        if step % 100 == 0 or step == 1:
            hist.append((step, loss.item()))
            if step % 500 == 0 or step == 1:
                log(f"step {step} loss {hist[-1][1]:.4f} ({time.time() - t0:.0f} s)")
    return params, hist


PLAIN = ("r1", "r2", "r3", "r4")


def equal_error(eps, wall):
    """The lowest plain order whose error reaches the learned one (mean over
    seeds), with the learned form's throughput relative to it."""
    for key in PLAIN:
        if eps[key] <= eps["learned"]:
            return {"plain": key, "h_rms_error_m": eps[key], "learned_h_rms_error_m": eps["learned"],
                    "wall_s_per_run": wall[key], "learned_wall_s_per_run": wall["learned"],
                    "throughput_learned_over_plain": wall[key] / max(wall["learned"], 1e-12)}
    return {"plain": None, "note": "no plain order up to 4 reaches the learned error"}


def evaluate(args, model, seeds, t_eval, dtype="f64", fields=None):
    """Errors at the horizon against the r = 5 truth, and wall-clock, of
    plain r = 1..4 and learned r = 1 (trained and untrained network).  Every
    method starts from the cos-weighted projection of the same order-4
    polynomial (P_k P_4 = P_k, so at t = 0 all errors are zero in the
    order-1 norm).  fields(seed) -> (q4 host array, StateInfo) supplies the
    initial polynomials (default: band_limited_state)."""
    import torch
    import paper_2303_11767_amd as dg
    from paper_2303_11767_amd import learned
    href = 1e4 if dtype == "f32" else 0.0
    m1 = dg.Mesh(N_LON, N_LAT, 1, dtype=dtype, h_ref=href)
    m2 = dg.Mesh(N_LON, N_LAT, 2, dtype=dtype, h_ref=href)
    m3 = dg.Mesh(N_LON, N_LAT, 3, dtype=dtype, h_ref=href)
    m4 = dg.Mesh(N_LON, N_LAT, 4, dtype=dtype, h_ref=href)
    m5 = dg.Mesh(N_LON, N_LAT, 5, dtype=dtype, h_ref=href)
    tdt = m1.dtype
    nets = {"learned": learned.LearnedRHS(m1, model["params"], model["feat_mean"], model["feat_istd"],
                                          model["out_mean"], model["out_std"], kappa=args.kappa)}
    untrained = torch.from_numpy(he_params(4242)).cuda()
    nets["untrained"] = learned.LearnedRHS(m1, untrained, model["feat_mean"], model["feat_istd"],
                                           model["out_mean"], model["out_std"], kappa=args.kappa)
    res = {k: [] for k in ("r1", "learned", "untrained", "r2", "r3", "r4")}
    wall = {"r1": 0.0, "learned": 0.0, "r2": 0.0, "r3": 0.0, "r4": 0.0, "r5": 0.0}
    fallbacks = 0
    if fields is None:
        from dg_inputs import band_limited_state

        def fields(seed):
            return band_limited_state(N_LON, N_LAT, 4, L_MAX, seed)

    def run(mesh, q, dt, nsteps, key, net=None):
        w = mesh.empty_work()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(True), torch.cuda.Event(True)
        a.record()
        if net is None:
            mesh.rk_step(q, w, dt, nsteps=nsteps)
        else:
            net.rk_step(q, w, dt, nsteps=nsteps)
        b.record()
        torch.cuda.synchronize()
        if key in wall:
            wall[key] += a.elapsed_time(b) * 1e-3
        return q

    meshes = {"r1": m1, "r2": m2, "r3": m3, "r4": m4, "r5": m5}
    for seed in seeds:
        q4h, info = fields(seed)
        q4 = torch.from_numpy(q4h).to("cuda", tdt)
        q5 = learned.project(m4, m5, q4)
        q1 = learned.project(m4, m1, q4)
        steps = {}
        for key, mesh in meshes.items():
            dt = dg.cfl_time_step(mesh, info.cmax, CFL)
            n = max(1, int(math.ceil(t_eval / dt)))
            steps[key] = (t_eval / n, n)
        out = {}
        out["r5"] = run(m5, q5, *steps["r5"], "r5")
        out["r4"] = run(m4, q4.clone(), *steps["r4"], "r4")
        for key in ("r2", "r3"):
            out[key] = run(meshes[key], learned.project(m4, meshes[key], q4), *steps[key], key)
        out["r1"] = run(m1, q1.clone(), *steps["r1"], "r1")
        for key in ("learned", "untrained"):
            nets[key].fallbacks.zero_()
            out[key] = run(m1, q1.clone(), *steps["r1"], key, nets[key])
            if key == "learned":
                fallbacks += int(nets[key].fallbacks.item())
        truth = learned.project(m5, m1, out["r5"]).cpu().numpy()[:, 0, :]
        for key in ("r1", "learned", "untrained"):
            res[key].append(h_rms(out[key].cpu().numpy()[:, 0, :] - truth, N_LON, N_LAT))
        for key in ("r2", "r3", "r4"):
            res[key].append(h_rms(learned.project(meshes[key], m1, out[key]).cpu().numpy()[:, 0, :] - truth,
                                  N_LON, N_LAT))
        log(f"seed {seed}: " + ", ".join(f"{k} {v[-1]:.3e} m" for k, v in res.items()))
    eps = {k: float(np.mean(v)) for k, v in res.items()}
    n_seeds = len(seeds)
    return {
        "horizon_s": t_eval, "seeds": list(seeds), "dtype": dtype, "kappa": args.kappa,
        "h_rms_error_m": eps,
        "ratio_learned_to_r4": eps["learned"] / eps["r4"],
        "gain_learned_vs_plain_r1": eps["r1"] / eps["learned"],
        "gain_trained_vs_untrained": eps["untrained"] / eps["learned"],
        "wall_s_per_run": {k: v / n_seeds for k, v in wall.items()},
        "throughput_learned_over_r4": wall["r4"] / max(wall["learned"], 1e-12),
        "fallback_elements_per_run": fallbacks / n_seeds,
        "h_rms_error_per_seed_m": {k: [float(x) for x in v] for k, v in res.items()},
        "equal_error": equal_error(eps, {k: v / n_seeds for k, v in wall.items()}),
    }


KAPPAS = (1.0, 2.0, 4.0, 8.0, 16.0, 1.0e30)


def pick_kappa(errs, tol=0.05):
    """The smallest trust bound whose error is within tol of the best one
    (errs: kappa -> validation error); non-finite errors never qualify."""
    finite = {k: e for k, e in errs.items() if math.isfinite(e)}
    if not finite:
        raise ValueError("no finite validation error")
    best = min(finite.values())
    return min(k for k, e in finite.items() if e <= (1.0 + tol) * best)


def select_kappa(args):
    """The trust bound is a tuning choice of the fallback, so it is chosen on
    validation seeds (disjoint from the training seeds 0.. and the held-out
    seeds 200..): the smallest kappa whose learned error is within 5 % of the
    best one, recorded in the model's metadata; then the held-out evaluation."""
    model, meta = load_model(args.select_kappa)
    seeds = range(args.val_seed0, args.val_seed0 + args.val)
    errs = {}
    for k in KAPPAS:
        rep = evaluate(argparse.Namespace(kappa=k), model, seeds, args.t_eval)
        errs[k] = rep["h_rms_error_m"]["learned"]
        log(f"kappa {k:g}: learned {errs[k]:.4e} m (plain r1 {rep['h_rms_error_m']['r1']:.4e} m)")
    chosen = pick_kappa(errs)
    meta["kappa"] = chosen
    meta["kappa_selection"] = {"seeds": list(seeds), "t_eval_s": args.t_eval,
                               "learned_h_rms_m": {f"{k:g}": e for k, e in errs.items()}}
    save(args.select_kappa, model, meta)
    args.kappa = chosen
    report = evaluate(args, model, range(200, 200 + args.heldout), args.t_eval)
    report["model"] = os.path.basename(args.select_kappa)
    report["kappa_selection"] = meta["kappa_selection"]
    report["training"] = {k: meta[k] for k in ("traj", "snapshots", "t_train_s", "steps", "batch", "lr")
                          if k in meta}
    log(json.dumps(report))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


def save(path, model, meta):
    np.savez(path, **{k: v.detach().cpu().numpy() for k, v in model.items()},
             meta=np.array(json.dumps(meta)))


def load_model(path, device="cuda"):
    import torch
    z = np.load(path, allow_pickle=False)
    model = {k: torch.from_numpy(z[k]).to(device) for k in
             ("params", "feat_mean", "feat_istd", "out_mean", "out_std")}
    return model, json.loads(str(z["meta"]))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--traj", type=int, default=200)
    ap.add_argument("--seed0", type=int, default=0)
    ap.add_argument("--snapshots", type=int, default=5)
    ap.add_argument("--t-train", type=float, default=30.0)
    ap.add_argument("--rows-per-snapshot", type=int, default=8192)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--kappa", type=float, default=None,
                    help="trust bound of the fallback (default: the model's stored one; 1 for a new model)")
    ap.add_argument("--heldout", type=int, default=20)
    ap.add_argument("--t-eval", type=float, default=30.0)
    ap.add_argument("--out", default="learned_r1_360x180.npz")
    ap.add_argument("--report", default=None)
    ap.add_argument("--evaluate-only", default=None, metavar="MODEL",
                    help="evaluate a saved model (no training)")
    ap.add_argument("--select-kappa", default=None, metavar="MODEL",
                    help="pick the trust bound kappa of a saved model on validation seeds "
                         "(--val-seed0, --val), store it in the model, then evaluate it")
    ap.add_argument("--val-seed0", type=int, default=300)
    ap.add_argument("--val", type=int, default=4)
    args = ap.parse_args()
    if args.select_kappa:
        select_kappa(args)
        return
    if args.evaluate_only:
        model, meta = load_model(args.evaluate_only)
        if args.kappa is None:
            args.kappa = meta.get("kappa", 1.0)
        report = evaluate(args, model, range(200, 200 + args.heldout), args.t_eval)
        report["model"] = os.path.basename(args.evaluate_only)
        log(json.dumps(report))
        if args.report:
            with open(args.report, "w") as f:
                json.dump(report, f, indent=1)
        return
    if args.kappa is None:
        args.kappa = 1.0
    wb = Workbench("f32")
    t0 = time.time()
    X, T, stats = build_dataset(args, wb)
    log(f"dataset {tuple(X.shape)} in {time.time() - t0:.0f} s")
    params, hist = fit(args, wb, X, T)
    model = dict(stats, params=params)
    meta = {"mesh": [N_LON, N_LAT], "traj": args.traj, "snapshots": args.snapshots,
            "t_train_s": args.t_train, "steps": args.steps, "batch": args.batch, "lr": args.lr,
            "loss_history": hist, "kappa": args.kappa}
    save(args.out, model, meta)
    report = evaluate(args, model, range(200, 200 + args.heldout), args.t_eval)
    report["training"] = {k: meta[k] for k in ("traj", "snapshots", "t_train_s", "steps", "batch", "lr")}
    report["final_loss"] = hist[-1][1]
    log(json.dumps(report))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
