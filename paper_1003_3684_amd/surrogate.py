"""MLP surrogate: generator parameters -> graph statistics, trained on the
ensembles the generators produce and inverted to choose Kronecker parameters
for a target degree exponent.  The real generator has the last word: a proposal
is accepted only when the generated graph's measured exponent is within the
tolerance, and the generator-only search takes over when the surrogate's
share of the budget runs out (fit_exponent).

Everything numerical runs in the library's kernels: ensemble_generate makes
the training data, mlp_forward / mlp_backward / mlp_mse_grad / adam_step train
the network and give input gradients for the inversion.  This module only
encodes features, schedules the steps and keeps score.
"""
import math

import numpy as np
import torch

from . import native as sfg

D_IN = 10      # [is_pba, is_kron, log2(n)/20, m/8, 2p, W00, W01, W10, W11, k/20]
D_OUT = 34     # 32 degree-bin shares, log(gamma - 1), closed-wedge fraction
GAMMA_COL = 32


def features(rows):
    X = np.zeros((len(rows), D_IN), np.float32)
    for i, r in enumerate(rows):
        if r["kind"] == "pba":
            X[i, 0] = 1
            X[i, 2] = math.log2(r["n"]) / 20
            X[i, 3] = r["m"] / 8
            X[i, 4] = 2 * r["p_inter"]
        else:
            X[i, 1] = 1
            X[i, 2] = r["k"] / 20
            X[i, 5:9] = np.asarray(r["initiator"], np.float32).ravel()[:4]
            X[i, 9] = r["k"] / 20
    return X


def targets(rows, hist, gamma, closed, samples):
    """(Y, mask): share of vertices per degree bin, log(gamma - 1), closed
    share; missing values masked.  The estimated exponent is heavy-tailed
    (nearly regular graphs give very large values); log(gamma - 1), the log
    of the tail index, is the smooth quantity to regress on."""
    n = np.array([r["n"] if r["kind"] == "pba" else r["n0"] ** r["k"] for r in rows], np.float64)
    Y = np.zeros((len(rows), D_OUT), np.float32)
    M = np.ones((len(rows), D_OUT), np.float32)
    Y[:, :32] = hist / n[:, None]
    g = np.asarray(gamma, np.float64)
    ok = np.isfinite(g) & (g > 1)
    Y[:, GAMMA_COL] = np.log(np.where(ok, g, 2.0) - 1.0)
    M[:, GAMMA_COL] = ok
    c = np.asarray(closed, np.float64)
    Y[:, 33] = np.where(c >= 0, c / max(samples, 1), 0)
    M[:, 33] = c >= 0
    return Y, M


def generate_dataset(rows, samples=10_000, stat_seed=0, max_batch_edges=1 << 28, ws=None):
    """Statistics of every graph in `rows` via the batched ensemble."""
    descs = sfg.graph_descs(rows)
    hist, gamma, closed = sfg.ensemble_generate(descs, num_samples=samples, stat_seed=stat_seed,
                                                max_batch_edges=max_batch_edges, ws=ws, check=True)
    return targets(rows, hist.cpu().numpy().astype(np.float64), gamma.cpu().numpy(), closed.cpu().numpy(), samples)


class Surrogate:
    def __init__(self, width=256, hidden=3, seed=0, batch=4096):
        self.shape = sfg.mlp_shape(D_IN, width, D_OUT, hidden)
        rng = np.random.default_rng(seed)
        P = sfg.mlp_param_count(self.shape)
        p = np.zeros(P, np.float32)
        off = 0
        dims = [D_IN] + [width] * hidden + [D_OUT]
        for i in range(len(dims) - 1):
            n_in, n_out = dims[i], dims[i + 1]
            p[off:off + n_in * n_out] = rng.normal(0, math.sqrt(2.0 / n_in), size=n_in * n_out)
            off += n_in * n_out + n_out
        self.params = torch.tensor(p).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.batch = batch
        self.ws = sfg.workspace(sfg.mlp_workspace_bytes(self.shape, batch))
        self.lws = sfg.workspace(4 * batch)
        # The fused training step's workspace (None when the network is wider
        # than the fused step takes).
        tb = sfg.mlp_train_workspace_bytes(self.shape, batch)
        self.tws = sfg.workspace(tb) if tb > 0 else None
        self.mu = np.zeros(D_OUT, np.float32)
        self.sd = np.ones(D_OUT, np.float32)

    def fit(self, X, Y, M, epochs=30, lr=1e-3, seed=0, col_weight=None, graph=True, fused=True):
        """Adam on standardized targets over full batches; returns the
        per-epoch mean loss.  A training step is forward, loss gradient,
        backward and Adam over the batch's rows: with fused=True (and a
        network the fused step takes) one mlp_train_step, which reads the
        rows through the shuffled index list; otherwise the batch is gathered
        and the unfused kernels run.  The learning rate (cosine schedule) and
        the step counter live in device memory, so with graph=True the step
        is captured once into a HIP graph after a first eager step and
        replayed; the result is bit-identical to the eager loop."""
        rng = np.random.default_rng(seed)
        Mb = M.astype(bool)
        for j in range(D_OUT):
            col = Y[Mb[:, j], j]
            if col.size:
                self.mu[j] = col.mean()
                self.sd[j] = max(col.std(), 1e-3)
        Ys = (Y - self.mu) / self.sd * M
        cw = torch.tensor(np.ones(D_OUT, np.float32) if col_weight is None else col_weight).cuda()
        Xg, Yg, Mg = (torch.tensor(a).cuda() for a in (X, Ys.astype(np.float32), M.astype(np.float32)))
        N, B = X.shape[0], self.batch
        nb = N // B
        if nb == 0:
            raise ValueError(f"fit needs at least one full batch of {B} rows")
        dev = self.params.device
        idx = torch.empty(B, dtype=torch.int64, device=dev)
        xs = torch.empty((B, D_IN), dtype=torch.float32, device=dev)
        ys = torch.empty((B, D_OUT), dtype=torch.float32, device=dev)
        ms = torch.empty((B, D_OUT), dtype=torch.float32, device=dev)
        y, dy = torch.empty_like(ys), torch.empty_like(ys)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        grad = torch.empty_like(self.params)
        lr_dev = torch.zeros(1, dtype=torch.float32, device=dev)
        step_dev = torch.tensor([self.step], dtype=torch.int32, device=dev)
        loss_acc = torch.zeros(1, dtype=torch.float32, device=dev)

        fused = fused and self.tws is not None

        def step():
            if fused:
                sfg.mlp_train_step(self.shape, B, self.params, Xg, Yg, self.m, self.v, lr_dev, step_dev, self.tws,
                                   rows=idx, mask=Mg, col_weight=cw, loss=loss)
                loss_acc.add_(loss)
                return
            torch.index_select(Xg, 0, idx, out=xs)
            torch.index_select(Yg, 0, idx, out=ys)
            torch.index_select(Mg, 0, idx, out=ms)
            sfg.mlp_forward(self.shape, self.params, xs, self.ws, y=y)
            sfg.mlp_mse_grad(y, ys, self.lws, mask=ms, col_weight=cw, dy=dy, loss=loss)
            sfg.mlp_backward(self.shape, self.params, dy, self.ws, grad=grad)
            sfg.adam_step_device(self.params, grad, self.m, self.v, lr_dev, step_dev)
            loss_acc.add_(loss)

        g = None
        history = []
        for ep in range(epochs):
            order = torch.tensor(rng.permutation(N)).to(dev)
            lr_dev.fill_(lr * 0.5 * (1 + math.cos(math.pi * ep / max(epochs, 1))))
            loss_acc.zero_()
            for b in range(nb):
                idx.copy_(order[b * B:(b + 1) * B])
                if g is not None:
                    g.replay()
                    continue
                step()
                if graph:  # every kernel has run once: capture the step
                    torch.cuda.synchronize()
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g):
                        step()
            history.append(float(loss_acc.item()) / nb)
        self.step = int(step_dev.item())
        return history

    def predict(self, X):
        out = []
        for b0 in range(0, X.shape[0], self.batch):
            xb = torch.tensor(X[b0:b0 + self.batch]).cuda()
            y = sfg.mlp_forward(self.shape, self.params, xb, self.ws)
            out.append(y.cpu().numpy() * self.sd + self.mu)
        return np.concatenate(out, 0)

    def log_tail_and_grad(self, X):
        """Predicted u = log(gamma - 1) and du / dX for a batch of feature rows."""
        xb = torch.tensor(X).cuda()
        y = sfg.mlp_forward(self.shape, self.params, xb, self.ws)
        dy = torch.zeros_like(y)
        dy[:, GAMMA_COL] = 1.0
        _, dx = sfg.mlp_backward(self.shape, self.params, dy, self.ws, want_grad=False, want_dx=True)
        u = y[:, GAMMA_COL].cpu().numpy().astype(np.float64) * self.sd[GAMMA_COL] + self.mu[GAMMA_COL]
        return u, dx.cpu().numpy().astype(np.float64) * self.sd[GAMMA_COL]

    def gamma_and_grad(self, X):
        """Predicted gamma and d gamma / dX for a batch of feature rows."""
        u, du = self.log_tail_and_grad(X)
        e = np.exp(u)
        return 1.0 + e, du * e[:, None]

    @staticmethod
    def gamma_of(Y):
        """Exponent from the target encoding."""
        return 1.0 + np.exp(np.asarray(Y)[:, GAMMA_COL].astype(np.float64))


# ----------------------------------------------------------------------------- inversion
def kron_row(a, b, k, seed, graph_id=0):
    """The 2x2 row-stochastic initiator family [[a, 1-a], [b, 1-b]]."""
    W = np.array([[a, 1 - a], [b, 1 - b]], np.float32)
    return dict(kind="kron", graph_id=graph_id, n0=2, initiator=W, k=k, num_edges=16 << k, seed=seed)


class Judge:
    """Runs the real generator and measures the exponent; counts the calls."""

    def __init__(self, k=14, seeds=(101,), samples=2000):
        self.k, self.seeds, self.samples, self.calls = k, seeds, samples, 0
        E = 16 << k
        self.ws = sfg.workspace(sfg.graph_stats_workspace_bytes(2 ** k, E, 4))

    def gamma(self, a, b):
        vals = []
        for s in self.seeds:
            r = kron_row(a, b, self.k, s)
            src, dst = sfg.kron_generate(2, r["initiator"], self.k, r["num_edges"], seed=s)
            _, g, _ = sfg.graph_stats(2 ** self.k, src, dst, num_samples=self.samples, seed=s, ws=self.ws)
            self.calls += 1
            vals.append(float(g.item()))
        return float(np.mean(vals))


def invert(model, target, k, restarts=16, iters=40, damping=0.5, max_step=0.1, seed=0, bounds=(0.03, 0.97)):
    """Solve predicted gamma(a, b) = target from several random starts by
    damped minimum-norm Newton steps on u = log(gamma - 1), projected onto
    the box; returns the candidates ordered by predicted error and their
    predicted exponents."""
    rng = np.random.default_rng(seed)
    ab = rng.uniform(bounds[0], bounds[1], size=(restarts, 2))
    ut = math.log(target - 1.0)
    for _ in range(iters):
        X = features([kron_row(a, b, k, 0) for a, b in ab])
        u, dX = model.log_tail_and_grad(X)
        # x5..x8 = (a, 1-a, b, 1-b): chain rule to (a, b)
        grad = np.stack([dX[:, 5] - dX[:, 6], dX[:, 7] - dX[:, 8]], 1)
        step = damping * (u - ut)[:, None] * grad / ((grad * grad).sum(1, keepdims=True) + 1e-9)
        norm = np.sqrt((step * step).sum(1, keepdims=True))
        step *= np.minimum(1.0, max_step / np.maximum(norm, 1e-12))
        ab = np.clip(ab - step, *bounds)
    X = features([kron_row(a, b, k, 0) for a, b in ab])
    g, _ = model.gamma_and_grad(X)
    order = np.argsort(np.abs(g - target))
    return ab[order], g[order]


def search_generator_only(judge, target, tol, budget=40, seed=0):
    """Baseline without the surrogate: random search over the (a, b) family,
    one generator run per candidate; returns (accepted, calls)."""
    rng = np.random.default_rng(seed)
    calls0 = judge.calls
    while judge.calls - calls0 < budget:
        a, b = rng.uniform(0.03, 0.97, size=2)
        if abs(judge.gamma(a, b) - target) <= tol:
            return True, judge.calls - calls0
    return False, judge.calls - calls0


def _u_grad(model, k, ab):
    """Predicted u = log(gamma - 1) at (a, b) and its gradient in (a, b)."""
    u, dX = model.log_tail_and_grad(features([kron_row(ab[0], ab[1], k, 0)]))
    # x5..x8 = (a, 1-a, b, 1-b): chain rule to (a, b)
    return float(u[0]), np.array([dX[0, 5] - dX[0, 6], dX[0, 7] - dX[0, 8]])


def search_with_surrogate(model, judge, target, tol, budget=40, seed=0, refine=6, max_step=0.15,
                          bounds=(0.03, 0.97)):
    """Surrogate-guided search, each proposal judged by one generator run.

    A start is the best inversion of the surrogate for the target.  From it
    the search moves along the surrogate's gradient of u = log(gamma - 1),
    by secant steps on the measured u: the first step uses the surrogate's
    slope, later ones the slope measured between the last two runs (kept
    when it agrees in sign with the surrogate and lies within a factor of 5
    of it).  The surrogate's level sets differ from the generator's by a
    smooth offset, so these local steps converge where re-inverting for a
    shifted target from scattered starts would not.  After `refine` steps
    without success, or an unusable measurement, the search restarts from
    another inversion.  Returns (accepted, calls)."""
    calls0 = judge.calls
    ut = math.log(target - 1.0)
    r = 0
    while judge.calls - calls0 < budget:
        cands, _ = invert(model, target, judge.k, seed=seed * 1000 + r)
        r += 1
        x = np.array(cands[0], np.float64)
        prev = None
        for _ in range(refine + 1):
            if judge.calls - calls0 >= budget:
                break
            g = judge.gamma(float(x[0]), float(x[1]))
            if abs(g - target) <= tol:
                return True, judge.calls - calls0
            if not (math.isfinite(g) and g > 1):
                break
            u = math.log(g - 1.0)
            _, grad = _u_grad(model, judge.k, x)
            gn = float(np.sqrt((grad * grad).sum()))
            if gn < 1e-9:
                break
            d = grad / gn
            slope = gn  # du per unit distance along d, from the surrogate
            if prev is not None:
                dist = float(np.dot(x - prev[0], d))
                if abs(dist) > 1e-9:
                    meas = (u - prev[1]) / dist
                    if 0.2 * gn < meas < 5.0 * gn:
                        slope = meas
            step = -(u - ut) / slope
            step = max(-max_step, min(max_step, step))
            prev = (x.copy(), u)
            x = np.clip(x + step * d, *bounds)
    return False, judge.calls - calls0


def fit_exponent(model, judge, target, tol, budget=40, seed=0, surrogate_share=0.5):
    """Parameters for a target exponent: the surrogate-guided search with a
    share of the budget, then the generator-only search with the rest.
    Returns (accepted, calls, which) with which in {"surrogate", "generator"}."""
    ok, c = search_with_surrogate(model, judge, target, tol, budget=max(1, int(budget * surrogate_share)), seed=seed)
    if ok:
        return True, c, "surrogate"
    ok2, c2 = search_generator_only(judge, target, tol, budget=budget - c, seed=seed)
    return ok2, c + c2, "generator"


# ----------------------------------------------------------------------------- the ensemble-scale study
def generate_dataset_chunked(rows, samples=10_000, stat_seed=0, chunk=4096, max_batch_edges=1 << 28):
    """(Y, M) of every graph in `rows`, made by ensemble_generate over
    consecutive chunks of `chunk` members (one workspace reused; the batch
    sequence is enqueued directly, since every chunk is a new table)."""
    import numpy as np
    Ys, Ms = [], []
    ws = None
    tu = sfg.ensemble_tuning(max_batch_edges, 8, 8, graph=False)
    for c0 in range(0, len(rows), chunk):
        part = rows[c0:c0 + chunk]
        descs = sfg.graph_descs(part)
        need = sfg.ensemble_workspace_bytes(descs, max_batch_edges)
        if ws is None or ws.numel() < need:
            ws = None
            torch.cuda.empty_cache()
            ws = sfg.workspace(need)
        hist, gamma, closed = sfg.ensemble_generate(descs, num_samples=samples, stat_seed=stat_seed, ws=ws,
                                                    tuning=tu, check=True)
        Y, M = targets(part, hist.cpu().numpy().astype(np.float64), gamma.cpu().numpy(), closed.cpu().numpy(),
                       samples)
        Ys.append(Y)
        Ms.append(M)
    del ws
    torch.cuda.empty_cache()
    return np.concatenate(Ys, 0), np.concatenate(Ms, 0)


def ensemble_study(rows, *, targets_gamma=tuple(round(2.1 + 0.1 * i, 1) for i in range(10)), k=14, tol=0.05,
                   budget=40, heldout=4096, epochs=60, lr=2e-3, samples=10_000, stat_seed=5, judge_seeds=(31,),
                   model_seed=1, log=None):
    """Train the surrogate on the statistics of the ensemble `rows` (the
    generators' own output), then fit the 2x2 Kronecker initiator
    [[a, 1-a], [b, 1-b]] at k levels to every target exponent twice: with
    the surrogate-guided search and with the generator-only search, each
    judged by the real generator.  A target is reported infeasible when
    neither search reaches it within the budget; the surrogate's closest
    prediction over its inversion starts is reported beside it.  Returns a
    dict of the figures (generator calls and seconds per target, with and
    without the surrogate)."""
    import time

    import numpy as np
    t0 = time.perf_counter()
    Y, M = generate_dataset_chunked(rows, samples=samples, stat_seed=stat_seed)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    if log:
        log(f"dataset: {len(rows)} graphs in {gen_s:.1f} s")
    X = features(rows)
    n_train = len(rows) - heldout
    model = Surrogate(batch=4096, seed=model_seed)
    t1 = time.perf_counter()
    hist = model.fit(X[:n_train], Y[:n_train], M[:n_train], epochs=epochs, lr=lr)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t1
    pred = Surrogate.gamma_of(model.predict(X[n_train:]))
    ok = M[n_train:, GAMMA_COL] > 0
    y = Surrogate.gamma_of(Y[n_train:])[ok]
    err = np.abs(pred[ok] - y)
    if log:
        log(f"fit: {epochs} epochs in {fit_s:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}, "
            f"held-out median |gamma error| {np.median(err):.4f}")
    judge = Judge(k=k, seeds=judge_seeds, samples=2000)
    per = []
    for i, t in enumerate(targets_gamma):
        _, gpred = invert(model, float(t), k, seed=1000 + i)
        ta = time.perf_counter()
        ok1, c1 = search_with_surrogate(model, judge, float(t), tol, budget=budget, seed=i)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ok2, c2 = search_generator_only(judge, float(t), tol, budget=budget, seed=i)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        per.append({"target": float(t), "feasible": bool(ok1 or ok2),
                    "predicted_closest": float(gpred[0]),
                    "with_surrogate": {"reached": bool(ok1), "generator_calls": int(c1), "seconds": tb - ta},
                    "generator_only": {"reached": bool(ok2), "generator_calls": int(c2), "seconds": tc - tb}})
        if log:
            log(f"target {t}: with surrogate {c1} calls ({'ok' if ok1 else 'missed'}), "
                f"generator only {c2} ({'ok' if ok2 else 'missed'})")
    feasible = [p for p in per if p["feasible"]]

    def mean(key, field):
        return float(np.mean([p[key][field] for p in feasible])) if feasible else None

    return {"train_graphs": n_train, "heldout_graphs": heldout, "dataset_s": gen_s, "fit_s": fit_s,
            "epochs": epochs, "loss_first": hist[0], "loss_last": hist[-1],
            "heldout_median_gamma_error": float(np.median(err)), "family": f"2x2 [[a,1-a],[b,1-b]], k={k}",
            "tolerance": tol, "budget": budget, "targets": per,
            "infeasible": [p["target"] for p in per if not p["feasible"]],
            "mean_calls_with_surrogate": mean("with_surrogate", "generator_calls"),
            "mean_calls_generator_only": mean("generator_only", "generator_calls"),
            "mean_seconds_with_surrogate": mean("with_surrogate", "seconds"),
            "mean_seconds_generator_only": mean("generator_only", "seconds")}
