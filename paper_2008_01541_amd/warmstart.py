"""Learned warm start for the collision-region PD iterations.

Frames are solved to convergence with Algorithm 1 (the plain solver); the
network learns the region displacement increment of the next frame from the
previous increment and the active-penalty mask detected at the start of the
frame.  At run time the prediction moves the region nodes before the first
outer iteration; the iterations then run exactly as without it, so the
converged state is still decided by the method.  The plain iteration
converged to a tighter tolerance judges every warm result (evaluate).
Everything here is call order and bookkeeping; the arithmetic runs in the
library's kernels (pd_* and pd_mlp_* entry points).
"""
import time

import numpy as np


def converge(run, tol=1e-6, max_outer=200, n_inner=1):
    """Outer iterations until ||x_k - x_{k-1}|| <= tol ||x_k - X|| (free nodes).
    Returns the number of outer iterations."""
    import torch
    prev = torch.empty_like(run.x)
    for it in range(1, max_outer + 1):
        prev.copy_(run.x)
        run.outer_iteration(n_inner=n_inner)
        d, s = run.ctx.displacement_change(run.x, prev)
        if s == 0.0 or d <= tol * s:
            return it
    return max_outer


def detect_at_start(run):
    """Penalty set of the frame detected at the current positions (fills run.c).
    The network's mask input assumes the runner's node proxies (run.prox)."""
    if run.mode != "nodes":
        raise ValueError("the learned warm start takes node proxies (one mask entry per proxy node)")
    c = run.ctx
    c.region_gather(run.x, run.x2)
    run.detect()


def generate_trajectory(run, centers_fn, radii, n_frames, tol=1e-6, max_outer=200, residual=True):
    """Solve n_frames frames from rest (cold start from the previous frame).
    Returns the network samples (inputs [du_{t-1}, mask_t]; targets du_t, or
    with residual the change du_t - du_{t-1}; unscaled) and the iteration
    counts."""
    import torch
    c = run.ctx
    run.set_positions(run.rest_np)
    m = c.m
    xs, ys, iters = [], [], []
    prev2 = prev1 = None            # region positions two and one frames back
    for fr in range(1, n_frames + 1):
        run.set_spheres(centers_fn(fr), radii)
        detect_at_start(run)
        inp = None
        if prev2 is not None:
            inp = torch.empty(4 * m, dtype=torch.float32, device=run.x.device)
            c.warmstart_input(prev1, prev2, 1.0, run.prox, run.c, inp)
        iters.append(converge(run, tol, max_outer))
        c.region_gather(run.x, run.x2)
        cur = run.x2.clone()
        if inp is not None:
            if residual:
                tgt = torch.empty(3 * m, dtype=torch.float32, device=run.x.device)
                c.warmstart_target(cur, prev1, prev2, 1.0, tgt)
            else:
                tgt = torch.empty(4 * m, dtype=torch.float32, device=run.x.device)
                c.warmstart_input(cur, prev1, 1.0, run.prox, run.c, tgt)   # first 3m = du_t
            xs.append(inp)
            ys.append(tgt[:3 * m].clone())
        prev2, prev1 = prev1, cur
    X = torch.stack(xs) if xs else None
    Y = torch.stack(ys) if ys else None
    return X, Y, iters


class WarmStart:
    """The network 4m -> hidden -> hidden -> 3m.  With residual (default) it
    predicts the change of the region increment from the previous frame's
    (the prediction is du_{t-1} + output), and its output layer starts at zero,
    so before training it is the extrapolation du_t = du_{t-1}."""

    def __init__(self, m, hidden=512, seed=4, max_batch=64, residual=True):
        from pd_inputs.mlp_init import mlp_init_params, pack
        from ._lib import MLP
        self.m = m
        self.residual = residual
        n_in, n_out = 4 * m, 3 * m
        p = mlp_init_params(n_in, hidden, hidden, n_out, seed, out_scale=0.0 if residual else 0.1)
        self.net = MLP(n_in, hidden, hidden, n_out, max_batch, pack(p))
        self.scale = 1.0
        self.max_batch = max_batch

    def close(self):
        self.net.close()

    def train(self, X, Y, epochs=30, lr=1e-3, seed=4):
        """Adam on standardised increments (inputs and targets divided by the
        mean |target|); returns the loss history.  Batches are gathered and
        scaled by the library (pd_mlp_gather_rows) from a seeded permutation."""
        import torch
        s = self.net.abs_mean(Y.contiguous())
        self.scale = 1.0 / s if s > 0 else 1.0
        X = X.contiguous()
        Y = Y.contiguous()
        rng = np.random.default_rng(seed)
        hist = []
        n = X.shape[0]
        B = self.max_batch
        xb = torch.empty((B, X.shape[1]), dtype=torch.float32, device=X.device)
        yb = torch.empty((B, Y.shape[1]), dtype=torch.float32, device=X.device)
        for ep in range(epochs):
            perm = rng.permutation(n).astype(np.int32)
            tot = 0.0
            for b0 in range(0, n, B):
                sel = torch.as_tensor(perm[b0:b0 + B], device=X.device)
                nb = sel.numel()
                self.net.gather_rows(X, sel, xb[:nb], n_scaled=3 * self.m, scale=self.scale)
                self.net.gather_rows(Y, sel, yb[:nb], n_scaled=Y.shape[1], scale=self.scale)
                tot += self.net.train_step(xb[:nb], yb[:nb], lr) * nb
            hist.append(tot / n)
        return hist

    def predict_into(self, run, x2_prev1, x2_prev2, extend=True):
        """Predict du for the next frame and apply it to run.x: with extend
        (default) to the region nodes together with the interior's static
        response to it (pd_warmstart_apply), else to the region nodes alone."""
        import torch
        c = run.ctx
        m = self.m
        inp = torch.empty((1, 4 * m), dtype=torch.float32, device=run.x.device)
        c.warmstart_input(x2_prev1, x2_prev2, self.scale, run.prox, run.c, inp)
        y = torch.empty((1, 3 * m), dtype=torch.float32, device=run.x.device)
        self.net.forward(inp, y)
        if self.residual:
            c.warmstart_apply(y, 1.0 / self.scale, run.x, x2_prev1, x2_prev2)
        elif extend:
            c.warmstart_apply(y, 1.0 / self.scale, run.x)
        else:
            c.region_add_f32(y, 1.0 / self.scale, run.x)


def extrapolate_into(run, x2_prev1, x2_prev2):
    """The non-learned predictor for comparison: the previous frame's region
    increment repeated (applied with the interior's static response)."""
    import torch
    c = run.ctx
    zero = torch.zeros(3 * c.m, dtype=torch.float32, device=run.x.device)
    c.warmstart_apply(zero, 1.0, run.x, x2_prev1, x2_prev2)


def evaluate(run, ws, centers_fn, radii, n_frames, tol=1e-8, judge_tol=1e-9, accept=1e-6,
             max_outer=2000, extend=True, predictor="mlp"):
    """Per frame, from the previous frame's judged state: the judge (the plain
    iteration, no prediction, to ||x_k - x_{k-1}|| <= judge_tol ||x_k - X||),
    the cold start (the same iteration to tol) and the learned warm start
    (prediction, applied with the interior's static response when extend,
    then the same iteration to tol).  A warm result is accepted
    when ||x_warm - x_judge|| <= accept ||x_judge - X||; otherwise the frame
    falls back to the cold solve and is charged both runs (iterations and
    wall time).  The judge's run is a measuring device and is not charged.
    predictor="extrapolate" replaces the network by extrapolate_into.  Each
    record also holds the distance of the cold and warm starting points from
    the judged result (relative to its displacement from rest).
    Returns one record per frame."""
    import torch
    run.set_positions(run.rest_np)
    c = run.ctx
    rows = []
    prev2 = prev1 = None
    for fr in range(1, n_frames + 1):
        run.set_spheres(centers_fn(fr), radii)
        start = run.x.clone()
        detect_at_start(run)
        judge_it = converge(run, judge_tol, max_outer)
        x_judge = run.x.clone()
        run.x.copy_(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it_cold = converge(run, tol, max_outer)
        torch.cuda.synchronize()
        t_cold = time.perf_counter() - t0
        d, s = c.displacement_change(run.x, x_judge)
        d0, _ = c.displacement_change(start, x_judge)
        rec = {"frame": fr, "judge_iters": judge_it, "cold_iters": it_cold, "cold_s": t_cold,
               "cold_rel_diff": d / max(s, 1e-300), "cold_start_err": d0 / max(s, 1e-300)}
        if prev2 is not None:
            run.x.copy_(start)
            detect_at_start(run)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if predictor == "extrapolate":
                extrapolate_into(run, prev1, prev2)
            else:
                ws.predict_into(run, prev1, prev2, extend=extend)
            d0, _ = c.displacement_change(run.x, x_judge)
            it_warm = converge(run, tol, max_outer)
            torch.cuda.synchronize()
            t_warm = time.perf_counter() - t0
            d, s = c.displacement_change(run.x, x_judge)
            rel = d / max(s, 1e-300)
            ok = rel <= accept
            rec.update({"warm_iters": it_warm, "warm_s": t_warm, "rel_diff": rel,
                        "warm_start_err": d0 / max(s, 1e-300),
                        "fell_back": not ok,
                        "charged_iters": it_warm if ok else it_warm + it_cold,
                        "charged_s": t_warm if ok else t_warm + t_cold})
        run.x.copy_(x_judge)
        c.region_gather(run.x, run.x2)
        prev2, prev1 = prev1, run.x2.clone()
        rows.append(rec)
    return rows


def summarize(rows):
    """Totals over the frames that had a warm start."""
    warm = [r for r in rows if "warm_iters" in r]
    if not warm:
        return {}
    cold_it = sum(r["cold_iters"] for r in warm)
    chg_it = sum(r["charged_iters"] for r in warm)
    cold_s = sum(r["cold_s"] for r in warm)
    chg_s = sum(r["charged_s"] for r in warm)
    return {"eval_frames": len(warm),
            "cold_outer_iters_per_frame": cold_it / len(warm),
            "warm_outer_iters_per_frame": sum(r["warm_iters"] for r in warm) / len(warm),
            "charged_outer_iters_per_frame": chg_it / len(warm),
            "iters_saved_frac": 1.0 - chg_it / cold_it if cold_it else None,
            "cold_s_per_frame": cold_s / len(warm),
            "charged_s_per_frame": chg_s / len(warm),
            "wall_saved_frac": 1.0 - chg_s / cold_s if cold_s else None,
            "fell_back": sum(1 for r in warm if r["fell_back"]),
            "cold_start_err_mean": float(np.mean([r["cold_start_err"] for r in warm])),
            "warm_start_err_mean": float(np.mean([r["warm_start_err"] for r in warm])),
            "rel_diff_max": max(r["rel_diff"] for r in warm),
            "cold_rel_diff_max": max(r["cold_rel_diff"] for r in warm)}
