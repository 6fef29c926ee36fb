"""Training and use of the learned warm start (see gmgm_ws_* in gmgm.h).

Orchestration only: features, targets, the network, its gradient, the
optimiser and the solves all run in the library's kernels.
"""
from __future__ import annotations

import numpy as np

import paper_2407_19892_amd as g


class WarmStart:
    """Parameters (FP32 master copy) and AdamW state of the warm-start network
    on one device.  Training and inference run the BF16-weight mode
    (gmgm_warmstart_train_step / gmgm_warmstart_infer: BF16 operands on the
    matrix cores, FP32 accumulation); the weight decay is fixed at creation."""

    def __init__(self, seed: int = 0, device: str = "cuda", weight_decay: float = 1e-4):
        import torch
        n = g.ws_param_count()
        dev = torch.device(device)
        self.params = torch.empty(n, dtype=torch.float32, device=dev)
        g.ws_init(self.params, seed)
        self.state = g.warmstart_state(weight_decay=weight_decay, device=dev.index)

    @property
    def step(self):
        return int(self.state[:8].cpu().numpy().view("int64")[0])

    def train_step(self, feats, targets, mask=None, lr=1e-3, want_loss=True):
        return g.warmstart_train_step(self.params, self.state, feats, targets, mask, lr, want_loss)

    def infer(self, feats):
        """Network outputs (batch x 1024) of a batch of features."""
        return g.warmstart_infer(self.params, feats)

    def predict(self, Ec, Eg, dc, dg):
        """Warm-start eigenvalues (lam_c, lam_g) of one axis pair."""
        f = g.ws_features(Ec, Eg, dc, dg)
        y = g.warmstart_infer(self.params, f.view(1, -1))
        return g.ws_apply(y.view(-1), Ec, Eg)

    def solve(self, Ec, Eg, dc, dg, tol=1e-12, max_iter=200):
        """gmgm_solve_eigs of the pair started from the network's prediction."""
        lc, lg = self.predict(Ec, Eg, dc, dg)
        return g.solve_eigs([Ec, Eg], [(0, 1)], warm=[lc, lg], tol=tol, max_iter=max_iter)

    def state_dict(self):
        return {"params": self.params.cpu(), "state": self.state.cpu()}

    def load_state_dict(self, sd):
        self.params.copy_(sd["params"])
        self.state.copy_(sd["state"])


def make_examples(pairs, tol=1e-12, max_iter=200):
    """Features and targets of solved axis pairs.

    pairs: iterable of (Ec, Eg, dc, dg) with FP64 device spectra.  Each pair is
    solved from the cold start by gmgm_solve_eigs; returns (feats, targets) as
    (N, 1028) and (N, 1024) FP32 device tensors and the cold iteration counts."""
    import torch
    feats, targs, iters = [], [], []
    for Ec, Eg, dc, dg in pairs:
        r = g.solve_eigs([Ec, Eg], [(0, 1)], tol=tol, max_iter=max_iter)
        feats.append(g.ws_features(Ec, Eg, dc, dg))
        targs.append(g.ws_targets(Ec, r.lam[0], Eg, r.lam[1]))
        iters.append(r.info["iterations"])
    return torch.stack(feats), torch.stack(targs), iters


def train(model: WarmStart, feats, targets, steps: int, batch: int = 64, lr: float = 1e-3, seed: int = 0,
          loss_every: int = 1):
    """Minibatch AdamW on (feats, targets); returns the loss of every
    `loss_every`-th step (reading a loss back synchronises)."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = feats.shape[0]
    losses = []
    for s in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=gen).to(feats.device)
        want = (s % loss_every == 0) or s == steps - 1
        loss = model.train_step(feats[idx].contiguous(), targets[idx].contiguous(), lr=lr, want_loss=want)
        if want:
            losses.append(loss)
    return losses


# ---------------------------------------------------------------------------
# The warm start at the scale of its training recipe: spectra of NB/log1p data
# of the three workloads' generator (axis sizes log-uniform in 200..20000,
# 8..40 clusters of equal or Zipf sizes, dense or 5%-sparse counts), the
# smaller axis' Gram and FP64 eigendecomposition in the library, cold solves
# with the cell axis at ranks 25, 50, 100, 200 and (up to 512) full.

def _draw_instance(rng, beta_sparse):
    n = int(round(float(np.exp(rng.uniform(np.log(200), np.log(20_000))))))
    p = int(round(float(np.exp(rng.uniform(np.log(200), np.log(20_000))))))
    ncl = int(rng.integers(8, 41))
    zipf = bool(rng.random() < 0.5)
    beta0 = 0.0 if rng.random() < 0.5 else beta_sparse[ncl]
    return n, p, ncl, zipf, beta0


def gram_spectrum(X):
    """Nonzero spectrum (FP64, descending, numerical rank) of the smaller
    axis' Gram of a dense device matrix, through gmgm_gram and gmgm_eigh_small."""
    import torch
    A = X if X.shape[0] >= X.shape[1] else X.t().contiguous()
    m, q = A.shape
    rp = torch.arange(m + 1, dtype=torch.int64, device=A.device) * q
    col = torch.arange(q, dtype=torch.int32, device=A.device).repeat(m)
    G = g.gram(rp, col, A.reshape(-1), m, q)
    del rp, col
    w, _, rank = g.eigh_small(G, vectors=False)
    return w[:rank].contiguous()


_BETA = {}


def _sparse_beta(seed=77):
    """beta0 giving a 5% nonzero fraction per cluster count (calibrated at 8, 24
    and 40 clusters, the nearest used in between)."""
    import synth
    if seed in _BETA:
        return _BETA[seed]
    cal = {}
    for ncl in (8, 24, 40):
        labels = synth.cluster_labels(2000, ncl, True, seed)
        cal[ncl] = synth._calibrate_beta0(0.05, 2000, ncl, labels, seed)
    _BETA[seed] = {ncl: cal[min(cal, key=lambda c: abs(c - ncl))] for ncl in range(8, 41)}
    return _BETA[seed]


def spectra_stream(seed, count, budget_s=None, log=None):
    """Yields (Ec_full, n, p) for `count` seeded instances (fewer if the time
    budget runs out)."""
    import time
    import synth
    rng = np.random.default_rng(seed)
    beta_sparse = _sparse_beta()
    t0 = time.perf_counter()
    for i in range(count):
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            return
        n, p, ncl, zipf, beta0 = _draw_instance(rng, beta_sparse)
        X = synth.nb_log1p_gpu(n, p, ncl, zipf, seed * 1_000_003 + i, beta0=beta0)
        E = gram_spectrum(X)
        del X
        if log and i % 100 == 0:
            log(f"instance {i}: {n} x {p}, rank {E.numel()}, {time.perf_counter() - t0:.0f} s")
        yield E, n, p


FULL_RANK_MAX = 512


def _ranks(m):
    """Cell-axis ranks solved per instance: 50 and 100 (the 100k x 2000 and
    1M x 20k workloads' ranks), 25 and 200 around them (clipped to m), and the
    full rank when the spectrum is at most FULL_RANK_MAX long (the 2000 x 500
    workload's r = 500; a full-rank pair of longer spectra makes the Newton
    system the whole smaller axis, too slow to repeat thousands of times)."""
    rs = {min(m, 25), min(m, 50), min(m, 100), min(m, 200)}
    if m <= FULL_RANK_MAX:
        rs.add(m)
    return sorted(rs)


def build_dataset(seed, n_solves, budget_s, tol=1e-12, log=None):
    """Features and targets of cold solves (every instance solved at each of
    its cell-axis ranks): returns feats (N x 1028), targets (N x 1024) on the
    device, the cold iteration counts and the instance sizes."""
    import torch
    feats, targs, iters, sizes = [], [], [], []
    for E, n, p in spectra_stream(seed, 10 ** 9, budget_s, log):
        for rc in _ranks(E.numel()):
            Ec = E[:rc].contiguous()
            r = g.solve_eigs([Ec, E], [(0, 1)], tol=tol, max_iter=300, raise_on_noconv=False)
            if not r.info["converged"]:
                continue
            feats.append(g.ws_features(Ec, E, n, p))
            targs.append(g.ws_targets(Ec, r.lam[0], E, r.lam[1]))
            iters.append(r.info["iterations"])
            sizes.append((n, p, rc, E.numel()))
        if len(feats) >= n_solves:
            break
    return torch.stack(feats), torch.stack(targs), iters, sizes


def evaluate(model, seed, count, tol=1e-12, log=None):
    """Cold vs warm (features + network + apply + solve) on `count` fresh
    instances: iterations, wall time and the warm result's distance from the
    cold one (in units of the solver's parity bar, 1e-10 relative plus 1e-12 of
    the axis maximum)."""
    import time
    import torch
    rows = []
    rng = np.random.default_rng(seed + 1)
    for E, n, p in spectra_stream(seed, count, None, log):
        rc = int(rng.choice(_ranks(E.numel())))
        Ec = E[:rc].contiguous()
        torch.cuda.synchronize()
        t = time.perf_counter()
        cold = g.solve_eigs([Ec, E], [(0, 1)], tol=tol, max_iter=300, raise_on_noconv=False)
        torch.cuda.synchronize()
        t_cold = time.perf_counter() - t
        t = time.perf_counter()
        warm = model.solve(Ec, E, n, p, tol=tol, max_iter=300)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t
        err = 0.0
        for x, y in zip(warm.lam, cold.lam):
            bar = 1e-10 * y.abs() + 1e-12 * y.max()
            err = max(err, float(((x - y).abs() / bar).max().item()))
        rows.append({"n": n, "p": p, "r_c": rc, "r_g": E.numel(), "cold_iters": cold.info["iterations"],
                     "warm_iters": warm.info["iterations"], "cold_s": t_cold, "warm_s": t_warm,
                     "warm_used": warm.info["warm_used"], "converged": bool(cold.info["converged"] and
                                                                           warm.info["converged"]),
                     "err_over_bar": err})
    return rows


def train_and_evaluate(out_path, seed=10_000, n_solves=20_000, budget_s=720.0, steps=4000, batch=512,
                       lr=1e-3, eval_count=512):
    """Build the training set (cold solves), train in the BF16-weight mode,
    evaluate on fresh instances; writes a JSON report and the weights."""
    import json
    import sys
    import time
    import torch

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    g.load()
    t0 = time.perf_counter()
    feats, targs, iters, sizes = build_dataset(seed, n_solves, budget_s, log=log)
    t_data = time.perf_counter() - t0
    log(f"dataset: {feats.shape[0]} solves from {len(set(s[:2] for s in sizes))} instances in {t_data:.0f} s")
    model = WarmStart(seed=3, weight_decay=1e-5)
    t0 = time.perf_counter()
    losses = train(model, feats, targs, steps=steps, batch=batch, lr=lr, seed=0, loss_every=100)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {steps} steps in {t_train:.0f} s: loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    rows = evaluate(model, seed + 500_000, eval_count, log=log)
    ok = [r for r in rows if r["converged"]]
    ci = np.array([r["cold_iters"] for r in ok], float)
    wi = np.array([r["warm_iters"] for r in ok], float)
    cs = np.array([r["cold_s"] for r in ok])
    ws = np.array([r["warm_s"] for r in ok])
    errs = np.array([r["err_over_bar"] for r in ok])
    nn = np.array([max(r["r_c"], r["r_g"]) for r in ok])
    rep = {"train": {"solves": int(feats.shape[0]), "instances": len(set((s[0], s[1]) for s in sizes)),
                     "axis_sizes": [int(min(min(s[0], s[1]) for s in sizes)), int(max(max(s[0], s[1]) for s in sizes))],
                     "spectrum_sizes": [int(min(s[3] for s in sizes)), int(max(s[3] for s in sizes))],
                     "cold_iterations_mean": float(np.mean(iters)), "data_s": t_data, "steps": steps,
                     "batch": batch, "train_s": t_train, "loss_first": losses[0], "loss_last": losses[-1],
                     "mode": "BF16 operands on MFMA, FP32 accumulation, FP32 master weights"},
           "eval": {"instances": len(rows), "converged": len(ok),
                    "cold_iterations_mean": float(ci.mean()), "warm_iterations_mean": float(wi.mean()),
                    "iterations_saved_frac": float(1 - wi.sum() / ci.sum()),
                    "cold_s_total": float(cs.sum()), "warm_s_total_incl_inference": float(ws.sum()),
                    "wall_time_saved_frac": float(1 - ws.sum() / cs.sum()),
                    "cold_s_median": float(np.median(cs)), "warm_s_median": float(np.median(ws)),
                    "large_r_over_2000": {"count": int((nn > 2000).sum()),
                                          "cold_s": float(cs[nn > 2000].sum()),
                                          "warm_s": float(ws[nn > 2000].sum())},
                    "warm_used_frac": float(np.mean([r["warm_used"] for r in ok])),
                    "psi_err_over_bar_max": float(errs.max()), "psi_within_bar_frac": float(np.mean(errs <= 1))},
           "eval_rows": rows,
           }
    with open(out_path, "w") as f:
        json.dump(rep, f, indent=1)
    torch.save({"params": model.params.cpu()}, out_path.replace(".json", "_weights.pt"))
    log(json.dumps(rep["eval"]))
    return rep


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="build the warm-start training set, train, evaluate")
    ap.add_argument("--out", required=True)
    ap.add_argument("--budget", type=float, default=720.0, help="seconds for building the training set")
    ap.add_argument("--solves", type=int, default=20_000)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--eval", type=int, default=512)
    a = ap.parse_args()
    train_and_evaluate(a.out, n_solves=a.solves, budget_s=a.budget, steps=a.steps, eval_count=a.eval)
