"""Training and use of the learned warm start (see gmgm_ws_* in gmgm.h).

Orchestration only: features, targets, the network, its gradient, the
optimiser and the solves all run in the library's kernels.
"""
from __future__ import annotations

import paper_2407_19892_amd as g


class WarmStart:
    """Parameters and AdamW state of the warm-start network on one device."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        import torch
        n = g.ws_param_count()
        self.params = torch.empty(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.step = 0
        g.ws_init(self.params, seed)

    def train_step(self, feats, targets, mask=None, lr=1e-3, weight_decay=1e-4, want_loss=True):
        self.step += 1
        return g.ws_train_step(self.params, self.m, self.v, self.step, feats, targets, mask, lr, weight_decay,
                               want_loss)

    def predict(self, Ec, Eg, dc, dg):
        """Warm-start eigenvalues (lam_c, lam_g) of one axis pair."""
        f = g.ws_features(Ec, Eg, dc, dg)
        y = g.ws_forward(self.params, f.view(1, -1))
        return g.ws_apply(y.view(-1), Ec, Eg)

    def solve(self, Ec, Eg, dc, dg, tol=1e-12, max_iter=200):
        """gmgm_solve_eigs of the pair started from the network's prediction."""
        lc, lg = self.predict(Ec, Eg, dc, dg)
        return g.solve_eigs([Ec, Eg], [(0, 1)], warm=[lc, lg], tol=tol, max_iter=max_iter)

    def state_dict(self):
        return {"params": self.params.cpu(), "m": self.m.cpu(), "v": self.v.cpu(), "step": self.step}

    def load_state_dict(self, sd):
        self.params.copy_(sd["params"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step = int(sd["step"])


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


def train(model: WarmStart, feats, targets, steps: int, batch: int = 64, lr: float = 1e-3,
          weight_decay: float = 1e-4, seed: int = 0):
    """Minibatch AdamW on (feats, targets); returns the loss of every step."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = feats.shape[0]
    losses = []
    for _ in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=gen).to(feats.device)
        losses.append(model.train_step(feats[idx].contiguous(), targets[idx].contiguous(), lr=lr,
                                       weight_decay=weight_decay))
    return losses
