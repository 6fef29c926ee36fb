"""Inputs built so that the operand rounding of a low-precision sweep pulls the
true largest |Psi_ij| of a row below a block of decoys.

Row `row` of Psi = V diag(1) V^T (psi = 1, so W = V) is built on the first
`r1` coordinates around 1, where the operand format keeps p significant bits
and u = 2^-p (BF16 u = 2^-8; FP8 e4m3 u = 2^-4 after its power-of-two scale):
  - the row itself and a hidden column h: entries a = 1 + u - u^2/2, which
    round DOWN to 1 (exact Psi_ih = r1 a^2 ~ r1 (1 + 2u), rounded value r1);
  - k "D" columns: two entries 1 + u + u^2/2 (round UP to 1 + 2u), the rest
    just below 1 + u/2 (round to 1); exact ~ r1 (1 + 1.5u), rounded r1 + 4u;
    their exact values are spread so that no two are within 1e-6 relative;
  - cap - k small decoys: one entry 1 + u + u^2/2, the rest 1 - u/2 + u^2/2
    (round UP to 1); exact ~ r1 (1 + u/2), rounded r1 + 2u.
So in rounded arithmetic the decoys fill a candidate list of length `cap`
ahead of h, although h's exact value is the largest.  The error on h is
~2 u ||W_row|| ||V_h||: a rounding bound that charges only u per product of two
rounded operands lets a certificate accept the decoys.

A second block on the remaining coordinates holds a row `tie_row` whose
largest values are `n_tie` identical columns (exact ties), more than the
candidate lists of both half rows of an FP32 sweep hold (2 x 32): no list can
certify it, so it reaches the exact scan of the whole row.

Every other row is small background noise.  Only inputs are built here.
"""
import numpy as np

U = {"bf16": 2.0 ** -8, "fp8": 2.0 ** -4}


def aligned_rounding_rows(prec="bf16", k=1, n=2048, r=100, cap=32, n_tie=72, seed=0):
    u = U[prec]
    r1 = r // 2
    rng = np.random.default_rng(seed)
    V = (rng.standard_normal((n, r)) * 1e-3).astype(np.float32)
    row, h = 5, 70
    d_cols = list(range(h + 1, h + 1 + k))
    s_cols = list(range(h + 1 + k, h + cap + 1))
    a = np.float32(1 + u - u * u / 2)
    up = np.float32(1 + u + u * u / 2)
    for j in [row, h]:
        V[j, :] = 0
        V[j, :r1] = a
    step = u / 64      # per-entry spread of the D columns (stays below the rounding midpoints)
    for q, j in enumerate(d_cols):
        V[j, :] = 0
        V[j, :r1] = np.float32(1 + u / 2 - q * step)
        V[j, :2] = up
    for j in s_cols:
        V[j, :] = 0
        V[j, :r1] = np.float32(1 - u / 2 + u * u / 2)
        V[j, 0] = up
    tie_row = 300
    tie_cols = list(range(400, 400 + n_tie))
    for j in [tie_row] + tie_cols:
        V[j, :] = 0
        V[j, r1:] = 1.0
    psi = np.ones(r, np.float64)
    return {"V": V, "psi": psi, "row": row, "hidden": h, "d_cols": d_cols, "s_cols": s_cols,
            "tie_row": tie_row, "tie_cols": tie_cols, "r1": r1, "u": u,
            # a threshold between the hidden value and everything else of the row
            "thr": float(r1 * (1 + 1.6 * u))}
