"""Writes solver_closed_forms.json from closed forms derived by hand from the
eigenvalue-gradient Proposition (no oracle code is used).

single_pair: r_c = r_g = 1 and E_c = E_g = E.  Stationarity gives
  E = 1/(psi + phi); Algorithm 1's start lambda^0 = 1/E has psi - phi = 0 and
  Newton/gradient steps keep psi - phi, so psi = phi = 1/(2E).
box: r_c = 1, r_g = 2, E_g = (E_ga, E_gb) descending, E_ga + E_gb > E_c >= 2 E_gb.
  With phi_a pinned at eps_g: psi + phi_b = 1/E_gb and E_c = 1/(psi + eps_g) + E_gb,
  so psi = 1/(E_c - E_gb) - eps_g and phi_b = 1/E_gb - psi; the pinned
  coordinate's gradient 1/2 (E_ga - (E_c - E_gb)) is >= 0.  (eps_g depends on the
  default 1e-10 / max E_g, so the test evaluates these formulas itself.)
"""
import json
import os

single = [{"E": E, "psi": 1.0 / (2 * E), "phi": 1.0 / (2 * E)} for E in (3.0, 0.25, 1234.5)]
box = [{"Ec": 4.5, "Eg": [3.0, 2.0]}, {"Ec": 7.0, "Eg": [6.0, 3.0]}, {"Ec": 2.5, "Eg": [2.0, 1.0]}]
out = {"source": "eigenvalue-gradient Proposition (appendix on the MLE) + Existence lemma box",
       "single_pair": single, "box": box}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "solver_closed_forms.json"), "w") as f:
    json.dump(out, f, indent=1)
