"""Writes the stored expected values under tests/golden/ (calls the oracle only).

chebyshev_scaling.json: for the bounds a = 2, b = 12.5, a0 = -3 of Algorithm 1
(Sec. 3.4), the scaling values T_m(tau) and the first ten sigma_k, with
T_m(tau) evaluated from the hyperbolic closed form
T_m(t) = sign(t)^m cosh(m arccosh|t|), |t| > 1, independently of the oracle's
recurrences.
"""
import json
import math
import os

a, b, a0 = 2.0, 12.5, -3.0
e, c = (b - a) / 2, (b + a) / 2
tau = (a0 - c) / e


def t_closed(m, t):
    return math.copysign(1.0, t) ** m * math.cosh(m * math.acosh(abs(t)))


out = {
    "source": "closed form of Chebyshev polynomials outside [-1, 1]; bounds of the "
              "full-size filter workload (Algorithm 1, Sec. 3.4)",
    "a": a, "b": b, "a0": a0,
    "T_m_tau": {str(m): t_closed(m, tau) for m in (1, 2, 10, 16, 20, 24)},
    "sigma_1_to_10": [t_closed(k - 1, tau) / t_closed(k, tau) for k in range(1, 11)],
}
here = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(here, "chebyshev_scaling.json"), "w") as f:
    json.dump(out, f, indent=1)
