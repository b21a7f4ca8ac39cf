"""Writes closed_forms.json: compositing closed forms evaluated with Python's
``decimal`` module at 40 significant digits.  Independent of the oracle.

Homogeneous density sigma on n midpoint bins of width dt starting at t0
(bin centres t_i = t0 + (i+1/2) dt), q = exp(-sigma dt), w_i = q^i (1-q):

  T_n = q^n = exp(-sigma n dt)                            (Eq. 6 telescoped)
  A   = 1 - q^n
  d*  = a (1-q^n) + dt q (1 - n q^(n-1) + (n-1) q^n)/(1-q),   a = t0 + dt/2
  M2  = (1-q) [a^2 S0 + 2 a dt S1 + dt^2 S2],  S_k = sum_{i<n} i^k q^i
  V*  = M2 - d*^2 (2 - A)

with the geometric sums S0 = (1-q^n)/(1-q),
S1 = q (1 - n q^(n-1) + (n-1) q^n)/(1-q)^2 and
S2 = q(1+q)/(1-q)^3 - q^n [n^2/(1-q) + 2 n q/(1-q)^2 + q(1+q)/(1-q)^3].

Cases:
  homogeneous: sigma = 1 on [1, 3], n = 32 (the tiny workload's sampler).
  slab:        the tiny workload's centre pixel (16,16) through the analytic
               sphere (radius 0.5, density 50): bins 8..23 of the same
               sampler lie inside, so the ray sees sigma = 50 on n = 16 bins
               starting at t0 = 1.5 and nothing elsewhere.
"""
import json
import os
from decimal import Decimal, getcontext

getcontext().prec = 40


def closed_form(sigma, t0, dt, n):
    sigma, t0, dt = Decimal(sigma), Decimal(t0), Decimal(dt)
    q = (-sigma * dt).exp()
    one = Decimal(1)
    qn = q ** n
    a = t0 + dt / 2
    S0 = (one - qn) / (one - q)
    S1 = q * (one - n * q ** (n - 1) + (n - 1) * qn) / (one - q) ** 2
    S2 = q * (one + q) / (one - q) ** 3 - qn * (Decimal(n * n) / (one - q)
                                                 + 2 * n * q / (one - q) ** 2
                                                 + q * (one + q) / (one - q) ** 3)
    A = one - qn
    d = a * A + dt * (one - q) * S1
    M2 = (one - q) * (a * a * S0 + 2 * a * dt * S1 + dt * dt * S2)
    V = M2 - d * d * (2 - A)
    return dict(T_end=str(qn), opacity=str(A), depth=str(d), var=str(V))


if __name__ == "__main__":
    out = dict(
        source="closed forms of Eq. 5/6 with midpoint bins; see make_closed_forms.py",
        homogeneous=dict(sigma="1", t0="1", dt="0.0625", n=32, **closed_form("1", "1", "0.0625", 32)),
        slab=dict(sigma="50", t0="1.5", dt="0.0625", n=16, **closed_form("50", "1.5", "0.0625", 16)),
    )
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
