"""Write the textbook oblique-shock values used by the ramp plateau test.

Relations (NACA Report 1135, oblique shock, perfect gas): for upstream Mach
M1 and deflection theta the weak-shock angle beta solves
  tan(theta) = 2 cot(beta) (M1^2 sin^2 beta - 1) / (M1^2 (gamma + cos 2 beta) + 2)
and with Mn1 = M1 sin beta:
  p2/p1   = 1 + 2 gamma/(gamma+1) (Mn1^2 - 1)
  rho2/rho1 = (gamma+1) Mn1^2 / ((gamma-1) Mn1^2 + 2)
  Mn2^2   = (1 + (gamma-1)/2 Mn1^2) / (gamma Mn1^2 - (gamma-1)/2),  M2 = Mn2 / sin(beta - theta)
"""
import json
import math
import os

from scipy.optimize import brentq


def oblique(M1, theta_deg, gamma=1.4):
    th = math.radians(theta_deg)

    def f(b):
        return (2.0 / math.tan(b) * (M1 ** 2 * math.sin(b) ** 2 - 1.0)
                / (M1 ** 2 * (gamma + math.cos(2 * b)) + 2.0) - math.tan(th))

    mu = math.asin(1.0 / M1)
    beta = brentq(f, mu + 1e-9, math.radians(64.0))  # weak branch lies below the max-deflection angle
    Mn1 = M1 * math.sin(beta)
    p21 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (Mn1 ** 2 - 1.0)
    r21 = (gamma + 1.0) * Mn1 ** 2 / ((gamma - 1.0) * Mn1 ** 2 + 2.0)
    Mn2 = math.sqrt((1.0 + 0.5 * (gamma - 1.0) * Mn1 ** 2) / (gamma * Mn1 ** 2 - 0.5 * (gamma - 1.0)))
    M2 = Mn2 / math.sin(beta - th)
    return {"M1": M1, "theta_deg": theta_deg, "gamma": gamma, "beta_deg": math.degrees(beta),
            "p2_p1": p21, "rho2_rho1": r21, "T2_T1": p21 / r21, "M2": M2,
            "source": "oblique-shock relations, NACA Report 1135 (perfect gas)"}


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oblique_shock_M2p5_10deg.json")
    with open(out, "w") as fh:
        json.dump(oblique(2.5, 10.0), fh, indent=2)
        fh.write("\n")
    print(open(out).read())
