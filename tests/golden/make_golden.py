"""Writes the closed-form fixtures under tests/golden/.

tgv2d_decay.json: the 2D Taylor-Green vortex u = u0 exp(-2 nu k^2 t)(sin x cos y,
-cos x sin y) is an exact solution of the incompressible Navier-Stokes equations
(Taylor & Green 1937).  With the lattice viscosity nu = (tau - 1/2)/3 (paper,
Sec. 3.1) and k = 2 pi / n this gives the velocity amplitude and the kinetic energy
ratio at the listed steps for the 64x64, tau = 0.6, u0 = 0.05 workload.  The
tolerance is the one the BGK truncation error O(k^2) allows (Krueger 2016, Sec. 4.5).

Run:  python tests/golden/make_golden.py
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def tgv2d(n=64, tau=0.6, u0=0.05, steps=(0, 100, 250, 500, 750, 1000)):
    nu = (tau - 0.5) / 3.0
    k = 2.0 * math.pi / n
    rate = 2.0 * nu * k * k
    return {
        "source": "Taylor-Green closed form; nu = (tau-1/2)/3 from the paper's Sec. 3.1",
        "n": n, "tau": tau, "u0": u0,
        "t": list(steps),
        "amplitude": [math.exp(-rate * t) for t in steps],
        "energy_ratio": [math.exp(-2.0 * rate * t) for t in steps],
        "rel_tol": 1e-2,
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "tgv2d_decay.json"), "w") as fh:
        json.dump(tgv2d(), fh, indent=1)
        fh.write("\n")
