"""Writes the stored expected values under tests/golden/ from oracle/closed_forms.py.

Run from the repository root:  python tests/golden/make_golden.py
It calls nothing but ``oracle.closed_forms`` (closed forms and 1-D quadratures);
no value comes from a random walk or from the HIP path.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import closed_forms as cf  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    alphas = [float(a) for a in np.linspace(0.5, 0.99, 16).astype(np.float32)]
    plane = {
        "what": "total diffuse reflectance and its albedo derivative, isotropic scattering, "
                "index-matched boundary, normal incidence, semi-infinite homogeneous medium: "
                "R = 1 - H(1) sqrt(1 - alpha) (Chandrasekhar, Radiative Transfer, ch. V)",
        "generator": "tests/golden/make_golden.py -> oracle.closed_forms.R_plane / dR_plane_dalpha",
        "alpha": alphas,
        "R": [cf.R_plane(a) for a in alphas],
        "dR_dalpha": [cf.dR_plane_dalpha(a) for a in alphas],
    }
    with open(os.path.join(HERE, "plane_albedo_16.json"), "w") as f:
        json.dump(plane, f, indent=1)

    ss = {
        "what": "single-scattering contribution per unit albedo (exactly one collision, then "
                "transmission through the smooth Fresnel surface), normal incidence, "
                "semi-infinite Henyey-Greenstein medium",
        "generator": "tests/golden/make_golden.py -> oracle.closed_forms.R1_total",
        "cases": [{"g": g, "n": n, "R1": cf.R1_total(1.0, g, n)}
                  for g in (0.0, 0.5, 0.9) for n in (1.0, 1.4)],
    }
    with open(os.path.join(HERE, "single_scatter.json"), "w") as f:
        json.dump(ss, f, indent=1)


if __name__ == "__main__":
    main()
