"""Runs the oracle pin battery against one build of the oracle source.

Usage: python -m tests.mutation_runner <liborc.so> [rocrand_ref_exe]
Exit status 0 when every check passes, 1 as soon as one fails (its name and
detail are printed).  Used by test_oracle_mutations.py on copies of the oracle
with planted mistakes; the checks are ordered cheapest first."""
import math
import sys

import numpy as np
from scipy import integrate

from oracle import closed_forms as cf
from oracle import oracle as O
from tests import oracle_pins as P

# Philox4x32-10 blocks produced by rocRAND's engine (from tests/rocrand_philox_ref.cpp)
# are compared when the helper executable is given.


def pieces(rr_exe):
    if rr_exe:
        import subprocess
        ctrs = [[0, 0, 0, 0], [1, 2, 3, 4], [7, 4000000000, 123, 99], [5, 17, 3, 0]]
        keys = [[0, 0], [5, 6], [3, 4], [11, 0]]
        lines = "\n".join(" ".join(map(str, c + k)) for c, k in zip(ctrs, keys)) + "\n"
        out = subprocess.run([rr_exe], input=lines, capture_output=True, text=True, check=True)
        ref = np.array([[int(t) for t in ln.split()] for ln in out.stdout.strip().splitlines()])
        for c, k, r in zip(ctrs, keys, ref):
            if not np.array_equal(O.philox([c], k)[0].astype(np.int64), r):
                return False, "philox vs rocRAND"
    if not (O.u01(0) == 2.0 ** -24 and O.u01(0xFFFFFFFF) == 1 - 2.0 ** -24):
        return False, "u01 end points"
    for n in (1.4, 1.6):
        for c in np.linspace(0.0, 1.0, 41):
            if abs(O.fresnel(c, n) - cf.fresnel_hecht(c, n)) > 1e-12:
                return False, "fresnel vs Hecht"
    for g in (0.0, 0.5, 0.9):
        for u in (0.1, 0.5, 0.9):
            p, _ = integrate.quad(lambda m: float(cf.hg_pdf(m, g)), -1.0, O.hg_cos(g, u))
            if abs(p - u) > 1e-9:
                return False, "HG inverse CDF"
        for mu in (-0.5, 0.5):
            h = 1e-6
            fd = (math.log(cf.hg_pdf(mu, g + h)) - math.log(cf.hg_pdf(mu, g - h))) / (2 * h)
            if abs(O.hg_dlog_dg(g, mu) - fd) > 1e-5 * max(1, abs(fd)):
                return False, "HG score"
    return True, ""


ORDER = ["energy", "special", "plane", "beer", "mixture", "single_scatter", "analog", "scale",
         "brute", "adj_plane", "adj_mixture", "jacobian", "second_moment", "trace", "spherical",
         "analog_cosine", "layers_trace", "layers_beer", "layers_plane", "layers_absorbing_top",
         "layers_adj_absorbing_top",
         "layers_stack", "layers_analog", "hero_reductions", "hero_closed_forms",
         "dwivedi_nu0", "dwivedi_telescope", "dwivedi_vs_plain", "dwivedi_closed_forms",
         "adding_doubling"]


def main():
    lib_path = sys.argv[1]
    rr_exe = sys.argv[2] if len(sys.argv) > 2 else None
    battery = dict(P.BATTERY_SMALL)
    with O.use_library(lib_path):
        ok, detail = pieces(rr_exe)
        if not ok:
            print(f"FAIL pieces: {detail}")
            return 1
        for name in ORDER:
            try:
                ok, detail = battery[name]()
            except Exception as e:  # a broken oracle may also reject its own input
                ok, detail = False, f"raised {e!r}"
            if not ok:
                print(f"FAIL {name}: {detail}")
                return 1
        ok, detail = P.check_adjoint_vs_crn_fd(paths=1 << 13, reps=6, k=5.0)
        if not ok:
            print(f"FAIL adj_fd: {detail}")
            return 1
    print("PASS")
    return 0


if __name__ == "__main__":
    sys.exit(main())
