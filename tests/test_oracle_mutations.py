"""Planted mistakes in a copy of the oracle must be caught by its pins (CPU only).

Each case edits one line of oracle/rw_oracle.c the way a plausible slip would
(a dropped term, a wrong sign or index, a transposed operand), builds the copy
in a temporary directory and runs the pin battery of tests/oracle_pins.py
against it in a subprocess.  The unmodified source must pass the same battery.
Nothing here touches the GPU or the product path."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("philox_transposed_products", "uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi0 ^ c1 ^ k0;"),
    ("philox_wrong_multiplier", "uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;",
     "uint64_t p1 = (uint64_t)M0 * (uint64_t)c2;"),
    ("philox_nine_rounds", "round < 10", "round < 9"),
    ("u01_wrong_shift", "((double)(w >> 9) + 0.5) * 0x1p-23", "((double)(w >> 8) + 0.5) * 0x1p-23"),
    ("fresnel_p_amplitude", "double rp = (cos_i - n * cos_t) / (cos_i + n * cos_t);",
     "double rp = (n * cos_i - cos_t) / (n * cos_i + cos_t);"),
    ("fresnel_refracted_cosine", "double cos_t = sqrt(1.0 - sin_t2);",
     "double cos_t = sqrt(1.0 - sin_i2);"),
    ("hg_orientation", "(1.0 - g + 2.0 * g * u)", "(1.0 + g - 2.0 * g * u)"),
    ("hg_score_dropped_term", "return -2.0 * g / (1.0 - g * g) + 3.0 * (mu - g)",
     "return 3.0 * (mu - g)"),
    ("frame_sign", "t2[2] = -d[1];", "t2[2] = d[1];"),
    ("azimuth_sin_cos", "b = st * sin(phi);", "b = st * cos(phi);"),
    ("free_flight_scale", "double s = -log(u[0]) / (dw ? sig_d : sig);",
     "double s = -log(u[0]) * (dw ? sig_d : sig);"),
    ("boundary_distance_sign", "db = -p[2] / d[2];", "db = p[2] / d[2];"),
    ("no_absorption", "W *= alb;", "W *= 1.0;"),
    ("absorbed_after_update", "res->absorbed += W * (1.0 - alb);\n    W *= alb;",
     "W *= alb;\n    res->absorbed += W * (1.0 - alb);"),
    ("roulette_weight", "W /= geo->rr_survive;", "W *= geo->rr_survive;"),
    ("medium_choice_uncumulated", "if (u[0] < up->cum[j])", "if (u[0] < up->w[j])"),
    ("entry_fresnel_dropped", "*W = 1.0 - F_in;", "*W = 1.0;"),
    ("cosine_lobe_not_cosine", "(1.0 - u[1]) / (n * n)", "(1.0 - u[1] * u[1]) / (n * n)"),
    ("cosine_lobe_no_snell", "(1.0 - u[1]) / (n * n)", "(1.0 - u[1])"),
    ("cosine_entry_fresnel_angle", "F_in = fresnel(ct, n);", "F_in = fresnel(st, n);"),
    ("bin_log_origin", "log(r / g->r_min_mm)", "log(r)"),
    ("exit_radius_component", "sqrt(p[0] * p[0] + p[1] * p[1])", "sqrt(p[0] * p[0] + p[2] * p[2])"),
    ("reflect_wrong_component", "d[2] = -d[2];", "d[0] = -d[0];"),
    ("scatter_sign", "scatter_dir(d, mu, 2.0 * M_PI * u[2]);", "scatter_dir(d, -mu, 2.0 * M_PI * u[2]);"),
    ("score_sigma_sign", "score[k] = (double)r.n_coll / up.sigma_t[k] - r.L;",
     "score[k] = (double)r.n_coll / up.sigma_t[k] + r.L;"),
    ("score_alpha_inverted", "(double)r.n_coll / up.albedo[k]", "(double)r.n_coll * up.albedo[k]"),
    ("score_logit_no_baseline", "(j == k ? 1.0 : 0.0) - up.w[j]", "(j == k ? 1.0 : 0.0)"),
    ("boundary_segment_not_counted", "      res->L += db;\n", ""),
    ("hg_score_not_accumulated", "res->Sg += hg_dlog_dg(g, mu);", "res->Sg = hg_dlog_dg(g, mu);"),
    ("interface_index_inverted", "const double rel = lp->n[layer] / lp->n[1 - layer];",
     "const double rel = lp->n[1 - layer] / lp->n[layer];"),
    ("refraction_sign_lost", "d[2] = d[2] > 0.0 ? ct : -ct;", "d[2] = ct;"),
    ("layer_not_switched", "        layer = 1 - layer;\n", ""),
    ("bottom_face_top_index", "const double F = fresnel(fabs(d[2]), lp->n[layer]);",
     "const double F = fresnel(fabs(d[2]), lp->n[0]);"),
    ("flight_top_sigma", "-log(u[0]) / lp->sigma_t[layer]", "-log(u[0]) / lp->sigma_t[0]"),
    ("layer_score_face_length_dropped", "      res->L_l[layer] += db;\n", ""),
    ("layer_score_flight_wrong_layer", "res->L_l[layer] += flight;", "res->L_l[0] += flight;"),
    ("layer_score_collisions_wrong_layer", "res->n_coll_l[layer] += res->n_coll - nc0;",
     "res->n_coll_l[0] += res->n_coll - nc0;"),
    ("refraction_tangent_unscaled", "        d[1] *= rel;\n", ""),
    ("interface_missed_upward", "if (d[2] < 0.0 && zn <= lp->d) { face = 2; zf = lp->d; }",
     "if (d[2] < 0.0 && zn <= 0.0) { face = 2; zf = lp->d; }"),
    ("jacobian_slot_index_transposed", "jacB[(int64_t)r.slot * P + j] += r.x * score[j];",
     "jacB[(int64_t)j * (nb + 2) + r.slot] += r.x * score[j];"),
    ("jacobian_total_times_cotangent", "jacR[j] += r.x * score[j];",
     "jacR[j] += r.x * cot * score[j];"),
    ("hero_no_group_factor", "hw->F[i] = (double)hw->C * hw->x[i] * exp(lp[i] - m) / S;",
     "hw->F[i] = hw->x[i] * exp(lp[i] - m) / S;"),
    ("hero_density_with_hero_sigma", "(double)res->n_coll_l[l] * log(hw->lps[i].sigma_t[l]) -",
     "(double)res->n_coll_l[l] * log(hw->lps[hw->hero].sigma_t[l]) -"),
    ("hero_density_length_sign", "-\n               hw->lps[i].sigma_t[l] * res->L_l[l];",
     "+\n               hw->lps[i].sigma_t[l] * res->L_l[l];"),
    ("hero_phase_density_of_hero_g", "hw->hg[i] += hg_log_pdf(hw->lps[i].g[layer], mu);",
     "hw->hg[i] += hg_log_pdf(hw->lps[hw->hero].g[layer], mu);"),
    ("hero_weight_with_hero_albedo", "hw->x[i] *= hw->lps[i].albedo[layer];",
     "hw->x[i] *= hw->lps[hw->hero].albedo[layer];"),
    ("hero_never_rotates", "const int hero = (int)(pth % C);", "const int hero = 0;"),
    ("dwivedi_flight_sign", "*sig_d = up->sigma_t[k] * (1.0 - *mu_s / nu0);",
     "*sig_d = up->sigma_t[k] * (1.0 + *mu_s / nu0);"),
    ("dwivedi_pdf_no_2pi", "return 1.0 / (2.0 * M_PI * lam * (nu0 - mu_s));",
     "return 1.0 / (lam * (nu0 - mu_s));"),
    ("dwivedi_flight_density_inverted", "(sig_d / sig)", "(sig / sig_d)"),
    ("dwivedi_surface_exp_sign", "exp(sig * mu_s * db / up->nu0[k])",
     "exp(-sig * mu_s * db / up->nu0[k])"),
    ("dwivedi_surface_weight_dropped", "W *= p_hg / (dw_q * p_d * exp(sig * mu_s * db",
     "W = W + 0.0 * p_hg / (dw_q * p_d * exp(sig * mu_s * db"),
    ("dwivedi_inverse_cdf", "const double m = nu0 - (nu0 + 1.0) * exp(-u[1] * lam);",
     "const double m = nu0 - (nu0 - 1.0) * exp(-u[1] * lam);"),
    ("dwivedi_hg_cosine_wrong", "const double c = nd[0] * d[0] + nd[1] * d[1] + nd[2] * d[2];",
     "const double c = nd[2];"),
    ("dwivedi_nu0_bisection", "if (a * f < 1.0) lo = x;", "if (a * f > 1.0) lo = x;"),
]


@pytest.fixture(scope="module")
def rr_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    exe = str(tmp_path_factory.mktemp("rrm") / "rr_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(ROOT, "tests", "rocrand_philox_ref.cpp")],
                          cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def _run(lib, rr, threads=None):
    cmd = [sys.executable, "-m", "tests.mutation_runner", lib] + ([rr] if rr else [])
    env = dict(os.environ)
    if threads:
        env["ORC_THREADS"] = str(threads)
        # the battery's small dense solves (adding-doubling) run one BLAS thread:
        # parallel batteries with a full BLAS pool each oversubscribe the host
        for var in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
            env[var] = "1"
    try:
        p = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=240, env=env)
    except subprocess.TimeoutExpired:
        return None, "timeout"
    return p.returncode, (p.stdout + p.stderr).strip()[-400:]


def test_unmodified_oracle_passes_battery(tmp_path, rr_exe):
    lib = O.compile_source(O.source_text(), str(tmp_path / "liborc_ok.so"))
    rc, out = _run(lib, rr_exe)
    assert rc == 0, out


def test_planted_mistakes_are_caught(tmp_path, rr_exe):
    src = O.source_text()
    libs = []
    for name, old, new in MUTATIONS:
        assert src.count(old) == 1, f"mutation site for {name} not unique"
        libs.append((name, O.compile_source(src.replace(old, new), str(tmp_path / f"liborc_{name}.so"))))
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda nl: (nl[0],) + _run(nl[1], rr_exe, threads=2), libs))
    survivors = [(name, out) for name, rc, out in results if rc == 0]
    assert not survivors, f"planted mistakes not caught: {survivors}"
