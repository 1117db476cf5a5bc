"""The oracle's pins are strong enough to catch plausible mistakes: each test
plants one mistake in a copy of oracle/pdhcg_oracle.c, compiles it, and
checks that at least one pin of tests/test_oracle_pins.py or
tests/test_oracle_adaptive.py fails against it.
CPU only; the planted copies live in a temporary directory."""
import os
import subprocess

import pytest

import test_oracle_adaptive as adaptive
import test_oracle_pins as pins
from oracle import oracle as O

SRC = os.path.join(os.path.dirname(O.__file__), "pdhcg_oracle.c")

# (name, original text, mistaken text) -- every mutation keeps memory safety
MUTATIONS = [
    ("dual step sign", "yn[i] = fmax(0.0, y[i] + sigma *", "yn[i] = fmax(0.0, y[i] - sigma *"),
    ("no extrapolation", "(2.0 * Axn[i] - Ax[i] - b[i])", "(Axn[i] - b[i])"),
    ("average weight", "double w = 1.0 / (double)(k + 1);", "double w = 1.0 / (double)(k + 2);"),
    ("gap sign", "fabs(xQx + cx + by)", "fabs(xQx + cx - by)"),
    ("dual residual drops A'y", "fabs(Qx[j] + Aty[j] + c[j])", "fabs(Qx[j] + c[j])"),
    ("CG residual update sign", "r[j] -= alpha * q[j];", "r[j] += alpha * q[j];"),
    ("proximal term scaled wrongly", "q[j] += p[j] / tau;", "q[j] += p[j] * tau;"),
    ("CG direction update", "p[j] = r[j] + beta * p[j];", "p[j] = r[j];"),
    ("primal weight mixes scales", "(1.0 - theta) * log(omega)", "(1.0 - theta) * omega"),
    ("restart condition (ii) direction", "K_c <= beta_nec * K_anchor && K_c > K_prev", "K_c <= beta_nec * K_anchor && K_c < K_prev"),
    ("step size uses ||A|| instead of 1/||A||", "s->eta_factor / (normA > 0.0 ? normA : 1.0)", "s->eta_factor * (normA > 0.0 ? normA : 1.0)"),
    ("primal residual ignores b", "maxp(Ax[i] - b[i], 0.0)", "maxp(Ax[i], 0.0)"),
    ("CG stop certificate without tau", "tau * sqrt(rho_new) <= eps", "sqrt(rho_new) <= eps"),
    ("power iteration normalisation", "v[j] = w[j] / lam;", "v[j] = w[j];"),
    # adaptive step size (Sec. 4)
    ("step limit drops the Q term", "double den = 2.0 * fabs(dot(m, dy, Adx)) + dot(n, dx, Qdx);",
     "double den = 2.0 * fabs(dot(m, dy, Adx));"),
    ("step limit bilinear term by sign", "double den = 2.0 * fabs(dot(m, dy, Adx)) + dot(n, dx, Qdx);",
     "double den = 2.0 * dot(m, dy, Adx) + dot(n, dx, Qdx);"),
    ("step limit weights inverted", "double num = omega * dot(n, dx, dx) + dot(m, dy, dy) / omega;",
     "double num = dot(n, dx, dx) / omega + omega * dot(m, dy, dy);"),
    ("step update exponents swapped", "double a = (1.0 - pow((double)t + 1.0, -0.3)) * eta_bar;",
     "double a = (1.0 - pow((double)t + 1.0, -0.6)) * eta_bar;"),
    ("acceptance test reversed", "int accept = eta <= eta_bar || attempts >= 64;",
     "int accept = eta >= eta_bar || attempts >= 64;"),
    ("repeated trial keeps the old tau", "            tau = eta / omega;\n            sigma = eta * omega;\n            if (accept) break;",
     "            sigma = eta * omega;\n            if (accept) break;"),
]

PINS = [
    pins.test_relkkt_worked_example,
    pins.test_relkkt_dual_gap_signs,
    pins.test_first_two_iterations_exact_cg,
    pins.test_first_iteration_cg_capped_at_one_step,
    pins.test_opnorm_matches_svd,
    pins.test_cg_to_convergence_matches_dense_solve,
    pins.test_cg_one_step_closed_form,
    pins.test_cg_stop_rule_and_error_bound,
    pins.test_primal_weight_worked_value,
    pins.test_invariants_along_iterations,
    pins.test_manufactured_solution_tiny_case_size,
    pins.test_warm_start_resume_and_negative_y0,
    adaptive.test_step_limit_worked_example,
    adaptive.test_next_step_closed_form,
    adaptive.test_first_adaptive_iteration_on_w_is_accepted,
    adaptive.test_rejected_trial_on_w,
] + [lambda row=row: pins.test_restart_decision_table(row) for row in pins._load_restart_table()]


def build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(path), "-lm"])
    return str(lib)


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    O.use_library(build_mutant(tmp_path, old, new))
    caught = []
    try:
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                caught.append(getattr(pin, "__name__", "restart table"))
                break
    finally:
        O.use_library(None)
    assert caught, f"no pin caught the planted mistake: {name}"
