"""Mistakes planted in copies of the oracle's restart rule are caught.

Each case copies ``oracle/pdhg_oracle.c``, changes one expression of the
Section 2.4.2 / Algorithm 4 logic, builds the copy with gcc on the CPU and
runs the restart pins of test_oracle.py against it: at least one of them must
fail.  This keeps those pins able to tell the rule as the paper states it from
plausible misreadings of it.
"""
import os

import pytest

import test_oracle as T

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "pdhg_oracle.c")

OMEGA_UPDATE = ("                if (o->use_pw_update && dx > o->eps_zero && dy > o->eps_zero)\n"
                "                    omega = exp(0.5 * log(dy / dx) + 0.5 * log(omega));\n")
NEW_REF = "                kkt0 = kkt_omega(ks_cand, omega);\n"

MUTANTS = {
    # "no progress" read as an improvement
    "progress_inverted": ("kw_cand > kkt_prev) restart = 1;", "kw_cand < kkt_prev) restart = 1;"),
    # the new epoch's reference value taken at the old primal weight
    "reference_at_old_omega": (OMEGA_UPDATE + "                /* the new epoch's reference value is the "
                               "candidate's metric at the new omega */\n" + NEW_REF,
                               NEW_REF + OMEGA_UPDATE),
    # beta_necessary in place of beta_sufficient
    "sufficient_0.8": ("if (kw_cand <= o->beta_suff * kkt0) restart = 1;",
                       "if (kw_cand <= o->beta_nec * kkt0) restart = 1;"),
    # ties of the candidate go to the iterate
    "tie_to_iterate": ("int cand_avg = o->use_restarts && !(kw_c < kw_a);",
                       "int cand_avg = o->use_restarts && !(kw_c <= kw_a);"),
    # the previous candidate survives a restart
    "prev_kept": ("                kkt_prev = INFINITY;\n                t_inner = 0;",
                  "                kkt_prev = kw_cand;\n                t_inner = 0;"),
    # Delta_x / Delta_y swapped in Algorithm 4
    "omega_swapped": ("log(dy / dx) + 0.5", "log(dx / dy) + 0.5"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_restart_pins_reject_mutant(orc, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = orc._load(orc.build(force=True, src=str(path), out=str(tmp_path / "libmut.so")))
    failures = []
    for check in [lambda: T.check_golden_1x1(orc, lib)] + \
                 [lambda c=c: T.check_restart_properties(orc, c, lib) for c in sorted(T.RESTART_CASES)]:
        try:
            check()
        except AssertionError as e:
            failures.append(str(e)[:200])
    assert failures, f"mutant {name} passes every restart pin"
