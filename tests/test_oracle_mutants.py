"""The driver pins fail when the oracle carries the slip each one targets (CPU).

Each case copies the oracle's C sources, plants one plausible mistake by a textual replacement, builds the copy
into a separate library and runs the pins of tests/test_oracle_driver_pins.py against it: at least one of the
listed pins must fail.  The committed oracle is never modified.
"""
import glob
import os
import shutil
import subprocess

import pytest

from tests import test_oracle_driver_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

CFL = [lambda m, n=n: pins.test_cfl_step_closed_form(m, n) for n in pins.CFL_CASES]
PRE = [lambda m, a=a: pins.test_tuning_pre_smoothing_stop_test(m, *a) for a in
       (("constant", 0.0, 1), ("orthogonal", None, 4), ("mixed", 0.05, 1), ("mixed", 0.2, 4))]
FIX = [pins.test_tuning_exact_fixed_point]
FMG = [pins.test_fmg_threshold_met_everywhere, pins.test_fmg_threshold_never_met,
       pins.test_fmg_threshold_crossed_after_two_cycles]

MUTANTS = {
    # CFL step, Sec. 2
    "size_J_over_Ja": ("residual.c", "double h = 2.0 * L->J[o + p] /", "double h = 1.0 * L->J[o + p] /", CFL),
    "order_plus_one": ("residual.c", "double N = L->ord[3 * e + d];", "double N = L->ord[3 * e + d] + 1;", CFL),
    "nu_without_rho": ("residual.c", "double nu = or_mu(ph, T) / (rho * ph->reynolds);",
                       "double nu = or_mu(ph, T) / (ph->reynolds);", CFL),
    # smoothing tuning, Sec. 3.1.2
    "pre_test_not_strict": ("multigrid.c", "if (or_norm_inf(Rfine, n) < prm->eta * or_norm_inf(rc, 5 * Lc->nn))",
                            "if (or_norm_inf(Rfine, n) <= prm->eta * or_norm_inf(rc, 5 * Lc->nn))", FIX + PRE),
    "pre_test_unrestricted": ("multigrid.c", "if (or_norm_inf(Rfine, n) < prm->eta * or_norm_inf(rc, 5 * Lc->nn))",
                              "if (or_norm_inf(Rfine, n) < prm->eta * or_norm_inf(Rfine, n))", FIX + PRE),
    "eta_on_wrong_side": ("multigrid.c", "if (or_norm_inf(Rfine, n) < prm->eta * or_norm_inf(rc, 5 * Lc->nn))",
                          "if (prm->eta * or_norm_inf(Rfine, n) < or_norm_inf(rc, 5 * Lc->nn))", FIX + PRE),
    "post_test_strict": ("multigrid.c", "if (or_norm_inf(R, n) <= rnorm_pre) break;",
                         "if (or_norm_inf(R, n) < rnorm_pre) break;", FIX),
    # FMG start, Sec. 3.1.1
    "fmg_test_inverted": ("multigrid.c", "if (r < prm->fmg_threshold || cycles >= max_cycles) break;",
                          "if (r > prm->fmg_threshold || cycles >= max_cycles) break;", FMG),
    "fmg_no_restriction": ("multigrid.c",
                           "for (int l = top; l > 0; l--) or_restrict(P, mg->L[l], mg->L[l - 1], mg->Q[l], mg->Q[l - 1]);",
                           "for (int l = top; l > 0; l--) memset(mg->Q[l - 1], 0, 0);", FMG),
}


@pytest.fixture
def mutant(tmp_path, monkeypatch):
    from oracle import oracle as O

    def make(fname, old, new):
        src = tmp_path / "src"
        src.mkdir()
        for f in glob.glob(os.path.join(ORACLE, "*.[ch]")):
            shutil.copy(f, src)
        text = (src / fname).read_text()
        assert text.count(old) == 1, (fname, old)
        (src / fname).write_text(text.replace(old, new))
        lib = tmp_path / "liboracle_mutant.so"
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib)] +
                       sorted(str(p) for p in src.glob("*.c")) + ["-lm"], check=True)
        monkeypatch.setattr(O, "LIB", str(lib))
        monkeypatch.setattr(O, "_lib", None)
        return O

    yield make


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_catch_the_slip(mutant, name):
    fname, old, new, checks = MUTANTS[name]
    O = mutant(fname, old, new)
    failed = 0
    for check in checks:
        try:
            check(O)
        except AssertionError:
            failed += 1
    assert failed > 0, f"no pin caught the planted slip {name}"
