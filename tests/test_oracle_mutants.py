"""The pins are sharp: each plausible mistake planted in a copy of the oracle's
source (on the CPU, in a temporary directory) makes at least one pin fail."""
import os
import shutil
import subprocess

import pytest

import oracle
from tests import pins

# (name, original text, mistaken text); each original must occur exactly once
MUTANTS = [
    ("drop_ND_factor", "(double)nd * log(S)", "log(S)"),
    ("conjugate_V_in_sum", "r += vr * ar - vi * ai;", "r += vr * ar + vi * ai;"),
    ("imag_sign_in_sum", "i += vr * ai + vi * ar;", "i += vr * ai - vi * ar;"),
    ("conj_wrong_operand", "nadd(&g[2 * a + 1], ar * ui - ai * ur);", "nadd(&g[2 * a + 1], ai * ur - ar * ui);"),
    ("u_without_1_over_I", "ur = zr / I;", "ur = zr;"),
    ("mc_weight_dropped_in_S", "nadd(&t, wj * I);", "nadd(&t, I);"),
    ("mc_weight_dropped_in_grad", "ur = wj * zr;", "ur = zr;"),
    ("intensity_minus", "double I = zr * zr + zi * zi;\n        double ur", "double I = zr * zr - zi * zi;\n        double ur"),
    ("c_missing_ngen", "c = (double)nd / s_raw;", "c = (double)nd / S;"),
    ("ext_c_missing_ngen", "c = 1.0 / n_gen;", "c = 1.0;"),
    ("grad_factor_2", "grad[a] = 2.0 * (-GD[a] + c * HM[a]);", "grad[a] = (-GD[a] + c * HM[a]);"),
    ("grad_sign", "grad[a] = 2.0 * (-GD[a] + c * HM[a]);", "grad[a] = 2.0 * (GD[a] - c * HM[a]);"),
    ("gram_transposed", "nadd(&acc[2 * (a * k + b) + 1], wj * (ar * bi - ai * br));",
     "nadd(&acc[2 * (a * k + b) + 1], wj * (ai * br - ar * bi));"),
    ("gram_no_ngen", "M[e] = (nm > 0) ? nval(&acc[e]) / n_gen : 0.0;", "M[e] = (nm > 0) ? nval(&acc[e]) : 0.0;"),
    ("gram_S_conj", "Si += V[2 * a] * i - V[2 * a + 1] * r;\n    }", "Si += V[2 * a] * i - V[2 * a + 1] * r;\n        Sr -= 2 * V[2 * a + 1] * i;\n    }"),
    ("gram_MV_index", "double mr = M[2 * (a * k + b)], mi = M[2 * (a * k + b) + 1];",
     "double mr = M[2 * (b * k + a)], mi = M[2 * (b * k + a) + 1];"),
    ("extended_uses_log", "*nll = -sum_log + S;", "*nll = -sum_log + log(S);"),
    ("no_compensation", "if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;\n    else                       a->c += (x - t) + a->s;", ""),
]


def _fails_some_pin(orc):
    failed = []
    for pin in pins.PINS:
        try:
            pin(orc)
        except Exception as e:   # AssertionError, or an error a broken oracle raises
            failed.append(pin.__name__)
    return failed


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(mut), out=str(tmp_path / "libmut.so"))
    failed = _fails_some_pin(oracle.Oracle(lib))
    assert failed, f"mutant {name} passed every pin"
