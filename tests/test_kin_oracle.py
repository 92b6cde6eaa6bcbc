"""The kinematic-amplitude oracle (oracle/kin.c) against its pins, and each
plausible mistake planted in a copy of kin.c caught by at least one pin (CPU)."""
import shutil

import pytest

import oracle
from tests import kin_pins


@pytest.mark.parametrize("pin", kin_pins.PINS, ids=lambda p: p.__name__[4:])
def test_pin(pin):
    pin(oracle.default())


# (name, original text, mistaken text); each original occurs exactly once in kin.c
MUTANTS = [
    ("width_sign", "1.0 / (ma * ma - m * m - _Complex_I * ma * ga)", "1.0 / (ma * ma - m * m + _Complex_I * ma * ga)"),
    ("width_without_mass", "1.0 / (ma * ma - m * m - _Complex_I * ma * ga)", "1.0 / (ma * ma - m * m - _Complex_I * ga)"),
    ("mass_not_squared", "1.0 / (ma * ma - m * m - _Complex_I * ma * ga)", "1.0 / (ma - m - _Complex_I * ma * ga)"),
    ("ylm_norm_2pi", "sqrt((2.0 * J + 1.0) / (4.0 * pi))", "sqrt((2.0 * J + 1.0) / (2.0 * pi))"),
    ("bonnet_coefficient", "((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0)", "((2.0 * n + 1.0) * x * p1 - n * p0) / n"),
    ("dm_sign_of_width", "-(2.0 * ma - _Complex_I * ga) * b2", "-(2.0 * ma + _Complex_I * ga) * b2"),
    ("dm_factor_2", "-(2.0 * ma - _Complex_I * ga) * b2", "-(ma - _Complex_I * ga) * b2"),
    ("dg_not_imaginary", "_Complex_I * ma * b2", "ma * b2"),
    ("dI_without_2", "kadd(&gr[2 * a], ce * 2.0 * creal(q * dm));", "kadd(&gr[2 * a], ce * creal(q * dm));"),
    ("bw_not_squared", "const double complex b2 = bw[a] * bw[a];", "const double complex b2 = bw[a];"),
    ("q_without_y", "conj(z) * V[a] * y[a];", "conj(z) * V[a];"),
    ("res_grad_sign", "grad_res[i] = -RD[i] + c * RM[i];", "grad_res[i] = RD[i] + c * RM[i];"),
    ("res_grad_mc_dropped", "grad_res[i] = -RD[i] + c * RM[i];", "grad_res[i] = -RD[i];"),
    ("mc_weight_dropped", "ce = w ? w[e] : 1.0;", "ce = 1.0;"),
    ("v_conj", "z += V[a] * bw[a] * y[a];", "z += conj(V[a]) * bw[a] * y[a];"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(oracle.KIN_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mut = tmp_path / "kin_mut.c"
    mut.write_text(src.replace(old, new))
    lib = oracle.build(force=True, out=str(tmp_path / "libmut.so"), kin_src=str(mut))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in kin_pins.PINS:
        try:
            pin(orc)
        except Exception:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
