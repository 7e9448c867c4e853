"""Plants plausible mistakes in copies of the oracle's C source (on the CPU)
and checks that the pins in test_oracle_pins catch every one of them: a
dropped term, a wrong sign, a transposed index, a swapped operand, the
textbook 2 l^2 in place of eq. (1)'s printed 2 l, noise put on the wrong
covariance. The error metrics (Python) get the same treatment: a mutated
copy of each metric function replaces it, and the hand-worked metric pins
must fail."""
import inspect
import os
import subprocess
import textwrap

import pytest

import oracle
from oracle import build as obuild
import test_oracle_pins as pins

MUTANTS = [
    ("exponent uses 2 l^2", "exp(-sqdist(a, b, D) / (2 * l))", "exp(-sqdist(a, b, D) / (2 * l * l))"),
    ("noise dropped from K", "if (i == j) k += s2r;", ";"),
    ("noise on cross covariance", "Ks[i * n + j] = kse(Xs + i * D, X + j * D, D, lr, vr);",
     "Ks[i * n + j] = kse(Xs + i * D, X + j * D, D, lr, vr) + (i == j ? s2r : 0);"),
    ("noise on test covariance", "real s = kse(Xs + i * D, Xs + j * D, D, lr, vr);",
     "real s = kse(Xs + i * D, Xs + j * D, D, lr, vr) + (i == j ? s2r : 0);"),
    ("distance skips first feature", "for (int d = 0; d < D; ++d) {", "for (int d = 1; d < D; ++d) {"),
    ("pivot sign", "d -= Lj[k] * Lj[k];", "d += Lj[k] * Lj[k];"),
    ("off-diagonal uses row j twice", "s -= Li[k] * Lj[k];", "s -= Lj[k] * Lj[k];"),
    ("backward substitution transposed", "s -= L[k * n + i] * x[k];", "s -= L[i * n + k] * x[k];"),
    ("mean uses beta", "Ks[i * n + j] * alpha[j]", "Ks[i * n + j] * beta[j]"),
    ("covariance sign", "s -= vi[k] * vj[k];", "s += vi[k] * vj[k];"),
    ("forward substitution drops division", "x[i] = s / L[i * n + i];\n    }\n}\n\n/* Backward",
     "x[i] = s;\n    }\n}\n\n/* Backward"),
    ("lengthscale gradient misses 1/l", "s / (2 * lr * lr)", "s / (2 * lr)"),
    ("logdet halved", "quad / 2 + logdet +", "quad / 2 + logdet / 2 +"),
    ("noise gradient uses off-diagonal", "if (i == j) rows[i] = a;", "if (j == 0) rows[i] = a;"),
]

# cheap pins first; each mutant must fail at least one
PINS = [
    pins.test_kernel_closed_form_points,
    pins.test_kernel_matrix_structure,
    lambda: pins.test_cholesky_vs_lapack(17),
    pins.test_substitutions_vs_scipy,
    lambda: pins.test_predict_vs_gauss_jordan(8, 5),
    pins.test_mean_identity_test_equals_train,
    pins.test_cov_identity_test_equals_train,
    pins.test_nlml_closed_form_n1,
    pins.test_nlml_closed_form_n2,
    lambda: pins.test_gradient_vs_finite_differences((0.3, 2.0, 0.5)),
]


def _build_mutant(tmp_path, src, name):
    path = tmp_path / f"m_{abs(hash(name))}.c"
    path.write_text(src)
    out = tmp_path / f"m_{abs(hash(name))}.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fopenmp", "-fPIC", "-shared",
                    "-DOR_REAL=double", str(path), "-o", str(out), "-lm"], check=True)
    return str(out)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, monkeypatch, name, old, new):
    src = open(obuild.SRC).read()
    assert old in src, f"mutation site not found: {old!r}"
    so = _build_mutant(tmp_path, src.replace(old, new), name)
    real_lib = oracle._lib("double")      # ensure the signatures are set up once
    import ctypes
    mlib = ctypes.CDLL(so)
    for attr in ["orc_kernel_matrix", "orc_assemble_K", "orc_cholesky", "orc_forward",
                 "orc_backward", "orc_predict", "orc_nlml_grad", "orc_gauss_jordan_inverse"]:
        f, g = getattr(real_lib, attr), getattr(mlib, attr)
        g.argtypes, g.restype = f.argtypes, f.restype
    monkeypatch.setitem(oracle._LIBS, "double", mlib)
    for pin in PINS:
        try:
            pin()
        except (AssertionError, oracle.OracleError, ZeroDivisionError, FloatingPointError):
            return
    pytest.fail(f"no pin caught mutant: {name}")


def test_unmutated_oracle_passes_all_listed_pins():
    for pin in PINS:
        pin()


METRIC_MUTANTS = [
    ("rel_err divides by ||A||", "rel_err", "nb = float(np.linalg.norm(B))",
     "nb = float(np.linalg.norm(A))"),
    ("rel_err uses the max norm", "rel_err", "d = float(np.linalg.norm(A - B))",
     "d = float(np.max(np.abs(A - B)))"),
    ("rel_err without the division", "rel_err", "return d / nb if nb > 0 else d", "return d"),
    ("rel_err squared norms", "rel_err", "return d / nb if nb > 0 else d",
     "return (d / nb) ** 2 if nb > 0 else d"),
    ("rel_err_lower takes upper triangles", "rel_err_lower",
     "return rel_err(np.tril(A), np.tril(B))", "return rel_err(np.triu(A), np.triu(B))"),
    ("rel_err_lower drops the diagonal", "rel_err_lower",
     "return rel_err(np.tril(A), np.tril(B))", "return rel_err(np.tril(A, -1), np.tril(B, -1))"),
    ("max_rel signed max", "max_rel", "mb = float(np.max(np.abs(B))) if B.size else 0.0",
     "mb = float(np.max(B)) if B.size else 0.0"),
    ("max_rel uses the mean difference", "max_rel",
     "md = float(np.max(np.abs(A - B))) if A.size else 0.0",
     "md = float(np.mean(np.abs(A - B))) if A.size else 0.0"),
]

METRIC_PINS = [pins.test_rel_err_hand_values, pins.test_rel_err_lower_hand_values,
               pins.test_max_rel_hand_values]


@pytest.mark.parametrize("name,func,old,new", METRIC_MUTANTS, ids=[m[0] for m in METRIC_MUTANTS])
def test_metric_pins_catch_mutant(monkeypatch, name, func, old, new):
    src = textwrap.dedent(inspect.getsource(getattr(oracle, func)))
    assert old in src, f"mutation site not found: {old!r}"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    monkeypatch.setattr(oracle, func, ns[func])
    if func == "rel_err":
        # rel_err_lower calls rel_err through the module namespace
        src_l = textwrap.dedent(inspect.getsource(oracle.rel_err_lower))
        exec(compile(src_l, "<rel_err_lower>", "exec"), ns)
        monkeypatch.setattr(oracle, "rel_err_lower", ns["rel_err_lower"])
    for pin in METRIC_PINS:
        try:
            pin()
        except AssertionError:
            return
    pytest.fail(f"no metric pin caught mutant: {name}")


def test_unmutated_metrics_pass_their_pins():
    for pin in METRIC_PINS:
        pin()
