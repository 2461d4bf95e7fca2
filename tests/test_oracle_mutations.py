"""The pins are sharp: plausible mistakes planted in the numpy oracle (on the
CPU, by monkeypatching) make at least one pin fail.  Each mutant is restored
after its check."""

import math

import numpy as np
import pytest

from oracle import gl_oracle as go

from . import test_oracle_pins as pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _run_pins():
    """Run a set of pin checks against gl_oracle; return names that failed."""
    failed = []
    checks = {
        "golden": lambda: pins.test_two_node_golden(go, "two_node.json"),
        "golden_unnormalized": lambda: pins.test_two_node_golden(go, "two_node_unnormalized.json"),
        "laplacian": lambda: pins.test_laplacian_properties(go, 1),
        "power": lambda: pins.test_power_method_closed_form(go, "C7", pins._cycle(7),
                                                            1 - math.cos(2 * math.pi * 3 / 7)),
        "sweeps_damped": lambda: pins.test_sweeps_closed_form(go, "damped_jacobi", 3, math.inf),
        "sweeps_richardson": lambda: pins.test_sweeps_closed_form(go, "richardson", 3, math.inf),
        "sweeps_k": lambda: pins.test_sweeps_closed_form(go, "perturbed_jacobi", 3, 0.5),
        "energy": pins.test_energy_double_sum_form,
        "decay": lambda: pins.test_energy_decreases(go, "damped_jacobi", 1),
        "fixed_point": lambda: pins.test_fixed_point_on_cycle(go),
    }
    for name, fn in checks.items():
        try:
            fn()
        except (AssertionError, ValueError, np.linalg.LinAlgError, FloatingPointError):
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_every_pin():
    assert _run_pins() == []


_orig = {name: getattr(go, name) for name in
         ("rhs", "double_well_grad", "precond_diag", "normalized_weights", "fidelity",
          "energy", "normalized_adjacency", "operator_parts")}


def _m_grad_sign(u, eps):
    return -(u ** 3 - u) / eps


def _m_rhs_no_fidelity(u, lam, y, eps, c, eta):
    return c * u - go.double_well_grad(u, eps)


def _m_rhs_wrong_c(u, lam, y, eps, c, eta):
    return u - go.double_well_grad(u, eps) + eta * lam[:, None] * y


def _m_precond_half(kind, lam, eps, c, eta, delta0=1e-6, lambda_max=2.0, step_k=math.inf, d=None):
    return 0.5 * _orig["precond_diag"](kind, lam, eps, c, eta, delta0, lambda_max, step_k, d)


def _m_precond_no_eta(kind, lam, eps, c, eta, delta0=1e-6, lambda_max=2.0, step_k=math.inf, d=None):
    return _orig["precond_diag"](kind, 0 * lam, eps, c, eta, delta0, lambda_max, step_k, d)


def _m_precond_no_degree(kind, lam, eps, c, eta, delta0=1e-6, lambda_max=2.0, step_k=math.inf,
                         d=None):
    # the unnormalized preconditioners with D replaced by I
    return _orig["precond_diag"](kind, lam, eps, c, eta, delta0, lambda_max, step_k, None)


def _m_parts_normalized(n, row_ptr, col, w, laplacian="normalized"):
    # the unnormalized Laplacian silently replaced by L_s
    return _orig["operator_parts"](n, row_ptr, col, w, "normalized")


def _m_weights_row_only(n, row_ptr, col, w):
    d = go.degrees(n, row_ptr, col, w)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    return w / d[rows]


def _m_weights_wrong_index(n, row_ptr, col, w):
    d = go.degrees(n, row_ptr, col, w)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    return w / np.sqrt(d[rows] * d[rows])


def _m_fidelity_flip(labels, K):
    lam, y = _orig["fidelity"](labels, K)
    return lam, -y


def _m_energy_factor(n, row_ptr, col, w, U, labels, eps, eta, laplacian="normalized"):
    U2 = np.asarray(U, dtype=np.float64)
    if U2.ndim == 1:
        U2 = U2[:, None]
    lam, y = go.fidelity(labels, U2.shape[1])
    LU = go.laplacian_apply(n, row_ptr, col, w, U2, laplacian)
    return eps * (U2 * LU).sum(0) + ((U2 ** 2 - 1) ** 2).sum(0) / (4 * eps) \
        + 0.5 * eta * (lam[:, None] * (U2 - y) ** 2).sum(0)


MUTANTS = {
    "double_well_grad sign": ("double_well_grad", _m_grad_sign),
    "rhs drops fidelity": ("rhs", _m_rhs_no_fidelity),
    "rhs uses 1 for c": ("rhs", _m_rhs_wrong_c),
    "preconditioner halved": ("precond_diag", _m_precond_half),
    "preconditioner drops eta Lambda": ("precond_diag", _m_precond_no_eta),
    "random-walk normalisation": ("normalized_weights", _m_weights_row_only),
    "degree index i for j": ("normalized_weights", _m_weights_wrong_index),
    "labels sign flipped": ("fidelity", _m_fidelity_flip),
    "energy Laplacian factor": ("energy", _m_energy_factor),
    "unnormalized preconditioner without D": ("precond_diag", _m_precond_no_degree),
    "unnormalized Laplacian replaced by L_s": ("operator_parts", _m_parts_normalized),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(go, attr, fn)
    failed = _run_pins()
    assert failed, f"mutant '{name}' passed every pin"
