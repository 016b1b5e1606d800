"""Scaling analysis of S(t, k) (Eq. (1)): recovery of known exponents from
spectra built exactly from the scaling form, the infrared constraint
alpha = d beta, independence of the reference time, bootstrap errors."""
import numpy as np
import pytest

from paper_2310_03636_amd import scaling


def scaling_form(t, k, t_ref, alpha, beta, zeta=2.6):
    """S(t, k) = (t/t_ref)^alpha f((t/t_ref)^beta k), f(x) = (1 + x^2)^(-zeta/2)."""
    s = (t[:, None] / t_ref)
    return s ** alpha * (1.0 + (s ** beta * k[None, :]) ** 2) ** (-zeta / 2)


T = np.linspace(200.0, 2000.0, 10)
K = np.exp(np.linspace(np.log(0.01), np.log(10.0), 600))


@pytest.mark.parametrize("alpha,beta", [(0.27, 0.25), (0.5, 0.25), (-0.4, -0.2), (0.0, 0.0)])
def test_recovers_exponents_of_exact_scaling_data(alpha, beta):
    S = scaling_form(T, K, T[3], alpha, beta)
    r = scaling.fit_scaling(T, K, S, T[3], (0.05, 2.0))
    assert abs(r["alpha"] - alpha) < 2e-4 and abs(r["beta"] - beta) < 2e-4, r
    assert r["residual"] < 1e-7 and r["points"] > 100


def test_infrared_constraint_and_reference_time():
    d = 2
    S = scaling_form(T, K, T[0], d * 0.21, 0.21)
    a = scaling.fit_scaling(T, K, S, T[0], (0.05, 1.0), alpha_per_beta=d)
    assert abs(a["beta"] - 0.21) < 2e-4 and abs(a["alpha"] - d * a["beta"]) < 1e-12
    # the exponents do not depend on which time serves as reference
    b = scaling.fit_scaling(T, K, S, T[6], (0.05, 1.0), alpha_per_beta=d)
    assert abs(a["beta"] - b["beta"]) < 3e-4


def test_bootstrap_errors_cover_the_truth():
    rng = np.random.default_rng(5)
    S = scaling_form(T, K, T[4], 0.3, 0.25)
    samples = S[:, None, :] * rng.exponential(1.0, size=(T.size, 40, K.size))  # Wigner-like spread
    r = scaling.bootstrap_scaling(T, K, samples, T[4], (0.05, 2.0), n_boot=30, seed=1)
    assert r["alpha_se"] > 0 and r["beta_se"] > 0
    assert abs(r["alpha"] - 0.3) < 4 * r["alpha_se"] + 1e-3
    assert abs(r["beta"] - 0.25) < 4 * r["beta_se"] + 1e-3


def test_input_checks():
    S = scaling_form(T, K, T[0], 0.3, 0.25)
    with pytest.raises(ValueError):
        scaling.fit_scaling(T, K, S[:, :-1], T[0], (0.1, 1.0))
    with pytest.raises(ValueError):
        scaling.fit_scaling(T, K, -S, T[0], (0.1, 1.0))
    with pytest.raises(ValueError):
        scaling.fit_scaling(T, K, S, 123.0, (0.1, 1.0))
    with pytest.raises(ValueError):
        scaling.fit_scaling(T, K, S, T[0], (5.0, 5.001))
