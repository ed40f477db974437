"""Planted mistakes in the oracle (CPU only).  Each plausible slip -- the
Euclidean instead of the squared distance, a cross term counted once, a
dropped 1/eps or a flipped sign in the log-sum-exp, the wrong exponent of
the conjugate gradient, a missing 1/p, a flipped McCann step -- is patched
into the oracle module for one test, and a committed pin must then fail;
so are the schedule slips (alpha_k as a share of the whole path, progress
as a plain sum of the alpha_k, eps without its 1/20, Alg. 4's eps_0 without
its 1/20, its hold-out score unsquared or averaged, the warm start scaled by
the previous step's alpha) and the metrics slips
(the divergence without its 1/2, a flipped entropy sign, <P, C> as a
product of sums).
This is what makes the pins a check of the oracle rather than of itself."""
import importlib

import numpy as np
import pytest

import oracle as oracle_pkg
from oracle import metrics, pcost, schedules
import tests.test_oracle_metrics as mpins
import tests.test_oracle_pcost as ppins
import tests.test_oracle_progot as spins
import tests.test_oracle_sinkhorn as pins

# the module (the package re-exports its sinkhorn function under that name)
osk = importlib.import_module("oracle.sinkhorn")

_cost = osk.cost_matrix
_softmin_rows = osk.softmin_rows
_grad_h_star = pcost.grad_h_star
_h_p = pcost.h_p
_map_p = pcost.entropic_map_p


def _cross_term_once(X, Y):
    X, Y = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    return (X ** 2).sum(1)[:, None] + (Y ** 2).sum(1)[None, :] - X @ Y.T


COST_MISTAKES = {
    "euclidean": lambda X, Y: np.sqrt(_cost(X, Y)),
    "cross_term_once": _cross_term_once,
    "half": lambda X, Y: 0.5 * _cost(X, Y),
}

SOFTMIN_MISTAKES = {
    "no_1_over_eps": lambda C, v, eps: _softmin_rows(C, v, 1.0),
    "cost_sign": lambda C, v, eps: _softmin_rows(-C, v, eps),
}


@pytest.mark.parametrize("name", sorted(COST_MISTAKES))
def test_cost_mistakes_fail_a_pin(monkeypatch, name):
    """The textbook-scaling pin builds its kernel from the correct cost, the
    oracle's Sinkhorn from the planted one."""
    monkeypatch.setattr(osk, "cost_matrix", COST_MISTAKES[name])
    with pytest.raises(AssertionError):
        pins.test_matches_textbook_scaling_iterations()


@pytest.mark.parametrize("name", sorted(SOFTMIN_MISTAKES))
def test_update_mistakes_fail_a_pin(monkeypatch, name):
    monkeypatch.setattr(osk, "softmin_rows", SOFTMIN_MISTAKES[name])
    with pytest.raises(AssertionError):
        pins.test_matches_textbook_scaling_iterations()


def test_conjugate_exponent_mistake_fails_a_pin(monkeypatch):
    # grad h*(w) = sign(w)|w|^(p-1) instead of |w|^(1/(p-1))
    monkeypatch.setattr(pcost, "grad_h_star",
                        lambda W, p: np.sign(W) * np.abs(np.asarray(W, np.float64)) ** (p - 1.0))
    with pytest.raises(AssertionError):
        ppins.test_conjugate_identities(1.5)


def test_missing_one_over_p_fails_a_pin(monkeypatch):
    monkeypatch.setattr(pcost, "h_p", lambda Z, p: _h_p(Z, p) * p)
    with pytest.raises(AssertionError):
        ppins.test_h_exact_values()


def test_flipped_mccann_step_fails_a_pin(monkeypatch):
    # x + grad h*(...) instead of x - grad h*(...)
    monkeypatch.setattr(pcost, "entropic_map_p",
                        lambda Xq, Y, g, eps, p, alpha=1.0: 2 * np.asarray(Xq, np.float64)
                        - _map_p(Xq, Y, g, eps, p, alpha))
    with pytest.raises(AssertionError):
        ppins.test_map_is_x_minus_grad_h_star_of_potential_gradient(1.5)


def test_pins_pass_on_the_unpatched_oracle():
    """The same pins, unpatched, pass (so the failures above come from the
    planted mistakes)."""
    pins.test_matches_textbook_scaling_iterations()
    ppins.test_conjugate_identities(1.5)
    ppins.test_h_exact_values()
    ppins.test_map_is_x_minus_grad_h_star_of_potential_gradient(1.5)


_alpha = schedules.alpha_schedule


def _alpha_unnormalised(K, kind="constant"):
    # alpha_k = t_k - t_{k-1}: the step as a share of the whole path rather
    # than of the rest of it
    t = schedules.progress(_alpha(K, kind))
    a = np.diff(np.concatenate([[0.0], t]))
    a[-1] = 1.0
    return a


def test_unnormalised_alpha_fails_a_pin(monkeypatch):
    monkeypatch.setattr(schedules, "alpha_schedule", _alpha_unnormalised)
    with pytest.raises(AssertionError):
        spins.test_alpha_schedule_golden("accelerated")


def test_progress_as_cumulative_sum_fails_a_pin(monkeypatch):
    monkeypatch.setattr(schedules, "progress", lambda alpha: np.cumsum(np.asarray(alpha, np.float64)))
    with pytest.raises(AssertionError):
        spins.test_alpha_schedule_golden("constant")


def test_eps_without_the_twentieth_fails_a_pin(monkeypatch):
    monkeypatch.setattr(schedules, "eps_mean_cost",
                        lambda X, Y, theta=1.0: float(theta * _cost(X, Y).mean()))
    with pytest.raises(AssertionError):
        spins.test_eps_mean_cost_closed_form()


def test_alg4_eps0_without_the_twentieth_fails_a_pin(monkeypatch):
    monkeypatch.setattr(schedules, "eps_zero", lambda C: float(np.asarray(C).mean()))
    with pytest.raises(AssertionError):
        spins.test_eps_scheduler_eps0_closed_form()


_score = schedules.holdout_score


def test_alg4_unsquared_score_fails_a_pin(monkeypatch):
    monkeypatch.setattr(schedules, "holdout_score",
                        lambda Yt, TY: float(np.linalg.norm(np.asarray(Yt, np.float64)
                                                            - np.asarray(TY), axis=1).sum()))
    with pytest.raises(AssertionError):
        spins.test_eps_scheduler_score_large_eps_limit()


def test_alg4_mean_score_fails_a_pin(monkeypatch):
    monkeypatch.setattr(schedules, "holdout_score",
                        lambda Yt, TY: _score(Yt, TY) / np.asarray(Yt).shape[0])
    with pytest.raises(AssertionError):
        spins.test_eps_scheduler_score_large_eps_limit()


_progot = importlib.import_module("oracle.progot").progot


def test_warm_start_from_previous_alpha_fails_a_pin(monkeypatch):
    # (1 - alpha_{k-1}) instead of the printed (1 - alpha_k)
    monkeypatch.setattr(oracle_pkg, "progot",
                        lambda *a, **k: _progot(*a, **{**k, "warm_start": "alpha_prev"}))
    with pytest.raises(AssertionError):
        spins.test_last_step_starts_cold()


def _progot_unscaled_warm_start(a, X, b, Y, K, n_iter=None, **_):
    """Alg. 2 with the previous potentials reused unscaled (no (1 - alpha_k)
    factor), built from the oracle's own steps."""
    al = schedules.alpha_schedule(K)
    Xk = np.asarray(X, np.float64).copy()
    f, g = np.zeros(Xk.shape[0]), np.zeros(np.asarray(Y).shape[0])
    G, eps = np.zeros((K, g.shape[0])), np.zeros(K)
    X_last = Xk
    for k in range(K):
        C = _cost(Xk, Y)
        eps[k] = C.mean() / 20.0
        r = osk.sinkhorn(a, Xk, b, Y, eps[k], 0.0, f, g, n_iter=n_iter, C=C)
        f, g = r.f, r.g
        G[k] = g
        X_last = Xk
        Xk = oracle_pkg.entropic_map(Xk, Y, g, eps[k], alpha=al[k])
    return importlib.import_module("oracle.progot").ProgOTResult(
        f=f, G=G, eps=eps, alpha=al, X_last=X_last, TX=Xk)


def test_warm_start_unscaled_fails_a_pin(monkeypatch):
    monkeypatch.setattr(oracle_pkg, "progot", _progot_unscaled_warm_start)
    with pytest.raises(AssertionError):
        spins.test_last_step_starts_cold()


def test_schedule_pins_pass_unpatched():
    spins.test_alpha_schedule_golden("accelerated")
    spins.test_alpha_schedule_golden("constant")
    spins.test_eps_mean_cost_closed_form()
    spins.test_eps_scheduler_eps0_closed_form()
    spins.test_eps_scheduler_score_large_eps_limit()
    spins.test_last_step_starts_cold()


_ot_value = metrics.ot_value
_p_log_p = metrics.p_log_p


def _divergence_without_half(a, X, b, Y, eps=None, tau=1e-6, max_iter=100_000, cost_p=None):
    if eps is None:
        eps = metrics.eps_divergence_default(Y, cost_p)
    oxy = _ot_value(a, X, b, Y, eps, tau, max_iter, cost_p)
    oxx = _ot_value(a, X, a, X, eps, tau, max_iter, cost_p)
    oyy = _ot_value(b, Y, b, Y, eps, tau, max_iter, cost_p)
    return oxy - (oxx + oyy), oxy, oxx, oyy, eps


def test_divergence_without_half_fails_a_pin(monkeypatch):
    monkeypatch.setattr(metrics, "sinkhorn_divergence", _divergence_without_half)
    with pytest.raises(AssertionError):
        mpins.test_divergence_translation_identity()


def test_entropy_sign_fails_a_pin(monkeypatch):
    monkeypatch.setattr(metrics, "p_log_p", lambda P: -_p_log_p(P))
    with pytest.raises(AssertionError):
        mpins.test_primal_parts_match_the_dual()


def test_transport_cost_as_product_of_sums_fails_a_pin(monkeypatch):
    monkeypatch.setattr(metrics, "transport_cost",
                        lambda P, C: float(np.asarray(P, np.float64).sum() * np.asarray(C).mean()))
    with pytest.raises(AssertionError):
        mpins.test_primal_parts_match_the_dual()


def test_metrics_pins_pass_unpatched():
    mpins.test_divergence_translation_identity()
    mpins.test_primal_parts_match_the_dual()
