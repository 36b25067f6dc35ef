"""Pins of the oracle's Metropolis VMC and fixed-node DMC walks (Sec. 2.3).

VMC energies of one-parameter trial functions have closed forms:
  H,  exp(-a r^2), a = 8/(9 pi):             E = 3a/2 - 2 sqrt(2a/pi) = -4/(3 pi)
  He, exp(-z r1 - z r2), z = 27/16:           E = z^2 - 27 z / 8 = -(27/16)^2
  He, exp(-a r1^2 - a r2^2), optimal a:       E = 3a - (8 sqrt2 - 2) sqrt(a/pi) = -3a
DMC of a nodeless one-electron problem is exact (no fixed-node error): H with
a Gaussian trial function projects to -1/2 up to time-step error; with the
exact trial function every weight stays 1 and the population is constant.
"""

import json
import math
import os

import numpy as np
import pytest

import systems as S

CLOSED = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _vmc_mean(o, R0, steps, burn, seed, step_size, all_electron):
    b = o.vmc(R0, burn, seed, 0, step_size, all_electron)
    R = b["R"]
    r = o.vmc(R, steps, seed, burn, step_size, all_electron)
    per_walker = r["e_sum"] / steps
    return per_walker.mean(), per_walker.std(ddof=1) / math.sqrt(len(per_walker)), r


def test_vmc_hydrogen_gaussian_energy(oracle_mod):
    a = 8 / (9 * math.pi)
    o = oracle_mod.Oracle(S.hydrogen_gaussian(a))
    R0 = np.random.default_rng(1).normal(size=(2000, 1, 3))
    m, s, r = _vmc_mean(o, R0, 200, 100, 11, 1.0, True)
    assert abs(m - CLOSED["hydrogen_gaussian_opt_energy"]) < 3 * s, (m, s)
    assert 0.2 < r["n_acc"].sum() / (2000 * 200) < 0.9


def test_vmc_helium_sto_energy(oracle_mod):
    o = oracle_mod.Oracle(S.helium_sto(CLOSED["helium_sto_opt_zeta"]))
    R0 = np.random.default_rng(2).normal(scale=0.6, size=(1000, 2, 3))
    m, s, _ = _vmc_mean(o, R0, 200, 100, 12, 0.6, False)
    assert abs(m - CLOSED["helium_sto_opt_energy"]) < 3 * s, (m, s)


def test_vmc_helium_gaussian_energy(oracle_mod):
    o = oracle_mod.Oracle(S.helium_gaussian(CLOSED["helium_gaussian_opt_alpha"]))
    R0 = np.random.default_rng(3).normal(scale=0.6, size=(1000, 2, 3))
    m, s, _ = _vmc_mean(o, R0, 200, 100, 13, 0.8, False)
    assert abs(m - CLOSED["helium_gaussian_opt_energy"]) < 3 * s, (m, s)


def test_vmc_exact_orbital_zero_variance(oracle_mod):
    o = oracle_mod.Oracle(S.hydrogen_sto_1s(1.0))
    R0 = np.random.default_rng(4).normal(size=(200, 1, 3))
    r = o.vmc(R0, 50, 5, 0, 1.0, True)
    np.testing.assert_allclose(r["e_sum"] / 50, -0.5, atol=1e-13)
    np.testing.assert_allclose(r["e2_sum"] / 50 - (r["e_sum"] / 50) ** 2, 0.0, atol=1e-12)


def test_vmc_is_deterministic_in_the_seed(oracle_mod):
    sysd = S.h2_heitler_london()
    o = oracle_mod.Oracle(sysd)
    R0 = S.initial_walkers(sysd, 64, seed=3)
    a = o.vmc(R0, 20, 99, 0, 0.5, True)
    b = o.vmc(R0, 20, 99, 0, 0.5, True)
    np.testing.assert_array_equal(a["R"], b["R"])
    np.testing.assert_array_equal(a["e_sum"], b["e_sum"])
    c = o.vmc(R0, 20, 98, 0, 0.5, True)
    assert not np.array_equal(a["R"], c["R"])


def test_dmc_exact_trial_function_keeps_population(oracle_mod):
    o = oracle_mod.Oracle(S.hydrogen_sto_1s(1.0))
    R0 = np.random.default_rng(5).normal(size=(300, 1, 3))
    e0 = o.evaluate(R0)["eloc"]
    r = o.dmc(R0, e0, 40, 21, 0, 0.01, -0.5, 300)
    assert r["rc"] == 0
    np.testing.assert_array_equal(r["pop"], 300)
    np.testing.assert_allclose(r["wsum"], 300, rtol=1e-13)
    np.testing.assert_allclose(r["wesum"] / r["wsum"], -0.5, atol=1e-13)


def test_dmc_move_lengths_give_the_effective_time_step(oracle_mod):
    """Hydrogen with its exact trial orbital e^-r: the drift is -r/|r| (unit
    length), so a proposal r' = r + tau v + sqrt(tau) chi has mean squared
    length 3 tau + tau^2; the accepted moves are a subset, so
    tau_eff = tau dr2_acc / dr2_prop lies below tau and above tau times the
    acceptance's lower part."""
    sysd = S.hydrogen_sto_1s(1.0)
    o = oracle_mod.Oracle(sysd)
    W, tau, steps = 2000, 0.05, 5
    R0 = np.random.default_rng(5).normal(size=(W, 1, 3))
    e0 = o.evaluate(R0)["eloc"]
    r = o.dmc(R0, e0, steps, 23, 0, tau, -0.5, W)
    n = r["pop"].sum()  # one electron per walker: proposals = walker-steps
    np.testing.assert_array_equal(r["prop"], r["pop"])
    mean = r["dr2_prop"].sum() / n
    # chi^2 with 3 degrees of freedom: variance of |sqrt(tau) chi + tau v|^2
    # about 6 tau^2 (plus O(tau^3)); 5 sigma
    assert abs(mean - (3 * tau + tau * tau)) < 5 * np.sqrt(6 * tau * tau / n) + 4 * tau ** 2, mean
    ratio = r["dr2_acc"] / r["dr2_prop"]
    acc = r["acc"] / r["prop"]
    assert np.all(ratio < 1.0) and np.all(ratio > 0.9), ratio
    assert np.all(np.abs(ratio - acc) < 0.05), (ratio, acc)


def test_dmc_nodeless_projection_reaches_exact_energy(oracle_mod):
    """Gaussian trial (VMC energy -0.424) projects to the exact -0.5 within the time-step error."""
    o = oracle_mod.Oracle(S.hydrogen_gaussian(0.3))
    R0 = np.random.default_rng(6).normal(size=(1000, 1, 3))
    e0 = o.evaluate(R0)["eloc"]
    r = o.dmc(R0, e0, 200, 31, 0, 0.01, float(e0.mean()), 1000)
    assert r["rc"] == 0
    r2 = o.dmc(r["R"], r["eloc"], 300, 31, 200, 0.01, r["e_trial"], 1000)
    assert r2["rc"] == 0
    blk = (r2["wesum"] / r2["wsum"]).reshape(30, 10).mean(1)
    m, s = blk.mean(), blk.std(ddof=1) / math.sqrt(len(blk))
    assert abs(m + 0.5) < 3 * s + 0.005, (m, s)
    assert np.all(np.abs(r2["pop"] / 1000 - 1) < 0.1)


def test_dmc_population_clamp_factor(oracle_mod):
    """A trial energy far above the energy makes every weight exceed 1; the
    population control scales all weights of the step by the one factor that
    brings their sum to 1.05 W_target, i.e. the step runs at the trial energy
    E_T + ln(f) / tau (logged as that step's E_T)."""
    o = oracle_mod.Oracle(S.hydrogen_gaussian(0.3))
    W, tau, et = 400, 0.01, 5.0
    R0 = np.random.default_rng(9).normal(size=(W, 1, 3))
    e0 = o.evaluate(R0)["eloc"]
    r = o.dmc(R0, e0, 1, 41, 0, tau, et, W)
    assert r["rc"] == 0
    assert r["wsum"][0] == pytest.approx(1.05 * W, rel=1e-12)
    assert r["etrial"][0] < et
    # a second step starts from the clamped population and stays in the band
    r2 = o.dmc(r["R"], r["eloc"], 1, 41, 1, tau, r["e_trial"], W)
    assert abs(r2["pop"][0] / W - 1) <= 0.1


def test_dmc_population_stays_in_band(oracle_mod):
    """The F2-shaped trial function has local energies over several thousand
    hartree (no cusps, exponents up to 1e4); the birth/death population must
    still stay within +-10 % of the target at every step, and the trial
    energy must stay finite and within the range of the sampled energies."""
    sysd = S.f2_shaped()
    o = oracle_mod.Oracle(sysd)
    W = 600
    R0 = S.initial_walkers(sysd, W, seed=8)
    e0 = o.evaluate(R0)["eloc"]
    r = o.dmc(R0, e0, 15, 77, 0, 0.005, float(np.median(e0)), W, capacity=4 * W)
    assert r["rc"] == 0
    assert np.all(np.abs(r["pop"] / W - 1) <= 0.1), r["pop"]
    assert abs(r["W"] / W - 1) <= 0.1
    lo, hi = np.percentile(e0, [5, 95])
    assert np.all((r["etrial"] > lo) & (r["etrial"] < hi)), r["etrial"]


def test_blocking_error_of_a_correlated_series():
    """bench.reblock against the closed-form error of an AR(1) series
    x_k = phi x_{k-1} + eps_k (unit noise): sigma_mean = 1 / ((1 - phi) sqrt(n))
    for long series, while the naive estimate is far too small."""
    import bench
    rng = np.random.default_rng(3)
    n, phi = 1 << 14, 0.8
    x = np.zeros(n)
    for k in range(1, n):
        x[k] = phi * x[k - 1] + rng.normal()
    mean, err, levels = bench.reblock(x, np.ones(n))
    exact = 1.0 / ((1.0 - phi) * np.sqrt(n))
    assert abs(mean - x.mean()) < 1e-12
    assert 0.8 * exact < err < 1.3 * exact, (err, exact)
    assert x.std() / np.sqrt(n) < 0.5 * exact
    # a constant series has that constant as its weighted mean, whatever the weights
    w = rng.uniform(0.5, 2.0, 64)
    m2, _, _ = bench.reblock(np.full(64, 3.0), w)
    assert abs(m2 - 3.0) < 1e-14
