"""Pins of the oracle's population control (comb, weight cap, force-bias cap,
energy-shift feedback) against properties that hold independently of how it is
written: conservation, the floor/ceil copy counts of systematic resampling, its
unbiasedness over the uniform offset, a hand-worked example and limits."""
import numpy as np
import pytest

from oracle import afqmc
from paper_2003_01831_amd import synth


def test_comb_hand_worked_example():
    # weights 1, 2, 3: W = 6, three teeth at (k + 1/2) * 2 = 1, 3, 5 against the
    # running sums 1, 3, 6: tooth 1 lies in [1, 3) -> walker 1, teeth 3 and 5 in [3, 6) -> walker 2
    src, wnew, total = afqmc.comb([1.0, 2.0, 3.0], 0.5)
    assert list(src) == [1, 2, 2]
    assert wnew == 2.0 and total == 6.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_comb_counts_are_floor_or_ceil_and_conserve_weight(seed):
    rng = np.random.default_rng(seed)
    n = 57
    w = rng.uniform(0.2, 3.0, n)
    w[rng.choice(n, 9, replace=False)] = 0.0          # dead walkers
    for xi in rng.uniform(0.0, 1.0, 20):
        src, wnew, total = afqmc.comb(w, xi)
        counts = np.bincount(src, minlength=n)
        expect = n * w / total
        assert np.all(counts >= np.floor(expect - 1e-9)) and np.all(counts <= np.ceil(expect + 1e-9))
        assert np.all(counts[w == 0.0] == 0)
        assert counts.sum() == n
        assert abs(n * wnew - total) <= 1e-12 * total


def test_comb_is_unbiased_over_the_offset():
    rng = np.random.default_rng(5)
    n = 13
    w = rng.uniform(0.1, 2.0, n)
    grid = (np.arange(4000) + 0.5) / 4000
    mean = np.zeros(n)
    for xi in grid:
        mean += np.bincount(afqmc.comb(w, xi)[0], minlength=n)
    mean /= grid.size
    assert np.max(np.abs(mean - n * w / w.sum())) < 2e-3


def test_comb_of_equal_weights_is_the_identity():
    for xi in (1e-6, 0.25, 0.999999):   # away from the boundaries, where rounding decides
        src, _, _ = afqmc.comb(np.full(31, 0.7), xi)
        assert list(src) == list(range(31))


def test_comb_rejects_an_empty_population():
    with pytest.raises(ValueError):
        afqmc.comb(np.zeros(4), 0.5)


def test_force_bias_cap():
    rng = np.random.default_rng(7)
    vbar = (rng.standard_normal(200) + 1j * rng.standard_normal(200)) * 3.0
    dt = 0.04
    plain = afqmc.force_bias_shift(vbar, dt)
    capped = afqmc.force_bias_shift(vbar, dt, cap=0.5)
    assert np.all(np.abs(capped) <= 0.5 * (1 + 1e-15))
    big = np.abs(plain) > 0.5
    assert big.any() and (~big).any()
    assert np.array_equal(capped[~big], plain[~big])
    assert np.allclose(np.angle(capped[big]), np.angle(plain[big]), atol=1e-14)
    assert np.allclose(np.abs(capped[big]), 0.5, rtol=1e-15)
    assert np.array_equal(afqmc.force_bias_shift(vbar, dt, cap=1e9), plain)


def _small():
    s = synth.make_system(10, 3, 2, 30, seed=8)
    s.chol = s.chol * 2.5
    nw = 10
    W0 = synth.perturbed_walkers(s, nw, 0.1, seed=9)
    fields = synth.make_fields(6, nw, 30, seed=10)
    return s, nw, W0, fields


def test_weight_cap_bounds_the_weights_and_is_inert_when_loose():
    s, nw, W0, fields = _small()
    args = (s.h1, s.chol, s.phi_t, 3, 2, W0, np.ones(nw), fields, 0.05)
    free = afqmc.run(*args, qr_every=2)
    cap = float(np.quantile(free["weights"][free["weights"] > 0], 0.5))
    capped = afqmc.run(*args, qr_every=2, w_cap=cap)
    assert np.all(capped["weights"] <= cap)
    assert not np.array_equal(capped["weights"], free["weights"])
    loose = afqmc.run(*args, qr_every=2, w_cap=1e30)
    assert np.array_equal(loose["weights"], free["weights"])
    assert np.array_equal(loose["eloc"], free["eloc"])


def test_comb_inside_the_walk():
    s, nw, W0, fields = _small()
    xi = [0.3, 0.8, 0.1]
    out = afqmc.run(s.h1, s.chol, s.phi_t, 3, 2, W0, np.linspace(0.5, 1.5, nw), fields, 0.05, qr_every=2,
                    comb_every=2, comb_xi=xi)
    assert len(out["comb_src"]) == 3
    # after a comb every walker has the same weight, so the next step's mixed
    # energy is the plain mean of Re E_L over the walkers
    for k in (2, 4):
        assert abs(out["emix"][k] - np.mean(out["eloc"][k].real)) < 1e-12 * abs(out["emix"][k])
    # each comb keeps n walkers, each a copy of a surviving walker
    for src in out["comb_src"]:
        assert len(src) == nw


def test_eshift_update():
    assert afqmc.eshift_update(-3.0, 100.0, 100.0, 0.01, 10) == -3.0
    # W = e W_target: the shift drops by 1 / (g dt) = 10
    assert abs(afqmc.eshift_update(-3.0, 100.0 * np.e, 100.0, 0.01, 10) - (-13.0)) < 1e-12
    assert afqmc.eshift_update(-3.0, 50.0, 100.0, 0.01, 10) > -3.0
