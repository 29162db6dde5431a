"""Pins of the oracle's mean-field background subtraction.

For any real vector c the two-body term of the paper's Eq. hamil in Cholesky
form is 1/2 sum_n (v_n - c_n)^2 + sum_n c_n v_n - 1/2 sum_n c_n^2, so a walk
that samples the shifted operators v_n - c_n, moves sum_n c_n L^n into the
one-body factor, and carries the c-number part and the constant in the
importance factor must still average to the short-time propagator
exp(-dt (H - E_shift)) with an O(dt^2) error (the Gauss-Hermite pin of
tests/test_oracle_propagator.py, here with c the trial's mean field and with
an arbitrary vector). Planted mistakes in each of the three pieces fail it.
With a large background the phaseless angle of a step shrinks when it is
subtracted, which is what the subtraction is for.
"""
import numpy as np
import pytest

from oracle import afqmc, fci
from paper_2003_01831_amd import synth
from prop_pin import averaged_step_error

NU, ND, M, X = 2, 2, 6, 2


@pytest.fixture(scope="module")
def case():
    s = synth.make_system(M, NU, ND, X, seed=7)
    # a diagonal part in every vector gives the walk a large mean field
    chol = 1.5 * s.chol + np.array([0.25, -0.15])[:, None, None] * np.eye(M)[None]
    H, _ = fci.hamiltonian(s.h1, afqmc.two_body_tensor(chol), NU, ND)
    rng = np.random.default_rng(5)
    W = s.phi_t + 0.3 * (rng.standard_normal(s.phi_t.shape) + 1j * rng.standard_normal(s.phi_t.shape))
    return s, chol, H, W


def _errors(case, vmf, dts, e_shift=-0.4):
    s, chol, H, W = case

    def step(W0, fields, dt, es):
        return afqmc.run(s.h1, chol, s.phi_t, NU, ND, W0, np.ones(W0.shape[0]), fields, dt, qr_every=0,
                         e_shift=es, vmf=vmf)

    return [averaged_step_error(step, H, W, NU, ND, X, dt, e_shift) for dt in dts]


def test_mean_field_bias_is_the_trials_own_force_bias(case):
    s, chol, _, _ = case
    vmf = afqmc.mean_field_bias(chol, s.phi_t, NU, ND)
    G = afqmc.greens_function(s.phi_t, s.phi_t, NU, ND)
    assert np.max(np.abs(vmf - afqmc.force_bias_plain(chol, G).real)) < 1e-14
    assert np.max(np.abs(vmf)) > 0.5                      # the diagonal part makes it large


@pytest.mark.parametrize("which", ["mean_field", "arbitrary"])
def test_subtracted_walk_averages_to_short_time_propagator(case, which):
    s, chol, _, _ = case
    vmf = afqmc.mean_field_bias(chol, s.phi_t, NU, ND) if which == "mean_field" else np.array([0.7, -0.4])
    e1, e2 = _errors(case, vmf, (0.02, 0.01))
    assert e1 < 5e-5 and e2 < 1.5e-5
    assert 3.5 < e1 / e2 < 4.5


@pytest.mark.parametrize("plant", ["one_body_sign", "no_cnumber", "no_constant"])
def test_pin_catches_planted_mistakes(case, plant, monkeypatch):
    s, chol, _, _ = case
    vmf = afqmc.mean_field_bias(chol, s.phi_t, NU, ND)
    good = _errors(case, vmf, (0.02,))[0]
    if plant == "one_body_sign":           # h' - sum c L instead of h' + sum c L
        orig = afqmc.prepare

        def bad_prepare(h1, ch, phi, nu, nd, dt, vmf=None):
            pre = orig(h1, ch, phi, nu, nd, dt, vmf=None)
            hp = pre["hp"] - np.tensordot(vmf, ch, axes=1)
            pre.update(hp=hp, B1=afqmc.sym_expm(-0.5 * dt * hp), vmf=vmf)
            return pre
        monkeypatch.setattr(afqmc, "prepare", bad_prepare)
    elif plant == "no_cnumber":            # the c-number factor of the shifted operators dropped
        orig_run = afqmc.run

        def strip_c0(h1, ch, phi, nu, nd, W0, w0, fields, dt, **k):
            o = orig_run(h1, ch, phi, nu, nd, W0, w0, fields, dt, **k)
            v = k["vmf"]
            ht, Lt = afqmc.half_rotate(h1, ch, phi, nu, nd)
            for i in range(W0.shape[0]):
                xbar = afqmc.force_bias_shift(afqmc.local_energy_half(ht, Lt, phi, W0[i], nu, nd)[2] - v, dt)
                o["log_I"][0, i] -= -1j * np.sqrt(dt) * np.sum((fields[0, i] - xbar) * v)
            return o
        monkeypatch.setattr(afqmc, "run", strip_c0)
    else:                                  # the constant exp(dt/2 sum c^2) dropped
        orig_run = afqmc.run

        def strip_const(h1, ch, phi, nu, nd, W0, w0, fields, dt, **k):
            o = orig_run(h1, ch, phi, nu, nd, W0, w0, fields, dt, **k)
            o["log_I"] = o["log_I"] - 0.5 * dt * np.sum(k["vmf"] ** 2)
            return o
        monkeypatch.setattr(afqmc, "run", strip_const)
    e1, e2 = _errors(case, vmf, (0.02, 0.01))
    assert e1 > 30 * good
    assert e1 / e2 < 3.0                   # no longer second order


def test_zero_background_is_the_plain_walk(case):
    s, chol, _, W = case
    nw, steps = 4, 6
    fields = synth.make_fields(steps, nw, X, seed=3)
    W0 = np.repeat(W[None], nw, axis=0)
    a = afqmc.run(s.h1, chol, s.phi_t, NU, ND, W0, np.ones(nw), fields, 0.01, qr_every=3)
    b = afqmc.run(s.h1, chol, s.phi_t, NU, ND, W0, np.ones(nw), fields, 0.01, qr_every=3, vmf=np.zeros(X))
    for k in ("eloc", "weights", "ratio", "log_I", "W"):
        assert np.array_equal(a[k], b[k]), k


def test_subtraction_shrinks_the_phaseless_angle(case):
    """Walkers at the trial, one step with 400 random field draws: with the
    mean field subtracted the mean 1 - cos(angle) is far smaller."""
    s, chol, _, _ = case
    vmf = afqmc.mean_field_bias(chol, s.phi_t, NU, ND)
    nw = 400
    fields = np.random.default_rng(9).standard_normal((1, nw, X))
    W0 = synth.trial_walkers(s, nw)
    kw = dict(qr_every=0)
    plain = afqmc.run(s.h1, chol, s.phi_t, NU, ND, W0, np.ones(nw), fields, 0.02, **kw)
    sub = afqmc.run(s.h1, chol, s.phi_t, NU, ND, W0, np.ones(nw), fields, 0.02, vmf=vmf, **kw)
    d_plain = np.mean(1.0 - plain["cosdt"][0])
    d_sub = np.mean(1.0 - sub["cosdt"][0])
    assert d_sub < 0.05 * d_plain
