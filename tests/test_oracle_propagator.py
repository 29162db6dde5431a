"""Pin of the oracle walk's short-time propagator against the Hamiltonian.

One step of the oracle's own walk (its B1 = exp(-dt h'/2), the order
B1 T_K(A) B1 and the importance factor, taken before the phaseless
projection) is averaged over the auxiliary fields with Gauss-Hermite
quadrature and mapped to the determinant space. The state a walker stands for
is I |W'> / <T|W'> for the start state |W> / <T|W>, so the average of
exp(log I - log r) |W'> must equal exp(-dt (H - E_shift)) |W> up to the
Trotter and Hubbard-Stratonovich error, O(dt^2) per step: the error falls
about four-fold when dt halves. H is the FCI matrix of the paper's Eq. hamil
with the Cholesky form of the two-electron tensor (Section "Auxiliary Field
Quantum Monte Carlo"); the FCI code shares no arithmetic with the walk.

A walk that exponentiates h instead of h' = h - 1/2 sum L L (the
normal-ordering correction) is off by O(dt) and fails: the planted-mistake
tests patch the oracle on the CPU and check that the pin catches it.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import afqmc, fci, kpoint
from paper_2003_01831_amd import synth

from prop_pin import averaged_step_error as _averaged_step_error


# --------------------------------------------------------------------------
# real symmetric Cholesky vectors: oracle/afqmc.py
# --------------------------------------------------------------------------
NU, ND, M_REAL, X_REAL = 2, 2, 6, 2


@pytest.fixture(scope="module")
def real_case():
    s = synth.make_system(M_REAL, NU, ND, X_REAL, seed=7)
    chol = 1.5 * s.chol                      # two-body part comparable to the one-body part
    H, _ = fci.hamiltonian(s.h1, afqmc.two_body_tensor(chol), NU, ND)
    rng = np.random.default_rng(5)
    W = s.phi_t + 0.3 * (rng.standard_normal(s.phi_t.shape) + 1j * rng.standard_normal(s.phi_t.shape))
    return s, chol, H, W


def _real_errors(case, dts):
    s, chol, H, W = case

    def step(W0, fields, dt, e_shift):
        return afqmc.run(s.h1, chol, s.phi_t, NU, ND, W0, np.ones(W0.shape[0]), fields, dt,
                         qr_every=0, e_shift=e_shift)

    return [_averaged_step_error(step, H, W, NU, ND, X_REAL, dt, e_shift=-1.3) for dt in dts]


def test_prepare_one_body_factor_is_exp_of_corrected_h(real_case):
    s, chol, _, _ = real_case
    dt = 0.02
    pre = afqmc.prepare(s.h1, chol, s.phi_t, NU, ND, dt)
    hp = s.h1 - 0.5 * sum(L @ L for L in chol)
    assert np.max(np.abs(pre["B1"] - expm(-0.5 * dt * hp))) < 1e-14


def test_walk_step_averages_to_short_time_propagator(real_case):
    e1, e2 = _real_errors(real_case, (0.02, 0.01))
    assert e1 < 5e-5 and e2 < 1.5e-5
    assert 3.5 < e1 / e2 < 4.5                       # O(dt^2) per step


def test_pin_catches_walk_without_normal_ordering_correction(real_case, monkeypatch):
    """Planted mistake: B1 = exp(-dt h/2). The error becomes O(dt) and hundreds
    of times larger, so the pin above fails."""
    good = _real_errors(real_case, (0.02,))[0]
    monkeypatch.setattr(afqmc, "one_body_corrected", lambda h1, chol: h1)
    e1, e2 = _real_errors(real_case, (0.02, 0.01))
    assert e1 > 100 * good
    assert 1.7 < e1 / e2 < 2.3                       # first order


# --------------------------------------------------------------------------
# general complex Cholesky vectors (two fields each): oracle/kpoint.py
# --------------------------------------------------------------------------
KU, KD, M_GEN = 2, 1, 5


@pytest.fixture(scope="module")
def general_case():
    rng = np.random.default_rng(11)
    a = rng.standard_normal((M_GEN, M_GEN)) + 1j * rng.standard_normal((M_GEN, M_GEN))
    h = (a + a.conj().T) / (2 * M_GEN)
    L = (rng.standard_normal((1, M_GEN, M_GEN)) + 1j * rng.standard_normal((1, M_GEN, M_GEN))) / M_GEN
    q, _ = np.linalg.qr(rng.standard_normal((M_GEN, M_GEN)) + 1j * rng.standard_normal((M_GEN, M_GEN)))
    T = np.concatenate([q[:, :KU], q[:, :KD]], axis=1)
    W = T + 0.3 * (rng.standard_normal(T.shape) + 1j * rng.standard_normal(T.shape))
    H, _ = fci.hamiltonian(h, kpoint.two_body_tensor(L), KU, KD)
    return h, L, T, H, W


def _general_errors(case, dts):
    h, L, T, H, W = case

    def step(W0, fields, dt, e_shift):
        return kpoint.run(h, L, T, KU, KD, W0, np.ones(W0.shape[0]), fields, dt, qr_every=0, e_shift=e_shift)

    return [_averaged_step_error(step, H, W, KU, KD, 2, dt, e_shift=0.7) for dt in dts]


def test_general_walk_step_averages_to_short_time_propagator(general_case):
    e1, e2 = _general_errors(general_case, (0.02, 0.01))
    assert e1 < 5e-5 and e2 < 1.5e-5
    assert 3.5 < e1 / e2 < 4.5


def test_pin_catches_general_walk_without_correction(general_case, monkeypatch):
    good = _general_errors(general_case, (0.02,))[0]
    monkeypatch.setattr(kpoint, "one_body_corrected", lambda h, L: h)
    e1, e2 = _general_errors(general_case, (0.02, 0.01))
    assert e1 > 100 * good
    assert 1.7 < e1 / e2 < 2.3
