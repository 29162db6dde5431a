"""Pins of the oracle's orthogonal multi-determinant trial against the full
determinant space: the CI vector of the trial gives the overlap, the mixed
energy and the force bias as plain matrix elements; the determinants are
orthonormal; a complete expansion of the exact ground state has zero-variance
local energy."""
import itertools

import numpy as np
import pytest

from oracle import afqmc, fci, msd
from paper_2003_01831_amd import synth

M, NU, ND, X = 6, 2, 2, 5


@pytest.fixture(scope="module")
def case():
    s = synth.make_system(M, NU, ND, X, seed=201)
    s.chol = s.chol * 3.0
    C, exc, coeffs = synth.make_msd(s, 12, 2, 3, 2, seed=202, decay=0.8)
    dets = msd.determinants(C, NU, ND, exc)
    v = afqmc.two_body_tensor(s.chol)
    H, _ = fci.hamiltonian(s.h1, v, NU, ND, e_core=0.7)
    cT = sum(c * fci.coefficients(D, NU, ND) for D, c in zip(dets, coeffs))
    return s, C, exc, coeffs, dets, H, cT


def test_determinants_are_orthonormal(case):
    s, C, exc, coeffs, dets, H, cT = case
    V = np.array([fci.coefficients(D, NU, ND) for D in dets])
    assert np.max(np.abs(V.conj() @ V.T - np.eye(len(dets)))) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_msd_mixed_estimates_are_the_determinant_space_matrix_elements(case, seed):
    s, C, exc, coeffs, dets, H, cT = case
    W = synth.perturbed_walkers(s, 1, 0.4, seed=210 + seed)[0]
    cW = fci.coefficients(W, NU, ND)
    ov = np.vdot(cT, cW)
    assert abs(msd.overlap(dets, coeffs, W, NU, ND) - ov) < 1e-12 * abs(ov)
    e, e1, e2, vb = msd.local_energy(s.h1, s.chol, dets, coeffs, W, NU, ND, e_core=0.7)
    assert abs(e - np.vdot(cT, H @ cW) / ov) < 1e-10
    H1 = fci.one_body_operator(s.h1, NU, ND)
    assert abs(e1 - np.vdot(cT, H1 @ cW) / ov) < 1e-10
    assert abs(e - 0.7 - e1 - e2) < 1e-12
    for n in range(X):
        ref = np.vdot(cT, fci.one_body_operator(s.chol[n], NU, ND) @ cW) / ov
        assert abs(vb[n] - ref) < 1e-10


def test_complete_expansion_of_the_ground_state_has_zero_variance():
    """Every determinant of the 2+2-in-6 space is an excitation of the
    reference in the basis C; with coefficients <D_I|psi_0> the trial is the
    exact ground state and E_L(W) = E_0 for any walker."""
    s = synth.make_system(M, NU, ND, X, seed=221)
    s.chol = s.chol * 3.0
    C = synth._lowest_eigvecs(s.h1, M).astype(np.complex128)
    H, _ = fci.hamiltonian(s.h1, afqmc.two_body_tensor(s.chol), NU, ND)
    e0, v0 = fci.ground_state(H)
    exc = []
    for up in itertools.combinations(range(M), NU):
        for dn in itertools.combinations(range(M), ND):
            spins = []
            for occ, n in ((up, NU), (dn, ND)):
                holes = tuple(h for h in range(n) if h not in occ)
                parts = tuple(p for p in occ if p >= n)
                spins.append((holes, parts))
            exc.append(tuple(spins))
    dets = msd.determinants(C, NU, ND, exc)
    coeffs = np.array([np.vdot(fci.coefficients(D, NU, ND), v0) for D in dets])
    assert abs(np.linalg.norm(coeffs) - 1.0) < 1e-12            # the expansion is complete
    for seed in (0, 1, 2):
        W = synth.perturbed_walkers(s, 1, 0.5, seed=230 + seed)[0]
        e, _, _, _ = msd.local_energy(s.h1, s.chol, dets, coeffs, W, NU, ND)
        assert abs(e - e0) < 1e-10
    # a truncated expansion is not exact
    e_ref, _, _, _ = msd.local_energy(s.h1, s.chol, dets[:1], coeffs[:1], W, NU, ND)
    assert abs(e_ref - e0) > 1e-4


def test_single_determinant_expansion_is_the_single_determinant_trial(case):
    s, C, exc, coeffs, dets, H, cT = case
    W = synth.perturbed_walkers(s, 1, 0.3, seed=240)[0]
    e, e1, e2, vb = msd.local_energy(s.h1, s.chol, dets[:1], [0.3 - 0.2j], W, NU, ND, e_core=0.7)
    ref = afqmc.local_energy_plain(s.h1, s.chol, s.phi_t, W, NU, ND, 0.7)
    assert abs(e - ref[0]) < 1e-12 and abs(e2 - ref[2] - ref[3]) < 1e-12


def test_walk_with_a_one_determinant_expansion_is_the_plain_walk(case):
    s, C, exc, coeffs, dets, H, cT = case
    nw, steps, dt = 4, 4, 0.05
    W0 = synth.perturbed_walkers(s, nw, 0.1, seed=250)
    w0 = synth.random_weights(nw, seed=251)
    f = synth.make_fields(steps, nw, X, seed=252)
    a = afqmc.run(s.h1, s.chol, s.phi_t, NU, ND, W0, w0, f, dt, qr_every=2, energy="plain")
    b = afqmc.run(s.h1, s.chol, s.phi_t, NU, ND, W0, w0, f, dt, qr_every=2,
                  msd=dict(dets=dets[:1], coeffs=[1.0]))
    assert np.max(np.abs(a["eloc"] - b["eloc"])) < 1e-12
    assert np.max(np.abs(a["weights"] - b["weights"])) < 1e-12
    c = afqmc.run(s.h1, s.chol, s.phi_t, NU, ND, W0, w0, f, dt, qr_every=2, msd=dict(dets=dets, coeffs=coeffs))
    assert np.all(np.isfinite(c["eloc"])) and np.all(c["weights"] > 0)
