"""Pins of the oracle's adjoint of the weighted mixed energy
Ebar = sum_w w Re E_L / sum_w w: central finite differences, the explicit mixed
one-body density matrix from FCI, and the gauge invariant of the walker gradient."""
import numpy as np
import pytest

from oracle import afqmc, fci
from paper_2003_01831_amd import synth


@pytest.fixture(scope="module")
def case():
    s = synth.make_system(6, 2, 2, 5, seed=13)
    nw = 3
    W = synth.perturbed_walkers(s, nw, 0.3, seed=14)
    w = synth.random_weights(nw, seed=15)
    grads = afqmc.energy_grad(s.h1, s.chol, s.phi_t, 2, 2, W, w)
    return s, W, w, grads


def _ebar(s, h1, chol, W, w):
    return afqmc.energy(h1, chol, s.phi_t, 2, 2, W, w, form="plain")[2]


def test_grad_h1_finite_differences(case):
    s, W, w, (dh, dl, dw) = case
    eps = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(6):
        i, j = rng.integers(0, s.M, 2)
        hp, hm = s.h1.copy(), s.h1.copy()
        hp[i, j] += eps
        hm[i, j] -= eps
        fd = (_ebar(s, hp, s.chol, W, w) - _ebar(s, hm, s.chol, W, w)) / (2 * eps)
        assert abs(fd - dh[i, j]) < 1e-6 * max(1.0, abs(fd))


def test_grad_chol_finite_differences(case):
    s, W, w, (dh, dl, dw) = case
    eps = 1e-6
    rng = np.random.default_rng(1)
    for _ in range(8):
        n = rng.integers(0, s.n_chol)
        i, j = rng.integers(0, s.M, 2)
        cp, cm = s.chol.copy(), s.chol.copy()
        cp[n, i, j] += eps
        cm[n, i, j] -= eps
        fd = (_ebar(s, s.h1, cp, W, w) - _ebar(s, s.h1, cm, W, w)) / (2 * eps)
        assert abs(fd - dl[n, i, j]) < 1e-6 * max(1.0, abs(fd))


def test_grad_walkers_finite_differences(case):
    """torch convention: grad = dE/dRe W + i dE/dIm W."""
    s, W, w, (dh, dl, dw) = case
    eps = 1e-6
    rng = np.random.default_rng(2)
    for _ in range(8):
        k = rng.integers(0, W.shape[0])
        i = rng.integers(0, s.M)
        a = rng.integers(0, 4)
        for unit, part in ((1.0, "re"), (1j, "im")):
            Wp, Wm = W.copy(), W.copy()
            Wp[k, i, a] += eps * unit
            Wm[k, i, a] -= eps * unit
            fd = (_ebar(s, s.h1, s.chol, Wp, w) - _ebar(s, s.h1, s.chol, Wm, w)) / (2 * eps)
            got = dw[k, i, a].real if part == "re" else dw[k, i, a].imag
            assert abs(fd - got) < 1e-6 * max(1.0, abs(fd))


def test_grad_h1_is_fci_mixed_rdm(case):
    """dEbar/dh_ij = Re sum_w wh_w <T|c+_i c_j|W>/<T|W> (summed over spin), with the
    density matrix formed explicitly on FCI vectors."""
    s, W, w, (dh, dl, dw) = case
    cT = fci.coefficients(s.phi_t, 2, 2)
    wh = w / w.sum()
    P = np.zeros((s.M, s.M), np.complex128)
    cWs = [fci.coefficients(Wk, 2, 2) for Wk in W]
    for i in range(s.M):
        for j in range(s.M):
            E = np.zeros((s.M, s.M))
            E[i, j] = 1.0
            op = fci.one_body_operator(E, 2, 2)
            P[i, j] = sum(wh[k] * np.vdot(cT, op @ cW) / np.vdot(cT, cW)
                          for k, cW in enumerate(cWs))
    assert np.max(np.abs(dh - P.real)) < 1e-12
    assert np.max(np.abs(afqmc.mixed_rdm1(s.phi_t, 2, 2, W, w) - P)) < 1e-12


def test_walker_gradient_gauge_invariance(case):
    """E_L is invariant under W -> W R, so W^T dE/dW = 0 per spin (holomorphic
    derivative dE/dW = conj(grad)/wh)."""
    s, W, w, (dh, dl, dw) = case
    for k in range(W.shape[0]):
        for b in afqmc.spin_blocks(2, 2):
            g = np.conj(dw[k][:, b])
            assert np.max(np.abs(W[k][:, b].T @ g)) < 1e-12
