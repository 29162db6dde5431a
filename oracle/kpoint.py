"""k-point-symmetric Cholesky factorisation for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/afqmc.py).

The AFQMC section of the paper factorises the two-electron tensor of a
periodic system per momentum transfer Q (the explicitly k-point dependent
factorisation): V_{(i k+Q, l k), (p k', j k'-Q)} = sum_n L^{Q,k}_{il,n} conj(L^{Q,k'-Q}_{pj,n}).
Read as a dense factorisation over orbitals (i, k) -> k*m + i, every (Q, n)
is one complex Cholesky vector L^{(Q,n)} whose only non-zero blocks are
(k + Q, k) = L^{Q,k}_n, and the tensor is the general form of the paper's
Cholesky equation, v_ijkl = sum_g L^g_ik conj(L^g_lj), with non-Hermitian
L^g. The walk below is written for that general form; `dense_factors` maps
the k-point blocks onto it.

General complex Cholesky vectors (second quantisation, textbook steps):
  H2 = 1/2 sum_ijkl v_ijkl c+_i c+_j c_l c_k
     = 1/2 sum_g rho_g rho_g^+ - 1/2 sum_g (L^g L^g+)_ik c+_i c_k,
  rho_g = sum_ik L^g_ik c+_i c_k.
  With a_g = (L^g + L^g+)/2 and b_g = (L^g - L^g+)/(2i) (both Hermitian),
  rho rho^+ = A^2 + B^2 - i[A, B], so
  H = sum_ik h'_ik c+_i c_k + 1/2 sum_g (A_g^2 + B_g^2),
  h' = h - 1/4 sum_g (L^g L^g+ + L^g+ L^g),
  and every A_g, B_g gets its own Hubbard-Stratonovich field.
  Local energy (Wick, G = sum_s G^s):
  E_L = E_II + sum_s tr(h G^s)
        + 1/2 sum_g [ tr(L^g G) tr(L^g+ G) - sum_s tr(L^g G^s L^g+ G^s) ].
  Force bias: abar_g = tr(a_g G), bbar_g = tr(b_g G); the shifts are
  -i sqrt(dt) times these, and A = i sqrt(dt) sum_g [(x_g - xbar_g) a_g + (y_g - ybar_g) b_g].
Fields are ordered (x_0 .. x_{X-1}, y_0 .. y_{X-1}) for X vectors.
"""
from __future__ import annotations

import numpy as np

from . import afqmc


# ---------------------------------------------------------------------------
# k-point blocks -> dense vectors
# ---------------------------------------------------------------------------
def dense_factors(Lk, kq):
    """Lk[Q, k, n] (m x m complex) and the addition table kq[Q][k] = k + Q
    -> dense L[(Q, n)] (M x M) with block (kq[Q][k], k) = Lk[Q, k, n]."""
    nk, _, xq, m, _ = Lk.shape
    M = nk * m
    L = np.zeros((nk * xq, M, M), np.complex128)
    for Q in range(nk):
        for k in range(nk):
            r = kq[Q][k]
            L[Q * xq:(Q + 1) * xq, r * m:(r + 1) * m, k * m:(k + 1) * m] = Lk[Q, k]
    return L


def dense_one_body(hk):
    """Block-diagonal h from per-k blocks hk[k] (m x m)."""
    nk, m, _ = hk.shape
    h = np.zeros((nk * m, nk * m), np.complex128)
    for k in range(nk):
        h[k * m:(k + 1) * m, k * m:(k + 1) * m] = hk[k]
    return h


def dense_trial(phik, n_up, n_dn):
    """Block-diagonal trial: phik[k] (m x (n_up + n_dn)) per k-point; the dense
    trial has columns (k, a) k-major within each spin, up spin first."""
    nk, m, _ = phik.shape
    T = np.zeros((nk * m, nk * (n_up + n_dn)), np.complex128)
    for k in range(nk):
        T[k * m:(k + 1) * m, k * n_up:(k + 1) * n_up] = phik[k][:, :n_up]
        T[k * m:(k + 1) * m, nk * n_up + k * n_dn:nk * n_up + (k + 1) * n_dn] = phik[k][:, n_up:]
    return T


# ---------------------------------------------------------------------------
# general complex Cholesky vectors
# ---------------------------------------------------------------------------
def two_body_tensor(L):
    """v_ijkl = sum_g L^g_ik conj(L^g_lj)."""
    return np.einsum("gik,glj->ijkl", L, np.conj(L))


def hermitian_parts(L):
    """a_g = (L + L^+)/2, b_g = (L - L^+)/(2i)."""
    Lh = np.conj(np.swapaxes(L, 1, 2))
    return 0.5 * (L + Lh), (L - Lh) / 2j


def one_body_corrected(h, L):
    """h' = h - 1/4 sum_g (L L^+ + L^+ L)."""
    Lh = np.conj(np.swapaxes(L, 1, 2))
    return h - 0.25 * (np.einsum("gij,gjk->ik", L, Lh) + np.einsum("gij,gjk->ik", Lh, L))


def local_energy(h, L, T, W, n_up, n_dn, e_core=0.0):
    """(E, E1, EJ, EK) with EJ = 1/2 sum_g tr(L G) tr(L^+ G) and
    EK = -1/2 sum_g sum_s tr(L G^s L^+ G^s)."""
    G = afqmc.greens_function(T, W, n_up, n_dn)
    Gt = G[0] + G[1]
    Lh = np.conj(np.swapaxes(L, 1, 2))
    e1 = sum(np.trace(h @ g) for g in G)
    trL = np.einsum("gik,ki->g", L, Gt)
    trLh = np.einsum("gik,ki->g", Lh, Gt)
    ej = 0.5 * np.sum(trL * trLh)
    ek = 0.0
    for g in G:
        LG = L @ g
        LhG = Lh @ g
        ek = ek - 0.5 * np.sum(np.einsum("gij,gji->g", LG, LhG))
    return e_core + e1 + ej + ek, e1, ej, ek


def force_bias(L, T, W, n_up, n_dn):
    """(abar, bbar) = (tr(a_g G), tr(b_g G)) as one vector of length 2X."""
    G = afqmc.greens_function(T, W, n_up, n_dn)
    Gt = G[0] + G[1]
    a, b = hermitian_parts(L)
    return np.concatenate([np.einsum("gik,ki->g", a, Gt), np.einsum("gik,ki->g", b, Gt)])


def run(h, L, T, n_up, n_dn, W0, weights0, fields, dt, qr_every=5, e_shift=0.0, order=6, e_core=0.0,
        bp_start=None, bp_len=0):
    """The phaseless walk of oracle/afqmc.run for general complex Cholesky
    vectors: fields[k, w] has 2X entries (x for the a_g, then y for the b_g);
    B1 = exp(-dt h'/2) with h' Hermitian; energy and force bias at the
    start-of-step walker; QR every qr_every steps. With bp_start set, the
    back-propagation window of oracle/afqmc.run is recorded (coefficients
    i sqrt(dt) (z - zbar) of the 2X Hermitian operators out["ops"]); out["B1"]
    is the one-body factor and out["log_I"][k, w] the complex log of the
    importance factor I before the phaseless projection."""
    nw = W0.shape[0]
    X = L.shape[0]
    hp = one_body_corrected(h, L)
    lam, V = np.linalg.eigh(hp)
    B1 = (V * np.exp(-0.5 * dt * lam)) @ V.conj().T
    a, b = hermitian_parts(L)
    ops = np.concatenate([a, b])                     # 2X Hermitian one-body matrices
    W = W0.astype(np.complex128).copy()
    w = np.asarray(weights0, dtype=np.float64).copy()
    logO = np.array([afqmc.theta(T, W[i], n_up, n_dn)[1] for i in range(nw)])
    alive = w > 0
    n_steps = fields.shape[0]
    out = dict(emix=np.zeros(n_steps), eloc=np.zeros((n_steps, nw), np.complex128),
               weights=np.zeros((n_steps, nw)), ratio=np.zeros((n_steps, nw), np.complex128),
               log_I=np.zeros((n_steps, nw), np.complex128))
    out.update(B1=B1, ops=ops)
    for k in range(n_steps):
        if bp_start == k:
            out["bp_W0"] = W.copy()
            out["bp_coefs"] = np.zeros((bp_len, nw, 2 * X), np.complex128)
        vb = np.zeros((nw, 2 * X), np.complex128)
        for i in range(nw):
            out["eloc"][k, i] = local_energy(h, L, T, W[i], n_up, n_dn, e_core)[0]
            vb[i] = force_bias(L, T, W[i], n_up, n_dn)
        sw = np.sum(w)
        out["emix"][k] = np.sum(w * out["eloc"][k].real) / sw if sw > 0 else 0.0
        for i in range(nw):
            if not alive[i]:
                continue
            x = fields[k, i]
            xbar = afqmc.force_bias_shift(vb[i], dt)
            A = np.tensordot(1j * np.sqrt(dt) * (x - xbar), ops, axes=1)
            if bp_start is not None and bp_start <= k < bp_start + bp_len:
                out["bp_coefs"][k - bp_start, i] = 1j * np.sqrt(dt) * (x - xbar)
            Wn = B1 @ afqmc.taylor_apply(A, B1 @ W[i], order)
            logOn = afqmc.theta(T, Wn, n_up, n_dn)[1]
            log_r = logOn - logO[i]
            log_I = log_r + afqmc.importance_log_factor(x, xbar) + dt * e_shift
            out["log_I"][k, i] = log_I
            cos_dth = np.cos(log_r.imag)
            wn = w[i] * np.exp(log_I.real) * cos_dth if cos_dth > 0.0 else 0.0
            out["ratio"][k, i] = np.exp(log_r)
            if not np.isfinite(wn) or wn <= 0.0:
                w[i] = 0.0
                alive[i] = False
                continue
            w[i] = wn
            W[i] = Wn
            logO[i] = logOn
        if qr_every > 0 and (k + 1) % qr_every == 0:
            for i in range(nw):
                if not alive[i]:
                    continue
                for bl in afqmc.spin_blocks(n_up, n_dn):
                    Q, R = afqmc.qr_positive(W[i][:, bl])
                    W[i][:, bl] = Q
                    logO[i] -= np.sum(np.log(np.diag(R).real))
        out["weights"][k] = w
        if bp_start is not None and k == bp_start + bp_len - 1:
            out["bp_weights"] = w.copy()
    out.update(W=W, w=w, logO=logO, alive=alive)
    return out
