"""Brute-force full configuration interaction (FCI) for tiny systems.

TEST INFRASTRUCTURE ONLY (see oracle/afqmc.py).

This module writes the paper's second-quantised Hamiltonian (Eq. "hamil",
Section "Auxiliary Field Quantum Monte Carlo")

    H = sum_ij h_ij c+_i c_j + 1/2 sum_ijkl v_ijkl c+_i c+_j c_l c_k + E_II

out literally on the space of all determinants with n_up up and n_dn down
electrons in M spatial orbitals, by applying each creation/annihilation string
to occupation bit-strings with the fermionic sign. The spin structure is that
of a spin-free interaction: i and k carry the same spin, and so do j and l.

It shares no arithmetic with oracle/afqmc.py: no Green's function, no Wick
contraction, no normal ordering. It is used to pin the oracle (local energy,
overlap, operator identities, the Hubbard-Stratonovich identity).

Spin-orbital index: p = s*M + i (s = 0 up, 1 down). A determinant is the
bit-string of occupied spin orbitals; |D> = c+_{p1} c+_{p2} ... |0> with
p1 < p2 < ... .
"""
from __future__ import annotations

import itertools
import numpy as np


def determinants(M, n_up, n_dn):
    ups = [sum(1 << i for i in c) for c in itertools.combinations(range(M), n_up)]
    dns = [sum(1 << (M + i) for i in c) for c in itertools.combinations(range(M), n_dn)]
    return [u | d for u in ups for d in dns]


def _annihilate(det, p):
    if not (det >> p) & 1:
        return None, 0
    sign = -1 if bin(det & ((1 << p) - 1)).count("1") % 2 else 1
    return det ^ (1 << p), sign


def _create(det, p):
    if (det >> p) & 1:
        return None, 0
    sign = -1 if bin(det & ((1 << p) - 1)).count("1") % 2 else 1
    return det | (1 << p), sign


def _occ(det, nso):
    return [p for p in range(nso) if (det >> p) & 1]


def hamiltonian(h1, v, n_up, n_dn, e_core=0.0):
    """Dense FCI matrix of H in the determinant basis (real-valued inputs)."""
    M = h1.shape[0]
    nso = 2 * M
    dets = determinants(M, n_up, n_dn)
    index = {d: i for i, d in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)), dtype=np.result_type(h1, v))
    for col, det in enumerate(dets):
        H[col, col] += e_core
        occ = _occ(det, nso)
        # one-body: h_ij c+_i c_j over both spins
        for q in occ:
            d1, s1 = _annihilate(det, q)
            sq, j = divmod(q, M)
            for i in range(M):
                p = sq * M + i
                d2, s2 = _create(d1, p)
                if d2 is None:
                    continue
                H[index[d2], col] += h1[i, j] * s1 * s2
        # two-body: 1/2 v_ijkl c+_i c+_j c_l c_k ; first c_k, then c_l, c+_j, c+_i
        for K in occ:
            dk, sk = _annihilate(det, K)
            sK, k = divmod(K, M)
            for Lp in occ:
                if Lp == K:
                    continue
                dl, sl = _annihilate(dk, Lp)
                sL, l = divmod(Lp, M)
                for j in range(M):
                    J = sL * M + j
                    dj, sj = _create(dl, J)
                    if dj is None:
                        continue
                    for i in range(M):
                        I = sK * M + i
                        di, si = _create(dj, I)
                        if di is None:
                            continue
                        H[index[di], col] += 0.5 * v[i, j, k, l] * sk * sl * sj * si
    return H, dets


def one_body_operator(A, n_up, n_dn, spin=None):
    """FCI matrix of sum_s sum_ik A_ik c+_is c_ks (A may be complex); with
    spin = 0 or 1 only that spin's term."""
    M = A.shape[0]
    nso = 2 * M
    dets = determinants(M, n_up, n_dn)
    index = {d: i for i, d in enumerate(dets)}
    out = np.zeros((len(dets), len(dets)), dtype=np.result_type(A, np.float64))
    for col, det in enumerate(dets):
        for q in _occ(det, nso):
            d1, s1 = _annihilate(det, q)
            sq, k = divmod(q, M)
            if spin is not None and sq != spin:
                continue
            for i in range(M):
                d2, s2 = _create(d1, sq * M + i)
                if d2 is None:
                    continue
                out[index[d2], col] += A[i, k] * s1 * s2
    return out


def coefficients(W, n_up, n_dn):
    """Expansion of the Slater determinant with orbitals W = [W_up | W_dn] (M x N):
    c(D) = det W_up[D_up, :] * det W_dn[D_dn, :]."""
    M = W.shape[0]
    dets = determinants(M, n_up, n_dn)
    Wu, Wd = W[:, :n_up], W[:, n_up:n_up + n_dn]
    c = np.zeros(len(dets), dtype=np.complex128)
    for idx, det in enumerate(dets):
        up = [i for i in range(M) if (det >> i) & 1]
        dn = [i for i in range(M) if (det >> (M + i)) & 1]
        c[idx] = np.linalg.det(Wu[up, :]) * np.linalg.det(Wd[dn, :])
    return c


def ground_state(H):
    vals, vecs = np.linalg.eigh(H)
    return vals[0], vecs[:, 0]


def mixed_estimate(H, cT, cW):
    """<T|H|W> / <T|W> and <T|W>."""
    ov = np.vdot(cT, cW)
    return np.vdot(cT, H @ cW) / ov, ov
