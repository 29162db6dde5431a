"""Orthogonal multi-determinant trial for the CPU oracle.

TEST INFRASTRUCTURE ONLY (see oracle/afqmc.py).

The AFQMC section of the paper allows a trial that is a linear combination of
Slater determinants, psi_T = sum_I c_I |D_I>, and singles out expansions whose
determinants are orthogonal, <D_I|D_J> = delta_IJ (configuration-interaction
expansions of one orthonormal orbital set). Here every D_I is built from an
orthonormal basis C (M x M, shared by both spins): the reference determinant
occupies the first n_up (n_dn) columns of C in the up (down) block, and
determinant I replaces, in each spin, the hole orbitals h_q by the particle
orbitals p_q slot by slot (column h_q of the reference block becomes column
p_q of C). Distinct occupation sets make the determinants orthonormal.

The mixed estimates are written as plain sums over the determinants, each
term taken from the single-determinant formulas of oracle/afqmc.py:
    <psi_T|W>  = sum_I conj(c_I) <D_I|W>
    E_L(W)     = sum_I conj(c_I) <D_I|W> E_L[D_I](W) / <psi_T|W>
    vbar_n(W)  = sum_I conj(c_I) <D_I|W> vbar_n[D_I](W) / <psi_T|W>
(the mixed estimate of an operator for a sum of bras is the overlap-weighted
average of the per-determinant mixed estimates). No low-rank updates are
used here.
"""
from __future__ import annotations

import numpy as np

from . import afqmc


def determinant(C, n_up, n_dn, exc):
    """Orbitals (M x (n_up + n_dn)) of the determinant with excitation
    exc = ((holes_up, parts_up), (holes_dn, parts_dn))."""
    blocks = []
    for n, (holes, parts) in zip((n_up, n_dn), exc):
        if len(holes) != len(parts):
            raise ValueError("holes and particles differ in number")
        D = C[:, :n].astype(np.complex128).copy()
        for h, p in zip(holes, parts):
            if not (0 <= h < n <= p < C.shape[0]):
                raise ValueError("hole or particle out of range")
            D[:, h] = C[:, p]
        blocks.append(D)
    return np.concatenate(blocks, axis=1)


def determinants(C, n_up, n_dn, excitations):
    return [determinant(C, n_up, n_dn, e) for e in excitations]


def overlap(dets, coeffs, W, n_up, n_dn):
    """<psi_T|W> = sum_I conj(c_I) prod_s det(D_I^sH W^s)."""
    return sum(np.conj(c) * afqmc.overlap(D, W, n_up, n_dn)[0] for D, c in zip(dets, coeffs))


def local_energy(h1, chol, dets, coeffs, W, n_up, n_dn, e_core=0.0):
    """Mixed E_L of the multi-determinant trial, its one-body and two-body
    parts (E1, E2 = EJ + EK) and the force bias vbar_n, all complex."""
    num_e = num_e1 = num_e2 = 0.0
    num_v = 0.0
    den = 0.0
    for D, c in zip(dets, coeffs):
        o = afqmc.overlap(D, W, n_up, n_dn)[0]
        if o == 0.0:
            raise ValueError("a determinant is orthogonal to the walker: its per-determinant estimate "
                             "is undefined (use the determinant-space form in the tests)")
        wt = np.conj(c) * o
        e, e1, ej, ek = afqmc.local_energy_plain(h1, chol, D, W, n_up, n_dn, e_core)
        vb = afqmc.force_bias_plain(chol, afqmc.greens_function(D, W, n_up, n_dn))
        num_e = num_e + wt * e
        num_e1 = num_e1 + wt * e1
        num_e2 = num_e2 + wt * (ej + ek)
        num_v = num_v + wt * vb
        den = den + wt
    return num_e / den, num_e1 / den, num_e2 / den, num_v / den
