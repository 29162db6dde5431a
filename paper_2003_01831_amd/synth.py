"""Seeded synthetic inputs for the phaseless-AFQMC walker step.

This module only draws random numbers and assembles input arrays; it holds none
of the method's arithmetic (no Green's function, propagator, energy or weight).
Both the CPU oracle tests and the GPU path take their inputs from here, so a
parity test feeds the two sides bit-identical arrays.

Recipe (shared by every workload):

* ``h1`` is a real symmetric M x M matrix. The upper triangle, diagonal
  included, is drawn i.i.d. N(0,1)/M and mirrored, so every entry has exactly
  that distribution.
* ``chol[n]`` (n = 0..X-1) are real symmetric M x M matrices drawn the same way
  with scale exp(-n/8)/M, so that the two-electron tensor
  v_ijkl = sum_n L^n_ik L^n_jl (the modified-Cholesky form of the paper's
  Section "Auxiliary Field Quantum Monte Carlo") is positive semi-definite.
* The trial ``phi_t`` holds the lowest-N eigenvectors of h1 (ascending order)
  for each spin, with the sign of each column fixed so that its largest-modulus
  entry is positive. Columns 0..n_up-1 are the up spin, the rest the down spin.
* Auxiliary fields are i.i.d. standard normal, shape (steps, walkers, X).

The paper's own AFQMC workloads (NaCl, acenes, ...) need molecular integrals that
are not available; these arrays stand in with the shape regime of the dense
3-index factorisation (M <= 1000, X = x_c M).
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class System:
    M: int
    n_up: int
    n_dn: int
    n_chol: int
    h1: np.ndarray        # (M, M) float64
    chol: np.ndarray      # (X, M, M) float64
    phi_t: np.ndarray     # (M, n_up + n_dn) complex128
    e_core: float = 0.0

    @property
    def n_tot(self) -> int:
        return self.n_up + self.n_dn


def _sym_draw(rng, shape_prefix, M, scale):
    a = rng.standard_normal(tuple(shape_prefix) + (M, M))
    up = np.triu(a)
    out = up + np.swapaxes(np.triu(a, 1), -1, -2)
    return out * scale


def _lowest_eigvecs(h, n):
    vals, vecs = np.linalg.eigh(h)
    v = vecs[:, :n].copy()
    for j in range(n):
        k = int(np.argmax(np.abs(v[:, j])))
        if v[k, j] < 0:
            v[:, j] = -v[:, j]
    return v


def make_system(M: int, n_up: int, n_dn: int, n_chol: int, seed: int,
                decay: float = 8.0, e_core: float = 0.0) -> System:
    rng = np.random.default_rng(seed)
    h1 = _sym_draw(rng, (), M, 1.0 / M)
    scales = np.exp(-np.arange(n_chol) / decay) / M
    chol = np.empty((n_chol, M, M))
    # draw one matrix at a time to keep peak memory at one chol copy
    for n in range(n_chol):
        chol[n] = _sym_draw(rng, (), M, scales[n])
    vu = _lowest_eigvecs(h1, n_up)
    vd = _lowest_eigvecs(h1, n_dn)
    phi_t = np.concatenate([vu, vd], axis=1).astype(np.complex128)
    return System(M, n_up, n_dn, n_chol, h1, chol, phi_t, e_core)


def make_fields(n_steps: int, n_walkers: int, n_chol: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_steps, n_walkers, n_chol))


def trial_walkers(sys: System, n_walkers: int) -> np.ndarray:
    return np.broadcast_to(sys.phi_t, (n_walkers,) + sys.phi_t.shape).copy()


def perturbed_walkers(sys: System, n_walkers: int, scale: float, seed: int) -> np.ndarray:
    """W = T + scale (Z1 + i Z2)/sqrt(2), independently per walker and spin."""
    rng = np.random.default_rng(seed)
    shape = (n_walkers,) + sys.phi_t.shape
    z = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    return sys.phi_t[None] + scale * z


def random_weights(n_walkers: int, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, n_walkers)


def make_msd(sys: System, n_det: int, n_occ_act: int, n_vir_act: int, k_max: int, seed: int,
             decay: float = 0.3):
    """Orthogonal multi-determinant trial for `sys`: the basis C holds every
    eigenvector of h1 with the sign rule of the trial (its first n columns are
    the trial's spin blocks); determinant 0 is the reference and the others
    draw, per spin, k <= k_max holes among the n_occ_act highest occupied and
    as many particles among the n_vir_act lowest virtual orbitals (holes and
    particles each ascending, paired in that order), every (up, down) pair
    distinct. Coefficients: 1 for the reference, complex normal times
    decay^(k_up + k_dn) otherwise. Returns (C (M x M complex128), excitations,
    coeffs (complex128)); excitations[I] = ((holes_up, parts_up), (holes_dn, parts_dn))."""
    rng = np.random.default_rng(seed)
    C = _lowest_eigvecs(sys.h1, sys.M).astype(np.complex128)
    seen = {((), (), (), ())}
    exc = [(((), ()), ((), ()))]
    coeffs = [1.0 + 0.0j]
    tries = 0
    while len(exc) < n_det:
        tries += 1
        if tries > 100 * n_det:
            raise ValueError("make_msd: the active space has too few distinct determinants")
        per_spin = []
        for n in (sys.n_up, sys.n_dn):
            k = int(rng.integers(0, k_max + 1))
            k = min(k, n_occ_act, n_vir_act, n)
            holes = tuple(sorted(rng.choice(np.arange(n - min(n_occ_act, n), n), k, replace=False).tolist()))
            parts = tuple(sorted(rng.choice(np.arange(n, min(n + n_vir_act, sys.M)), k, replace=False).tolist()))
            per_spin.append((holes, parts))
        key = per_spin[0] + per_spin[1]
        if key in seen:
            continue
        seen.add(key)
        exc.append(tuple(per_spin))
        rank = len(per_spin[0][0]) + len(per_spin[1][0])
        coeffs.append(decay ** rank * (rng.standard_normal() + 1j * rng.standard_normal()) / np.sqrt(2.0))
    return C, exc, np.asarray(coeffs, dtype=np.complex128)


@dataclasses.dataclass
class KpSystem:
    """k-point-blocked system: nk k-points on a ring (k + Q = (k + Q) mod nk),
    m orbitals per k-point, n_up/n_dn electrons per k-point and spin."""
    nk: int
    m: int
    n_up: int
    n_dn: int
    xq: int
    kq: np.ndarray        # (nk, nk) int: kq[Q][k] = index of k + Q
    hk: np.ndarray        # (nk, m, m) complex128 Hermitian blocks
    Lk: np.ndarray        # (nk, nk, xq, m, m) complex128: Lk[Q, k, n] couples (k + Q) <- k
    phik: np.ndarray      # (nk, m, n_up + n_dn) complex128 trial blocks
    e_core: float = 0.0


def _fix_phase(v):
    """Column phases: the entry of largest modulus made real positive."""
    v = v.copy()
    for j in range(v.shape[1]):
        k = int(np.argmax(np.abs(v[:, j])))
        v[:, j] *= np.abs(v[k, j]) / v[k, j]
    return v


def make_kpoint_system(nk: int, m: int, n_up: int, n_dn: int, xq: int, seed: int,
                       decay: float = 8.0) -> KpSystem:
    """Random Hermitian h^k (scale 1/M) and Cholesky blocks with the symmetry of
    a periodic Hermitian interaction, L^{-Q, k+Q}_n = (L^{Q,k}_n)^+ (drawn for
    one Q of each (Q, -Q) pair; Q = -Q blocks made consistent), scaled by
    exp(-n / decay) / M. The trial takes the n lowest eigenvectors of each h^k."""
    rng = np.random.default_rng(seed)
    M = nk * m
    kq = np.array([[(k + Q) % nk for k in range(nk)] for Q in range(nk)], dtype=np.int64)
    a = rng.standard_normal((nk, m, m)) + 1j * rng.standard_normal((nk, m, m))
    hk = (a + np.conj(np.swapaxes(a, 1, 2))) / (2.0 * M)
    scales = np.exp(-np.arange(xq) / decay) / M
    Lk = np.zeros((nk, nk, xq, m, m), np.complex128)
    done = np.zeros((nk, nk), bool)
    for Q in range(nk):
        mQ = (-Q) % nk
        for k in range(nk):
            if done[Q, k]:
                continue
            z = (rng.standard_normal((xq, m, m)) + 1j * rng.standard_normal((xq, m, m))) * scales[:, None, None]
            k2 = kq[Q][k]
            if (mQ, k2) == (Q, k):              # Q = -Q and k + Q = k: the block must be Hermitian
                z = 0.5 * (z + np.conj(np.swapaxes(z, 1, 2)))
            Lk[Q, k] = z
            Lk[mQ, k2] = np.conj(np.swapaxes(z, 1, 2))
            done[Q, k] = done[mQ, k2] = True
    phik = np.zeros((nk, m, n_up + n_dn), np.complex128)
    for k in range(nk):
        _, v = np.linalg.eigh(hk[k])
        phik[k, :, :n_up] = _fix_phase(v[:, :n_up])
        phik[k, :, n_up:] = _fix_phase(v[:, :n_dn])
    return KpSystem(nk, m, n_up, n_dn, xq, kq, hk, Lk, phik)


# ---------------------------------------------------------------------------
# Named workloads. Seeds: systems 1..5, fields 1001..1005, uneven systems 4000+s.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "tiny_m8": dict(M=8, n_up=2, n_dn=2, n_chol=24, n_walkers=32, dt=0.01,
                    n_steps=50, qr_every=5, seed=1, field_seed=1001),
    "m128": dict(M=128, n_up=32, n_dn=32, n_chol=512, n_walkers=256, dt=0.005,
                 n_steps=200, qr_every=5, seed=2, field_seed=1002),
    "grad_m64": dict(M=64, n_up=16, n_dn=16, n_chol=256, n_walkers=64, dt=0.005,
                     n_steps=0, qr_every=5, seed=3, field_seed=1003, perturb=0.1),
    "m400": dict(M=400, n_up=100, n_dn=100, n_chol=1600, n_walkers=512, dt=0.005,
                 n_steps=100, qr_every=5, seed=5, field_seed=1005),
    # orthogonal multi-determinant trial: 256 determinants drawn in an active
    # space of 8 occupied and 16 virtual orbitals per spin, rank <= 4 per spin
    # k-point-blocked Cholesky: 8 k-points on a ring, 24 orbitals and 6 + 6
    # electrons per k-point, 96 vectors per momentum transfer (M = 192, N = 48
    # per spin, 768 complex vectors, 1536 auxiliary fields)
    "kp_m192": dict(nk=8, m=24, n_up=6, n_dn=6, xq=96, n_walkers=256, dt=0.005, n_steps=100, qr_every=5,
                    seed=7, field_seed=1007),
    "msd_m128": dict(M=128, n_up=16, n_dn=16, n_chol=512, n_walkers=256, dt=0.005,
                     n_steps=100, qr_every=5, seed=6, field_seed=1006, n_det=256, occ_act=8,
                     vir_act=16, k_max=4, msd_seed=2006),
}


def uneven_systems(n_systems: int = 24, seed: int = 4000, m_lo: int = 32, m_hi: int = 256,
                   nw_lo: int = 16, nw_hi: int = 128):
    """Shapes for many uneven systems: M uniform over multiples of 4 in [m_lo, m_hi],
    N_up = N_dn = M/4, X = 4M, walker count uniform in [nw_lo, nw_hi]."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo // 4, m_hi // 4 + 1, n_systems) * 4
    nws = rng.integers(nw_lo, nw_hi + 1, n_systems)
    out = []
    for s in range(n_systems):
        M = int(ms[s])
        out.append(dict(M=M, n_up=M // 4, n_dn=M // 4, n_chol=4 * M, n_walkers=int(nws[s]),
                        seed=seed + s))
    return out
