"""Counter-based Philox4x32-10 generator and Box-Muller normals, on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/afqmc.py).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
  (c0, c1, c2, c3) -> (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))
with A = 0xD2511F53, B = 0xCD9E8D57, and the key bumped by the Weyl constants
(0x9E3779B9, 0xBB67AE85) between rounds.

Auxiliary-field mapping used by the library (an interface, restated here
independently of the GPU code): field x[step, w, n] of system `sys_id` comes
from the block with counter (n // 2, w, step, sys_id) and key (seed lo32,
seed hi32). From its outputs r0..r3,
  u1 = ((r1 << 32 | r0) >> 11 + 0.5) * 2^-53     in (0, 1)
  u2 = ((r3 << 32 | r2) >> 11) * 2^-53           in [0, 1)
  x[2j]   = sqrt(-2 ln u1) cos(2 pi u2)
  x[2j+1] = sqrt(-2 ln u1) sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_A = np.uint64(0xD2511F53)
_B = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32-valued, key: (..., 2). Returns (..., 4) uint32 array."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & _MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & _MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _A * c[0]
        p1 = _B * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [(hi1 ^ c[1] ^ k0) & _MASK, lo1, (hi0 ^ c[3] ^ k1) & _MASK, lo0]
    return np.stack(c, axis=-1).astype(np.uint32)


def normal_fields(seed, n_steps, n_walkers, n_chol, step0=0, sys_id=0):
    """Standard-normal fields x[step, w, n] for steps step0..step0+n_steps-1."""
    npair = (n_chol + 1) // 2
    s, w, j = np.meshgrid(np.arange(step0, step0 + n_steps, dtype=np.uint64),
                          np.arange(n_walkers, dtype=np.uint64),
                          np.arange(npair, dtype=np.uint64), indexing="ij")
    ctr = np.stack([j, w, s, np.full_like(j, sys_id)], axis=-1)
    seed = int(seed)
    key = np.broadcast_to(np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF],
                                   dtype=np.uint64), ctr.shape[:-1] + (2,))
    r = philox4x32_10(ctr, key).astype(np.uint64)
    a = (r[..., 1] << np.uint64(32)) | r[..., 0]
    b = (r[..., 3] << np.uint64(32)) | r[..., 2]
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(u1.shape + (2,))
    z[..., 0] = rad * np.cos(2.0 * np.pi * u2)
    z[..., 1] = rad * np.sin(2.0 * np.pi * u2)
    return z.reshape(n_steps, n_walkers, 2 * npair)[:, :, :n_chol]
