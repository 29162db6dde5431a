"""MI355X (gfx950) phaseless-AFQMC walker step.

The batched walker step of Cholesky-factorised phaseless auxiliary-field QMC
(mixed Green's function, force bias, Taylor propagator with the phaseless
weight update, half-rotated Coulomb/exchange local energy, periodic QR, the
adjoint of the local energy) as a C-ABI HIP library (include/afq.h,
libafq.so) with a thin torch binding.

Importing the package does not load the library; the binding does on first
use and raises if it has not been built (there is no CPU fallback).
"""
from __future__ import annotations

__all__ = ["System", "Walkers", "Batch", "energy_backward", "fields_generate", "LocalEnergy", "synth"]


def __getattr__(name):
    if name in ("System", "Walkers", "Batch", "energy_backward", "fields_generate"):
        from . import api
        return getattr(api, name)
    if name == "LocalEnergy":
        from .autograd import LocalEnergy
        return LocalEnergy
    if name == "Batch":
        from .batch import Batch
        return Batch
    raise AttributeError(name)
