"""Thin torch-facing binding of the C ABI (include/afq.h).

torch provides device memory and the stream; the walker step itself runs in
the HIP library. Arrays passed to the library are CUDA (HIP) tensors:
float64 for real data, complex128 for complex data, contiguous.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import EXCHANGE_FORM, PRECISION, check


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2003_01831_amd needs a ROCm GPU (gfx950); no device is visible")
    return torch.device("cuda", torch.cuda.current_device())


def _as_dev(x, dtype):
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device=_dev(), dtype=dtype).contiguous()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class System:
    """h1 (M x M), chol (X x M x M), trial phi_t (M x (n_up+n_dn)) and E_II.

    numpy inputs are handed to the library as host pointers (AFQ_HOST_PTRS:
    one host-to-device copy, no staging tensors); torch tensors are moved to
    the current device and handed over as device pointers. The library keeps
    its own copies either way."""

    def __init__(self, h1, chol, phi_t, n_up, n_dn, e_core=0.0, precision="fp64", stream=None,
                 exchange_form="auto"):
        self.lib = _lib.load()
        _dev()
        host = all(isinstance(a, np.ndarray) for a in (h1, chol, phi_t))
        if host:
            ins = [np.ascontiguousarray(h1, dtype=np.float64), np.ascontiguousarray(chol, dtype=np.float64),
                   np.ascontiguousarray(phi_t, dtype=np.complex128)]
            ptrs = [C.c_void_p(a.ctypes.data) for a in ins]
            flags = _lib.AFQ_HOST_PTRS
        else:
            ins = [_as_dev(h1, torch.float64), _as_dev(chol, torch.float64), _as_dev(phi_t, torch.complex128)]
            ptrs = [_ptr(a) for a in ins]
            flags = 0
        self.M = int(ins[0].shape[0])
        self.n_up, self.n_dn = int(n_up), int(n_dn)
        self.n_chol = int(ins[1].shape[0])
        self.e_core = float(e_core)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.precision = precision
        # a non-default exchange form is set before the precision, so that the
        # automatic choice never builds a tensor that is dropped at once (complex
        # FP32 mode has no four-index form)
        first = precision if exchange_form == "auto" else "cfp32"
        h = C.c_void_p()
        check(self.lib.afq_system_create(C.byref(h), self.M, self.n_up, self.n_dn, self.n_chol, *ptrs,
                                         self.e_core, PRECISION[first], _stream_handle(self.stream), flags))
        self.handle = h
        del ins, ptrs                 # the create call synchronised; the library owns copies
        if exchange_form != "auto":
            self.set_exchange_form(exchange_form)
            self.set_precision(precision)

    @classmethod
    def from_synth(cls, s, precision="fp64", exchange_form="auto"):
        return cls(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, s.e_core, precision, exchange_form=exchange_form)

    @classmethod
    def from_kpoint(cls, ks, precision="fp64", stream=None):
        """k-point-blocked system from a synth.KpSystem-like object (nk, m,
        n_up / n_dn per k-point, xq, kq, hk, Lk, phik, e_core)."""
        self = cls.__new__(cls)
        self.lib = _lib.load()
        self.hk = _as_dev(ks.hk, torch.complex128)
        self.Lk = _as_dev(ks.Lk, torch.complex128)
        self.phik = _as_dev(ks.phik, torch.complex128)
        kq = np.ascontiguousarray(np.asarray(ks.kq, dtype=np.int32))
        self.M = int(ks.nk * ks.m)
        self.n_up, self.n_dn = int(ks.nk * ks.n_up), int(ks.nk * ks.n_dn)
        self.n_chol = int(2 * ks.nk * ks.xq)          # auxiliary fields
        self.e_core = float(ks.e_core)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.precision = precision
        h = C.c_void_p()
        check(self.lib.afq_kp_system_create(C.byref(h), int(ks.nk), kq.ctypes.data_as(C.c_void_p), int(ks.m),
                                            int(ks.n_up), int(ks.n_dn), int(ks.xq), _ptr(self.hk), _ptr(self.Lk),
                                            _ptr(self.phik), self.e_core, PRECISION[precision],
                                            _stream_handle(self.stream)))
        self.handle = h
        return self

    def set_precision(self, precision):
        check(self.lib.afq_system_set_precision(self.handle, PRECISION[precision]))
        self.precision = precision

    def set_exchange_form(self, form):
        """"auto", "cholesky" or "four_index" (the half-rotated two-electron
        tensor; split-BF16x3 mode with a real trial only)."""
        check(self.lib.afq_system_set_exchange_form(self.handle, EXCHANGE_FORM[form]))

    def set_propagator_tile(self, tile):
        """Tile of the split-BF16x3 propagator products: 0 (224 x 160), 1 (128 x
        128), 2 (64 x 64), or -1 for the per-system choice by padded work."""
        check(self.lib.afq_system_set_propagator_tile(self.handle, int(tile)))

    def propagator_tile(self):
        """The propagator-product tile the next step uses (0..2)."""
        t = C.c_int()
        check(self.lib.afq_system_propagator_tile(self.handle, C.byref(t)))
        return int(t.value)

    def exchange_form(self):
        """(form the next step uses, device bytes of the four-index tensor)."""
        f, b = C.c_int(), C.c_uint64()
        check(self.lib.afq_system_exchange_form(self.handle, C.byref(f), C.byref(b)))
        names = {v: k for k, v in EXCHANGE_FORM.items()}
        return names[f.value], int(b.value)

    def set_background(self, on=True, vector=None):
        """Mean-field background subtraction for later steps: on with vector None
        uses the trial's own force bias; a vector (n_chol reals) is used as given."""
        v = None if vector is None else _as_dev(vector, torch.float64)
        check(self.lib.afq_system_set_background(self.handle, 1 if on else 0, _ptr(v)))

    def background(self):
        """The subtracted background vector (device tensor), or None when off."""
        on = C.c_int()
        out = torch.zeros(self.n_chol, dtype=torch.float64, device=_dev())
        check(self.lib.afq_system_background(self.handle, C.byref(on), _ptr(out)))
        torch.cuda.synchronize()
        return out if on.value else None

    MSD_KMAX = 4

    def set_msd(self, basis, excitations, coeffs):
        """Orthogonal multi-determinant trial: basis (M x M orthonormal, its first
        n columns equal to each spin block of phi_t); excitations[I] =
        ((holes_up, parts_up), (holes_dn, parts_dn)) with particle p_q taking the
        slot of hole h_q; coeffs[I] complex. Empty excitations detach it."""
        n = len(excitations)
        k = self.MSD_KMAX
        table = np.zeros((max(n, 1), 2, 1 + 2 * k), dtype=np.int32)
        for i, e in enumerate(excitations):
            for sp in range(2):
                holes, parts = e[sp]
                if len(holes) != len(parts) or len(holes) > k:
                    raise ValueError("each spin needs as many particles as holes, at most %d" % k)
                table[i, sp, 0] = len(holes)
                table[i, sp, 1:1 + len(holes)] = holes
                table[i, sp, 1 + k:1 + k + len(parts)] = parts
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.complex128).reshape(-1))
        if c.size != n:
            raise ValueError("one coefficient per determinant")
        self._msd_basis = _as_dev(basis, torch.complex128)
        check(self.lib.afq_system_set_msd(self.handle, _ptr(self._msd_basis), n, c.ctypes.data_as(C.c_void_p),
                                          table.ctypes.data_as(C.c_void_p)))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.afq_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Walkers:
    def __init__(self, system: System, n_walkers: int, w0=None, weights=None):
        self.sys = system
        self.lib = system.lib
        self.nw = int(n_walkers)
        w0t = None if w0 is None else _as_dev(w0, torch.complex128)
        wtt = None if weights is None else _as_dev(weights, torch.float64)
        h = C.c_void_p()
        check(self.lib.afq_walkers_create(C.byref(h), system.handle, self.nw, _ptr(w0t), _ptr(wtt)))
        self.handle = h

    def step(self, n_steps, dt, fields=None, seed=0, qr_every=5, e_shift=0.0, taylor_order=6,
             outputs=("emix", "eloc", "weights", "ratio")):
        dev = _dev()
        f = None if fields is None else _as_dev(fields, torch.float64)
        out = {}
        if "emix" in outputs:
            out["emix"] = torch.zeros(n_steps, dtype=torch.float64, device=dev)
        if "eloc" in outputs:
            out["eloc"] = torch.zeros(n_steps, self.nw, dtype=torch.complex128, device=dev)
        if "weights" in outputs:
            out["weights"] = torch.zeros(n_steps, self.nw, dtype=torch.float64, device=dev)
        if "ratio" in outputs:
            out["ratio"] = torch.zeros(n_steps, self.nw, dtype=torch.complex128, device=dev)
        check(self.lib.afq_step(self.sys.handle, self.handle, int(n_steps), float(dt), _ptr(f), int(seed),
                                int(qr_every), float(e_shift), int(taylor_order), _ptr(out.get("emix")),
                                _ptr(out.get("eloc")), _ptr(out.get("weights")), _ptr(out.get("ratio"))))
        return out

    def energy(self, want_vbar=False):
        dev = _dev()
        el = torch.zeros(self.nw, dtype=torch.complex128, device=dev)
        parts = torch.zeros(self.nw, 3, dtype=torch.complex128, device=dev)
        vb = torch.zeros(self.nw, self.sys.n_chol, dtype=torch.complex128, device=dev) if want_vbar else None
        em = torch.zeros(1, dtype=torch.float64, device=dev)
        check(self.lib.afq_energy(self.sys.handle, self.handle, _ptr(el), _ptr(parts), _ptr(vb), _ptr(em)))
        return el, parts, vb, em

    def get(self, want_logovlp=False):
        dev = _dev()
        W = torch.zeros(self.nw, self.sys.M, self.sys.n_up + self.sys.n_dn, dtype=torch.complex128, device=dev)
        wt = torch.zeros(self.nw, dtype=torch.float64, device=dev)
        al = torch.zeros(self.nw, dtype=torch.int32, device=dev)
        lo = torch.zeros(self.nw, dtype=torch.complex128, device=dev) if want_logovlp else None
        ctr = C.c_uint64()
        check(self.lib.afq_walkers_get(self.handle, _ptr(W), _ptr(wt), _ptr(lo), _ptr(al), C.byref(ctr)))
        return dict(W=W, weights=wt, alive=al, logovlp=lo, counter=int(ctr.value))

    def set(self, W=None, weights=None, alive=None, counter=0):
        Wt = None if W is None else _as_dev(W, torch.complex128)
        wt = None if weights is None else _as_dev(weights, torch.float64)
        al = None if alive is None else _as_dev(alive, torch.int32)
        check(self.lib.afq_walkers_set(self.handle, _ptr(Wt), _ptr(wt), _ptr(al), int(counter)))
        torch.cuda.synchronize()

    def stats(self):
        na, nk = C.c_int(), C.c_int64()
        check(self.lib.afq_walkers_stats(self.handle, C.byref(na), C.byref(nk)))
        return int(na.value), int(nk.value)

    def autotune(self, reps=3):
        """Pick the fastest exchange-kernel variant for these walkers (returned
        per spin) and, in split-BF16x3 mode, the fastest propagator-product
        tile for the system (System.propagator_tile)."""
        ch = (C.c_int * 2)()
        check(self.lib.afq_autotune(self.sys.handle, self.handle, int(reps), C.cast(ch, C.c_void_p)))
        return int(ch[0]), int(ch[1])

    def set_controls(self, fb_cap=0.0, w_cap=0.0):
        """Force-bias and weight caps for later steps (0 = off)."""
        check(self.lib.afq_walkers_set_controls(self.handle, float(fb_cap), float(w_cap)))

    def comb(self, xi):
        """Systematic resampling to equal weights; returns (source indices, total weight)."""
        src = np.zeros(self.nw, dtype=np.int32)
        tot = C.c_double()
        check(self.lib.afq_walkers_comb(self.handle, float(xi), src.ctypes.data_as(C.c_void_p), C.byref(tot)))
        return src, float(tot.value)

    def bp_begin(self, n_bp):
        """Open a back-propagation window of n_bp steps on the current walkers."""
        check(self.lib.afq_bp_begin(self.handle, int(n_bp)))

    def bp_rdm1(self, qr_every=0):
        """Back-propagated spin-resolved 1-RDM P[s, i, j] = <c+_is c_js> (2 x M x M
        complex128 on the device) and the total weight at the end of the window."""
        M = self.sys.M
        out = torch.zeros(2, M, M, dtype=torch.complex128, device=_dev())
        wsum = C.c_double()
        check(self.lib.afq_bp_rdm1(self.handle, int(qr_every), _ptr(out), C.byref(wsum)))
        return out, float(wsum.value)

    def bp_end(self):
        check(self.lib.afq_bp_end(self.handle))

    def set_exchange_variant(self, spin, variant):
        check(self.lib.afq_exchange_variant(self.handle, int(spin), int(variant)))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.afq_walkers_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy_backward(system: System, walkers: Walkers, scale=1.0, want=("h1", "chol", "walkers")):
    dev = _dev()
    M, X = system.M, system.n_chol
    dh = torch.zeros(M, M, dtype=torch.float64, device=dev) if "h1" in want else None
    dl = torch.zeros(X, M, M, dtype=torch.float64, device=dev) if "chol" in want else None
    dw = (torch.zeros(walkers.nw, M, system.n_up + system.n_dn, dtype=torch.complex128, device=dev)
          if "walkers" in want else None)
    check(system.lib.afq_energy_backward(system.handle, walkers.handle, float(scale), _ptr(dh), _ptr(dl), _ptr(dw)))
    return dh, dl, dw


def eshift_update(e_est, w_total, w_target, dt, gain_steps):
    out = C.c_double()
    check(_lib.load().afq_eshift_update(float(e_est), float(w_total), float(w_target), float(dt), float(gain_steps),
                                        C.byref(out)))
    return float(out.value)


def fields_generate(seed, n_steps, n_walkers, n_chol, step0=0, sys_id=0):
    lib = _lib.load()
    out = torch.zeros(n_steps, n_walkers, n_chol, dtype=torch.float64, device=_dev())
    check(lib.afq_fields_generate(int(seed), int(sys_id), int(step0), int(n_steps), int(n_walkers), int(n_chol),
                                  _ptr(out), _stream_handle(None)))
    return out


class Batch:
    """Several (System, Walkers) pairs stepped together as branches of one
    captured HIP graph (system i draws Philox fields with sys_id = i)."""

    def __init__(self, pairs):
        self.pairs = list(pairs)
        if not self.pairs:
            raise ValueError("Batch needs at least one (system, walkers) pair")
        self.lib = self.pairs[0][0].lib
        n = len(self.pairs)
        self._sys = (C.c_void_p * n)(*[p[0].handle.value for p in self.pairs])
        self._wk = (C.c_void_p * n)(*[p[1].handle.value for p in self.pairs])
        h = C.c_void_p()
        check(self.lib.afq_batch_create(C.byref(h), n, C.cast(self._sys, C.c_void_p), C.cast(self._wk, C.c_void_p)))
        self.handle = h

    def step(self, n_steps, dt, seed=0, qr_every=5, e_shift=0.0, taylor_order=6, emix=True):
        n = len(self.pairs)
        es = np.broadcast_to(np.asarray(e_shift, dtype=np.float64), (n,)).copy()
        out = torch.zeros(n, n_steps, dtype=torch.float64, device=_dev()) if emix else None
        check(self.lib.afq_batch_step(self.handle, int(n_steps), float(dt), int(seed), int(qr_every),
                                      es.ctypes.data_as(C.c_void_p), int(taylor_order), _ptr(out)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.afq_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
