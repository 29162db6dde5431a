"""Parity at the full benchmark size (M=400, 100+100 electrons, 1600 Cholesky
vectors, 512 walkers, dt 0.005) in the launch configuration the benchmark
times. The oracle cannot afford 512 walkers, so sampled walkers are checked
one by one (walkers are independent given their fields) and the mixed energy
is checked as the weighted mean of the GPU's own per-walker outputs. The walk
takes 6 steps with QR every 5, so the re-orthonormalisation at 100 electrons
per spin runs and the sixth step starts from its output."""
import numpy as np
import pytest

from oracle import afqmc
from paper_2003_01831_amd import synth
from gpu_util import rel_fro, rel_vec, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.WORKLOADS["m400"]
    s = synth.make_system(cfg["M"], cfg["n_up"], cfg["n_dn"], cfg["n_chol"], seed=cfg["seed"])
    pre = afqmc.prepare(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, cfg["dt"])
    return cfg, s, pre


_oracle_cache = {}


@pytest.mark.parametrize("prec,form,tol", [("bf16x3", "auto", 1e-5), ("bf16x3", "cholesky", 1e-5),
                                           ("fp64", "auto", 1e-10)])
def test_full_size_sampled_walkers(full, prec, form, tol):
    """Split-BF16x3 in both exchange forms (the automatic choice takes the
    four-index form at this size), and FP64."""
    from paper_2003_01831_amd import api
    cfg, s, pre = full
    nw, steps, dt = cfg["n_walkers"], 6, cfg["dt"]
    fields = synth.make_fields(steps, nw, cfg["n_chol"], seed=cfg["field_seed"])
    sysg = api.System.from_synth(s, precision=prec, exchange_form=form)
    if prec == "bf16x3":
        assert sysg.exchange_form()[0] == ("four_index" if form == "auto" else "cholesky")
    wk = api.Walkers(sysg, nw)
    if "e_var" not in _oracle_cache:   # one shift for every mode, so the oracle runs once
        _oracle_cache["e_var"] = afqmc.local_energy_plain(s.h1, s.chol, s.phi_t, s.phi_t, s.n_up, s.n_dn)[0].real
    e_var = _oracle_cache["e_var"]
    out = wk.step(steps, dt, fields=fields, qr_every=cfg["qr_every"], e_shift=e_var)
    Wg = to_np(wk.get()["W"])
    torch.cuda.synchronize()
    g = {k: to_np(v) for k, v in out.items()}
    sample = np.array([0, 300, 511])
    if "run" not in _oracle_cache:
        _oracle_cache["run"] = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn,
                                         synth.trial_walkers(s, len(sample)), np.ones(len(sample)),
                                         fields[:, sample], dt, qr_every=cfg["qr_every"], e_shift=e_var, pre=pre)
    o = _oracle_cache["run"]
    for k in ("eloc", "weights", "ratio"):
        err = rel_vec(g[k][:, sample], o[k])
        print(prec, form, k, f"{err:.2e}")
        assert err < tol, k
    err = rel_fro(Wg[sample], o["W"])
    print(prec, form, "W", f"{err:.2e}")
    assert err < tol
    # E_mix is the weighted mean of the per-walker energies with the pre-step weights
    wprev = np.vstack([np.ones(nw), g["weights"][:-1]])
    ref = np.sum(wprev * g["eloc"].real, axis=1) / np.sum(wprev, axis=1)
    assert rel_vec(g["emix"], ref) < 1e-12


@pytest.mark.parametrize("prec,tol", [("bf16x3", 1e-5), ("fp64", 1e-10)])
def test_full_size_back_propagation(full, prec, tol):
    """Back-propagated 1-RDM over a 2-step window at the full size. With all 512
    walkers alive the trace of every spin block must be its electron count; with
    only the 4 sampled walkers alive (the others ride along frozen at weight 0,
    same launches) the estimate must match the oracle's over those 4."""
    from paper_2003_01831_amd import api
    cfg, s, pre = full
    nw, n_bp, dt = cfg["n_walkers"], 2, cfg["dt"]
    fields = synth.make_fields(n_bp, nw, cfg["n_chol"], seed=cfg["field_seed"])
    sysg = api.System.from_synth(s, precision=prec)
    wk = api.Walkers(sysg, nw)
    wk.bp_begin(n_bp)
    wk.step(n_bp, dt, fields=fields, qr_every=cfg["qr_every"])
    P, _ = wk.bp_rdm1(qr_every=cfg["qr_every"])
    P = to_np(P)
    for sp, n in enumerate((s.n_up, s.n_dn)):
        assert abs(np.trace(P[sp]) - n) < 1e-9 * n
    del wk
    sample = np.array([0, 137, 300, 511])
    w0 = np.zeros(nw)
    w0[sample] = 1.0
    wk = api.Walkers(sysg, nw, None, w0)
    wk.bp_begin(n_bp)
    wk.step(n_bp, dt, fields=fields, qr_every=cfg["qr_every"])
    P, wsum = wk.bp_rdm1(qr_every=cfg["qr_every"])
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, synth.trial_walkers(s, 4), np.ones(4),
                  fields[:, sample], dt, qr_every=cfg["qr_every"], pre=pre, bp_start=0, bp_len=n_bp)
    ref = afqmc.back_propagated_rdm1(pre["B1"], s.chol, s.phi_t, s.n_up, s.n_dn, o["bp_W0"], o["bp_coefs"],
                                     o["bp_weights"], order=6, qr_every=cfg["qr_every"])
    err = rel_fro(to_np(P), ref)
    print(prec, f"full-size bp rdm1 rel err {err:.2e}")
    assert err < tol
