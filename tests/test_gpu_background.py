"""Mean-field background subtraction on the GPU (afq_system_set_background)
against the CPU FP64 oracle's subtracted walk: the trial's mean-field vector,
walks in every precision with the trial's background and with a caller's
vector, a multi-determinant trial, switching the subtraction off again, and
the state checks. The Cholesky vectors get a diagonal part so the mean field
is large (about 1 per vector), as in real molecules."""
import numpy as np
import pytest

from oracle import afqmc, msd
from paper_2003_01831_amd import synth
from gpu_util import rel_fro, rel_vec, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-10, "cfp32": 1e-5, "bf16x3": 1e-5}


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api
    return api


def _system(M=24, nu=5, nd=4, X=30, seed=501):
    s = synth.make_system(M, nu, nd, X, seed=seed, e_core=0.3)
    diag = np.random.default_rng(seed).uniform(-0.2, 0.2, X)
    s.chol = s.chol + diag[:, None, None] * np.eye(M)[None]
    return s


def test_background_vector_is_the_trials_mean_field(api):
    s = _system()
    g = api.System.from_synth(s)
    assert g.background() is None
    g.set_background(True)
    got = to_np(g.background())
    ref = afqmc.mean_field_bias(s.chol, s.phi_t, s.n_up, s.n_dn)
    assert np.max(np.abs(ref)) > 0.5
    assert rel_vec(got, ref) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "cfp32", "bf16x3"])
@pytest.mark.parametrize("which", ["mean_field", "given"])
def test_subtracted_walk_matches_the_oracle(api, prec, which):
    s = _system()
    nw, steps, dt = 8, 10, 0.01
    # a caller's background: the mean field moved by up to 0.1 per vector (a far-off
    # vector adds phase instead of removing it and leaves weights ill-conditioned)
    vmf = afqmc.mean_field_bias(s.chol, s.phi_t, s.n_up, s.n_dn)
    if which == "given":
        vmf = vmf + np.random.default_rng(7).uniform(-0.1, 0.1, s.n_chol)
    W0 = synth.perturbed_walkers(s, nw, 0.05, seed=502)
    w0 = synth.random_weights(nw, seed=503)
    fields = synth.make_fields(steps, nw, s.n_chol, seed=504)
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, w0, fields, dt, qr_every=5, e_shift=-0.5,
                  e_core=s.e_core, vmf=vmf)
    g = api.System.from_synth(s, precision=prec)
    g.set_background(True, None if which == "mean_field" else vmf)
    wk = api.Walkers(g, nw, W0, w0)
    out = wk.step(steps, dt, fields=fields, qr_every=5, e_shift=-0.5)
    W = to_np(wk.get()["W"])
    torch.cuda.synchronize()
    errs = {k: rel_vec(to_np(out[k]), o[k]) for k in ("emix", "eloc", "weights", "ratio")}
    errs["W"] = rel_fro(W, o["W"])
    print(prec, which, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < TOL[prec], (k, v)


def test_subtracted_walk_with_a_multi_determinant_trial(api):
    s = synth.make_system(16, 5, 4, 30, seed=511, e_core=0.4)
    s.chol = 2.0 * s.chol + 0.1 * np.eye(16)[None]
    C, exc, coeffs = synth.make_msd(s, 30, 4, 6, 4, seed=512, decay=0.6)
    dets = msd.determinants(C, s.n_up, s.n_dn, exc)
    nw, steps, dt = 6, 4, 0.02
    W0 = synth.perturbed_walkers(s, nw, 0.1, seed=513)
    fields = synth.make_fields(steps, nw, s.n_chol, seed=514)
    vmf = afqmc.mean_field_bias(s.chol, s.phi_t, s.n_up, s.n_dn)
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, np.ones(nw), fields, dt, qr_every=2, e_core=0.4,
                  msd=dict(dets=dets, coeffs=coeffs), vmf=vmf)
    g = api.System.from_synth(s)
    g.set_msd(C, exc, coeffs)
    g.set_background(True)
    wk = api.Walkers(g, nw, W0)
    out = wk.step(steps, dt, fields=fields, qr_every=2, outputs=("eloc", "weights", "ratio"))
    torch.cuda.synchronize()
    for k in ("eloc", "weights", "ratio"):
        assert rel_vec(to_np(out[k]), o[k]) < 1e-10, k


def test_switching_off_restores_the_plain_walk_and_state_checks(api):
    s = _system(seed=521)
    nw = 5
    fields = synth.make_fields(6, nw, s.n_chol, seed=522)
    ref_sys = api.System.from_synth(s)
    ref = api.Walkers(ref_sys, nw).step(6, 0.01, fields=fields, qr_every=3)
    g = api.System.from_synth(s)
    g.set_background(True)
    api.Walkers(g, nw).step(2, 0.01, fields=fields[:2], qr_every=3)     # B1 built with the background
    g.set_background(False)
    got = api.Walkers(g, nw).step(6, 0.01, fields=fields, qr_every=3)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
    from paper_2003_01831_amd._lib import AfqError
    wk = api.Walkers(g, nw)
    wk.bp_begin(3)
    wk.step(1, 0.01, fields=fields[:1], qr_every=0)
    g.set_background(True)
    with pytest.raises(AfqError):                 # a window must not span a change
        wk.step(1, 0.01, fields=fields[1:2], qr_every=0)
    with pytest.raises(AfqError):
        g.set_background(True, np.full(s.n_chol, np.nan))
    ks = synth.make_kpoint_system(2, 3, 1, 1, 2, seed=523)
    gk = api.System.from_kpoint(ks)
    with pytest.raises(AfqError):
        gk.set_background(True)
