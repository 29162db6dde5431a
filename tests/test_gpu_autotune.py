"""Launch variants of the generic exchange kernel and the autotuner: every
variant that fits a shape gives the oracle's energies, and tuning leaves the
walkers unchanged."""
import numpy as np
import pytest

from oracle import afqmc
from paper_2003_01831_amd import synth
from gpu_util import rel_vec, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api
    return api


TOL = {"fp64": 1e-10, "cfp32": 1e-5, "bf16x3": 1e-5}


@pytest.mark.parametrize("prec", ["fp64", "cfp32", "bf16x3"])
@pytest.mark.parametrize("shape", [(24, 5, 3, 40), (64, 16, 16, 96), (128, 40, 33, 64), (200, 60, 60, 32),
                                   (160, 100, 100, 24), (240, 120, 120, 48)])
def test_every_variant_matches_oracle(api, prec, shape):
    M, nu, nd, X = shape
    if prec == "fp64" and max(nu, nd) > 100:
        pytest.skip("FP64 mode holds at most 100 electrons per spin")
    s = synth.make_system(M, nu, nd, X, seed=M + 3 * X)
    nw = 5
    W = synth.perturbed_walkers(s, nw, 0.1, seed=12)
    w = synth.random_weights(nw, seed=13)
    ht, Lt = afqmc.half_rotate(s.h1, s.chol, s.phi_t, nu, nd)
    ref = np.zeros((nw, 3), complex)
    for i in range(nw):
        ref[i] = afqmc.local_energy_half(ht, Lt, s.phi_t, W[i], nu, nd, s.e_core)[1]
    g = api.System.from_synth(s, precision=prec)
    wk = api.Walkers(g, nw, W, w)
    from paper_2003_01831_amd._lib import AfqError
    ran = 0
    for v in range(3):
        wk.set_exchange_variant(0, v)
        wk.set_exchange_variant(1, v)
        try:
            _, parts, _, _ = wk.energy()
        except AfqError as e:
            assert "LDS" in str(e) or "UNSUPPORTED" in str(e), str(e)
            continue
        torch.cuda.synchronize()
        p = to_np(parts)
        for c in (1, 2):
            err = rel_vec(p[:, c], ref[:, c])
            assert err < TOL[prec], (v, c, err)
        ran += 1
    assert ran >= 1


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_autotune_keeps_walkers_and_energy(api, prec):
    s = synth.make_system(96, 24, 20, 192, seed=21)
    nw = 12
    W = synth.perturbed_walkers(s, nw, 0.05, seed=22)
    g = api.System.from_synth(s, precision=prec)
    wk = api.Walkers(g, nw, W)
    e0 = to_np(wk.energy()[0])
    before = wk.get()
    choice = wk.autotune(reps=2)
    assert all(c in (0, 1, 2) for c in choice), choice
    after = wk.get()
    assert torch.equal(before["W"], after["W"]) and torch.equal(before["weights"], after["weights"])
    e1 = to_np(wk.energy()[0])
    assert rel_vec(e1, e0) < TOL[prec]
    # a second walker set of the same shape starts from the tuned table
    wk2 = api.Walkers(g, nw, W)
    assert rel_vec(to_np(wk2.energy()[0]), e0) < TOL[prec]


def test_autotune_reports_single_kernel_shapes(api):
    s = synth.make_system(128, 80, 70, 32, seed=23)
    g = api.System.from_synth(s, precision="bf16x3")
    wk = api.Walkers(g, 4)
    assert wk.autotune(reps=1) == (-1, -1)
