"""Tiles of the split-BF16x3 propagator products (the Horner products of the
Taylor propagator and the two B1 products): every tile gives the oracle's
walk, the tiles agree with each other bit for bit (each output element sums
the same 32-element chunks in the same order whatever the tile), the
padded-work model picks the small tile for a small system and the large one
for the large walker shape, and the autotuner's pick leaves the walkers
unchanged."""
import numpy as np
import pytest

from oracle import afqmc
from paper_2003_01831_amd import synth
from gpu_util import rel_fro, rel_vec, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api
    return api


# (M, n_up, n_dn, X, walkers): ragged against every tile (n_tot = 11 and 2M =
# 60 against 64-row tiles; n_tot = 58 and 2M = 136 against 128 and 224 x 160)
SHAPES = [(30, 6, 5, 40, 5), (68, 30, 28, 90, 7)]


def _walk(api, s, tile, nw, steps, dt):
    g = api.System.from_synth(s, precision="bf16x3")
    g.set_propagator_tile(tile)
    assert g.propagator_tile() == tile
    W0 = synth.perturbed_walkers(s, nw, 0.05, seed=601)
    fields = synth.make_fields(steps, nw, s.n_chol, seed=602)
    wk = api.Walkers(g, nw, W0)
    out = wk.step(steps, dt, fields=fields, qr_every=3)
    res = {k: to_np(v) for k, v in out.items()}
    res["W"] = to_np(wk.get()["W"])
    torch.cuda.synchronize()
    return res, W0, fields


@pytest.mark.parametrize("shape", SHAPES)
def test_every_tile_matches_the_oracle_and_the_others(api, shape):
    M, nu, nd, X, nw = shape
    s = synth.make_system(M, nu, nd, X, seed=M + X)
    steps, dt = 4, 0.01
    runs = [_walk(api, s, t, nw, steps, dt) for t in (0, 1, 2)]
    _, W0, fields = runs[0]
    o = afqmc.run(s.h1, s.chol, s.phi_t, nu, nd, W0, np.ones(nw), fields, dt, qr_every=3)
    for t, (r, _, _) in enumerate(runs):
        for k in ("emix", "eloc", "weights", "ratio"):
            assert rel_vec(r[k], o[k]) < 1e-5, (t, k)
        assert rel_fro(r["W"], o["W"]) < 1e-5, t
    for t in (1, 2):
        for k in runs[0][0]:
            assert np.array_equal(runs[t][0][k], runs[0][0][k]), (t, k)


def test_model_choice_and_pinning(api):
    small = api.System.from_synth(synth.make_system(64, 16, 16, 64, seed=611), precision="bf16x3")
    assert small.propagator_tile() == 2            # n_tot = 32, 2M = 128: the 64 x 64 tile
    # the M = 400 walker shape (n_tot = 200, 2M = 800) keeps the 224 x 160 tile;
    # only the shape matters to the model, so few vectors suffice
    big = api.System.from_synth(synth.make_system(400, 100, 100, 8, seed=612), precision="bf16x3")
    assert big.propagator_tile() == 0
    big.set_propagator_tile(1)
    assert big.propagator_tile() == 1
    big.set_propagator_tile(-1)
    assert big.propagator_tile() == 0
    from paper_2003_01831_amd._lib import AfqError
    with pytest.raises(AfqError):
        big.set_propagator_tile(3)


def test_autotune_picks_a_tile_and_keeps_the_walkers(api):
    s = synth.make_system(68, 30, 28, 90, seed=621)
    nw, steps, dt = 7, 3, 0.01
    g = api.System.from_synth(s, precision="bf16x3")
    W0 = synth.perturbed_walkers(s, nw, 0.05, seed=622)
    fields = synth.make_fields(2 * steps, nw, s.n_chol, seed=623)
    wk = api.Walkers(g, nw, W0)
    wk.step(steps, dt, fields=fields[:steps], qr_every=0)
    before = wk.get()
    wk.autotune(reps=2)
    assert g.propagator_tile() in (0, 1, 2)
    after = wk.get()
    assert torch.equal(before["W"], after["W"]) and torch.equal(before["weights"], after["weights"])
    out = wk.step(steps, dt, fields=fields[steps:], qr_every=0)
    torch.cuda.synchronize()
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, np.ones(nw), fields, dt, qr_every=0)
    assert rel_vec(to_np(out["weights"])[-1], o["weights"][-1]) < 1e-5
    assert rel_fro(to_np(wk.get()["W"]), o["W"]) < 1e-5
