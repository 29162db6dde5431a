"""Population control on the GPU (force-bias cap, weight cap, comb resampling,
energy-shift feedback) against the CPU oracle."""
import numpy as np
import pytest

from oracle import afqmc
from paper_2003_01831_amd import synth
from gpu_util import rel_vec, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api
    return api


def test_comb_indices_match_the_oracle_bitwise(api):
    s = synth.make_system(12, 3, 3, 20, seed=31)
    nw = 300
    rng = np.random.default_rng(32)
    w = rng.uniform(0.1, 2.5, nw)
    w[rng.choice(nw, 40, replace=False)] = 0.0
    g = api.System.from_synth(s)
    wk = api.Walkers(g, nw)
    W0 = wk.get()["W"]
    alive = (w > 0).astype(np.int32)
    for xi in (0.0, 0.37, 0.999):
        wk.set(W0, w, alive, counter=0)
        src, total = wk.comb(xi)
        osrc, onew, ototal = afqmc.comb(w, xi)
        assert np.array_equal(src, osrc), xi
        assert total == ototal
        st = wk.get()
        assert np.all(to_np(st["weights"]) == onew)
        assert np.all(to_np(st["alive"]) == 1)
        assert torch.equal(st["W"], W0[torch.as_tensor(osrc, device=W0.device).long()])


def test_comb_of_a_dead_population_is_an_error(api):
    s = synth.make_system(8, 2, 2, 12, seed=33)
    g = api.System.from_synth(s)
    wk = api.Walkers(g, 6)
    wk.set(weights=np.zeros(6), alive=np.zeros(6, dtype=np.int32))
    from paper_2003_01831_amd._lib import AfqError
    with pytest.raises(AfqError):
        wk.comb(0.5)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 1e-5)])
def test_controlled_walk_matches_the_oracle(api, prec, tol):
    """Force-bias cap that binds, a weight cap, and a comb every 3 steps over 9
    steps (QR every 2): energies and weights against the oracle, comb sources
    identical."""
    s = synth.make_system(16, 4, 3, 40, seed=34)
    s.chol = s.chol * 2.0
    nw, steps, dt = 24, 9, 0.02
    W0 = synth.perturbed_walkers(s, nw, 0.1, seed=35)
    w0 = synth.random_weights(nw, seed=36)
    fields = synth.make_fields(steps, nw, 40, seed=37)
    xi = [0.21, 0.64, 0.05]
    ht, Lt = afqmc.half_rotate(s.h1, s.chol, s.phi_t, 4, 3)
    vb = np.array([afqmc.local_energy_half(ht, Lt, s.phi_t, W0[i], 4, 3)[2] for i in range(nw)])
    fb_cap = 0.5 * float(np.quantile(np.abs(afqmc.force_bias_shift(vb, dt)), 0.9))
    o = afqmc.run(s.h1, s.chol, s.phi_t, 4, 3, W0, w0, fields, dt, qr_every=2, fb_cap=fb_cap, w_cap=1.2,
                  comb_every=3, comb_xi=xi)
    g = api.System.from_synth(s, precision=prec)
    wk = api.Walkers(g, nw, W0, w0)
    wk.set_controls(fb_cap=fb_cap, w_cap=1.2)
    em, wt, srcs = [], [], []
    for c in range(3):
        out = wk.step(3, dt, fields=fields[3 * c:3 * c + 3], qr_every=2, outputs=("emix", "weights"))
        torch.cuda.synchronize()
        em.append(to_np(out["emix"]))
        wt.append(to_np(out["weights"]))
        srcs.append(wk.comb(xi[c])[0])
    em, wt = np.concatenate(em), np.concatenate(wt)
    print(prec, f"emix {rel_vec(em, o['emix']):.1e} weights {rel_vec(wt, o['weights']):.1e}")
    assert rel_vec(em, o["emix"]) < tol
    assert rel_vec(wt[wt > 0], o["weights"][wt > 0]) < tol
    assert np.array_equal(wt == 0, o["weights"] == 0)
    for a, b in zip(srcs, o["comb_src"]):
        assert np.array_equal(a, b)
    assert rel_fro(to_np(wk.get()["W"]), o["W"]) < tol
    # the cap binds: without it the trajectory differs
    o_free = afqmc.run(s.h1, s.chol, s.phi_t, 4, 3, W0, w0, fields[:3], dt, qr_every=2)
    assert rel_vec(o["emix"][1:3], o_free["emix"][1:3]) > 1e-8


def test_eshift_update(api):
    assert api.eshift_update(-3.0, 100.0, 100.0, 0.01, 10) == -3.0
    assert abs(api.eshift_update(-3.0, 100.0 * np.e, 100.0, 0.01, 10) + 13.0) < 1e-12
    from paper_2003_01831_amd._lib import AfqError
    with pytest.raises(AfqError):
        api.eshift_update(-3.0, 0.0, 100.0, 0.01, 10)
