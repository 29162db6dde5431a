"""The widened paths together: back-propagation on a k-point-blocked system,
and one captured batch that mixes a plain system, a multi-determinant trial
and a k-point-blocked system."""
import numpy as np
import pytest

from oracle import afqmc, kpoint
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


def _kp_case(seed):
    ks = synth.make_kpoint_system(4, 5, 2, 1, 6, seed=seed)
    ks.Lk = ks.Lk * 3.0
    h = kpoint.dense_one_body(ks.hk)
    L = kpoint.dense_factors(ks.Lk, ks.kq)
    T = kpoint.dense_trial(ks.phik, ks.n_up, ks.n_dn)
    return ks, h, L, T


def test_kpoint_back_propagation_matches_the_oracle(api):
    """Two steps, then a window of four (walk QR every 2, bra QR every 2); the
    bra walks back through the Hermitian parts a_g, b_g with the recorded
    coefficients."""
    ks, h, L, T = _kp_case(501)
    Nu, Nd = ks.nk * ks.n_up, ks.nk * ks.n_dn
    nw, dt = 5, 0.02
    rng = np.random.default_rng(502)
    W0 = T[None] + 0.1 * (rng.standard_normal((nw,) + T.shape) + 1j * rng.standard_normal((nw,) + T.shape))
    w0 = synth.random_weights(nw, seed=503)
    fields = rng.standard_normal((6, nw, 2 * L.shape[0]))
    o = kpoint.run(h, L, T, Nu, Nd, W0, w0, fields, dt, qr_every=2, bp_start=2, bp_len=4)
    ref = afqmc.back_propagated_rdm1(o["B1"], o["ops"], T, Nu, Nd, o["bp_W0"], o["bp_coefs"], o["bp_weights"],
                                     order=6, qr_every=2)
    g = api.System.from_kpoint(ks)
    wk = api.Walkers(g, nw, W0, w0)
    wk.step(2, dt, fields=fields[:2], qr_every=2)
    wk.bp_begin(4)
    wk.step(4, dt, fields=fields[2:], qr_every=2)
    P, _ = wk.bp_rdm1(qr_every=2)
    err = rel_fro(to_np(P), ref)
    print(f"k-point bp rdm1 rel err {err:.2e}")
    assert err < 1e-10


def test_batch_mixes_plain_multideterminant_and_kpoint_systems(api):
    dt, seed, qr, steps = 0.01, 17, 3, 8
    builds = []
    for _ in range(2):
        s0 = synth.make_system(12, 3, 3, 24, seed=511)
        g0 = api.System.from_synth(s0)
        s1 = synth.make_system(14, 4, 3, 20, seed=512)
        C, exc, coeffs = synth.make_msd(s1, 20, 3, 4, 3, seed=513)
        g1 = api.System.from_synth(s1)
        g1.set_msd(C, exc, coeffs)
        ks, _, _, _ = _kp_case(514)
        g2 = api.System.from_kpoint(ks)
        sysg = [g0, g1, g2]
        wk = [api.Walkers(g0, 6, synth.perturbed_walkers(s0, 6, 0.05, seed=515)),
              api.Walkers(g1, 5, synth.perturbed_walkers(s1, 5, 0.05, seed=516)),
              api.Walkers(g2, 4)]
        builds.append((sysg, wk))
    (sa, wa), (sb, wb) = builds
    b = api.Batch(list(zip(sa, wa)))
    got = b.step(steps, dt, seed=seed, qr_every=qr, e_shift=[0.0, 0.1, 0.2])
    torch.cuda.synchronize()
    for i in range(3):
        f = api.fields_generate(seed, steps, wb[i].nw, sb[i].n_chol, step0=0, sys_id=i)
        ref = wb[i].step(steps, dt, fields=f, qr_every=qr, e_shift=[0.0, 0.1, 0.2][i], outputs=("emix",))["emix"]
        torch.cuda.synchronize()
        err = rel_vec(to_np(got[i]), to_np(ref))
        print(f"batch member {i}: emix rel {err:.1e}")
        assert err < 1e-12, i
        assert rel_fro(to_np(wa[i].get()["W"]), to_np(wb[i].get()["W"])) < 1e-12
    b.close()
