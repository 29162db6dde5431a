"""Many uneven systems stepped as branches of one captured HIP graph
(afq_batch_*): against the same systems stepped one by one, and against the
CPU FP64 oracle."""
import numpy as np
import pytest

from oracle import afqmc, philox
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


def _shapes(n, m_hi, nw_hi, seed):
    return synth.uneven_systems(n, seed=seed, m_lo=8, m_hi=m_hi, nw_lo=3, nw_hi=nw_hi)


def _build(api, shapes, prec="fp64", perturb=0.05):
    systems, walkers, synths = [], [], []
    for c in shapes:
        s = synth.make_system(c["M"], c["n_up"], c["n_dn"], c["n_chol"], seed=c["seed"])
        g = api.System.from_synth(s, precision=prec)
        W0 = synth.perturbed_walkers(s, c["n_walkers"], perturb, seed=c["seed"] + 7)
        w0 = synth.random_weights(c["n_walkers"], seed=c["seed"] + 8)
        systems.append(g)
        walkers.append(api.Walkers(g, c["n_walkers"], W0, w0))
        synths.append((s, W0, w0))
    return systems, walkers, synths


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batch_equals_individual_steps(api, prec):
    """Two calls (13 then 7 steps, QR every 5): eager warm-up, graph capture,
    replays and eager tails; each system equals afq_step driven by the device
    fields of its sys_id."""
    shapes = _shapes(4, 48, 9, seed=4100)
    dt, seed, qr = 0.01, 31, 5
    es = [0.1 * i for i in range(len(shapes))]
    sysA, wkA, _ = _build(api, shapes, prec)
    sysB, wkB, _ = _build(api, shapes, prec)
    b = api.Batch(list(zip(sysA, wkA)))
    e1 = b.step(13, dt, seed=seed, qr_every=qr, e_shift=es)
    e2 = b.step(7, dt, seed=seed, qr_every=qr, e_shift=es)
    torch.cuda.synchronize()
    got = torch.cat([e1, e2], dim=1)
    for i, c in enumerate(shapes):
        f = api.fields_generate(seed, 20, c["n_walkers"], c["n_chol"], step0=0, sys_id=i)
        ref = wkB[i].step(20, dt, fields=f, qr_every=qr, e_shift=es[i], outputs=("emix",))["emix"]
        torch.cuda.synchronize()
        err = rel_vec(to_np(got[i]), to_np(ref))
        print(f"system {i} M={c['M']} nw={c['n_walkers']}: emix rel {err:.1e}")
        assert err < 1e-12, i
        ga, gb = wkA[i].get(), wkB[i].get()
        assert ga["counter"] == gb["counter"] == 20
        assert rel_fro(to_np(ga["W"]), to_np(gb["W"])) < 1e-12
        assert rel_vec(to_np(ga["weights"]), to_np(gb["weights"])) < 1e-12
        assert torch.equal(ga["alive"], gb["alive"])
    b.close()


def test_batch_system0_bitwise_and_replays_repeat(api):
    """System 0 (sys_id 0) equals afq_step with fields=None bit for bit, and a
    second batch over fresh walkers reproduces the first bit for bit."""
    shapes = _shapes(3, 40, 8, seed=4200)
    runs = []
    for _ in range(2):
        sysg, wk, _ = _build(api, shapes)
        b = api.Batch(list(zip(sysg, wk)))
        e = torch.cat([b.step(9, 0.01, seed=5, qr_every=3), b.step(6, 0.01, seed=5, qr_every=3)], dim=1)
        torch.cuda.synchronize()
        runs.append((e, [w.get()["W"] for w in wk]))
        b.close()
    assert torch.equal(runs[0][0], runs[1][0])
    for a, c in zip(runs[0][1], runs[1][1]):
        assert torch.equal(a, c)
    sysg, wk, _ = _build(api, shapes[:1])
    ref = wk[0].step(15, 0.01, seed=5, qr_every=3, outputs=("emix",))["emix"]
    torch.cuda.synchronize()
    assert torch.equal(runs[0][0][0], ref)


def test_batch_parameter_change_recaptures(api):
    """Changing dt between calls rebuilds the graph; the result equals stepping
    each system with the same dt sequence."""
    shapes = _shapes(2, 32, 6, seed=4300)
    sysA, wkA, _ = _build(api, shapes)
    sysB, wkB, _ = _build(api, shapes)
    b = api.Batch(list(zip(sysA, wkA)))
    ea = b.step(4, 0.01, seed=9, qr_every=2)
    eb = b.step(4, 0.02, seed=9, qr_every=2)
    torch.cuda.synchronize()
    for i, c in enumerate(shapes):
        f = api.fields_generate(9, 8, c["n_walkers"], c["n_chol"], sys_id=i)
        ra = wkB[i].step(4, 0.01, fields=f[:4], qr_every=2, outputs=("emix",))["emix"]
        rb = wkB[i].step(4, 0.02, fields=f[4:], qr_every=2, outputs=("emix",))["emix"]
        torch.cuda.synchronize()
        assert rel_vec(to_np(ea[i]), to_np(ra)) < 1e-12
        assert rel_vec(to_np(eb[i]), to_np(rb)) < 1e-12
    b.close()


def test_batch_grouped_overlaps_mixed_shapes(api):
    """Grouped overlap and Theta launches over systems of different electron
    block counts (1 and 2 sixteen-wide blocks), wave counts (M = 72: 4 waves;
    M = 128: 8 waves) and trial kinds (one complex trial): the batch equals
    the same systems stepped one by one, QR every 3."""
    cfg = [dict(M=72, n_up=18, n_dn=17, n_chol=40, n_walkers=5, seed=4601, cplx=False),
           dict(M=128, n_up=32, n_dn=32, n_chol=48, n_walkers=4, seed=4602, cplx=False),
           dict(M=40, n_up=10, n_dn=9, n_chol=36, n_walkers=6, seed=4603, cplx=True)]
    dt, seed, qr = 0.01, 17, 3

    def build():
        systems, walkers = [], []
        for c in cfg:
            s = synth.make_system(c["M"], c["n_up"], c["n_dn"], c["n_chol"], seed=c["seed"])
            if c["cplx"]:
                rng = np.random.default_rng(c["seed"])
                s.phi_t = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, c["M"]))) @ s.phi_t
            g = api.System.from_synth(s, precision="fp64")
            W0 = synth.perturbed_walkers(s, c["n_walkers"], 0.05, seed=c["seed"] + 7)
            systems.append(g)
            walkers.append(api.Walkers(g, c["n_walkers"], W0, np.ones(c["n_walkers"])))
        return systems, walkers

    sysA, wkA = build()
    sysB, wkB = build()
    b = api.Batch(list(zip(sysA, wkA)))
    got = b.step(7, dt, seed=seed, qr_every=qr)
    torch.cuda.synchronize()
    for i, c in enumerate(cfg):
        f = api.fields_generate(seed, 7, c["n_walkers"], c["n_chol"], step0=0, sys_id=i)
        ref = wkB[i].step(7, dt, fields=f, qr_every=qr, outputs=("emix",))["emix"]
        torch.cuda.synchronize()
        assert rel_vec(to_np(got[i]), to_np(ref)) < 1e-12, i
        assert rel_fro(to_np(wkA[i].get()["W"]), to_np(wkB[i].get()["W"])) < 1e-12, i
    b.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 1e-5)])
def test_batch_uneven_systems_vs_oracle(api, prec, tol):
    """Five uneven systems (M in [8, 64], N = M/4 per spin, X = 4M), 8 steps,
    QR every 4: every system's E_mix trajectory and final weights against the
    oracle run on the CPU Philox fields of its sys_id."""
    shapes = _shapes(5, 64, 10, seed=4400)
    dt, seed, qr = 0.005, 123, 4
    sysg, wk, syn = _build(api, shapes, prec)
    b = api.Batch(list(zip(sysg, wk)))
    em = to_np(b.step(8, dt, seed=seed, qr_every=qr))
    for i, (c, (s, W0, w0)) in enumerate(zip(shapes, syn)):
        f = philox.normal_fields(seed, 8, c["n_walkers"], c["n_chol"], sys_id=i)
        o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, w0, f, dt, qr_every=qr, e_core=s.e_core)
        g = wk[i].get()
        err = rel_vec(em[i], o["emix"])
        print(f"system {i} M={c['M']} nw={c['n_walkers']} {prec}: emix rel {err:.1e}")
        assert err < tol, i
        assert rel_vec(to_np(g["weights"]), o["w"]) < tol, i
    b.close()


def test_batch_rejects_mismatched_precision(api):
    shapes = _shapes(2, 24, 4, seed=4500)
    sysg, wk, _ = _build(api, shapes)
    sysg[1].set_precision("cfp32")
    from paper_2003_01831_amd._lib import AfqError
    with pytest.raises(AfqError):
        api.Batch(list(zip(sysg, wk)))
