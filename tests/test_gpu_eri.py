"""The four-index exchange form (split-BF16x3 and FP64 modes, real trial)
against the FP64 oracle and against the Cholesky form: sum_n tr(Omega_n Omega_n) as the
quadratic form of the half-rotated two-electron tensor, contracted over its
upper block triangle. Shapes cover one and several 256-row blocks with ragged
tails, work units of a single chunk and several runs per row block, walker
counts that leave padding columns, shared and distinct spin tensors."""
import numpy as np
import pytest

from oracle import afqmc
from paper_2003_01831_amd import synth
from gpu_util import rel_fro, rel_scalar, rel_vec, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api
    return api


def _oracle_energy(s, W, w):
    ht, Lt = afqmc.half_rotate(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn)
    el = np.zeros(W.shape[0], complex)
    parts = np.zeros((W.shape[0], 3), complex)
    vb = np.zeros((W.shape[0], s.n_chol), complex)
    for i in range(W.shape[0]):
        el[i], parts[i], vb[i] = afqmc.local_energy_half(ht, Lt, s.phi_t, W[i], s.n_up, s.n_dn, s.e_core)
    return el, parts, vb, np.sum(w * el.real) / np.sum(w)


def _rotate_down_block(s, seed):
    """Same spin counts, different trial blocks (the spins get distinct tensors)."""
    rng = np.random.default_rng(seed)
    n = s.n_dn
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s.phi_t = s.phi_t.copy()
    s.phi_t[:, s.n_up:] = s.phi_t[:, s.n_up:] @ Q
    return s


# (M, n_up, n_dn, X, walkers, distinct spin blocks):
#   NM = 280: two row blocks, the second a unit of one chunk;
#   NM = 1280 / 1088: five row blocks, several runs each, 70 walkers (two
#   column blocks, the second mostly padding);
#   NM = 450 / 350: ragged everywhere; equal spin counts with distinct blocks
CASES = [(20, 14, 14, 50, 5, False), (64, 20, 17, 100, 70, False), (50, 9, 9, 120, 7, True),
         (30, 5, 3, 40, 3, False)]


TOL = {"bf16x3": 1e-5, "fp64": 1e-10}


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
@pytest.mark.parametrize("case", CASES)
def test_four_index_energy_matches_the_oracle(api, case, prec):
    M, nu, nd, X, nw, distinct = case
    s = synth.make_system(M, nu, nd, X, seed=M + X + 7)
    s.e_core = 0.21
    if distinct:
        s = _rotate_down_block(s, seed=M)
    W = synth.perturbed_walkers(s, nw, 0.15, seed=11)
    w = synth.random_weights(nw, seed=12)
    sysg = api.System.from_synth(s, precision=prec, exchange_form="four_index")
    form, nbytes = sysg.exchange_form()
    assert form == "four_index" and nbytes > 0
    wk = api.Walkers(sysg, nw, W, w)
    el, parts, vb, em = (to_np(t) for t in wk.energy(want_vbar=True))
    rel, rparts, rvb, rem = _oracle_energy(s, W, w)
    errs = {"E_L": rel_vec(el, rel), "E1": rel_vec(parts[:, 0], rparts[:, 0]),
            "EJ": rel_vec(parts[:, 1], rparts[:, 1]), "EK": rel_vec(parts[:, 2], rparts[:, 2]),
            "vbar": rel_fro(vb, rvb), "E_mix": rel_scalar(float(em[0]), rem)}
    print(prec, case, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < TOL[prec], (k, v)
    # the Cholesky form of the same mode gives the same exchange energy
    chol = api.System.from_synth(s, precision=prec, exchange_form="cholesky")
    assert chol.exchange_form() == ("cholesky", 0)
    parts_c = to_np(api.Walkers(chol, nw, W, w).energy()[1])
    assert rel_vec(parts[:, 2], parts_c[:, 2]) < TOL[prec]


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_four_index_walk_matches_the_oracle(api, prec):
    """Ten steps with QR every 5 through the four-index exchange (N M = 1024)."""
    s = synth.make_system(64, 16, 16, 256, seed=3)
    nw, steps, dt = 6, 10, 0.005
    fields = synth.make_fields(steps, nw, 256, seed=1003)
    W0 = synth.perturbed_walkers(s, nw, 0.05, seed=9)
    sysg = api.System.from_synth(s, precision=prec, exchange_form="four_index")
    wk = api.Walkers(sysg, nw, W0, np.ones(nw))
    out = wk.step(steps, dt, fields=fields, qr_every=5)
    torch.cuda.synchronize()
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, np.ones(nw), fields, dt, qr_every=5)
    for k in ("emix", "eloc", "weights", "ratio"):
        err = rel_vec(to_np(out[k]), o[k])
        print(prec, k, f"{err:.2e}")
        assert err < TOL[prec], k


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_four_index_is_repeatable_bitwise(api, prec):
    """Fixed-order partial sums: two identical runs agree bit for bit."""
    s = synth.make_system(48, 12, 11, 60, seed=21)
    outs = []
    for _ in range(2):
        sysg = api.System.from_synth(s, precision=prec, exchange_form="four_index")
        wk = api.Walkers(sysg, 9)
        outs.append(wk.step(3, 0.005, seed=4, qr_every=2))
    torch.cuda.synchronize()
    for k in outs[0]:
        assert torch.equal(outs[0][k], outs[1][k]), k


def test_exchange_form_selection(api):
    s = synth.make_system(24, 4, 4, 30, seed=31)
    g = api.System.from_synth(s, precision="bf16x3")
    assert g.exchange_form() == ("cholesky", 0)          # auto: N M = 96 is below the size floor
    g.set_exchange_form("four_index")
    # split BF16: hi and lo planes of the upper block triangle, N M = 96 in three
    # 32-column chunks that each keep one 256-row block of 64-byte rows
    assert g.exchange_form() == ("four_index", 2 * 3 * 256 * 64)
    g.set_precision("cfp32")                              # not in complex FP32 mode
    assert g.exchange_form() == ("cholesky", 0)
    g.set_precision("fp64")   # FP64 keeps W' in three 32-column blocks, each down to its diagonal block
    assert g.exchange_form() == ("four_index", (32 + 64 + 96) * 32 * 8)
    g.set_precision("bf16x3")
    assert g.exchange_form()[0] == "four_index"
    g.set_exchange_form("cholesky")
    assert g.exchange_form() == ("cholesky", 0)
    with pytest.raises(KeyError):
        g.set_exchange_form("dense")
    assert g.lib.afq_system_set_exchange_form(g.handle, 7) == -1     # AFQ_E_INVALID
    # a complex trial keeps the Cholesky form
    rng = np.random.default_rng(1)
    sc = synth.make_system(24, 4, 4, 30, seed=31)
    sc.phi_t = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 24))) @ sc.phi_t
    gc = api.System.from_synth(sc, precision="bf16x3", exchange_form="four_index")
    assert gc.exchange_form() == ("cholesky", 0)


def test_batch_captures_again_after_a_form_switch(api):
    """A captured batch replays the kernel sequence of its capture: switching a
    member's exchange form must make the next call capture again."""
    dt, seed, qr = 0.01, 41, 2
    s0 = synth.make_system(32, 8, 8, 48, seed=42)
    s1 = synth.make_system(28, 9, 6, 40, seed=43)
    g = [api.System.from_synth(x, precision="bf16x3", exchange_form="four_index") for x in (s0, s1)]
    w = [api.Walkers(g[0], 6), api.Walkers(g[1], 5)]
    b = api.Batch(list(zip(g, w)))
    b.step(4, dt, seed=seed, qr_every=qr)
    g[0].set_exchange_form("cholesky")
    got = b.step(4, dt, seed=seed, qr_every=qr)
    torch.cuda.synchronize()
    # eager reference: the same walkers, the first 4 steps in the four-index
    # form, the next 4 in the form each member had then
    r = [api.System.from_synth(x, precision="bf16x3", exchange_form="four_index") for x in (s0, s1)]
    rw = [api.Walkers(r[0], 6), api.Walkers(r[1], 5)]
    for i in range(2):
        f = api.fields_generate(seed, 4, rw[i].nw, r[i].n_chol, step0=0, sys_id=i)
        rw[i].step(4, dt, fields=f, qr_every=qr)
    r[0].set_exchange_form("cholesky")
    for i in range(2):
        f = api.fields_generate(seed, 4, rw[i].nw, r[i].n_chol, step0=4, sys_id=i)
        ref = rw[i].step(4, dt, fields=f, qr_every=qr, outputs=("emix",))["emix"]
        torch.cuda.synchronize()
        assert rel_vec(to_np(got[i]), to_np(ref)) < 1e-12, i
        assert rel_fro(to_np(w[i].get()["W"]), to_np(rw[i].get()["W"])) < 1e-12, i
    b.close()
