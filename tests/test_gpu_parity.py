"""GPU parity of the HIP walker step against the CPU FP64 oracle, through the
C ABI (torch binding). Tolerances: 1e-10 relative in FP64 mode, 1e-5 in the
reduced-precision modes (complex FP32, split-BF16x3)."""
import numpy as np
import pytest

from oracle import afqmc, philox
from paper_2003_01831_amd import synth
from gpu_util import rel_scalar, rel_vec, rel_fro, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api
    return api


def _energy_case(api, s, W, w, prec, form="auto"):
    sysg = api.System.from_synth(s, precision=prec, exchange_form=form)
    wk = api.Walkers(sysg, W.shape[0], W, w)
    el, parts, vb, em = wk.energy(want_vbar=True)
    torch.cuda.synchronize()
    return to_np(el), to_np(parts), to_np(vb), float(em[0])


def _oracle_energy(s, W, w):
    ht, Lt = afqmc.half_rotate(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn)
    el = np.zeros(W.shape[0], complex)
    parts = np.zeros((W.shape[0], 3), complex)
    vb = np.zeros((W.shape[0], s.n_chol), complex)
    for i in range(W.shape[0]):
        el[i], p, vb[i] = afqmc.local_energy_half(ht, Lt, s.phi_t, W[i], s.n_up, s.n_dn, s.e_core)
        parts[i] = p
    emix = np.sum(w * el.real) / np.sum(w)
    return el, parts, vb, emix


@pytest.mark.parametrize("shape", [(8, 2, 2, 24), (20, 5, 3, 37), (64, 16, 16, 256), (128, 32, 32, 512),
                                   (100, 50, 47, 60), (120, 100, 65, 40)])
def test_energy_fp64(api, shape):
    M, nu, nd, X = shape
    s = synth.make_system(M, nu, nd, X, seed=M + X)
    s.e_core = 0.37
    W = synth.perturbed_walkers(s, 5, 0.2, seed=3)
    w = synth.random_weights(5, seed=4)
    el, parts, vb, em = _energy_case(api, s, W, w, "fp64")
    rel, rparts, rvb, rem = _oracle_energy(s, W, w)
    print(f"shape {shape}: max rel E_L {rel_vec(el, rel):.2e}")
    assert rel_vec(el, rel) < 1e-10
    for c in range(3):
        assert rel_vec(parts[:, c], rparts[:, c]) < 1e-10, c
    assert rel_fro(vb, rvb) < 1e-10
    assert rel_scalar(em, rem) < 1e-10


def test_energy_fp64_many_electrons(api):
    """113..128 electrons per spin (eight 16-wide MFMA blocks in the overlap
    and Theta kernels, a ragged basis tail and electron counts that are not
    multiples of 4): FP64 takes the four-index exchange form here."""
    s = synth.make_system(136, 120, 117, 48, seed=11)
    W = synth.perturbed_walkers(s, 3, 0.2, seed=3)
    w = synth.random_weights(3, seed=4)
    el, parts, vb, em = _energy_case(api, s, W, w, "fp64", "four_index")
    rel, rparts, rvb, rem = _oracle_energy(s, W, w)
    assert rel_vec(el, rel) < 1e-10
    for c in range(3):
        assert rel_vec(parts[:, c], rparts[:, c]) < 1e-10, c
    assert rel_fro(vb, rvb) < 1e-10
    assert rel_scalar(em, rem) < 1e-10


def test_energy_complex_trial(api):
    """A complex trial doubles the contraction length (Re/Im stacked along k)."""
    s = synth.make_system(24, 4, 5, 30, seed=8)
    rng = np.random.default_rng(1)
    U = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 24)))
    s.phi_t = U @ s.phi_t
    W = synth.perturbed_walkers(s, 4, 0.2, seed=5)
    w = np.ones(4)
    for prec, tol in (("fp64", 1e-10), ("cfp32", 1e-5), ("bf16x3", 1e-5)):
        el, parts, vb, em = _energy_case(api, s, W, w, prec)
        rel, rparts, rvb, rem = _oracle_energy(s, W, w)
        assert rel_vec(el, rel) < tol, prec


@pytest.mark.parametrize("prec,form", [("cfp32", "auto"), ("bf16x3", "cholesky"), ("bf16x3", "four_index")])
@pytest.mark.parametrize("shape", [(64, 16, 16, 256), (128, 32, 32, 512), (160, 80, 70, 96), (224, 100, 100, 128),
                                   (240, 100, 97, 40)])
def test_energy_reduced_precision(api, prec, form, shape):
    """Split-BF16x3 in both exchange forms: the Cholesky form (the 65..100
    electron shapes take the one-wave-per-SIMD kernel) and the four-index form."""
    M, nu, nd, X = shape
    s = synth.make_system(M, nu, nd, X, seed=M + X)
    W = synth.perturbed_walkers(s, 6, 0.1, seed=3)
    w = synth.random_weights(6, seed=4)
    el, parts, vb, em = _energy_case(api, s, W, w, prec, form)
    rel, rparts, rvb, rem = _oracle_energy(s, W, w)
    errs = {"E_L": rel_vec(el, rel), "E1": rel_vec(parts[:, 0], rparts[:, 0]),
            "EJ": rel_vec(parts[:, 1], rparts[:, 1]), "EK": rel_vec(parts[:, 2], rparts[:, 2]),
            "vbar": rel_fro(vb, rvb), "E_mix": rel_scalar(em, rem)}
    print(prec, form, shape, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < 1e-5, (k, v)


def _run_both(api, s, W0, w0, fields, dt, qr_every, e_shift, prec="fp64"):
    sysg = api.System.from_synth(s, precision=prec)
    wk = api.Walkers(sysg, W0.shape[0], W0, w0)
    out = wk.step(fields.shape[0], dt, fields=fields, qr_every=qr_every, e_shift=e_shift)
    st = wk.get()
    torch.cuda.synchronize()
    g = {k: to_np(v) for k, v in out.items()}
    g["W"] = to_np(st["W"])
    g["alive"] = to_np(st["alive"])
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, w0, fields, dt, qr_every=qr_every,
                  e_shift=e_shift, e_core=s.e_core)
    return g, o


def test_step_tiny_full_trajectory(api):
    """8 orbitals, 2+2 electrons, 24 Cholesky vectors, 32 walkers at the trial,
    dt 0.01, 50 steps, QR every 5: every per-step output against the oracle."""
    cfg = synth.WORKLOADS["tiny_m8"]
    s = synth.make_system(cfg["M"], cfg["n_up"], cfg["n_dn"], cfg["n_chol"], seed=cfg["seed"])
    nw = cfg["n_walkers"]
    fields = synth.make_fields(cfg["n_steps"], nw, cfg["n_chol"], seed=cfg["field_seed"])
    evar = afqmc.local_energy_plain(s.h1, s.chol, s.phi_t, s.phi_t, 2, 2)[0].real
    g, o = _run_both(api, s, synth.trial_walkers(s, nw), np.ones(nw), fields, cfg["dt"], cfg["qr_every"], evar)
    assert rel_vec(g["emix"], o["emix"]) < 1e-10
    assert rel_vec(g["eloc"], o["eloc"]) < 1e-10
    assert rel_vec(g["weights"], o["weights"]) < 1e-10
    assert rel_vec(g["ratio"], o["ratio"]) < 1e-10
    assert np.array_equal(g["alive"].astype(bool), o["alive"])
    assert rel_fro(g["W"], o["W"]) < 1e-10


def test_step_moderate_subset(api):
    """M=128, 32+32 electrons, X=512, dt 0.005, QR every 5: 8 walkers x 10 steps."""
    cfg = synth.WORKLOADS["m128"]
    s = synth.make_system(cfg["M"], cfg["n_up"], cfg["n_dn"], cfg["n_chol"], seed=cfg["seed"])
    nw, steps = 8, 10
    fields = synth.make_fields(steps, nw, cfg["n_chol"], seed=cfg["field_seed"])
    evar = afqmc.local_energy_plain(s.h1, s.chol, s.phi_t, s.phi_t, 32, 32)[0].real
    g, o = _run_both(api, s, synth.trial_walkers(s, nw), np.ones(nw), fields, cfg["dt"], cfg["qr_every"], evar)
    for k in ("emix", "eloc", "weights", "ratio"):
        print(k, f"{rel_vec(g[k], o[k]):.2e}")
        assert rel_vec(g[k], o[k]) < 1e-10, k
    assert rel_fro(g["W"], o["W"]) < 1e-10


def test_step_many_electrons_qr_every_step(api):
    """120 + 117 electrons (eight 16-wide blocks in the overlap, Theta, Gram
    and Q kernels, odd electron counts, a ragged basis tail at M = 136) with
    CholeskyQR after every step: FP64 (two CholeskyQR passes, four-index
    exchange) against the oracle over 3 steps."""
    s = synth.make_system(136, 120, 117, 48, seed=12)
    nw, steps = 3, 3
    fields = synth.make_fields(steps, nw, 48, seed=1012)
    W0 = synth.perturbed_walkers(s, nw, 0.1, seed=5)
    w0 = np.ones(nw)
    sysg = api.System.from_synth(s, precision="fp64", exchange_form="four_index")
    wk = api.Walkers(sysg, nw, W0, w0)
    out = wk.step(steps, 0.005, fields=fields, qr_every=1, e_shift=0.0)
    st = wk.get()
    torch.cuda.synchronize()
    g = {k: to_np(v) for k, v in out.items()}
    o = afqmc.run(s.h1, s.chol, s.phi_t, s.n_up, s.n_dn, W0, w0, fields, 0.005, qr_every=1, e_shift=0.0,
                  e_core=s.e_core)
    for k in ("emix", "eloc", "weights", "ratio"):
        assert rel_vec(g[k], o[k]) < 1e-10, k
    assert rel_fro(to_np(st["W"]), o["W"]) < 1e-10


@pytest.mark.parametrize("prec", ["cfp32", "bf16x3"])
@pytest.mark.parametrize("shape", [(64, 16, 16, 256), (37, 9, 6, 70)])
def test_step_reduced_precision(api, prec, shape):
    """Reduced-precision contractions against the FP64 oracle over 10 steps.
    M = 37 leaves ragged tails in every packed chunk (2M = 74, M = 37 against
    16- and 32-element chunks) and in the walker-column tiles (n_tot = 15)."""
    M, nu, nd, X = shape
    s = synth.make_system(M, nu, nd, X, seed=3)
    nw, steps = 6, 10
    fields = synth.make_fields(steps, nw, X, seed=1003)
    W0 = synth.perturbed_walkers(s, nw, 0.05, seed=9)
    g, o = _run_both(api, s, W0, np.ones(nw), fields, 0.005, 5, 0.0, prec=prec)
    errs = {k: rel_vec(g[k], o[k]) for k in ("emix", "eloc", "weights", "ratio")}
    print(prec, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v < 1e-5, (k, v)


def test_uneven_spins_and_dead_walkers(api):
    """n_up != n_dn, a huge time step: walkers die and stay frozen, exactly as in the oracle."""
    s = synth.make_system(8, 3, 1, 24, seed=1)
    s.chol = s.chol * 3.0
    nw = 16
    fields = synth.make_fields(4, nw, 24, seed=6)
    g, o = _run_both(api, s, synth.trial_walkers(s, nw), np.ones(nw), fields, 0.3, 1, 0.0)
    assert np.array_equal(g["alive"].astype(bool), o["alive"])
    assert not o["alive"].all() and o["alive"].any()
    assert np.array_equal(g["weights"] == 0, o["weights"] == 0)
    live = o["alive"]
    assert rel_vec(g["weights"][-1][live], o["weights"][-1][live]) < 1e-9
    assert rel_vec(g["emix"], o["emix"]) < 1e-9
    # a dead walker keeps the W of its last committed step; a live one took every step's W'
    assert rel_fro(g["W"][~live], o["W"][~live]) < 1e-8
    assert rel_fro(g["W"][live], o["W"][live]) < 1e-8


def test_dead_walkers_between_qr_steps(api):
    """Walkers that die on steps without QR (the new S^-1 carried to the next
    step): the commit keeps their W, S^-1 and log det, so their local energies
    on the following steps still follow the frozen walkers, as in the oracle."""
    s = synth.make_system(8, 3, 2, 24, seed=2)
    s.chol = s.chol * 2.0
    nw = 16
    fields = synth.make_fields(5, nw, 24, seed=7)
    # dt 0.2: 1, 3, 4, 6 and 7 walkers dead after steps 1..5 (oracle), none QR
    g, o = _run_both(api, s, synth.trial_walkers(s, nw), np.ones(nw), fields, 0.2, 0, 0.0)
    assert np.array_equal(g["alive"].astype(bool), o["alive"])
    assert not o["alive"].all() and o["alive"].any()
    assert rel_vec(g["eloc"], o["eloc"]) < 1e-9   # every walker, every step, dead ones included
    assert rel_vec(g["emix"], o["emix"]) < 1e-9
    live = o["alive"]
    assert rel_fro(g["W"][~live], o["W"][~live]) < 1e-8
    assert rel_fro(g["W"][live], o["W"][live]) < 1e-8


def test_device_philox_matches_cpu(api):
    x = to_np(api.fields_generate(987654321987, 3, 7, 257, step0=11, sys_id=2))
    ref = philox.normal_fields(987654321987, 3, 7, 257, step0=11, sys_id=2)
    assert np.max(np.abs(x - ref)) < 1e-13


def test_philox_fields_drive_the_step(api):
    """fields=None draws from the device Philox stream keyed by the step counter:
    identical to passing the CPU generator's fields explicitly."""
    s = synth.make_system(10, 2, 2, 12, seed=4)
    nw = 5
    sysg = api.System.from_synth(s)
    a = api.Walkers(sysg, nw)
    oa = a.step(6, 0.01, fields=None, seed=77, qr_every=2)
    f = philox.normal_fields(77, 6, nw, 12)
    b = api.Walkers(sysg, nw)
    ob = b.step(6, 0.01, fields=f, seed=0, qr_every=2)
    torch.cuda.synchronize()
    assert rel_vec(to_np(oa["eloc"]), to_np(ob["eloc"])) < 1e-12


def test_checkpoint_resume_is_bitwise(api):
    s = synth.make_system(12, 3, 3, 20, seed=5)
    nw = 6
    sysg = api.System.from_synth(s)
    a = api.Walkers(sysg, nw)
    full = a.step(10, 0.01, seed=5, qr_every=3)
    b = api.Walkers(sysg, nw)
    first = b.step(5, 0.01, seed=5, qr_every=3)
    st = b.get()
    c = api.Walkers(sysg, nw)
    c.set(st["W"], st["weights"], st["alive"], st["counter"])
    second = c.step(5, 0.01, seed=5, qr_every=3)
    torch.cuda.synchronize()
    got = torch.cat([first["eloc"], second["eloc"]])
    assert torch.equal(got, full["eloc"])
    assert torch.equal(c.get()["W"], a.get()["W"])


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_walkers_replaced_between_steps(api, prec):
    """Without QR at the end of a step the next step reuses S^-1 and log det
    from the weight phase. Walkers replaced by set() or resampled by the comb
    must not: the continued run equals fresh walkers started from the same
    state, bit for bit."""
    s = synth.make_system(12, 3, 3, 20, seed=5)
    nw = 6
    sysg = api.System.from_synth(s, precision=prec)
    a = api.Walkers(sysg, nw)
    a.step(4, 0.01, seed=5, qr_every=5)              # step 4 has no QR: the inverse is carried
    W2 = synth.perturbed_walkers(s, nw, 0.1, seed=8)
    a.set(W2, np.ones(nw), np.ones(nw, dtype=np.int32), 4)
    got = a.step(3, 0.01, seed=5, qr_every=5)
    b = api.Walkers(sysg, nw)
    b.set(W2, np.ones(nw), np.ones(nw, dtype=np.int32), 4)
    ref = b.step(3, 0.01, seed=5, qr_every=5)
    torch.cuda.synchronize()
    for k in ("eloc", "weights", "ratio"):
        assert torch.equal(got[k], ref[k]), k
    # the comb copies walkers over others: their carried inverses would be stale
    a.comb(0.37)
    st = a.get()
    c = api.Walkers(sysg, nw)
    c.set(st["W"], st["weights"], st["alive"], st["counter"])
    got = a.step(3, 0.01, seed=5, qr_every=5)
    ref = c.step(3, 0.01, seed=5, qr_every=5)
    torch.cuda.synchronize()
    for k in ("eloc", "weights", "ratio"):
        assert torch.equal(got[k], ref[k]), k


def test_precision_switch_between_steps(api):
    """The FP32 and the split-BF16 propagator kernels pack their operands in
    different layouts with zero padding in different places: walkers continued
    after a precision switch equal fresh walkers started from the same state."""
    s = synth.make_system(37, 9, 6, 70, seed=8)
    nw = 5
    sysg = api.System.from_synth(s, precision="cfp32")
    a = api.Walkers(sysg, nw)
    a.step(3, 0.01, seed=2, qr_every=2)
    for prec in ("bf16x3", "cfp32", "bf16x3"):
        sysg.set_precision(prec)
        st = a.get()
        b = api.Walkers(sysg, nw)
        b.set(st["W"], st["weights"], st["alive"], st["counter"])
        got = a.step(3, 0.01, seed=2, qr_every=2)
        ref = b.step(3, 0.01, seed=2, qr_every=2)
        torch.cuda.synchronize()
        for k in ("eloc", "weights", "ratio"):
            assert torch.equal(got[k], ref[k]), (prec, k)
        b.close()


def test_repeatable_bitwise(api):
    """Fixed-order reductions: two identical runs agree bit for bit."""
    s = synth.make_system(40, 10, 10, 80, seed=6)
    outs = []
    for _ in range(2):
        sysg = api.System.from_synth(s, precision="bf16x3")
        wk = api.Walkers(sysg, 12)
        outs.append(wk.step(4, 0.005, seed=3, qr_every=2))
    torch.cuda.synchronize()
    for k in outs[0]:
        assert torch.equal(outs[0][k], outs[1][k]), k


def test_singular_initial_overlap_is_reported(api):
    from paper_2003_01831_amd._lib import AfqError
    s = synth.make_system(8, 2, 2, 4, seed=2)
    W0 = synth.trial_walkers(s, 3)
    W0[1, :, 0] = 0.0
    sysg = api.System.from_synth(s)
    with pytest.raises(AfqError, match="AFQ_E_SINGULAR"):
        api.Walkers(sysg, 3, W0)
    # a dead (zero-weight) walker may be singular
    api.Walkers(sysg, 3, W0, np.array([1.0, 0.0, 1.0]))


def test_asymmetric_input_is_rejected(api):
    from paper_2003_01831_amd._lib import AfqError
    s = synth.make_system(8, 2, 2, 4, seed=2)
    s.h1[0, 1] += 1e-3
    with pytest.raises(AfqError, match="AFQ_E_INVALID"):
        api.System.from_synth(s)
