"""k-point-blocked Cholesky on the GPU against the oracle's general complex
Cholesky walk over the dense block vectors: local energy and both force-bias
sets, a multi-step walk with explicit fields, and the set-up checks."""
import numpy as np
import pytest

from oracle import kpoint
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


def _dense(ks):
    h = kpoint.dense_one_body(ks.hk)
    L = kpoint.dense_factors(ks.Lk, ks.kq)
    T = kpoint.dense_trial(ks.phik, ks.n_up, ks.n_dn)
    return h, L, T


def _walkers(T, nw, scale, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((nw,) + T.shape) + 1j * rng.standard_normal((nw,) + T.shape)
    return T[None] + scale * z / np.sqrt(2.0)


def _pin_valu(wk):
    """Pins the FP64 VALU trace kernel (variant 1) instead of the MFMA one."""
    wk.set_exchange_variant(0, 1)
    wk.set_exchange_variant(1, 1)


# (4, 5, 4, 5) and (5, 4, 3, 4): the spin with fewer electrons per k-point runs
# more vectors per pass and needs the larger LDS layout of the VALU trace
# kernel; (8, 4, 1, 1, 5): eight row blocks per MFMA workgroup (G ns = 8);
# (3, 5, 1, 2, 6): three (k-point counts without a power of two); (2, 68, 1, 1,
# 3): m > 32, which only the VALU kernel takes (both parametrisations run it)
@pytest.mark.parametrize("kernel", ["mfma", "valu"])
@pytest.mark.parametrize("nk,m,nu,nd,xq", [(4, 6, 2, 1, 8), (3, 5, 1, 2, 6), (8, 4, 1, 1, 5), (4, 5, 4, 5, 8),
                                          (5, 4, 3, 4, 3), (2, 68, 1, 1, 3)])
def test_kpoint_energy_and_force_bias_match_the_oracle(api, nk, m, nu, nd, xq, kernel):
    ks = synth.make_kpoint_system(nk, m, nu, nd, xq, seed=400 + nk)
    ks.Lk = ks.Lk * 3.0
    ks.e_core = 0.25
    h, L, T = _dense(ks)
    Nu, Nd = nk * nu, nk * nd
    nw = 6
    W = _walkers(T, nw, 0.2, seed=401)
    g = api.System.from_kpoint(ks)
    wk = api.Walkers(g, nw, W)
    if kernel == "valu":
        _pin_valu(wk)
    el, parts, vb, _ = wk.energy(want_vbar=True)
    el, parts, vb = to_np(el), to_np(parts), to_np(vb)
    for i in range(nw):
        e, e1, ej, ek = kpoint.local_energy(h, L, T, W[i], Nu, Nd, e_core=0.25)
        assert abs(el[i] - e) < 1e-10 * abs(e)
        assert abs(parts[i, 0] - e1) < 1e-10 * abs(e)
        assert abs(parts[i, 1] - ej) < 1e-10 * abs(e) and abs(parts[i, 2] - ek) < 1e-10 * abs(e)
        assert rel_fro(vb[i], kpoint.force_bias(L, T, W[i], Nu, Nd)) < 1e-10


def test_kpoint_walk_matches_the_oracle(api):
    ks = synth.make_kpoint_system(4, 5, 2, 1, 6, seed=410)
    ks.Lk = ks.Lk * 3.0
    h, L, T = _dense(ks)
    Nu, Nd = 4 * 2, 4 * 1
    nw, steps, dt = 6, 5, 0.02
    W0 = _walkers(T, nw, 0.1, seed=411)
    w0 = synth.random_weights(nw, seed=412)
    fields = np.random.default_rng(413).standard_normal((steps, nw, 2 * L.shape[0]))
    o = kpoint.run(h, L, T, Nu, Nd, W0, w0, fields, dt, qr_every=2)
    g = api.System.from_kpoint(ks)
    wk = api.Walkers(g, nw, W0, w0)
    out = wk.step(steps, dt, fields=fields, qr_every=2, outputs=("emix", "eloc", "weights", "ratio"))
    torch.cuda.synchronize()
    for k in ("eloc", "weights", "ratio"):
        err = rel_vec(to_np(out[k]), o[k])
        print("kpoint walk", k, f"{err:.2e}")
        assert err < 1e-10, k
    assert rel_vec(to_np(out["emix"]), o["emix"]) < 1e-10


def test_kpoint_trace_kernels_agree_and_repeat(api):
    """The MFMA and VALU trace kernels sum in different orders: their energies
    agree to rounding, and each is bitwise repeatable."""
    ks = synth.make_kpoint_system(4, 8, 3, 2, 10, seed=430)
    ks.Lk = ks.Lk * 3.0
    _, _, T = _dense(ks)
    W = _walkers(T, 7, 0.2, seed=431)
    g = api.System.from_kpoint(ks)
    res = {}
    for kernel in ("mfma", "valu"):
        wk = api.Walkers(g, 7, W)
        if kernel == "valu":
            _pin_valu(wk)
        a = to_np(wk.energy()[1])
        b = to_np(wk.energy()[1])
        assert np.array_equal(a, b), kernel
        res[kernel] = a
    assert np.max(np.abs(res["mfma"] - res["valu"])) < 1e-12 * np.max(np.abs(res["valu"]))


def test_kpoint_setup_errors(api):
    from paper_2003_01831_amd._lib import AfqError
    ks = synth.make_kpoint_system(4, 3, 1, 1, 3, seed=420)
    bad = synth.make_kpoint_system(4, 3, 1, 1, 3, seed=420)
    bad.kq = bad.kq.copy()
    bad.kq[1, 2], bad.kq[1, 3] = bad.kq[1, 3], bad.kq[1, 2]      # not a group law
    with pytest.raises(AfqError):
        api.System.from_kpoint(bad)
    with pytest.raises(AfqError):                                # FP64 only
        api.System.from_kpoint(ks, precision="bf16x3")
    g = api.System.from_kpoint(ks)
    with pytest.raises(AfqError):
        g.set_precision("cfp32")
    wk = api.Walkers(g, 2)
    from paper_2003_01831_amd.api import energy_backward
    with pytest.raises(AfqError):
        energy_backward(g, wk)
