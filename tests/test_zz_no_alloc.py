"""afq_walkers_comb_noalloc (the allocation-free comb) against afq_walkers_comb,
through the C ABI: identical source indices, total weight, walkers, weights and
alive flags, on two calls in a row with the second on a smaller walker set
(the static scratch keeps the first call's larger contents), and its error
cases (too many walkers, an open back-propagation window, xi out of range)."""
import ctypes as C

import numpy as np
import pytest

from paper_2003_01831_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_01831_amd import api, _lib
    return api, _lib, _lib.load()


def _comb(lib, fn, wk, xi):
    src = np.full(wk.nw, -7, dtype=np.int32)
    tot = C.c_double()
    rc = getattr(lib, fn)(wk.handle, float(xi), src.ctypes.data_as(C.c_void_p), C.byref(tot))
    return rc, src, tot.value


def _pair(api, s, sysg, nw, seed, dead=()):
    W0 = synth.perturbed_walkers(s, nw, 0.2, seed=seed)
    w0 = np.random.default_rng(seed + 1).uniform(0.2, 2.0, nw)
    w0[list(dead)] = 0.0
    return api.Walkers(sysg, nw, W0, w0), api.Walkers(sysg, nw, W0, w0)


def test_noalloc_comb_equals_comb_on_two_calls(env):
    api, _lib, lib = env
    s = synth.make_system(24, 4, 3, 30, seed=61)
    sysg = api.System.from_synth(s)
    for nw, seed, xi in ((512, 62, 0.37), (100, 63, 0.81)):     # second call: fewer walkers
        ref, got = _pair(api, s, sysg, nw, seed, dead=(3, nw - 1))
        for rep in range(2):                                      # and twice on the same sets
            x = (xi + 0.29 * rep) % 1.0
            rc_a, src_a, tot_a = _comb(lib, "afq_walkers_comb", ref, x)
            rc_b, src_b, tot_b = _comb(lib, "afq_walkers_comb_noalloc", got, x)
            assert rc_a == 0 and rc_b == 0, _lib.load().afq_last_error()
            assert np.array_equal(src_a, src_b)
            assert tot_a == tot_b
            ga, gb = ref.get(), got.get()
            torch.cuda.synchronize()
            assert torch.equal(ga["W"], gb["W"])
            assert torch.equal(ga["weights"], gb["weights"])
            assert torch.equal(ga["alive"], gb["alive"])
            if rep == 0:
                assert 3 not in src_b and nw - 1 not in src_b     # dead walkers get no copies


def test_noalloc_comb_errors(env):
    api, _lib, lib = env
    s = synth.make_system(2, 1, 1, 1, seed=64)
    sysg = api.System.from_synth(s)
    big = api.Walkers(sysg, 4097)
    rc, _, _ = _comb(lib, "afq_walkers_comb_noalloc", big, 0.5)
    assert rc == -1 and b"scratch limit" in lib.afq_last_error()
    big.close()
    wk = api.Walkers(sysg, 8)
    assert _comb(lib, "afq_walkers_comb_noalloc", wk, 1.0)[0] == -1
    wk.bp_begin(2)
    assert _comb(lib, "afq_walkers_comb_noalloc", wk, 0.5)[0] == -6
    wk.bp_end()
    assert _comb(lib, "afq_walkers_comb_noalloc", wk, 0.5)[0] == 0
    wk.set(weights=np.zeros(8))
    assert _comb(lib, "afq_walkers_comb_noalloc", wk, 0.5)[0] == -5
