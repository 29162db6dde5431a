"""CPU FP64 oracle for the phaseless-AFQMC walker step (Cholesky form).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module. The GPU library never
calls it and shares no code with it.

Everything here is plain numpy in complex128/float64, written to be checked by
eye against the definitions:

* Hamiltonian: H = sum_ij h_ij c+_i c_j + 1/2 sum_ijkl v_ijkl c+_i c+_j c_l c_k
  + E_II (the paper's Eq. "hamil", Section "Auxiliary Field Quantum Monte
  Carlo").
* Modified-Cholesky factorisation v_ijkl = sum_n L^n_ik L^n*_lj (same section);
  for the real symmetric L^n used here this is sum_n L^n_ik L^n_jl.
* The phaseless random walk and the Hubbard-Stratonovich transformation are
  only cited by the paper (its references to Zhang & Krakauer's phaseless
  method and Motta & Zhang's review). The steps below are the standard ones,
  derived from the two statements above with Wick's theorem and a Gaussian
  integral:

  - mixed Green's function G^s = W^s (T^sH W^s)^-1 T^sH with <c+_i c_k> = G_ki;
  - local energy E_L = E_II + sum_s tr(h G^s)
        + 1/2 sum_n [ (sum_s tr(L^n G^s))^2 - sum_s tr(L^n G^s L^n G^s) ];
  - one-body correction from normal ordering: h' = h - 1/2 sum_n L^n L^n;
  - HS: exp(-dt v^2/2) = E_x[exp(i sqrt(dt) x v)], shifted by the force bias
    xbar_n = -i sqrt(dt) vbar_n, vbar_n = sum_s tr(L^n G^s);
  - walker update W <- B1 T_K(A) B1 W with B1 = exp(-dt h'/2),
    A = i sqrt(dt) sum_n (x_n - xbar_n) L^n and T_K the order-K Taylor series;
  - importance function I = (O'/O) exp(sum_n x_n xbar_n - xbar_n^2/2) exp(dt E_shift),
    phaseless weight w <- w |I| max(0, cos(arg(O'/O)));
  - periodic thin QR with a positive diagonal R, O <- O / prod_s det R^s;
  - optional mean-field background subtraction (cited with the phaseless
    method, not described in the paper): for any real vector c (normally the
    trial's mean field c_n = sum_s tr(L^n G_T^s)) the two-body term is
    1/2 sum_n (v_n - c_n)^2 + sum_n c_n v_n - 1/2 sum_n c_n^2, so the one-body
    factor uses h' + sum_n c_n L^n, the force bias is taken for v_n - c_n, the
    c-number part of exp(i sqrt(dt) (x - xbar)(v - c)) multiplies the
    overlap ratio (and so enters the phaseless angle), and the constant
    exp(dt/2 sum_n c_n^2) multiplies every weight.

Walkers are stored as W[w] with shape (M, n_up + n_dn): up columns first.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Small helpers
# ---------------------------------------------------------------------------
def spin_blocks(n_up, n_dn):
    return [slice(0, n_up), slice(n_up, n_up + n_dn)]


def two_body_tensor(chol):
    """v_ijkl = sum_n L^n_ik L^n_jl (real symmetric L^n)."""
    return np.einsum("nik,njl->ijkl", chol, chol)


def one_body_corrected(h1, chol):
    """h' = h - 1/2 sum_n L^n L^n (normal-ordering correction of the two-body term)."""
    return h1 - 0.5 * np.tensordot(chol, chol, axes=([0, 2], [0, 1]))


def sym_expm(a):
    """exp(a) for a real symmetric matrix through its eigendecomposition."""
    lam, v = np.linalg.eigh(a)
    return (v * np.exp(lam)) @ v.T


def taylor_apply(A, V, order):
    """sum_{j=0}^{order} A^j V / j!  (the order-K Taylor propagator applied to V)."""
    term = V.copy()
    out = V.copy()
    for j in range(1, order + 1):
        term = (A @ term) / j
        out = out + term
    return out


def qr_positive(W):
    """Thin QR with a positive real diagonal in R (unique for full column rank)."""
    Q, R = np.linalg.qr(W)
    d = np.diag(R)
    ph = d / np.abs(d)
    Q = Q * ph[None, :]
    R = R / ph[:, None]
    return Q, R


# ---------------------------------------------------------------------------
# Green's function, overlap, force bias, local energy (plain form)
# ---------------------------------------------------------------------------
def overlap(T, W, n_up, n_dn):
    """O = prod_s det(T^sH W^s) and the per-spin S^s."""
    S = [T[:, b].conj().T @ W[:, b] for b in spin_blocks(n_up, n_dn)]
    return np.prod([np.linalg.det(s) for s in S]), S


def greens_function(T, W, n_up, n_dn):
    """Per-spin mixed Green's function G^s = W^s (T^sH W^s)^-1 T^sH (M x M)."""
    out = []
    for b in spin_blocks(n_up, n_dn):
        Ts, Ws = T[:, b], W[:, b]
        S = Ts.conj().T @ Ws
        out.append(Ws @ np.linalg.solve(S, Ts.conj().T))
    return out


def force_bias_plain(chol, G):
    """vbar_n = sum_s tr(L^n G^s) = sum_s sum_ik L^n_ik G^s_ki."""
    return sum(np.tensordot(chol, g.T, axes=([1, 2], [0, 1])) for g in G)


def local_energy_plain(h1, chol, T, W, n_up, n_dn, e_core=0.0):
    """E_L from the full Green's function. Returns (E, E1, EJ, EK), all complex."""
    G = greens_function(T, W, n_up, n_dn)
    e1 = sum(np.trace(h1 @ g) for g in G)
    vbar = force_bias_plain(chol, G)
    ej = 0.5 * np.sum(vbar * vbar)
    ek = 0.0
    for g in G:
        LG = np.matmul(chol, g)                          # L^n G
        ek = ek - 0.5 * np.sum(LG * np.swapaxes(LG, 1, 2))   # tr(L G L G)
    return e_core + e1 + ej + ek, e1, ej, ek


# ---------------------------------------------------------------------------
# Half-rotated form: tr(L G) = tr(Lt Theta), tr(LGLG) = tr(Omega Omega)
# ---------------------------------------------------------------------------
def half_rotate(h1, chol, T, n_up, n_dn):
    """ht^s = T^sH h (N x M), Lt^s[n] = T^sH L^n (N x M)."""
    ht, Lt = [], []
    for b in spin_blocks(n_up, n_dn):
        Th = T[:, b].conj().T
        ht.append(Th @ h1)
        Lt.append(np.matmul(Th, chol))
    return ht, Lt


def theta(T, W, n_up, n_dn):
    """Theta^s = W^s (T^sH W^s)^-1 and log det S^s."""
    th, logdet = [], 0.0 + 0.0j
    for b in spin_blocks(n_up, n_dn):
        S = T[:, b].conj().T @ W[:, b]
        th.append(W[:, b] @ np.linalg.inv(S))
        sign, ld = np.linalg.slogdet(S)
        logdet += ld + np.log(sign)
    return th, logdet


def local_energy_half(ht, Lt, T, W, n_up, n_dn, e_core=0.0):
    """Half-rotated E_L and vbar: Omega^{ns} = Lt^{ns} Theta^s (N x N)."""
    th, _ = theta(T, W, n_up, n_dn)
    e1 = sum(np.sum(ht[s] * th[s].T) for s in range(2))
    vbar = 0.0
    ek = 0.0
    for s in range(2):
        Om = np.matmul(Lt[s], th[s])                     # Omega^{ns} = Lt^{ns} Theta^s
        vbar = vbar + np.trace(Om, axis1=1, axis2=2)
        ek = ek - 0.5 * np.sum(Om * np.swapaxes(Om, 1, 2))
    ej = 0.5 * np.sum(vbar * vbar)
    return e_core + e1 + ej + ek, (e1, ej, ek), vbar


# ---------------------------------------------------------------------------
# One-body propagator pieces (Hubbard-Stratonovich with the force-bias shift)
# ---------------------------------------------------------------------------
def force_bias_shift(vbar, dt, cap=0.0):
    """xbar_n = -i sqrt(dt) vbar_n. With cap > 0 every xbar_n of modulus above
    cap is scaled back to modulus cap, its phase kept (the usual force-bias cap
    of production phaseless AFQMC; the paper does not discuss it)."""
    xbar = -1j * np.sqrt(dt) * np.asarray(vbar)
    if cap > 0.0:
        mag = np.abs(xbar)
        big = mag > cap
        xbar = np.where(big, xbar * (cap / np.where(big, mag, 1.0)), xbar)
    return xbar


def mean_field_bias(chol, phi_t, n_up, n_dn):
    """c_n = sum_s tr(L^n G_T^s), G_T^s = T^s T^sH: the force bias of the trial
    itself (real for real symmetric L^n), the usual background vector."""
    out = np.zeros(chol.shape[0])
    for b in spin_blocks(n_up, n_dn):
        T = phi_t[:, b]
        out += np.einsum("nik,ki->n", chol, T @ T.conj().T).real
    return out


def hs_operator(chol, x, xbar, dt):
    """A = i sqrt(dt) sum_n (x_n - xbar_n) L^n (M x M)."""
    return np.tensordot(1j * np.sqrt(dt) * (x - xbar), chol, axes=1)


def importance_log_factor(x, xbar):
    """log of p(x - xbar)/p(x) for the standard normal p: sum_n x_n xbar_n - xbar_n^2/2."""
    return np.sum(x * xbar - 0.5 * xbar * xbar)


# ---------------------------------------------------------------------------
# The walk
# ---------------------------------------------------------------------------
def prepare(h1, chol, phi_t, n_up, n_dn, dt, vmf=None):
    """One-time set-up of the walk. With a background vector vmf (mean-field
    subtraction) the one-body factor is exp(-dt/2 (h' + sum_n vmf_n L^n))."""
    hp = one_body_corrected(h1, chol)
    if vmf is not None:
        vmf = np.asarray(vmf, dtype=np.float64)
        hp = hp + np.tensordot(vmf, chol, axes=1)
    B1 = sym_expm(-0.5 * dt * hp)
    ht, Lt = half_rotate(h1, chol, phi_t, n_up, n_dn)
    return dict(hp=hp, B1=B1, ht=ht, Lt=Lt, vmf=vmf)


def run(h1, chol, phi_t, n_up, n_dn, W0, weights0, fields, dt, qr_every=5,
        e_shift=0.0, order=6, e_core=0.0, energy="half", record_walkers=False, pre=None,
        fb_cap=0.0, w_cap=0.0, comb_every=0, comb_xi=None, bp_start=None, bp_len=0, msd=None, vmf=None):
    """Run len(fields) steps. fields[k, w, n] are the standard-normal HS fields.
    `pre` may hold prepare(h1, chol, phi_t, n_up, n_dn, dt) computed beforehand.

    Per step k (energy and force bias both at the start-of-step walker W_k):
      1. Theta, E_L (E1, EJ, EK) and vbar at W_k;
         E_mix(k) = sum_w w_k Re E_L / sum_w w_k with the pre-update weights.
      2. For live walkers: W' = B1 T_K(A) B1 W, r = O'/O, phaseless weight
         (the force bias capped at fb_cap and the new weight at w_cap when
         these are positive). A walker whose weight becomes 0 (or non-finite)
         is frozen (W not updated).
      3. QR of the live walkers when (k+1) % qr_every == 0.
      4. Population control when comb_every > 0 and (k+1) % comb_every == 0:
         comb() with the next uniform number of comb_xi. out["weights"][k]
         holds the weights before this step's comb.
    With bp_start set, a back-propagation window of bp_len steps opens at the
    start of step bp_start: out["bp_W0"] holds the walkers then, out["bp_coefs"]
    [j, w] the coefficients c_n = i sqrt(dt) (x_n - xbar_n) of A = sum_n c_n L^n
    drawn by walker w in step bp_start + j (zero for frozen walkers), and
    out["bp_weights"] the weights at the end of the window. A comb inside the
    window hands every copy its source walker's history (ket and coefficients).
    out["log_I"][k, w] is the complex log of the importance factor I of
    walker w in step k, before the phaseless projection (zero for frozen
    walkers).
    With vmf (a real vector of n_chol entries, or taken from `pre`) the walk
    subtracts that background: B1 from h' + sum vmf L, xbar for vbar - vmf,
    log I += c0 + dt/2 sum vmf^2 with c0 = -i sqrt(dt) sum_n (x_n - xbar_n)
    vmf_n, and the phaseless angle is Im(log r + c0).
    With msd = dict(dets=[...], coeffs=[...]) the trial is the orthogonal
    multi-determinant expansion of oracle/msd.py (phi_t is then unused):
    overlaps, E_L and the force bias come from its determinant sums, and the
    recorded parts are (E1, E2, 0) with E2 the whole two-body term.
    """
    M = h1.shape[0]
    nw = W0.shape[0]
    if pre is None:
        pre = prepare(h1, chol, phi_t, n_up, n_dn, dt, vmf=vmf)
    elif vmf is not None:
        assert pre.get("vmf") is not None and np.array_equal(pre["vmf"], vmf), "pre was prepared for another vmf"
    B1, ht, Lt = pre["B1"], pre["ht"], pre["Lt"]
    vmf = pre.get("vmf")
    W = W0.astype(np.complex128).copy()
    w = np.asarray(weights0, dtype=np.float64).copy()
    if msd is not None:
        from . import msd as msd_mod

        def log_ovlp(Wi):
            return np.log(msd_mod.overlap(msd["dets"], msd["coeffs"], Wi, n_up, n_dn))
    else:
        def log_ovlp(Wi):
            return theta(phi_t, Wi, n_up, n_dn)[1]
    logO = np.empty(nw, dtype=np.complex128)
    for i in range(nw):
        logO[i] = log_ovlp(W[i])
    alive = w > 0
    n_steps = fields.shape[0]
    out = dict(emix=np.zeros(n_steps), eloc=np.zeros((n_steps, nw), np.complex128),
               parts=np.zeros((n_steps, nw, 3), np.complex128),
               weights=np.zeros((n_steps, nw)), ratio=np.zeros((n_steps, nw), np.complex128),
               log_I=np.zeros((n_steps, nw), np.complex128), cosdt=np.ones((n_steps, nw)))
    if record_walkers:
        out["walkers"] = np.zeros((n_steps,) + W.shape, np.complex128)
    def open_window():
        out["bp_W0"] = W.copy()
        out["bp_coefs"] = np.zeros((bp_len, nw, chol.shape[0]), np.complex128)
        if bp_len == 0:
            out["bp_weights"] = w.copy()

    in_window = lambda k: bp_start is not None and bp_start <= k < bp_start + bp_len
    for k in range(n_steps):
        if bp_start == k:
            open_window()
        vb = np.zeros((nw, chol.shape[0]), np.complex128)
        for i in range(nw):
            if msd is not None:
                e, e1, e2, vb[i] = msd_mod.local_energy(h1, chol, msd["dets"], msd["coeffs"], W[i], n_up, n_dn,
                                                        e_core)
                parts = (e1, e2, 0.0)
            elif energy == "plain":
                e, e1, ej, ek = local_energy_plain(h1, chol, phi_t, W[i], n_up, n_dn, e_core)
                parts = (e1, ej, ek)
                G = greens_function(phi_t, W[i], n_up, n_dn)
                vb[i] = force_bias_plain(chol, G)
            else:
                e, parts, vb[i] = local_energy_half(ht, Lt, phi_t, W[i], n_up, n_dn, e_core)
            out["eloc"][k, i] = e
            out["parts"][k, i] = parts
        sw = np.sum(w)
        out["emix"][k] = np.sum(w * out["eloc"][k].real) / sw if sw > 0 else 0.0
        for i in range(nw):
            if not alive[i]:
                continue
            x = fields[k, i]
            xbar = force_bias_shift(vb[i] if vmf is None else vb[i] - vmf, dt, fb_cap)
            A = hs_operator(chol, x, xbar, dt)
            if in_window(k):
                out["bp_coefs"][k - bp_start, i] = 1j * np.sqrt(dt) * (x - xbar)
            Wn = B1 @ taylor_apply(A, B1 @ W[i], order)
            logOn = log_ovlp(Wn)
            log_r = logOn - logO[i]
            r = np.exp(log_r)
            log_I = log_r + importance_log_factor(x, xbar) + dt * e_shift
            phase = log_r.imag
            if vmf is not None:        # c-number part of the shifted operators, and the constant
                c0 = -1j * np.sqrt(dt) * np.sum((x - xbar) * vmf)
                log_I = log_I + c0 + 0.5 * dt * np.sum(vmf * vmf)
                phase = phase + c0.imag
            out["log_I"][k, i] = log_I
            cos_dth = np.cos(phase)
            wn = w[i] * np.exp(log_I.real) * cos_dth if cos_dth > 0.0 else 0.0
            out["ratio"][k, i] = r
            out["cosdt"][k, i] = cos_dth
            if not np.isfinite(wn) or wn <= 0.0:
                w[i] = 0.0
                alive[i] = False
                continue
            if w_cap > 0.0:
                wn = min(wn, w_cap)
            w[i] = wn
            W[i] = Wn
            logO[i] = logOn
        if qr_every > 0 and (k + 1) % qr_every == 0:
            for i in range(nw):
                if not alive[i]:
                    continue
                for b in spin_blocks(n_up, n_dn):
                    Q, R = qr_positive(W[i][:, b])
                    W[i][:, b] = Q
                    logO[i] -= np.sum(np.log(np.diag(R).real))
        out["weights"][k] = w
        if comb_every > 0 and (k + 1) % comb_every == 0:
            src, wnew, _ = comb(w, comb_xi[len(out.setdefault("comb_src", []))])
            out["comb_src"].append(src)
            W = W[src].copy()
            logO = logO[src].copy()
            w = np.full(nw, wnew)
            alive = np.ones(nw, dtype=bool)
            if in_window(k):
                out["bp_W0"] = out["bp_W0"][src].copy()
                out["bp_coefs"] = out["bp_coefs"][:, src].copy()
        if in_window(k) and k == bp_start + bp_len - 1:
            out["bp_weights"] = w.copy()
        if record_walkers:
            out["walkers"][k] = W
    if bp_start == n_steps:
        open_window()
    out.update(W=W, w=w, logO=logO, alive=alive)
    return out


# ---------------------------------------------------------------------------
# Population control (production bookkeeping around the walk; the paper only
# cites the method, so these follow the standard phaseless-AFQMC practice)
# ---------------------------------------------------------------------------
def comb(weights, xi):
    """Systematic resampling ("comb") of a weighted population of n walkers
    into n walkers of equal weight W/n, W = sum of the weights.

    The running sums C_i = w_0 + ... + w_i are formed left to right; tooth k of
    the comb sits at u_k = (k + xi) W / n (0 <= xi < 1) and selects the walker
    i with C_{i-1} <= u_k < C_i. A tooth that rounding puts at or beyond W
    selects the last walker of positive weight. Returns (source index of every
    new walker, the new common weight W/n, W)."""
    w = np.asarray(weights, dtype=np.float64)
    n = w.size
    cum = np.cumsum(w)
    total = cum[-1]
    if not total > 0.0:
        raise ValueError("comb: no walker has positive weight")
    step = total / n
    u = (np.arange(n, dtype=np.float64) + xi) * step
    src = np.searchsorted(cum, u, side="right")
    last = int(np.nonzero(w > 0.0)[0][-1])
    return np.minimum(src, last), step, total


def eshift_update(e_est, w_total, w_target, dt, gain_steps):
    """Population-control energy shift: E_shift = E_est - ln(W / W_target) / (g dt)
    with g = gain_steps, pulling the total weight W back toward W_target."""
    return e_est - np.log(w_total / w_target) / (gain_steps * dt)


def energy(h1, chol, phi_t, n_up, n_dn, W, weights, e_core=0.0, form="half"):
    """Per-walker E_L, parts (E1, EJ, EK) and the weighted mixed energy."""
    nw = W.shape[0]
    el = np.zeros(nw, np.complex128)
    parts = np.zeros((nw, 3), np.complex128)
    if form == "half":
        ht, Lt = half_rotate(h1, chol, phi_t, n_up, n_dn)
    for i in range(nw):
        if form == "half":
            el[i], p, _ = local_energy_half(ht, Lt, phi_t, W[i], n_up, n_dn, e_core)
        else:
            e, e1, ej, ek = local_energy_plain(h1, chol, phi_t, W[i], n_up, n_dn, e_core)
            el[i], p = e, (e1, ej, ek)
        parts[i] = p
    w = np.asarray(weights, dtype=np.float64)
    emix = np.sum(w * el.real) / np.sum(w)
    return el, parts, emix


# ---------------------------------------------------------------------------
# Adjoint of the weighted mixed energy  Ebar = sum_w w Re E_L / sum_w w
# (weights and the trial held fixed; gradients w.r.t. every entry of h1, L^n
# and, in torch's convention d/dRe + i d/dIm, the walker orbitals).
# ---------------------------------------------------------------------------
def energy_grad(h1, chol, phi_t, n_up, n_dn, W, weights):
    nw = W.shape[0]
    X, M, _ = chol.shape
    w = np.asarray(weights, dtype=np.float64)
    wh = w / np.sum(w)
    d_h1 = np.zeros((M, M))
    d_chol = np.zeros((X, M, M))
    d_W = np.zeros_like(W, dtype=np.complex128)
    ht, Lt = half_rotate(h1, chol, phi_t, n_up, n_dn)
    for i in range(nw):
        G = greens_function(phi_t, W[i], n_up, n_dn)
        Gsum = G[0] + G[1]
        vbar = force_bias_plain(chol, G)
        # dE/dh_ij = G_ji ; dE/dL^n_ij = vbar_n G_ji - sum_s (G L^n G)_ji
        d_h1 += wh[i] * Gsum.T.real
        dl = vbar[:, None, None] * Gsum.T[None]
        for g in G:
            GLG = np.matmul(np.matmul(g, chol), g)          # G L^n G
            dl = dl - np.transpose(GLG, (0, 2, 1))
        d_chol += wh[i] * dl.real
        # dE/dW^s = (I - G^s)^T Gamma^s S^-T, Gamma = dE/dTheta (holomorphic)
        th, _ = theta(phi_t, W[i], n_up, n_dn)
        for s, b in enumerate(spin_blocks(n_up, n_dn)):
            Om = np.matmul(Lt[s], th[s])
            gam = ht[s].T + np.tensordot(vbar, Lt[s], axes=1).T \
                - np.sum(np.matmul(Om, Lt[s]), axis=0).T
            S = phi_t[:, b].conj().T @ W[i][:, b]
            dEdW = (np.eye(M) - G[s]).T @ gam @ np.linalg.inv(S).T
            d_W[i][:, b] = wh[i] * np.conj(dEdW)
    return d_h1, d_chol, d_W


def mixed_rdm1(phi_t, n_up, n_dn, W, weights):
    """Weighted mixed one-body density matrix P_ij = sum_w wh_w sum_s <c+_i c_j>_w = G_ji."""
    w = np.asarray(weights, dtype=np.float64)
    wh = w / np.sum(w)
    P = 0.0
    for i in range(W.shape[0]):
        G = greens_function(phi_t, W[i], n_up, n_dn)
        P = P + wh[i] * (G[0] + G[1]).T
    return P



# ---------------------------------------------------------------------------
# Back-propagated one-body density matrix (the back-propagation paragraph of
# the AFQMC section; the method itself is only cited there). For an operator
# that does not commute with H the mixed form <T|O|phi>/<T|phi> is biased; the
# back-propagated form replaces the bra <T| by <T| B_{n-1} ... B_0, the trial
# carried through the n steps that followed the ket phi (the walker at the
# start of the window) with the fields those steps drew, and weighs each walker
# by its weight at the end of the window. No path restoration of the phases is
# applied.
# ---------------------------------------------------------------------------
def back_propagate(B1, chol, phi_t, n_up, n_dn, coefs, order, qr_every=0):
    """Ket form of the back-propagated bra of one walker.

    coefs[j, n] are the propagator coefficients of step j of the window,
    A_j = sum_n coefs[j, n] L^n and B_j = B1 T_K(A_j) B1. The bra
    <T| B_{n-1} ... B_0 is the ket B_0^H ... B_{n-1}^H |T>; with L^n and B1
    real symmetric, B_j^H = B1 T_K(A_j^H) B1 with A_j^H = sum_n conj(c_jn) L^n
    (the Taylor polynomial commutes with the adjoint). B_{n-1}^H acts first.
    With qr_every > 0 each spin block is replaced by the Q of its
    positive-diagonal QR after every qr_every of these steps; the estimator
    depends on the bra only through the column space of each spin block, so
    this changes nothing but rounding."""
    psi = phi_t.astype(np.complex128).copy()
    n = coefs.shape[0]
    for t, j in enumerate(range(n - 1, -1, -1)):
        AH = np.tensordot(np.conj(coefs[j]), chol, axes=1)
        psi = B1 @ taylor_apply(AH, B1 @ psi, order)
        if qr_every > 0 and (t + 1) % qr_every == 0:
            for b in spin_blocks(n_up, n_dn):
                psi[:, b], _ = qr_positive(psi[:, b])
    return psi


def back_propagated_rdm1(B1, chol, phi_t, n_up, n_dn, W0, coefs, weights, order, qr_every=0):
    """Spin-resolved back-propagated 1-RDM
        P[s, i, j] = sum_w w_w <psi_w| c+_is c_js |phi_w> / <psi_w|phi_w> / sum_w w_w
    with phi_w = W0[w] (walkers at the start of the window), psi_w the
    back-propagated bra of walker w (coefs[:, w, :]) and w_w the weights at the
    end of the window. Per spin, <psi|c+_i c_j|phi>/<psi|phi> = G_ji with
    G = phi (psi^H phi)^-1 psi^H (the same Wick form as the mixed estimate, bra
    psi in place of T). Walkers of weight 0 are skipped."""
    w = np.asarray(weights, dtype=np.float64)
    M = phi_t.shape[0]
    P = np.zeros((2, M, M), np.complex128)
    for i in range(W0.shape[0]):
        if w[i] == 0.0:
            continue
        psi = back_propagate(B1, chol, phi_t, n_up, n_dn, coefs[:, i], order, qr_every)
        G = greens_function(psi, W0[i], n_up, n_dn)
        for s in range(2):
            P[s] += w[i] * G[s].T
    return P / np.sum(w)
