"""Gauss-Hermite average of one oracle walk step over its auxiliary fields,
mapped to the determinant space (shared by the propagator pins).

One step of the oracle's walk from |W> for every node of a product
Gauss-Hermite grid, each node's walker weighted by exp(log I - log r) (the
importance factor without the determinant ratio: the state a walker stands for
is I |W'> / <T|W'> for the start state |W> / <T|W>), must average to
exp(-dt (H - E_shift)) |W> up to O(dt^2) per step.
"""
import numpy as np
from numpy.polynomial.hermite_e import hermegauss
from scipy.linalg import expm

from oracle import fci

N_NODES = 16          # per field; the integrand is a degree-24 polynomial times exp(x xbar)


def grid(n_fields):
    t, g = hermegauss(N_NODES)
    g = g / np.sqrt(2.0 * np.pi)
    xs = np.stack([m.ravel() for m in np.meshgrid(*([t] * n_fields), indexing="ij")], axis=1)
    gs = np.prod(np.stack([m.ravel() for m in np.meshgrid(*([g] * n_fields), indexing="ij")], axis=1), axis=1)
    return xs, gs


def averaged_step_error(step, H, W, n_up, n_dn, n_fields, dt, e_shift):
    """|| sum_q g_q exp(log I_q - log r_q) c(W'_q) - exp(-dt (H - E_shift)) c(W) || / ||.||"""
    xs, gs = grid(n_fields)
    nq = len(gs)
    o = step(np.repeat(W[None], nq, axis=0), xs[None], dt, e_shift)
    assert o["alive"].all(), "a quadrature node was killed by the phaseless projection"
    acc = 0.0
    for q in range(nq):
        acc = acc + gs[q] * np.exp(o["log_I"][0, q] - np.log(o["ratio"][0, q])) * fci.coefficients(
            o["W"][q], n_up, n_dn)
    exact = expm(-dt * (H - e_shift * np.eye(len(H)))) @ fci.coefficients(W, n_up, n_dn)
    return np.linalg.norm(acc - exact) / np.linalg.norm(exact)
