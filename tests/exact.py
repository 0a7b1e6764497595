"""Exact small-system results used to pin the CPU oracle.

Everything here is computed by exhaustive enumeration of the 2^n spin states
(n <= 16) in numpy, directly from the definitions in arXiv:2509.23043:
Boltzmann weights pi_beta(x) = exp(-beta E(x)) / Z (Supp. S2, Part 1) and the
transition matrices of Supp. S2, Part 2 (single-site updates composed into a
sweep, the swap matrix W_swap, the Delta-E-rule proposal matrix W_DeltaE).
Nothing here calls the oracle or the HIP path.
"""
from __future__ import annotations

import numpy as np

from paper_2509_23043_amd.inputs import csr_to_dense


def all_states(n):
    """[2^n, n] int8 +-1; state index k has spin i = +1 iff bit i of k is set."""
    k = np.arange(1 << n, dtype=np.int64)
    bits = (k[:, None] >> np.arange(n)) & 1
    return (bits * 2 - 1).astype(np.int8)


def dense(problem):
    return csr_to_dense(problem["n"], problem["row_ptr"], problem["col"], problem["J"])


def energies(problem, states=None):
    """E(x) = -sum_{i<j} J_ij x_i x_j - sum_i h_i x_i for all states."""
    n = problem["n"]
    if states is None:
        states = all_states(n)
    Jd = dense(problem).astype(np.float64)
    h = np.asarray(problem.get("h", np.zeros(n)), np.float64)
    out = np.empty(len(states), np.int64)
    for a in range(0, len(states), 1 << 16):
        x = states[a:a + (1 << 16)].astype(np.float64)
        e = -0.5 * ((x @ Jd) * x).sum(axis=1) - x @ h
        out[a:a + len(x)] = np.rint(e).astype(np.int64)
    return out


def boltzmann(E, beta):
    w = np.exp(-beta * (E - E.min()))
    return w / w.sum()


def level_distribution(E, beta):
    """{energy level: probability} under pi_beta."""
    p = boltzmann(E, beta)
    lv = np.unique(E)
    return lv, np.array([p[E == e].sum() for e in lv])


def flip_prob(rule, beta, dE):
    dE = np.asarray(dE, np.float64)
    if rule == "gibbs":
        return 1.0 / (1.0 + np.exp(beta * dE))
    return np.minimum(1.0, np.exp(-beta * dE))


def sweep_matrix(problem, beta, rule, order):
    """Column-stochastic W_sweep = W_{order[-1]} ... W_{order[0]} over 2^n states
    (single-site updates of the sites in ``order``, first applied first)."""
    n = problem["n"]
    S = all_states(n)
    E = energies(problem, S)
    N = 1 << n
    W = np.eye(N)
    idx = np.arange(N)
    for i in order:
        j = idx ^ (1 << i)          # state with spin i flipped
        dE = E[j] - E[idx]
        pf = flip_prob(rule, beta, dE)
        Wi = np.zeros((N, N))
        Wi[idx, idx] = 1.0 - pf
        Wi[j, idx] += pf
        W = Wi @ W
    return W


def prop_matrix_delta_e(E, beta, q):
    """W_DeltaE(x' <- x) = q(x') min[1, exp(-beta (E(x') - E(x)))], rejected mass
    on the diagonal (Supp. S2, Part 2)."""
    A = np.minimum(1.0, np.exp(-beta * (E[:, None] - E[None, :])))  # [x', x]
    W = q[:, None] * A
    np.fill_diagonal(W, 0.0)
    W[np.diag_indices_from(W)] = 1.0 - W.sum(axis=0)
    return W


def apply_axis(p, W, axis):
    """Apply a single-replica matrix W along replica ``axis`` of joint p."""
    return np.moveaxis(np.tensordot(W, p, axes=([1], [axis])), 0, axis)


def apply_swap(p, E, dbeta, r):
    """W_swap for pair (r, r+1) on the joint distribution p (Supp. S2, Part 2):
    from (a, b) the pair moves to (b, a) with min{1, exp(dbeta (E(b) - E(a)))}."""
    pm = np.moveaxis(p, (r, r + 1), (0, 1))
    A = np.minimum(1.0, np.exp(dbeta * (E[None, :] - E[:, None])))  # A[a, b]
    Ax = A.reshape(A.shape + (1,) * (pm.ndim - 2))
    out = pm * (1.0 - Ax) + np.swapaxes(pm * Ax, 0, 1)
    return np.moveaxis(out, (0, 1), (r, r + 1))


def tapt_cycle_marginals(problem, betas, rule, order, props, n_iter=4000):
    """Stationary per-slot marginals of the TAPT cycle chain of Algorithm 1 with
    M = 1: sweep all slots, proposals on the slots in ``props`` ({slot: q}),
    then the swap stage whose parity alternates with the cycle number.
    Returns the average of the marginals after odd and after even cycles."""
    n = problem["n"]
    N = 1 << n
    R = len(betas)
    E = energies(problem)
    Ws = [sweep_matrix(problem, b, rule, order) for b in betas]
    Wp = {r: prop_matrix_delta_e(E, betas[r], q) for r, q in props.items()}

    def cycle(p, odd):
        for r in range(R):
            p = apply_axis(p, Ws[r], r)
        for r in sorted(Wp):
            p = apply_axis(p, Wp[r], r)
        for r in range(0 if odd else 1, R - 1, 2):
            p = apply_swap(p, E, betas[r + 1] - betas[r], r)
        return p

    p = np.full((N,) * R, 1.0 / N ** R)
    for _ in range(n_iter):
        p_odd = cycle(p, True)
        p_new = cycle(p_odd, False)
        done = np.abs(p_new - p).max() < 1e-14
        p = p_new
        if done:
            break
    p_odd = cycle(p, True)
    marg = []
    for r in range(R):
        axes = tuple(a for a in range(R) if a != r)
        marg.append(0.5 * (p.sum(axis=axes) + p_odd.sum(axis=axes)))
    return np.array(marg)


def kl(p, q):
    m = p > 0
    return float(np.sum(p[m] * np.log(p[m] / q[m])))
