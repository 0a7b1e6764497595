"""Pins of the CPU oracle against things fixed by the paper and by mathematics.

Each test names what it pins. None retypes the oracle's own formula: they
compare it with an independent Philox implementation (rocRAND), with the
gadget truth tables and closed forms of Supp. S4, with exact Boltzmann
distributions and exact transition-matrix stationary distributions obtained
by enumeration (Supp. S2), and with invariants of Algorithm 1.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_2509_23043_amd import inputs
from tests import exact

# ---------------------------------------------------------------------------
# Philox4x32-10


def test_philox_known_answers():
    # known-answer vectors of the Philox4x32-10 definition (Salmon et al., SC'11)
    cases = [
        ([0, 0, 0, 0], 0, [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, 0xFFFFFFFFFFFFFFFF, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], 0x299F31D0A4093822,
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in cases:
        assert [int(x) for x in oracle.philox(ctr, key)] == want


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  probe e; unsigned a, b, c, d, k0, k1;
  while (scanf("%x %x %x %x %x %x", &a, &b, &c, &d, &k0, &k1) == 6) {
    uint4 o = e.run(uint4{a, b, c, d}, uint2{k0, k1});
    printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
  }
}
"""


def test_philox_matches_rocrand():
    """The oracle's Philox against rocRAND's independent implementation."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, 2 ** 32, size=(300, 4), dtype=np.uint64)
    keys = rng.integers(0, 2 ** 64, size=300, dtype=np.uint64)
    ctrs[:10] = [[k, 5, 7, 2 << 24] for k in range(10)]   # counters of the sweep stream
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(src, "w").write(ROCRAND_PROBE)
        subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe, src], check=True,
                       capture_output=True)
        lines = "".join(f"{c[0]:x} {c[1]:x} {c[2]:x} {c[3]:x} {int(k) & 0xFFFFFFFF:x} {int(k) >> 32:x}\n"
                        for c, k in zip(ctrs, keys))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, k, line in zip(ctrs, keys, out):
        want = [int(x, 16) for x in line.split()]
        assert [int(x) for x in oracle.philox(c, int(k))] == want


def test_sweep_uniform_layout():
    """u = (half (i&7) of the SWEEP block << 16) | same half of the REFINE block."""
    seed, t, r = 0x1234_5678_9ABC_DEF0, 17, 5
    for i in [0, 1, 7, 8, 13, 511]:
        hi = oracle.philox([i >> 3, t, r, 2], seed)[(i & 7) >> 1]
        lo = oracle.philox([i >> 3, t, r, 3], seed)[(i & 7) >> 1]
        sh = 16 * (i & 1)
        want = (((int(hi) >> sh) & 0xFFFF) << 16) | ((int(lo) >> sh) & 0xFFFF)
        assert oracle.sweep_uniform(seed, i, t, r) == want


# ---------------------------------------------------------------------------
# thresholds


def test_threshold_edges():
    assert oracle.threshold(1.0) == 0xFFFFFFFF
    assert oracle.threshold(2.0) == 0xFFFFFFFF
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(0.5) == 1 << 31
    assert oracle.threshold(2.0 ** -32) == 1
    assert oracle.threshold(2.0 ** -33) == 0
    assert oracle.threshold(1.0 - 2.0 ** -40) == 0xFFFFFFFF


@pytest.mark.parametrize("beta", [0.2, 0.7, 1.3, 3.0])
def test_flip_tables(beta):
    D = 40
    met = oracle.flip_table("metropolis", beta, D).astype(np.int64)
    gib = oracle.flip_table("gibbs", beta, D).astype(np.int64)
    d = np.arange(-D, D + 1)
    # Metropolis: downhill and flat moves always accepted; uphill decreasing
    assert np.all(met[d <= 0] == 0xFFFFFFFF)
    assert np.all(np.diff(met) <= 0)
    # Gibbs: P(dE) + P(-dE) = 1 (heat bath), so the thresholds sum to 2^32 within 1
    s = gib + gib[::-1]
    assert np.all((s == 2 ** 32) | (s == 2 ** 32 - 1))
    assert gib[D] == 1 << 31
    assert np.all(np.diff(gib) <= 0)
    # Gibbs never exceeds Metropolis for the same move
    assert np.all(gib <= met)


# ---------------------------------------------------------------------------
# energy function against Supp. S4 truth tables and closed forms


def _all_energies(g):
    S = exact.all_states(g["n"])
    run = oracle.Run(g, [1.0], seed=0)
    return S, np.array([run.energy(s) for s in S])


def test_and_gadget_truth_table():
    g = inputs.gadget_graph("and")
    S, E = _all_energies(g)
    bits = (S > 0).astype(int)
    valid = (bits[:, 2] == (bits[:, 0] & bits[:, 1]))
    assert set(E[valid]) == {-3}
    assert E[~valid].min() > -3
    assert sorted(set(E)) == [-3, 1, 9]
    # decimal labels of Fig. S7 read (A, B, C) as a binary number, A the MSB
    dec = bits[:, 0] * 4 + bits[:, 1] * 2 + bits[:, 2]
    assert sorted(dec[E == -3]) == [0, 2, 4, 7]


def test_full_adder_truth_table():
    g = inputs.gadget_graph("fa")
    S, E = _all_energies(g)
    b = (S > 0).astype(int)
    tot = b[:, 0] + b[:, 1] + b[:, 2]
    valid = (b[:, 3] == tot % 2) & (b[:, 4] == tot // 2)
    assert valid.sum() == 8
    assert set(E[valid]) == {-4}
    assert E[~valid].min() > -4
    assert sorted(set(E)) == [-4, -2, 4, 14]


def test_and_gate_boltzmann_beta1():
    """Fig. S7: at beta = 1 the four valid states carry most of the weight."""
    g = inputs.gadget_graph("and")
    S, E = _all_energies(g)
    p = np.exp(-E) / np.exp(-E).sum()
    valid = E == -3
    assert np.allclose(p[valid], 0.24661, atol=5e-6)
    assert np.allclose(np.sort(p[~valid])[-3:], 0.00452, atol=5e-6)


@pytest.mark.parametrize("L", [4, 6])
def test_ferromagnet_ground_energy(L):
    g = inputs.ea_lattice(L, 0, ferro=True)
    n = L ** 3
    run = oracle.Run(g, [1.0], seed=0)
    assert run.energy(np.ones(n, np.int8)) == -3 * n
    assert run.energy(-np.ones(n, np.int8)) == -3 * n
    # one flipped spin breaks its 6 bonds: +12
    m = np.ones(n, np.int8)
    m[5] = -1
    assert run.energy(m) == -3 * n + 12


def test_multiplier_spin_count_law():
    """N_spin = 3/4 n^2 + 1/2 n with n = 2m product bits (Supp. S5) and the
    sizes of Table S3: 200, 252, 310, 374, 444 spins for 16..24-bit products."""
    table_s3 = {16: 200, 18: 252, 20: 310, 22: 374, 24: 444}
    for nbits, N in table_s3.items():
        g = inputs.multiplier(nbits // 2)
        assert g["n"] == N == (3 * nbits * nbits) // 4 + nbits // 2


@pytest.mark.parametrize("m", [2, 3, 5, 8, 10, 12])
def test_multiplier_valid_assignment_is_ground(m):
    """A correct multiplication puts every gadget in its ground state:
    E = -3 m^2 (ANDs) - 4 m (m-1) (full adders)."""
    rng = np.random.default_rng(m)
    for _ in range(3):
        A, B = (int(x) for x in rng.integers(0, 1 << m, size=2))
        g = inputs.multiplier(m, A * B)
        s = inputs.multiplier_assignment(g, A, B)
        assert np.all((g["clamp"] == 0) | (g["clamp"] == s))
        run = oracle.Run(g, [1.0], seed=0)
        assert run.energy(s) == -3 * m * m - 4 * m * (m - 1)
        assert inputs.bits_to_int(s, g["a_idx"]) * inputs.bits_to_int(s, g["b_idx"]) == A * B


def test_paper_example_1022117():
    """Fig. 4d: C = 1,022,117 = 1009 x 1013, a 20-bit product (m = 10)."""
    C = 1022117
    assert C == 1009 * 1013 and C < (1 << 20)
    g = inputs.multiplier(10, C)
    assert g["n"] == 310
    s = inputs.multiplier_assignment(g, 1009, 1013)
    run = oracle.Run(g, [1.0], seed=0)
    assert run.energy(s) == -3 * 100 - 4 * 10 * 9


def _free_enumeration_energies(g):
    free = np.nonzero(g["clamp"] == 0)[0]
    base = g["clamp"].astype(np.int8).copy()
    S = exact.all_states(len(free))
    full = np.repeat(base[None, :], len(S), axis=0)
    full[:, free] = S
    return full, exact.energies(g, full)


def test_multiplier_m2_ground_states_are_all_products():
    g = inputs.multiplier(2)          # product free; only the zero spins clamped
    full, E = _free_enumeration_energies(g)
    gnd = full[E == E.min()]
    assert E.min() == -3 * 4 - 4 * 2
    seen = set()
    for s in gnd:
        A = inputs.bits_to_int(s, g["a_idx"])
        B = inputs.bits_to_int(s, g["b_idx"])
        C = inputs.bits_to_int(s, g["c_idx"])
        assert A * B == C
        seen.add((A, B))
    assert seen == {(a, b) for a in range(4) for b in range(4)}
    # the oracle energy agrees with enumeration on ground states
    run = oracle.Run(g, [1.0], seed=0)
    assert all(run.energy(s) == E.min() for s in gnd[:8])


def test_multiplier_m3_reverse_mode_35():
    g = inputs.multiplier(3, 35)
    full, E = _free_enumeration_energies(g)
    gnd = full[E == E.min()]
    assert E.min() == -3 * 9 - 4 * 6
    facs = {(inputs.bits_to_int(s, g["a_idx"]), inputs.bits_to_int(s, g["b_idx"])) for s in gnd}
    assert facs == {(5, 7), (7, 5)}


# ---------------------------------------------------------------------------
# chain dynamics


def _batch_z(series, exact_mean, nb=40):
    """z-score of the mean of a correlated series via batch means."""
    series = np.asarray(series, np.float64)
    k = len(series) // nb
    b = series[: k * nb].reshape(nb, k).mean(axis=1)
    se = b.std(ddof=1) / np.sqrt(nb)
    return (b.mean() - exact_mean) / max(se, 1e-12)


def _state_series(problem, betas, rule, n_sweeps, seed, **kw):
    """Per-slot state-index histograms in 40 consecutive blocks."""
    run = oracle.Run(problem, betas, seed=seed, rule=rule, **kw)
    blocks = [run.run_sampled(n_sweeps // 40) for _ in range(40)]
    return run, np.stack(blocks)          # [40, R, 2^n]


@pytest.mark.parametrize("rule", ["metropolis", "gibbs"])
def test_pt_stationary_boltzmann_2d(rule):
    """Sweeps + alternating swaps preserve the product Boltzmann measure, so
    each slot's energy distribution is exact g(E) e^{-beta E} / Z."""
    g = inputs.square_lattice_2d(4)
    rng = np.random.default_rng(11)
    g["J"] = g["J"] * 0 + 1
    # +-J couplings, kept symmetric
    Jd = exact.dense(g)
    up = np.triu(Jd != 0)
    signs = rng.choice([-1, 1], size=Jd.shape)
    Jd = np.where(up, Jd * signs, 0)
    Jd = Jd + Jd.T
    g = inputs.graph(16, *inputs.dense_to_csr(Jd))
    betas = np.array([0.3, 0.55, 0.8, 1.1])
    E = exact.energies(g)
    run, H = _state_series(g, betas, rule, 120_000, seed=3)
    levels = np.unique(E)
    for r, b in enumerate(betas):
        pex = exact.boltzmann(E, b)
        # mean energy
        per_block_E = (H[:, r, :] * E[None, :]).sum(axis=1) / H[:, r, :].sum(axis=1)
        z = _batch_z(per_block_E, float((pex * E).sum()), nb=40)
        assert abs(z) < 5, (r, z)
        # every energy level with probability > 2%
        for e in levels:
            pe = pex[E == e].sum()
            if pe < 0.02:
                continue
            frac = H[:, r, E == e].sum(axis=1) / H[:, r, :].sum(axis=1)
            z = _batch_z(frac, pe, nb=40)
            assert abs(z) < 5, (r, e, z)
    # swap acceptance equals E_{pi_r x pi_r+1}[min(1, exp(dbeta dE))]
    for r in range(len(betas) - 1):
        lv, p1 = exact.level_distribution(E, betas[r])
        _, p2 = exact.level_distribution(E, betas[r + 1])
        dE = lv[None, :] - lv[:, None]                # E(x_{r+1}) - E(x_r)
        acc = (p1[:, None] * p2[None, :] * np.minimum(1, np.exp((betas[r + 1] - betas[r]) * dE))).sum()
        rate = run.swap_acc[r] / run.swap_att[r]
        se = np.sqrt(acc * (1 - acc) / run.swap_att[r]) * 6   # generous: correlated
        assert abs(rate - acc) < max(5 * se, 0.01), (r, rate, acc)


def test_pt_stationary_detects_wrong_beta():
    """Discriminating power: the exact law at the neighbouring beta is rejected."""
    g = inputs.square_lattice_2d(4)
    betas = np.array([0.3, 0.45])
    E = exact.energies(g)
    run, H = _state_series(g, betas, "metropolis", 40_000, seed=5)
    per_block_E = (H[:, 0, :] * E[None, :]).sum(axis=1) / H[:, 0, :].sum(axis=1)
    wrong = float((exact.boltzmann(E, 0.45) * E).sum())
    assert abs(_batch_z(per_block_E, wrong)) > 10


@pytest.mark.parametrize("rule", ["gibbs", "metropolis"])
def test_tapt_full_adder_transition_matrix(rule):
    """Fig. S2: three replicas of the full adder at beta = {0.5, 1.7, 4.6},
    independent exact-equilibrium proposals on the two hotter replicas under
    the Delta-E rule (Eq. 2). The oracle's per-slot state frequencies must
    match the stationary marginals of the exact transition-matrix chain of
    Supp. S2 (sequential sweep over the five spins, then proposals, then the
    alternating swap stage), which differ from Boltzmann."""
    g = inputs.gadget_graph("fa")          # one color per site: sweep in index order
    betas = np.array([0.5, 1.7, 4.6])
    E = exact.energies(g)
    S = exact.all_states(5)
    rng = np.random.default_rng(2024)
    B = 1 << 17
    banks, qs = {}, {}
    for r in (0, 1):
        pi = exact.boltzmann(E, betas[r])
        draw = rng.choice(32, size=B, p=pi)
        banks[r] = S[draw]
        qs[r] = np.bincount(draw, minlength=32) / B      # exact proposal law of this bank
    marg = exact.tapt_cycle_marginals(g, betas, rule, order=list(range(5)), props=qs)
    n_cyc = 120_000
    run, H = _state_series(g, betas, rule, n_cyc, seed=9, banks=banks, prop_start=1, prop_period=1)
    assert run.prop_att[0] == n_cyc and run.prop_att[2] == 0
    for r in range(3):
        emp_blocks = H[:, r, :] / H[:, r, :].sum(axis=1, keepdims=True)
        for x in range(32):
            if marg[r, x] < 0.01:
                continue
            z = _batch_z(emp_blocks[:, x], marg[r, x])
            assert abs(z) < 5, (r, x, marg[r, x], z)
    # the Delta-E rule biases the hot replica away from Boltzmann (Supp. S2)
    pi0 = exact.boltzmann(E, betas[0])
    assert exact.kl(marg[0], pi0) > 1e-3
    emp0 = H[:, 0, :].sum(axis=0) / H[:, 0, :].sum()
    big = np.argmax(np.abs(marg[0] - pi0))
    emp_blocks = H[:, 0, :] / H[:, 0, :].sum(axis=1, keepdims=True)
    assert abs(_batch_z(emp_blocks[:, big], pi0[big])) > 8, emp0[big]


def test_and_gate_sampling_beta1():
    """Single replica of the AND gate at beta = 1 samples Fig. S7's law."""
    g = inputs.gadget_graph("and")
    E = exact.energies(g)
    run, H = _state_series(g, [1.0], "gibbs", 200_000, seed=4)
    p = exact.boltzmann(E, 1.0)
    blocks = H[:, 0, :] / H[:, 0, :].sum(axis=1, keepdims=True)
    for x in range(8):
        if p[x] > 0.001:
            assert abs(_batch_z(blocks[:, x], p[x])) < 5


def test_single_spin_in_field():
    """N = 1 with field h: stationary P(+1) = e^{beta h} / (2 cosh beta h)."""
    g = inputs.graph(1, np.array([0, 0]), np.zeros(0), np.zeros(0), h=np.array([1]))
    for rule in ("metropolis", "gibbs"):
        run, H = _state_series(g, [0.7], rule, 200_000, seed=1)
        frac = H[:, 0, 1] / H[:, 0, :].sum(axis=1)
        assert abs(_batch_z(frac, np.exp(0.7) / (2 * np.cosh(0.7)))) < 5


# ---------------------------------------------------------------------------
# invariants of Algorithm 1


def test_incremental_energy_matches_recompute():
    g = inputs.ea_lattice(4, 1)
    betas = inputs.geometric_ladder(16)
    run = oracle.Run(g, betas, seed=1001, check_energy=True)
    run.run(300)
    assert run.energy_mismatch == 0
    for r in range(16):
        assert run.E[r] == run.energy(run.spins[r])


@pytest.mark.parametrize("M", [1, 2, 3])
def test_swap_parity_and_counts(M):
    """Cycle n odd attempts pairs (0,1),(2,3),...; even n attempts (1,2),(3,4),..."""
    g = inputs.ea_lattice(4, 2)
    R = 7
    run = oracle.Run(g, inputs.geometric_ladder(R), seed=5, M=M)
    T = 61 * M + (M - 1)          # an odd number of cycles, and a partial one
    run.run(T)
    cycles = T // M
    n_odd, n_even = (cycles + 1) // 2, cycles // 2
    assert n_odd != n_even
    for r in range(R - 1):
        assert run.swap_att[r] == (n_odd if r % 2 == 0 else n_even)


def test_proposal_schedule_and_cursor():
    g = inputs.ea_lattice(4, 3)
    R = 6
    B = 5
    banks = {r: inputs.random_bank(64, B, seed=100 + r) for r in (0, 2)}
    run = oracle.Run(g, inputs.geometric_ladder(R), seed=8, banks=banks,
                     prop_start=10, prop_period=7, prop_stop=50)
    start = run.cursor.copy()
    for r in (0, 2):
        assert start[r] == int(oracle.philox([r, 0, 0, 6], 8)[0]) % B
    run.run(60)
    n_prop = len(range(10, 51, 7))
    for r in range(R):
        assert run.prop_att[r] == (n_prop if r in banks else 0)
    for r in banks:
        assert run.cursor[r] == (start[r] + n_prop) % B


def test_accepted_proposal_is_copied():
    """A bank holding the ground state of a ferromagnet: d <= 0, always accepted."""
    g = inputs.ea_lattice(4, 0, ferro=True)
    bank = np.ones((1, 64), np.int8)
    run = oracle.Run(g, [0.2, 0.3], seed=2, banks={0: bank}, prop_start=1, prop_period=1)
    run.run(1)
    assert run.prop_acc[0] == 1
    # after the proposal the swap stage (cycle 1, pair (0,1)) may move it
    assert -192 in run.E
    assert run.best == -192 and run.best_t == 1


def test_ferromagnet_reaches_ground_state():
    g = inputs.ea_lattice(4, 0, ferro=True)
    run = oracle.Run(g, inputs.geometric_ladder(16), seed=1001, target=-192)
    run.run(1000)
    assert run.best == -192
    assert 0 < run.first_hit <= 1000
    assert run.energy(run.best_spins) == -192


def test_factorization_solved():
    """Reverse-mode 4x4 multiplier: the chain reaches E_gnd and the factor
    spins multiply to the clamped product."""
    C = 11 * 13
    g = inputs.multiplier(4, C)
    egnd = -3 * 16 - 4 * 12
    run = oracle.Run(g, inputs.geometric_ladder(16, 0.2, 3.0), seed=77, target=egnd)
    run.run(3000)
    assert run.best == egnd
    s = run.best_spins
    A, B = inputs.bits_to_int(s, g["a_idx"]), inputs.bits_to_int(s, g["b_idx"])
    assert A * B == C and {A, B} == {11, 13}


def test_clamped_spins_never_move():
    g = inputs.multiplier(3, 35)
    run = oracle.Run(g, inputs.geometric_ladder(4), seed=3)
    run.run(200)
    fixed = g["clamp"] != 0
    assert np.all(run.spins[:, fixed] == g["clamp"][fixed])


def test_counter_wiring_brute_force():
    """Tiny-input brute force of the random-number contract: initial spins
    from the INIT stream and one full sweep (color 0 then color 1, increasing
    index) with the SWEEP/REFINE uniforms, recomputed here one site at a time."""
    g = inputs.ea_lattice(4, 9)
    betas = np.array([0.4, 1.5])
    seed = 0xABCDEF0123
    run = oracle.Run(g, betas, seed=seed)
    n = 64
    m = np.zeros((2, n), np.int64)
    for r in range(2):
        for i in range(n):
            w = int(oracle.philox([i >> 2, 0, r, 1], seed)[i & 3])
            m[r, i] = 1 if w >= 2 ** 31 else -1
    assert np.array_equal(run.spins, m)
    nbr = inputs.lattice_neighbours(4)
    J = inputs.csr_to_dense(n, g["row_ptr"], g["col"], g["J"])
    for r in range(2):
        for c in (0, 1):
            for i in range(n):
                if g["color"][i] != c:
                    continue
                I = sum(int(J[i, j]) * int(m[r, j]) for j in nbr[i])
                dE = 2 * int(m[r, i]) * I
                p = 1.0 if dE <= 0 else float(np.exp(-(betas[r] * dE)))
                T = oracle.threshold(p)
                u = oracle.sweep_uniform(seed, i, 1, r)
                if T == 0xFFFFFFFF or u < T:
                    m[r, i] = -m[r, i]
    run.run(1)
    # cycle 1 swaps pair (0, 1) or not; compare as a set of rows
    got = {run.spins[0].tobytes(), run.spins[1].tobytes()}
    want = {m[0].astype(np.int8).tobytes(), m[1].astype(np.int8).tobytes()}
    assert got == want


# ---------------------------------------------------------------------------
# independent chains (M = 0): the bank-generation runs of Supp. Table S3


def test_independent_chains_equal_a_run_without_cycle_ends():
    """With M = 0 no cycle ever ends: every slot is a plain Metropolis chain.
    That is the same chain as a ladder whose first cycle end lies beyond the
    run (M larger than the sweeps run), slot for slot."""
    g = inputs.ea_lattice(4, 7)
    betas = inputs.geometric_ladder(8)
    a = oracle.Run(g, betas, seed=77, M=0)
    b = oracle.Run(g, betas, seed=77, M=1000)
    a.run(300)
    b.run(300)
    assert np.array_equal(a.spins, b.spins) and np.array_equal(a.E, b.E)
    assert a.swap_att.sum() == 0 and b.swap_att.sum() == 0
    for r in range(8):
        assert a.E[r] == a.energy(a.spins[r])


def test_independent_chains_do_not_see_other_slots():
    """A slot's chain depends only on its own beta (equal betas allowed):
    changing every other slot's beta leaves it bit-identical."""
    g = inputs.ea_lattice(4, 8)
    a = oracle.Run(g, [1.0, 1.0, 1.0], seed=5, M=0)
    b = oracle.Run(g, [0.3, 1.0, 2.5], seed=5, M=0)
    a.run(200)
    b.run(200)
    assert np.array_equal(a.spins[1], b.spins[1]) and a.E[1] == b.E[1]
    assert not np.array_equal(a.spins[0], b.spins[0])


def test_independent_chain_samples_boltzmann():
    """One independent chain at beta = 0.7 on a single spin in a field samples
    P(+1) = e^{beta h} / (2 cosh beta h), as with swaps switched off."""
    g = inputs.graph(1, np.array([0, 0]), np.zeros(0), np.zeros(0), h=np.array([1]))
    run, H = _state_series(g, [0.7, 0.7], "metropolis", 200_000, seed=9, M=0)
    for r in range(2):
        frac = H[:, r, 1] / H[:, r, :].sum(axis=1)
        assert abs(_batch_z(frac, np.exp(0.7) / (2 * np.cosh(0.7)))) < 5
