"""Seeded synthetic problem generators shared by the tests, the benchmark and
the CPU reference.

This module only *describes problems*: coupling graphs, fields, clamps,
colorings, temperature ladders, proposal banks and semiprimes. It holds none
of the sampler's arithmetic (no energies, no acceptance rules, no random
numbers the sampler draws), so neither the HIP path nor the reference depends
on the other through it.

Problem conventions (arXiv:2509.23043, Supp. S4, energy convention):
E(m) = -sum_{i<j} J_ij m_i m_j - sum_i h_i m_i with m_i in {-1,+1}, J symmetric
with zero diagonal. Graphs are returned in CSR form with both directions of
every edge stored.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# small CSR helpers


def dense_to_csr(Jd: np.ndarray):
    """Dense symmetric integer coupling matrix -> (row_ptr, col, J) int32 CSR."""
    Jd = np.asarray(Jd)
    n = Jd.shape[0]
    assert Jd.shape == (n, n)
    assert np.array_equal(Jd, Jd.T), "J must be symmetric"
    assert not np.any(np.diag(Jd)), "J must have zero diagonal"
    row_ptr = np.zeros(n + 1, np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(Jd[i])[0]
        cols.append(nz)
        vals.append(Jd[i, nz])
        row_ptr[i + 1] = row_ptr[i] + len(nz)
    col = np.concatenate(cols).astype(np.int32) if n else np.zeros(0, np.int32)
    J = np.concatenate(vals).astype(np.int32) if n else np.zeros(0, np.int32)
    return row_ptr, col, J


def csr_to_dense(n, row_ptr, col, J):
    Jd = np.zeros((n, n), np.int64)
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            Jd[i, col[k]] = J[k]
    return Jd


def graph(n, row_ptr, col, J, h=None, clamp=None, color=None, **extra):
    """Bundle a general sparse Ising problem."""
    g = dict(
        kind="csr",
        n=int(n),
        row_ptr=np.ascontiguousarray(row_ptr, np.int32),
        col=np.ascontiguousarray(col, np.int32),
        J=np.ascontiguousarray(J, np.int32),
        h=np.zeros(n, np.int32) if h is None else np.ascontiguousarray(h, np.int32),
        clamp=np.zeros(n, np.int8) if clamp is None else np.ascontiguousarray(clamp, np.int8),
    )
    g["color"] = dsatur(n, g["row_ptr"], g["col"]) if color is None else np.ascontiguousarray(color, np.int32)
    g.update(extra)
    return g


# ---------------------------------------------------------------------------
# 3D periodic cubic lattice (Edwards-Anderson +-J spin glass and ferromagnet)
#
# Site index i = x + L*(y + L*z). Bond array J3[d][i] holds the coupling of the
# bond from site i to its +x (d=0), +y (d=1), +z (d=2) neighbour, periodic.


def lattice_site(L, x, y, z):
    return (x % L) + L * ((y % L) + L * (z % L))


def lattice_neighbours(L):
    """[n, 6] neighbour table in the order +x, -x, +y, -y, +z, -z."""
    n = L ** 3
    i = np.arange(n)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    nb = np.stack([
        lattice_site(L, x + 1, y, z), lattice_site(L, x - 1, y, z),
        lattice_site(L, x, y + 1, z), lattice_site(L, x, y - 1, z),
        lattice_site(L, x, y, z + 1), lattice_site(L, x, y, z - 1),
    ], axis=1)
    return nb.astype(np.int32)


def ea_lattice(L: int, seed: int, ferro: bool = False):
    """3D Edwards-Anderson +-J instance on the periodic L^3 cubic lattice.

    Couplings iid uniform in {-1,+1} from ``seed`` (numpy PCG64), h = 0.
    ``ferro=True`` gives the ferromagnet (all J = +1).
    """
    if L < 3:
        raise ValueError("periodic lattice needs L >= 3 (L=2 would double bonds)")
    n = L ** 3
    if ferro:
        J3 = np.ones((3, n), np.int8)
    else:
        rng = np.random.Generator(np.random.PCG64(seed))
        J3 = (rng.integers(0, 2, size=(3, n), dtype=np.int8) * 2 - 1).astype(np.int8)
    g = lattice_to_csr(L, J3)
    g.update(lattice_L=L, J3=J3, seed=seed)
    return g


def lattice_to_csr(L, J3):
    """Express a periodic cubic instance as a general CSR graph (both directions)."""
    n = L ** 3
    nb = lattice_neighbours(L)
    # coupling of each of the 6 bonds of site i
    Jn = np.empty((n, 6), np.int32)
    Jn[:, 0] = J3[0]
    Jn[:, 1] = J3[0][nb[:, 1]]
    Jn[:, 2] = J3[1]
    Jn[:, 3] = J3[1][nb[:, 3]]
    Jn[:, 4] = J3[2]
    Jn[:, 5] = J3[2][nb[:, 5]]
    row_ptr = (np.arange(n + 1) * 6).astype(np.int32)
    g = graph(n, row_ptr, nb.reshape(-1), Jn.reshape(-1), color=lattice_colors(L))
    return g


def lattice_colors(L):
    """Checkerboard coloring (x+y+z) mod 2; proper for even L."""
    if L % 2:
        raise ValueError("checkerboard coloring of a periodic lattice needs even L")
    i = np.arange(L ** 3)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    return ((x + y + z) & 1).astype(np.int32)


def square_lattice_2d(L: int, J: int = 1):
    """Periodic L x L square lattice (L >= 3), uniform coupling J, h=0."""
    n = L * L
    Jd = np.zeros((n, n), np.int64)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            for (dx, dy) in ((1, 0), (0, 1)):
                j = (x + dx) % L + L * ((y + dy) % L)
                Jd[i, j] += J
                Jd[j, i] += J
    return graph(n, *dense_to_csr(Jd))


def open_box(dims, seed=None):
    """Open-boundary grid graph of the given dims; +-1 couplings from seed or +1."""
    dims = tuple(dims)
    n = int(np.prod(dims))
    rng = None if seed is None else np.random.Generator(np.random.PCG64(seed))
    Jd = np.zeros((n, n), np.int64)
    idx = np.arange(n).reshape(dims[::-1])  # z, y, x
    for axis in range(len(dims)):
        a = np.moveaxis(idx, axis, 0)
        for k in range(a.shape[0] - 1):
            for i, j in zip(a[k].ravel(), a[k + 1].ravel()):
                v = 1 if rng is None else int(rng.integers(0, 2)) * 2 - 1
                Jd[i, j] = Jd[j, i] = v
    return graph(n, *dense_to_csr(Jd))


# ---------------------------------------------------------------------------
# Temperature ladders


def geometric_ladder(R: int, beta_min: float = 0.2, beta_max: float = 3.0) -> np.ndarray:
    """beta_r = beta_min * (beta_max/beta_min)^(r/(R-1)), r = 0 (hottest) .. R-1."""
    if R == 1:
        return np.array([beta_min], np.float64)
    r = np.arange(R, dtype=np.float64)
    b = beta_min * (beta_max / beta_min) ** (r / (R - 1))
    b[-1] = beta_max
    return b.astype(np.float64)


# ---------------------------------------------------------------------------
# Invertible-logic gadgets (Supp. S4). Logical 0 -> -1, 1 -> +1.

# AND gate, spin order (A, B, C)
AND_J = np.array([[0, -1, 2], [-1, 0, 2], [2, 2, 0]], np.int64)
AND_H = np.array([1, 1, -2], np.int64)

# Full adder, spin order (A, B, Cin, S, Cout), h = 0
FA_J = np.array([
    [0, -1, -1, 1, 2],
    [-1, 0, -1, 1, 2],
    [-1, -1, 0, 1, 2],
    [1, 1, 1, 0, -2],
    [2, 2, 2, -2, 0],
], np.int64)
FA_H = np.zeros(5, np.int64)


def gadget_graph(kind: str):
    Jd, h = (AND_J, AND_H) if kind == "and" else (FA_J, FA_H)
    n = Jd.shape[0]
    return graph(n, *dense_to_csr(Jd), h=h, color=np.arange(n, dtype=np.int32))


def multiplier(m: int, product: int | None = None):
    """m x m-bit array multiplier built from AND gadgets and full adders.

    Row 0 of partial products p_0j = a_j AND b_0 gives product bit c_0 = p_00.
    Row i >= 1 adds p_ij to the previous row's sum shifted down by one with a
    ripple-carry chain of full adders FA(i, j): inputs (p_ij, r_ij, carry-in),
    outputs (s_ij, cout_ij). The carry-in of FA(i, 0) is a spin clamped to
    logical 0; r_1,m-1 (the top input of row 1) is another clamped-0 spin;
    r_i,m-1 = cout_{i-1,m-1} for i >= 2. Product bits: c_i = s_i0 for
    1 <= i <= m-1, c_{m-1+j} = s_{m-1,j} for j >= 1, c_{2m-1} = cout_{m-1,m-1}.
    That is 3m^2 + m spins: m + m factor bits, m^2 AND outputs, 2m(m-1) adder
    outputs and m clamped zeros.

    With ``product`` given the 2m product spins are clamped to its bits
    (reverse mode); factor bits stay free.
    """
    if m < 2:
        raise ValueError("multiplier needs m >= 2")
    names = []

    def new(name):
        names.append(name)
        return len(names) - 1

    a = [new(f"a{j}") for j in range(m)]
    b = [new(f"b{i}") for i in range(m)]
    p = [[new(f"p{i}_{j}") for j in range(m)] for i in range(m)]
    s = {}
    co = {}
    for i in range(1, m):
        for j in range(m):
            s[i, j] = new(f"s{i}_{j}")
            co[i, j] = new(f"co{i}_{j}")
    zeros = [new(f"zero_cin{i}") for i in range(1, m)] + [new("zero_top")]
    n = len(names)
    assert n == 3 * m * m + m

    Jd = np.zeros((n, n), np.int64)
    h = np.zeros(n, np.int64)

    def place(idx, GJ, Gh):
        for u in range(len(idx)):
            h[idx[u]] += Gh[u]
            for v in range(len(idx)):
                if u != v:
                    Jd[idx[u], idx[v]] += GJ[u, v]

    for i in range(m):
        for j in range(m):
            place([a[j], b[i], p[i][j]], AND_J, AND_H)
    zero_cin = {i: zeros[i - 1] for i in range(1, m)}
    zero_top = zeros[-1]
    for i in range(1, m):
        for j in range(m):
            if j < m - 1:
                r = p[0][j + 1] if i == 1 else s[i - 1, j + 1]
            else:
                r = zero_top if i == 1 else co[i - 1, m - 1]
            cin = zero_cin[i] if j == 0 else co[i, j - 1]
            place([p[i][j], r, cin, s[i, j], co[i, j]], FA_J, FA_H)

    c = [p[0][0]] + [s[i, 0] for i in range(1, m)] + [s[m - 1, j] for j in range(1, m)] + [co[m - 1, m - 1]]
    assert len(c) == 2 * m
    clamp = np.zeros(n, np.int8)
    for z in zeros:
        clamp[z] = -1
    if product is not None:
        if not (0 <= product < (1 << (2 * m))):
            raise ValueError("product does not fit 2m bits")
        for k, idx in enumerate(c):
            clamp[idx] = 1 if (product >> k) & 1 else -1
    row_ptr, col, J = dense_to_csr(Jd)
    return graph(n, row_ptr, col, J, h=h, clamp=clamp,
                 m=m, product=product, a_idx=np.array(a), b_idx=np.array(b),
                 c_idx=np.array(c), zero_idx=np.array(zeros), names=names,
                 n_and=m * m, n_fa=m * (m - 1))


def bits_to_int(spins, idx):
    """Read an integer from spins (+1 = logical 1) at bit positions idx (LSB first)."""
    v = 0
    for k, i in enumerate(idx):
        if spins[i] > 0:
            v |= 1 << k
    return v


def multiplier_assignment(g, A: int, B: int):
    """The spin configuration of multiplier ``g`` that computes A*B correctly."""
    m = g["m"]
    names = g["names"]
    val = {}
    for j in range(m):
        val[f"a{j}"] = (A >> j) & 1
        val[f"b{j}"] = (B >> j) & 1
    for i in range(m):
        for j in range(m):
            val[f"p{i}_{j}"] = val[f"a{j}"] & val[f"b{i}"]
    for i in range(1, m):
        carry = 0
        for j in range(m):
            if j < m - 1:
                r = val[f"p0_{j + 1}"] if i == 1 else val[f"s{i - 1}_{j + 1}"]
            else:
                r = 0 if i == 1 else val[f"co{i - 1}_{m - 1}"]
            tot = val[f"p{i}_{j}"] + r + carry
            val[f"s{i}_{j}"] = tot & 1
            carry = tot >> 1
            val[f"co{i}_{j}"] = carry
    for nm in names:
        if nm.startswith("zero"):
            val[nm] = 0
    return np.array([1 if val[nm] else -1 for nm in names], np.int8)


# ---------------------------------------------------------------------------
# Graph coloring: DSATUR (Brelaz 1979)


def dsatur(n, row_ptr, col):
    """Greedy DSATUR coloring. Picks the uncolored vertex with the most distinct
    neighbour colors (ties: larger degree, then lower index) and gives it the
    smallest color absent from its neighbours."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    color = np.full(n, -1, np.int64)
    deg = np.diff(row_ptr)
    sat = [set() for _ in range(n)]
    for _ in range(n):
        best, key = -1, None
        for v in range(n):
            if color[v] >= 0:
                continue
            k = (len(sat[v]), deg[v], -v)
            if key is None or k > key:
                best, key = v, k
        v = best
        used = sat[v]
        c = 0
        while c in used:
            c += 1
        color[v] = c
        for k in range(row_ptr[v], row_ptr[v + 1]):
            sat[col[k]].add(c)
    return color.astype(np.int32)


def is_proper_coloring(n, row_ptr, col, color):
    for i in range(n):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            if color[col[k]] == color[i]:
                return False
    return True


# ---------------------------------------------------------------------------
# Semiprimes, banks


def primes_in(lo: int, hi: int):
    """Primes p with lo <= p < hi."""
    out = []
    for p in range(max(lo, 2), hi):
        if all(p % d for d in range(2, int(p ** 0.5) + 1)):
            out.append(p)
    return out


def semiprimes(m: int, count: int, seed: int):
    """``count`` products p*q of distinct primes drawn from [2^(m-1), 2^m)."""
    ps = primes_in(1 << (m - 1), 1 << m)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        i, j = rng.choice(len(ps), size=2, replace=False)
        p, q = ps[i], ps[j]
        out.append((p * q, min(p, q), max(p, q)))
    return out


def random_bank(n: int, B: int, seed: int, clamp=None):
    """B configurations of n spins, iid uniform +-1, clamped sites forced."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bank = (rng.integers(0, 2, size=(B, n), dtype=np.int8) * 2 - 1).astype(np.int8)
    if clamp is not None:
        clamp = np.asarray(clamp, np.int8)
        fixed = clamp != 0
        bank[:, fixed] = clamp[fixed]
    return bank
