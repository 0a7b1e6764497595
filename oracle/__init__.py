"""CPU oracle for the TAPT hot path -- test infrastructure only.

Python face of ``oracle.c`` (a plain, single-threaded C implementation of
Algorithm 1 of arXiv:2509.23043). Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product library
(``paper_2509_23043_amd``) never imports it and shares no code with it.

Use:
    st = oracle.Run(problem, betas, seed=..., M=1, rule="metropolis", banks=...)
    st.run(n_sweeps)          # continue the chain
    st.spins, st.E, st.t ...  # numpy views of the state, slot order
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import build, library_path

RULES = {"metropolis": 0, "gibbs": 1}


class _Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("row_ptr", C.POINTER(C.c_int32)),
        ("col", C.POINTER(C.c_int32)),
        ("J", C.POINTER(C.c_int32)),
        ("h", C.POINTER(C.c_int32)),
        ("clamp", C.POINTER(C.c_int8)),
        ("color", C.POINTER(C.c_int32)),
        ("ncolors", C.c_int32),
        ("R", C.c_int32),
        ("beta", C.POINTER(C.c_double)),
        ("rule", C.c_int32),
        ("M", C.c_int32),
        ("prop_start", C.c_int64),
        ("prop_period", C.c_int64),
        ("prop_stop", C.c_int64),
        ("seed", C.c_uint64),
        ("bank", C.POINTER(C.POINTER(C.c_int8))),
        ("bank_n", C.POINTER(C.c_int32)),
        ("has_target", C.c_int32),
        ("target", C.c_int64),
        ("check_energy", C.c_int32),
        ("ctx_fraction", C.c_double),
        ("ctx_sweeps", C.c_int32),
    ]


class _State(C.Structure):
    _fields_ = [
        ("t", C.c_uint64),
        ("spins", C.POINTER(C.c_int8)),
        ("E", C.POINTER(C.c_int64)),
        ("cursor", C.POINTER(C.c_int32)),
        ("best", C.c_int64),
        ("best_t", C.c_int64),
        ("best_slot", C.c_int32),
        ("best_spins", C.POINTER(C.c_int8)),
        ("first_hit", C.c_int64),
        ("swap_att", C.POINTER(C.c_uint64)),
        ("swap_acc", C.POINTER(C.c_uint64)),
        ("prop_att", C.POINTER(C.c_uint64)),
        ("prop_acc", C.POINTER(C.c_uint64)),
        ("flips", C.POINTER(C.c_uint64)),
        ("energy_mismatch", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("TAPT_ORACLE_LIB") or library_path()
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        L.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.c_uint64, C.POINTER(C.c_uint32)]
        L.orc_philox.restype = None
        L.orc_sweep_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_sweep_uniform.restype = C.c_uint32
        L.orc_threshold.argtypes = [C.c_double]
        L.orc_threshold.restype = C.c_uint32
        L.orc_flip_prob.argtypes = [C.c_int32, C.c_double, C.c_int64]
        L.orc_flip_prob.restype = C.c_double
        L.orc_energy.argtypes = [C.POINTER(_Problem), C.POINTER(C.c_int8)]
        L.orc_energy.restype = C.c_int64
        L.orc_init.argtypes = [C.POINTER(_Problem), C.POINTER(_State)]
        L.orc_run.argtypes = [C.POINTER(_Problem), C.POINTER(_State), C.c_uint64]
        L.orc_flip_table.argtypes = [C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_uint32)]
        L.orc_flip_table.restype = None
        L.orc_run_sampled.argtypes = [C.POINTER(_Problem), C.POINTER(_State), C.c_uint64, C.c_uint64,
                                      C.POINTER(C.c_uint64)]
        L.orc_context_candidate.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_uint32, C.POINTER(C.c_int8),
                                            C.POINTER(C.c_int8), C.POINTER(C.c_int8), C.POINTER(C.c_uint8)]
        L.orc_context_candidate.restype = None
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, seed):
    """Philox4x32-10 of a 4-word counter under a 64-bit seed -> 4 uint32."""
    c = np.ascontiguousarray(ctr, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_p(c, C.c_uint32), C.c_uint64(seed), _p(out, C.c_uint32))
    return out


def sweep_uniform(seed, site, t, slot):
    return int(lib().orc_sweep_uniform(seed, site, t, slot))


def threshold(p):
    return int(lib().orc_threshold(float(p)))


def flip_table(rule, beta, dmax):
    out = np.zeros(2 * dmax + 1, np.uint32)
    lib().orc_flip_table(RULES[rule], float(beta), int(dmax), _p(out, C.c_uint32))
    return out


class Run:
    """One TAPT run of the oracle on one problem instance.

    problem: dict from ``paper_2509_23043_amd.inputs`` (n, row_ptr, col, J, h,
    clamp, color). banks: optional {slot: int8 [B, n]} proposal banks; a slot
    is proposal-enabled iff it has a bank. ctx_fraction / ctx_sweeps: the
    contextual proposals of the context ablation (a random choice of
    round(ctx_fraction * n_free) free sites is the context; the rest is
    completed by ctx_sweeps sweeps from the bank entry).
    """

    def __init__(self, problem, betas, seed, M=1, rule="metropolis", banks=None,
                 prop_start=0, prop_period=0, prop_stop=-1, target=None,
                 check_energy=True, ctx_fraction=0.0, ctx_sweeps=0):
        n = int(problem["n"])
        self.n = n
        self.R = R = len(betas)
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dt)
            self._keep.append(a)
            return a

        row_ptr = keep(problem["row_ptr"], np.int32)
        col = keep(problem["col"], np.int32)
        J = keep(problem["J"], np.int32)
        h = keep(problem.get("h", np.zeros(n)), np.int32)
        clamp = keep(problem.get("clamp", np.zeros(n)), np.int8)
        color = keep(problem["color"], np.int32)
        beta = keep(betas, np.float64)
        P = _Problem()
        P.n = n
        P.row_ptr, P.col, P.J, P.h = _p(row_ptr, C.c_int32), _p(col, C.c_int32), _p(J, C.c_int32), _p(h, C.c_int32)
        P.clamp = _p(clamp, C.c_int8)
        P.color = _p(color, C.c_int32)
        P.ncolors = int(color.max()) + 1 if n else 0
        P.R = R
        P.beta = _p(beta, C.c_double)
        P.rule = RULES[rule]
        P.M = int(M)
        P.prop_start, P.prop_period, P.prop_stop = int(prop_start), int(prop_period), int(prop_stop)
        P.seed = int(seed)
        if banks:
            ptrs = (C.POINTER(C.c_int8) * R)()
            bn = keep(np.zeros(R), np.int32)
            for r, b in banks.items():
                b = keep(b, np.int8)
                assert b.ndim == 2 and b.shape[1] == n
                ptrs[r] = _p(b, C.c_int8)
                bn[r] = b.shape[0]
            self._keep.append(ptrs)
            P.bank = C.cast(ptrs, C.POINTER(C.POINTER(C.c_int8)))
            P.bank_n = _p(bn, C.c_int32)
        else:
            P.bank = None
            P.bank_n = None
        P.has_target = 0 if target is None else 1
        P.target = 0 if target is None else int(target)
        P.check_energy = 1 if check_energy else 0
        P.ctx_fraction = float(ctx_fraction)
        P.ctx_sweeps = int(ctx_sweeps)
        self.P = P

        self.spins = np.zeros((R, n), np.int8)
        self.E = np.zeros(R, np.int64)
        self.cursor = np.zeros(R, np.int32)
        self.best_spins = np.zeros(n, np.int8)
        self.swap_att = np.zeros(max(R - 1, 1), np.uint64)
        self.swap_acc = np.zeros(max(R - 1, 1), np.uint64)
        self.prop_att = np.zeros(R, np.uint64)
        self.prop_acc = np.zeros(R, np.uint64)
        self.flips = np.zeros(R, np.uint64)
        S = _State()
        S.spins = _p(self.spins, C.c_int8)
        S.E = _p(self.E, C.c_int64)
        S.cursor = _p(self.cursor, C.c_int32)
        S.best_spins = _p(self.best_spins, C.c_int8)
        S.swap_att, S.swap_acc = _p(self.swap_att, C.c_uint64), _p(self.swap_acc, C.c_uint64)
        S.prop_att, S.prop_acc = _p(self.prop_att, C.c_uint64), _p(self.prop_acc, C.c_uint64)
        S.flips = _p(self.flips, C.c_uint64)
        self.S = S
        lib().orc_init(C.byref(P), C.byref(S))

    def run(self, n_sweeps):
        rc = lib().orc_run(C.byref(self.P), C.byref(self.S), C.c_uint64(int(n_sweeps)))
        if rc != 0:
            raise RuntimeError("oracle run failed")
        return self

    def run_sampled(self, n_sweeps, thin=1):
        """Run and return hist[R, 2^n] of slot states seen after every thin-th sweep."""
        hist = np.zeros((self.R, 1 << self.n), np.uint64)
        rc = lib().orc_run_sampled(C.byref(self.P), C.byref(self.S), C.c_uint64(int(n_sweeps)),
                                   C.c_uint64(int(thin)), _p(hist, C.c_uint64))
        if rc != 0:
            raise RuntimeError("oracle sampled run failed")
        return hist

    def context_candidate(self, r, cyc, start, current):
        """The contextual proposal of slot r at cycle cyc built from the bank
        entry ``start`` and the slot's ``current`` spins: (candidate, mask of
        the context sites)."""
        a = np.ascontiguousarray(start, np.int8)
        b = np.ascontiguousarray(current, np.int8)
        out = np.zeros(self.n, np.int8)
        mask = np.zeros(self.n, np.uint8)
        lib().orc_context_candidate(C.byref(self.P), int(r), C.c_uint32(int(cyc)), _p(a, C.c_int8),
                                    _p(b, C.c_int8), _p(out, C.c_int8), _p(mask, C.c_uint8))
        return out, mask

    def energy(self, spins):
        s = np.ascontiguousarray(spins, np.int8)
        return int(lib().orc_energy(C.byref(self.P), _p(s, C.c_int8)))

    # scalar views of the state
    t = property(lambda s: int(s.S.t))
    best = property(lambda s: int(s.S.best))
    best_t = property(lambda s: int(s.S.best_t))
    best_slot = property(lambda s: int(s.S.best_slot))
    first_hit = property(lambda s: int(s.S.first_hit))
    energy_mismatch = property(lambda s: int(s.S.energy_mismatch))


def energy(problem, spins):
    """E(m) of one configuration under ``problem`` (oracle energy function)."""
    return Run(problem, [1.0], seed=0).energy(spins)
