"""ctypes binding of libtapt.so (include/tapt.h). Argument marshalling only:
every step of the hot path runs in the library's HIP kernels. There is no CPU
fallback; a missing or unloadable library raises."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtapt.so")

PT_OK = 0
PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_ESTATE, PT_EUNSUPPORTED, PT_ETIMEOUT = -1, -2, -3, -4, -5, -6
RULES = {"metropolis": 0, "gibbs": 1}


class TaptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtapt error {code}: {msg}")
        self.code = code


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int32), ("lattice_L", C.c_int32), ("nnz", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("J", C.POINTER(C.c_int32)), ("h", C.POINTER(C.c_int32)),
                ("clamp", C.POINTER(C.c_int8)), ("color", C.POINTER(C.c_int32))]


class _Opts(C.Structure):
    _fields_ = [("rule", C.c_int32), ("sweeps_per_cycle", C.c_int32), ("prop_start", C.c_int64),
                ("prop_period", C.c_int64), ("prop_stop", C.c_int64), ("seed", C.c_uint64),
                ("has_target", C.c_int32), ("target", C.c_int32)]


class _Summary(C.Structure):
    _fields_ = [("t", C.c_uint64), ("best_energy", C.c_int32), ("best_t", C.c_int64),
                ("best_slot", C.c_int32), ("first_hit", C.c_int64)]


class _BatchOpts(C.Structure):
    _fields_ = [("replicas_per_wg", C.c_int32), ("replicas_per_thread", C.c_int32),
                ("chunk_sweeps", C.c_int32), ("use_graph", C.c_int32), ("kernel", C.c_int32)]


KERNELS = {"auto": 0, "block": 1, "wave": 2, "pm": 3, "pm1": 4, "row": 5, "row4": 6, "pml": 7, "csrw": 8}


class _ServeOpts(C.Structure):
    _fields_ = [("mem_budget", C.c_uint64), ("chunk_sweeps", C.c_int32), ("max_active", C.c_int32),
                ("replicas_per_wg", C.c_int32), ("replicas_per_thread", C.c_int32), ("pipeline", C.c_int32)]


class _Request(C.Structure):
    _fields_ = [("problem", C.c_int32), ("has_target", C.c_int32), ("target", C.c_int32), ("pad", C.c_int32),
                ("seed", C.c_uint64), ("sweep_cap", C.c_uint64), ("best_out", C.c_void_p),
                ("user_tag", C.c_uint64)]


class _Result(C.Structure):
    _fields_ = [("id", C.c_uint64), ("user_tag", C.c_uint64), ("status", C.c_int32), ("hit", C.c_int32),
                ("first_hit", C.c_int64), ("best_energy", C.c_int32), ("best_slot", C.c_int32),
                ("best_t", C.c_int64), ("sweeps", C.c_uint64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


class _ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("rejected", C.c_uint64), ("rounds", C.c_uint64), ("busy_s", C.c_double),
                ("attempts", C.c_double), ("active", C.c_int32), ("waiting", C.c_int32),
                ("peak_active", C.c_int32), ("peak_lanes", C.c_int32), ("mem_used", C.c_uint64),
                ("mem_peak", C.c_uint64), ("gpu_busy_s", C.c_double)]


EXPORTS = ["pt_create", "pt_destroy", "pt_propose", "pt_propose_device", "pt_set_context", "pt_sweep", "pt_energies",
           "pt_state", "pt_state_device", "pt_set_state", "pt_save_size", "pt_save", "pt_restore",
           "pt_summary_get", "pt_counters",
           "pt_energy_device", "pt_set_stream", "pt_batch_create", "pt_batch_sweep", "pt_batch_destroy",
           "pt_batch_set_stream", "pt_batch_kernel_time", "pt_batch_describe", "pt_batch_run_static", "pt_serve_start",
           "pt_serve_register",
           "pt_serve_submit", "pt_serve_poll", "pt_serve_stats_get", "pt_serve_clock", "pt_serve_stop",
           "pt_probe_lds", "pt_probe_valu", "pt_last_error"]

_lib = None


def lib():
    """Load libtapt.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7);
    # loading torch first makes libtapt bind to that one, so the process has a
    # single HIP runtime and torch tensors and streams can be passed in.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.pt_create.argtypes = [C.POINTER(_Graph), C.POINTER(C.c_double), C.c_int32, C.POINTER(_Opts), C.POINTER(vp)]
    L.pt_destroy.argtypes = [vp]
    L.pt_propose.argtypes = [vp, C.c_double, C.POINTER(C.c_int8), C.c_int32]
    L.pt_propose_device.argtypes = [vp, C.c_double, vp, C.c_int32]
    L.pt_set_context.argtypes = [vp, C.c_double, C.c_int32]
    L.pt_sweep.argtypes = [vp, C.c_uint64]
    L.pt_energies.argtypes = [vp, C.POINTER(C.c_int32)]
    L.pt_state.argtypes = [vp, C.POINTER(C.c_int8), C.POINTER(C.c_uint64)]
    L.pt_state_device.argtypes = [vp, vp]
    L.pt_set_state.argtypes = [vp, C.POINTER(C.c_int8), C.c_uint64]
    L.pt_save_size.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.pt_save.argtypes = [vp, vp, C.c_uint64]
    L.pt_restore.argtypes = [vp, vp, C.c_uint64]
    L.pt_summary_get.argtypes = [vp, C.POINTER(_Summary), C.POINTER(C.c_int8)]
    L.pt_counters.argtypes = [vp] + [C.POINTER(C.c_uint64)] * 5
    L.pt_energy_device.argtypes = [vp, vp, C.c_int32, vp]
    L.pt_set_stream.argtypes = [vp, vp]
    L.pt_batch_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(_BatchOpts), C.POINTER(vp)]
    L.pt_batch_sweep.argtypes = [vp, C.c_uint64]
    L.pt_batch_destroy.argtypes = [vp]
    L.pt_batch_set_stream.argtypes = [vp, vp]
    L.pt_batch_kernel_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    L.pt_batch_describe.argtypes = [vp, C.c_char_p, C.c_int32]
    L.pt_batch_run_static.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(_BatchOpts), C.c_uint64, vp]
    L.pt_serve_start.argtypes = [C.POINTER(_ServeOpts), C.POINTER(vp)]
    L.pt_serve_register.argtypes = [vp, vp, C.POINTER(C.c_int32)]
    L.pt_serve_submit.argtypes = [vp, C.POINTER(_Request), C.POINTER(C.c_uint64)]
    L.pt_serve_poll.argtypes = [vp, C.POINTER(_Result), C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.pt_serve_stats_get.argtypes = [vp, C.POINTER(_ServeStats)]
    L.pt_serve_clock.argtypes = [vp]
    L.pt_serve_stop.argtypes = [vp]
    L.pt_probe_lds.argtypes = [C.c_int32, C.c_int32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.pt_probe_valu.argtypes = [C.c_int32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.pt_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("pt_last_error", "pt_serve_clock"):
            getattr(L, name).restype = C.c_int
    L.pt_serve_clock.restype = C.c_double
    _lib = L
    return L


def _check(rc):
    if rc != PT_OK:
        raise TaptError(rc, lib().pt_last_error().decode())


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Context:
    """One problem instance and its replica ladder on the GPU (pt_ctx)."""

    def __init__(self, problem, betas, seed, rule="metropolis", M=1, prop_start=0, prop_period=0,
                 prop_stop=-1, target=None):
        L = lib()
        n = int(problem["n"])
        self.n = n
        self.R = len(betas)
        self.nfree = int(n - np.count_nonzero(np.asarray(problem.get("clamp", np.zeros(n)))))
        self.M = int(M)
        self.betas = np.ascontiguousarray(betas, np.float64)
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dt)
            self._keep.append(a)
            return a

        g = _Graph()
        g.n = n
        self.kind, self.L = "csr", 0
        self.pm = False     # the +-J 8^3 kernel applies (every coupling +-1, even ladder)
        self.pml = False    # the +-J row kernel applies (even L in 6..16, every coupling +-1)
        if problem.get("lattice_L") and not np.any(problem.get("h", 0)) and not np.any(problem.get("clamp", 0)):
            g.lattice_L = int(problem["lattice_L"])
            self.kind = "lattice" if g.lattice_L <= 16 else "csr"
            self.L = g.lattice_L
            pmj = bool(np.all(np.abs(np.asarray(problem["J3"])) == 1))
            self.pm = self.L == 8 and self.R % 2 == 0 and pmj
            self.pml = self.L % 2 == 0 and 6 <= self.L <= 16 and pmj
            g.J = _p(keep(np.asarray(problem["J3"]).reshape(-1), np.int32), C.c_int32)
            g.nnz = 0
        else:
            g.lattice_L = 0
            rp = keep(problem["row_ptr"], np.int32)
            g.row_ptr = _p(rp, C.c_int32)
            g.col = _p(keep(problem["col"], np.int32), C.c_int32)
            g.J = _p(keep(problem["J"], np.int32), C.c_int32)
            g.nnz = int(rp[-1])
            g.color = _p(keep(problem["color"], np.int32), C.c_int32)
        if "h" in problem:
            g.h = _p(keep(problem["h"], np.int32), C.c_int32)
        if "clamp" in problem:
            g.clamp = _p(keep(problem["clamp"], np.int8), C.c_int8)
        o = _Opts()
        o.rule = RULES[rule]
        o.sweeps_per_cycle = int(M)
        o.prop_start, o.prop_period, o.prop_stop = int(prop_start), int(prop_period), int(prop_stop)
        o.seed = int(seed)
        o.has_target = 0 if target is None else 1
        o.target = 0 if target is None else int(target)
        h = C.c_void_p()
        _check(L.pt_create(C.byref(g), _p(self.betas, C.c_double), self.R, C.byref(o), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().pt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propose(self, slot, configs):
        """Install a bank (int8 [B, n]) on the slot ``slot`` (by its beta)."""
        cfg = np.ascontiguousarray(configs, np.int8)
        assert cfg.ndim == 2 and cfg.shape[1] == self.n
        _check(lib().pt_propose(self.h, float(self.betas[slot]), _p(cfg, C.c_int8), cfg.shape[0]))

    def propose_device(self, slot, dev_ptr, count):
        _check(lib().pt_propose_device(self.h, float(self.betas[slot]), C.c_void_p(dev_ptr), int(count)))

    def set_context(self, fraction, sweeps):
        """Contextual proposals: a random ``fraction`` of each proposal's free
        sites takes the slot's current values, the rest is completed by
        ``sweeps`` sweeps from the bank entry (0, 0: plain bank proposals)."""
        _check(lib().pt_set_context(self.h, float(fraction), int(sweeps)))

    def sweep(self, n):
        """Plain path: n sweeps of Algorithm 1, per-sweep launches."""
        _check(lib().pt_sweep(self.h, int(n)))

    def energies(self):
        out = np.zeros(self.R, np.int32)
        _check(lib().pt_energies(self.h, _p(out, C.c_int32)))
        return out

    def state(self):
        s = np.zeros((self.R, self.n), np.int8)
        t = C.c_uint64()
        _check(lib().pt_state(self.h, _p(s, C.c_int8), C.byref(t)))
        return s, int(t.value)

    def state_device(self, dev_ptr):
        _check(lib().pt_state_device(self.h, C.c_void_p(dev_ptr)))

    def set_state(self, spins, t):
        s = np.ascontiguousarray(spins, np.int8)
        _check(lib().pt_set_state(self.h, _p(s, C.c_int8), int(t)))

    def save(self):
        """Checkpoint of the whole chain state (pt_save) as bytes."""
        nb = C.c_uint64()
        _check(lib().pt_save_size(self.h, C.byref(nb)))
        buf = C.create_string_buffer(nb.value)
        _check(lib().pt_save(self.h, buf, nb.value))
        return buf.raw

    def restore(self, blob):
        """Resume from a checkpoint taken by save() (pt_restore)."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(lib().pt_restore(self.h, buf, len(blob)))

    def summary(self):
        s = _Summary()
        b = np.zeros(self.n, np.int8)
        _check(lib().pt_summary_get(self.h, C.byref(s), _p(b, C.c_int8)))
        return dict(t=s.t, best=s.best_energy, best_t=s.best_t, best_slot=s.best_slot,
                    first_hit=s.first_hit, best_spins=b)

    def counters(self):
        R = self.R
        a = [np.zeros(max(R - 1, 1), np.uint64), np.zeros(max(R - 1, 1), np.uint64),
             np.zeros(R, np.uint64), np.zeros(R, np.uint64), np.zeros(R, np.uint64)]
        _check(lib().pt_counters(self.h, *[_p(x, C.c_uint64) for x in a]))
        return dict(swap_att=a[0][:R - 1], swap_acc=a[1][:R - 1], prop_att=a[2], prop_acc=a[3], flips=a[4])

    def energy_device(self, cfg_ptr, k, out_ptr):
        _check(lib().pt_energy_device(self.h, C.c_void_p(cfg_ptr), int(k), C.c_void_p(out_ptr)))

    def set_stream(self, stream_ptr):
        _check(lib().pt_set_stream(self.h, C.c_void_p(stream_ptr)))


def probe_lds(bytes_per_read=16, blocks_per_cu=4, iters=2048):
    """Measured LDS read bandwidth (TB/s, ms) of the current device."""
    tb, ms = C.c_double(), C.c_double()
    rc = lib().pt_probe_lds(int(bytes_per_read), int(blocks_per_cu), int(iters), C.byref(tb), C.byref(ms))
    if rc != PT_OK:
        raise TaptError(rc, "LDS probe failed")
    return tb.value, ms.value


def probe_valu(op, iters=4096):
    """VALU issue rate (wave-instructions per clock per CU, ms) of op 0
    (v_xor_b32), 1 (v_mul_hi_u32), 2 (v_mul_lo_u32) or 3 (v_mad_u64_u32)."""
    r, ms = C.c_double(), C.c_double()
    rc = lib().pt_probe_valu(int(op), int(iters), C.byref(r), C.byref(ms))
    if rc != PT_OK:
        raise TaptError(rc, "VALU probe failed")
    return r.value, ms.value


def run_static(contexts, n_sweeps, replicas_per_wg=0, replicas_per_thread=0, chunk_sweeps=0, kernel="auto",
               stream_ptr=None):
    """pt_batch_run_static: a batched run of the contexts that allocates no
    device memory (the launch's buffers live in the library's static scratch)."""
    contexts = list(contexts)
    arr = (C.c_void_p * len(contexts))(*[c.h for c in contexts])
    o = _BatchOpts(int(replicas_per_wg), int(replicas_per_thread), int(chunk_sweeps), 0, KERNELS[kernel])
    _check(lib().pt_batch_run_static(arr, len(contexts), C.byref(o), int(n_sweeps),
                                     C.c_void_p(stream_ptr) if stream_ptr else None))


class Batch:
    """Many contexts run by persistent chunk launches (pt_batch)."""

    def __init__(self, contexts, replicas_per_wg=0, replicas_per_thread=0, chunk_sweeps=0, use_graph=False,
                 kernel="auto"):
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h for c in self.contexts])
        o = _BatchOpts(int(replicas_per_wg), int(replicas_per_thread), int(chunk_sweeps), 1 if use_graph else 0,
                       KERNELS[kernel])
        h = C.c_void_p()
        _check(lib().pt_batch_create(arr, len(self.contexts), C.byref(o), C.byref(h)))
        self.h = h

    def sweep(self, n):
        _check(lib().pt_batch_sweep(self.h, int(n)))

    def set_stream(self, stream_ptr):
        _check(lib().pt_batch_set_stream(self.h, C.c_void_p(stream_ptr)))

    def kernel_time(self):
        """(ms, launches) of the chunk-kernel launches since the last call."""
        ms, n = C.c_double(), C.c_uint64()
        _check(lib().pt_batch_kernel_time(self.h, C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)

    def describe(self):
        """The launch plan: one dict per launch group (kernel, sweeper,
        contexts, grid, block, lds)."""
        buf = C.create_string_buffer(4096)
        _check(lib().pt_batch_describe(self.h, buf, len(buf)))
        out = []
        for line in buf.value.decode().splitlines():
            d = dict(kv.split("=", 1) for kv in line.split())
            out.append({k: (int(v) if v.isdigit() else v) for k, v in d.items()})
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().pt_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (pt_serve_*). Problems are Contexts
    with their banks installed; requests are (problem, seed, target, cap)."""

    def __init__(self, mem_budget=0, chunk_sweeps=0, max_active=0, replicas_per_wg=0, replicas_per_thread=0,
                 pipeline=False):
        o = _ServeOpts(int(mem_budget), int(chunk_sweeps), int(max_active), int(replicas_per_wg),
                       int(replicas_per_thread), 1 if pipeline else 0)
        h = C.c_void_p()
        _check(lib().pt_serve_start(C.byref(o), C.byref(h)))
        self.h = h
        self.problems = []
        self._best = {}

    def register(self, ctx):
        """Register a Context as a problem; returns its id. The context must
        stay alive and untouched until the server stops."""
        pid = C.c_int32()
        _check(lib().pt_serve_register(self.h, ctx.h, C.byref(pid)))
        self.problems.append(ctx)
        return int(pid.value)

    def submit(self, problem, seed, sweep_cap, target=None, want_best=True, user_tag=0):
        rq = _Request()
        rq.problem = int(problem)
        rq.has_target = 0 if target is None else 1
        rq.target = 0 if target is None else int(target)
        rq.seed = int(seed)
        rq.sweep_cap = int(sweep_cap)
        rq.user_tag = int(user_tag)
        buf = None
        if want_best:
            buf = np.zeros(self.problems[problem].n, np.int8)
            rq.best_out = buf.ctypes.data
        rid = C.c_uint64()
        _check(lib().pt_serve_submit(self.h, C.byref(rq), C.byref(rid)))
        if buf is not None:
            self._best[int(rid.value)] = buf
        return int(rid.value)

    def poll(self, max_results=256, wait_ms=0):
        """Finished requests as dicts (best_spins included when requested)."""
        arr = (_Result * max_results)()
        n = C.c_int32()
        _check(lib().pt_serve_poll(self.h, arr, int(max_results), int(wait_ms), C.byref(n)))
        out = []
        for k in range(n.value):
            r = arr[k]
            d = {f: getattr(r, f) for f, _ in _Result._fields_}
            d["best_spins"] = self._best.pop(int(r.id), None)
            out.append(d)
        return out

    def stats(self):
        st = _ServeStats()
        _check(lib().pt_serve_stats_get(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServeStats._fields_}

    def clock(self):
        return float(lib().pt_serve_clock(self.h))

    def stop(self):
        if getattr(self, "h", None):
            _check(lib().pt_serve_stop(self.h))
            self.h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
