"""Python binding of the C ABI in ``include/gtap.h`` (argument marshalling only).

Every step of the fork-join runtime runs in the HIP library
``libgtap.so``; this module only converts arguments.  The functions keep the
C names (``gtap_init``, ``gtap_submit``, ``gtap_run``, ``gtap_result``,
``gtap_finalize``, ...).  :class:`Runtime` wraps them for convenience and uses
PyTorch for the two things the runtime borrows from its caller: device memory
(the workspace tensor, k-clique CSR tensors) and the HIP stream.

If ``libgtap.so`` has not been built this module raises on import: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgtap.so")

# ---- status codes, kinds, modes (mirror include/gtap.h) --------------------
GTAP_OK = 0
GTAP_E_INVAL = -1
GTAP_E_NOMEM = -2
GTAP_E_HIP = -3
GTAP_E_STATE = -4
GTAP_E_FULL = -5
GTAP_E_CAPACITY = -6
GTAP_E_PENDING = -7
GTAP_E_TIMEOUT = -8
GTAP_E_NOJOB = -9

GTAP_MODE_THREAD = 0
GTAP_MODE_BLOCK = 1

GTAP_KIND_FIB = 1
GTAP_KIND_NQUEENS = 2
GTAP_KIND_UTS = 3
GTAP_KIND_KCLIQUE = 4
GTAP_KIND_FMM = 5
GTAP_KIND_CILKSORT = 6
GTAP_KIND_KCLIQUE_SPLIT = 7

GTAP_KCLIQUE_ORIENT = 0
GTAP_KCLIQUE_PIVOT = 1

GTAP_FMM_TASKS = 0
GTAP_FMM_LISTS = 1
GTAP_FMM_WORKLIST = 2

GTAP_DAQ_NONE = 0
GTAP_DAQ_BY_KIND = 1
GTAP_DAQ_KCLIQUE = 2
GTAP_DAQ_CILKSORT = 3

# scheduler variants (config.flags): the scheduler comparison of Sec. 6.5
GTAP_FLAG_NO_PRIVATE_STACK = 1
GTAP_FLAG_SCHED_SINGLE = 2
GTAP_FLAG_SCHED_CENTRAL = 4


class gtap_config(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("num_waves", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("num_queues", ctypes.c_int32),
        ("daq_policy", ctypes.c_int32),
        ("daq_bounds", ctypes.c_int32 * 7),
        ("deque_capacity", ctypes.c_uint32),
        ("steal_below", ctypes.c_uint32),
        ("steal_probes", ctypes.c_uint32),
        ("steal_div", ctypes.c_uint32),
        ("small_frames", ctypes.c_uint64),
        ("big_frames", ctypes.c_uint64),
        ("big_frame_ints", ctypes.c_uint32),
        ("max_jobs", ctypes.c_uint32),
        ("timeout_ms", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("workspace_dev", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
    ]


class gtap_fib_args(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gtap_nqueens_args(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gtap_uts_args(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("threshold", ctypes.c_uint64),
                ("max_depth", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gtap_kclique_args(ctypes.Structure):
    _fields_ = [("row_ptr_dev", ctypes.c_void_p), ("col_dev", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("range_leaf", ctypes.c_int32), ("max_outdeg", ctypes.c_int32)]


class gtap_kclique_split_args(ctypes.Structure):
    _fields_ = [("row_ptr_dev", ctypes.c_void_p), ("col_dev", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("range_leaf", ctypes.c_int32), ("max_outdeg", ctypes.c_int32),
                ("threshold", ctypes.c_int32), ("algorithm", ctypes.c_int32)]


class gtap_fmm_args(ctypes.Structure):
    _fields_ = [("x_dev", ctypes.c_void_p), ("y_dev", ctypes.c_void_p), ("z_dev", ctypes.c_void_p),
                ("q_dev", ctypes.c_void_p), ("phi_dev", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("theta_num", ctypes.c_int32), ("theta_den", ctypes.c_int32),
                ("order", ctypes.c_int32), ("traversal", ctypes.c_int32),
                ("m2l_capacity", ctypes.c_uint64), ("p2p_capacity", ctypes.c_uint64)]


class gtap_cilksort_args(ctypes.Structure):
    _fields_ = [("keys_dev", ctypes.c_void_p), ("tmp_dev", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("sort_cutoff", ctypes.c_int32), ("merge_cutoff", ctypes.c_int32)]


class gtap_fmm_result(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n_cells", "n_leaves", "max_level", "m2l_pairs", "p2p_pairs")] + \
               [("m2l_hash", ctypes.c_uint64), ("p2p_hash", ctypes.c_uint64),
                ("p2p_interactions", ctypes.c_int64), ("coincident", ctypes.c_int64)] + \
               [(f, ctypes.c_double) for f in ("tree_ms", "upward_ms", "traversal_ms", "downward_ms",
                                                "sort_ms", "m2l_ms", "p2p_ms")] + \
               [("dtt_rounds", ctypes.c_int64), ("list_retries", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class gtap_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "tasks", "conts", "spawns", "pushed", "push_batches", "popped", "pop_batches",
        "stolen", "steal_batches", "steal_attempts", "iterations", "idle_iterations",
        "small_frames_touched", "big_frames_touched", "depot_spills", "depot_refills",
        "busy_cycles", "idle_cycles", "admitted", "local_pushed", "atomics", "data_bytes")] + [
        ("kernel_ms", ctypes.c_double),
        ("num_waves", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("num_queues", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class gtap_trace_job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("args_bytes", ctypes.c_uint32),
                ("arrival_s", ctypes.c_double), ("args", ctypes.c_uint64 * 4)]


class gtap_trace_result(ctypes.Structure):
    _fields_ = [("result", ctypes.c_int64), ("submit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gtap_tune_space(ctypes.Structure):
    _fields_ = [("num_queues", ctypes.c_int32 * 4), ("daq_policies", ctypes.c_int32 * 4),
                ("waves_per_group", ctypes.c_int32 * 4), ("num_waves", ctypes.c_int32 * 4),
                ("bounds_sets", ctypes.c_int32), ("bounds", (ctypes.c_int32 * 7) * 4),
                ("repeats", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class gtap_tune_report(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("failed", ctypes.c_int32), ("best_ms", ctypes.c_double),
                ("base_ms", ctypes.c_double), ("small_frames_touched", ctypes.c_uint64),
                ("big_frames_touched", ctypes.c_uint64)]


class gtap_litmus_result(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("instances", "mp_reads", "mp_stale", "mp_overlap", "sb_rounds",
                                                "sb_both_new", "sb_a_new_only", "sb_b_new_only", "sb_both_old")] + \
               [("pairs", ctypes.c_int32), ("pairs_on_distinct_xcds", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class gtap_error_report(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("pool", ctypes.c_int32),
                ("capacity", ctypes.c_uint64), ("requested", ctypes.c_uint64),
                ("wave", ctypes.c_int32), ("job", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# ---- library loading --------------------------------------------------------
def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP runtime first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # PyTorch's wheel carries its own HIP runtime.  Loading it first makes the
    # library's libamdhip64 dependency resolve to that already-loaded copy, so
    # the process has one HIP runtime and tensors, streams and this library
    # share it; loading the library first would map a second runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.gtap_config_default.argtypes = [P(gtap_config)]
    lib.gtap_config_default.restype = None
    lib.gtap_workspace_size.argtypes = [P(gtap_config), P(ctypes.c_uint64)]
    lib.gtap_init.argtypes = [P(gtap_config), P(vp)]
    lib.gtap_submit.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_size_t, P(ctypes.c_uint64)]
    lib.gtap_run.argtypes = [vp]
    lib.gtap_kclique_split_buffer_ints.argtypes = [ctypes.c_int32]
    lib.gtap_kclique_split_buffer_ints.restype = ctypes.c_int32
    lib.gtap_result.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_size_t]
    lib.gtap_finalize.argtypes = [vp]
    lib.gtap_stats_get.argtypes = [vp, P(gtap_stats)]
    lib.gtap_last_error.argtypes = [vp, P(gtap_error_report)]
    lib.gtap_status_string.argtypes = [ctypes.c_int32]
    lib.gtap_status_string.restype = ctypes.c_char_p
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    lib.gtap_serve_start.argtypes = [vp, u32, u32, u32]
    lib.gtap_serve_submit.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_size_t, P(u64)]
    lib.gtap_serve_poll.argtypes = [vp, u64, P(ctypes.c_int64), P(u64)]
    lib.gtap_serve_stop.argtypes = [vp, u32]
    lib.gtap_trace_run.argtypes = [vp, P(gtap_trace_job), ctypes.c_size_t, P(gtap_trace_result), u32]
    lib.gtap_trace_run_plain.argtypes = [vp, P(gtap_trace_job), ctypes.c_size_t, P(gtap_trace_result)]
    lib.gtap_autotune.argtypes = [P(gtap_config), P(gtap_trace_job), ctypes.c_size_t, P(gtap_tune_space),
                                  P(gtap_config), P(gtap_tune_report)]
    lib.gtap_probe_atomics.argtypes = [ctypes.c_int32, u32, u32, vp, u64, vp, P(ctypes.c_double),
                                       P(ctypes.c_double)]
    lib.gtap_litmus.argtypes = [ctypes.c_int32, ctypes.c_int32, u32, u32, vp, u64, vp, P(gtap_litmus_result)]
    lib.gtap_run_static.argtypes = [P(gtap_config), P(gtap_trace_job), ctypes.c_size_t, P(ctypes.c_int64),
                                    P(gtap_error_report)]
    for fn in ("gtap_workspace_size", "gtap_init", "gtap_submit", "gtap_run", "gtap_result",
               "gtap_finalize", "gtap_stats_get", "gtap_last_error", "gtap_serve_start",
               "gtap_serve_submit", "gtap_serve_poll", "gtap_serve_stop", "gtap_trace_run",
               "gtap_trace_run_plain", "gtap_autotune", "gtap_probe_atomics",
               "gtap_litmus", "gtap_run_static"):
        getattr(lib, fn).restype = ctypes.c_int
    return lib


_lib = _load()

# Names every test checks the library exports (the declarations of gtap.h).
EXPORTED = ("gtap_config_default", "gtap_workspace_size", "gtap_init", "gtap_submit", "gtap_run",
            "gtap_result", "gtap_finalize", "gtap_stats_get", "gtap_last_error",
            "gtap_status_string", "gtap_serve_start", "gtap_serve_submit", "gtap_serve_poll",
            "gtap_serve_stop", "gtap_trace_run", "gtap_trace_run_plain", "gtap_autotune",
            "gtap_kclique_split_buffer_ints", "gtap_probe_atomics", "gtap_litmus", "gtap_run_static")


class GtapError(RuntimeError):
    def __init__(self, code: int, what: str, report: Optional[dict] = None):
        self.code = code
        self.report = report
        msg = f"{what}: {gtap_status_string(code)} ({code})"
        if report:
            msg += f" report={report}"
        super().__init__(msg)


def gtap_status_string(code: int) -> str:
    return _lib.gtap_status_string(int(code)).decode()


def kclique_split_buffer_ints(max_outdeg: int) -> int:
    """Big-frame buffer ints a split k-clique job needs (0 = out of range)."""
    return int(_lib.gtap_kclique_split_buffer_ints(int(max_outdeg)))


def gtap_config_default() -> gtap_config:
    cfg = gtap_config()
    _lib.gtap_config_default(ctypes.byref(cfg))
    return cfg


def gtap_workspace_size(cfg: gtap_config) -> int:
    out = ctypes.c_uint64(0)
    rc = _lib.gtap_workspace_size(ctypes.byref(cfg), ctypes.byref(out))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_workspace_size")
    return int(out.value)


def gtap_init(cfg: gtap_config) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    rc = _lib.gtap_init(ctypes.byref(cfg), ctypes.byref(ctx))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_init")
    return ctx


def gtap_submit(ctx, kind: int, args: ctypes.Structure) -> int:
    jid = ctypes.c_uint64(0)
    rc = _lib.gtap_submit(ctx, int(kind), ctypes.byref(args), ctypes.sizeof(args), ctypes.byref(jid))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_submit")
    return int(jid.value)


def gtap_last_error(ctx) -> dict:
    rep = gtap_error_report()
    _lib.gtap_last_error(ctx, ctypes.byref(rep))
    return rep.as_dict()


def gtap_run(ctx) -> None:
    rc = _lib.gtap_run(ctx)
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_run", gtap_last_error(ctx))


def gtap_result(ctx, job_id: int) -> int:
    out = ctypes.c_int64(0)
    rc = _lib.gtap_result(ctx, int(job_id), ctypes.byref(out), ctypes.sizeof(out))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_result")
    return int(out.value)


def gtap_stats_get(ctx) -> dict:
    st = gtap_stats()
    rc = _lib.gtap_stats_get(ctx, ctypes.byref(st))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_stats_get")
    return st.as_dict()


def gtap_finalize(ctx) -> None:
    rc = _lib.gtap_finalize(ctx)
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_finalize")


def gtap_serve_start(ctx, max_inflight: int, headroom_small: int, headroom_big: int) -> None:
    rc = _lib.gtap_serve_start(ctx, int(max_inflight), int(headroom_small), int(headroom_big))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_serve_start")


def gtap_serve_submit(ctx, kind: int, args: ctypes.Structure) -> int:
    t = ctypes.c_uint64(0)
    rc = _lib.gtap_serve_submit(ctx, int(kind), ctypes.byref(args), ctypes.sizeof(args), ctypes.byref(t))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_serve_submit")
    return int(t.value)


def gtap_serve_poll(ctx, ticket: int):
    """(result, done_ticks) once the job completed, else None."""
    r, d = ctypes.c_int64(0), ctypes.c_uint64(0)
    rc = _lib.gtap_serve_poll(ctx, int(ticket), ctypes.byref(r), ctypes.byref(d))
    if rc == GTAP_E_PENDING:
        return None
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_serve_poll")
    return int(r.value), int(d.value)


def gtap_serve_stop(ctx, wait_ms: int = 60000) -> None:
    rc = _lib.gtap_serve_stop(ctx, int(wait_ms))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_serve_stop", gtap_last_error(ctx))


def gtap_trace_run(ctx, jobs, results, timeout_ms: int) -> None:
    rc = _lib.gtap_trace_run(ctx, jobs, len(jobs), results, int(timeout_ms))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_trace_run", gtap_last_error(ctx))


def gtap_trace_run_plain(ctx, jobs, results) -> None:
    rc = _lib.gtap_trace_run_plain(ctx, jobs, len(jobs), results)
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_trace_run_plain", gtap_last_error(ctx))


def gtap_autotune(base: "gtap_config", jobs, space: "gtap_tune_space"):
    """(best gtap_config, report dict) over the candidates of `space`."""
    best = gtap_config()
    rep = gtap_tune_report()
    rc = _lib.gtap_autotune(ctypes.byref(base), jobs, len(jobs), ctypes.byref(space), ctypes.byref(best),
                            ctypes.byref(rep))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_autotune")
    return best, {f: getattr(rep, f) for f, _ in rep._fields_}


GTAP_PROBE_DISTINCT = 0
GTAP_PROBE_PER_WAVE = 1
GTAP_PROBE_ONE_WORD = 2
GTAP_STATIC_SCRATCH_BYTES = 256 << 20   # workspace bytes of gtap_run_static (per device)
GTAP_STATIC_MAX_JOBS = 4096


def gtap_probe_atomics(mode: int, blocks: int, iters: int, words_dev_ptr: int, words: int, stream=None):
    """(device-scope RMWs per second, kernel ms) of the atomic-throughput probe."""
    rate, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = _lib.gtap_probe_atomics(int(mode), int(blocks), int(iters), ctypes.c_void_p(int(words_dev_ptr)),
                                 int(words), stream, ctypes.byref(rate), ctypes.byref(ms))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_probe_atomics")
    return rate.value, ms.value


def gtap_litmus(test: int, ordered: bool, pairs: int, rounds: int, buf_dev_ptr: int, buf_bytes: int,
                stream=None) -> dict:
    """Message-passing (test 0) or store-buffering (test 1) litmus counts."""
    out = gtap_litmus_result()
    rc = _lib.gtap_litmus(int(test), int(bool(ordered)), int(pairs), int(rounds), ctypes.c_void_p(int(buf_dev_ptr)),
                          int(buf_bytes), stream, ctypes.byref(out))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_litmus")
    return out.as_dict()


def gtap_run_static(cfg: "gtap_config", jobs) -> list:
    """Results of a batch run in the library's static workspace (no device
    allocation).  jobs: a ctypes array of gtap_trace_job (Runtime.trace)."""
    out = (ctypes.c_int64 * max(1, len(jobs)))()
    rep = gtap_error_report()
    rc = _lib.gtap_run_static(ctypes.byref(cfg), jobs, len(jobs), out, ctypes.byref(rep))
    if rc != GTAP_OK:
        raise GtapError(rc, "gtap_run_static", rep.as_dict() if rep.code else None)
    return list(out[:len(jobs)])


def tune_space(num_queues=(1,), waves_per_group=(4,), num_waves=(0,), bounds=(), daq_policy=0,
               repeats=2, daq_policies=()) -> "gtap_tune_space":
    """Build a gtap_tune_space from Python lists (num_waves 0 = occupancy
    maximum; daq_policy is shorthand for a one-entry daq_policies)."""
    sp = gtap_tune_space()
    pols = list(daq_policies) or ([daq_policy] if daq_policy else [])
    for i, v in enumerate(pols[:4]):
        sp.daq_policies[i] = int(v)
    for i, v in enumerate(list(num_queues)[:4]):
        sp.num_queues[i] = int(v)
    for i, v in enumerate(list(waves_per_group)[:4]):
        sp.waves_per_group[i] = int(v)
    for i, v in enumerate(list(num_waves)[:4]):
        sp.num_waves[i] = -1 if int(v) == 0 else int(v)
    sp.bounds_sets = min(len(bounds), 4)
    for i, bset in enumerate(list(bounds)[:4]):
        full = list(bset) + [1 << 30] * (7 - len(bset))
        for k in range(7):
            sp.bounds[i][k] = int(full[k])
    sp.repeats = int(repeats)
    return sp


def uts_threshold(m: float) -> int:
    """floor(2^64 * m / (m+1)): continue-threshold of a geometric law with mean m."""
    from fractions import Fraction
    f = Fraction(m).limit_denominator(1 << 20)
    return int((Fraction(1 << 64) * f) // (f + 1))


class Runtime:
    """One runtime context on the current device, memory and stream from PyTorch."""

    def __init__(self, **overrides):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the GTaP runtime needs a HIP device")
        self._torch = torch
        cfg = gtap_config_default()
        for key, val in overrides.items():
            if key == "daq_bounds":
                arr = (ctypes.c_int32 * 7)(*(list(val) + [1 << 30] * (7 - len(val))))
                cfg.daq_bounds = arr
            elif hasattr(cfg, key):
                setattr(cfg, key, val)
            else:
                raise TypeError(f"unknown runtime option {key!r}")
        if cfg.stream is None:
            cfg.stream = torch.cuda.current_stream().cuda_stream
        nbytes = gtap_workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        cfg.workspace_dev = self.workspace.data_ptr()
        cfg.workspace_bytes = nbytes
        self.cfg = cfg
        self.ctx = gtap_init(cfg)
        self._keep = []          # device tensors borrowed by pending jobs

    # -- submission -----------------------------------------------------------
    def submit_fib(self, n: int) -> int:
        return gtap_submit(self.ctx, GTAP_KIND_FIB, gtap_fib_args(int(n), 0))

    def submit_nqueens(self, n: int) -> int:
        return gtap_submit(self.ctx, GTAP_KIND_NQUEENS, gtap_nqueens_args(int(n), 0))

    def submit_uts(self, seed: int, threshold: int, max_depth: int) -> int:
        return gtap_submit(self.ctx, GTAP_KIND_UTS,
                           gtap_uts_args(int(seed) & (2**64 - 1), int(threshold), int(max_depth), 0))

    def submit_kclique(self, row_ptr, col, k: int, range_leaf: int = 64,
                       max_outdeg: Optional[int] = None) -> int:
        torch = self._torch
        rp = row_ptr if isinstance(row_ptr, torch.Tensor) else torch.as_tensor(row_ptr)
        cl = col if isinstance(col, torch.Tensor) else torch.as_tensor(col)
        rp = rp.to(device="cuda", dtype=torch.int32).contiguous()
        cl = cl.to(device="cuda", dtype=torch.int32).contiguous()
        if cl.numel() == 0:
            cl = torch.zeros(1, dtype=torch.int32, device="cuda")
        n = rp.numel() - 1
        if max_outdeg is None:
            max_outdeg = int((rp[1:] - rp[:-1]).max().item()) if n > 0 else 0
        self._keep.append((rp, cl))
        return gtap_submit(self.ctx, GTAP_KIND_KCLIQUE,
                           gtap_kclique_args(rp.data_ptr(), cl.data_ptr(), n, int(k),
                                             int(range_leaf), int(max_outdeg)))

    def submit_kclique_split(self, row_ptr, col, k: int, threshold: int = 16,
                             algorithm: int = GTAP_KCLIQUE_ORIENT, range_leaf: int = 64,
                             max_outdeg: Optional[int] = None) -> int:
        """k-clique job with bitset candidate subgraphs and cost-threshold
        splitting (orientation or pivoting); needs a thread-mode runtime with
        waves_per_group 4 and, for k >= 4, big frames of at least
        kclique_split_buffer_ints(max_outdeg) ints."""
        torch = self._torch
        rp = row_ptr if isinstance(row_ptr, torch.Tensor) else torch.as_tensor(row_ptr)
        cl = col if isinstance(col, torch.Tensor) else torch.as_tensor(col)
        rp = rp.to(device="cuda", dtype=torch.int32).contiguous()
        cl = cl.to(device="cuda", dtype=torch.int32).contiguous()
        if cl.numel() == 0:
            cl = torch.zeros(1, dtype=torch.int32, device="cuda")
        n = rp.numel() - 1
        if max_outdeg is None:
            max_outdeg = int((rp[1:] - rp[:-1]).max().item()) if n > 0 else 0
        self._keep.append((rp, cl))
        return gtap_submit(self.ctx, GTAP_KIND_KCLIQUE_SPLIT,
                           gtap_kclique_split_args(rp.data_ptr(), cl.data_ptr(), n, int(k), int(range_leaf),
                                                   int(max_outdeg), int(threshold), int(algorithm)))

    def submit_fmm(self, x, y, z, q, phi, leaf_max: int = 64, theta=(1, 2), order: int = 6,
                   traversal: int = GTAP_FMM_TASKS, m2l_capacity: int = 0, p2p_capacity: int = 0) -> int:
        """FMM job: x, y, z, q, phi are float64 CUDA tensors of n entries, kept
        alive until run() returns; phi receives the potentials.  traversal
        GTAP_FMM_TASKS needs a block-mode runtime, LISTS and WORKLIST a
        thread-mode one."""
        torch = self._torch
        ts = [t.to(device="cuda", dtype=torch.float64).contiguous() for t in (x, y, z, q)]
        if not (phi.is_cuda and phi.dtype == torch.float64 and phi.is_contiguous()):
            raise ValueError("phi must be a contiguous float64 CUDA tensor")
        n = ts[0].numel()
        self._keep.append((*ts, phi))
        return gtap_submit(self.ctx, GTAP_KIND_FMM,
                           gtap_fmm_args(ts[0].data_ptr(), ts[1].data_ptr(), ts[2].data_ptr(), ts[3].data_ptr(),
                                         phi.data_ptr(), n, int(leaf_max), int(theta[0]), int(theta[1]),
                                         int(order), int(traversal), int(m2l_capacity), int(p2p_capacity)))

    def submit_cilksort(self, keys, tmp=None, sort_cutoff: int = 64, merge_cutoff: int = 256) -> int:
        """Cilksort job: keys is a contiguous uint32 (or int32 viewed as
        unsigned) CUDA tensor sorted in place by run(); tmp a scratch tensor of
        the same size (allocated here if not given), both kept alive until
        run() returns.  The job's result is the number of keys."""
        torch = self._torch
        if not (keys.is_cuda and keys.is_contiguous() and keys.element_size() == 4):
            raise ValueError("keys must be a contiguous 32-bit CUDA tensor")
        if tmp is None:
            tmp = torch.empty_like(keys)
        self._keep.append((keys, tmp))
        return gtap_submit(self.ctx, GTAP_KIND_CILKSORT,
                           gtap_cilksort_args(keys.data_ptr(), tmp.data_ptr(), keys.numel(), int(sort_cutoff),
                                              int(merge_cutoff)))

    def fmm_result(self, job_id: int) -> dict:
        r = gtap_fmm_result()
        rc = _lib.gtap_result(self.ctx, job_id, ctypes.byref(r), ctypes.sizeof(r))
        if rc != GTAP_OK:
            raise GtapError(rc, "gtap_result")
        return r.as_dict()

    # -- argument structs (for traces and serving) ----------------------------
    @staticmethod
    def fib_args(n):
        return GTAP_KIND_FIB, gtap_fib_args(int(n), 0)

    @staticmethod
    def nqueens_args(n):
        return GTAP_KIND_NQUEENS, gtap_nqueens_args(int(n), 0)

    @staticmethod
    def uts_args(seed, threshold, max_depth):
        return GTAP_KIND_UTS, gtap_uts_args(int(seed) & (2**64 - 1), int(threshold), int(max_depth), 0)

    def kclique_args(self, row_ptr, col, k, range_leaf=64, max_outdeg=None):
        """row_ptr/col must be int32 CUDA tensors kept alive by the caller."""
        n = row_ptr.numel() - 1
        if max_outdeg is None:
            max_outdeg = int((row_ptr[1:] - row_ptr[:-1]).max().item()) if n > 0 else 0
        return GTAP_KIND_KCLIQUE, gtap_kclique_args(row_ptr.data_ptr(), col.data_ptr(), n, int(k),
                                                    int(range_leaf), int(max_outdeg))

    @staticmethod
    def trace(entries):
        """entries: [(arrival_s, (kind, args_struct)), ...] -> ctypes array of gtap_trace_job."""
        arr = (gtap_trace_job * len(entries))()
        for i, (t, (kind, a)) in enumerate(entries):
            arr[i].kind = kind
            arr[i].args_bytes = ctypes.sizeof(a)
            arr[i].arrival_s = float(t)
            ctypes.memmove(ctypes.addressof(arr[i].args), ctypes.addressof(a), ctypes.sizeof(a))
        return arr

    # -- serving --------------------------------------------------------------
    def serve_start(self, max_inflight=1024, headroom_small=1 << 16, headroom_big=0):
        gtap_serve_start(self.ctx, max_inflight, headroom_small, headroom_big)

    def serve_submit(self, kind, args) -> int:
        return gtap_serve_submit(self.ctx, kind, args)

    def serve_poll(self, ticket):
        return gtap_serve_poll(self.ctx, ticket)

    def serve_stop(self, wait_ms=60000):
        gtap_serve_stop(self.ctx, wait_ms)

    def trace_run(self, jobs, timeout_ms=120000):
        res = (gtap_trace_result * len(jobs))()
        gtap_trace_run(self.ctx, jobs, res, timeout_ms)
        return res

    def autotune(self, jobs, space):
        """Best configuration for the calibration jobs (see gtap_autotune): a
        dict of the tuned gtap_config fields, and the report."""
        best, rep = gtap_autotune(self.cfg, jobs, space)
        keys = ("num_queues", "daq_policy", "waves_per_group", "num_waves", "small_frames", "big_frames")
        out = {k: getattr(best, k) for k in keys}
        out["daq_bounds"] = list(best.daq_bounds)
        return out, rep

    def trace_run_plain(self, jobs):
        res = (gtap_trace_result * len(jobs))()
        gtap_trace_run_plain(self.ctx, jobs, res)
        return res

    # -- execution ------------------------------------------------------------
    def run(self) -> None:
        try:
            gtap_run(self.ctx)
        finally:
            self._keep = []

    def result(self, job_id: int) -> int:
        return gtap_result(self.ctx, job_id)

    def stats(self) -> dict:
        return gtap_stats_get(self.ctx)

    def last_error(self) -> dict:
        return gtap_last_error(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            gtap_finalize(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
