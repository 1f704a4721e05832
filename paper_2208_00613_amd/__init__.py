"""Python binding of the gfx950 memory-efficient IMM library (``include/hbmax.h``).

Argument marshalling only: every step of sampling, encoding and selection runs
in the HIP kernels of ``libhbmax.so``.  PyTorch provides device memory (graph
upload) and the stream.  Importing the package fails loudly if the library has
not been built; there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhbmax.so")

HBM_OK, HBM_EINVAL, HBM_ENOMEM, HBM_EBUDGET, HBM_EDEVICE, HBM_ESTATE = range(6)
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EBUDGET", 4: "EDEVICE", 5: "ESTATE"}
HBM_IC, HBM_LT = 0, 1
HBM_PROB_EDGE, HBM_PROB_WC = 0, 1
ENC = {"NONE": 0, "HUFFMAN": 1, "HOT_BITMAP": 2, "HUFFMAN_HOT_BITMAP": 3, "BITMAX": 4, "AUTO": 5}
ARRAYS = {"IN_PTR": (0, np.int64), "IN_SRC": (1, np.int32), "THRESH": (2, np.uint32), "COUNTS": (3, np.uint32),
          "WARM": (4, np.uint32), "HOT": (5, np.int32), "BITMAP": (6, np.uint64), "RAW_OFF": (7, np.int64),
          "RAW_MEM": (8, np.int32), "LENS": (9, np.uint8), "CODES": (10, np.uint32), "BITOFF": (11, np.int64),
          "PAYLOAD": (12, np.uint32), "ARR_HOT": (13, np.int32), "ARR_OFF": (14, np.int64),
          "ARR_LOW": (15, np.uint16)}
EXPORTED = ["hbm_create", "hbm_destroy", "hbm_last_error", "hbm_set_budget", "hbm_load_graph", "hbm_set_encoding",
            "hbm_sample_rr", "hbm_select_seeds", "hbm_imm", "hbm_get_rr", "hbm_dump_sets", "hbm_get_store_stats",
            "hbm_export", "hbm_version", "hbm_set_tuning", "hbm_set_hot_density", "hbm_profile", "hbm_profile_read", "hbm_imm_batch",
            "hbm_server_create", "hbm_server_destroy", "hbm_server_last_error", "hbm_server_submit",
            "hbm_server_poll", "hbm_server_get_stats", "hbm_autotune", "hbm_select_seeds_noalloc",
            "hbm_get_memory", "hbm_bench_philox", "hbm_set_spill", "hbm_set_implicit_roots",
            "hbm_set_row_containers"]
TUNE = {"IC_TIER1": 0, "IC_T1_BUDGET": 1, "BLOCK_SETS": 2, "LT_PATH": 3, "T2_QUEUE": 4, "T2_SLOTS": 5,
        "LDS_THREADS": 6, "LDS_PER_CU": 7, "SPARSE_COUNTS": 8, "SELECT_GRAPH": 9, "SPILL_SLOTS": 10,
        "LDS_SMALL": 11}
TUNE_COUNT = 12


class HbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class StoreStats(C.Structure):
    _fields_ = [("nsets", C.c_int64), ("members", C.c_int64), ("warmup_sets", C.c_int64), ("encoding", C.c_int32),
                ("nhot", C.c_int32), ("alphabet", C.c_int32), ("max_code_len", C.c_int32),
                ("ustar_enc", C.c_int32), ("escape_bits", C.c_int32), ("escapes", C.c_int64),
                ("payload_bits", C.c_uint64), ("index_bytes", C.c_int64), ("bitmap_bytes", C.c_int64),
                ("raw_bytes", C.c_int64), ("codebook_bytes", C.c_int64), ("store_bytes", C.c_int64),
                ("skewness", C.c_double), ("density", C.c_double), ("narray", C.c_int32),
                ("array_entries", C.c_int64), ("array_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("alg_bytes", C.c_double), ("alg_ops", C.c_double)]


class ImmStats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("theta_round", C.c_int64 * 64), ("cov_round", C.c_uint64 * 64),
                ("lb", C.c_double), ("theta_final", C.c_int64), ("nsets_final", C.c_int64),
                ("coverage", C.c_uint64), ("influence", C.c_double), ("lambda_prime", C.c_double),
                ("lambda_star", C.c_double), ("t_sample_ms", C.c_double), ("t_encode_ms", C.c_double),
                ("t_select_ms", C.c_double), ("t_total_ms", C.c_double), ("store", StoreStats)]

    def as_dict(self):
        r = self.rounds
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("theta_round", "cov_round", "store")}
        d["theta_round"] = list(self.theta_round[:r])
        d["cov_round"] = list(self.cov_round[:r])
        d["store"] = self.store.as_dict()
        return d


class Query(C.Structure):
    _fields_ = [("k", C.c_int32), ("eps", C.c_double), ("l", C.c_double), ("seed", C.c_uint64)]


class ServeInfo(C.Structure):
    _fields_ = [("done", C.c_int32), ("status", C.c_int), ("preemptions", C.c_int32), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double), ("error", C.c_char * 128)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """hbm_allocator: device memory callbacks the library calls on the calling thread."""
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Backs a context's device memory with PyTorch's caching allocator (on the context's
    stream).  ``fail_after`` (for tests) makes the n-th and later requests return NULL until it
    is reset to None."""

    def __init__(self, device: int, stream):
        import torch

        self._torch = torch
        self.device, self.stream = device, stream
        self.fail_after = None
        self.requests = 0
        self.live = {}

        def _alloc(nbytes, _user):
            self.requests += 1
            if self.fail_after is not None and self.requests >= self.fail_after:
                return None
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except RuntimeError:
                return None
            self.live[p] = int(nbytes)
            return p

        def _release(ptr, _user):
            if ptr and self.live.pop(ptr, None) is not None:
                torch.cuda.caching_allocator_delete(ptr)

        self._fa, self._fr = _ALLOC_FN(_alloc), _RELEASE_FN(_release)  # kept alive with the context
        self.struct = Allocator(self._fa, self._fr, None)


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "admitted", "completed", "failed", "preemptions", "steps",
                                         "peak_active", "peak_store_bytes", "active", "queued")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libhbmax.so (built by ``_build.build()``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "hbm_create": ([C.POINTER(P), C.c_int, P, P], C.c_int),
        "hbm_destroy": ([P], None),
        "hbm_last_error": ([P], C.c_char_p),
        "hbm_set_budget": ([P, I64], C.c_int),
        "hbm_load_graph": ([P, I32, I64, P, P, P, C.c_int, C.c_int], C.c_int),
        "hbm_set_encoding": ([P, C.c_int, D, D], C.c_int),
        "hbm_set_hot_density": ([P, D], C.c_int),
        "hbm_set_spill": ([P, I64], C.c_int),
        "hbm_set_implicit_roots": ([P, I32], C.c_int),
        "hbm_set_row_containers": ([P, I32], C.c_int),
        "hbm_sample_rr": ([P, I64, U64], C.c_int),
        "hbm_select_seeds": ([P, I32, P, P, P], C.c_int),
        "hbm_select_seeds_noalloc": ([P, I32, P, P, P], C.c_int),
        "hbm_get_memory": ([P, C.POINTER(I64), C.POINTER(I64), I32], C.c_int),
        "hbm_bench_philox": ([P, I64, I32, C.POINTER(D), C.POINTER(C.c_uint32)], C.c_int),
        "hbm_imm": ([P, I32, D, D, U64, P, P, C.POINTER(ImmStats)], C.c_int),
        "hbm_get_rr": ([P, I64, P, I64, C.POINTER(I64)], C.c_int),
        "hbm_dump_sets": ([P, I64, I64, P, P, I64, C.POINTER(I64)], C.c_int),
        "hbm_get_store_stats": ([P, C.POINTER(StoreStats)], C.c_int),
        "hbm_export": ([P, C.c_int, P, I64, C.POINTER(I64)], C.c_int),
        "hbm_version": ([], C.c_char_p),
        "hbm_set_tuning": ([P, C.c_int, I64], C.c_int),
        "hbm_profile": ([P, I32], C.c_int),
        "hbm_profile_read": ([P, C.POINTER(KernelStat), I32, C.POINTER(I32)], C.c_int),
        "hbm_imm_batch": ([P, I32, C.POINTER(Query), P, P, C.POINTER(ImmStats), P], C.c_int),
        "hbm_server_create": ([C.POINTER(P), P, I64, I32], C.c_int),
        "hbm_server_destroy": ([P], None),
        "hbm_server_last_error": ([P], C.c_char_p),
        "hbm_server_submit": ([P, C.POINTER(Query), C.POINTER(I64)], C.c_int),
        "hbm_server_poll": ([P, I64, I32, P, P, C.POINTER(ImmStats), C.POINTER(ServeInfo)], C.c_int),
        "hbm_server_get_stats": ([P, C.POINTER(ServerStats)], C.c_int),
        "hbm_autotune": ([P, I32, C.POINTER(Query), P, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Context:
    """One hbm_ctx on a HIP device, issuing work on a torch stream.  Device memory comes from
    PyTorch's caching allocator (allocator="torch", the default) or from hipMalloc
    (allocator=None)."""

    def __init__(self, device: int = 0, stream=None, allocator="torch"):
        import torch

        self._torch = torch
        L = lib()
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = C.c_void_p()
        self.allocator = TorchAllocator(device, stream) if allocator == "torch" else None
        ap = C.c_void_p(C.addressof(self.allocator.struct)) if self.allocator else None
        st = L.hbm_create(C.byref(h), device, C.c_void_p(stream.cuda_stream), ap)
        if st != HBM_OK:
            raise HbmError(st, "hbm_create failed")
        self.h = h
        self.n = 0
        self._graph_dev = None

    def close(self):
        if getattr(self, "h", None):
            lib().hbm_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():  # the allocator callbacks cannot run any more: leave it to the OS
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != HBM_OK:
            msg = lib().hbm_last_error(self.h)
            raise HbmError(st, msg.decode() if msg else "")

    # ---------------------------------------------------------------- API (same names as the C ABI)
    def hbm_set_budget(self, nbytes: int):
        self._check(lib().hbm_set_budget(self.h, int(nbytes)))

    def hbm_profile(self, enable: bool):
        self._check(lib().hbm_profile(self.h, 1 if enable else 0))

    def hbm_profile_read(self) -> list:
        cnt = C.c_int32()
        self._check(lib().hbm_profile_read(self.h, None, 0, C.byref(cnt)))
        arr = (KernelStat * max(cnt.value, 1))()
        self._check(lib().hbm_profile_read(self.h, arr, cnt.value, C.byref(cnt)))
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                     alg_bytes=arr[i].alg_bytes, alg_ops=arr[i].alg_ops) for i in range(cnt.value)]

    def hbm_get_memory(self, reset_peak: bool = False):
        now, peak = C.c_int64(), C.c_int64()
        self._check(lib().hbm_get_memory(self.h, C.byref(now), C.byref(peak), 1 if reset_peak else 0))
        return now.value, peak.value

    def hbm_bench_philox(self, calls_per_thread: int, blocks: int):
        ms, chk = C.c_double(), C.c_uint32()
        self._check(lib().hbm_bench_philox(self.h, int(calls_per_thread), int(blocks), C.byref(ms), C.byref(chk)))
        return ms.value, chk.value

    def hbm_set_tuning(self, key: str, value: int):
        self._check(lib().hbm_set_tuning(self.h, TUNE[key], int(value)))

    def hbm_load_graph(self, n, row_ptr, dst, w=None, model="IC", prob="EDGE"):
        """Load a forward CSR given as numpy arrays (copied to the device for the call) or as
        contiguous device tensors of this context's GPU (int64 row_ptr, int32 dst, float32 w)."""
        torch = self._torch
        dev = torch.device("cuda", self.device)

        def on_dev(a, dt_np, dt_t):
            if isinstance(a, torch.Tensor):
                if a.device != dev or a.dtype != dt_t or not a.is_contiguous():
                    raise ValueError(f"device tensor must be contiguous {dt_t} on {dev}")
                return a
            return torch.as_tensor(np.ascontiguousarray(a, dtype=dt_np)).to(dev)

        torch.cuda.current_stream(self.device).synchronize()
        with torch.cuda.stream(self.stream):
            rp = on_dev(row_ptr, np.int64, torch.int64)
            ds = on_dev(dst, np.int32, torch.int32)
            ww = None if w is None else on_dev(w, np.float32, torch.float32)
        self.stream.synchronize()
        m = int(ds.numel())
        mod = HBM_IC if model in ("IC", HBM_IC) else HBM_LT
        pr = HBM_PROB_WC if prob in ("WC", HBM_PROB_WC) else HBM_PROB_EDGE
        st = lib().hbm_load_graph(self.h, int(n), m, C.c_void_p(rp.data_ptr()),
                                  C.c_void_p(ds.data_ptr() if m else 0),
                                  C.c_void_p(ww.data_ptr()) if ww is not None else None, mod, pr)
        self.stream.synchronize()
        del rp, ds, ww
        self._check(st)
        self.n = int(n)

    def load_synth(self, g, model="IC", prob="EDGE"):
        self.hbm_load_graph(g.n, g.row_ptr, g.dst, g.w if prob == "EDGE" else None, model=model, prob=prob)

    def hbm_set_encoding(self, enc="NONE", warmup_frac=0.1, hot_frac=0.01):
        self._check(lib().hbm_set_encoding(self.h, ENC[enc] if isinstance(enc, str) else int(enc),
                                           float(warmup_frac), float(hot_frac)))

    def hbm_set_implicit_roots(self, on: bool):
        self._check(lib().hbm_set_implicit_roots(self.h, 1 if on else 0))

    def hbm_set_row_containers(self, on: bool):
        self._check(lib().hbm_set_row_containers(self.h, 1 if on else 0))

    def hbm_set_spill(self, device_bytes: int):
        self._check(lib().hbm_set_spill(self.h, int(device_bytes)))

    def hbm_set_hot_density(self, min_density: float):
        self._check(lib().hbm_set_hot_density(self.h, float(min_density)))

    def hbm_sample_rr(self, theta: int, seed: int):
        self._check(lib().hbm_sample_rr(self.h, int(theta), int(seed)))

    def hbm_select_seeds(self, k: int):
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        cov = np.zeros(1, dtype=np.uint64)
        self._check(lib().hbm_select_seeds(self.h, int(k), _ptr(seeds), _ptr(gains), _ptr(cov)))
        return seeds, gains, int(cov[0])

    def hbm_select_seeds_noalloc(self, k: int):
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        cov = np.zeros(1, dtype=np.uint64)
        self._check(lib().hbm_select_seeds_noalloc(self.h, int(k), _ptr(seeds), _ptr(gains), _ptr(cov)))
        return seeds, gains, int(cov[0])

    def hbm_imm(self, k: int, eps: float, l: float, seed: int):
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        st = ImmStats()
        self._check(lib().hbm_imm(self.h, int(k), float(eps), float(l), int(seed), _ptr(seeds), _ptr(gains),
                                  C.byref(st)))
        return seeds, gains, st.as_dict()

    def hbm_get_rr(self, j: int) -> np.ndarray:
        ln = C.c_int64()
        st = lib().hbm_get_rr(self.h, int(j), None, 0, C.byref(ln))
        if st not in (HBM_OK, HBM_EINVAL):
            self._check(st)
        buf = np.zeros(max(ln.value, 1), dtype=np.int32)
        self._check(lib().hbm_get_rr(self.h, int(j), _ptr(buf), buf.size, C.byref(ln)))
        return buf[:ln.value]

    def hbm_dump_sets(self, j0: int, j1: int):
        off = np.zeros(j1 - j0 + 1, dtype=np.int64)
        tot = C.c_int64()
        st = lib().hbm_dump_sets(self.h, int(j0), int(j1), _ptr(off), None, 0, C.byref(tot))
        if st not in (HBM_OK, HBM_EINVAL):
            self._check(st)
        mem = np.zeros(max(tot.value, 1), dtype=np.int32)
        self._check(lib().hbm_dump_sets(self.h, int(j0), int(j1), _ptr(off), _ptr(mem), mem.size, C.byref(tot)))
        return off, mem[:tot.value]

    def hbm_get_store_stats(self) -> dict:
        s = StoreStats()
        self._check(lib().hbm_get_store_stats(self.h, C.byref(s)))
        return s.as_dict()

    def hbm_export(self, name: str) -> np.ndarray:
        code, dt = ARRAYS[name]
        nb = C.c_int64()
        st = lib().hbm_export(self.h, code, None, 0, C.byref(nb))
        if st not in (HBM_OK, HBM_EINVAL):
            self._check(st)
        buf = np.zeros(max(nb.value // np.dtype(dt).itemsize, 1), dtype=dt)
        self._check(lib().hbm_export(self.h, code, _ptr(buf), buf.nbytes, C.byref(nb)))
        return buf[:nb.value // np.dtype(dt).itemsize]


def imm_batch(contexts, queries):
    """hbm_imm_batch over Context objects; queries are (k, eps, l, seed) tuples.  Returns a list
    of (seeds, gains, stats) per instance; raises on the first failing instance."""
    L = lib()
    n = len(contexts)
    hs = (C.c_void_p * n)(*[c.h for c in contexts])
    q = (Query * n)(*[Query(int(k), float(e), float(l), int(sd)) for (k, e, l, sd) in queries])
    seeds = [np.zeros(int(k), dtype=np.int32) for (k, _, _, _) in queries]
    gains = [np.zeros(int(k), dtype=np.uint64) for (k, _, _, _) in queries]
    sp = (C.c_void_p * n)(*[s.ctypes.data for s in seeds])
    gp = (C.c_void_p * n)(*[g.ctypes.data for g in gains])
    stats = (ImmStats * n)()
    status = np.zeros(n, dtype=np.int32)
    st = L.hbm_imm_batch(hs, n, q, sp, gp, stats, _ptr(status))
    if st != HBM_OK:
        bad = [i for i in range(n) if status[i] != HBM_OK]
        i = bad[0] if bad else 0
        msg = L.hbm_last_error(contexts[i].h)
        raise HbmError(st, f"instance {i}: " + (msg.decode() if msg else ""))
    return [(seeds[i], gains[i], stats[i].as_dict()) for i in range(n)]


def imm_autotune(contexts, queries):
    """hbm_autotune over Context objects and (k, eps, l, seed) queries: the chosen launch shapes
    (left applied to every context) and the probe time of the chosen setting."""
    L = lib()
    n = len(contexts)
    hs = (C.c_void_p * n)(*[c.h for c in contexts])
    q = (Query * n)(*[Query(int(k), float(e), float(l), int(sd)) for (k, e, l, sd) in queries])
    chosen = np.zeros(TUNE_COUNT, dtype=np.int64)
    best = C.c_double()
    st = L.hbm_autotune(hs, n, q, _ptr(chosen), C.byref(best))
    if st != HBM_OK:
        msg = L.hbm_last_error(contexts[0].h)
        raise HbmError(st, msg.decode() if msg else "")
    return {k: int(chosen[v]) for k, v in TUNE.items()}, best.value


class Server:
    """hbm_server over the graph (and encoding) of a Context."""

    def __init__(self, ctx: Context, store_budget: int, max_active: int = 16):
        h = C.c_void_p()
        st = lib().hbm_server_create(C.byref(h), ctx.h, int(store_budget), int(max_active))
        if st != HBM_OK:
            raise HbmError(st, "hbm_server_create failed")
        self.h = h
        self.ctx = ctx  # keeps the graph alive
        self.k = {}

    def close(self):
        if getattr(self, "h", None):
            lib().hbm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hbm_server_submit(self, k: int, eps: float, l: float, seed: int) -> int:
        t = C.c_int64()
        q = Query(int(k), float(eps), float(l), int(seed))
        st = lib().hbm_server_submit(self.h, C.byref(q), C.byref(t))
        if st != HBM_OK:
            msg = lib().hbm_server_last_error(self.h)
            raise HbmError(st, msg.decode() if msg else "")
        self.k[t.value] = int(k)
        return t.value

    def hbm_server_poll(self, ticket: int, wait: bool = False):
        """None while pending; else a dict with status, seeds, gains, stats and times."""
        k = self.k.get(ticket, 1)
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        st = ImmStats()
        info = ServeInfo()
        rc = lib().hbm_server_poll(self.h, int(ticket), 1 if wait else 0, _ptr(seeds), _ptr(gains), C.byref(st),
                                   C.byref(info))
        if rc != HBM_OK:
            raise HbmError(rc, f"poll of ticket {ticket}")
        if not info.done:
            return None
        self.k.pop(ticket, None)
        out = dict(status=STATUS.get(info.status, info.status), preemptions=info.preemptions,
                   t_submit_ms=info.t_submit_ms, t_admit_ms=info.t_admit_ms, t_done_ms=info.t_done_ms,
                   error=info.error.decode())
        if info.status == HBM_OK:
            out.update(seeds=seeds, gains=gains, stats=st.as_dict())
        return out

    def hbm_server_get_stats(self) -> dict:
        s = ServerStats()
        lib().hbm_server_get_stats(self.h, C.byref(s))
        return s.as_dict()


def version() -> str:
    return lib().hbm_version().decode()
