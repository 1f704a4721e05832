"""Plain CPU oracle of the memory-efficient IMM hot path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``hbm_oracle.c`` (plain C, built with gcc) via
ctypes and returns numpy arrays.  It shares no code with the GPU library.

Functions and the passages they follow:

* ``philox``            Philox4x32-10 keyed counter RNG (Salmon et al. 2011).
* ``Graph``             transposed graph of the RR-set definition (Background,
                        RR set / RRR set definitions) with IC / LT parameters.
* ``Graph.sample``      one RR set per index: IC reverse BFS over live edges,
                        LT reverse walk (Background, IC and LT models; the
                        sampling step of IMM is a randomized BFS).
* ``greedy``            greedy max coverage (Seed Selection paragraph).
* ``imm``               two-phase IMM schedule (Eq. 1 and Tang et al. 2015).
* ``huffman_lengths``   Huffman code lengths (Huffmax encoding section).
* ``encode`` / ``decode_set``  Huffmax and hot-bitmap store (Alg. 1, Eq. 3).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hbm_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libhbm_oracle.so")

IC, LT = 0, 1
PROB_EDGE, PROB_WC = 0, 1
ENC = {"NONE": 0, "HUFFMAN": 1, "HOT_BITMAP": 2, "HUFFMAN_HOT_BITMAP": 3, "BITMAX": 4, "AUTO": 5}
ENC_NAME = {v: k for k, v in ENC.items()}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction of float expressions)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _ImmStats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("theta_round", C.c_int64 * 64), ("cov_round", C.c_uint64 * 64),
                ("lb", C.c_double), ("theta_final", C.c_int64), ("nsets_final", C.c_int64),
                ("coverage", C.c_uint64), ("l_adj", C.c_double), ("eps_prime", C.c_double),
                ("lnC", C.c_double), ("lambda_prime", C.c_double), ("lambda_star", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_graph_new.restype = P
        L.orc_graph_new.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int, C.c_int]
        L.orc_graph_free.argtypes = [P]
        L.orc_graph_in_ptr.restype = C.c_int64
        L.orc_graph_in_ptr.argtypes = [P, C.POINTER(C.c_void_p)]
        L.orc_graph_in_src.restype = C.c_int64
        L.orc_graph_in_src.argtypes = [P, C.POINTER(C.c_void_p)]
        L.orc_root.restype = C.c_int32
        L.orc_root.argtypes = [C.c_int32, C.c_uint64, C.c_uint64]
        L.orc_sample_one.restype = C.c_int64
        L.orc_sample_one.argtypes = [P, C.c_uint64, C.c_int64, P]
        L.orc_store_new.restype = P
        L.orc_store_free.argtypes = [P]
        L.orc_store_reset.argtypes = [P]
        L.orc_store_append_range.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int64]
        L.orc_scratch_new.restype = P
        L.orc_scratch_new.argtypes = [C.c_int32]
        L.orc_scratch_free.argtypes = [P]
        L.orc_bitmax_select.argtypes = [P, C.c_int32, P, P, P, P]
        L.orc_store_nsets.restype = C.c_int64
        L.orc_store_nsets.argtypes = [P]
        L.orc_store_nmem.restype = C.c_int64
        L.orc_store_nmem.argtypes = [P]
        L.orc_store_off.restype = P
        L.orc_store_off.argtypes = [P]
        L.orc_store_mem.restype = P
        L.orc_store_mem.argtypes = [P]
        L.orc_store_extend.restype = C.c_int
        L.orc_store_extend.argtypes = [P, P, C.c_uint64, C.c_int64]
        L.orc_store_set.restype = C.c_int
        L.orc_store_set.argtypes = [P, C.c_int64, P, P]
        L.orc_greedy_sets.restype = C.c_int
        L.orc_greedy_sets.argtypes = [C.c_int64, P, P, C.c_int32, C.c_int32, P, P, P]
        L.orc_greedy.restype = C.c_int
        L.orc_greedy.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.orc_counts.argtypes = [P, C.c_int32, C.c_int64, C.c_int64, P]
        L.orc_characterize.argtypes = [P, C.c_int32, C.c_int64, C.c_int64, P, P]
        L.orc_imm_params.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, P, P, P, P, P]
        L.orc_imm.restype = C.c_int
        L.orc_imm.argtypes = [P, P, C.c_int32, C.c_double, C.c_double, C.c_uint64, P, P, C.POINTER(_ImmStats)]
        L.orc_huffman_lengths.restype = C.c_int
        L.orc_huffman_lengths.argtypes = [C.c_int32, P, P]
        L.orc_canonical_codes.argtypes = [C.c_int32, P, P]
        L.orc_warmup_count.restype = C.c_int64
        L.orc_warmup_count.argtypes = [C.c_double, C.c_int64]
        L.orc_encode.restype = C.c_int
        L.orc_encode.argtypes = [P, C.c_int32, C.c_int, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_int,
                                 C.POINTER(C.c_void_p)]
        for nm in ("orc_encoded_ar_hot", "orc_encoded_ar_off", "orc_encoded_ar_low"):
            getattr(L, nm).restype = P
            getattr(L, nm).argtypes = [P]
        L.orc_encoded_free.argtypes = [P]
        L.orc_encoded_info.argtypes = [P, P]
        for nm in ["warm", "hot", "bitmap", "cold_off", "cold_mem", "lens", "codes", "bitoff", "payload"]:
            f = getattr(L, f"orc_encoded_{nm}")
            f.restype = P
            f.argtypes = [P]
        L.orc_decode_set.restype = C.c_int64
        L.orc_decode_set.argtypes = [P, C.c_int64, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _view(ptr, dtype, count) -> np.ndarray:
    if count == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    buf = (C.c_char * (count * np.dtype(dtype).itemsize)).from_address(ptr)
    return np.frombuffer(buf, dtype=dtype, count=count).copy()


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def root(n: int, seed: int, j: int) -> int:
    return int(lib().orc_root(n, seed, j))


class Graph:
    """Oracle view of a forward CSR graph under a diffusion model."""

    def __init__(self, n, row_ptr, dst, w=None, model="IC", prob="EDGE"):
        self.n = int(n)
        self._row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self._dst = np.ascontiguousarray(dst, dtype=np.int32)
        self._w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        self.model = IC if model in ("IC", IC) else LT
        self.prob = PROB_WC if prob in ("WC", PROB_WC) else PROB_EDGE
        self.m = int(self._dst.shape[0])
        self.h = lib().orc_graph_new(self.n, self.m, _p(self._row_ptr), _p(self._dst),
                                     _p(self._w) if self._w is not None else None, self.model, self.prob)

    @classmethod
    def from_synth(cls, g, model="IC", prob="EDGE"):
        return cls(g.n, g.row_ptr, g.dst, g.w, model=model, prob=prob)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_graph_free(self.h)
            self.h = None

    def in_csr(self):
        p = C.c_void_p()
        cnt = lib().orc_graph_in_ptr(self.h, C.byref(p))
        ptr = _view(p.value, np.int64, cnt)
        cnt = lib().orc_graph_in_src(self.h, C.byref(p))
        src = _view(p.value, np.int32, cnt)
        return ptr, src

    def sample(self, seed: int, j: int) -> np.ndarray:
        buf = np.empty(self.n, dtype=np.int32)
        ln = lib().orc_sample_one(self.h, seed, j, _p(buf))
        return buf[:ln].copy()


class Store:
    """Canonical RR sets 0..nsets-1."""

    def __init__(self):
        self.h = lib().orc_store_new()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_store_free(self.h)
            self.h = None

    @classmethod
    def from_sets(cls, off, mem):
        st = cls()
        off = np.ascontiguousarray(off, dtype=np.int64)
        mem = np.ascontiguousarray(mem, dtype=np.int32)
        lib().orc_store_set(st.h, len(off) - 1, _p(off), _p(mem))
        return st

    def extend(self, g: Graph, seed: int, theta: int):
        lib().orc_store_extend(self.h, g.h, seed, theta)

    def append_range(self, g: Graph, seed: int, j0: int, j1: int, scratch: "Scratch" = None):
        """Append RR sets j0..j1-1 as the next sets (a shard of the index range).  Threads that
        sample one graph at once each pass a Scratch of their own."""
        lib().orc_store_append_range(self.h, g.h, scratch.h if scratch else None, seed, j0, j1)

    @property
    def nsets(self) -> int:
        return int(lib().orc_store_nsets(self.h))

    def arrays(self):
        ns = self.nsets
        off = _view(lib().orc_store_off(self.h), np.int64, ns + 1)
        mem = _view(lib().orc_store_mem(self.h), np.int32, int(off[-1]))
        return off, mem

    def counts(self, n: int, j0: int = 0, j1: int = None) -> np.ndarray:
        j1 = self.nsets if j1 is None else j1
        out = np.zeros(n, dtype=np.uint64)
        lib().orc_counts(self.h, n, j0, j1, _p(out))
        return out

    def characterize(self, n: int, j0: int, j1: int):
        s = C.c_double()
        d = C.c_double()
        lib().orc_characterize(self.h, n, j0, j1, C.byref(s), C.byref(d))
        return s.value, d.value


class Scratch:
    """Sampling scratch for one thread (a visited flag per vertex and a BFS queue)."""

    def __init__(self, n: int):
        self.h = lib().orc_scratch_new(n)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_scratch_free(self.h)
            self.h = None


def sample_store(g: Graph, seed: int, theta: int) -> Store:
    s = Store()
    s.extend(g, seed, theta)
    return s


def greedy_sets(off, mem, n: int, k: int):
    off = np.ascontiguousarray(off, dtype=np.int64)
    mem = np.ascontiguousarray(mem, dtype=np.int32)
    seeds = np.zeros(k, dtype=np.int32)
    gains = np.zeros(k, dtype=np.uint64)
    cov = np.zeros(1, dtype=np.uint64)
    rc = lib().orc_greedy_sets(len(off) - 1, _p(off), _p(mem), n, k, _p(seeds), _p(gains), _p(cov))
    if rc:
        raise ValueError("invalid k")
    return seeds, gains, int(cov[0])


def greedy(store: Store, n: int, k: int):
    seeds = np.zeros(k, dtype=np.int32)
    gains = np.zeros(k, dtype=np.uint64)
    cov = np.zeros(1, dtype=np.uint64)
    rc = lib().orc_greedy(store.h, n, k, _p(seeds), _p(gains), _p(cov))
    if rc:
        raise ValueError("invalid k")
    return seeds, gains, int(cov[0])


def imm_params(n: int, k: int, eps: float, l: float):
    vals = [C.c_double() for _ in range(5)]
    lib().orc_imm_params(n, k, eps, l, *[C.byref(v) for v in vals])
    return dict(zip(["l_adj", "eps_prime", "lnC", "lambda_prime", "lambda_star"], [v.value for v in vals]))


def imm(g: Graph, k: int, eps: float, l: float, seed: int, store: Store = None):
    store = store or Store()
    seeds = np.zeros(k, dtype=np.int32)
    gains = np.zeros(k, dtype=np.uint64)
    st = _ImmStats()
    lib().orc_imm(g.h, store.h, k, eps, l, seed, _p(seeds), _p(gains), C.byref(st))
    r = st.rounds
    stats = dict(rounds=r, theta_round=list(st.theta_round[:r]), cov_round=list(st.cov_round[:r]), lb=st.lb,
                 theta_final=st.theta_final, nsets_final=st.nsets_final, coverage=st.coverage,
                 l_adj=st.l_adj, eps_prime=st.eps_prime, lnC=st.lnC, lambda_prime=st.lambda_prime,
                 lambda_star=st.lambda_star)
    return seeds, gains, stats, store


def huffman_lengths(weights) -> np.ndarray:
    w = np.ascontiguousarray(weights, dtype=np.uint64)
    lens = np.zeros(len(w), dtype=np.uint8)
    lib().orc_huffman_lengths(len(w), _p(w), _p(lens))
    return lens


def canonical_codes(lens) -> np.ndarray:
    lens = np.ascontiguousarray(lens, dtype=np.uint8)
    codes = np.zeros(len(lens), dtype=np.uint32)
    lib().orc_canonical_codes(len(lens), _p(lens), _p(codes))
    return codes


def warmup_count(frac: float, theta: int) -> int:
    return int(lib().orc_warmup_count(frac, theta))


class Encoded:
    """The oracle's encoded store (same layout the GPU library documents)."""

    def __init__(self, store: Store, n: int, enc: str, W: int, hot_frac: float = 0.0, hot_min_density: float = 0.0,
                 implicit_roots: bool = False, containers: bool = False):
        h = C.c_void_p()
        rc = lib().orc_encode(store.h, n, ENC[enc], W, hot_frac, hot_min_density, 1 if implicit_roots else 0,
                              1 if containers else 0, C.byref(h))
        if rc:
            raise ValueError("implicit roots need a sampled store (every set holds its root)")
        self.h = h.value
        info = np.zeros(17, dtype=np.int64)
        lib().orc_encoded_info(self.h, _p(info))
        (self.enc, self.n, self.nsets, self.W, self.nhot, self.nwords, ncold, self.ustar_enc, self.wbits,
         self.payload_bits, npay, self.n_escapes, self.n_coded, self.maxlen, self.nar, self.nchunks,
         nlow) = [int(x) for x in info]
        L = lib()
        self.warm = _view(L.orc_encoded_warm(self.h), np.uint64, n)
        self.hot = _view(L.orc_encoded_hot(self.h), np.int32, self.nhot)
        self.bitmap = _view(L.orc_encoded_bitmap(self.h), np.uint64, self.nwords * self.nhot)
        cold_off = L.orc_encoded_cold_off(self.h)
        self.cold_off = _view(cold_off, np.int64, self.nsets + 1) if cold_off else None
        self.cold_mem = _view(L.orc_encoded_cold_mem(self.h), np.int32, ncold) if cold_off else None
        lens = L.orc_encoded_lens(self.h)
        self.lens = _view(lens, np.uint8, n) if lens else None
        self.codes = _view(L.orc_encoded_codes(self.h), np.uint32, n) if lens else None
        bo = L.orc_encoded_bitoff(self.h)
        self.bitoff = _view(bo, np.int64, self.nsets + 1) if bo else None
        self.payload = _view(L.orc_encoded_payload(self.h), np.uint32, npay) if bo else None
        # array containers: rows in hot order; offsets per (chunk, row); 16-bit set offsets
        self.ar_hot = _view(L.orc_encoded_ar_hot(self.h), np.int32, self.nar) if self.nar else np.zeros(0, np.int32)
        self.ar_off = (_view(L.orc_encoded_ar_off(self.h), np.int64, self.nchunks * (self.nar + 1))
                       if self.nar and self.nchunks else np.zeros(0, np.int64))
        self.ar_low = _view(L.orc_encoded_ar_low(self.h), np.uint16, nlow) if nlow else np.zeros(0, np.uint16)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_encoded_free(self.h)
            self.h = None

    @property
    def enc_name(self) -> str:
        """The encoding in use (AUTO resolves to BITMAX or HUFFMAN)."""
        return ENC_NAME[self.enc]

    def bitmax_select(self, k: int, want_after: bool = False):
        """Alg. 3 on the Bitmax bit matrix: seeds, gains, coverage (and the matrix after the
        k-th subtraction, word-major like ``bitmap``)."""
        seeds = np.zeros(k, dtype=np.int32)
        gains = np.zeros(k, dtype=np.uint64)
        cov = np.zeros(1, dtype=np.uint64)
        after = np.zeros(self.nwords * self.nhot, dtype=np.uint64) if want_after else None
        rc = lib().orc_bitmax_select(self.h, k, _p(seeds), _p(gains), _p(cov), _p(after) if want_after else None)
        if rc:
            raise ValueError("bitmax_select needs a BITMAX store and 1 <= k <= n")
        return (seeds, gains, int(cov[0]), after) if want_after else (seeds, gains, int(cov[0]))

    def decode_set(self, j: int) -> np.ndarray:
        buf = np.empty(self.n, dtype=np.int32)
        ln = lib().orc_decode_set(self.h, j, _p(buf))
        if ln < 0:
            raise ValueError(f"undecodable set {j}")
        return buf[:ln].copy()
