"""Python binding of hgm (include/hgm.h): argument marshalling only.

Every step of the matching runs in the HIP library ``libhgm.so``; this module
builds the C structures from torch tensors (PyTorch provides device memory and
streams) and calls the C entry points of the same names.  There is no CPU
fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgm.so")

HGM_OK = 0
HGM_E_ARG = -1
HGM_E_CSR = -2
HGM_E_SIZE = -3
HGM_E_ROUND_LIMIT = -4
HGM_E_HIP = -5

HGM_VARIANT_AUTO = 0
HGM_VARIANT_CRCW = 1
HGM_VARIANT_CREW = 2
VARIANTS = {"auto": HGM_VARIANT_AUTO, "crcw": HGM_VARIANT_CRCW, "crew": HGM_VARIANT_CREW}

EXPORTED = ["hgm_workspace_size", "hgm_match", "hgm_batch_workspace_size", "hgm_match_batch",
            "hgm_server_create", "hgm_server_submit", "hgm_server_poll", "hgm_server_info",
            "hgm_server_destroy", "hgm_request_check", "hgm_strerror", "hgm_version",
            "hgm_source_digest", "hgm_match_noalloc", "hgm_noalloc_max_bytes",
            "hgm_solo_lds_vertices", "hgm_tune_workspace_size", "hgm_tune_batch_workspace_size",
            "hgm_tune", "hgm_tune_batch", "hgm_tuned_opts", "hgm_tuned_batch_opts"]


class HgmTuneReport(ctypes.Structure):
    _fields_ = [("ms_default", ctypes.c_double), ("ms_best", ctypes.c_double),
                ("evaluations", ctypes.c_int32), ("identical", ctypes.c_int32)]


class HgmCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("kappa", ctypes.c_int64),
                ("e_off", ctypes.c_void_p), ("e_pins", ctypes.c_void_p),
                ("v_off", ctypes.c_void_p), ("v_edges", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


class HgmOpts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("hub_threshold", ctypes.c_int32),
                ("rounds_per_sync", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("reseed", ctypes.c_int32),
                ("pairs", ctypes.c_int32), ("solo_max_kappa", ctypes.c_int32),
                ("edge_grid", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("clear_ratio", ctypes.c_int32), ("hot_degree", ctypes.c_int32),
                ("first_batch_pct", ctypes.c_int32), ("tail_pins", ctypes.c_int32),
                ("bin_shift", ctypes.c_int32)]

SCHEDULE_FIELDS = ["hub_threshold", "solo_max_kappa", "edge_grid", "blocks_per_cu",
                   "clear_ratio", "hot_degree", "first_batch_pct", "tail_pins", "bin_shift"]


class HgmBatch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n_total", ctypes.c_int64), ("m_total", ctypes.c_int64),
                ("kappa_total", ctypes.c_int64), ("words_total", ctypes.c_int64),
                ("v_base", ctypes.c_void_p), ("e_base", ctypes.c_void_p),
                ("pin_base", ctypes.c_void_p), ("word_base", ctypes.c_void_p),
                ("e_off", ctypes.c_void_p), ("e_pins", ctypes.c_void_p),
                ("v_off", ctypes.c_void_p), ("v_edges", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("seeds", ctypes.c_void_p)]


class HgmRequest(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("kappa", ctypes.c_int64), ("e_off", ctypes.c_void_p), ("e_pins", ctypes.c_void_p),
                ("v_off", ctypes.c_void_p), ("v_edges", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("seed", ctypes.c_uint32), ("bits_out", ctypes.c_void_p)]


class HgmResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("wave_size", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class HgmServerOpts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("match", HgmOpts),
                ("edge_side_only", ctypes.c_int32)]


class HgmServerState(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("submitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("arena_bytes", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64),
                ("stalls", ctypes.c_int64), ("stall_s", ctypes.c_double)]


(HGM_K_SETUP, HGM_K_SCATTER, HGM_K_VERTEX_MAX, HGM_K_TEST, HGM_K_RETIRE, HGM_K_SOLO,
 HGM_K_TAIL) = range(7)
HGM_K_CLASSES = 7
KERNEL_CLASS_NAMES = ["setup", "scatter", "vertex_max", "test", "retire", "solo", "tail"]


class HgmStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("matched", ctypes.c_int64),
                ("weight", ctypes.c_uint64), ("live_edges", ctypes.c_void_p),
                ("live_pins", ctypes.c_void_p), ("matched_per_round", ctypes.c_void_p),
                ("matched_pins", ctypes.c_void_p), ("cap", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("round_ms", ctypes.c_void_p),
                ("kernel_ms", ctypes.c_double * HGM_K_CLASSES),
                ("kernel_launches", ctypes.c_int32 * HGM_K_CLASSES)]


class HgmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {hgm_strerror(code)} (code {code})")
        self.code = code


_lib = None


def load():
    """Load libhgm.so; raises if it has not been built, or if it was built
    from other sources than the ones beside it (a stale build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "paper_2602_22976_amd.build.build() (hipcc, gfx950)")
    from . import build as _build
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.hgm_source_digest.restype = ctypes.c_char_p
    lib.hgm_source_digest.argtypes = []
    built, want = lib.hgm_source_digest().decode(), _build.source_digest()
    if built != want:
        raise RuntimeError(f"{LIB_PATH} was built from other sources (digest {built}, sources "
                           f"{want}): rebuild it with paper_2602_22976_amd.build.build()")
    lib.hgm_workspace_size.restype = ctypes.c_size_t
    lib.hgm_workspace_size.argtypes = [ctypes.POINTER(HgmCsr), ctypes.POINTER(HgmOpts)]
    lib.hgm_match.restype = ctypes.c_int
    lib.hgm_match.argtypes = [ctypes.POINTER(HgmCsr), ctypes.c_uint32, P, P, ctypes.c_size_t,
                              ctypes.POINTER(HgmOpts), P, ctypes.POINTER(HgmStats)]
    lib.hgm_match_noalloc.restype = ctypes.c_int
    lib.hgm_match_noalloc.argtypes = [ctypes.POINTER(HgmCsr), ctypes.c_uint32, P,
                                      ctypes.POINTER(HgmOpts), P, ctypes.POINTER(HgmStats)]
    lib.hgm_noalloc_max_bytes.restype = ctypes.c_size_t
    lib.hgm_noalloc_max_bytes.argtypes = []
    lib.hgm_tune_workspace_size.restype = ctypes.c_size_t
    lib.hgm_tune_workspace_size.argtypes = [ctypes.POINTER(HgmCsr), ctypes.POINTER(HgmOpts)]
    lib.hgm_tune_batch_workspace_size.restype = ctypes.c_size_t
    lib.hgm_tune_batch_workspace_size.argtypes = [ctypes.POINTER(HgmBatch),
                                                  ctypes.POINTER(HgmOpts)]
    lib.hgm_tune.restype = ctypes.c_int
    lib.hgm_tune.argtypes = [ctypes.POINTER(HgmCsr), ctypes.c_uint32, P, P, ctypes.c_size_t,
                             ctypes.POINTER(HgmOpts), P, ctypes.c_int32, ctypes.c_char_p,
                             ctypes.POINTER(HgmOpts), ctypes.POINTER(HgmTuneReport)]
    lib.hgm_tune_batch.restype = ctypes.c_int
    lib.hgm_tune_batch.argtypes = [ctypes.POINTER(HgmBatch), P, P, ctypes.c_size_t,
                                   ctypes.POINTER(HgmOpts), P, ctypes.c_int32, ctypes.c_char_p,
                                   ctypes.POINTER(HgmOpts), ctypes.POINTER(HgmTuneReport)]
    lib.hgm_tuned_opts.restype = ctypes.c_int
    lib.hgm_tuned_opts.argtypes = [ctypes.c_char_p, ctypes.POINTER(HgmCsr),
                                   ctypes.POINTER(HgmOpts)]
    lib.hgm_tuned_batch_opts.restype = ctypes.c_int
    lib.hgm_tuned_batch_opts.argtypes = [ctypes.c_char_p, ctypes.POINTER(HgmBatch),
                                         ctypes.POINTER(HgmOpts)]
    lib.hgm_solo_lds_vertices.restype = ctypes.c_int
    lib.hgm_solo_lds_vertices.argtypes = []
    lib.hgm_batch_workspace_size.restype = ctypes.c_size_t
    lib.hgm_batch_workspace_size.argtypes = [ctypes.POINTER(HgmBatch), ctypes.POINTER(HgmOpts)]
    lib.hgm_match_batch.restype = ctypes.c_int
    lib.hgm_match_batch.argtypes = [ctypes.POINTER(HgmBatch), P, P, ctypes.c_size_t,
                                    ctypes.POINTER(HgmOpts), P, ctypes.POINTER(HgmStats)]
    lib.hgm_server_create.restype = ctypes.c_int
    lib.hgm_server_create.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(HgmServerOpts),
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.hgm_server_submit.restype = ctypes.c_int
    lib.hgm_server_submit.argtypes = [P, ctypes.POINTER(HgmRequest)]
    lib.hgm_server_poll.restype = ctypes.c_int
    lib.hgm_server_poll.argtypes = [P, ctypes.POINTER(HgmResult), ctypes.c_int, ctypes.c_double]
    lib.hgm_server_info.restype = ctypes.c_int
    lib.hgm_server_info.argtypes = [P, ctypes.POINTER(HgmServerState)]
    lib.hgm_server_destroy.restype = ctypes.c_int
    lib.hgm_server_destroy.argtypes = [P]
    lib.hgm_request_check.restype = ctypes.c_int
    lib.hgm_request_check.argtypes = [ctypes.POINTER(HgmRequest), ctypes.c_int32]
    lib.hgm_strerror.restype = ctypes.c_char_p
    lib.hgm_strerror.argtypes = [ctypes.c_int]
    lib.hgm_version.restype = ctypes.c_int
    lib.hgm_version.argtypes = []
    _lib = lib
    return lib


def hgm_strerror(code: int) -> str:
    return load().hgm_strerror(int(code)).decode()


def hgm_version() -> int:
    return int(load().hgm_version())


def hgm_workspace_size(csr: HgmCsr, opts: HgmOpts | None = None) -> int:
    return int(load().hgm_workspace_size(ctypes.byref(csr),
                                         ctypes.byref(opts) if opts is not None else None))


def hgm_match(csr: HgmCsr, seed: int, bits_ptr: int, ws_ptr: int, ws_bytes: int,
              opts: HgmOpts | None = None, stream: int = 0,
              stats: HgmStats | None = None) -> int:
    """Raw call; returns the HGM_* code."""
    return int(load().hgm_match(ctypes.byref(csr), seed & 0xFFFFFFFF, bits_ptr or None,
                                ws_ptr or None, ws_bytes,
                                ctypes.byref(opts) if opts is not None else None,
                                stream or None,
                                ctypes.byref(stats) if stats is not None else None))


def hgm_match_noalloc(csr: HgmCsr, seed: int, bits_ptr: int, opts: HgmOpts | None = None,
                      stream: int = 0, stats: HgmStats | None = None) -> int:
    """Raw call; returns the HGM_* code."""
    return int(load().hgm_match_noalloc(ctypes.byref(csr), seed & 0xFFFFFFFF, bits_ptr or None,
                                        ctypes.byref(opts) if opts is not None else None,
                                        stream or None,
                                        ctypes.byref(stats) if stats is not None else None))


def hgm_noalloc_max_bytes() -> int:
    return int(load().hgm_noalloc_max_bytes())


def hgm_batch_workspace_size(batch: HgmBatch, opts: HgmOpts | None = None) -> int:
    return int(load().hgm_batch_workspace_size(ctypes.byref(batch),
                                               ctypes.byref(opts) if opts is not None else None))


def hgm_match_batch(batch: HgmBatch, bits_ptr: int, ws_ptr: int, ws_bytes: int,
                    opts: HgmOpts | None = None, stream: int = 0,
                    stats: HgmStats | None = None) -> int:
    """Raw call; returns the HGM_* code."""
    return int(load().hgm_match_batch(ctypes.byref(batch), bits_ptr or None, ws_ptr or None,
                                      ws_bytes, ctypes.byref(opts) if opts is not None else None,
                                      stream or None,
                                      ctypes.byref(stats) if stats is not None else None))


# ---------------------------------------------------------------------------
# torch-facing helpers (marshalling only)

def _torch():
    import torch
    return torch


class DeviceHypergraph:
    """Dual compressed hypergraph resident on a GPU (torch tensors)."""

    def __init__(self, n, m, e_off, e_pins, v_off, v_edges, w):
        self.n, self.m = int(n), int(m)
        self.e_off, self.e_pins, self.v_off, self.v_edges, self.w = e_off, e_pins, v_off, v_edges, w
        self.kappa = int(e_pins.numel())

    @classmethod
    def from_host(cls, g, device="cuda"):
        """Copy a host hypergraph (numpy arrays n, m, e_off, ...) to `device`."""
        torch = _torch()

        def t(a, dt):
            return torch.from_numpy(a.astype(dt, copy=False)).to(device)

        import numpy as np
        return cls(g.n, g.m, t(g.e_off, np.int32), t(g.e_pins, np.int32), t(g.v_off, np.int32),
                   t(g.v_edges, np.int32), t(g.w.view(np.int32), np.int32))

    def csr(self) -> HgmCsr:
        c = HgmCsr()
        c.n, c.m, c.kappa = self.n, self.m, self.kappa
        c.e_off = self.e_off.data_ptr() if self.e_off.numel() else None
        c.e_pins = self.e_pins.data_ptr() if self.e_pins.numel() else None
        c.v_off = self.v_off.data_ptr() if self.v_off.numel() else None
        c.v_edges = self.v_edges.data_ptr() if self.v_edges.numel() else None
        c.w = self.w.data_ptr() if self.w.numel() else None
        return c


class DeviceBatch:
    """Concatenated instances (instance-local ids) resident on a GPU."""

    def __init__(self, count, n_total, m_total, kappa_total, words_total, v_base, e_base,
                 pin_base, word_base, e_off, e_pins, v_off, v_edges, w, seeds):
        self.count = int(count)
        self.n_total, self.m_total = int(n_total), int(m_total)
        self.kappa_total, self.words_total = int(kappa_total), int(words_total)
        self.v_base, self.e_base, self.pin_base, self.word_base = v_base, e_base, pin_base, word_base
        self.e_off, self.e_pins, self.v_off, self.v_edges, self.w, self.seeds = (
            e_off, e_pins, v_off, v_edges, w, seeds)

    @classmethod
    def from_host(cls, b, device="cuda"):
        """Copy a host batch (synth.Batch-like numpy arrays) to `device`."""
        torch = _torch()
        import numpy as np

        def t(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a).astype(dt, copy=False)).to(device)

        return cls(b.count, int(b.v_base[-1]), int(b.e_base[-1]), int(b.pin_base[-1]),
                   int(b.word_base[-1]), t(b.v_base, np.int64), t(b.e_base, np.int64),
                   t(b.pin_base, np.int64), t(b.word_base, np.int64), t(b.e_off, np.int32),
                   t(b.e_pins, np.int32), t(b.v_off, np.int32), t(b.v_edges, np.int32),
                   t(np.asarray(b.w, dtype=np.uint32).view(np.int32), np.int32),
                   t(np.asarray(b.seeds, dtype=np.uint32).view(np.int32), np.int32))

    def c_struct(self) -> HgmBatch:
        c = HgmBatch()
        c.count, c.n_total, c.m_total = self.count, self.n_total, self.m_total
        c.kappa_total, c.words_total = self.kappa_total, self.words_total

        def p(x):
            return x.data_ptr() if x is not None and x.numel() else None

        c.v_base, c.e_base, c.pin_base, c.word_base = (p(self.v_base), p(self.e_base),
                                                       p(self.pin_base), p(self.word_base))
        c.e_off, c.e_pins, c.v_off, c.v_edges = (p(self.e_off), p(self.e_pins), p(self.v_off),
                                                 p(self.v_edges))
        c.w, c.seeds = p(self.w), p(self.seeds)
        return c


def make_opts(variant="auto", hub_threshold=0, rounds_per_sync=0, validate=False,
              max_rounds=0, reseed=False, pairs=False, solo_max_kappa=0, edge_grid=0,
              blocks_per_cu=0, clear_ratio=0, hot_degree=0, first_batch_pct=0,
              tail_pins=0, bin_shift=0) -> HgmOpts:
    o = HgmOpts()
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.hub_threshold = hub_threshold
    o.rounds_per_sync = rounds_per_sync
    o.validate = 1 if validate else 0
    o.max_rounds = max_rounds
    o.reseed = 1 if reseed else 0
    o.pairs = 1 if pairs else 0
    o.solo_max_kappa = solo_max_kappa
    o.edge_grid, o.blocks_per_cu, o.clear_ratio = edge_grid, blocks_per_cu, clear_ratio
    o.hot_degree, o.first_batch_pct = hot_degree, first_batch_pct
    o.tail_pins = tail_pins
    o.bin_shift = bin_shift
    return o


def alloc_batch_workspace(db: DeviceBatch, opts: HgmOpts | None = None):
    torch = _torch()
    nbytes = hgm_batch_workspace_size(db.c_struct(), opts)
    if nbytes == 0:
        raise HgmError(HGM_E_ARG, "hgm_batch_workspace_size")
    return torch.empty(nbytes, dtype=torch.uint8, device=db.e_pins.device)


# Per-round rows the wrappers collect unless a call asks for more (`cap`):
# instances that need more rounds are paths and chains of thousands of edges;
# "rounds" is exact either way, the per-round arrays then stop at the cap.
STATS_CAP = 4096


def _stats_struct(cap, timing):
    import numpy as np
    arrays = [np.zeros(max(cap, 1), dtype=np.int64) for _ in range(4)]
    rms = np.zeros(max(cap, 1), dtype=np.float32)
    st = HgmStats()
    st.cap = cap
    st.live_edges, st.live_pins, st.matched_per_round, st.matched_pins = [
        a.ctypes.data_as(ctypes.c_void_p) for a in arrays]
    st.timing = 1 if timing else 0
    st.round_ms = rms.ctypes.data_as(ctypes.c_void_p)
    return st, arrays, rms


def _stats_dict(st, arrays, rms, timing):
    r = st.rounds
    k = min(r, st.cap)
    d = {"rounds": r, "matched": st.matched, "weight": st.weight,
         "live_edges": arrays[0][:k].copy(), "live_pins": arrays[1][:k].copy(),
         "matched_per_round": arrays[2][:k].copy(), "matched_pins": arrays[3][:k].copy()}
    if timing:
        d["round_ms"] = rms[:k].copy()
        d["kernel_ms"] = {KERNEL_CLASS_NAMES[c]: st.kernel_ms[c] for c in range(HGM_K_CLASSES)}
        d["kernel_launches"] = {KERNEL_CLASS_NAMES[c]: st.kernel_launches[c]
                                for c in range(HGM_K_CLASSES)}
    return d


def match_batch(db: DeviceBatch, opts: HgmOpts | None = None, workspace=None, bits=None,
                stream=None, want_stats=True, cap=None, timing=False):
    """Run hgm_match_batch; returns (bits int32 tensor [words_total], stats or None)."""
    torch = _torch()
    dev = db.e_pins.device
    if workspace is None:
        workspace = alloc_batch_workspace(db, opts)
    if bits is None:
        bits = torch.empty(max(db.words_total, 1), dtype=torch.int32, device=dev)
    st = arrays = rms = None
    if want_stats or timing:
        st, arrays, rms = _stats_struct(min(db.m_total + 1, STATS_CAP) if cap is None else cap,
                                        timing)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = hgm_match_batch(db.c_struct(), bits.data_ptr(), workspace.data_ptr(), workspace.numel(),
                         opts, stream, st)
    if rc != HGM_OK:
        raise HgmError(rc, "hgm_match_batch")
    return bits[:db.words_total], (_stats_dict(st, arrays, rms, timing) if st is not None else None)


def alloc_workspace(dg: DeviceHypergraph, opts: HgmOpts | None = None):
    torch = _torch()
    nbytes = hgm_workspace_size(dg.csr(), opts)
    if nbytes == 0:
        raise HgmError(HGM_E_ARG, "hgm_workspace_size")
    return torch.empty(nbytes, dtype=torch.uint8, device=dg.e_pins.device)


def match(dg: DeviceHypergraph, seed: int, opts: HgmOpts | None = None, workspace=None,
          bits=None, stream=None, want_stats=True, cap=None, timing=False):
    """Run hgm_match; returns (bits int32 tensor [ceil(m/32)], stats dict or None)."""
    torch = _torch()
    import numpy as np
    dev = dg.e_pins.device
    if workspace is None:
        workspace = alloc_workspace(dg, opts)
    words = (dg.m + 31) // 32
    if bits is None:
        bits = torch.empty(max(words, 1), dtype=torch.int32, device=dev)
    st = arrays = rms = None
    if want_stats or timing:
        st, arrays, rms = _stats_struct(min(dg.m + 1, STATS_CAP) if cap is None else cap, timing)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = hgm_match(dg.csr(), seed, bits.data_ptr(), workspace.data_ptr(), workspace.numel(),
                   opts, stream, st)
    if rc != HGM_OK:
        raise HgmError(rc, "hgm_match")
    return bits[:words], (_stats_dict(st, arrays, rms, timing) if st is not None else None)


def opts_dict(o: HgmOpts) -> dict:
    return {f: int(getattr(o, f)) for f in SCHEDULE_FIELDS}


def _enc(path):
    return path.encode() if isinstance(path, str) else path


def tune(dg: DeviceHypergraph, seed: int, opts: HgmOpts | None = None, reps: int = 3,
         cache: str | None = None, stream=None):
    """Run hgm_tune on a device hypergraph; returns (best HgmOpts, report dict)."""
    torch = _torch()
    dev = dg.e_pins.device
    c = dg.csr()
    nbytes = int(load().hgm_tune_workspace_size(ctypes.byref(c),
                                                ctypes.byref(opts) if opts is not None else None))
    if nbytes == 0:
        raise HgmError(HGM_E_ARG, "hgm_tune_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    bits = torch.empty(max((dg.m + 31) // 32, 1), dtype=torch.int32, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    best, rep = HgmOpts(), HgmTuneReport()
    rc = load().hgm_tune(ctypes.byref(c), seed & 0xFFFFFFFF, bits.data_ptr(), ws.data_ptr(),
                         nbytes, ctypes.byref(opts) if opts is not None else None, stream or None,
                         reps, _enc(cache), ctypes.byref(best), ctypes.byref(rep))
    if rc != HGM_OK:
        raise HgmError(rc, "hgm_tune")
    return best, {"ms_default": rep.ms_default, "ms_best": rep.ms_best,
                  "evaluations": rep.evaluations, "identical": bool(rep.identical),
                  "opts": opts_dict(best)}


def tune_batch(db: DeviceBatch, opts: HgmOpts | None = None, reps: int = 3,
               cache: str | None = None, stream=None):
    """Run hgm_tune_batch; returns (best HgmOpts, report dict)."""
    torch = _torch()
    dev = db.e_pins.device
    c = db.c_struct()
    nbytes = int(load().hgm_tune_batch_workspace_size(
        ctypes.byref(c), ctypes.byref(opts) if opts is not None else None))
    if nbytes == 0:
        raise HgmError(HGM_E_ARG, "hgm_tune_batch_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    bits = torch.empty(max(db.words_total, 1), dtype=torch.int32, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    best, rep = HgmOpts(), HgmTuneReport()
    rc = load().hgm_tune_batch(ctypes.byref(c), bits.data_ptr(), ws.data_ptr(), nbytes,
                               ctypes.byref(opts) if opts is not None else None, stream or None,
                               reps, _enc(cache), ctypes.byref(best), ctypes.byref(rep))
    if rc != HGM_OK:
        raise HgmError(rc, "hgm_tune_batch")
    return best, {"ms_default": rep.ms_default, "ms_best": rep.ms_best,
                  "evaluations": rep.evaluations, "identical": bool(rep.identical),
                  "opts": opts_dict(best)}


def tuned_opts(dg: DeviceHypergraph, opts: HgmOpts | None = None, cache: str | None = None):
    """The cached schedule for this instance's bucket, or None."""
    o = HgmOpts() if opts is None else HgmOpts.from_buffer_copy(opts)
    rc = load().hgm_tuned_opts(_enc(cache), ctypes.byref(dg.csr()), ctypes.byref(o))
    return o if rc == HGM_OK else None


def tuned_batch_opts(db: DeviceBatch, opts: HgmOpts | None = None, cache: str | None = None):
    o = HgmOpts() if opts is None else HgmOpts.from_buffer_copy(opts)
    rc = load().hgm_tuned_batch_opts(_enc(cache), ctypes.byref(db.c_struct()), ctypes.byref(o))
    return o if rc == HGM_OK else None


# ---------------------------------------------------------------------------
# Request server (hgm_server_*): marshalling and bookkeeping of host buffers.

def request(g, seed, rid=0, vertex_side=True):
    """An HgmRequest over host hypergraph `g` (numpy arrays); returns
    (request, arrays it points into, output bitmap).  The arrays must stay
    alive while the request is in use."""
    import numpy as np
    arrs = [np.ascontiguousarray(g.e_off, dtype=np.int32),
            np.ascontiguousarray(g.e_pins, dtype=np.int32),
            np.ascontiguousarray(g.v_off, dtype=np.int32) if vertex_side else None,
            np.ascontiguousarray(g.v_edges, dtype=np.int32) if vertex_side else None,
            np.ascontiguousarray(g.w, dtype=np.uint32)]
    out = np.zeros(max((g.m + 31) // 32, 1), dtype=np.uint32)
    q = HgmRequest()
    q.id, q.n, q.m, q.kappa = rid, g.n, g.m, int(arrs[1].size)
    q.e_off, q.e_pins, q.v_off, q.v_edges, q.w = [
        a.ctypes.data_as(ctypes.c_void_p) if a is not None else None for a in arrs]
    q.seed = seed & 0xFFFFFFFF
    q.bits_out = out.ctypes.data_as(ctypes.c_void_p)
    return q, arrs, out


def hgm_request_check(q: HgmRequest, vertex_side: bool = True) -> int:
    """Raw call; returns the HGM_* code of the host-side content check."""
    return int(load().hgm_request_check(ctypes.byref(q), 1 if vertex_side else 0))

class Server:
    """Continuous-batching request server over a torch-allocated device arena.

    submit() takes a host hypergraph (numpy arrays, pinned or not), keeps its
    arrays alive until the result is polled, and returns the request id;
    poll() returns finished results as dicts with the output bitmap."""

    def __init__(self, arena_bytes, workers=2, max_batch=0, opts: HgmOpts | None = None,
                 device="cuda:0", edge_side_only=False):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        so = HgmServerOpts()
        so.workers, so.max_batch = workers, max_batch
        so.edge_side_only = 1 if edge_side_only else 0
        self.edge_side_only = bool(edge_side_only)
        if opts is not None:
            so.match = opts
        h = ctypes.c_void_p()
        rc = load().hgm_server_create(self.arena.data_ptr(), self.arena.numel(),
                                      ctypes.byref(so), ctypes.byref(h))
        if rc != HGM_OK:
            raise HgmError(rc, "hgm_server_create")
        self.h = h
        self.live = {}
        self.next_id = 0

    def submit(self, g, seed, req_id=None):
        """Queue a matching of host hypergraph `g`; returns its id.  A given
        req_id must not belong to a request whose result is not yet polled:
        the server writes each result into buffers kept under its id."""
        rid = self.next_id if req_id is None else int(req_id)
        if rid in self.live:
            raise ValueError(f"request id {rid} is still in flight")
        vside = not self.edge_side_only   # else the vertex side is not sent
        q, arrs, out = request(g, seed, rid, vside)
        self.next_id = max(self.next_id, rid) + 1
        self.live[rid] = (arrs, out, g.m)
        rc = load().hgm_server_submit(self.h, ctypes.byref(q))
        if rc != HGM_OK:
            del self.live[rid]
            raise HgmError(rc, "hgm_server_submit")
        return rid

    def poll(self, cap=256, timeout_s=0.0):
        buf = (HgmResult * cap)()
        k = load().hgm_server_poll(self.h, buf, cap, float(timeout_s))
        if k < 0:
            raise HgmError(k, "hgm_server_poll")
        res = []
        for r in buf[:k]:
            arrs, out, m = self.live.pop(r.id)
            res.append({"id": r.id, "status": r.status, "wave_size": r.wave_size,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "bits": out[:(m + 31) // 32]})
        return res

    def info(self):
        st = HgmServerState()
        rc = load().hgm_server_info(self.h, ctypes.byref(st))
        if rc != HGM_OK:
            raise HgmError(rc, "hgm_server_info")
        return {f: getattr(st, f) for f, _ in HgmServerState._fields_}

    def close(self):
        if self.h:
            load().hgm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
