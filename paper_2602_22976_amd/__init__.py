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

EXPORTED = ["hgm_workspace_size", "hgm_match", "hgm_strerror", "hgm_version"]


class HgmCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("kappa", ctypes.c_int64),
                ("e_off", ctypes.c_void_p), ("e_pins", ctypes.c_void_p),
                ("v_off", ctypes.c_void_p), ("v_edges", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


class HgmOpts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("hub_threshold", ctypes.c_int32),
                ("rounds_per_sync", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32)]


HGM_K_SETUP, HGM_K_SCATTER, HGM_K_VERTEX_MAX, HGM_K_TEST, HGM_K_RETIRE = range(5)
HGM_K_CLASSES = 5
KERNEL_CLASS_NAMES = ["setup", "scatter", "vertex_max", "test", "retire"]


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
    """Load libhgm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "paper_2602_22976_amd.build.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.hgm_workspace_size.restype = ctypes.c_size_t
    lib.hgm_workspace_size.argtypes = [ctypes.POINTER(HgmCsr), ctypes.POINTER(HgmOpts)]
    lib.hgm_match.restype = ctypes.c_int
    lib.hgm_match.argtypes = [ctypes.POINTER(HgmCsr), ctypes.c_uint32, P, P, ctypes.c_size_t,
                              ctypes.POINTER(HgmOpts), P, ctypes.POINTER(HgmStats)]
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


def make_opts(variant="auto", hub_threshold=0, rounds_per_sync=0, validate=False,
              max_rounds=0) -> HgmOpts:
    o = HgmOpts()
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.hub_threshold = hub_threshold
    o.rounds_per_sync = rounds_per_sync
    o.validate = 1 if validate else 0
    o.max_rounds = max_rounds
    return o


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
    st = None
    arrays = None
    if want_stats or timing:
        cap = min(dg.m + 1, 1 << 16) if cap is None else cap
        arrays = [np.zeros(max(cap, 1), dtype=np.int64) for _ in range(4)]
        rms = np.zeros(max(cap, 1), dtype=np.float32)
        st = HgmStats()
        st.cap = cap
        st.live_edges, st.live_pins, st.matched_per_round, st.matched_pins = [
            a.ctypes.data_as(ctypes.c_void_p) for a in arrays]
        st.timing = 1 if timing else 0
        st.round_ms = rms.ctypes.data_as(ctypes.c_void_p)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = hgm_match(dg.csr(), seed, bits.data_ptr(), workspace.data_ptr(), workspace.numel(),
                   opts, stream, st)
    if rc != HGM_OK:
        raise HgmError(rc, "hgm_match")
    stats = None
    if st is not None:
        r = st.rounds
        k = min(r, st.cap)
        stats = {"rounds": r, "matched": st.matched, "weight": st.weight,
                 "live_edges": arrays[0][:k].copy(), "live_pins": arrays[1][:k].copy(),
                 "matched_per_round": arrays[2][:k].copy(),
                 "matched_pins": arrays[3][:k].copy()}
        if timing:
            stats["round_ms"] = rms[:k].copy()
            stats["kernel_ms"] = {KERNEL_CLASS_NAMES[c]: st.kernel_ms[c] for c in range(HGM_K_CLASSES)}
            stats["kernel_launches"] = {KERNEL_CLASS_NAMES[c]: st.kernel_launches[c]
                                        for c in range(HGM_K_CLASSES)}
    return bits[:words], stats
