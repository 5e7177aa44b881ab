"""Python binding of the gfx950 Sprintz codec library (``libsprintz.so``).

Argument marshalling only: every step of compression and decompression runs
in the HIP kernels behind the C ABI declared in ``include/sprintz.h``. The
functions named ``sprintz_*`` mirror the C entry points one to one; the
``compress`` / ``decompress`` helpers wrap them for torch tensors on the GPU
(PyTorch supplies device memory and streams, nothing else). There is no CPU
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsprintz.so")

SPZ_OK, SPZ_EINVAL, SPZ_ENOSPC, SPZ_ECORRUPT, SPZ_EUNSUPPORTED, SPZ_EHIP, SPZ_ENOMEM = 0, -1, -2, -3, -4, -5, -6
SPZ_INT8, SPZ_UINT8, SPZ_INT16, SPZ_UINT16 = 1, 2, 3, 4
SPZ_DELTA, SPZ_FIRE = 0, 1
FORECASTERS = {"delta": SPZ_DELTA, "fire": SPZ_FIRE}


class spz_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("forecaster", ctypes.c_uint32), ("seg_rows", ctypes.c_uint32),
                ("hdr_group", ctypes.c_uint32), ("learn_shift", ctypes.c_uint32), ("entropy", ctypes.c_uint32)]


class spz_info(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint64), ("D", ctypes.c_uint32), ("dtype", ctypes.c_uint32),
                ("params", spz_params), ("compressed_size", ctypes.c_uint64),
                ("decompressed_size", ctypes.c_uint64), ("nseg", ctypes.c_uint32), ("w", ctypes.c_uint32)]


class SprintzError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = sprintz_strerror(status) if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")
        self.status = status


_lib = None

#: C entry points and their ctypes signatures (also checked by the CPU tests).
class spz_batch_item(ctypes.Structure):
    _fields_ = [("d_src", ctypes.c_void_p), ("src_size", ctypes.c_size_t),
                ("d_dst", ctypes.c_void_p), ("dst_cap", ctypes.c_size_t)]


class spz_compress_item(ctypes.Structure):
    _fields_ = [("d_src", ctypes.c_void_p), ("rows", ctypes.c_uint64), ("D", ctypes.c_uint32),
                ("dtype", ctypes.c_uint32), ("params", spz_params), ("d_dst", ctypes.c_void_p),
                ("dst_cap", ctypes.c_size_t), ("d_out_size", ctypes.c_void_p), ("d_ws", ctypes.c_void_p),
                ("ws_size", ctypes.c_size_t)]


_SIGNATURES = {
    "spz_params_default": (None, [ctypes.POINTER(spz_params)]),
    "sprintz_compress_bound": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                                 ctypes.POINTER(spz_params)]),
    "sprintz_workspace_size": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                                 ctypes.POINTER(spz_params)]),
    "sprintz_workspace_size_min": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                                     ctypes.POINTER(spz_params)]),
    "sprintz_compress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                        ctypes.POINTER(spz_params), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "sprintz_compress_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                                ctypes.POINTER(spz_params), ctypes.c_void_p, ctypes.c_size_t,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sprintz_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                        ctypes.POINTER(spz_params), ctypes.POINTER(ctypes.c_uint32), ctypes.c_void_p]),
    "sprintz_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(spz_info)]),
    "sprintz_decompress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(spz_info),
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "sprintz_decompress_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(spz_info)]),
    "sprintz_decompress_ws": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(spz_info),
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]),
    "sprintz_batch_create": (ctypes.c_int, [ctypes.POINTER(spz_batch_item), ctypes.POINTER(spz_info),
                                            ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "sprintz_batch_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(spz_batch_item), ctypes.POINTER(spz_info),
                                                       ctypes.c_uint32]),
    "sprintz_batch_create_in": (ctypes.c_int, [ctypes.POINTER(spz_batch_item), ctypes.POINTER(spz_info),
                                               ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                               ctypes.POINTER(ctypes.c_void_p)]),
    "sprintz_batch_decompress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sprintz_batch_destroy": (None, [ctypes.c_void_p]),
    "sprintz_compress_batch_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(spz_compress_item), ctypes.c_uint32]),
    "sprintz_compress_batch_create_in": (ctypes.c_int, [ctypes.POINTER(spz_compress_item), ctypes.c_uint32,
                                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                                        ctypes.POINTER(ctypes.c_void_p)]),
    "sprintz_compress_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sprintz_compress_batch_destroy": (None, [ctypes.c_void_p]),
    "sprintz_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sprintz_format_version": (ctypes.c_int, []),
}


def load(path: str = LIB_PATH):
    """Load ``libsprintz.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1808_02515_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# One-to-one wrappers of the C ABI
# ---------------------------------------------------------------------------
def spz_params_default() -> spz_params:
    p = spz_params()
    load().spz_params_default(ctypes.byref(p))
    return p


def make_params(forecaster: str = "fire", seg_rows: int = 1024, hdr_group: int = 0, learn_shift: int = 1,
                entropy: int = 0) -> spz_params:
    p = spz_params_default()
    p.forecaster = FORECASTERS[forecaster]
    p.seg_rows = seg_rows
    p.hdr_group = hdr_group
    p.learn_shift = learn_shift
    p.entropy = entropy
    return p


def sprintz_compress_bound(rows: int, D: int, dtype: int, p: spz_params) -> int:
    return int(load().sprintz_compress_bound(rows, D, dtype, ctypes.byref(p)))


def sprintz_workspace_size(rows: int, D: int, dtype: int, p: spz_params) -> int:
    return int(load().sprintz_workspace_size(rows, D, dtype, ctypes.byref(p)))


def sprintz_workspace_size_min(rows: int, D: int, dtype: int, p: spz_params) -> int:
    return int(load().sprintz_workspace_size_min(rows, D, dtype, ctypes.byref(p)))


def sprintz_compress(d_src: int, rows: int, D: int, dtype: int, p: spz_params, d_dst: int, dst_cap: int,
                     d_out_size: int, d_ws: int, ws_size: int, d_status: int, stream: int) -> int:
    return int(load().sprintz_compress(d_src, rows, D, dtype, ctypes.byref(p), d_dst, dst_cap, d_out_size, d_ws,
                                       ws_size, d_status, stream))


#: bytes of the static device workspace of sprintz_compress_noalloc
NOALLOC_WORKSPACE_BYTES = 4 << 20


def sprintz_compress_noalloc(d_src: int, rows: int, D: int, dtype: int, p: spz_params, d_dst: int, dst_cap: int,
                             d_out_size: int, d_status: int, stream: int) -> int:
    return int(load().sprintz_compress_noalloc(d_src, rows, D, dtype, ctypes.byref(p), d_dst, dst_cap, d_out_size,
                                               d_status, stream))


def sprintz_autotune(d_src: int, rows: int, D: int, dtype: int, p: spz_params, stream: int) -> int:
    """The library's segment-size autotuner (synchronous); returns seg_rows."""
    out = ctypes.c_uint32(0)
    rc = int(load().sprintz_autotune(d_src, rows, D, dtype, ctypes.byref(p), ctypes.byref(out), stream))
    if rc != SPZ_OK:
        raise SprintzError(rc, "sprintz_autotune")
    return int(out.value)


def sprintz_get_info(h_src: bytes) -> spz_info:
    info = spz_info()
    buf = ctypes.create_string_buffer(bytes(h_src), len(h_src))
    rc = load().sprintz_get_info(buf, len(h_src), ctypes.byref(info))
    if rc != SPZ_OK:
        raise SprintzError(rc, "sprintz_get_info")
    return info


def sprintz_decompress(d_src: int, src_size: int, info: spz_info, d_dst: int, dst_cap: int, d_status: int,
                       stream: int) -> int:
    return int(load().sprintz_decompress(d_src, src_size, ctypes.byref(info), d_dst, dst_cap, d_status, stream))


def sprintz_decompress_workspace_size(info: spz_info) -> int:
    return int(load().sprintz_decompress_workspace_size(ctypes.byref(info)))


def sprintz_decompress_ws(d_src: int, src_size: int, info: spz_info, d_dst: int, dst_cap: int, d_status: int,
                          d_ws: int, ws_size: int, stream: int) -> int:
    return int(load().sprintz_decompress_ws(d_src, src_size, ctypes.byref(info), d_dst, dst_cap, d_status, d_ws,
                                            ws_size, stream))


def sprintz_batch_create(items, infos) -> int:
    """items: sequence of spz_batch_item, infos: sequence of spz_info; returns
    the plan handle (an integer)."""
    n = len(items)
    arr_i = (spz_batch_item * max(n, 1))(*items)
    arr_f = (spz_info * max(n, 1))(*infos)
    h = ctypes.c_void_p()
    rc = load().sprintz_batch_create(arr_i, arr_f, n, ctypes.byref(h))
    if rc != SPZ_OK:
        raise SprintzError(rc, "sprintz_batch_create")
    return h.value


def sprintz_batch_workspace_size(items, infos) -> int:
    n = len(items)
    arr_i = (spz_batch_item * max(n, 1))(*items)
    arr_f = (spz_info * max(n, 1))(*infos)
    return int(load().sprintz_batch_workspace_size(arr_i, arr_f, n))


def sprintz_batch_create_in(items, infos, d_ws: int, ws_size: int, stream: int) -> int:
    n = len(items)
    arr_i = (spz_batch_item * max(n, 1))(*items)
    arr_f = (spz_info * max(n, 1))(*infos)
    h = ctypes.c_void_p()
    rc = load().sprintz_batch_create_in(arr_i, arr_f, n, d_ws, ws_size, stream, ctypes.byref(h))
    if rc != SPZ_OK:
        raise SprintzError(rc, "sprintz_batch_create_in")
    return h.value


def sprintz_batch_decompress(plan: int, d_status: int, stream: int) -> int:
    return int(load().sprintz_batch_decompress(plan, d_status, stream))


def sprintz_batch_destroy(plan: int) -> None:
    load().sprintz_batch_destroy(plan)


def sprintz_compress_batch_workspace_size(items) -> int:
    n = len(items)
    arr = (spz_compress_item * max(n, 1))(*items)
    return int(load().sprintz_compress_batch_workspace_size(arr, n))


def sprintz_compress_batch_create_in(items, d_ws: int, ws_size: int, stream: int) -> int:
    n = len(items)
    arr = (spz_compress_item * max(n, 1))(*items)
    h = ctypes.c_void_p()
    rc = load().sprintz_compress_batch_create_in(arr, n, d_ws, ws_size, stream, ctypes.byref(h))
    if rc != SPZ_OK:
        raise SprintzError(rc, "sprintz_compress_batch_create_in")
    return h.value


def sprintz_compress_batch(plan: int, d_status: int, stream: int) -> int:
    return int(load().sprintz_compress_batch(plan, d_status, stream))


def sprintz_compress_batch_destroy(plan: int) -> None:
    load().sprintz_compress_batch_destroy(plan)


def sprintz_strerror(status: int) -> str:
    return load().sprintz_strerror(status).decode()


def sprintz_format_version() -> int:
    return int(load().sprintz_format_version())


# ---------------------------------------------------------------------------
# torch helpers (device memory and streams only)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    m = {torch.int8: SPZ_INT8, torch.uint8: SPZ_UINT8, torch.int16: SPZ_INT16}
    if hasattr(torch, "uint16"):
        m[torch.uint16] = SPZ_UINT16
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def torch_dtype(code: int):
    torch = _torch()
    return {SPZ_INT8: torch.int8, SPZ_UINT8: torch.uint8, SPZ_INT16: torch.int16,
            SPZ_UINT16: getattr(torch, "uint16", torch.int16)}[code]


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


@dataclass
class Encoder:
    """Reusable device buffers for compressing series of one shape."""
    rows: int
    D: int
    dtype: int
    params: spz_params
    dst: object
    ws: object
    out_size: object
    status: object

    @classmethod
    def create(cls, rows: int, D: int, dtype: int, params: spz_params, device="cuda"):
        torch = _torch()
        cap = sprintz_compress_bound(rows, D, dtype, params)
        if cap == 0:
            raise SprintzError(SPZ_EINVAL, "sprintz_compress_bound")
        wsz = sprintz_workspace_size(rows, D, dtype, params)
        return cls(rows, D, dtype, params, torch.empty(cap, dtype=torch.uint8, device=device),
                   torch.empty(max(wsz, 8), dtype=torch.uint8, device=device),
                   torch.zeros(1, dtype=torch.int64, device=device),
                   torch.zeros(1, dtype=torch.int32, device=device))

    def run(self, x, stream=None):
        """Enqueue compression of x into self.dst (asynchronous)."""
        rc = sprintz_compress(x.data_ptr(), self.rows, self.D, self.dtype, self.params, self.dst.data_ptr(),
                              self.dst.numel(), self.out_size.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                              self.status.data_ptr(), _stream_handle(stream))
        if rc != SPZ_OK:
            raise SprintzError(rc, "sprintz_compress")


def compress(x, forecaster: str = "fire", seg_rows: int = 1024, hdr_group: int = 0, learn_shift: int = 1,
             stream=None, entropy: int = 0):
    """Compress a (rows, D) int8/uint8/int16/uint16 CUDA tensor; returns the
    container as a uint8 CUDA tensor of its exact size (synchronises).
    ``entropy=1`` adds the Huffman stage."""
    torch = _torch()
    if x.dim() == 1:
        x = x.reshape(-1, 1)
    if x.dim() != 2 or not x.is_cuda:
        raise ValueError("expected a 2-D CUDA tensor")
    x = x.contiguous()
    p = make_params(forecaster, seg_rows, hdr_group, learn_shift, entropy)
    enc = Encoder.create(x.shape[0], x.shape[1], dtype_code(x), p, device=x.device)
    enc.run(x, stream)
    torch.cuda.synchronize(x.device)
    if int(enc.status.item()) != 0:
        raise SprintzError(SPZ_EHIP, f"device status {int(enc.status.item())}")
    return enc.dst[: int(enc.out_size.item())].clone()


def info_of(container) -> spz_info:
    head = container[:64].cpu().numpy().tobytes() if hasattr(container, "cpu") else bytes(container[:64])
    return sprintz_get_info(head)


def decompress(container, out=None, stream=None, check: bool = True):
    """Decompress a uint8 CUDA tensor holding a container; returns the
    (rows, D) tensor. With check=True synchronises and raises on a corrupt
    container."""
    torch = _torch()
    info = info_of(container)
    if out is None:
        out = torch.empty((info.rows, info.D), dtype=torch_dtype(info.dtype), device=container.device)
    status = torch.zeros(1, dtype=torch.int32, device=container.device)
    wsz = sprintz_decompress_workspace_size(info)
    if wsz:
        ws = torch.empty(wsz, dtype=torch.uint8, device=container.device)
        if stream is not None:
            ws.record_stream(stream)
        rc = sprintz_decompress_ws(container.data_ptr(), container.numel(), info, out.data_ptr(),
                                   out.numel() * out.element_size(), status.data_ptr(), ws.data_ptr(), wsz,
                                   _stream_handle(stream))
    else:
        rc = sprintz_decompress(container.data_ptr(), container.numel(), info, out.data_ptr(),
                                out.numel() * out.element_size(), status.data_ptr(), _stream_handle(stream))
    if rc != SPZ_OK:
        raise SprintzError(rc, "sprintz_decompress")
    if check:
        torch.cuda.synchronize(container.device)
        if int(status.item()) != 0:
            raise SprintzError(SPZ_ECORRUPT, f"device status {int(status.item())}")
    return out


class BatchDecoder:
    """A decompression plan over many containers: one call decodes them all
    (per-class persistent launches over a device work list of segments).

    containers: uint8 CUDA tensors; outs: matching (rows, D) CUDA tensors
    (allocated here when None). The plan keeps pointers to both: keep them
    alive while it is used."""

    def __init__(self, containers, outs=None, device="cuda"):
        torch = _torch()
        self.containers = list(containers)
        self.infos = [info_of(c) for c in self.containers]
        if outs is None:
            outs = [torch.empty((i.rows, i.D), dtype=torch_dtype(i.dtype), device=device) for i in self.infos]
        self.outs = list(outs)
        items = [spz_batch_item(c.data_ptr(), c.numel(), o.data_ptr(), o.numel() * o.element_size())
                 for c, o in zip(self.containers, self.outs)]
        self.status = torch.zeros(max(len(items), 1), dtype=torch.int32, device=device)
        self.plan = sprintz_batch_create(items, self.infos)

    def run(self, stream=None, status=None):
        """Enqueue the decoding of every container (asynchronous)."""
        st = self.status if status is None else status
        rc = sprintz_batch_decompress(self.plan, st.data_ptr(), _stream_handle(stream))
        if rc != SPZ_OK:
            raise SprintzError(rc, "sprintz_batch_decompress")

    def close(self):
        if getattr(self, "plan", None):
            sprintz_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchEncoder:
    """A compression plan over many (rows, D) CUDA tensors: one call codes
    them all (per-class persistent launches over the series' segments, one
    offset scan per series, one compaction launch). Containers go to
    ``self.dsts`` (each at its bound); ``containers()`` returns them at their
    sizes. The plan keeps pointers to the inputs: keep them alive while it is
    used. With seg_rows 0 the library's autotuner runs once per class
    (dtype, D), on the class's longest series, and its choice
    (``self.tuned``) codes the whole class."""

    def __init__(self, xs, forecaster: str = "fire", seg_rows: int = 1024, learn_shift: int = 1, device="cuda",
                 stream=None):
        torch = _torch()
        self.xs = [x if x.dim() == 2 else x.reshape(-1, 1) for x in xs]
        sh = _stream_handle(stream)
        self.tuned = {}
        if seg_rows == 0:
            longest = {}
            for x in self.xs:
                key = (dtype_code(x), x.shape[1])
                if key not in longest or x.shape[0] > longest[key].shape[0]:
                    longest[key] = x
            for key, x in sorted(longest.items()):
                self.tuned[key] = sprintz_autotune(x.data_ptr(), x.shape[0], x.shape[1], key[0],
                                                   make_params(forecaster, 0, 0, learn_shift), sh)
        self.params = [make_params(forecaster, self.tuned[(dtype_code(x), x.shape[1])] if seg_rows == 0 else seg_rows,
                                   0, learn_shift) for x in self.xs]
        self.dsts = [torch.empty(sprintz_compress_bound(x.shape[0], x.shape[1], dtype_code(x), p), dtype=torch.uint8,
                                 device=device) for x, p in zip(self.xs, self.params)]
        self.out_sizes = torch.zeros(max(len(self.xs), 1), dtype=torch.int64, device=device)
        self.status = torch.zeros(max(len(self.xs), 1), dtype=torch.int32, device=device)
        self.wss = [torch.empty(max(sprintz_workspace_size(x.shape[0], x.shape[1], dtype_code(x), p), 16),
                                dtype=torch.uint8, device=device) for x, p in zip(self.xs, self.params)]
        items = [spz_compress_item(x.data_ptr(), x.shape[0], x.shape[1], dtype_code(x), p, d.data_ptr(), d.numel(),
                                   self.out_sizes.data_ptr() + 8 * k, w.data_ptr(), w.numel())
                 for k, (x, p, d, w) in enumerate(zip(self.xs, self.params, self.dsts, self.wss))]
        wsz = sprintz_compress_batch_workspace_size(items)
        if wsz == 0:
            raise SprintzError(SPZ_EINVAL, "sprintz_compress_batch_workspace_size")
        self.ws = torch.empty(wsz + 256, dtype=torch.uint8, device=device)
        base = (self.ws.data_ptr() + 255) & ~255
        self.plan = sprintz_compress_batch_create_in(items, base, wsz, sh)

    def run(self, stream=None, status=None):
        """Enqueue the compression of every series (asynchronous)."""
        st = self.status if status is None else status
        rc = sprintz_compress_batch(self.plan, st.data_ptr(), _stream_handle(stream))
        if rc != SPZ_OK:
            raise SprintzError(rc, "sprintz_compress_batch")

    def containers(self):
        """The containers as uint8 CUDA tensors of their exact sizes (synchronises)."""
        torch = _torch()
        torch.cuda.synchronize()
        sizes = self.out_sizes.cpu().tolist()
        return [d[: int(n)] for d, n in zip(self.dsts, sizes)]

    def close(self):
        if getattr(self, "plan", None):
            sprintz_compress_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
