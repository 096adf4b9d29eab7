"""Python binding of libmgard_hip.so (MI355X / gfx950 multilevel lossy compressor).

Argument marshalling only: every step runs in the HIP library.  Device
buffers are torch CUDA tensors; work is enqueued on torch's current stream.
The functions carry the C names of include/mgard_hip.h.  Importing this module
does not need a GPU; calling into it does.  If the shared library has not
been built, loading fails with an error naming the build command -- there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgard_hip.so")

MGARD_OK = 0
STATUS = {
    0: "MGARD_OK", -1: "MGARD_ERR_ARG", -2: "MGARD_ERR_SHAPE", -3: "MGARD_ERR_DTYPE", -4: "MGARD_ERR_TOL",
    -5: "MGARD_ERR_NONFINITE", -6: "MGARD_ERR_CAPACITY", -7: "MGARD_ERR_FORMAT", -8: "MGARD_ERR_DEVICE",
    -9: "MGARD_ERR_OOM",
}
F32, F64 = 0, 1
ABS, REL = 0, 1
NORM_LINF, NORM_S = 0, 1
ALLOC = {"plain": 0, "learned": 1, "count": 2}


class MgardError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class mgard_opts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("eb", C.c_uint32), ("alloc", C.c_uint32),
                ("dict_size", C.c_uint32), ("chunk_symbols", C.c_uint32), ("lossless", C.c_uint32),
                ("stream", C.c_void_p), ("model", C.c_void_p), ("norm", C.c_uint32), ("reserved2", C.c_uint32),
                ("s", C.c_double)]


class mgard_info(C.Structure):
    _fields_ = [("tol", C.c_double), ("tau_abs", C.c_double), ("maxabs", C.c_double),
                ("bin_width", C.c_double * 40), ("linf_err", C.c_double),
                ("n_symbols", C.c_uint64), ("n_outliers", C.c_uint64), ("payload_words", C.c_uint64),
                ("out_bytes", C.c_uint64), ("levels", C.c_uint32), ("fallback_used", C.c_uint32)]


class mgard_header(C.Structure):
    _fields_ = [("version", C.c_uint32), ("dtype", C.c_uint32), ("ndim", C.c_uint32), ("eb", C.c_uint32),
                ("alloc", C.c_uint32), ("fallback", C.c_uint32), ("coord_flags", C.c_uint32),
                ("levels", C.c_uint32), ("dict_size", C.c_uint32), ("chunk_symbols", C.c_uint32),
                ("shape", C.c_uint64 * 4), ("tol", C.c_double), ("tau_abs", C.c_double),
                ("maxabs", C.c_double), ("n_symbols", C.c_uint64), ("n_chunks", C.c_uint64),
                ("n_outliers", C.c_uint64), ("payload_words", C.c_uint64), ("total_bytes", C.c_uint64),
                ("norm", C.c_uint32), ("reserved", C.c_uint32), ("s", C.c_double)]


_lib = None


def load_library():
    """Loads libmgard_hip.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python {os.path.join(_HERE, 'build.py')}`")
    lib = C.CDLL(LIB_PATH)
    P, U32, U64, D = C.c_void_p, C.c_uint32, C.c_uint64, C.c_double
    PU64, PD = C.POINTER(C.c_uint64), C.POINTER(C.c_double)
    sig = {
        "mgard_default_opts": (None, [P]),
        "mgard_last_error": (C.c_char_p, []),
        "mgard_version": (C.c_char_p, []),
        "mgard_release_workspace": (C.c_int, []),
        "mgard_compress_bound": (U64, [U32, PU64, P, C.c_int, P]),
        "mgard_compress": (C.c_int, [U32, PU64, P, C.c_int, D, P, P, U64, PU64, P, P]),
        "mgard_decompress": (C.c_int, [P, U64, P, U64, P, P]),
        "mgard_inspect": (C.c_int, [P, U64, P]),
        "mgard_stream_layout": (C.c_int, [U32, PU64, C.POINTER(U32), PU64, U32]),
        "mgard_decompose": (C.c_int, [U32, PU64, P, C.c_int, P, P, P]),
        "mgard_recompose": (C.c_int, [U32, PU64, P, C.c_int, P, P, P]),
        "mgard_quantize": (C.c_int, [U32, PU64, C.c_int, P, PD, U32, P, P, P]),
        "mgard_dequantize": (C.c_int, [U32, PU64, C.c_int, P, P, PD, U32, P, P]),
        "mgard_histogram": (C.c_int, [P, U64, U32, U32, P, P, P]),
        "mgard_huffman_codebook": (C.c_int, [P, U32, P, P, P]),
        "mgard_huffman_encode": (C.c_int, [P, U64, U32, U32, P, P, P, P, U64, PU64, P]),
        "mgard_huffman_encode_noalloc": (C.c_int, [P, U64, U32, U32, P, P, P, P, U64, PU64, P]),
        "mgard_huffman_decode": (C.c_int, [P, U64, P, U64, U32, U32, P, P, P]),
        "mgard_maxabs": (C.c_int, [C.c_int, P, U64, PD, P]),
        "mgard_plain_constant": (C.c_int, [U32, PU64, P, PD, PD, U32]),
        "mgard_l2_norm": (C.c_int, [U32, PU64, P, C.c_int, P, PD, P]),
        "mgard_timing": (C.c_int, [C.c_int]),
        "mgard_timing_report": (C.c_int, [C.c_char_p, U64, PU64]),
        "mgard_autotune": (C.c_int, [U32, PU64, P, C.c_int, P, P]),
        "mgard_batch_bound": (U64, [U32, P, P]),
        "mgard_chunked_bound": (U64, [U32, PU64, P, C.c_int, U64, P]),
        "mgard_compress_chunked": (C.c_int, [U32, PU64, P, C.c_int, D, P, U64, P, U64, PU64, P]),
        "mgard_decompress_chunked": (C.c_int, [P, U64, P, U64, P]),
        "mgard_batch_create": (C.c_int, [U32, P, D, P, U64, PU64, P, P, C.POINTER(P)]),
        "mgard_batch_launch": (C.c_int, [P, P]),
        "mgard_batch_free": (None, [P]),
        "mgard_batch_launches": (U32, [P]),
        "mgard_refactor_bound": (U64, [U32, PU64, P, C.c_int, U32]),
        "mgard_refactor": (C.c_int, [U32, PU64, P, C.c_int, U32, P, P, U64, PU64, P]),
        "mgard_refactor_inspect": (C.c_int, [P, U64, PU64, C.POINTER(U32), C.POINTER(U32), PU64]),
        "mgard_refactor_request": (C.c_int, [P, U64, D, P, P, U32, PD, P]),
        "mgard_refactor_ranges": (C.c_int, [P, U64, P, P, U32, P, P, C.POINTER(U32)]),
        "mgard_reconstruct": (C.c_int, [P, U64, P, U32, P, U64, P]),
        "mgard_lossless_bound": (U64, [U64]),
        "mgard_lossless_encode": (C.c_int, [P, U64, P, U64, PU64, P]),
        "mgard_lossless_decode": (C.c_int, [P, U64, P, U64, PU64, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int):
    if code != MGARD_OK:
        msg = load_library().mgard_last_error().decode(errors="replace")
        raise MgardError(code, msg)


def _torch():
    import torch

    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _shape(shape):
    return (C.c_uint64 * len(shape))(*[int(s) for s in shape])


class _Coords:
    """Keeps host coordinate arrays alive for the duration of a call."""

    def __init__(self, coords, ndim):
        self.arrays = []
        if coords is None:
            self.ptr = None
            return
        if len(coords) != ndim:
            raise ValueError("one coordinate entry per dimension")
        arr = (C.c_void_p * ndim)()
        for d, x in enumerate(coords):
            if x is None:
                arr[d] = None
            else:
                a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
                self.arrays.append(a)
                arr[d] = a.ctypes.data
        self.arr = arr
        self.ptr = C.cast(arr, C.c_void_p)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("float32 or float64 tensor expected")


def make_opts(eb="rel", alloc="plain", dict_size=8192, chunk=1024, stream=None, norm="linf", s=0.0, lossless=False):
    """norm: "linf" (maximum error) or "s" (the s-norm of smoothness s; s = 0 is L2);
    lossless: the zero-suppression stage after the entropy coder."""
    o = mgard_opts()
    load_library().mgard_default_opts(C.byref(o))
    o.lossless = 1 if lossless else 0
    o.eb = REL if eb == "rel" else ABS
    o.alloc = ALLOC[alloc]
    o.dict_size = dict_size
    o.chunk_symbols = chunk
    o.norm = NORM_S if norm == "s" else NORM_LINF
    o.s = float(s)
    if stream is None:
        stream = _torch().cuda.current_stream().cuda_stream
    o.stream = stream
    return o


def mgard_compress_bound(shape, dtype=F32, coords=None, dict_size=8192, chunk=1024):
    lib = load_library()
    cc = _Coords(coords, len(shape))
    o = mgard_opts()
    lib.mgard_default_opts(C.byref(o))
    o.dict_size, o.chunk_symbols = dict_size, chunk
    b = lib.mgard_compress_bound(len(shape), _shape(shape), cc.ptr, dtype, C.byref(o))
    if b == 0:
        _check(-1)
    return int(b)


def mgard_compress(u, tol, coords=None, eb="rel", alloc="plain", dict_size=8192, chunk=1024, out=None, norm="linf",
                   s=0.0, lossless=False):
    """Compresses a CUDA float tensor.  Returns (uint8 CUDA buffer, nbytes, info dict).
    lossless: add the zero-suppression stage (its container when that is smaller)."""
    torch = _torch()
    lib = load_library()
    u = u.contiguous()
    dt = _dtype_code(u)
    shape = tuple(u.shape)
    cc = _Coords(coords, len(shape))
    o = make_opts(eb, alloc, dict_size, chunk, norm=norm, s=s, lossless=lossless)
    bound = mgard_compress_bound(shape, dt, coords, dict_size, chunk)
    if out is None:
        out = torch.empty(bound, dtype=torch.uint8, device=u.device)
    nbytes = C.c_uint64(0)
    info = mgard_info()
    _check(lib.mgard_compress(len(shape), _shape(shape), cc.ptr, dt, float(tol), _ptr(u), _ptr(out),
                              out.numel(), C.byref(nbytes), C.byref(o), C.byref(info)))
    L = info.levels
    d = {
        "tol": info.tol, "tau_abs": info.tau_abs, "maxabs": info.maxabs,
        "bins": [info.bin_width[i] for i in range(L + 1)], "levels": L,
        "n_outliers": info.n_outliers, "payload_words": info.payload_words, "out_bytes": info.out_bytes,
        "fallback_used": info.fallback_used, "linf_err": info.linf_err,
    }
    return out, int(nbytes.value), d


def mgard_decompress(buf, nbytes, out=None):
    """Decompresses a uint8 CUDA buffer; returns the field as a CUDA tensor."""
    torch = _torch()
    lib = load_library()
    if out is None:
        head = buf[: min(int(nbytes), 1 << 16)].cpu().numpy().tobytes()
        if head[:4] == b"MGZS":
            # the lossless stage's container: its stream is needed for the shape
            buf, nbytes = mgard_lossless_decode(buf, nbytes)
            head = buf[: min(int(nbytes), 1 << 16)].cpu().numpy().tobytes()
        hd = mgard_inspect(head)
        shape = tuple(hd["shape"])
        dtype = torch.float32 if hd["dtype"] == 0 else torch.float64
        out = torch.empty(shape, dtype=dtype, device=buf.device)
    o = make_opts()
    h = mgard_header()
    _check(lib.mgard_decompress(_ptr(buf), int(nbytes), _ptr(out), out.numel() * out.element_size(),
                                C.byref(o), C.byref(h)))
    return out


def mgard_compress_chunked(u_host, tol, slab_planes, coords=None, eb="rel", dict_size=8192, chunk=1024, out=None):
    """Out-of-core compression of a CPU tensor (pinned for overlapped copies)
    in slabs of slab_planes planes along dimension 0.  Returns (uint8 CPU
    tensor, nbytes)."""
    torch = _torch()
    lib = load_library()
    if u_host.is_cuda:
        raise ValueError("mgard_compress_chunked takes a host (CPU) tensor")
    u_host = u_host.contiguous()
    dt = _dtype_code(u_host)
    shape = tuple(u_host.shape)
    cc = _Coords(coords, len(shape))
    o = make_opts(eb, "plain", dict_size, chunk)
    bound = lib.mgard_chunked_bound(len(shape), _shape(shape), cc.ptr, dt, int(slab_planes), C.byref(o))
    if bound == 0:
        _check(-1)
    if out is None:
        out = torch.empty(bound, dtype=torch.uint8, pin_memory=True)
    nbytes = C.c_uint64(0)
    _check(lib.mgard_compress_chunked(len(shape), _shape(shape), cc.ptr, dt, float(tol), _ptr(u_host),
                                      int(slab_planes), _ptr(out), out.numel(), C.byref(nbytes), C.byref(o)))
    return out, int(nbytes.value)


def mgard_decompress_chunked(buf_host, nbytes, out=None):
    """Inverse of mgard_compress_chunked; returns a CPU tensor (pinned)."""
    import struct

    torch = _torch()
    lib = load_library()
    head = buf_host[:88].numpy().tobytes()
    if head[:4] != b"MGCK":
        raise MgardError(-7, "not a chunked container")
    ndim, dtc = struct.unpack("<II", head[8:16])
    shape = struct.unpack("<4Q", head[16:48])[:ndim]
    if out is None:
        out = torch.empty(shape, dtype=torch.float32 if dtc == 0 else torch.float64, pin_memory=True)
    o = make_opts()
    _check(lib.mgard_decompress_chunked(_ptr(buf_host), int(nbytes), _ptr(out), out.numel() * out.element_size(),
                                        C.byref(o)))
    return out


def mgard_inspect(host_bytes: bytes):
    lib = load_library()
    h = mgard_header()
    b = C.create_string_buffer(host_bytes, len(host_bytes))
    code = lib.mgard_inspect(b, len(host_bytes), C.byref(h))
    if code == -6:  # needs more bytes for the full header: still report the fixed fields
        pass
    else:
        _check(code)
    return {
        "version": h.version, "dtype": h.dtype, "ndim": h.ndim, "eb": h.eb, "alloc": h.alloc,
        "fallback": h.fallback, "coord_flags": h.coord_flags, "levels": h.levels, "dict_size": h.dict_size,
        "chunk_symbols": h.chunk_symbols, "shape": [h.shape[i] for i in range(h.ndim)], "tol": h.tol,
        "tau_abs": h.tau_abs, "maxabs": h.maxabs, "n_symbols": h.n_symbols, "n_chunks": h.n_chunks,
        "n_outliers": h.n_outliers, "payload_words": h.payload_words, "total_bytes": h.total_bytes,
        "norm": h.norm, "s": h.s, "complete": code == 0,
    }


def mgard_stream_layout(shape):
    lib = load_library()
    L = C.c_uint32(0)
    offs = (C.c_uint64 * 42)()
    _check(lib.mgard_stream_layout(len(shape), _shape(shape), C.byref(L), offs, 42))
    return int(L.value), [int(offs[i]) for i in range(L.value + 2)]


def mgard_decompose(u, coords=None):
    torch = _torch()
    lib = load_library()
    u = u.contiguous()
    cc = _Coords(coords, u.dim())
    out = torch.empty(u.numel(), dtype=u.dtype, device=u.device)
    o = make_opts()
    _check(lib.mgard_decompose(u.dim(), _shape(u.shape), cc.ptr, _dtype_code(u), _ptr(u), _ptr(out), C.byref(o)))
    return out


def mgard_recompose(coeff, shape, coords=None):
    torch = _torch()
    lib = load_library()
    coeff = coeff.contiguous()
    cc = _Coords(coords, len(shape))
    out = torch.empty(tuple(shape), dtype=coeff.dtype, device=coeff.device)
    o = make_opts()
    _check(lib.mgard_recompose(len(shape), _shape(shape), cc.ptr, _dtype_code(coeff), _ptr(coeff), _ptr(out),
                               C.byref(o)))
    return out


def mgard_quantize(coeff, shape, bins, dict_size=8192):
    torch = _torch()
    lib = load_library()
    coeff = coeff.contiguous()
    n = coeff.numel()
    sym = torch.empty(n, dtype=torch.int16, device=coeff.device)
    qside = torch.zeros(n, dtype=torch.int64, device=coeff.device)
    hb = (C.c_double * len(bins))(*bins)
    o = make_opts()
    _check(lib.mgard_quantize(len(shape), _shape(shape), _dtype_code(coeff), _ptr(coeff), hb, dict_size,
                              _ptr(sym), _ptr(qside), C.byref(o)))
    return sym, qside


def mgard_dequantize(sym, qside, shape, bins, dtype, dict_size=8192):
    torch = _torch()
    lib = load_library()
    out = torch.empty(sym.numel(), dtype=dtype, device=sym.device)
    hb = (C.c_double * len(bins))(*bins)
    o = make_opts()
    _check(lib.mgard_dequantize(len(shape), _shape(shape), _dtype_code(out), _ptr(sym), _ptr(qside), hb,
                                dict_size, _ptr(out), C.byref(o)))
    return out


def mgard_histogram(sym, dict_size=8192, chunk=1024):
    torch = _torch()
    lib = load_library()
    n = sym.numel()
    hist = torch.empty(dict_size, dtype=torch.int64, device=sym.device)
    esc = torch.empty(max((n + chunk - 1) // chunk, 1), dtype=torch.int32, device=sym.device)
    o = make_opts()
    _check(lib.mgard_histogram(_ptr(sym), n, dict_size, chunk, _ptr(hist), _ptr(esc), C.byref(o)))
    return hist, esc


def mgard_huffman_codebook(hist, dict_size=8192):
    torch = _torch()
    lib = load_library()
    lens = torch.empty(dict_size, dtype=torch.uint8, device=hist.device)
    codes = torch.empty(dict_size, dtype=torch.int64, device=hist.device)
    o = make_opts()
    _check(lib.mgard_huffman_codebook(_ptr(hist), dict_size, _ptr(lens), _ptr(codes), C.byref(o)))
    return lens, codes


def mgard_huffman_encode(sym, lens, codes, dict_size=8192, chunk=1024):
    torch = _torch()
    lib = load_library()
    n = sym.numel()
    nch = (n + chunk - 1) // chunk
    bits = torch.empty(max(nch, 1), dtype=torch.int32, device=sym.device)
    cap = (n * 64 + 31) // 32 + nch + 1
    payload = torch.empty(cap, dtype=torch.int32, device=sym.device)
    words = C.c_uint64(0)
    o = make_opts()
    _check(lib.mgard_huffman_encode(_ptr(sym), n, dict_size, chunk, _ptr(lens), _ptr(codes), _ptr(bits),
                                    _ptr(payload), cap, C.byref(words), C.byref(o)))
    return bits[:nch], payload[: words.value]


def mgard_huffman_encode_noalloc(sym, lens, codes, chunk_bits, payload, dict_size=8192, chunk=1024, stream=None):
    """mgard_huffman_encode into caller buffers (chunk_bits: int32, >= ceil(n/chunk);
    payload: int32 of any capacity) with the library's fixed scratch: nothing is
    allocated, here or in the library.  Returns the payload length in words."""
    lib = load_library()
    words = C.c_uint64(0)
    o = make_opts(stream=stream)
    _check(lib.mgard_huffman_encode_noalloc(_ptr(sym), sym.numel(), dict_size, chunk, _ptr(lens), _ptr(codes),
                                            _ptr(chunk_bits), _ptr(payload), payload.numel(), C.byref(words),
                                            C.byref(o)))
    return words.value


def mgard_huffman_decode(payload, bits, n, lens, dict_size=8192, chunk=1024):
    torch = _torch()
    lib = load_library()
    sym = torch.empty(n, dtype=torch.int16, device=payload.device)
    o = make_opts()
    _check(lib.mgard_huffman_decode(_ptr(payload), payload.numel(), _ptr(bits), n, dict_size, chunk, _ptr(lens),
                                    _ptr(sym), C.byref(o)))
    return sym


def mgard_maxabs(u):
    lib = load_library()
    m = C.c_double(0)
    o = make_opts()
    _check(lib.mgard_maxabs(_dtype_code(u), _ptr(u), u.numel(), C.byref(m), C.byref(o)))
    return m.value


def mgard_l2_norm(u, coords=None):
    """||u|| = sqrt(u^T M u) of a CUDA float tensor (the L2 norm of its multilinear interpolant)."""
    lib = load_library()
    u = u.contiguous()
    shape = tuple(u.shape)
    cc = _Coords(coords, len(shape))
    v = C.c_double(0)
    o = make_opts()
    _check(lib.mgard_l2_norm(len(shape), _shape(shape), cc.ptr, _dtype_code(u), _ptr(u), C.byref(v), C.byref(o)))
    return v.value


def mgard_plain_constant(shape, coords=None):
    lib = load_library()
    cc = _Coords(coords, len(shape))
    S = C.c_double(0)
    K = (C.c_double * 41)()
    _check(lib.mgard_plain_constant(len(shape), _shape(shape), cc.ptr, C.byref(S), K, 41))
    return S.value, list(K)


def mgard_release_workspace():
    _check(load_library().mgard_release_workspace())


def u16(t):
    """uint16 view (numpy) of an int16 symbol tensor."""
    return t.cpu().numpy().view(np.uint16)


def mgard_timing(enable: bool):
    _check(load_library().mgard_timing(1 if enable else 0))


def mgard_timing_report():
    """{kernel name: (launches, total ms)} recorded since mgard_timing(True)."""
    lib = load_library()
    need = C.c_uint64(0)
    lib.mgard_timing_report(None, 0, C.byref(need))
    buf = C.create_string_buffer(int(need.value) + 1)
    _check(lib.mgard_timing_report(buf, len(buf), C.byref(need)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out


# ------------------------------------------------------------- learned allocation
MLP_NPARAM, MLP_IN, MLP_HID, MLP_CACHE_PER_ROW = 4553, 4, 64, 260


def _learned_sigs(lib):
    P, U32, U64 = C.c_void_p, C.c_uint32, C.c_uint64
    sig = {
        "mgard_model_create": (C.c_int, [P, U64, C.POINTER(C.c_void_p)]),
        "mgard_model_free": (None, [P]),
        "mgard_level_stats": (C.c_int, [U32, C.POINTER(U64), C.c_int, P, C.POINTER(C.c_double), P]),
        "mgard_level_features": (C.c_int, [U32, C.POINTER(U64), C.c_int, P, C.c_double, P, U32, P]),
        "mgard_bin_widths": (C.c_int, [U32, C.POINTER(U64), P, C.c_int, C.c_double, P, C.POINTER(C.c_double),
                                       U32, C.POINTER(C.c_double), P]),
        "mgard_linf_error": (C.c_int, [C.c_int, P, P, U64, C.POINTER(C.c_double), P]),
        "mgard_mlp_forward": (C.c_int, [P, P, U32, P, P, P]),
        "mgard_mlp_backward": (C.c_int, [P, P, P, U32, P, P]),
        "mgard_mlp_mse": (C.c_int, [P, P, U32, P, C.POINTER(C.c_double), P]),
        "mgard_mlp_adam": (C.c_int, [P, P, P, P, U32, C.c_float, C.c_float, C.c_float, C.c_float, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        if f.argtypes is None:
            f.restype = res
            f.argtypes = args
    return lib


class Model:
    """Device copy of the network parameters (mgard_model*)."""

    def __init__(self, params):
        lib = _learned_sigs(load_library())
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != MLP_NPARAM:
            raise ValueError(f"{MLP_NPARAM} parameters expected")
        h = C.c_void_p(0)
        _check(lib.mgard_model_create(p.ctypes.data, p.size, C.byref(h)))
        self.handle = h
        self.params = p

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mgard_model_free(self.handle)
            self.handle = None


def mgard_compress_learned(u, tol, model: Model, coords=None, eb="rel", dict_size=8192, chunk=1024, out=None):
    """Compression with the learned per-level bin widths (plain widths when the check fails)."""
    torch = _torch()
    lib = load_library()
    u = u.contiguous()
    dt = _dtype_code(u)
    shape = tuple(u.shape)
    cc = _Coords(coords, len(shape))
    o = make_opts(eb, "learned", dict_size, chunk)
    o.model = model.handle
    bound = mgard_compress_bound(shape, dt, coords, dict_size, chunk)
    if out is None:
        out = torch.empty(bound, dtype=torch.uint8, device=u.device)
    nbytes = C.c_uint64(0)
    info = mgard_info()
    _check(lib.mgard_compress(len(shape), _shape(shape), cc.ptr, dt, float(tol), _ptr(u), _ptr(out),
                              out.numel(), C.byref(nbytes), C.byref(o), C.byref(info)))
    L = info.levels
    return out, int(nbytes.value), {
        "tau_abs": info.tau_abs, "bins": [info.bin_width[i] for i in range(L + 1)], "levels": L,
        "linf_err": info.linf_err, "fallback_used": info.fallback_used, "out_bytes": info.out_bytes,
        "n_outliers": info.n_outliers,
    }


def mgard_level_stats(coeff, shape):
    lib = _learned_sigs(load_library())
    L, _ = mgard_stream_layout(shape)
    st = (C.c_double * (3 * (L + 1)))()
    o = make_opts()
    _check(lib.mgard_level_stats(len(shape), _shape(shape), _dtype_code(coeff), _ptr(coeff), st, C.byref(o)))
    return np.array(list(st)).reshape(L + 1, 3)


def mgard_level_features(coeff, shape, tau_abs):
    """The network's raw input rows (levels + 1, 4) as the device computes them."""
    lib = _learned_sigs(load_library())
    L, _ = mgard_stream_layout(shape)
    x = (C.c_float * (4 * (L + 1)))()
    o = make_opts()
    _check(lib.mgard_level_features(len(shape), _shape(shape), _dtype_code(coeff), _ptr(coeff), float(tau_abs), x,
                                    L + 1, C.byref(o)))
    return np.array(list(x), dtype=np.float32).reshape(L + 1, 4)


def mgard_bin_widths(u, tol, coords=None, eb="rel", alloc="plain", norm="linf", s=0.0):
    """The a-priori bin widths (plain or count; L-infinity or s-norm) of u under tol, and
    tau_abs, from the device."""
    lib = _learned_sigs(load_library())
    u = u.contiguous()
    shape = tuple(u.shape)
    L, _ = mgard_stream_layout(shape)
    cc = _Coords(coords, len(shape))
    bins = (C.c_double * (L + 1))()
    tau = C.c_double(0)
    o = make_opts(eb, alloc, norm=norm, s=s)
    _check(lib.mgard_bin_widths(len(shape), _shape(shape), cc.ptr, _dtype_code(u), float(tol), _ptr(u), bins, L + 1,
                                C.byref(tau), C.byref(o)))
    return list(bins), tau.value


def mgard_linf_error(a, b):
    lib = _learned_sigs(load_library())
    e = C.c_double(0)
    o = make_opts()
    _check(lib.mgard_linf_error(_dtype_code(a), _ptr(a), _ptr(b), a.numel(), C.byref(e), C.byref(o)))
    return e.value


def mgard_mlp_forward(params, x, cache=True):
    """params: float32 CUDA (MLP_NPARAM); x: float32 CUDA (B, 4) raw features."""
    torch = _torch()
    lib = _learned_sigs(load_library())
    B = x.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=x.device)
    cch = torch.empty(B * MLP_CACHE_PER_ROW, dtype=torch.float32, device=x.device) if cache else None
    o = make_opts()
    _check(lib.mgard_mlp_forward(_ptr(params), _ptr(x.contiguous()), B, _ptr(out), _ptr(cch), C.byref(o)))
    return out, cch


def mgard_mlp_backward(params, cache, dout, batch):
    torch = _torch()
    lib = _learned_sigs(load_library())
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=params.device)
    o = make_opts()
    _check(lib.mgard_mlp_backward(_ptr(params), _ptr(cache), _ptr(dout), batch, _ptr(g), C.byref(o)))
    return g


def mgard_mlp_mse(pred, target):
    torch = _torch()
    lib = _learned_sigs(load_library())
    d = torch.empty_like(pred)
    loss = C.c_double(0)
    o = make_opts()
    _check(lib.mgard_mlp_mse(_ptr(pred), _ptr(target), pred.numel(), _ptr(d), C.byref(loss), C.byref(o)))
    return d, loss.value


def mgard_mlp_adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    lib = _learned_sigs(load_library())
    o = make_opts()
    _check(lib.mgard_mlp_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(step), lr, beta1, beta2, eps,
                              C.byref(o)))


# ---------------------------------------------------------------- batches


class mgard_field(C.Structure):
    _fields_ = [("ndim", C.c_uint32), ("dtype", C.c_uint32), ("shape", C.c_uint64 * 4),
                ("coords", C.c_void_p * 4), ("d_in", C.c_void_p)]


def mgard_autotune(u, coords=None, dict_size=8192, chunk=1024):
    """Runs the launch-shape tuner for the levels of u's shape (see mgard_autotune in the header)."""
    lib = load_library()
    u = u.contiguous()
    cc = _Coords(coords, u.dim())
    o = make_opts(dict_size=dict_size, chunk=chunk)
    _check(lib.mgard_autotune(u.dim(), _shape(u.shape), cc.ptr, _dtype_code(u), _ptr(u), C.byref(o)))


class Batch:
    """A captured batch plan: many fields compressed by one graph launch.

    fields: CUDA float tensors (kept alive by the plan); coords: None or one
    entry per field (None or a per-dimension list).  launch() replays the
    graph on the current stream; results() waits and returns, per field, the
    compressed bytes as a view of the shared output buffer.
    """

    def __init__(self, fields, tol, coords=None, eb="rel", alloc="plain", dict_size=8192, chunk=1024):
        torch = _torch()
        lib = load_library()
        self.fields = [f.contiguous() for f in fields]
        n = len(self.fields)
        arr = (mgard_field * n)()
        self._coords = []
        for i, f in enumerate(self.fields):
            arr[i].ndim = f.dim()
            arr[i].dtype = _dtype_code(f)
            for d in range(f.dim()):
                arr[i].shape[d] = int(f.shape[d])
            cf = coords[i] if coords is not None else None
            if cf is not None:
                for d, x in enumerate(cf):
                    if x is not None:
                        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
                        self._coords.append(a)
                        arr[i].coords[d] = a.ctypes.data
            arr[i].d_in = f.data_ptr()
        self._arr = arr
        o = make_opts(eb, alloc, dict_size, chunk)
        bound = lib.mgard_batch_bound(n, C.cast(arr, C.c_void_p), C.byref(o))
        if bound == 0:
            _check(-1)
        dev = self.fields[0].device
        self.out = torch.empty(int(bound), dtype=torch.uint8, device=dev)
        self.sizes = torch.zeros(n, dtype=torch.int64, device=dev)
        offs = (C.c_uint64 * n)()
        plan = C.c_void_p()
        _check(lib.mgard_batch_create(n, C.cast(arr, C.c_void_p), float(tol), _ptr(self.out), self.out.numel(),
                                      offs, _ptr(self.sizes), C.byref(o), C.byref(plan)))
        self.plan = plan
        self.offsets = [int(offs[i]) for i in range(n)]
        self.launches = int(lib.mgard_batch_launches(plan))

    def launch(self, stream=None):
        if stream is None:
            stream = _torch().cuda.current_stream().cuda_stream
        _check(load_library().mgard_batch_launch(self.plan, C.c_void_p(stream)))

    def results(self):
        torch = _torch()
        torch.cuda.synchronize()
        sizes = self.sizes.cpu().tolist()
        return [(self.out[o:o + s], s) for o, s in zip(self.offsets, sizes)]

    def close(self):
        if getattr(self, "plan", None):
            load_library().mgard_batch_free(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ refactoring
def mgard_refactor_bound(shape, dtype=F32, planes=32, coords=None):
    lib = load_library()
    cc = _Coords(coords, len(shape))
    b = lib.mgard_refactor_bound(len(shape), _shape(shape), cc.ptr, dtype, planes)
    if b == 0:
        _check(-1)
    return int(b)


def mgard_refactor(u, planes=32, coords=None, out=None):
    """Refactors a CUDA float tensor into bitplane segments.  Returns (uint8 CUDA buffer, nbytes)."""
    torch = _torch()
    lib = load_library()
    u = u.contiguous()
    dt = _dtype_code(u)
    shape = tuple(u.shape)
    cc = _Coords(coords, len(shape))
    if out is None:
        out = torch.empty(mgard_refactor_bound(shape, dt, planes, coords), dtype=torch.uint8, device=u.device)
    nb = C.c_uint64(0)
    o = make_opts()
    _check(lib.mgard_refactor(len(shape), _shape(shape), cc.ptr, dt, planes, _ptr(u), _ptr(out), out.numel(),
                              C.byref(nb), C.byref(o)))
    return out, int(nb.value)


def mgard_refactor_inspect(meta: bytes):
    """(metadata bytes, levels, planes, total bytes) of a refactored buffer's first bytes."""
    lib = load_library()
    mb, L, B, tot = C.c_uint64(0), C.c_uint32(0), C.c_uint32(0), C.c_uint64(0)
    b = C.create_string_buffer(bytes(meta), len(meta))
    _check(lib.mgard_refactor_inspect(b, len(meta), C.byref(mb), C.byref(L), C.byref(B), C.byref(tot)))
    return int(mb.value), int(L.value), int(B.value), int(tot.value)


def _u32s(v):
    return None if v is None else (C.c_uint32 * len(v))(*[int(x) for x in v])


def mgard_refactor_request(meta: bytes, tol, have=None, eb="rel", norm="linf", s=0.0):
    """Planes per level to hold for tol (greedy, from `have`), and the estimate."""
    lib = load_library()
    _, L, _, _ = mgard_refactor_inspect(meta)
    want = (C.c_uint32 * (L + 1))()
    est = C.c_double(0.0)
    o = mgard_opts()
    lib.mgard_default_opts(C.byref(o))
    o.eb = REL if eb == "rel" else ABS
    o.norm = NORM_S if norm == "s" else NORM_LINF
    o.s = float(s)
    b = C.create_string_buffer(bytes(meta), len(meta))
    _check(lib.mgard_refactor_request(b, len(meta), float(tol), _u32s(have), want, L + 1, C.byref(est), C.byref(o)))
    return [int(x) for x in want], float(est.value)


def mgard_refactor_ranges(meta: bytes, have, want):
    """Byte ranges (offset, length) of the buffer to fetch to go from `have` to `want` planes."""
    lib = load_library()
    n = len(want)
    offs, lens, cnt = (C.c_uint64 * n)(), (C.c_uint64 * n)(), C.c_uint32(0)
    b = C.create_string_buffer(bytes(meta), len(meta))
    _check(lib.mgard_refactor_ranges(b, len(meta), _u32s(have), _u32s(want), n, offs, lens, C.byref(cnt)))
    return [(int(offs[i]), int(lens[i])) for i in range(cnt.value)]


def mgard_reconstruct(buf, nbytes, planes, out=None):
    """Reconstruction from the first planes[l] planes of every level of a refactored CUDA buffer."""
    torch = _torch()
    lib = load_library()
    if out is None:
        import struct

        head = buf[: min(nbytes, 64)].cpu().numpy().tobytes()
        if len(head) < 40 or head[:4] != b"MGRF" or not 1 <= head[7] <= 4:
            raise MgardError(-7, "not a refactored buffer")
        dt, nd = head[6], head[7]
        shape = struct.unpack_from("<%dQ" % nd, head, 32)
        out = torch.empty(shape, dtype=torch.float64 if dt else torch.float32, device=buf.device)
    o = make_opts()
    _check(lib.mgard_reconstruct(_ptr(buf), nbytes, _u32s(planes), len(planes), _ptr(out),
                                 out.numel() * out.element_size(), C.byref(o)))
    return out


# ------------------------------------------------------------------ lossless stage
def mgard_lossless_bound(raw_bytes):
    return int(load_library().mgard_lossless_bound(int(raw_bytes)))


def mgard_lossless_encode(buf, nbytes, out=None):
    """Zero-suppression container of the first nbytes of a uint8 CUDA buffer: (buffer, nbytes)."""
    torch = _torch()
    lib = load_library()
    if out is None:
        out = torch.empty(mgard_lossless_bound(nbytes), dtype=torch.uint8, device=buf.device)
    nb = C.c_uint64(0)
    o = make_opts()
    _check(lib.mgard_lossless_encode(_ptr(buf), int(nbytes), _ptr(out), out.numel(), C.byref(nb), C.byref(o)))
    return out, int(nb.value)


def mgard_lossless_decode(buf, nbytes, out=None, raw_bytes=None):
    """Inverse of mgard_lossless_encode: (uint8 CUDA buffer, raw bytes)."""
    torch = _torch()
    lib = load_library()
    if out is None:
        if raw_bytes is None:
            import struct

            raw_bytes = struct.unpack_from("<Q", buf[:24].cpu().numpy().tobytes(), 8)[0]
        out = torch.empty(4 * ((raw_bytes + 3) // 4), dtype=torch.uint8, device=buf.device)
    rb = C.c_uint64(0)
    o = make_opts()
    _check(lib.mgard_lossless_decode(_ptr(buf), int(nbytes), _ptr(out), out.numel(), C.byref(rb), C.byref(o)))
    return out, int(rb.value)
