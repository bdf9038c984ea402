"""Thin Python binding of the rngx C-ABI (include/rngx.h).

Per-thread random-number streams (LCG32, LCG64, MWC, XORWOW, Philox4x32-10
and the XORShift-1024/Weyl generator of Manssen, Weigel & Hartmann) and their
checkerboard Metropolis Ising consumer, as HIP kernels for gfx950 in
librngx.so.  This module only marshals arguments: device buffers are torch
tensors (or raw device addresses as ints), streams default to torch's current
stream, and every non-OK status raises RngxError.  There is no fallback: if
librngx.so is absent the import of the library fails.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import torch  # loaded first so that librngx.so binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librngx.so")

KINDS = {"lcg32": 1, "lcg64": 2, "mwc": 3, "xorwow": 4, "philox4x32_10": 5, "xs1024w": 6, "philox4x32_7": 7,
         "lcg32_sub": 8, "lcg64_sub": 9, "lfg521": 10, "lfg1279": 11, "mwc_diff": 12}
KIND_NAMES = {v: k for k, v in KINDS.items()}
STATUS = {0: "RNGX_OK", -1: "RNGX_E_INVALID", -2: "RNGX_E_ALIGN", -3: "RNGX_E_NOMEM", -4: "RNGX_E_HIP",
          -5: "RNGX_E_OVERFLOW", -6: "RNGX_E_STATE", -7: "RNGX_E_BUSY"}

# Names exported by the C-ABI and their ctypes signatures.
_u64, _i32, _vp, _sz = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
SIGNATURES = {
    "rng_create": (_i32, [_i32, _u64, _u64, ctypes.POINTER(_vp)]),
    "rng_create_substreams": (_i32, [_i32, _u64, _u64, ctypes.POINTER(_vp)]),
    "rng_destroy": (_i32, [_vp]),
    "rng_info": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_u64)]),
    "rng_fill_u32": (_i32, [_vp, _vp, _u64, _vp]),
    "rng_fill_f32": (_i32, [_vp, _vp, _u64, _vp]),
    "rng_consume": (_i32, [_vp, _vp, _u64, _vp]),
    "rng_skip": (_i32, [_vp, _u64, _vp]),
    "rng_fill_configs": (_i32, [_i32, _vp, ctypes.POINTER(_i32)]),
    "rng_set_fill_config": (_i32, [_vp, _i32]),
    "rng_get_fill_config": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "rng_autotune_fill": (_i32, [_vp, _vp, _u64, _i32, _vp, _vp]),
    "ising_plans": (_i32, [_vp, _vp, ctypes.POINTER(_i32)]),
    "ising_set_plan": (_i32, [_vp, ctypes.c_uint32]),
    "ising_autotune": (_i32, [_vp, ctypes.c_double, _u64, _i32, _vp, _vp]),
    "rng_ragged_create": (_i32, [_vp, _vp, _u64, ctypes.POINTER(_vp)]),
    "rng_fill_ragged_u32": (_i32, [_vp, _vp, _vp]),
    "rng_ragged_destroy": (_i32, [_vp]),
    "rng_ragged_shapes": (_i32, [_i32, ctypes.POINTER(_u64), ctypes.POINTER(_i32)]),
    "rng_ragged_set_shape": (_i32, [_vp, _i32]),
    "rng_ragged_get_shape": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "rng_ragged_autotune": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "rng_fill_ragged_u32_noalloc": (_i32, [_vp, _vp, _u64, _vp, _vp]),
    "rng_get_state": (_i32, [_vp, _vp, ctypes.POINTER(_sz), _vp]),
    "rng_set_state": (_i32, [_vp, _vp, _sz, _vp]),
    "ising_create": (_i32, [ctypes.c_uint32, _i32, _u64, ctypes.POINTER(_vp)]),
    "ising_sweep": (_i32, [_vp, ctypes.c_double, _u64, _vp, _vp]),
    "ising_sweep_hits": (_i32, [_vp, ctypes.c_double, _u64, ctypes.c_uint32, _vp, _vp]),
    "ising_info": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_uint32)]),
    "ising_spins": (_i32, [_vp, ctypes.POINTER(_vp)]),
    "ising_get_spins": (_i32, [_vp, _vp, _vp]),
    "ising_set_spins": (_i32, [_vp, _vp, _vp]),
    "ising_rng": (_i32, [_vp, ctypes.POINTER(_vp)]),
    "ising_status": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), _vp]),
    "ising_destroy": (_i32, [_vp]),
    "ising_batch_create": (_i32, [ctypes.POINTER(_vp), ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(_u64), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "ising_batch_run": (_i32, [_vp, _vp]),
    "ising_batch_status": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), _vp]),
    "ising_batch_info": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(ctypes.c_uint32)]),
    "ising_batch_destroy": (_i32, [_vp]),
    "ising_batch_shapes": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "ising_batch_set_shape": (_i32, [_vp, _i32]),
    "ising_batch_get_shape": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "ising_batch_autotune": (_i32, [_vp, _u64, _i32, _vp, _vp]),
    "srv_create": (_i32, [ctypes.c_void_p, ctypes.POINTER(_vp)]),
    "srv_submit_fill": (_i32, [_vp, ctypes.c_uint32, _i32, _u64, _i32, ctypes.POINTER(_u64)]),
    "srv_submit_ising": (_i32, [_vp, ctypes.c_uint32, _i32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32,
                                ctypes.POINTER(_u64)]),
    "srv_wait": (_i32, [_vp, _u64, ctypes.c_double, ctypes.c_void_p]),
    "srv_wait_any": (_i32, [_vp, ctypes.c_double, ctypes.POINTER(_u64), ctypes.c_void_p]),
    "srv_release": (_i32, [_vp, _u64]),
    "srv_cancel": (_i32, [_vp, _u64]),
    "srv_get_client_state": (_i32, [_vp, ctypes.c_uint32, _i32, _vp, ctypes.POINTER(_sz)]),
    "srv_set_client_state": (_i32, [_vp, ctypes.c_uint32, _i32, _vp, _sz]),
    "srv_destroy": (_i32, [_vp]),
    "rngx_last_error": (ctypes.c_char_p, []),
}


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32), ("memory_budget", ctypes.c_uint64),
                ("seed", ctypes.c_uint64)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("d_output", ctypes.c_void_p), ("n_values", ctypes.c_uint64),
                ("latency_s", ctypes.c_double)]


class RngxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
# Set when the interpreter starts to exit: handles still alive then are not
# destroyed by their finalizers (which would call into the HIP runtime while
# it, torch and any attached profiler are being torn down); the process exit
# releases their device memory.  Destroy handles explicitly to free it sooner.
_exiting = False


def _mark_exiting():
    global _exiting
    _exiting = True


atexit.register(_mark_exiting)


def _finalizing() -> bool:
    return _exiting or _lib is None


def load():
    """Load librngx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(st: int):
    if st != 0:
        raise RngxError(st, load().rngx_last_error().decode())


def _kind(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dptr(buf, min_elems: int, elem_size: int):
    """Device address of `buf` (a CUDA tensor, or an int address)."""
    if isinstance(buf, int) or buf is None:
        return buf
    if not buf.is_cuda:
        raise ValueError("buffer must be a device tensor")
    if not buf.is_contiguous():
        raise ValueError("buffer must be contiguous")
    if buf.element_size() != elem_size:
        raise ValueError(f"buffer elements must be {elem_size} bytes")
    if buf.numel() < min_elems:
        raise ValueError(f"buffer holds {buf.numel()} elements, needs {min_elems}")
    return buf.data_ptr()


class Gen:
    """A handle of S streams (owns the device state unless borrowed)."""

    def __init__(self, handle, owned=True):
        self.handle = handle
        self.owned = owned
        k = ctypes.c_int()
        s = ctypes.c_uint64()
        _check(load().rng_info(handle, ctypes.byref(k), ctypes.byref(s)))
        self.kind = KIND_NAMES[k.value]
        self.n_streams = s.value

    def __del__(self):
        if getattr(self, "owned", False) and self.handle and not _finalizing():
            _lib.rng_destroy(self.handle)
            self.handle = None

    def destroy(self):
        if self.owned and self.handle:
            _check(load().rng_destroy(self.handle))
        self.handle = None


def rng_create(kind, n_streams: int, seed: int) -> Gen:
    h = _vp()
    _check(load().rng_create(_kind(kind), n_streams, seed, ctypes.byref(h)))
    return Gen(h.value)


def rng_create_substreams(kind, n_streams: int, seed: int) -> Gen:
    """XS1024W: instance g = instance 0 of rng_create skipped g * 2^137 steps."""
    h = _vp()
    _check(load().rng_create_substreams(_kind(kind), n_streams, seed, ctypes.byref(h)))
    return Gen(h.value)


def rng_destroy(g: Gen):
    g.destroy()


def rng_fill_u32(g: Gen, out, count_per_stream: int, stream=None):
    _check(load().rng_fill_u32(g.handle, _dptr(out, g.n_streams * count_per_stream, 4), count_per_stream,
                               _stream(stream)))


def rng_fill_f32(g: Gen, out, count_per_stream: int, stream=None):
    _check(load().rng_fill_f32(g.handle, _dptr(out, g.n_streams * count_per_stream, 4), count_per_stream,
                               _stream(stream)))


def rng_consume(g: Gen, out_xor, count_per_stream: int, stream=None):
    _check(load().rng_consume(g.handle, _dptr(out_xor, g.n_streams, 4), count_per_stream, _stream(stream)))


def rng_skip(g: Gen, n: int, stream=None):
    _check(load().rng_skip(g.handle, n, _stream(stream)))


class FillConfig(ctypes.Structure):
    """rngx_fill_config: paced, streams per thread, threads per workgroup."""
    _fields_ = [("paced", ctypes.c_int32), ("streams_per_thread", ctypes.c_int32), ("block", ctypes.c_int32)]


def rng_fill_configs(kind) -> list[tuple[int, int, int]]:
    """The fill configurations of `kind` in index order, as (paced, streams_per_thread, block)."""
    n = ctypes.c_int()
    _check(load().rng_fill_configs(_kind(kind), None, ctypes.byref(n)))
    arr = (FillConfig * n.value)()
    _check(load().rng_fill_configs(_kind(kind), ctypes.cast(arr, _vp), ctypes.byref(n)))
    return [(c.paced, c.streams_per_thread, c.block) for c in arr]


def rng_set_fill_config(g: Gen, index: int):
    _check(load().rng_set_fill_config(g.handle, index))


def rng_get_fill_config(g: Gen) -> int:
    i = ctypes.c_int()
    _check(load().rng_get_fill_config(g.handle, ctypes.byref(i)))
    return i.value


def rng_autotune_fill(g: Gen, out, count_per_stream: int, reps: int = 3, stream=None) -> list[float]:
    """Time every fill configuration on `out` (S*count u32, overwritten), keep the fastest for `g`
    and leave g's stream state unchanged; returns the mean launch time (ms) of each configuration."""
    n = len(rng_fill_configs(g.kind))
    ms = (ctypes.c_float * n)()
    _check(load().rng_autotune_fill(g.handle, _dptr(out, g.n_streams * count_per_stream, 4), count_per_stream, reps,
                                    ctypes.cast(ms, _vp), _stream(stream)))
    return list(ms)


class Ragged:
    """A plan of uneven per-stream requests (keeps its generator alive)."""

    def __init__(self, handle, gen, total):
        self.handle = handle
        self.gen = gen
        self.total = total

    def __del__(self):
        if getattr(self, "handle", None) and not _finalizing():
            _lib.rng_ragged_destroy(self.handle)
            self.handle = None

    def destroy(self):
        if self.handle:
            _check(load().rng_ragged_destroy(self.handle))
        self.handle = None


def rng_ragged_create(g: Gen, offsets) -> Ragged:
    """offsets: n_units + 1 non-decreasing element indices (host array-like)."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    h = _vp()
    _check(load().rng_ragged_create(g.handle, off.ctypes.data, off.size, ctypes.byref(h)))
    return Ragged(h.value, g, int(off[-1]))


def rng_fill_ragged_u32(r: Ragged, out, stream=None):
    _check(load().rng_fill_ragged_u32(r.handle, _dptr(out, r.total, 4), _stream(stream)))


def rng_ragged_destroy(r: Ragged):
    r.destroy()


def rng_ragged_shapes(kind) -> list[int]:
    """The ragged shape values of `kind` in index order (XS1024W: rows per CU; else outputs per chunk)."""
    n = ctypes.c_int()
    _check(load().rng_ragged_shapes(_kind(kind), None, ctypes.byref(n)))
    arr = (_u64 * n.value)()
    _check(load().rng_ragged_shapes(_kind(kind), arr, ctypes.byref(n)))
    return [int(v) for v in arr]


def rng_ragged_set_shape(r: Ragged, index: int):
    _check(load().rng_ragged_set_shape(r.handle, int(index)))


def rng_ragged_get_shape(r: Ragged) -> int:
    v = ctypes.c_int()
    _check(load().rng_ragged_get_shape(r.handle, ctypes.byref(v)))
    return v.value


def rng_ragged_autotune(r: Ragged, out, reps: int = 2, stream=None) -> list[float]:
    """Time every ragged shape on fills into `out` (overwritten), keep the fastest and restore the
    streams; returns the mean fill time (ms) of each shape."""
    n = len(rng_ragged_shapes(r.gen.kind))
    ms = (ctypes.c_float * n)()
    _check(load().rng_ragged_autotune(r.handle, _dptr(out, r.total, 4), int(reps), ctypes.cast(ms, _vp),
                                      _stream(stream)))
    return list(ms)


def rng_fill_ragged_u32_noalloc(g: Gen, offsets, out, stream=None):
    """rng_ragged_create + rng_fill_ragged_u32 in one synchronous call that
    allocates no device memory (the plan is staged in the library's static
    device scratch)."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    total = int(off[-1]) if off.size else 0
    _check(load().rng_fill_ragged_u32_noalloc(g.handle, off.ctypes.data, off.size, _dptr(out, total, 4),
                                              _stream(stream)))


def rng_get_state(g: Gen, stream=None):
    """State image as a numpy uint8 array (layout in include/rngx.h)."""
    import numpy as np
    n = ctypes.c_size_t()
    _check(load().rng_get_state(g.handle, None, ctypes.byref(n), _stream(stream)))
    buf = np.zeros(n.value, dtype=np.uint8)
    _check(load().rng_get_state(g.handle, buf.ctypes.data, ctypes.byref(n), _stream(stream)))
    return buf


def rng_set_state(g: Gen, image, stream=None):
    import numpy as np
    buf = np.ascontiguousarray(image, dtype=np.uint8)
    _check(load().rng_set_state(g.handle, buf.ctypes.data, buf.nbytes, _stream(stream)))


class Ising:
    """An L x L lattice with its L*L/4 streams."""

    def __init__(self, handle, L, kind):
        self.handle = handle
        self.L = L
        self.kind = kind

    def __del__(self):
        if getattr(self, "handle", None) and not _finalizing():
            _lib.ising_destroy(self.handle)
            self.handle = None

    def destroy(self):
        if self.handle:
            _check(load().ising_destroy(self.handle))
        self.handle = None


def ising_create(L: int, kind, seed: int) -> Ising:
    h = _vp()
    _check(load().ising_create(L, _kind(kind), seed, ctypes.byref(h)))
    return Ising(h.value, L, kind)


def ising_sweep(lat: Ising, beta: float, n_sweeps: int, energy_trace=None, stream=None):
    _check(load().ising_sweep(lat.handle, beta, n_sweeps, _dptr(energy_trace, n_sweeps, 4), _stream(stream)))


def ising_sweep_hits(lat: Ising, beta: float, n_sweeps: int, hits: int, energy_trace=None, stream=None):
    """Multi-hit sweeps: `hits` Metropolis updates per visited site."""
    _check(load().ising_sweep_hits(lat.handle, beta, n_sweeps, hits, _dptr(energy_trace, n_sweeps, 4),
                                   _stream(stream)))


def ising_info(lat: Ising) -> dict:
    """{"L", "kind", "strips"}: strips = on-chip strip workgroups (0 = one launch per colour pass)."""
    L = ctypes.c_uint32()
    k = ctypes.c_int()
    n = ctypes.c_uint32()
    _check(load().ising_info(lat.handle, ctypes.byref(L), ctypes.byref(k), ctypes.byref(n)))
    return {"L": L.value, "kind": KIND_NAMES[k.value], "strips": n.value}


def ising_plans(lat: Ising) -> list[int]:
    """Strip counts that fit this lattice, most strips first, then 0 (one launch per colour pass)."""
    n = ctypes.c_int()
    _check(load().ising_plans(lat.handle, None, ctypes.byref(n)))
    arr = (ctypes.c_uint32 * n.value)()
    _check(load().ising_plans(lat.handle, ctypes.cast(arr, _vp), ctypes.byref(n)))
    return list(arr)


def ising_set_plan(lat: Ising, strips: int):
    _check(load().ising_set_plan(lat.handle, strips))


def ising_autotune(lat: Ising, beta: float, n_sweeps: int, reps: int = 2, stream=None) -> list[float]:
    """Time every plan (ising_plans order), keep the fastest, restore spins and streams; returns ms per call."""
    n = len(ising_plans(lat))
    ms = (ctypes.c_float * n)()
    _check(load().ising_autotune(lat.handle, beta, n_sweeps, reps, ctypes.cast(ms, _vp), _stream(stream)))
    return list(ms)


def ising_spins(lat: Ising) -> int:
    """Device address of the L*L int8 spins (borrowed)."""
    p = _vp()
    _check(load().ising_spins(lat.handle, ctypes.byref(p)))
    return p.value


_hip = None


def copy_to_host(d_ptr: int, nbytes: int, dtype="uint8"):
    """Copy nbytes of device memory (e.g. a server result) into a new numpy
    array, with the HIP runtime torch loaded (same process-wide runtime)."""
    import numpy as np
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(nbytes, dtype=np.uint8)
    rc = _hip.hipMemcpy(out.ctypes.data, d_ptr, nbytes, 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")
    return out.view(dtype)


class _DeviceArray:
    """Exposes a borrowed device allocation through __cuda_array_interface__."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}


def ising_spins_view(lat: Ising) -> torch.Tensor:
    """Zero-copy int8 device tensor [L, L] over the lattice's spins (borrowed:
    valid until the lattice is destroyed)."""
    L = lat.L
    return torch.as_tensor(_DeviceArray(ising_spins(lat), L * L, "|i1"), device="cuda").view(L, L)


def ising_get_spins(lat: Ising, stream=None):
    """Spins as a numpy int8 array [L, L] (host copy)."""
    import numpy as np
    out = np.zeros(lat.L * lat.L, dtype=np.int8)
    _check(load().ising_get_spins(lat.handle, out.ctypes.data, _stream(stream)))
    return out.reshape(lat.L, lat.L)


def ising_set_spins(lat: Ising, spins, stream=None):
    import numpy as np
    buf = np.ascontiguousarray(spins, dtype=np.int8).ravel()
    if buf.size != lat.L * lat.L:
        raise ValueError(f"need {lat.L * lat.L} spins, got {buf.size}")
    _check(load().ising_set_spins(lat.handle, buf.ctypes.data, _stream(stream)))


def ising_status(lat: Ising, stream=None) -> int:
    """1 if a strip gave up waiting for a neighbour (the lattice is invalid), else 0."""
    v = ctypes.c_uint32()
    _check(load().ising_status(lat.handle, ctypes.byref(v), _stream(stream)))
    return v.value


def ising_rng(lat: Ising) -> Gen:
    h = _vp()
    _check(load().ising_rng(lat.handle, ctypes.byref(h)))
    return Gen(h.value, owned=False)


def ising_destroy(lat: Ising):
    lat.destroy()


class IsingBatch:
    """Lattices swept together by one launch per run (keeps its members alive)."""

    def __init__(self, handle, members, traces):
        self.handle = handle
        self.members = members
        self.traces = traces

    def __del__(self):
        if getattr(self, "handle", None) and not _finalizing():
            _lib.ising_batch_destroy(self.handle)
            self.handle = None

    def destroy(self):
        if self.handle:
            _check(load().ising_batch_destroy(self.handle))
        self.handle = None


def ising_batch_create(lats, betas, n_sweeps, traces=None) -> IsingBatch:
    """traces: None, or a list of int32 device tensors (or None entries) of n_sweeps[i] elements."""
    n = len(lats)
    harr = (_vp * n)(*[l.handle for l in lats])
    barr = (ctypes.c_double * n)(*[float(b) for b in betas])
    sarr = (_u64 * n)(*[int(x) for x in n_sweeps])
    tarr = None
    if traces is not None:
        tarr = (_vp * n)(*[_dptr(t, int(x), 4) if t is not None else None for t, x in zip(traces, n_sweeps)])
    h = _vp()
    _check(load().ising_batch_create(harr, n, barr, sarr, tarr, ctypes.byref(h)))
    return IsingBatch(h.value, list(lats), traces)


def ising_batch_run(batch: IsingBatch, stream=None):
    _check(load().ising_batch_run(batch.handle, _stream(stream)))


def ising_batch_status(batch: IsingBatch, stream=None) -> int:
    """Number of replicas of the batch that are invalid (see ising_status)."""
    v = ctypes.c_uint32()
    _check(load().ising_batch_status(batch.handle, ctypes.byref(v), _stream(stream)))
    return v.value


def ising_batch_info(batch: IsingBatch) -> dict:
    """{"items": work items, "resident": workgroups that fit at once,
    "grid": workgroups of the persistent launch}."""
    n, r, g = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().ising_batch_info(batch.handle, ctypes.byref(n), ctypes.byref(r), ctypes.byref(g)))
    return {"items": n.value, "resident": r.value, "grid": g.value}


class BatchShape(ctypes.Structure):
    """rngx_batch_shape: threads per workgroup, most sites per thread, most LDS bytes of a strip."""
    _fields_ = [("threads", ctypes.c_uint32), ("sites_per_thread", ctypes.c_uint32), ("lds_cap", ctypes.c_uint32)]


def ising_batch_shapes() -> list[tuple[int, int, int]]:
    """The batch launch shapes in index order, as (threads, sites_per_thread, lds_cap)."""
    n = ctypes.c_int()
    _check(load().ising_batch_shapes(None, ctypes.byref(n)))
    arr = (BatchShape * n.value)()
    _check(load().ising_batch_shapes(ctypes.cast(arr, _vp), ctypes.byref(n)))
    return [(c.threads, c.sites_per_thread, c.lds_cap) for c in arr]


def ising_batch_set_shape(batch: IsingBatch, index: int):
    _check(load().ising_batch_set_shape(batch.handle, int(index)))


def ising_batch_get_shape(batch: IsingBatch) -> int:
    v = ctypes.c_int()
    _check(load().ising_batch_get_shape(batch.handle, ctypes.byref(v)))
    return v.value


def ising_batch_autotune(batch: IsingBatch, max_sweeps: int = 200, reps: int = 2, stream=None) -> list[float]:
    """Time every batch shape (sweep counts scaled so the longest is max_sweeps), keep the fastest and
    restore the replicas; returns the mean run time (ms) of each shape."""
    n = len(ising_batch_shapes())
    ms = (ctypes.c_float * n)()
    _check(load().ising_batch_autotune(batch.handle, int(max_sweeps), int(reps), ctypes.cast(ms, _vp),
                                       _stream(stream)))
    return list(ms)


def ising_batch_destroy(batch: IsingBatch):
    batch.destroy()


class Server:
    """Request server (continuous batching over `slots` streams, memory budget)."""

    def __init__(self, slots=8, max_inflight=32, memory_budget=8 << 30, seed=1):
        cfg = ServerConfig(slots, max_inflight, memory_budget, seed)
        h = _vp()
        _check(load().srv_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h.value

    def submit_fill(self, client: int, kind, count: int, f32: bool = False) -> int:
        t = _u64()
        _check(load().srv_submit_fill(self.handle, client, _kind(kind), count, int(f32), ctypes.byref(t)))
        return t.value

    def submit_ising(self, client: int, kind, L: int, beta: float, sweeps: int) -> int:
        t = _u64()
        _check(load().srv_submit_ising(self.handle, client, _kind(kind), L, beta, sweeps, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0) -> RequestResult:
        r = RequestResult()
        _check(load().srv_wait(self.handle, ticket, timeout_s, ctypes.byref(r)))
        return r

    def wait_any(self, timeout_s: float = -1.0):
        """(ticket, RequestResult) of the next request to finish."""
        r = RequestResult()
        t = _u64()
        _check(load().srv_wait_any(self.handle, timeout_s, ctypes.byref(t), ctypes.byref(r)))
        return t.value, r

    def release(self, ticket: int):
        _check(load().srv_release(self.handle, ticket))

    def cancel(self, ticket: int):
        """Withdraw a request that has not been admitted yet."""
        _check(load().srv_cancel(self.handle, ticket))

    def get_client_state(self, client: int, kind):
        """State image (numpy uint8) of the (client, kind) stream."""
        import numpy as np
        n = _sz()
        _check(load().srv_get_client_state(self.handle, client, _kind(kind), None, ctypes.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint8)
        _check(load().srv_get_client_state(self.handle, client, _kind(kind), buf.ctypes.data, ctypes.byref(n)))
        return buf

    def set_client_state(self, client: int, kind, image):
        import numpy as np
        buf = np.ascontiguousarray(image, dtype=np.uint8)
        _check(load().srv_set_client_state(self.handle, client, _kind(kind), buf.ctypes.data, buf.size))

    def destroy(self):
        if self.handle:
            _check(load().srv_destroy(self.handle))
        self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and not _finalizing():
            _lib.srv_destroy(self.handle)
            self.handle = None
