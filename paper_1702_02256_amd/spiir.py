"""Python binding of libspiir.so: argument marshalling only.

Every step of the filtering path runs in the library's HIP kernels; this module
converts numpy tables and torch device tensors into the C ABI's pointers and
sizes.  The functions ``spiir_*`` mirror the C entry points one to one;
``Bank`` is a thin object wrapper over them.  Importing this module fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SPIIR_LIB_PATH selects another build of the same library (same ABI).
LIB_PATH = os.environ.get("SPIIR_LIB_PATH") or os.path.join(_PKG, "libspiir.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "spiir.h")

SPIIR_OK = 0
SPIIR_EINVAL = -1
SPIIR_ENOMEM = -2
SPIIR_EDEVICE = -3
SPIIR_EORDER = -4
SPIIR_ENONFINITE = -5
SPIIR_FP32 = 0
SPIIR_FP32_COMPENSATED = 1
MAX_BATCH = 16
NOALLOC_MAX_WORKSPACE = 32 << 20  # bytes of the static workspace (spiir_process_block_noalloc)
TIME_CHUNKS_AUTO = -1  # time_chunks: the library chooses the split
WORKSPACE_OWN = 0      # spiir_create allocates the bank's workspace
WORKSPACE_CALLER = 1   # every request brings one (spiir_request.ws_dev)
ENGINE_VALU = 0        # the filter bank sample by sample on the vector units
ENGINE_MFMA = 1        # prototype: single-rate banks through the matrix cores

_PRECISION = {"fp32": SPIIR_FP32, "fp32_compensated": SPIIR_FP32_COMPENSATED,
              "compensated": SPIIR_FP32_COMPENSATED}


class BankDesc(C.Structure):
    _fields_ = [
        ("n_templates", C.c_int32),
        ("n_bands", C.c_int32),
        ("base_rate_hz", C.c_int32),
        ("n_filters", C.POINTER(C.c_int32)),
        ("a1", C.POINTER(C.c_double)),
        ("b0", C.POINTER(C.c_double)),
        ("delay", C.POINTER(C.c_int32)),
        ("n_taps_down", C.c_int32),
        ("h_down", C.POINTER(C.c_double)),
        ("n_taps_up", C.c_int32),
        ("h_up", C.POINTER(C.c_double)),
        ("max_block", C.c_int32),
        ("precision", C.c_int32),
        ("carry_chunk", C.c_int32),
        ("filters_per_lane", C.c_int32),
        ("waves_per_group", C.c_int32),
        ("device", C.c_int32),
        ("time_chunks", C.c_int32),
        ("window_copies", C.c_int32),
        ("workspace", C.c_int32),
        ("engine", C.c_int32),
    ]


class Request(C.Structure):
    _fields_ = [
        ("bank", C.c_void_p),
        ("x_dev", C.c_void_p),
        ("n", C.c_int64),
        ("z_dev", C.c_void_p),
        ("ldz", C.c_int64),
        ("ws_dev", C.c_void_p),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("total_filters", C.c_int64),
        ("filter_slots", C.c_int64),
        ("n_groups", C.c_int32),
        ("n_pieces", C.c_int32),
        ("lanes_per_group", C.c_int32),
        ("filters_per_lane", C.c_int32),
        ("lds_bytes", C.c_int32),
        ("carry_chunk", C.c_int32),
        ("footprint", C.c_size_t),
        ("time_chunks", C.c_int32),
        ("window_copies", C.c_int32),
        ("workspace_bytes", C.c_size_t),
        ("workspace", C.c_int32),
        ("engine", C.c_int32),
    ]


class ProfileData(C.Structure):
    _fields_ = [("launches", C.c_int64 * 3), ("ms", C.c_double * 3)]


class SpiirError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {spiir_strerror(code)} ({code})")


_lib = None


def load_library():
    """Load libspiir.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (there is no fallback path)")
    _torch_hip_first()
    lib = C.CDLL(LIB_PATH)
    paths = hip_runtime_paths()
    if len(paths) > 1:
        raise ImportError("two HIP runtimes are mapped in this process (%s): the library and the "
                          "GPU memory it is given must use one" % ", ".join(paths))
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "spiir_footprint": (C.c_int, [C.POINTER(BankDesc), C.POINTER(C.c_size_t)]),
        "spiir_create": (C.c_int, [C.POINTER(BankDesc), vp, C.POINTER(vp)]),
        "spiir_clone": (C.c_int, [vp, vp, C.POINTER(vp)]),
        "spiir_process_block": (C.c_int, [vp, vp, i64, vp, i64, vp]),
        "spiir_process_block_noalloc": (C.c_int, [vp, vp, i64, vp, i64, vp]),
        "spiir_process_batch": (C.c_int, [i32, C.POINTER(Request), vp]),
        "spiir_reset": (C.c_int, [vp]),
        "spiir_state_size": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "spiir_save_state": (C.c_int, [vp, vp, vp]),
        "spiir_load_state": (C.c_int, [vp, vp, vp]),
        "spiir_status": (C.c_int, [vp, C.POINTER(C.c_int32)]),
        "spiir_destroy": (C.c_int, [vp]),
        "spiir_strerror": (C.c_char_p, [C.c_int]),
        "spiir_samples_done": (C.c_int, [vp, C.POINTER(C.c_int64)]),
        "spiir_plan": (C.c_int, [C.POINTER(BankDesc), C.POINTER(PlanInfo)]),
        "spiir_bank_plan": (C.c_int, [vp, C.POINTER(PlanInfo)]),
        "spiir_profile_enable": (C.c_int, [C.c_int]),
        "spiir_profile_read": (C.c_int, [C.POINTER(ProfileData)]),
        "spiir_process_peaks": (C.c_int, [vp, vp, i64, vp, i64, vp, C.c_float, vp]),
        "spiir_process_batch_peaks": (C.c_int, [i32, C.POINTER(Request), C.POINTER(vp), C.c_float, vp]),
        "spiir_graph_create": (C.c_int, [i32, C.POINTER(Request), C.POINTER(vp)]),
        "spiir_graph_launch": (C.c_int, [vp, vp]),
        "spiir_graph_destroy": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def hip_runtime_paths() -> list:
    """Distinct files of the HIP runtime (libamdhip64) mapped in this process.

    The library links libamdhip64.so.7 by that soname.  When torch is imported
    first, its bundled runtime, which carries the same soname, is already
    mapped and the loader binds the library to it, so the library, torch's
    allocator and torch's streams share one runtime; a process without torch
    maps ROCm's.  Two distinct files here would mean two runtimes."""
    out = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                i = line.find("/")
                if i >= 0 and os.path.basename(line[i:].strip()).startswith("libamdhip64"):
                    out.add(os.path.realpath(line[i:].strip()))
    except OSError:
        pass
    return sorted(out)


def header_symbols() -> list:
    """Entry points declared in include/spiir.h."""
    txt = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^(?:int|const char\s*\*)\s*(spiir_[a-z_]+)\s*\(", txt, re.M)))


def spiir_strerror(code: int) -> str:
    return load_library().spiir_strerror(int(code)).decode()


def _check(rc: int, where: str) -> int:
    if rc != SPIIR_OK:
        raise SpiirError(rc, where)
    return rc


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class _DescHolder:
    """A BankDesc plus the numpy arrays its pointers refer to."""

    def __init__(self, tables, max_block, precision="fp32", carry_chunk=0, filters_per_lane=0,
                 waves_per_group=0, device=0, time_chunks=0, window_copies=0, workspace=WORKSPACE_OWN,
                 engine=ENGINE_VALU):
        self.nf = np.ascontiguousarray(tables.n_filters.reshape(-1), dtype=np.int32)
        self.a1 = np.ascontiguousarray(np.asarray(tables.a1, np.complex128)).view(np.float64)
        self.b0 = np.ascontiguousarray(np.asarray(tables.b0, np.complex128)).view(np.float64)
        self.d = np.ascontiguousarray(tables.delay, dtype=np.int32)
        self.hd = np.ascontiguousarray(tables.h_down, dtype=np.float64)
        self.hu = np.ascontiguousarray(tables.h_up, dtype=np.float64)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        prec = _PRECISION[precision] if isinstance(precision, str) else int(precision)
        self.desc = BankDesc(
            n_templates=int(tables.n_filters.shape[0]),
            n_bands=int(tables.n_filters.shape[1]),
            base_rate_hz=int(tables.base_rate),
            n_filters=ip(self.nf), a1=dp(self.a1), b0=dp(self.b0), delay=ip(self.d),
            n_taps_down=len(self.hd), h_down=dp(self.hd),
            n_taps_up=len(self.hu), h_up=dp(self.hu),
            max_block=int(max_block), precision=prec, carry_chunk=int(carry_chunk),
            filters_per_lane=int(filters_per_lane), waves_per_group=int(waves_per_group),
            device=int(device), time_chunks=int(time_chunks), window_copies=int(window_copies),
            workspace=int(workspace), engine=int(engine))


# ---------------------------------------------------------------- C-named functions


def spiir_plan(tables, max_block, **kw) -> dict:
    h = _DescHolder(tables, max_block, **kw)
    info = PlanInfo()
    _check(load_library().spiir_plan(C.byref(h.desc), C.byref(info)), "spiir_plan")
    return {k: getattr(info, k) for k, _ in PlanInfo._fields_}


def spiir_footprint(tables, max_block, **kw) -> int:
    h = _DescHolder(tables, max_block, **kw)
    out = C.c_size_t()
    _check(load_library().spiir_footprint(C.byref(h.desc), C.byref(out)), "spiir_footprint")
    return int(out.value)


def spiir_create(tables, max_block, stream=None, **kw) -> "Bank":
    return Bank(tables, max_block, stream=stream, **kw)


def spiir_process_block(bank: "Bank", x, z, stream=None) -> None:
    bank.process_block(x, z, stream)


def _ws_ptr(bank, ws):
    """Device address of a caller workspace (a torch tensor or an int), or None."""
    if ws is None:
        return None
    if isinstance(ws, int):
        return ws
    if not ws.is_cuda or ws.numel() * ws.element_size() < bank.workspace_bytes:
        raise ValueError("the workspace must be a device tensor of at least workspace_bytes")
    return ws.data_ptr()


def _request(item, z_optional=False):
    """(bank, x, z[, ws]) -> Request; z may be None where z_optional."""
    bank, x, z = item[:3]
    ws = item[3] if len(item) > 3 else None
    _validate_io(bank, x, z, z_optional=z_optional)
    return Request(bank._h, x.data_ptr(), int(x.numel()), z.data_ptr() if z is not None else None,
                   int(z.stride(0)) if z is not None else 0, _ws_ptr(bank, ws))


def workspace_empty(nbytes: int, device="cuda"):
    """A device buffer usable as a request workspace (256-byte aligned by torch)."""
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def spiir_process_batch(requests, stream=None) -> None:
    """requests: list of (bank, x, z) or (bank, x, z, workspace) with torch device tensors."""
    n = len(requests)
    arr = (Request * max(n, 1))()
    for i, item in enumerate(requests):
        arr[i] = _request(item)
    _check(load_library().spiir_process_batch(n, arr, _stream_handle(stream)), "spiir_process_batch")


class Graph:
    """A recorded batch (spiir_graph_*): the launch sequence of one
    spiir_process_batch call over fixed buffers, replayed by `launch`.

    requests: list of (bank, x, z) device tensors; x is refilled and z read by
    the caller between launches, in stream order.
    """

    def __init__(self, requests):
        lib = load_library()
        self._lib = lib
        n = len(requests)
        arr = (Request * max(n, 1))()
        for i, item in enumerate(requests):
            arr[i] = _request(item)
        # keep the tensors alive as long as the recorded pointers are used
        self._keep = [tuple(item) for item in requests]
        h = C.c_void_p()
        _check(lib.spiir_graph_create(n, arr, C.byref(h)), "spiir_graph_create")
        self._h = h.value

    def launch(self, stream=None) -> None:
        _check(self._lib.spiir_graph_launch(self._h, _stream_handle(stream)), "spiir_graph_launch")

    def destroy(self) -> None:
        if getattr(self, "_h", None):
            self._lib.spiir_graph_destroy(self._h)
            self._h = None
        self._keep = []

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def spiir_profile_enable(on: bool = True) -> None:
    _check(load_library().spiir_profile_enable(1 if on else 0), "spiir_profile_enable")


def spiir_profile_read() -> dict:
    d = ProfileData()
    _check(load_library().spiir_profile_read(C.byref(d)), "spiir_profile_read")
    names = ("stage", "filter", "upadd")
    return {names[i]: {"launches": int(d.launches[i]), "ms": float(d.ms[i])} for i in range(3)}


def peaks_empty(n_templates: int, device="cuda"):
    """Device buffer for spiir_peak[n_templates] (int32 [T, 4]; see peaks_unpack)."""
    import torch
    return torch.empty((n_templates, 4), dtype=torch.int32, device=device)


def peaks_unpack(peaks) -> dict:
    """Host copy of a spiir_peak buffer: peak2 (float32), index, n_above (int32)."""
    a = peaks.cpu().numpy()
    return {"peak2": a[:, 0].copy().view(np.float32), "index": a[:, 1].copy(),
            "n_above": a[:, 2].copy()}


def _validate_peaks(bank, peaks):
    import torch
    if (peaks.dtype != torch.int32 or not peaks.is_cuda or tuple(peaks.shape) != (bank.n_templates, 4)
            or not peaks.is_contiguous()):
        raise ValueError("peaks must be a contiguous int32 device tensor of shape (n_templates, 4)")


def spiir_process_batch_peaks(requests, peaks, threshold: float, stream=None) -> None:
    """requests: list of (bank, x, z or None[, workspace]); peaks: one peaks_empty buffer per request."""
    n = len(requests)
    arr = (Request * max(n, 1))()
    pk = (C.c_void_p * max(n, 1))()
    for i, (item, p) in enumerate(zip(requests, peaks)):
        arr[i] = _request(item, z_optional=True)
        _validate_peaks(item[0], p)
        pk[i] = p.data_ptr()
    _check(load_library().spiir_process_batch_peaks(n, arr, pk, float(threshold), _stream_handle(stream)),
           "spiir_process_batch_peaks")


def _validate_io(bank, x, z, z_optional=False):
    import torch
    if z is None and not z_optional:
        raise ValueError("z is required")
    if x.dtype != torch.float32 or not x.is_cuda or x.dim() != 1 or not x.is_contiguous():
        raise ValueError("x must be a contiguous 1-D float32 device tensor")
    if z is None:
        return
    if z.dtype != torch.complex64 or not z.is_cuda or z.dim() != 2 or z.stride(1) != 1:
        raise ValueError("z must be a 2-D complex64 device tensor with unit inner stride")
    if z.shape[0] < bank.n_templates or z.shape[1] < x.numel():
        raise ValueError("z is too small for this block")


def _torch_hip_first():
    """Start torch's HIP runtime before the library makes its first device call.

    The torch wheel ships its own HIP runtime next to the one the library links;
    when the library's runtime opens the GPU first, torch's finds no device.
    Started in this order both work on the same device memory."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


class Bank:
    """One template bank bound to one input stream (owns its device memory)."""

    def __init__(self, tables, max_block, stream=None, precision="fp32", carry_chunk=0,
                 filters_per_lane=0, waves_per_group=0, device=0, time_chunks=0, window_copies=0,
                 workspace=WORKSPACE_OWN, engine=ENGINE_VALU, _clone_of=None):
        _torch_hip_first()
        lib = load_library()
        self._lib = lib
        h = C.c_void_p()
        s = _stream_handle(stream) if stream is not None else C.c_void_p(0)
        if _clone_of is not None:
            self.n_templates, self.n_bands = _clone_of.n_templates, _clone_of.n_bands
            self.max_block = _clone_of.max_block
            _check(lib.spiir_clone(_clone_of._h, s, C.byref(h)), "spiir_clone")
        else:
            hold = _DescHolder(tables, max_block, precision, carry_chunk, filters_per_lane,
                               waves_per_group, device, time_chunks, window_copies, workspace, engine)
            self.n_templates = int(tables.n_filters.shape[0])
            self.n_bands = int(tables.n_filters.shape[1])
            self.max_block = int(max_block)
            _check(lib.spiir_create(C.byref(hold.desc), s, C.byref(h)), "spiir_create")
        self._h = h.value
        info = PlanInfo()
        _check(lib.spiir_bank_plan(self._h, C.byref(info)), "spiir_bank_plan")
        self.plan = {k: getattr(info, k) for k, _ in PlanInfo._fields_}
        self.workspace_bytes = int(self.plan["workspace_bytes"])

    def clone(self, stream=None) -> "Bank":
        """spiir_clone: the same tables and plan, zero state, a stream of its own."""
        return Bank(None, None, stream=stream, _clone_of=self)

    def process_block(self, x, z, stream=None, ws=None) -> None:
        """spiir_process_block, or with a caller workspace `ws` a one-request
        spiir_process_batch (the same launch sequence)."""
        if ws is not None:
            spiir_process_batch([(self, x, z, ws)], stream)
            return
        _validate_io(self, x, z)
        rc = self._lib.spiir_process_block(self._h, x.data_ptr(), int(x.numel()), z.data_ptr(),
                                           int(z.stride(0)), _stream_handle(stream))
        _check(rc, "spiir_process_block")

    def process_block_noalloc(self, x, z, stream=None) -> None:
        """spiir_process_block_noalloc: the workspace is the library's static array."""
        _validate_io(self, x, z)
        rc = self._lib.spiir_process_block_noalloc(self._h, x.data_ptr(), int(x.numel()), z.data_ptr(),
                                                   int(z.stride(0)), _stream_handle(stream))
        _check(rc, "spiir_process_block_noalloc")

    def process_peaks(self, x, z, peaks, threshold: float, stream=None, ws=None) -> None:
        """process_block plus the trigger reduction into `peaks` (z may be None)."""
        if ws is not None:
            spiir_process_batch_peaks([(self, x, z, ws)], [peaks], threshold, stream)
            return
        _validate_io(self, x, z, z_optional=True)
        _validate_peaks(self, peaks)
        rc = self._lib.spiir_process_peaks(self._h, x.data_ptr(), int(x.numel()),
                                           z.data_ptr() if z is not None else None,
                                           int(z.stride(0)) if z is not None else 0,
                                           peaks.data_ptr(), float(threshold), _stream_handle(stream))
        _check(rc, "spiir_process_peaks")

    def process_raw(self, x_ptr: int, n: int, z_ptr: int, ldz: int, stream=None) -> int:
        """Unchecked pointer form (returns the status code)."""
        return self._lib.spiir_process_block(self._h, x_ptr, n, z_ptr, ldz, _stream_handle(stream))

    @property
    def samples_done(self) -> int:
        v = C.c_int64()
        _check(self._lib.spiir_samples_done(self._h, C.byref(v)), "spiir_samples_done")
        return int(v.value)

    def reset(self) -> None:
        _check(self._lib.spiir_reset(self._h), "spiir_reset")

    def state_size(self) -> int:
        v = C.c_size_t()
        _check(self._lib.spiir_state_size(self._h, C.byref(v)), "spiir_state_size")
        return int(v.value)

    def save_state(self, stream=None) -> bytes:
        buf = C.create_string_buffer(self.state_size())
        _check(self._lib.spiir_save_state(self._h, buf, _stream_handle(stream)), "spiir_save_state")
        return buf.raw

    def load_state(self, blob: bytes, stream=None) -> None:
        # the library reads state_size() bytes: a blob of another length is refused here
        if len(blob) != self.state_size():
            raise SpiirError(SPIIR_EINVAL, "spiir_load_state")
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(self._lib.spiir_load_state(self._h, buf, _stream_handle(stream)), "spiir_load_state")

    def status(self):
        """(status code, per-template non-finite flags)."""
        flags = np.zeros(self.n_templates, np.int32)
        rc = self._lib.spiir_status(self._h, flags.ctypes.data_as(C.POINTER(C.c_int32)))
        return rc, flags

    def destroy(self) -> None:
        if getattr(self, "_h", None):
            self._lib.spiir_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
