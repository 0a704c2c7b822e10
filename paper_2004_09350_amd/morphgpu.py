"""Thin Python binding of libmorphgpu.so (argument marshalling only).

Every step of every operator runs in the HIP library; this module converts
arguments, registers PyTorch's caching allocator as the library's device memory
provider and uses PyTorch streams.  There is no CPU fallback: if the library is
missing the import of this module fails.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# MS_LIBMORPHGPU selects another build of the library (e.g. one with host-side sanitizers)
LIB_PATH = os.environ.get("MS_LIBMORPHGPU") or os.path.join(HERE, "libmorphgpu.so")

UNCOMPR, STATIC_BP, DYN_BP, DELTA_DYN_BP, FOR_DYN_BP, RLE = range(6)
KINDS = (UNCOMPR, STATIC_BP, DYN_BP, DELTA_DYN_BP, FOR_DYN_BP, RLE)
KIND_NAMES = ("UNCOMPR", "STATIC_BP", "DYN_BP", "DELTA_DYN_BP", "FOR_DYN_BP", "RLE")
EQ, NE, LT, LE, GT, GE, BETWEEN = range(7)
BW_AUTO = 0xFFFFFFFF
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "VALUE_TOO_WIDE", 4: "OUT_OF_RANGE", 5: "NOT_SORTED",
          6: "LENGTH_MISMATCH", 7: "OOM", 8: "HIP", 9: "NOT_INITIALIZED"}
SEC_WIDTHS, SEC_OFFSETS, SEC_BASES, SEC_PAYLOAD, SEC_REM, SEC_RVALUES, SEC_RSTARTS = range(7)


class MorphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Format(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("bit_width", ctypes.c_uint32)]


class ColumnInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("kind", ctypes.c_uint32), ("bit_width", ctypes.c_uint32),
                ("n_main", ctypes.c_uint64), ("n_rem", ctypes.c_uint64), ("n_blocks", ctypes.c_uint64),
                ("runs", ctypes.c_uint64), ("payload_words", ctypes.c_uint64), ("payload_extent", ctypes.c_uint64),
                ("footprint", ctypes.c_uint64), ("capacity_bytes", ctypes.c_uint64), ("or_all", ctypes.c_uint32),
                ("sorted", ctypes.c_uint32)]


def fmt(kind, bit_width: int = BW_AUTO) -> Format:
    if isinstance(kind, str):
        kind = KIND_NAMES.index(kind)
    return Format(int(kind), int(bit_width) if kind == STATIC_BP else 0)


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_PP = ctypes.POINTER(ctypes.c_void_p)
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p)

class Step(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("cmp", ctypes.c_uint32),
                ("c0", ctypes.c_uint32), ("c1", ctypes.c_uint32), ("param", ctypes.c_uint64), ("out", Format)]


class Tune(ctypes.Structure):
    _fields_ = [("branches", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32), ("chunks_per_wg", ctypes.c_uint32),
                ("batch", ctypes.c_uint32)]


_sigs = {
    "ms_init": [_ALLOC_T, _FREE_T, _P],
    "ms_column_encode": [_P, _U64, Format, _P, _PP],
    "ms_column_wrap_uncompr": [_P, _U64, _P, _PP],
    "ms_column_decode": [_P, _P, _P],
    "ms_column_free": [_P],
    "ms_column_info_get": [_P, _P, ctypes.POINTER(ColumnInfo)],
    "ms_column_read_section": [_P, _U32, _P, _U64, _P, ctypes.POINTER(_U64)],
    "ms_column_shrink": [_P, _P],
    "ms_morph": [_P, Format, _P, _PP],
    "ms_select": [_P, _U32, _U32, _U32, Format, _P, _PP],
    "ms_bitmap_from_positions": [_P, _U64, _P, _P],
    "ms_semijoin": [_P, _P, _U64, Format, _P, _PP],
    "ms_project": [_P, _P, Format, _P, _PP],
    "ms_intersect": [_P, _P, _U64, Format, _P, _PP],
    "ms_sum": [_P, _P, _P],
    "ms_group_sum": [_P, _P, _U32, _P, _P],
    "ms_group_sum_noalloc": [_P, _P, _U32, _P, _P],
    "ms_sync": [_P],
    "ms_footprints": [_P, _P, _P],
    "ms_calc": [_P, _P, _U32, Format, _P, _PP],
    "ms_join": [_P, _P, _U64, Format, Format, _P, _PP, _PP],
    "ms_group_by": [_P, _U64, Format, Format, _P, _PP, _PP],
    "ms_stats": [_P, _P, _P],
    "ms_mlp_forward": [_P, _P, _U64, _P, _P, _P],
    "ms_mlp_grad": [_P, _P, _P, _U64, _P, _P, _P],
    "ms_plan_create": [ctypes.POINTER(Step), _U32, ctypes.POINTER(_P), _U32, _PP],
    "ms_plan_destroy": [_P],
    "ms_plan_set_format": [_P, _U32, Format],
    "ms_plan_set_tune": [_P, ctypes.POINTER(Tune)],
    "ms_plan_get_format": [_P, _U32, ctypes.POINTER(Format)],
    "ms_plan_get_tune": [_P, ctypes.POINTER(Tune)],
    "ms_plan_run": [_P, _P],
    "ms_plan_launch": [_P, _P],
    "ms_plan_result": [_P, _U32, _PP, _PP],
    "ms_plan_read_result": [_P, _U32, _P, _U64, _P, ctypes.POINTER(_U64)],
    "ms_plan_autotune": [_P, _P, _U32, ctypes.c_char_p, ctypes.POINTER(Tune), ctypes.POINTER(ctypes.c_float)],
    "ms_adam_step": [_P, _P, _P, _P, _U64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P],
    "ms_selector_create": [_P, _P, _PP],
    "ms_selector_destroy": [_P],
    "ms_selector_params": [_P, _U32, _P, _P],
    "ms_selector_save": [_P, ctypes.c_char_p],
    "ms_selector_load": [ctypes.c_char_p, _PP],
    "ms_selector_size_targets": [_P, _P, _U64, _P, _P],
    "ms_selector_cost_targets": [_P, _P, _U64, _P, _P],
    "ms_selector_train": [_P, _U32, _P, _P, _U64, _P, ctypes.POINTER(ctypes.c_float), _P],
    "ms_selector_pick": [_P, _U32, _P, _U64, _P, _P, _P],
    "ms_select_exhaustive": [_P, _P, _P, _P],
    "ms_select_argmin": [_P, _U64, _P, _P],
    "ms_decode_cost": [_P, _U32, _P, _P],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.ms_last_error.restype = ctypes.c_char_p
_lib.ms_last_error.argtypes = []
_lib.ms_prof_enable.argtypes = [ctypes.c_int]
_lib.ms_prof_enable.restype = None
_lib.ms_prof_count.argtypes = []
_lib.ms_prof_count.restype = ctypes.c_uint64
_lib.ms_prof_get.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float)]
_lib.ms_prof_get.restype = ctypes.c_int
_lib.ms_prof_reset.argtypes = []
_lib.ms_prof_reset.restype = None
_lib.ms_mlp_nparam.argtypes = []
_lib.ms_mlp_nparam.restype = ctypes.c_uint32
MLP_NPARAM = int(_lib.ms_mlp_nparam())
_lib.ms_plan_arena_bytes.argtypes = [_P]
_lib.ms_plan_arena_bytes.restype = ctypes.c_uint64
_lib.ms_selector_trained.argtypes = [_P]
_lib.ms_selector_trained.restype = ctypes.c_uint32


def lib():
    return _lib


def _check(st: int):
    if st != 0:
        raise MorphError(st, _lib.ms_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# --------------------------------------------------------------------------------- allocator
_alloc_calls = [0, 0]  # allocator callbacks made by the library: [alloc, free]


def allocator_calls() -> tuple:
    """(alloc, free) callbacks the library has made through this binding so far."""
    return tuple(_alloc_calls)


@_ALLOC_T
def _torch_alloc(nbytes, stream, ctx):
    _alloc_calls[0] += 1
    try:
        p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
        return p
    except Exception:  # allocation failure is reported to the library as NULL (MS_ERR_OOM)
        return None


@_FREE_T
def _torch_free(ptr, nbytes, stream, ctx):
    _alloc_calls[1] += 1
    if ptr:
        torch.cuda.caching_allocator_delete(ptr)


_initialized = False


def init(use_torch_allocator: bool = True):
    """Initialise the library on the current device (idempotent)."""
    global _initialized
    if _initialized:
        return
    if not torch.cuda.is_available():
        raise RuntimeError("libmorphgpu needs a ROCm GPU; none is visible")
    torch.cuda.init()
    if use_torch_allocator:
        _check(_lib.ms_init(_torch_alloc, _torch_free, None))
    else:
        _check(_lib.ms_init(_ALLOC_T(), _FREE_T(), None))
    _initialized = True


# --------------------------------------------------------------------------------- columns
class Column:
    """A compressed column on the device (owns an ms_column*)."""

    def __init__(self, handle: int, keep=None, stream=None, owned: bool = True):
        self._h = ctypes.c_void_p(handle)
        self._keep = keep  # device tensors a wrapped column borrows (or the plan owning a result)
        self._stream = _stream(stream)
        self._owned = owned

    @property
    def handle(self):
        if not self._h.value and self._stale:
            raise MorphError(1, "borrowed plan result used after the plan's results changed (run, launch after a "
                                "change, set_format, set_tune, autotune or close); take plan.column() again")
        return self._h

    _stale = False

    def _invalidate(self):
        """Drop a borrowed handle whose results the plan is about to free."""
        self._h = ctypes.c_void_p(0)
        self._stale = True

    def free(self):
        if self._h and self._h.value and self._owned:
            _lib.ms_column_free(self._h)
        self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self, stream=None) -> dict:
        ci = ColumnInfo()
        _check(_lib.ms_column_info_get(self.handle, _stream(stream), ctypes.byref(ci)))
        return {f: getattr(ci, f) for f, _ in ColumnInfo._fields_}

    def read_section(self, sec: int, nbytes: int, dtype, stream=None) -> np.ndarray:
        buf = np.zeros(max(nbytes, 1), np.uint8)
        got = _U64(0)
        _check(_lib.ms_column_read_section(self.handle, sec, buf.ctypes.data, nbytes, _stream(stream),
                                           ctypes.byref(got)))
        return buf[: got.value].view(dtype).copy()

    def sections(self, stream=None) -> dict:
        """The column's sections on the host, in the dictionary shape the oracle's decoder reads."""
        i = self.info(stream)
        nb = i["n_blocks"]
        out = dict(kind=i["kind"], n=i["n"], bit_width=i["bit_width"], n_main=i["n_main"], n_rem=i["n_rem"],
                   nb=nb, runs=i["runs"], payload_words=i["payload_words"], footprint=i["footprint"])
        out["widths"] = self.read_section(SEC_WIDTHS, nb, np.uint8, stream)
        out["offsets"] = self.read_section(SEC_OFFSETS, 4 * nb, np.uint32, stream)
        out["bases"] = self.read_section(SEC_BASES, 4 * nb, np.uint32, stream)
        out["payload"] = self.read_section(SEC_PAYLOAD, 4 * i["payload_extent"], np.uint32, stream)
        out["rem"] = self.read_section(SEC_REM, 4 * i["n_rem"], np.uint32, stream)
        out["rvalues"] = self.read_section(SEC_RVALUES, 4 * i["runs"], np.uint32, stream)
        out["rstarts"] = self.read_section(SEC_RSTARTS, 4 * i["runs"], np.uint32, stream)
        return out

    def decode(self, n: int | None = None, stream=None) -> torch.Tensor:
        """Decode into a new int32 device tensor holding the uint32 bit patterns."""
        if n is None:
            n = self.info(stream)["n"]
        out = torch.empty(max(n, 4), dtype=torch.int32, device="cuda")
        _check(_lib.ms_column_decode(self.handle, out.data_ptr(), _stream(stream)))
        return out[:n]

    def shrink(self, stream=None):
        _check(_lib.ms_column_shrink(self.handle, _stream(stream)))
        return self

    def __len__(self):
        return self.info()["n"]


def _out(fn, *args, keep=None, stream=None) -> Column:
    h = ctypes.c_void_p(0)
    _check(fn(*args, ctypes.byref(h)))
    return Column(h.value, keep=keep, stream=stream)


def _as_u32_tensor(values) -> torch.Tensor:
    if isinstance(values, torch.Tensor):
        t = values
        if t.dtype not in (torch.int32, torch.uint32):
            raise TypeError("device values must be int32/uint32 tensors (uint32 bit patterns)")
        if not t.is_cuda:
            t = t.cuda()
        return t.contiguous()
    a = np.ascontiguousarray(values, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).cuda()


def encode(values, f: Format, stream=None) -> Column:
    t = _as_u32_tensor(values)
    return _out(_lib.ms_column_encode, t.data_ptr() if t.numel() else None, t.numel(), f, _stream(stream),
                stream=stream)


def wrap(values, stream=None) -> Column:
    t = _as_u32_tensor(values)
    return _out(_lib.ms_column_wrap_uncompr, t.data_ptr() if t.numel() else None, t.numel(), _stream(stream),
                keep=t, stream=stream)


def morph(col: Column, f: Format, stream=None) -> Column:
    return _out(_lib.ms_morph, col.handle, f, _stream(stream), stream=stream)


def select(col: Column, cmp: int, c0: int, c1: int = 0, f: Format = None, stream=None) -> Column:
    f = f if f is not None else fmt(DELTA_DYN_BP)
    return _out(_lib.ms_select, col.handle, cmp, c0 & 0xFFFFFFFF, c1 & 0xFFFFFFFF, f, _stream(stream), stream=stream)


def bitmap_from_positions(pos: Column, domain: int, stream=None) -> torch.Tensor:
    bm = torch.empty(max((domain + 31) // 32, 1), dtype=torch.int32, device="cuda")
    _check(_lib.ms_bitmap_from_positions(pos.handle, domain, bm.data_ptr(), _stream(stream)))
    return bm


def semijoin(keys: Column, bitmap: torch.Tensor, domain: int, f: Format = None, stream=None) -> Column:
    f = f if f is not None else fmt(DELTA_DYN_BP)
    return _out(_lib.ms_semijoin, keys.handle, bitmap.data_ptr(), domain, f, _stream(stream), stream=stream)


def project(data: Column, pos: Column, f: Format = None, stream=None) -> Column:
    f = f if f is not None else fmt(STATIC_BP)
    return _out(_lib.ms_project, data.handle, pos.handle, f, _stream(stream), stream=stream)


def intersect(a: Column, b: Column, domain: int, f: Format = None, stream=None) -> Column:
    f = f if f is not None else fmt(DELTA_DYN_BP)
    return _out(_lib.ms_intersect, a.handle, b.handle, domain, f, _stream(stream), stream=stream)


CALC_ADD, CALC_SUB, CALC_MUL = range(3)


def calc(a: Column, b: Column, op: int, f: Format = None, stream=None) -> Column:
    """Element-wise a op b modulo 2^32 (op: CALC_ADD, CALC_SUB, CALC_MUL)."""
    f = f if f is not None else fmt(STATIC_BP)
    return _out(_lib.ms_calc, a.handle, b.handle, op, f, _stream(stream), stream=stream)


def join(keys: Column, bitmap: torch.Tensor, domain: int, f_left: Format = None, f_right: Format = None,
         stream=None):
    """Position pairs of the join of keys with the dimension rows marked in bitmap:
    (ascending fact positions, the matching dimension positions)."""
    f_left = f_left if f_left is not None else fmt(DELTA_DYN_BP)
    f_right = f_right if f_right is not None else fmt(STATIC_BP)
    l, r = ctypes.c_void_p(0), ctypes.c_void_p(0)
    _check(_lib.ms_join(keys.handle, bitmap.data_ptr(), domain, f_left, f_right, _stream(stream), ctypes.byref(l),
                        ctypes.byref(r)))
    return Column(l.value, stream=stream), Column(r.value, stream=stream)


def group_by(keys: Column, domain: int, f_ids: Format = None, f_keys: Format = None, stream=None):
    """(group id of every row = rank of its key among the distinct keys, the distinct keys
    in ascending order); every key must be below domain (<= 2^28)."""
    f_ids = f_ids if f_ids is not None else fmt(STATIC_BP)
    f_keys = f_keys if f_keys is not None else fmt(DELTA_DYN_BP)
    i, d = ctypes.c_void_p(0), ctypes.c_void_p(0)
    _check(_lib.ms_group_by(keys.handle, domain, f_ids, f_keys, _stream(stream), ctypes.byref(i), ctypes.byref(d)))
    return Column(i.value, stream=stream), Column(d.value, stream=stream)


def sum_(col: Column, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device="cuda")
    _check(_lib.ms_sum(col.handle, out.data_ptr(), _stream(stream)))
    return out


def group_sum(groups: Column, vals: Column, G: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(max(G, 1), dtype=torch.int64, device="cuda")
    _check(_lib.ms_group_sum(groups.handle, vals.handle, G, out.data_ptr(), _stream(stream)))
    return out[:G]


def group_sum_noalloc(groups: Column, vals: Column, G: int, out: torch.Tensor, stream=None) -> torch.Tensor:
    """ms_group_sum_noalloc: group-sum with the library's static scratch; `out` (int64[G],
    caller-allocated) receives the sums."""
    if out.dtype != torch.int64 or not out.is_cuda or out.numel() < G:
        raise ValueError("out must be an int64 CUDA tensor with room for G sums")
    _check(_lib.ms_group_sum_noalloc(groups.handle, vals.handle, G, out.data_ptr(), _stream(stream)))
    return out[:G]


def footprints(col: Column, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Exact bytes of the column in each of the six formats (int64[6], index = kind)."""
    if out is None:
        out = torch.empty(6, dtype=torch.int64, device="cuda")
    _check(_lib.ms_footprints(col.handle, out.data_ptr(), _stream(stream)))
    return out


def stats(col: Column, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The 32 selector features of the column (float32[32], see ms_stats)."""
    if out is None:
        out = torch.empty(32, dtype=torch.float32, device="cuda")
    _check(_lib.ms_stats(col.handle, out.data_ptr(), _stream(stream)))
    return out


def _f32(t: torch.Tensor, *shape) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if shape and tuple(t.shape) != shape:
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


def mlp_forward(params: torch.Tensor, x: torch.Tensor, want_y: bool = True, want_pick: bool = True, stream=None):
    """Selector network outputs (n x 6) and argmin picks (n) for features x (n x 32)."""
    _f32(params, MLP_NPARAM)
    n = x.shape[0]
    _f32(x, n, 32)
    y = torch.empty((n, 6), dtype=torch.float32, device="cuda") if want_y else None
    pick = torch.empty(n, dtype=torch.int32, device="cuda") if want_pick else None
    _check(_lib.ms_mlp_forward(params.data_ptr(), x.data_ptr(), n, y.data_ptr() if y is not None else None,
                               pick.data_ptr() if pick is not None else None, _stream(stream)))
    return y, pick


def mlp_grad(params: torch.Tensor, x: torch.Tensor, t: torch.Tensor, grad: torch.Tensor | None = None,
             stream=None):
    """Gradient (6662) and loss (1) of the mean squared error of the network on (x, t)."""
    _f32(params, MLP_NPARAM)
    n = x.shape[0]
    _f32(x, n, 32)
    _f32(t, n, 6)
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(_lib.ms_mlp_grad(params.data_ptr(), x.data_ptr(), t.data_ptr(), n, grad.data_ptr(), loss.data_ptr(),
                            _stream(stream)))
    return grad, loss


def adam_step(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
    """One Adam update of params, m and v in place (step counts from 1)."""
    for t in (params, grad, m, v):
        _f32(t, MLP_NPARAM)
    _check(_lib.ms_adam_step(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, beta1, beta2,
                             eps, _stream(stream)))


# ----------------------------------------------------------------------------------- selection
NET_SIZE, NET_COST = 0, 1
OBJ_FOOTPRINT, OBJ_DECODE = 0, 1


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


def _u64_tensor(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a if a.is_cuda else a.cuda()
        return t.to(torch.int64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def _f32_tensor(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a if a.is_cuda else a.cuda()
        return t.to(torch.float32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


class Selector:
    """The size and decode-cost networks of the learned format selector (ms_selector)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @classmethod
    def create(cls, init_size: np.ndarray, init_cost: np.ndarray) -> "Selector":
        a = np.ascontiguousarray(init_size, dtype=np.float32)
        b = np.ascontiguousarray(init_cost, dtype=np.float32)
        if a.shape != (MLP_NPARAM,) or b.shape != (MLP_NPARAM,):
            raise ValueError(f"initial parameters must be float32[{MLP_NPARAM}]")
        h = ctypes.c_void_p(0)
        _check(_lib.ms_selector_create(a.ctypes.data, b.ctypes.data, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path: str) -> "Selector":
        h = ctypes.c_void_p(0)
        _check(_lib.ms_selector_load(os.fsencode(path), ctypes.byref(h)))
        return cls(h.value)

    def save(self, path: str):
        _check(_lib.ms_selector_save(self._h, os.fsencode(path)))

    def params(self, net: int, stream=None) -> torch.Tensor:
        """A copy of network `net`'s parameters (float32[6662] on the device)."""
        out = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        _check(_lib.ms_selector_params(self._h, net, out.data_ptr(), _stream(stream)))
        return out

    def trained(self) -> int:
        return int(_lib.ms_selector_trained(self._h))

    def train(self, net: int, x, t, epochs: int = 40, batch: int = 1024, lr: float = 2e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, seed: int = 77, stream=None) -> float:
        """Mini-batch Adam on network `net` over features x (n x 32) and targets t (n x 6);
        returns the mean batch loss of the last pass."""
        xd, td = _f32_tensor(x), _f32_tensor(t)
        n = xd.shape[0]
        _f32(xd, n, 32)
        _f32(td, n, 6)
        cfg = TrainCfg(epochs, batch, lr, beta1, beta2, eps, seed)
        loss = ctypes.c_float(0)
        _check(_lib.ms_selector_train(self._h, net, xd.data_ptr(), td.data_ptr(), n, ctypes.byref(cfg),
                                      ctypes.byref(loss), _stream(stream)))
        return float(loss.value)

    def pick(self, x, objective: int = OBJ_FOOTPRINT, want_pred: bool = False, stream=None):
        """Per row of x (n x 32): the format of least predicted cost (int32[n]), and the
        network's outputs (n x 6) when want_pred."""
        xd = _f32_tensor(x)
        n = xd.shape[0]
        _f32(xd, n, 32)
        kinds = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        pred = torch.empty((max(n, 1), 6), dtype=torch.float32, device="cuda") if want_pred else None
        _check(_lib.ms_selector_pick(self._h, objective, xd.data_ptr(), n, kinds.data_ptr(),
                                     pred.data_ptr() if pred is not None else None, _stream(stream)))
        return (kinds[:n], pred[:n]) if want_pred else kinds[:n]

    def close(self):
        if self._h and self._h.value:
            _lib.ms_selector_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def size_targets(bytes6, n, stream=None) -> torch.Tensor:
    """Training targets of the size network: log2(1 + 8 * bytes / n) / 6 (n x 6 float32)."""
    b, nn = _u64_tensor(bytes6), _u64_tensor(n)
    cnt = nn.numel()
    out = torch.empty((max(cnt, 1), 6), dtype=torch.float32, device="cuda")
    _check(_lib.ms_selector_size_targets(b.data_ptr(), nn.data_ptr(), cnt, out.data_ptr(), _stream(stream)))
    return out[:cnt]


def cost_targets(ns6, n, stream=None) -> torch.Tensor:
    """Training targets of the decode-cost network: log2(1 + 1000 * ns / n) / 16 (n x 6)."""
    c, nn = _f32_tensor(ns6), _u64_tensor(n)
    cnt = nn.numel()
    out = torch.empty((max(cnt, 1), 6), dtype=torch.float32, device="cuda")
    _check(_lib.ms_selector_cost_targets(c.data_ptr(), nn.data_ptr(), cnt, out.data_ptr(), _stream(stream)))
    return out[:cnt]


def select_exhaustive(col: Column, stream=None):
    """(least-footprint kind as an int32[1] device tensor, the six footprints int64[6])."""
    b = torch.empty(6, dtype=torch.int64, device="cuda")
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    _check(_lib.ms_select_exhaustive(col.handle, b.data_ptr(), k.data_ptr(), _stream(stream)))
    return k, b


def select_argmin(bytes6, stream=None) -> torch.Tensor:
    """Exhaustive choice for rows of footprints (n x 6): int32[n], ties to the lower kind."""
    b = _u64_tensor(bytes6)
    cnt = b.numel() // 6
    k = torch.empty(max(cnt, 1), dtype=torch.int32, device="cuda")
    _check(_lib.ms_select_argmin(b.data_ptr(), cnt, k.data_ptr(), _stream(stream)))
    return k[:cnt]


def decode_cost(col: Column, reps: int = 3, stream=None) -> np.ndarray:
    """Measured ns per decode of the column in each of the six formats (float32[6])."""
    out = np.zeros(6, np.float32)
    _check(_lib.ms_decode_cost(col.handle, reps, out.ctypes.data, _stream(stream)))
    return out


# ----------------------------------------------------------------------------------- plans
OP_MORPH, OP_SELECT, OP_BITMAP, OP_SEMIJOIN, OP_PROJECT, OP_INTERSECT, OP_SUM, OP_GROUP_SUM, OP_FOOTPRINTS, \
    OP_STATS = range(10)
_RESULT_BYTES = {OP_SUM: lambda p: 8, OP_GROUP_SUM: lambda p: 8 * max(p, 1), OP_FOOTPRINTS: lambda p: 48,
                 OP_STATS: lambda p: 128, OP_BITMAP: lambda p: 4 * ((p + 31) // 32)}


def step(op: int, a: int = -1, b: int = -1, out: Format | None = None, cmp: int = 0, c0: int = 0, c1: int = 0,
         param: int = 0) -> Step:
    """One plan step; operands: k >= 0 the result of step k, -1 - j input column j."""
    return Step(op, a, b, cmp, c0 & 0xFFFFFFFF, c1 & 0xFFFFFFFF, param, out if out is not None else fmt(UNCOMPR))


def inp(j: int) -> int:
    """Operand reference to input column j."""
    return -1 - j


class Plan:
    """An operator plan over input columns, run eagerly (run) or as a replayed HIP graph (launch)."""

    def __init__(self, steps, inputs):
        self.steps = list(steps)
        self.inputs = list(inputs)  # kept alive: the plan borrows them
        arr = (Step * max(len(self.steps), 1))(*self.steps)
        ins = (_P * max(len(self.inputs), 1))(*[c.handle.value for c in self.inputs])
        h = ctypes.c_void_p(0)
        _check(_lib.ms_plan_create(arr, len(self.steps), ins, len(self.inputs), ctypes.byref(h)))
        self._h = h
        self._borrowed = weakref.WeakSet()  # result views handed out by column()
        self._borrowed_graph = False        # whether they view the captured graph's results

    def _drop_borrowed(self):
        for c in list(self._borrowed):
            c._invalidate()
        self._borrowed = weakref.WeakSet()
        self._borrowed_graph = False

    def close(self):
        self._drop_borrowed()
        if self._h and self._h.value:
            _lib.ms_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_format(self, i: int, f: Format):
        self._drop_borrowed()
        _check(_lib.ms_plan_set_format(self._h, i, f))
        self.steps[i].out = f

    def set_tune(self, branches: int, wg_per_cu: int, chunks_per_wg: int = 0, batch: int = 0):
        """Launch shape (see ms_tune): batch=1 runs the plan level by level with batched
        persistent launches (branches must be 1)."""
        self._drop_borrowed()
        t = Tune(branches, wg_per_cu, chunks_per_wg, batch)
        _check(_lib.ms_plan_set_tune(self._h, ctypes.byref(t)))

    def tune(self) -> tuple:
        t = Tune()
        _check(_lib.ms_plan_get_tune(self._h, ctypes.byref(t)))
        return t.branches, t.wg_per_cu, t.chunks_per_wg, t.batch

    def run(self, stream=None):
        self._drop_borrowed()
        _check(_lib.ms_plan_run(self._h, _stream(stream)))

    def launch(self, stream=None):
        # a replay of the captured graph keeps its results in place; a (re)capture or a
        # switch from eager results does not
        if not self._borrowed_graph:
            self._drop_borrowed()
        _check(_lib.ms_plan_launch(self._h, _stream(stream)))
        self._borrowed_graph = True

    def autotune(self, reps: int = 3, cache: str | None = None, stream=None):
        self._drop_borrowed()
        t = Tune()
        ms = ctypes.c_float(0)
        _check(_lib.ms_plan_autotune(self._h, _stream(stream), reps, cache.encode() if cache else None,
                                     ctypes.byref(t), ctypes.byref(ms)))
        return (t.branches, t.wg_per_cu, t.chunks_per_wg, t.batch), ms.value

    def formats(self) -> list:
        """The output format kind of every step as the library holds it."""
        out = []
        for i in range(len(self.steps)):
            f = Format()
            _check(_lib.ms_plan_get_format(self._h, i, ctypes.byref(f)))
            out.append(f.kind)
        return out

    def arena_bytes(self) -> int:
        return int(_lib.ms_plan_arena_bytes(self._h))

    def column(self, i: int) -> Column:
        """Borrowed view of step i's result column (valid until the next run, capture or close)."""
        c = ctypes.c_void_p(0)
        _check(_lib.ms_plan_result(self._h, i, ctypes.byref(c), None))
        if not c.value:
            raise MorphError(1, "step has no column result")
        col = Column(c.value, keep=self, owned=False)
        self._borrowed.add(col)
        return col

    def read(self, i: int, stream=None) -> np.ndarray:
        """Host copy of a non-column result: uint64 for sums, group sums and footprints,
        float32 for statistics, uint32 words for bitmaps."""
        s = self.steps[i]
        nbytes = _RESULT_BYTES[s.op](s.param)
        buf = np.zeros(max(nbytes, 8), np.uint8)
        got = _U64(0)
        _check(_lib.ms_plan_read_result(self._h, i, buf.ctypes.data, nbytes, _stream(stream), ctypes.byref(got)))
        dt = {OP_STATS: np.float32, OP_BITMAP: np.uint32}.get(s.op, np.uint64)
        return buf[: got.value].view(dt).copy()


def sync(stream=None):
    """Synchronise and raise the first data-dependent device error, if any."""
    _check(_lib.ms_sync(_stream(stream)))


def prof_enable(on: bool = True):
    """Bracket every kernel launch with HIP events on its stream (see ms_prof_enable)."""
    _lib.ms_prof_enable(1 if on else 0)


def prof_count() -> int:
    return int(_lib.ms_prof_count())


def prof_records(start: int = 0) -> list:
    """[(kernel name, milliseconds)] for records start.. (synchronise first)."""
    out = []
    name = ctypes.c_char_p()
    ms = ctypes.c_float()
    for i in range(start, prof_count()):
        _check(_lib.ms_prof_get(i, ctypes.byref(name), ctypes.byref(ms)))
        out.append((name.value.decode(), float(ms.value)))
    return out


def prof_reset():
    _lib.ms_prof_reset()


def u64(t: torch.Tensor) -> np.ndarray:
    """int64 device tensor holding uint64 results -> numpy uint64."""
    return t.cpu().numpy().view(np.uint64)


def u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)
