"""Plain CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, the package's smoke() check and bench.py's cpu_baseline leg may
import this package.  It wraps ``ms_oracle.c`` (plain C, built with gcc by
``build()``) with numpy arrays and composes the two queries of the paper's
evaluation shape from the plain operators.  It imports nothing from the GPU
package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

UNCOMPR, STATIC_BP, DYN_BP, DELTA_DYN_BP, FOR_DYN_BP, RLE = range(6)
KINDS = (UNCOMPR, STATIC_BP, DYN_BP, DELTA_DYN_BP, FOR_DYN_BP, RLE)
KIND_NAMES = ("UNCOMPR", "STATIC_BP", "DYN_BP", "DELTA_DYN_BP", "FOR_DYN_BP", "RLE")
EQ, NE, LT, LE, GT, GE, BETWEEN = range(7)
BW_AUTO = 0xFFFFFFFF
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_VALUE_TOO_WIDE, ERR_OUT_OF_RANGE, ERR_NOT_SORTED, ERR_LENGTH_MISMATCH = range(7)
MLP_NPARAM = 64 * 32 + 64 + 64 * 64 + 64 + 6 * 64 + 6


class OracleError(Exception):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "ms_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Col(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_uint32), ("bit_width", ctypes.c_uint32),
        ("n", ctypes.c_uint64), ("n_main", ctypes.c_uint64), ("n_rem", ctypes.c_uint64),
        ("nb", ctypes.c_uint64), ("payload_words", ctypes.c_uint64), ("runs", ctypes.c_uint64),
        ("widths", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("bases", ctypes.c_void_p),
        ("payload", ctypes.c_void_p), ("rem", ctypes.c_void_p),
        ("rvalues", ctypes.c_void_p), ("rstarts", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.c_void_p
        L.or_encode.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_Col)]
        L.or_decode.argtypes = [ctypes.POINTER(_Col), u32p]
        L.or_footprint.argtypes = [ctypes.POINTER(_Col)]
        L.or_footprint.restype = ctypes.c_uint64
        L.or_bw.argtypes = [ctypes.c_uint32]
        L.or_bw.restype = ctypes.c_uint32
        L.or_select.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.or_select.restype = ctypes.c_uint64
        L.or_bitmap_from_positions.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, u32p]
        L.or_semijoin.argtypes = [u32p, ctypes.c_uint64, u32p, ctypes.c_uint64, u32p]
        L.or_semijoin.restype = ctypes.c_uint64
        L.or_project.argtypes = [u32p, ctypes.c_uint64, u32p, ctypes.c_uint64, u32p]
        L.or_intersect.argtypes = [u32p, ctypes.c_uint64, u32p, ctypes.c_uint64, u32p, ctypes.POINTER(ctypes.c_uint64)]
        L.or_sum.argtypes = [u32p, ctypes.c_uint64]
        L.or_sum.restype = ctypes.c_uint64
        L.or_group_sum.argtypes = [u32p, ctypes.c_uint64, u32p, ctypes.c_uint64, ctypes.c_uint32, u32p]
        L.or_stats.argtypes = [u32p, ctypes.c_uint64, u32p]
        L.or_footprints.argtypes = [u32p, ctypes.c_uint64, u32p]
        L.or_mlp_forward.argtypes = [u32p, u32p, ctypes.c_uint64, u32p]
        L.or_mlp_loss_grad.argtypes = [u32p, u32p, u32p, ctypes.c_uint64, u32p]
        L.or_mlp_loss_grad.restype = ctypes.c_double
        L.or_adam_step.argtypes = [u32p, u32p, u32p, u32p, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_uint64]
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def bw(x: int) -> int:
    return int(lib().or_bw(x))


# ----------------------------------------------------------------------------- formats
def encode(values, kind: int, bit_width: int = BW_AUTO) -> dict:
    """Encode into `kind`; returns the sections as numpy arrays (canonical layout)."""
    v = _u32(values)
    n = v.size
    nbk = n // 512 + 1
    arr = dict(
        widths=np.zeros(nbk, np.uint8), offsets=np.zeros(nbk, np.uint32), bases=np.zeros(nbk, np.uint32),
        payload=np.zeros(n + 16, np.uint32), rem=np.zeros(512, np.uint32),
        rvalues=np.zeros(max(n, 1), np.uint32), rstarts=np.zeros(max(n, 1), np.uint32),
    )
    c = _Col()
    for k, a in arr.items():
        setattr(c, k, _p(a))
    st = lib().or_encode(_p(v), n, kind, bit_width, ctypes.byref(c))
    if st != OK:
        raise OracleError(st, "encode")
    return dict(
        kind=kind, n=n, bit_width=c.bit_width, n_main=c.n_main, n_rem=c.n_rem, nb=c.nb,
        payload_words=c.payload_words, runs=c.runs,
        widths=arr["widths"][: c.nb].copy(), offsets=arr["offsets"][: c.nb].copy(),
        bases=arr["bases"][: c.nb].copy(), payload=arr["payload"][: c.payload_words].copy(),
        rem=arr["rem"][: c.n_rem].copy(), rvalues=arr["rvalues"][: c.runs].copy(),
        rstarts=arr["rstarts"][: c.runs].copy(),
        footprint=int(lib().or_footprint(ctypes.byref(c))),
    )


def _colstruct(enc: dict, keep: list) -> _Col:
    c = _Col()
    for k in ("kind", "bit_width", "n", "n_main", "n_rem", "nb", "runs"):
        setattr(c, k, int(enc[k]))
    pw = enc["payload"]
    c.payload_words = int(pw.size)
    for k, dt in (("widths", np.uint8), ("offsets", np.uint32), ("bases", np.uint32),
                  ("payload", np.uint32), ("rem", np.uint32), ("rvalues", np.uint32), ("rstarts", np.uint32)):
        a = np.ascontiguousarray(enc[k], dtype=dt)
        if a.size == 0:
            a = np.zeros(1, dt)
        keep.append(a)
        setattr(c, k, _p(a))
    return c


def decode(enc: dict) -> np.ndarray:
    """Decode sections (from the oracle or from the GPU library) back to values."""
    keep: list = []
    c = _colstruct(enc, keep)
    out = np.zeros(max(int(enc["n"]), 1), np.uint32)
    st = lib().or_decode(ctypes.byref(c), _p(out))
    if st != OK:
        raise OracleError(st, "decode")
    return out[: int(enc["n"])]


def footprint(enc: dict) -> int:
    keep: list = []
    c = _colstruct(enc, keep)
    return int(lib().or_footprint(ctypes.byref(c)))


def footprints(values) -> np.ndarray:
    v = _u32(values)
    out = np.zeros(6, np.uint64)
    lib().or_footprints(_p(v) if v.size else None, v.size, _p(out))
    return out


# ----------------------------------------------------------------------------- operators
def select(values, cmp: int, c0: int, c1: int = 0) -> np.ndarray:
    v = _u32(values)
    out = np.zeros(max(v.size, 1), np.uint32)
    k = lib().or_select(_p(v), v.size, cmp, c0, c1, _p(out))
    return out[:k].copy()


def bitmap_from_positions(pos, domain: int) -> np.ndarray:
    p = _u32(pos)
    bm = np.zeros(max((domain + 31) // 32, 1), np.uint32)
    st = lib().or_bitmap_from_positions(_p(p), p.size, domain, _p(bm))
    if st != OK:
        raise OracleError(st, "bitmap_from_positions")
    return bm[: (domain + 31) // 32]


def semijoin(keys, bitmap, domain: int) -> np.ndarray:
    k = _u32(keys)
    bm = _u32(bitmap) if len(bitmap) else np.zeros(1, np.uint32)
    out = np.zeros(max(k.size, 1), np.uint32)
    cnt = lib().or_semijoin(_p(k), k.size, _p(bm), domain, _p(out))
    return out[:cnt].copy()


def project(data, pos) -> np.ndarray:
    d = _u32(data)
    p = _u32(pos)
    out = np.zeros(max(p.size, 1), np.uint32)
    st = lib().or_project(_p(d) if d.size else None, d.size, _p(p), p.size, _p(out))
    if st != OK:
        raise OracleError(st, "project")
    return out[: p.size].copy()


def intersect(a, b) -> np.ndarray:
    a = _u32(a)
    b = _u32(b)
    out = np.zeros(max(min(a.size, b.size), 1), np.uint32)
    k = ctypes.c_uint64(0)
    st = lib().or_intersect(_p(a), a.size, _p(b), b.size, _p(out), ctypes.byref(k))
    if st != OK:
        raise OracleError(st, "intersect")
    return out[: k.value].copy()


def sum_(values) -> int:
    v = _u32(values)
    return int(lib().or_sum(_p(v), v.size))


def group_sum(groups, values, G: int) -> np.ndarray:
    g = _u32(groups)
    v = _u32(values)
    out = np.zeros(max(G, 1), np.uint64)
    st = lib().or_group_sum(_p(g), g.size, _p(v), v.size, G, _p(out))
    if st != OK:
        raise OracleError(st, "group_sum")
    return out[:G]


def stats(values) -> np.ndarray:
    v = _u32(values)
    out = np.zeros(32, np.float64)
    lib().or_stats(_p(v) if v.size else None, v.size, _p(out))
    return out


# ----------------------------------------------------------------------------- selector network
def mlp_forward(params, x) -> np.ndarray:
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 32)
    y = np.zeros((x.shape[0], 6), np.float64)
    lib().or_mlp_forward(_p(p), _p(x), x.shape[0], _p(y))
    return y


def mlp_loss_grad(params, x, t):
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 32)
    t = np.ascontiguousarray(t, np.float64).reshape(-1, 6)
    g = np.zeros(MLP_NPARAM, np.float64)
    loss = lib().or_mlp_loss_grad(_p(p), _p(x), _p(t), x.shape[0], _p(g))
    return float(loss), g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays params, m, v."""
    lib().or_adam_step(_p(params), _p(np.ascontiguousarray(grad, np.float64)), _p(m), _p(v), step, lr,
                       beta1, beta2, eps, params.size)


# ----------------------------------------------------------------------------- format selection
def exhaustive_choice(bytes6) -> np.ndarray:
    """Section 5.2's exhaustive selection for rows of six footprints: the format of least
    physical size, scanning the formats in their fixed order so that ties keep the lower
    format number."""
    F = np.asarray(bytes6, np.uint64).reshape(-1, 6)
    out = np.zeros(F.shape[0], np.int64)
    for i in range(F.shape[0]):
        best = 0
        for k in range(1, 6):
            if int(F[i, k]) < int(F[i, best]):
                best = k
        out[i] = best
    return out


def size_targets(bytes6, n) -> np.ndarray:
    """Targets of the size network: t_k = log2(1 + bits per value of format k) / 6, with
    bits per value = 8 * footprint_k / n (an empty column counts as n = 1), in float64."""
    F = np.asarray(bytes6, np.float64).reshape(-1, 6)
    nv = np.maximum(np.asarray(n, np.float64).reshape(-1, 1), 1.0)
    return np.log2(1.0 + 8.0 * F / nv) / 6.0


def cost_targets(ns6, n) -> np.ndarray:
    """Targets of the decode-cost network: t_k = log2(1 + picoseconds per value spent
    decoding format k) / 16, from measured nanoseconds per decode (negative times count
    as 0; an empty column counts as n = 1), in float64."""
    C = np.maximum(np.asarray(ns6, np.float64).reshape(-1, 6), 0.0)
    nv = np.maximum(np.asarray(n, np.float64).reshape(-1, 1), 1.0)
    return np.log2(1.0 + 1000.0 * C / nv) / 16.0


# ----------------------------------------------------------------------------- wider operator set
# The operators of the paper's star-schema plans beyond select / semi-join / intersect /
# project / aggregation (section 4.2's operator list, section 5.2's SSB plans): element-wise
# arithmetic on two columns ("calc"), a join that emits position pairs, and a group-by that
# assigns group ids itself.
CALC_ADD, CALC_SUB, CALC_MUL = range(3)


def calc(a, b, op: int) -> np.ndarray:
    """out_i = a_i (+, -, *) b_i, unsigned 32-bit arithmetic wrapping modulo 2^32."""
    a = _u32(a).astype(np.uint64)
    b = _u32(b).astype(np.uint64)
    if a.size != b.size:
        raise OracleError(ERR_LENGTH_MISMATCH, "calc")
    with np.errstate(over="ignore"):
        if op == CALC_ADD:
            r = a + b
        elif op == CALC_SUB:
            r = a + (np.uint64(1 << 32) - b)
        elif op == CALC_MUL:
            r = a * b  # both factors < 2^32: the product fits 64 bits
        else:
            raise OracleError(ERR_INVALID_ARG, "calc")
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def join_pairs(keys, bitmap, domain: int):
    """Join of a foreign-key column with a dimension whose qualifying rows are marked in
    `bitmap` (bit k of word k // 32): the ascending fact positions i with keys_i < domain
    and bit keys_i set (left), and the matching dimension positions keys_i (right)."""
    k = _u32(keys)
    bm = _u32(bitmap)
    left = []
    for i in range(k.size):
        x = int(k[i])
        if x < domain and (int(bm[x >> 5]) >> (x & 31)) & 1:
            left.append(i)
    left = np.asarray(left, np.uint32)
    return left, k[left.astype(np.int64)].astype(np.uint32) if left.size else np.zeros(0, np.uint32)


def group_by(keys):
    """Group ids assigned from the data: the distinct keys in ascending order, and for
    every row the rank of its key among them (ids 0 .. #groups - 1)."""
    k = _u32(keys)
    distinct = np.array(sorted(set(int(x) for x in k)), np.uint32)
    rank = {int(v): i for i, v in enumerate(distinct)}
    return np.array([rank[int(x)] for x in k], np.uint32), distinct
