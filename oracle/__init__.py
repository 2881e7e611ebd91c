"""ctypes binding of the CPU oracle (``libcqref.so``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use this module; the product package never imports it.  The oracle is
single-threaded C (FP64 distances, exact integer histogram and sums) written
from Celebi's Weighted Sort-Means description (Section 2.2, Algo. 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcqref.so")
SRC_PATH = os.path.join(_HERE, "cqref.c")

(INIT_FORGY, INIT_MAXMIN, INIT_KMEANSPP, INIT_USER, INIT_VAR, INIT_SFF, INIT_WU, INIT_LBG,
 INIT_DEN) = 0, 1, 2, 3, 4, 5, 6, 7, 8
OK, EINVAL, ECAPACITY, ENOMEM = 0, 1, 2, 5

BUILD_CMD = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-Wextra",
             "-fPIC", "-shared", "-o", LIB_PATH, SRC_PATH, "-lm"]


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    subprocess.run(BUILD_CMD, check=True)
    return LIB_PATH


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("k_used", ctypes.c_int32),
        ("prune", ctypes.c_int32),
        ("n_unique", ctypes.c_int64),
        ("ndc_total", ctypes.c_int64),
        ("near_ties", ctypes.c_int64),
        ("sse_final", ctypes.c_double),
        ("mse_float", ctypes.c_double),
        ("mse_img", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.cqref_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
        L.cqref_splitmix64_next.restype = u64
        L.cqref_uniform_below.argtypes = [ctypes.POINTER(u64), u64]
        L.cqref_uniform_below.restype = u64
        L.cqref_histogram.argtypes = [P, i32, i32, i64, i32, P, P, i64, ctypes.POINTER(i64)]
        L.cqref_init.argtypes = [P, P, i64, i32, i32, u64, P, ctypes.POINTER(i32)]
        L.cqref_wu_boxes.argtypes = [P, P, i64, i32, P, ctypes.POINTER(i32)]
        L.cqref_den_quotas.argtypes = [P, i64, i32, P]
        L.cqref_sff_subset.argtypes = [i32, i64]
        L.cqref_sff_subset.restype = i64
        L.cqref_kmeans.argtypes = [P, P, i64, i32, P, i32, f64, i32, P, P, P, ctypes.POINTER(Stats)]
        L.cqref_map.argtypes = [P, i32, i32, i64, P, i32, P, P, ctypes.POINTER(u64)]
        L.cqref_quantize.argtypes = [P, i32, i32, i64, i32, i32, i32, u64, i32, f64, i32, P, P, P,
                                     ctypes.POINTER(Stats)]
        for f in ("cqref_histogram", "cqref_init", "cqref_kmeans", "cqref_map", "cqref_quantize", "cqref_wu_boxes",
                  "cqref_den_quotas"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} returned status {code}")
        self.code = code


def _check(fn: str, rc: int):
    if rc != OK:
        raise OracleError(fn, rc)


def splitmix64(seed: int, count: int) -> list[int]:
    s = ctypes.c_uint64(seed)
    return [lib().cqref_splitmix64_next(ctypes.byref(s)) for _ in range(count)]


def uniform_below(seed: int, T: int, count: int) -> list[int]:
    s = ctypes.c_uint64(seed)
    return [lib().cqref_uniform_below(ctypes.byref(s), T) for _ in range(count)]


def _img_args(img: np.ndarray):
    if img.dtype != np.uint8 or img.ndim != 3 or img.shape[2] != 3:
        raise ValueError("image must be uint8 [H, W, 3]")
    if not (img.strides[2] == 1 and img.strides[1] == 3):
        img = np.ascontiguousarray(img)
    return img, img.shape[0], img.shape[1], img.strides[0]


def histogram(img: np.ndarray, capacity: int | None = None, subsample: bool = False):
    """Unique colours (ascending 0xRRGGBB keys) and their pixel counts
    (optionally of the 2:1-subsampled image)."""
    img, H, W, stride = _img_args(img)
    cap = H * W if capacity is None else capacity
    keys = np.zeros(max(cap, 1), np.uint32)
    counts = np.zeros(max(cap, 1), np.uint32)
    n = ctypes.c_int64(0)
    rc = lib().cqref_histogram(_ptr(img), H, W, stride, int(bool(subsample)), _ptr(keys), _ptr(counts), cap,
                               ctypes.byref(n))
    if rc == ECAPACITY:
        raise OracleError("cqref_histogram", rc)
    _check("cqref_histogram", rc)
    return keys[: n.value].copy(), counts[: n.value].copy()


def init(keys: np.ndarray, counts: np.ndarray, K: int, scheme: int, seed: int):
    keys = np.ascontiguousarray(keys, np.uint32)
    counts = np.ascontiguousarray(counts, np.uint32)
    centers = np.zeros((K, 3), np.float64)
    k_used = ctypes.c_int32(0)
    _check("cqref_init", lib().cqref_init(_ptr(keys), _ptr(counts), len(keys), K, scheme, seed,
                                          _ptr(centers), ctypes.byref(k_used)))
    return centers, k_used.value


@dataclass
class KMeansResult:
    centers: np.ndarray
    assign: np.ndarray
    palette: np.ndarray
    sse_trace: np.ndarray
    stats: dict


def kmeans(keys, counts, centers0, max_iters: int, tol: float, prune: bool,
           assign0: np.ndarray | None = None) -> KMeansResult:
    keys = np.ascontiguousarray(keys, np.uint32)
    counts = np.ascontiguousarray(counts, np.uint32)
    centers = np.array(centers0, dtype=np.float64, copy=True).reshape(-1, 3)
    K = centers.shape[0]
    assign = (np.zeros(len(keys), np.uint8) if assign0 is None
              else np.array(assign0, dtype=np.uint8, copy=True))
    palette = np.zeros((K, 3), np.uint8)
    trace = np.zeros(max_iters, np.float64)
    st = Stats()
    _check("cqref_kmeans", lib().cqref_kmeans(_ptr(keys), _ptr(counts), len(keys), K,
                                              _ptr(centers), max_iters, tol, int(bool(prune)),
                                              _ptr(assign), _ptr(palette), _ptr(trace),
                                              ctypes.byref(st)))
    return KMeansResult(centers, assign, palette, trace[: st.iters].copy(), st.as_dict())


def map_image(img: np.ndarray, palette: np.ndarray):
    img, H, W, stride = _img_args(img)
    palette = np.ascontiguousarray(palette, np.uint8).reshape(-1, 3)
    idx = np.zeros((H, W), np.uint8)
    rgb = np.zeros((H, W, 3), np.uint8)
    err = ctypes.c_uint64(0)
    _check("cqref_map", lib().cqref_map(_ptr(img), H, W, stride, _ptr(palette), palette.shape[0],
                                        _ptr(idx), _ptr(rgb), ctypes.byref(err)))
    return idx, rgb, err.value


def quantize(img: np.ndarray, K: int, scheme: int, seed: int, max_iters: int, tol: float,
             prune: bool = True, want_images: bool = True, subsample: bool = False):
    img, H, W, stride = _img_args(img)
    palette = np.zeros((K, 3), np.uint8)
    idx = np.zeros((H, W), np.uint8) if want_images else None
    rgb = np.zeros((H, W, 3), np.uint8) if want_images else None
    st = Stats()
    _check("cqref_quantize", lib().cqref_quantize(_ptr(img), H, W, stride, int(bool(subsample)), K, scheme, seed,
                                                  max_iters, tol, int(bool(prune)), _ptr(palette),
                                                  _ptr(idx), _ptr(rgb), ctypes.byref(st)))
    return palette, idx, rgb, st.as_dict()


def sff_subset(K: int, n: int) -> int:
    """Size of the SFF subset: max(K, ceil(2 K ln K)), at most n."""
    return int(lib().cqref_sff_subset(K, n))


def wu_boxes(keys: np.ndarray, counts: np.ndarray, K: int) -> np.ndarray:
    """WU's boxes for K, in box index order: rows (lo_r, lo_g, lo_b, hi_r,
    hi_g, hi_b) over the 32 levels value >> 3, inclusive."""
    keys = np.ascontiguousarray(keys, np.uint32)
    counts = np.ascontiguousarray(counts, np.uint32)
    boxes = np.zeros((K, 6), np.int32)
    nb = ctypes.c_int32(0)
    _check("cqref_wu_boxes", lib().cqref_wu_boxes(_ptr(keys), _ptr(counts), len(keys), K, _ptr(boxes),
                                                  ctypes.byref(nb)))
    return boxes[: nb.value].copy()


def den_quotas(keys: np.ndarray, K: int) -> np.ndarray:
    """DEN's centres per cell (512 cells, (r >> 5) * 64 + (g >> 5) * 8 + (b >> 5))."""
    keys = np.ascontiguousarray(keys, np.uint32)
    quota = np.zeros(512, np.int32)
    _check("cqref_den_quotas", lib().cqref_den_quotas(_ptr(keys), len(keys), K, _ptr(quota)))
    return quota
