"""FP64 CPU oracle for FSR (test infrastructure): the block-independent
method and the sequential variant that reuses reconstructed pixels.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``fsr_oracle.c`` (plain C,
double precision) through ctypes and shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsr_oracle.c")
_LIB = os.path.join(_HERE, "libfsr_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libfsr_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u16p = ctypes.POINTER(ctypes.c_uint16)
        i64p = ctypes.POINTER(ctypes.c_int64)
        c_int, c_long, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_double
        lib.fsro_twiddles.argtypes = [c_int, dp, dp]
        lib.fsro_spatial_weight.argtypes = [c_int, c_double, u8p, dp]
        lib.fsro_freq_weight.argtypes = [c_int, dp]
        lib.fsro_dft2_real.argtypes = [c_int, dp, dp, dp]
        lib.fsro_block.argtypes = [c_int, c_int, c_double, c_double, c_int, dp, u8p,
                                   dp, dp, dp, dp, u16p, dp, dp]
        lib.fsro_block.restype = c_int
        lib.fsro_model_pixel.argtypes = [c_int, dp, dp, c_int, c_int]
        lib.fsro_model_pixel.restype = c_double
        lib.fsro_reconstruct.argtypes = [dp, u8p, dp, c_int, c_int, c_long, c_int, c_int, c_int,
                                         c_double, c_double, c_int, u16p, dp, c_int]
        lib.fsro_reconstruct.restype = c_long
        lib.fsro_reconstruct_blocks.argtypes = [dp, u8p, c_int, c_int, c_long, c_int, c_int,
                                                c_int, c_double, c_double, c_int, i64p, c_long,
                                                dp, u16p, dp, dp, c_int]
        lib.fsro_reconstruct_blocks.restype = c_long
        lib.fsro_block_weighted.argtypes = [c_int, c_int, c_double, c_int, dp, dp,
                                            dp, dp, dp, dp, u16p, dp, dp]
        lib.fsro_block_weighted.restype = c_int
        lib.fsro_reconstruct_reuse.argtypes = [dp, u8p, dp, c_int, c_int, c_long, c_int, c_int,
                                               c_int, c_double, c_double, c_double, c_int, u16p]
        lib.fsro_reconstruct_reuse.restype = c_long
        lib.fsro_reconstruct_reuse_given.argtypes = [dp, u8p, dp, dp, c_int, c_int, c_long, c_int,
                                                     c_int, c_int, c_double, c_double, c_double,
                                                     c_int, u16p, c_int]
        lib.fsro_reconstruct_reuse_given.restype = c_long
        lib.fsro_max_threads.restype = c_int
        _lib = lib
    return _lib


def _p(a, ctype):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(np.asarray(a) != 0, dtype=np.uint8)


def twiddles(S: int) -> np.ndarray:
    tr, ti = np.empty(S), np.empty(S)
    _load().fsro_twiddles(S, _p(tr, ctypes.c_double), _p(ti, ctypes.c_double))
    return tr + 1j * ti


def spatial_weight(known: np.ndarray, rho: float) -> np.ndarray:
    k = _u8(known)
    S = k.shape[0]
    w = np.empty((S, S))
    _load().fsro_spatial_weight(S, rho, _p(k, ctypes.c_uint8), _p(w, ctypes.c_double))
    return w


def freq_weight(S: int) -> np.ndarray:
    wf = np.empty((S, S))
    _load().fsro_freq_weight(S, _p(wf, ctypes.c_double))
    return wf


def dft2_real(x: np.ndarray) -> np.ndarray:
    x = _f64(x)
    S = x.shape[0]
    Xr, Xi = np.empty((S, S)), np.empty((S, S))
    _load().fsro_dft2_real(S, _p(x, ctypes.c_double), _p(Xr, ctypes.c_double),
                           _p(Xi, ctypes.c_double))
    return Xr + 1j * Xi


def dft2_real_parts(x: np.ndarray):
    """Like :func:`dft2_real` but returns the (re, im) arrays as computed."""
    x = _f64(x)
    S = x.shape[0]
    Xr, Xi = np.empty((S, S)), np.empty((S, S))
    _load().fsro_dft2_real(S, _p(x, ctypes.c_double), _p(Xr, ctypes.c_double),
                           _p(Xi, ctypes.c_double))
    return Xr, Xi


def block(ft: np.ndarray, known: np.ndarray, iters: int, rho: float, gamma: float,
          tie_larger: bool = False):
    """Run O2-O6 on one S x S support block.

    Returns a dict with the final model ``G`` and residual ``R`` (complex
    S x S), the per-iteration picks ``idx`` (u*S + v), the projection
    coefficients ``p`` (complex), the winning objectives ``obj`` and their
    relative separations ``sep`` from the next objective (the winner's
    exactly tied conjugate passed over), and ``empty`` (no known pixel)."""
    ft = _f64(ft)
    k = _u8(known)
    S = ft.shape[0]
    Gr, Gi, Rr, Ri = (np.empty((S, S)) for _ in range(4))
    idx = np.empty(max(iters, 1), np.uint16)
    p = np.empty(2 * max(iters, 1))
    sep = np.empty(2 * max(iters, 1))
    D = ctypes.c_double
    empty = _load().fsro_block(S, iters, rho, gamma, int(tie_larger), _p(ft, D),
                               _p(k, ctypes.c_uint8), _p(Gr, D), _p(Gi, D), _p(Rr, D),
                               _p(Ri, D), _p(idx, ctypes.c_uint16), _p(p, D), _p(sep, D))
    return {"G": Gr + 1j * Gi, "R": Rr + 1j * Ri, "Gr": Gr, "Gi": Gi, "Rr": Rr, "Ri": Ri,
            "idx": idx[:iters].copy(), "p": (p[0::2] + 1j * p[1::2])[:iters],
            "obj": sep[0::2][:iters].copy(), "sep": sep[1::2][:iters].copy(),
            "empty": bool(empty)}


def block_weighted(ft: np.ndarray, w: np.ndarray, iters: int, gamma: float,
                   tie_larger: bool = False):
    """Run O3-O6 on one support block with a given spatial weight ``w``
    (S x S).  Returns the same dict as :func:`block`."""
    ft = _f64(ft)
    w = _f64(w)
    S = ft.shape[0]
    Gr, Gi, Rr, Ri = (np.empty((S, S)) for _ in range(4))
    idx = np.empty(max(iters, 1), np.uint16)
    p = np.empty(2 * max(iters, 1))
    D = ctypes.c_double
    empty = _load().fsro_block_weighted(S, iters, gamma, int(tie_larger), _p(ft, D), _p(w, D),
                                        _p(Gr, D), _p(Gi, D), _p(Rr, D), _p(Ri, D),
                                        _p(idx, ctypes.c_uint16), _p(p, D), None)
    return {"G": Gr + 1j * Gi, "R": Rr + 1j * Ri, "Gr": Gr, "Gi": Gi, "Rr": Rr, "Ri": Ri,
            "idx": idx[:iters].copy(), "p": (p[0::2] + 1j * p[1::2])[:iters],
            "empty": bool(empty)}


def model_pixel(G: np.ndarray, m: int, n: int) -> float:
    S = G.shape[0]
    Gr, Gi = _f64(G.real), _f64(G.imag)
    return _load().fsro_model_pixel(S, _p(Gr, ctypes.c_double), _p(Gi, ctypes.c_double), m, n)


def reconstruct(image: np.ndarray, mask: np.ndarray, iters: int, block_size: int = 4,
                border: int = 14, rho: float = 0.7, gamma: float = 0.5,
                tie_larger: bool = False, log: bool = False, threads: int = 0,
                separations: bool = False):
    """Whole-image FP64 reconstruction.  Returns ``(out, log_idx, n_empty)``;
    ``log_idx`` is an (N, I) uint16 array when ``log`` is set, else None.
    With ``separations`` a fourth item holds the (N, I) winning objectives
    and the (N, I) relative separations of each pick (see :func:`block`)."""
    img = _f64(image)
    m = _u8(mask)
    H, W = img.shape
    B = block_size
    N = (-(-H // B)) * (-(-W // B))
    out = np.empty_like(img)
    lg = np.empty((N, max(iters, 1)), np.uint16) if log else None
    ls = np.empty((N, max(iters, 1), 2)) if separations else None
    n_empty = _load().fsro_reconstruct(_p(img, ctypes.c_double), _p(m, ctypes.c_uint8),
                                       _p(out, ctypes.c_double), H, W, W, B, border, iters,
                                       rho, gamma, int(tie_larger), _p(lg, ctypes.c_uint16),
                                       _p(ls, ctypes.c_double), threads)
    if lg is not None:
        lg = lg[:, :iters]
    if separations:
        return out, lg, int(n_empty), (ls[:, :iters, 0].copy(), ls[:, :iters, 1].copy())
    return out, lg, int(n_empty)


def reconstruct_blocks(image: np.ndarray, mask: np.ndarray, block_ids, iters: int,
                       block_size: int = 4, border: int = 14, rho: float = 0.7,
                       gamma: float = 0.5, tie_larger: bool = False, log: bool = False,
                       log_p: bool = False, threads: int = 0):
    """FP64 reconstruction of selected blocks.  Returns ``(targets, log_idx,
    p, n_empty)``; ``targets`` is (n, B, B) with NaN outside the image."""
    img = _f64(image)
    m = _u8(mask)
    H, W = img.shape
    B = block_size
    ids = np.ascontiguousarray(block_ids, dtype=np.int64)
    n = ids.shape[0]
    tg = np.empty((n, B, B))
    lg = np.empty((n, max(iters, 1)), np.uint16) if log else None
    lp = np.empty((n, max(iters, 1), 2)) if log_p else None
    n_empty = _load().fsro_reconstruct_blocks(
        _p(img, ctypes.c_double), _p(m, ctypes.c_uint8), H, W, W, B, border, iters, rho, gamma,
        int(tie_larger), _p(ids, ctypes.c_int64), n, _p(tg, ctypes.c_double),
        _p(lg, ctypes.c_uint16), _p(lp, ctypes.c_double), None, threads)
    if lg is not None:
        lg = lg[:, :iters]
    p = None if lp is None else (lp[:, :iters, 0] + 1j * lp[:, :iters, 1])
    return tg, lg, p, int(n_empty)


def reconstruct_reuse(image: np.ndarray, mask: np.ndarray, iters: int, delta: float = 0.5,
                      block_size: int = 4, border: int = 14, rho: float = 0.7,
                      gamma: float = 0.5, tie_larger: bool = False, log: bool = False):
    """Sequential FP64 reconstruction that reuses reconstructed pixels (O9):
    blocks in raster order, missing pixels of earlier blocks' targets taking
    part with their reconstruction and the weight ``delta`` rho^dist.
    Returns ``(out, log_idx, n_empty)`` like :func:`reconstruct`."""
    img = _f64(image)
    m = _u8(mask)
    H, W = img.shape
    B = block_size
    N = (-(-H // B)) * (-(-W // B))
    out = np.zeros_like(img)
    lg = np.empty((N, max(iters, 1)), np.uint16) if log else None
    n_empty = _load().fsro_reconstruct_reuse(_p(img, ctypes.c_double), _p(m, ctypes.c_uint8),
                                             _p(out, ctypes.c_double), H, W, W, B, border, iters,
                                             rho, gamma, delta, int(tie_larger),
                                             _p(lg, ctypes.c_uint16))
    if lg is not None:
        lg = lg[:, :iters]
    return out, lg, int(n_empty)


def reconstruct_reuse_given(image: np.ndarray, mask: np.ndarray, reused: np.ndarray, iters: int,
                            delta: float = 0.5, block_size: int = 4, border: int = 14,
                            rho: float = 0.7, gamma: float = 0.5, tie_larger: bool = False,
                            log: bool = False, threads: int = 0):
    """Every block of the sequential variant on its own, its reused pixels
    taken from the frame ``reused`` (same shape as ``image``) rather than
    from the oracle's own earlier blocks.  Returns ``(out, log_idx, n_empty)``
    like :func:`reconstruct_reuse`; fed that function's own output it
    returns the same output and log."""
    img = _f64(image)
    m = _u8(mask)
    src = _f64(reused)
    H, W = img.shape
    assert src.shape == img.shape
    B = block_size
    N = (-(-H // B)) * (-(-W // B))
    out = np.zeros_like(img)
    lg = np.empty((N, max(iters, 1)), np.uint16) if log else None
    n_empty = _load().fsro_reconstruct_reuse_given(
        _p(img, ctypes.c_double), _p(m, ctypes.c_uint8), _p(src, ctypes.c_double),
        _p(out, ctypes.c_double), H, W, W, B, border, iters, rho, gamma, delta, int(tie_larger),
        _p(lg, ctypes.c_uint16), threads)
    if lg is not None:
        lg = lg[:, :iters]
    return out, lg, int(n_empty)


def max_threads() -> int:
    return int(_load().fsro_max_threads())
