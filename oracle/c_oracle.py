"""ctypes loader for the plain-C cascade in chw_oracle.c.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The shared object liborc_chw.so is built next to its source with gcc (by the
repository's build step, or here on first use when it is missing).  It is a
separate, self-contained library: nothing from the GPU library is linked in.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chw_oracle.c")
_LIB = os.path.join(_HERE, "liborc_chw.so")
# ORC_CHW_LIBRARY names another build of the same source (the sanitizer build
# of the host checks); it is loaded as it is, never rebuilt here
_LIB_OVERRIDE = os.environ.get("ORC_CHW_LIBRARY")
_lib = None


def build_sanitized(path):
    """Compile chw_oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
    (clang, sharing the sanitizer runtime of the library's host build) into
    `path`."""
    clang = "/opt/rocm/llvm/bin/clang"
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.check_call([clang, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-fno-fast-math", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-shared-libsan",
                           "-fno-omit-frame-pointer", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, path)
    return path


def build(force=False):
    """Compile chw_oracle.c into liborc_chw.so (plain gcc, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-pthread", "-fno-fast-math", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build()
            lib = ctypes.CDLL(_LIB)
        for name, ptr in (("orc_chw_batch_f64", ctypes.c_double),
                          ("orc_chw_batch_i64", ctypes.c_int64)):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.POINTER(ptr), ctypes.POINTER(ptr),
                           ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                           ctypes.c_int, ctypes.c_int]
        _lib = lib
    return _lib


def chw_batch(x, log2_sizes, offsets=None, adjoint=False, threads=1, out=None):
    """Apply the CHW cascade (or its adjoint) to every signal of a packed batch.

    x: 1-D float64 or int64 array holding all signals; signal i occupies
    x[offsets[i] : offsets[i] + 2^log2_sizes[i]].  offsets=None packs the
    signals back to back.  Elements outside every signal are copied through
    unchanged.  Returns the transformed array (float64 orthonormal, or int64
    unnormalized).
    """
    lib = _load()
    x = np.ascontiguousarray(x)
    if np.issubdtype(x.dtype, np.integer):
        x = x.astype(np.int64, copy=False)
        fn, ct = lib.orc_chw_batch_i64, ctypes.c_int64
    else:
        x = x.astype(np.float64, copy=False)
        fn, ct = lib.orc_chw_batch_f64, ctypes.c_double
    sizes = np.ascontiguousarray(log2_sizes, dtype=np.int32)
    if offsets is None:
        offsets = np.zeros(len(sizes), dtype=np.int64)
        if len(sizes) > 1:
            offsets[1:] = np.cumsum(np.left_shift(np.int64(1), sizes[:-1].astype(np.int64)))
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    y = np.array(x, copy=True) if out is None else out
    rc = fn(x.ctypes.data_as(ctypes.POINTER(ct)), y.ctypes.data_as(ctypes.POINTER(ct)),
            sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ctypes.c_int64(len(sizes)), ctypes.c_int(1 if adjoint else 0),
            ctypes.c_int(int(threads)))
    if rc != 0:
        raise RuntimeError("C oracle failed with status %d" % rc)
    return y


def chw_rows(x2d, adjoint=False, threads=1):
    """Convenience: transform each row of a (batch, 2^m) array."""
    x2d = np.asarray(x2d)
    b, n = x2d.shape
    m = n.bit_length() - 1
    flat = chw_batch(x2d.reshape(-1), np.full(b, m, dtype=np.int32),
                     adjoint=adjoint, threads=threads)
    return flat.reshape(b, n)
