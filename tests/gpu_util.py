"""Helpers for the GPU tests: move seeded inputs to the device, run the HIP
path through the binding, and compare with the oracle."""

import numpy as np

from oracle import c_oracle, metrics

TOL = {"f32": 1e-5, "bf16": 4e-3, "f16": 4e-3, "f64": 1e-13}
TORCH_DT = {"f32": "float32", "bf16": "bfloat16", "f16": "float16", "i32": "int32",
            "f64": "float64"}


def torch():
    import torch as t
    return t


def dev_tensor(a, dtype):
    """numpy array (or torch CPU tensor) -> contiguous device tensor of dtype."""
    t = torch()
    if isinstance(a, np.ndarray):
        a = t.from_numpy(np.ascontiguousarray(a))
    return a.to(getattr(t, TORCH_DT[dtype])).contiguous().to("cuda")


def host_f64(t):
    """device/CPU tensor -> float64 numpy (exact for every supported dtype)."""
    tt = torch()
    return t.detach().to("cpu").to(tt.float64).numpy()


def host_i64(t):
    tt = torch()
    return t.detach().to("cpu").to(tt.int64).numpy()


def oracle_packed(x_flat, log2_sizes, offsets=None, adjoint=False, threads=8):
    """Oracle on a flat array (float64 or int64) with the plan's layout."""
    offs = None if offsets is None else np.asarray(offsets[:-1], dtype=np.int64)
    return c_oracle.chw_batch(x_flat, np.asarray(log2_sizes, dtype=np.int32), offs,
                              adjoint=adjoint, threads=threads)


def per_signal_rel(y_hat, y_ref, log2_sizes, offsets=None):
    """Per-signal relative L2 of flat arrays laid out by sizes/offsets."""
    sizes = np.asarray(log2_sizes, dtype=np.int64)
    if offsets is None:
        offs = np.zeros(len(sizes), dtype=np.int64)
        if len(sizes) > 1:
            offs[1:] = np.cumsum(np.left_shift(1, sizes[:-1]))
    else:
        offs = np.asarray(offsets[:-1], dtype=np.int64)
    out = np.empty(len(sizes))
    for i, (k, o) in enumerate(zip(sizes, offs)):
        n = 1 << int(k)
        out[i] = metrics.rel_l2(y_hat[o:o + n], y_ref[o:o + n])
    return out


def rne_narrow(t32, dtype):
    """float32 tensor -> bf16 / f16 by torch's round-to-nearest-even
    conversion, done on the CPU (c10's software rounding, independent of the
    kernels' converts)."""
    tt = torch()
    return t32.detach().to("cpu").to(getattr(tt, TORCH_DT[dtype]))


def narrowing_mismatches(y_half, y32, dtype):
    """Elements where a bf16 / f16 result differs, bit for bit, from the RNE
    narrowing of the float32 result of the same stages: 0 when the narrowing
    is round to nearest even."""
    tt = torch()
    want = rne_narrow(y32, dtype).view(tt.int16)
    got = y_half.detach().to("cpu").view(tt.int16)
    if got.shape != want.shape:
        raise ValueError("shapes differ: %s vs %s" % (tuple(got.shape), tuple(want.shape)))
    return int((got != want).sum())
