"""The seeded input generators are deterministic and have the stated shapes."""

import numpy as np

import workloads


def test_same_seed_same_bytes():
    a = workloads.float_signals(2001, 3, 10)
    b = workloads.float_signals(2001, 3, 10)
    assert a.dtype == np.float32 and a.shape == (3, 1024)
    assert a.tobytes() == b.tobytes()
    # signal i can be regenerated alone
    c = workloads.float_signals(2001, 1, 10, first=2)
    assert np.array_equal(c[0], a[2])
    assert not np.array_equal(a[0], a[1])


def test_int_range():
    x = workloads.int_signals(1002, 4, 12)
    assert x.dtype == np.int32 and x.min() == -128 and x.max() == 127


def test_outliers():
    x = workloads.outlier_signals(3001, 4, 12)
    frac = np.mean(np.abs(x) > 8)
    assert 0.004 < frac < 0.02
    bf = workloads.to_half_precision(x, "bf16")
    assert str(bf.dtype) == "torch.bfloat16"


def test_ragged_draw():
    k = workloads.ragged_log2_sizes()
    assert len(k) == 20000 and k.min() == 6 and k.max() == 20
    tot = int(np.sum(np.left_shift(np.int64(1), k.astype(np.int64))))
    assert tot == 1 << 30
    hist = np.bincount(k, minlength=21)[6:].tolist()
    assert hist == [12990, 487, 495, 489, 535, 494, 521, 480, 485, 488, 477,
                    507, 508, 543, 501]
    off = workloads.packed_offsets(k)
    assert off[-1] == 1 << 30 and off[0] == 0


def test_sign_diagonal():
    d = workloads.sign_diagonal(5002, 1 << 14)
    assert set(np.unique(d)) == {-1.0, 1.0}
