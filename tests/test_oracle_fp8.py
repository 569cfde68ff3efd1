"""Pins of the E4M3 rounding of the oracle (FP8 storage of H and S), CPU only.

F1  the decoded table: 127 distinct non-negative finite values, 2^-9 the
    smallest subnormal, 2^-6 the smallest normal, 448 the largest;
F2  rounding equals torch's float32 -> float8_e4m3fn conversion on inputs that
    are exact in float32 (so torch's float32 path rounds once), over random
    magnitudes from the subnormals to 448, and on every midpoint between
    neighbouring values (ties to even);
F3  worked values: 0.1 -> 0.1015625, 17 -> 16 (tie, even mantissa), 2^-10 -> 0
    (tie), 3 2^-10 -> 2^-8 (tie), 460 -> 448, 465 overflows, -0.0 keeps its sign.
"""
import numpy as np
import pytest

from oracle import fp8

torch = pytest.importorskip("torch")


def test_f1_table():
    v = fp8.VALUES
    assert len(np.unique(v)) == 127 and np.all(np.diff(v) > 0)
    assert v[1] == 2.0 ** -9 and v[8] == 2.0 ** -6 and v[-1] == 448.0


def _torch_codes(x32):
    return torch.from_numpy(x32).to(torch.float8_e4m3fn).view(torch.uint8).numpy()


def test_f2_matches_torch_on_float32_inputs():
    rng = np.random.default_rng(0)
    mag = 2.0 ** rng.uniform(-11, np.log2(447.0), 200000)
    x32 = (mag * rng.choice([-1.0, 1.0], mag.size)).astype(np.float32)
    codes, over = fp8.round_e4m3(x32.astype(np.float64))
    assert not over.any()
    assert np.array_equal(codes, _torch_codes(x32))
    mids = ((fp8.VALUES[:-1] + fp8.VALUES[1:]) / 2.0).astype(np.float32)
    assert np.array_equal(mids.astype(np.float64), (fp8.VALUES[:-1] + fp8.VALUES[1:]) / 2.0)
    codes, _ = fp8.round_e4m3(mids.astype(np.float64))
    assert np.array_equal(codes, _torch_codes(mids))
    assert np.all(codes % 2 == 0)


def test_f3_worked_values():
    x = np.array([0.1, 17.0, 2.0 ** -10, 3 * 2.0 ** -10, 460.0, 465.0, -0.0, -3.0])
    codes, over = fp8.round_e4m3(x)
    vals = fp8.decode(codes)
    assert vals[0] == 0.1015625 and vals[1] == 16.0 and vals[2] == 0.0 and vals[3] == 2.0 ** -8
    assert vals[4] == 448.0 and over[5] and not over[4]
    assert codes[6] == 0x80 and vals[7] == -3.0
