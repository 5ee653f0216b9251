"""Checkpoint file format (host side): round trip of FP64 and FP32 states
with their header, and rejection of a foreign file, a damaged state and a
truncated file."""
import numpy as np
import pytest

from paper_2604_02125_amd import checkpoint


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_round_trip(tmp_path, dtype):
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 6, 16)).astype(dtype)
    head = dict(config=dict(nx=3, ny=2, degree=3), t=1.25, step=17, extra={"note": "x"})
    p = str(tmp_path / "a.ckpt")
    checkpoint.write_file(p, head, u)
    h, v = checkpoint.read_file(p)
    assert v.dtype == dtype and v.shape == u.shape and np.array_equal(v, u)
    assert h["t"] == 1.25 and h["step"] == 17 and h["config"]["nx"] == 3 and h["extra"]["note"] == "x"
    assert h["version"] == checkpoint.VERSION


def test_rejects_damage(tmp_path):
    u = np.arange(24, dtype=np.float64).reshape(2, 3, 4)
    p = str(tmp_path / "b.ckpt")
    checkpoint.write_file(p, {"t": 0.0}, u)
    data = bytearray(open(p, "rb").read())
    bad = str(tmp_path / "bad.ckpt")
    data[-3] ^= 0x40                                   # one flipped bit in the state
    open(bad, "wb").write(bytes(data))
    with pytest.raises(ValueError, match="checksum"):
        checkpoint.read_file(bad)
    open(bad, "wb").write(bytes(data[:-8]))            # truncated
    with pytest.raises(ValueError, match="bytes"):
        checkpoint.read_file(bad)
    open(bad, "wb").write(b"NOTACKPT" + bytes(data[8:]))
    with pytest.raises(ValueError, match="not a checkpoint"):
        checkpoint.read_file(bad)
    with pytest.raises(ValueError):
        checkpoint.write_file(p, {}, np.zeros(3, dtype=np.int32))
