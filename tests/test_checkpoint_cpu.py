"""The committed network checkpoint is a valid integer network (CPU only)."""
import os

import numpy as np

from paper_2604_14411_amd.learn import load_checkpoint

HERE = os.path.dirname(os.path.abspath(__file__))


def test_checkpoint_is_a_valid_integer_network():
    q, w, ck = load_checkpoint(os.path.join(HERE, "..", "paper_2604_14411_amd", "mlp_v2.json"))
    assert ck["format"] == "hgp-mlp-1" and 1 <= q["k"] <= 8
    for key in ("w1", "w2", "w3"):
        assert np.abs(q[key]).max() <= 255
    for key in ("b1", "b2"):
        assert np.abs(q[key]).max() <= 2 ** 22
    assert abs(q["b3"]) <= 2 ** 22 and 0 <= q["r1"] <= 30 and 0 <= q["r2"] <= 30
    assert np.all(q["w1"][10:] == 0)
    # the training record names graphs that are not evaluation instances
    names = [g["graph"] for g in ck["train"]["graphs"]]
    assert names and all("8x(96x16x17)" not in n and "8x(42x30x30)" not in n for n in names)
    assert ck["train"]["loss"][-1] < ck["train"]["loss"][0]


# ------------------------------------------------------- binary checkpoint file
def _lib_or_skip():
    import pytest

    from paper_2604_14411_amd import hgp

    if not os.path.exists(hgp.LIB_PATH):
        pytest.skip("libhgp.so not built")
    return hgp


def _state(hgp, seed):
    rng = np.random.default_rng(seed)
    st = hgp.train_state(hgp.mlp_init(seed), seed=seed)
    m = hgp.f32_from_dict({k: (rng.standard_normal(np.shape(v)).astype(np.float32) if k != "b3" else 0.25)
                           for k, v in hgp.mlp_init(1).items()})
    st.m = m
    st.v = hgp.f32_from_dict({k: (rng.random(np.shape(v)).astype(np.float32) if k != "b3" else 0.5)
                              for k, v in hgp.mlp_init(2).items()})
    st.step, st.epoch, st.rng = 1234, 5, 0xDEADBEEF12345678
    return st


def _int_net():
    q, _, _ = load_checkpoint(os.path.join(HERE, "..", "paper_2604_14411_amd", "mlp_v2.json"))
    return q


def test_binary_checkpoint_round_trip_and_layout(tmp_path):
    import struct
    import zlib

    hgp = _lib_or_skip()
    st = _state(hgp, 3)
    q = _int_net()
    path = str(tmp_path / "net.hgpmlp")
    hgp.mlp_save(path, st, q, score_shift=-7)
    raw = open(path, "rb").read()
    # header fields, sizes and the CRC-32 (IEEE) recomputed by zlib
    magic, ver, hb, fin, hid, npar, sec, shift, res, pay = struct.unpack("<8sIIIIIIiIQ", raw[:48])
    assert magic == b"HGPMLP\0\0" and ver == 1 and hb == 48 and (fin, hid) == (16, 64)
    assert npar == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1 and sec == 3 and shift == -7 and res == 0
    state_bytes = 3 * 4 * npar + 24
    int_bytes = 4 * (4 + 16 * 64 + 64 + 64 * 64 + 64 + 64)
    assert pay == state_bytes + int_bytes and len(raw) == 48 + pay + 4
    assert struct.unpack("<I", raw[-4:])[0] == zlib.crc32(raw[:-4])
    # the stored weights are the state's floats, in order
    w = np.frombuffer(raw[48:48 + 4 * npar], dtype="<f4")
    assert np.array_equal(w[:16 * 64], np.ctypeslib.as_array(st.w.w1))
    st2, q2, sh2 = hgp.mlp_load(path)
    assert bytes(st2) == bytes(st) or (
        bytes(st2.w) == bytes(st.w) and bytes(st2.m) == bytes(st.m) and bytes(st2.v) == bytes(st.v))
    assert (st2.step, st2.epoch, st2.rng) == (st.step, st.epoch, st.rng)
    for k in ("k", "r1", "r2", "b3"):
        assert q2[k] == q[k]
    for k in ("w1", "b1", "w2", "b2", "w3"):
        assert np.array_equal(np.asarray(q2[k]).reshape(-1), np.asarray(q[k]).reshape(-1))
    assert sh2 == -7


def test_binary_checkpoint_sections(tmp_path):
    hgp = _lib_or_skip()
    only_net = str(tmp_path / "net.hgpmlp")
    hgp.mlp_save(only_net, None, _int_net(), 3)
    st, q, sh = hgp.mlp_load(only_net, state=False)
    assert st is None and q is not None and sh == 3
    import pytest

    with pytest.raises(hgp.HgpError) as e:
        hgp.mlp_load(only_net, state=True)
    assert e.value.code == hgp.EFORMAT
    only_state = str(tmp_path / "state.hgpmlp")
    hgp.mlp_save(only_state, _state(hgp, 4), None, 0)
    st, q, _ = hgp.mlp_load(only_state, network=False)
    assert st.step == 1234 and q is None
    with pytest.raises(hgp.HgpError) as e:
        hgp.mlp_save(str(tmp_path / "none"), None, None, 0)
    assert e.value.code == hgp.EINVAL
    bad = _int_net()
    bad["w2"] = np.array(bad["w2"]).copy()
    bad["w2"][0, 0] = 300
    with pytest.raises(hgp.HgpError) as e:
        hgp.mlp_save(str(tmp_path / "bad"), None, bad, 0)
    assert e.value.code == hgp.EINVAL


def test_binary_checkpoint_rejects_damaged_files(tmp_path):
    import struct
    import zlib

    import pytest

    hgp = _lib_or_skip()
    path = str(tmp_path / "net.hgpmlp")
    hgp.mlp_save(path, _state(hgp, 5), _int_net(), 0)
    raw = bytearray(open(path, "rb").read())

    def expect(data, code, name):
        p = str(tmp_path / name)
        open(p, "wb").write(bytes(data))
        with pytest.raises(hgp.HgpError) as e:
            hgp.mlp_load(p)
        assert e.value.code == code, name

    flipped = bytearray(raw)
    flipped[100] ^= 0x10
    expect(flipped, hgp.EFORMAT, "flipped")
    expect(raw[:-9], hgp.EFORMAT, "truncated")
    expect(raw + b"\0", hgp.EFORMAT, "trailing")
    magic = bytearray(raw)
    magic[0:1] = b"X"
    expect(magic, hgp.EFORMAT, "magic")

    def with_header(off, fmt, value, name):
        d = bytearray(raw)
        struct.pack_into(fmt, d, off, value)
        struct.pack_into("<I", d, len(d) - 4, zlib.crc32(bytes(d[:-4])))  # a valid CRC: the field itself is checked
        expect(d, hgp.EFORMAT, name)

    with_header(8, "<I", 2, "version")
    with_header(20, "<I", 32, "hidden")
    with_header(28, "<I", 4, "sections")
    with_header(40, "<Q", 10, "payload")
    with pytest.raises(hgp.HgpError) as e:
        hgp.mlp_load(str(tmp_path / "missing.hgpmlp"))
    assert e.value.code == hgp.EIO
