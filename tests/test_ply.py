"""PLY reader/writer of the standard 3DGS layout (CPU)."""
import numpy as np
import pytest

from paper_2603_16103_amd.ply import FIELDS, read_ply, write_ply
from paper_2603_16103_amd.synth import gen_scene


def test_round_trip_is_exact(tmp_path):
    sc = gen_scene(1000, 3)
    p = tmp_path / "scene.ply"
    write_ply(str(p), sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    got = read_ply(str(p))
    for a, b in zip(got, (sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)):
        assert a.dtype == np.float32 and a.shape == b.shape
        assert np.array_equal(a.view(np.uint32), np.asarray(b, np.float32).view(np.uint32))


def test_layout_is_the_standard_one(tmp_path):
    sc = gen_scene(5, 4)
    p = tmp_path / "s.ply"
    write_ply(str(p), sc.pos, sc.log_scale, sc.rot, sc.opacity, sc.sh)
    raw = p.read_bytes()
    head, body = raw.split(b"end_header\n", 1)
    props = [ln.split()[-1].decode() for ln in head.splitlines() if ln.startswith(b"property")]
    assert props == FIELDS and len(FIELDS) == 62
    assert len(body) == 5 * 62 * 4
    rec = np.frombuffer(body, dtype="<f4").reshape(5, 62)
    np.testing.assert_array_equal(rec[:, 0:3], sc.pos)
    np.testing.assert_array_equal(rec[:, 6:54], sc.sh)     # f_dc then f_rest
    np.testing.assert_array_equal(rec[:, 54], sc.opacity)
    np.testing.assert_array_equal(rec[:, 55:58], sc.log_scale)
    np.testing.assert_array_equal(rec[:, 58:62], sc.rot)


def test_reader_accepts_extra_properties_and_rejects_ascii(tmp_path):
    sc = gen_scene(7, 5)
    extra = FIELDS[:6] + ["red"] + FIELDS[6:]
    n = 7
    dt = np.dtype([(f, "<f4") for f in extra])
    rec = np.zeros(n, dtype=dt)
    rec["x"], rec["y"], rec["z"] = sc.pos.T
    for i in range(48):
        rec[f"f_dc_{i}" if i < 3 else f"f_rest_{i - 3}"] = sc.sh[:, i]
    rec["opacity"] = sc.opacity
    for i in range(3):
        rec[f"scale_{i}"] = sc.log_scale[:, i]
    for i in range(4):
        rec[f"rot_{i}"] = sc.rot[:, i]
    p = tmp_path / "e.ply"
    hdr = "ply\nformat binary_little_endian 1.0\nelement vertex 7\n"
    hdr += "".join(f"property float {f}\n" for f in extra) + "end_header\n"
    p.write_bytes(hdr.encode() + rec.tobytes())
    pos, ls, rot, op, sh = read_ply(str(p))
    np.testing.assert_array_equal(sh, sc.sh)
    np.testing.assert_array_equal(rot, sc.rot)
    q = tmp_path / "a.ply"
    q.write_bytes(b"ply\nformat ascii 1.0\nelement vertex 0\nend_header\n")
    with pytest.raises(ValueError):
        read_ply(str(q))
