"""Pins of the oracle's counter-based generator against numpy's Philox4x64-10 and the
published known-answer vector (Salmon et al., SC'11, Random123 KAT)."""
import numpy as np

from oracle import philox


def test_known_answer_zero():
    assert philox.philox4x64_int((0, 0, 0, 0), (0, 0)) == (
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B)


def test_matches_numpy_philox_raw_stream():
    # numpy advances its counter before each block, so raw block b uses counter b + 1.
    for key in ((5, 7), (philox.MASK64, 123456789), (0x191001031, 0)):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array([0, 11, 22, 33], dtype=np.uint64))
        raw = bg.random_raw(4 * 64)
        c0 = np.arange(1, 65, dtype=np.uint64)
        out = philox.philox4x64(c0, 11, 22, 33, key[0], key[1])
        mine = np.stack(out, axis=1).reshape(-1)
        assert np.array_equal(mine, raw)


def test_vectorised_equals_integer_reference():
    c = np.array([0, 1, 2**40 + 3, 2**63 + 5], dtype=np.uint64)
    out = philox.philox4x64(c, 9, 2**60, 77, 0xDEADBEEF, 3)
    for i, ci in enumerate(c):
        ref = philox.philox4x64_int((int(ci), 9, 2**60, 77), (0xDEADBEEF, 3))
        assert tuple(int(w[i]) for w in out) == ref


def test_normals_are_standard():
    z = philox.normals(200_000, 42, 3, philox.TAG_MODEL_ERROR, 0, 1)
    assert abs(z.mean()) < 4 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / len(z))
    # streams differ by every counter word
    a = philox.normals(64, 42, 3, philox.TAG_XI, 0, 1)
    for args in ((43, 3, philox.TAG_XI, 0, 1), (42, 4, philox.TAG_XI, 0, 1),
                 (42, 3, philox.TAG_NU, 0, 1), (42, 3, philox.TAG_XI, 1, 1),
                 (42, 3, philox.TAG_XI, 0, 2)):
        assert not np.allclose(a, philox.normals(64, *args))


def test_box_muller_lane_order():
    x = philox.philox4x64(np.arange(2, dtype=np.uint64), *philox.counter_words(5, 2, 0, 3), 99, 0)
    z = philox.normals(8, 99, 5, 2, 0, 3)
    a0, a1 = philox.box_muller(x[0], x[1])
    a2, a3 = philox.box_muller(x[2], x[3])
    assert np.array_equal(z[0::4], a0) and np.array_equal(z[1::4], a1)
    assert np.array_equal(z[2::4], a2) and np.array_equal(z[3::4], a3)
