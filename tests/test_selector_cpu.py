"""CPU checks of the selector model file: the writer's layout and the
library's loader rejecting damaged files before any device work."""
import ctypes
import struct

import numpy as np

from paper_1902_02250_amd import bltc, selector


def _write(tmp_path, **kw):
    k = selector.K
    params = np.arange(selector.bltc_param_count(k), dtype=np.float32) * 1e-4
    path = str(tmp_path / "m.bin")
    selector.write_model(path, params, np.zeros(12), np.ones(12), 0.25, **kw)
    return path, params


def test_model_layout(tmp_path):
    path, params = _write(tmp_path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"BLTCSEL1"
    assert struct.unpack("<4i", raw[8:24]) == (1, 12, 64, selector.K)
    k = selector.K
    off = 24 + 4 * k + 8 * k
    assert struct.unpack("<4d", raw[off:off + 32]) == (selector.THETA_REF, selector.COST_FAR,
                                                      selector.COST_NEAR, 0.25)
    assert len(raw) == off + 32 + 96 + 4 * params.size + 8
    assert struct.unpack("<Q", raw[-8:])[0] == selector._fnv1a(raw[:-8])
    assert bltc.mlp_params(k) == params.size


def _status(path):
    h = ctypes.c_void_p()
    rc = bltc.load().bltc_selector_load(path.encode(), ctypes.byref(h))
    assert h.value is None
    return bltc.STATUS[rc]


def test_loader_rejects_damage(tmp_path):
    path, _ = _write(tmp_path)
    raw = bytearray(open(path, "rb").read())
    bad = tmp_path / "bad.bin"
    for mutate in (lambda b: b.__setitem__(100, b[100] ^ 1),      # checksum
                   lambda b: b.__setitem__(0, ord("X")),         # magic
                   lambda b: b.__setitem__(8, 2)):               # version
        b = bytearray(raw)
        mutate(b)
        bad.write_bytes(bytes(b))
        assert _status(str(bad)) == "EMODEL"
    bad.write_bytes(bytes(raw[:-20]))                            # truncated
    assert _status(str(bad)) == "EMODEL"
    bad.write_bytes(bytes(raw) + b"\0")                          # trailing bytes
    assert _status(str(bad)) == "EMODEL"
    assert _status(str(tmp_path / "missing.bin")) == "EMODEL"
    path2, _ = _write(tmp_path, cand=[(13, 0.5)] * selector.K)   # degree out of range
    assert _status(path2) == "EMODEL"
