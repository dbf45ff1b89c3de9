"""CPU checks of the selector model file: the writer's layout and the
library's loader rejecting damaged files before any device work."""
import ctypes
import struct

import numpy as np
import pytest

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
    assert struct.unpack("<5i", raw[8:28]) == (4, 12, 64, selector.K, selector.DEG_MIN)
    k = selector.K
    off = 28 + 4 * k + 8 * k
    assert struct.unpack("<7d", raw[off:off + 56]) == (
        selector.THETA_REF, selector.COST_FAR, selector.COST_ROW, selector.COST_CLU,
        selector.COST_NEAR, 0.25, 0.25)
    assert len(raw) == off + 56 + 96 + 4 * params.size + 8
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
                   lambda b: b.__setitem__(8, 5)):               # version
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
    path3, _ = _write(tmp_path, costs=(-1.0, 0.5, 2.5, 1.0))     # negative cost weight
    assert _status(path3) == "EMODEL"
    path4, _ = _write(tmp_path, deg_min=13)                      # rule out of range
    assert _status(path4) == "EMODEL"


def _toy(seed, nb=300):
    rng = np.random.default_rng(seed)
    k = selector.K
    n1 = np.array([c[0] + 1 for c in selector.CANDIDATES], float)
    th = np.array([c[1] for c in selector.CANDIDATES])
    # error falls with n and rises with theta; cost rises with n and falls with theta
    Y = (-0.45 * n1[None, :] + 3.0 * th[None, :] - 1.0 + rng.normal(0, 0.3, (nb, 1))
         + rng.normal(0, 0.05, (nb, k))).astype(np.float32)
    cost = (n1[None, :] ** 3 * (1.5 - th[None, :]) * rng.uniform(0.5, 2.0, (nb, 1)))
    wt = rng.uniform(0.1, 10.0, nb)
    return Y, cost, wt


def _budget(Y, wt, ch, tau):
    e2 = 10.0 ** (2.0 * Y.astype(np.float64))
    return (wt * e2[np.arange(Y.shape[0]), ch]).sum() / (wt.sum() * tau * tau)


def test_allocation_extremes():
    Y, cost, wt = _toy(1)
    ch = selector.allocate(Y, cost, wt, 10.0)              # any choice meets it
    assert np.array_equal(ch, cost.argmin(1))
    ch = selector.allocate(Y, cost, wt, 1e-30)             # nothing meets it
    assert np.array_equal(ch, Y.argmin(1))


@pytest.mark.parametrize("tau", [1e-2, 1e-3, 1e-4])
def test_allocation_meets_budget_at_least_cost(tau):
    """The allocation meets the budget, and any single-batch move to a cheaper
    candidate breaks it or costs accuracy the budget does not have: the total
    cost is below that of every uniform choice that meets the budget."""
    Y, cost, wt = _toy(2)
    ch = selector.allocate(Y, cost, wt, tau)
    assert _budget(Y, wt, ch, tau) <= 1.0
    tot = cost[np.arange(cost.shape[0]), ch].sum()
    for j in range(selector.K):
        uni = np.full(cost.shape[0], j)
        if _budget(Y, wt, uni, tau) <= 1.0:
            assert tot <= cost[:, j].sum() * (1 + 1e-12), j
