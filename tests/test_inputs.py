"""The seeded input generators: SplitMix64 against its published reference
outputs, counter independence, and the shape of every workload."""
import numpy as np

from paper_1902_02250_amd import inputs


def test_splitmix64_reference_outputs():
    """SplitMix64 with state 0: the first outputs of the reference
    generator (state += golden gamma, then the two xor-shift-multiply
    rounds) are 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F."""
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    with np.errstate(over="ignore"):
        ctr = np.arange(1, 4, dtype=np.uint64)
        got = inputs._mix(ctr * inputs._GAMMA)
    assert [int(v) for v in got] == want


def test_counter_independence():
    a = inputs.uniform01(7, 3, 0, 100)
    b = inputs.uniform01(7, 3, 40, 20)
    assert np.array_equal(a[40:60], b)
    assert np.all((a >= 0) & (a < 1))


def test_pairs_workload():
    """Section 8.1: bodies in a cube of side 10, flagella 0.02 away, unit
    forces in opposite directions along the organism."""
    p, w, cfg = inputs.workload("e1", n=2001)
    assert p.shape == (3, 2001) and w.shape == (3, 2001)
    body, flag = p[:, 0:2000:2], p[:, 1:2000:2]
    assert np.allclose(np.linalg.norm(flag - body, axis=0), 0.02, rtol=1e-12)
    assert np.all((body >= 0) & (body <= 10))
    assert np.allclose(np.linalg.norm(w, axis=0), 1.0, rtol=1e-12)
    assert np.array_equal(w[:, 0:2000:2], -w[:, 1:2000:2])
    d = (flag - body) / 0.02
    assert np.allclose(d, w[:, 0:2000:2], atol=1e-12)
    # directions cover the sphere evenly: mean near 0, second moments near 1/3
    assert np.abs(d.mean(axis=1)).max() < 0.1
    assert np.allclose((d * d).mean(axis=1), 1 / 3, atol=0.05)
    p2, w2, _ = inputs.workload("e1", n=2001)
    assert np.array_equal(p, p2) and np.array_equal(w, w2)


def test_distributions_in_cube():
    for dist in ("uniform", "mixture", "union"):
        p = inputs.points(dist, 5000, 3)
        assert p.shape == (3, 5000)
        assert np.all((p >= -1) & (p <= 1))


def test_rods_workload():
    """Section 8.2: N = N_r (M + 1) particles on helices of radius 0.3 about
    base points of a square grid, 0 <= z <= 9; 15 x 15 rods fill [-8, 8]^2
    and 80 x 80 rods give N = 966400; a force and a torque per particle."""
    per = inputs.ROD_SEGMENTS + 1
    p = inputs.rods(225 * per)
    assert p.shape == (3, 33975)
    rod = p.reshape(3, 225, per)
    z = rod[2]
    assert np.all(z[:, 0] == 0.0) and np.all(z[:, -1] == 9.0)
    assert np.allclose(np.diff(z, axis=1), 9.0 / 150, rtol=1e-12)
    base = rod[:2, :, 0] - np.array([[0.3], [0.0]])          # z = 0: cos 0 = 1, sin 0 = 0
    assert np.allclose(np.hypot(rod[0] - base[0][:, None], rod[1] - base[1][:, None]), 0.3)
    # angle advances by 2 dz along the rod
    ang = np.unwrap(np.arctan2(rod[1] - base[1][:, None], rod[0] - base[0][:, None]), axis=1)
    assert np.allclose(ang, 2.0 * z, atol=1e-12)
    xs, ys = np.unique(np.round(base[0], 12)), np.unique(np.round(base[1], 12))
    assert xs.size == ys.size == 15
    assert np.allclose(np.diff(xs), 16 / 15) and np.isclose(xs[0] - 8 / 15, -8.0)
    assert np.isclose(xs[-1] + 8 / 15, 8.0)
    pe, we, cfg = inputs.workload("e2")
    assert pe.shape == (3, 966400) and we.shape == (6, 966400) and cfg["kernel"] == "full"
    assert np.all(np.abs(we) <= 1.0) and cfg["eps"] == 0.3
    xe = np.unique(np.round(pe[0].reshape(-1, per)[:, 0] - 0.3, 9))
    assert xe.size == 80 and np.isclose(xe[0] - 8 / 15, -80 * 8 / 15)
    # a ragged count cuts the last rod
    assert inputs.rods(1000).shape == (3, 1000)
    assert np.array_equal(inputs.rods(1000), inputs.rods(7 * per)[:, :1000])
