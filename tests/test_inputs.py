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
