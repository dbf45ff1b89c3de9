"""Pins of the oracle's regularized Stokes kernels (Section 7).

Checked against facts the formulas must satisfy rather than the formulas
themselves: values at r = 0, the classical singular Stokes kernels as
eps -> 0 with their leading correction factors, the derivative relations
Q = H2 - H1'/r, D1 = 2Q + r Q', D2 = -Q'/r (the rotlet is half the vorticity
of the Stokeslet, and the angular velocity of a rotlet half its vorticity),
incompressibility of the Stokeslet field, symmetry of the mobility matrices
and rotation covariance.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_values_at_zero(orc):
    rows = {}
    with open(os.path.join(GOLDEN, "mrs_at_zero.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, c, p = line.split()
            rows[name] = (float(c), int(p))
    for eps in (0.3, 0.01, 0.002):
        got = orc.mrs_functions(0.0, eps)
        for i, name in enumerate(["H1", "H2", "Q", "D1", "D2"]):
            c, p = rows[name]
            assert got[i] == pytest.approx(c / (np.pi * eps ** p), rel=1e-14)


def _fd(f, r, h):
    return (f(r + h) - f(r - h)) / (2 * h)


@pytest.mark.parametrize("eps", [0.005, 0.05, 0.3])
@pytest.mark.parametrize("r", [0.001, 0.02, 0.3, 2.0])
def test_derivative_relations(orc, eps, r):
    H1 = lambda x: orc.mrs_functions(x * x, eps)[0]
    H2 = orc.mrs_functions(r * r, eps)[1]
    Qf = lambda x: orc.mrs_functions(x * x, eps)[2]
    Q, D1, D2 = orc.mrs_functions(r * r, eps)[2:]
    h = 1e-4 * min(r, eps)
    dH1 = _fd(H1, r, h)
    dQ = _fd(Qf, r, h)
    assert Q == pytest.approx(H2 - dH1 / r, rel=1e-7)
    assert D2 == pytest.approx(-dQ / r, rel=1e-7)
    assert D1 == pytest.approx(2 * Q + r * dQ, rel=1e-6, abs=1e-7 * abs(2 * Q))


def _curl(field, x, h):
    J = np.zeros((3, 3))       # J[a, b] = d field_a / d x_b
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        J[:, b] = (field(x + e) - field(x - e)) / (2 * h)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]]), np.trace(J)


@pytest.mark.parametrize("seed", range(4))
def test_rotlet_is_half_vorticity(orc, seed):
    rng = np.random.default_rng(seed)
    eps = [0.01, 0.1, 0.5, 0.05][seed]
    y = rng.uniform(-1, 1, 3)
    x = y + rng.uniform(-0.3, 0.3, 3)
    g = rng.uniform(-1, 1, 3)
    stok = lambda p: orc.pair("stokeslet", p, y, g, eps=eps)
    rot = lambda p: orc.pair("rotlet", p, y, g, eps=eps)
    h = 1e-5 * max(eps, np.linalg.norm(x - y))
    curl_s, div_s = _curl(stok, x, h)
    u_rot = rot(x)
    scale = np.linalg.norm(u_rot) + np.linalg.norm(curl_s)
    # velocity of a torque = half the vorticity of a force of the same vector
    assert np.max(np.abs(u_rot[:3] - 0.5 * curl_s)) < 1e-7 * scale
    # the regularized Stokeslet field is divergence free
    assert abs(div_s) < 1e-7 * np.linalg.norm(stok(x)) / np.linalg.norm(x - y)
    # angular velocity of a torque = half the vorticity of its velocity
    curl_r, div_r = _curl(lambda p: rot(p)[:3], x, h)
    assert np.max(np.abs(u_rot[3:] - 0.5 * curl_r)) < 1e-7 * (np.linalg.norm(u_rot[3:]) + np.linalg.norm(curl_r))
    assert abs(div_r) < 1e-7 * np.linalg.norm(u_rot[:3]) / np.linalg.norm(x - y)


@pytest.mark.parametrize("r", [0.1, 0.5, 2.0])
def test_eps_to_zero_limit(orc, r):
    """As eps -> 0 the kernels tend to the singular Stokes kernels, with
    H1 ~ (1 + eps^2/(2 r^2)) and H2 ~ (1 - 3 eps^2/(2 r^2)) times their limits."""
    rng = np.random.default_rng(int(r * 10))
    d = rng.normal(size=3)
    d *= r / np.linalg.norm(d)
    y = rng.uniform(-1, 1, 3)
    x = y + d
    g = rng.uniform(-1, 1, 3)
    stokes = (g / r + np.dot(g, d) * d / r ** 3) / (8 * np.pi)
    rotlet_u = np.cross(g, d) / (8 * np.pi * r ** 3)
    rotlet_w = (-g / r ** 3 + 3 * np.dot(g, d) * d / r ** 5) / (16 * np.pi)
    prev = None
    for eps in (1e-2 * r, 1e-3 * r, 1e-4 * r):
        su = orc.pair("stokeslet", x, y, g, eps=eps)
        ro = orc.pair("rotlet", x, y, g, eps=eps)
        err = max(np.linalg.norm(su - stokes) / np.linalg.norm(stokes),
                  np.linalg.norm(ro[:3] - rotlet_u) / np.linalg.norm(rotlet_u),
                  np.linalg.norm(ro[3:] - rotlet_w) / np.linalg.norm(rotlet_w))
        assert err < 10 * (eps / r) ** 2
        if prev is not None:
            assert err < prev / 50
        prev = err
        H1, H2 = orc.mrs_functions(r * r, eps)[:2]
        assert H1 * 8 * np.pi * r == pytest.approx(1 + eps ** 2 / (2 * r ** 2), abs=5 * (eps / r) ** 4)
        assert H2 * 8 * np.pi * r ** 3 == pytest.approx(1 - 1.5 * eps ** 2 / r ** 2, abs=5 * (eps / r) ** 4)
    # eps = 0 exactly reproduces the singular kernels
    assert np.allclose(orc.pair("stokeslet", x, y, g, eps=0.0), stokes, rtol=1e-14, atol=0)


def _mobility(orc, kernel, pts, eps, rows):
    n = pts.shape[1]
    M = np.zeros((rows * n, 3 * n))
    for j in range(n):
        for b in range(3):
            g = np.zeros(3)
            g[b] = 1.0
            for i in range(n):
                M[rows * i:rows * i + rows, 3 * j + b] = orc.pair(kernel, pts[:, i], pts[:, j], g, eps=eps)
    return M


def test_mobility_symmetry(orc):
    rng = np.random.default_rng(7)
    pts = rng.uniform(-1, 1, (3, 9))
    eps = 0.05
    Ms = _mobility(orc, "stokeslet", pts, eps, 3)
    assert np.max(np.abs(Ms - Ms.T)) < 1e-13 * np.max(np.abs(Ms))
    Mr = _mobility(orc, "rotlet", pts, eps, 6)
    n = pts.shape[1]
    Mu = Mr.reshape(n, 6, 3 * n)[:, :3, :].reshape(3 * n, 3 * n)
    Mw = Mr.reshape(n, 6, 3 * n)[:, 3:, :].reshape(3 * n, 3 * n)
    assert np.max(np.abs(Mu - Mu.T)) < 1e-13 * np.max(np.abs(Mu))
    assert np.max(np.abs(Mw - Mw.T)) < 1e-13 * np.max(np.abs(Mw))
    # the Stokeslet mobility is positive definite for this regularization
    assert np.min(np.linalg.eigvalsh(0.5 * (Ms + Ms.T))) > 0


def test_rotation_covariance(orc):
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    R, _ = np.linalg.qr(A)
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    for _ in range(5):
        x, y, g = rng.uniform(-1, 1, (3, 3))
        for kern in ("stokeslet", "rotlet"):
            a = orc.pair(kern, R @ x, R @ y, R @ g, eps=0.07)
            b = orc.pair(kern, x, y, g, eps=0.07)
            assert np.allclose(a[:3], R @ b[:3], rtol=1e-12, atol=1e-12 * np.abs(b).max())
            if kern == "rotlet":
                assert np.allclose(a[3:], R @ b[3:], rtol=1e-12, atol=1e-12 * np.abs(b).max())


def test_poly_kernel_integer_values(orc):
    x = np.array([1.0, -2.0, 3.0])
    y = np.array([2.0, 1.0, -1.0])
    g = np.array([1.0, 2.0, -3.0])
    out = orc.pair("poly", x, y, g, poly_p=3, poly_c=2.0)
    v = (2 + (1 * 2 - 2 * 1 - 3 * 1)) ** 3
    assert np.array_equal(out, v * g)
