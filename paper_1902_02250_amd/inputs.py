"""Seeded synthetic particle sets (no treecode arithmetic lives here).

One counter-based generator serves every workload: SplitMix64 (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
evaluated at counters 1, 2, 3, ... of a stream, so any draw can be produced
independently of the others.  A 64-bit output z becomes the double
(z >> 11) * 2**-53 in [0, 1).  Normals use Box-Muller on pairs of draws.

Workloads (particle positions are (3, n) float64, weights (3, n) float64):
  uniform   - i.i.d. uniform points in [-1, 1]^3
  mixture   - a 32-component isotropic Gaussian mixture in [-1, 1]^3: means
              uniform in the cube, standard deviations uniform in
              [0.01, 0.2], mixture weights Dirichlet(1) (normalised Exp(1)
              draws); a point falling outside the cube is drawn again
  union     - half uniform, half mixture, concatenated and then shuffled by
              a seeded permutation
  pairs     - the microorganism pairs of the paper's first example (Section
              8.1): bodies uniform in a cube of side 10, each with a
              flagellum particle at distance 0.02 along a direction uniform on
              the sphere; the two exert unit forces in opposite directions
              along that direction (body +u, flagellum -u)
  rods      - the helical rods of the paper's second example (Section 8.2):
              rods of M = 150 segments (151 particles) at
              (x0 + 0.3 cos 2z, y0 + 0.3 sin 2z, z), z = 9 m / M, with base
              points (x0, y0) at the centers of a square grid of spacing
              16/15 centred on the origin (15 x 15 rods fill [-8, 8]^2), the
              grid widening with the rod count at constant density; weights
              are a force and a torque per particle (6 rows)
Weights (forces or torques) are i.i.d. uniform in [-1, 1] per component and
come from their own stream of the same seed, except for `pairs`, whose forces
follow from the orientations.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream identifiers, so positions, weights, etc. never share counters
S_POS, S_WEIGHT, S_MIX_PARAM, S_MIX_POINT, S_SHUFFLE, S_SAMPLE, S_PAIR = range(7)


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed, stream, start, count):
    """count uniform doubles in [0, 1) from counters start+1 .. start+count of
    (seed, stream)."""
    with np.errstate(over="ignore"):
        key = _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ _mix(np.uint64(stream + 1) * _GAMMA))
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = _mix(key + ctr * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_points(n, seed, lo=-1.0, hi=1.0):
    u = uniform01(seed, S_POS, 0, 3 * n).reshape(n, 3).T
    return np.ascontiguousarray(lo + (hi - lo) * u)


def weights(n, seed, wdim=3):
    u = uniform01(seed, S_WEIGHT, 0, wdim * n).reshape(n, wdim).T
    return np.ascontiguousarray(-1.0 + 2.0 * u)


def shape_args(cfg):
    """Keyword arguments of points() / weights_for() that a config sets."""
    return {"pair_length": cfg["pair_length"]} if "pair_length" in cfg else {}


def weights_for(dist, n, seed, pair_length=0.02):
    """The weights of a workload: the pair forces for `pairs`, a force and a
    torque per particle for `rods`, else weights()."""
    if dist == "pairs":
        return _pairs(n, seed, length=pair_length)[1]
    if dist == "rods":
        return weights(n, seed, 6)
    return weights(n, seed)


def mixture_params(seed, ncomp=32):
    """Means (ncomp, 3), standard deviations (ncomp,), weights (ncomp,)."""
    u = uniform01(seed, S_MIX_PARAM, 0, 5 * ncomp).reshape(ncomp, 5)
    means = -1.0 + 2.0 * u[:, 0:3]
    sigma = 0.01 + (0.2 - 0.01) * u[:, 3]
    e = -np.log1p(-u[:, 4])                   # Exp(1)
    return means, sigma, e / e.sum()


def mixture_points(n, seed, ncomp=32):
    means, sigma, wts = mixture_params(seed, ncomp)
    cdf = np.cumsum(wts)
    cdf[-1] = 1.0
    out = np.empty((n, 3))
    todo = np.arange(n)
    rnd = 0
    while todo.size:
        # round rnd draws attempt rnd for every still-missing point i from
        # counters that depend only on (i, rnd)
        base = (rnd * n + todo).astype(np.int64)
        rows = _draw_rows(seed, base, 4)
        comp = np.searchsorted(cdf, rows[:, 0], side="right")
        comp = np.minimum(comp, ncomp - 1)
        g = _box_muller_rows(rows[:, 1:4], seed, base)
        p = means[comp] + sigma[comp, None] * g
        inside = np.all((p >= -1.0) & (p <= 1.0), axis=1)
        out[todo[inside]] = p[inside]
        todo = todo[~inside]
        rnd += 1
    return np.ascontiguousarray(out.T)


def _draw_rows(seed, base, width):
    """Row r holds the draws base[r]*width+1 .. base[r]*width+width."""
    with np.errstate(over="ignore"):
        key = _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ _mix(np.uint64(S_MIX_POINT + 1) * _GAMMA))
        ctr = (base.astype(np.uint64)[:, None] * np.uint64(width)
               + np.arange(1, width + 1, dtype=np.uint64)[None, :])
        z = _mix(key + ctr * _GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _box_muller_rows(u3, seed, base):
    """Three normals per row: two from (u0, u1) and one from (u2, extra)."""
    extra = _draw_rows(seed + 0x5EED, base, 1)[:, 0]
    r01 = np.sqrt(-2.0 * np.log1p(-u3[:, 0]))
    a01 = 2.0 * np.pi * u3[:, 1]
    r2 = np.sqrt(-2.0 * np.log1p(-u3[:, 2]))
    a2 = 2.0 * np.pi * extra
    return np.stack([r01 * np.cos(a01), r01 * np.sin(a01), r2 * np.cos(a2)], axis=1)


def shuffle_perm(n, seed):
    keys = uniform01(seed, S_SHUFFLE, 0, n)
    return np.argsort(keys, kind="stable")


def union_points(n, seed):
    a = uniform_points(n // 2, seed)
    b = mixture_points(n - n // 2, seed)
    p = np.concatenate([a, b], axis=1)
    return np.ascontiguousarray(p[:, shuffle_perm(n, seed)])


def _pairs(n, seed, side=10.0, length=0.02):
    """Positions and forces of n particles as body-flagellum pairs (a last
    unpaired body when n is odd)."""
    m = (n + 1) // 2
    body = side * uniform01(seed, S_POS, 0, 3 * m).reshape(m, 3)
    u = uniform01(seed, S_PAIR, 0, 2 * m).reshape(m, 2)
    z = 2.0 * u[:, 0] - 1.0
    phi = 2.0 * np.pi * u[:, 1]
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)
    pos = np.empty((2 * m, 3))
    pos[0::2] = body
    pos[1::2] = body + length * d
    frc = np.empty((2 * m, 3))
    frc[0::2] = d
    frc[1::2] = -d
    return np.ascontiguousarray(pos[:n].T), np.ascontiguousarray(frc[:n].T)


ROD_SEGMENTS = 150
ROD_SPACING = 16.0 / 15.0


def rods(n, segments=ROD_SEGMENTS, spacing=ROD_SPACING, height=9.0, radius=0.3):
    """Particles of ceil(n / (segments + 1)) helical rods, rod after rod, cut
    to n.  The rods take the first places, row by row, of the smallest square
    grid that holds them; no draw is random."""
    per = segments + 1
    nr = -(-n // per)
    side = int(np.ceil(np.sqrt(nr))) if nr else 0
    while side * side < nr:
        side += 1
    r = np.arange(nr)
    c = (np.arange(side) - 0.5 * (side - 1)) * spacing
    x0, y0 = c[r % side], c[r // side]
    z = height * np.arange(per) / segments
    px = x0[:, None] + radius * np.cos(2.0 * z)[None, :]
    py = y0[:, None] + radius * np.sin(2.0 * z)[None, :]
    pz = np.broadcast_to(z[None, :], px.shape)
    pts = np.stack([px.ravel(), py.ravel(), pz.ravel()])[:, :n]
    return np.ascontiguousarray(pts)


def points(dist, n, seed, pair_length=0.02):
    if dist == "pairs":
        return _pairs(n, seed, length=pair_length)[0]
    if dist == "rods":
        return rods(n)
    if dist == "uniform":
        return uniform_points(n, seed)
    if dist == "mixture":
        return mixture_points(n, seed)
    if dist == "union":
        return union_points(n, seed)
    raise ValueError(f"unknown distribution {dist!r}")


def sample_indices(m, k, seed):
    """k distinct target indices out of m (seeded), sorted."""
    if k >= m:
        return np.arange(m, dtype=np.int64)
    keys = uniform01(seed, S_SAMPLE, 0, m)
    return np.sort(np.argsort(keys, kind="stable")[:k]).astype(np.int64)


SEED_BASE = 1902022500

# The five workloads: positions, kernel, eps and treecode parameters.
CONFIGS = {
    "c1": dict(n=8000, dist="uniform", kernel="stokeslet", eps=0.01, degree=4,
               theta=0.7, leaf=500, seed=SEED_BASE + 1),
    "c2": dict(n=100000, dist="uniform", kernel="stokeslet", eps=0.01,
               degree=6, theta=0.7, leaf=2000, seed=SEED_BASE + 2,
               degrees=(2, 4, 6, 8, 10), thetas=(0.5, 0.7, 0.9)),
    "c3": dict(n=1000000, dist="uniform", kernel="stokeslet", eps=0.005,
               degree=8, theta=0.7, leaf=2000, seed=SEED_BASE + 3,
               error_sample=10000),
    "c4": dict(n=1000000, dist="mixture", kernel="rotlet", eps=0.01, degree=6,
               theta=0.7, leaf=2000, seed=SEED_BASE + 4, error_sample=10000),
    "c5": dict(n=4000000, dist="union", kernel="stokeslet", eps=0.002,
               degree=10, theta=0.6, leaf=2000, seed=SEED_BASE + 5,
               error_sample=10000, tol=1e-6),
    # the paper's first example at its 640K size (Section 8.1, Tables 1 and 4)
    "e1": dict(n=640000, dist="pairs", kernel="stokeslet", eps=0.02, degree=7,
               theta=0.7, leaf=2000, seed=SEED_BASE + 11, error_sample=10000),
    # the paper's second example with 80 x 80 rods (Section 8.2, Table 5):
    # Stokeslets and rotlets together, eps = 5 L / M = 0.3
    "e2": dict(n=966400, dist="rods", kernel="full", eps=0.3, degree=7,
               theta=0.7, leaf=1000, seed=SEED_BASE + 12, error_sample=10000),
}


def workload(name, n=None):
    """(points (3, n), weights (3, n), config dict) for a named workload; n
    overrides the size (same recipe, smaller set)."""
    cfg = dict(CONFIGS[name])
    if n is not None:
        cfg["n"] = n
    pts = points(cfg["dist"], cfg["n"], cfg["seed"], **shape_args(cfg))
    w = weights_for(cfg["dist"], cfg["n"], cfg["seed"], **shape_args(cfg))
    return pts, w, cfg
