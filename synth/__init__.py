"""Seeded synthetic particle snapshots (input generators only).

This module draws the particle sets that both the HIP path and the CPU
oracle consume.  It holds none of the level-of-detail method: it only
places points in the unit cube and assigns masses.  Every generator is
numpy ``Generator(PCG64(seed))`` in float64, cast to float32 at the end.

The paper's own data (the Aquarius dark-matter runs, 150 million particles
per snapshot) are not available; these clustered sets stand in for them:

* ``plummer_mix``    -- Plummer spheres plus a uniform background
* ``nfw_mix``        -- NFW haloes with power-law masses plus a background
* ``soneira_peebles``-- hierarchical Soneira-Peebles clustering
* ``uniform``        -- uniform in the unit cube

Common finishing rules (``finish``): positions are wrapped periodically into
[0, 1), a coordinate that rounds to 1.0f is replaced by 1 - 2**-24, the
particle order is shuffled with a permutation drawn from seed + 1 (so ids
carry no spatial order), and masses are float32 1/N.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Snapshot", "finish", "uniform", "plummer_mix", "nfw_mix", "soneira_peebles",
    "config1", "config2", "config3", "config5_sizes", "config5_snapshot",
    "small_clustered", "Attributes", "evolve",
]

_ONE_MINUS = np.float32(1.0 - 2.0 ** -24)


@dataclass
class Snapshot:
    x: np.ndarray  # float32 [N]
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray  # float32 [N]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, count: int) -> "Snapshot":
        return Snapshot(self.x[:count].copy(), self.y[:count].copy(),
                        self.z[:count].copy(), self.m[:count].copy())


def _wrap32(a: np.ndarray) -> np.ndarray:
    a = a - np.floor(a)
    f = a.astype(np.float32)
    f[f >= np.float32(1.0)] = _ONE_MINUS
    f[f < np.float32(0.0)] = np.float32(0.0)
    return f


def finish(pos: np.ndarray, seed: int, shuffle: bool = True) -> Snapshot:
    """Wrap float64 positions [N,3] into the unit cube, shuffle, set masses."""
    n = pos.shape[0]
    x = _wrap32(pos[:, 0])
    y = _wrap32(pos[:, 1])
    z = _wrap32(pos[:, 2])
    if shuffle and n > 1:
        perm = np.random.Generator(np.random.PCG64(seed + 1)).permutation(n)
        x, y, z = x[perm], y[perm], z[perm]
    m = np.full(n, np.float32(1.0 / n) if n else np.float32(0.0), dtype=np.float32)
    return Snapshot(np.ascontiguousarray(x), np.ascontiguousarray(y),
                    np.ascontiguousarray(z), m)


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    nrm = np.sqrt((v * v).sum(axis=1))
    nrm[nrm == 0.0] = 1.0
    return v / nrm[:, None]


def uniform(n: int, seed: int, shuffle: bool = True) -> Snapshot:
    rng = np.random.Generator(np.random.PCG64(seed))
    return finish(rng.random((n, 3)), seed, shuffle)


def plummer_mix(n: int, seed: int, n_spheres: int = 20, frac: float = 0.7,
                a_range=(0.01, 0.05), shuffle: bool = True) -> Snapshot:
    """Plummer spheres (r = a / sqrt(u^(-2/3) - 1)) plus a uniform remainder."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = int(round(n * frac / n_spheres)) if n_spheres else 0
    n_cl = per * n_spheres
    n_bg = n - n_cl
    a = rng.uniform(a_range[0], a_range[1], n_spheres)
    centres = rng.random((n_spheres, 3))
    u = rng.random(n_cl)
    u = np.clip(u, 1e-300, 1.0 - 1e-16)
    sc = np.repeat(np.arange(n_spheres), per)
    r = a[sc] / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    cl = centres[sc] + r[:, None] * _unit_vectors(rng, n_cl)
    bg = rng.random((n_bg, 3))
    return finish(np.concatenate([cl, bg]), seed, shuffle)


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    q = weights / weights.sum() * total
    base = np.floor(q).astype(np.int64)
    short = total - int(base.sum())
    if short > 0:
        order = np.argsort(-(q - base), kind="stable")
        base[order[:short]] += 1
    return base


def nfw_mix(n: int, seed: int, n_halos: int = 500, bg_frac: float = 0.2,
            slope: float = -1.9, mass_range: float = 1e3, rvir_max: float = 0.05,
            c_range=(5.0, 15.0), shuffle: bool = True) -> Snapshot:
    """NFW haloes truncated at the virial radius plus a uniform background.

    Halo masses follow dN/dM ~ M^slope on [Mmax/mass_range, Mmax]; particle
    counts are proportional to mass (largest remainder); R_vir scales as
    M^(1/3); the radius is drawn from the closed-form inverse of the NFW
    enclosed-mass profile, x = -1 - 1/W0(-exp(-1 - mu(c) u)).
    """
    from scipy.special import lambertw

    rng = np.random.Generator(np.random.PCG64(seed))
    n_bg = int(round(n * bg_frac))
    n_cl = n - n_bg
    g = slope + 1.0
    lo, hi = 1.0 / mass_range, 1.0
    u = rng.random(n_halos)
    mh = (lo ** g + u * (hi ** g - lo ** g)) ** (1.0 / g)
    counts = _largest_remainder(mh, n_cl)
    rvir = rvir_max * (mh / mh.max()) ** (1.0 / 3.0)
    conc = rng.uniform(c_range[0], c_range[1], n_halos)
    centres = rng.random((n_halos, 3))
    hid = np.repeat(np.arange(n_halos), counts)
    c = conc[hid]
    mu_c = np.log1p(c) - c / (1.0 + c)
    uu = rng.random(n_cl)
    w0 = lambertw(-np.exp(-1.0 - mu_c * uu), 0).real
    xs = -1.0 - 1.0 / w0
    r = np.minimum(xs, c) * (rvir[hid] / c)
    cl = centres[hid] + r[:, None] * _unit_vectors(rng, n_cl)
    bg = rng.random((n_bg, 3))
    return finish(np.concatenate([cl, bg]), seed, shuffle)


def soneira_peebles(n: int, seed: int, levels: int = 8, eta: int = 4,
                    lam: float = 1.9, shuffle: bool = True) -> Snapshot:
    """Soneira-Peebles hierarchical clustering.

    ceil(n / eta^levels) top spheres with uniform centres and radius R0 chosen
    so that the top spheres fill the box once, R0 = (3 / (4 pi n_top))^(1/3).
    Each sphere places eta child centres uniformly inside its ball; children
    have radius / lam.  The level-`levels` centres are emitted; the first n
    are kept.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    per_top = eta ** levels
    n_top = max(1, -(-n // per_top))
    r0 = (3.0 / (4.0 * math.pi * n_top)) ** (1.0 / 3.0)
    pos = rng.random((n_top, 3))
    radius = r0
    for _ in range(levels):
        parents = np.repeat(pos, eta, axis=0)
        k = parents.shape[0]
        rr = radius * np.cbrt(rng.random(k))
        pos = parents + rr[:, None] * _unit_vectors(rng, k)
        del parents
        radius = radius / lam
    return finish(pos[:n], seed, shuffle)


def small_clustered(n: int, seed: int) -> Snapshot:
    """A small Plummer mix used by quick tests (5 spheres, 60% clustered)."""
    return plummer_mix(n, seed, n_spheres=5, frac=0.6)


# --- the five benchmark configurations ------------------------------------

def config1() -> Snapshot:
    """262,144 particles, seed 0: 20 Plummer spheres (70%) + 30% uniform."""
    return plummer_mix(262144, 0, n_spheres=20, frac=183500 / 262144)


def config2() -> Snapshot:
    """16,777,216 particles, seed 2: 500 NFW haloes + 20% uniform."""
    return nfw_mix(16777216, 2)


def config3(count: int = 150_000_000) -> Snapshot:
    """150M particles, seed 3: Soneira-Peebles, 8 levels, eta 4, lambda 1.9."""
    return soneira_peebles(count, 3)


def config5_sizes(n_snap: int = 128, lo: float = 5e5, hi: float = 8e6) -> np.ndarray:
    """Snapshot sizes, log-uniform on [lo, hi], drawn from seed 5."""
    rng = np.random.Generator(np.random.PCG64(5))
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_snap))).astype(np.int64)


def config5_snapshot(s: int, size: int) -> Snapshot:
    return soneira_peebles(int(size), 5000 + s)


# --- a second, ID-matched snapshot (time interpolation) -----------------------

@dataclass
class Attributes:
    """Per-particle world radius h and colour value c of one snapshot."""
    h: np.ndarray   # float32 [N]
    c: np.ndarray   # float32 [N], in [0, 1]


def evolve(s: Snapshot, seed: int, step: float = 0.01, modes: int = 6, h0: float = 0.002):
    """The next snapshot of the same particles (same ids, same masses):
    positions moved by a smooth random flow, displacement
    step * sum_k a_k sin(2 pi k.x + phi_k) per axis (unit wave vectors k with
    integer components up to 3, amplitudes a_k ~ N(0, 1/modes)), plus
    isotropic noise of 0.05 step; clipped into [0, 1 - 2^-24].  Also per-particle
    world radii (h0 (1 + U) at A, times 1 + 0.4 (U' - 1/2) at B) and colours
    (speed of the flow at each position, scaled to [0, 1]).
    Returns (snapshot B, attributes A, attributes B)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = rng.integers(-3, 4, (modes, 3)).astype(np.float64)
    ks[np.all(ks == 0, axis=1)] = (1.0, 0.0, 0.0)
    amp = rng.standard_normal((modes, 3)) / math.sqrt(modes)
    ph = rng.random(modes) * 2 * math.pi

    def flow(x, y, z):
        v = np.zeros((x.shape[0], 3))
        for k in range(modes):
            arg = 2 * math.pi * (ks[k, 0] * x + ks[k, 1] * y + ks[k, 2] * z) + ph[k]
            v += np.sin(arg)[:, None] * amp[k][None, :]
        return v

    xa, ya, za = (a.astype(np.float64) for a in (s.x, s.y, s.z))
    va = flow(xa, ya, za)
    d = step * va + 0.05 * step * rng.standard_normal((s.n, 3))
    hi = 1.0 - 2.0 ** -24
    nb = [np.clip(a + d[:, i], 0.0, hi).astype(np.float32) for i, a in enumerate((xa, ya, za))]
    vb = flow(*(b.astype(np.float64) for b in nb))
    sa = np.sqrt((va * va).sum(axis=1)); sb = np.sqrt((vb * vb).sum(axis=1))
    top = max(float(sa.max(initial=0.0)), float(sb.max(initial=0.0)), 1e-30)
    ha = (h0 * (1.0 + rng.random(s.n))).astype(np.float32)
    hb = (ha.astype(np.float64) * (1.0 + 0.4 * (rng.random(s.n) - 0.5))).astype(np.float32)
    B = Snapshot(nb[0], nb[1], nb[2], s.m.copy())
    return B, Attributes(ha, (sa / top).astype(np.float32)), Attributes(hb, (sb / top).astype(np.float32))
