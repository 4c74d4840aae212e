"""Seeded synthetic sky catalogues for the positional cross-match.

This module only *generates inputs*. It holds none of the matching arithmetic
(no separation test, no zone or cell logic) and is imported by the tests, by
``bench.py`` and by ``__graft_entry__.smoke``; neither ``oracle/`` nor the HIP
library imports it.

The paper's catalogues (its Table 2: SDSS, 2MASS and Gaia extracts) are not
available, so every workload here is synthetic, with the shapes those
catalogues have: area-uniform backgrounds, counterparts displaced by a small
positional error, a dense band like the Galactic plane, tight clumps, and
sources crowding the poles and the RA 0/360 seam.

Conventions
-----------
* All positions are FP64 (ra, dec) in degrees, ra in [0, 360), dec in
  [-90, 90], stored as separate contiguous arrays (structure of arrays).
* ``rng(k, sub)`` is numpy ``Generator(PCG64(SeedSequence([2301073310, k, sub])))``.
* Uniform on the sphere: ra ~ U[0, 360), sin(dec) ~ U[-1, 1).
* Isotropic Gaussian offset of width sigma: tangent-plane components
  xi, eta ~ N(0, sigma^2); the source is moved by rho = hypot(xi, eta) along
  position angle atan2(xi, eta) with the exact spherical "direct" formula.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 2301073310
ARCSEC = 1.0 / 3600.0


def rng(k: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, k, sub])))


# ---------------------------------------------------------------------------
# elementary samplers
# ---------------------------------------------------------------------------

def _wrap_ra(ra: np.ndarray) -> np.ndarray:
    ra = np.mod(ra, 360.0)
    ra[ra >= 360.0] = 0.0  # np.mod can round a tiny negative up to exactly 360
    return ra


def uniform_sphere(g: np.random.Generator, n: int):
    ra = g.uniform(0.0, 360.0, n)
    dec = np.degrees(np.arcsin(g.uniform(-1.0, 1.0, n)))
    return ra, dec


def uniform_patch(g: np.random.Generator, n: int, ra0, ra1, dec0, dec1):
    """Area-uniform in the box ra0..ra1, dec0..dec1 (degrees)."""
    ra = g.uniform(ra0, ra1, n)
    s0, s1 = math.sin(math.radians(dec0)), math.sin(math.radians(dec1))
    dec = np.degrees(np.arcsin(g.uniform(s0, s1, n)))
    return ra, dec


def polar_caps(g: np.random.Generator, n: int, cap_deg: float):
    """Uniform on the two caps |dec| > 90 - cap_deg (hemisphere chosen with p=1/2)."""
    ra = g.uniform(0.0, 360.0, n)
    s = g.uniform(math.cos(math.radians(cap_deg)), 1.0, n)
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    dec = sign * np.degrees(np.arcsin(s))
    return ra, dec


def ra_seam_strip(g: np.random.Generator, n: int, half_width_deg: float):
    """Uniform in sin(dec), ra within +-half_width of the 0/360 seam."""
    x = g.uniform(-half_width_deg, half_width_deg, n)
    ra = _wrap_ra(x)
    dec = np.degrees(np.arcsin(g.uniform(-1.0, 1.0, n)))
    return ra, dec


def direct(ra, dec, rho_deg, pa_rad):
    """Move (ra, dec) by angular distance rho along position angle pa (N through E)."""
    d = np.radians(dec)
    rho = np.radians(rho_deg)
    sd, cd = np.sin(d), np.cos(d)
    sr, cr = np.sin(rho), np.cos(rho)
    s2 = np.clip(sd * cr + cd * sr * np.cos(pa_rad), -1.0, 1.0)
    d2 = np.arcsin(s2)
    dra = np.arctan2(np.sin(pa_rad) * sr * cd, cr - sd * s2)
    return _wrap_ra(ra + np.degrees(dra)), np.degrees(d2)


def gaussian_offset(g: np.random.Generator, ra, dec, sigma_deg: float):
    n = len(ra)
    xi = g.normal(0.0, sigma_deg, n)
    eta = g.normal(0.0, sigma_deg, n)
    return direct(ra, dec, np.hypot(xi, eta), np.arctan2(xi, eta))


def ring_offset(g: np.random.Generator, ra, dec, rho_lo_deg, rho_hi_deg):
    """Offset by rho ~ U[rho_lo, rho_hi] along a uniform position angle."""
    n = len(ra)
    rho = g.uniform(rho_lo_deg, rho_hi_deg, n)
    pa = g.uniform(0.0, 2.0 * math.pi, n)
    return direct(ra, dec, rho, pa)


def cone(g: np.random.Generator, n: int, ra_c: float, dec_c: float, radius_deg: float):
    """Area-uniform inside a cone of the given radius around (ra_c, dec_c)."""
    cr = g.uniform(math.cos(math.radians(radius_deg)), 1.0, n)
    rho = np.degrees(np.arccos(cr))
    pa = g.uniform(0.0, 2.0 * math.pi, n)
    return direct(np.full(n, ra_c), np.full(n, dec_c), rho, pa)


def band_sphere(g: np.random.Generator, n: int, pole_ra=270.0, pole_dec=30.0,
                half_width_deg=10.0, contrast=5.0):
    """Uniform sphere thinned outside a band around a great circle.

    Points within half_width of the great circle whose pole is (pole_ra,
    pole_dec) are always kept; others are kept with probability 1/contrast,
    so the band is `contrast` times denser than the rest of the sky.
    """
    pr, pd = math.radians(pole_ra), math.radians(pole_dec)
    p = np.array([math.cos(pd) * math.cos(pr), math.cos(pd) * math.sin(pr), math.sin(pd)])
    lim = math.sin(math.radians(half_width_deg))
    out_ra, out_dec, have = [], [], 0
    while have < n:
        m = int((n - have) * 2.6) + 1024
        ra, dec = uniform_sphere(g, m)
        r, d = np.radians(ra), np.radians(dec)
        dot = np.cos(d) * np.cos(r) * p[0] + np.cos(d) * np.sin(r) * p[1] + np.sin(d) * p[2]
        keep = (np.abs(dot) <= lim) | (g.random(m) < 1.0 / contrast)
        out_ra.append(ra[keep])
        out_dec.append(dec[keep])
        have += int(keep.sum())
    return np.concatenate(out_ra)[:n], np.concatenate(out_dec)[:n]


def quantize(x: np.ndarray, bits: int = 30) -> np.ndarray:
    """Round to a multiple of 2**-bits degrees (exact RA-shift invariance tests)."""
    q = 2.0 ** bits
    return np.round(x * q) / q


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclass
class Catalogues:
    name: str
    a_ra: np.ndarray
    a_dec: np.ndarray
    b_ra: np.ndarray
    b_dec: np.ndarray
    r_arcsec: float
    meta: dict = field(default_factory=dict)

    @property
    def na(self):
        return len(self.a_ra)

    @property
    def nb(self):
        return len(self.b_ra)


def _shuffle(g, ra, dec):
    p = g.permutation(len(ra))
    return np.ascontiguousarray(ra[p]), np.ascontiguousarray(dec[p])


def _counterparts(g, a_ra, a_dec, n, sigma_deg):
    idx = g.choice(len(a_ra), size=n, replace=False)
    return gaussian_offset(g, a_ra[idx], a_dec[idx], sigma_deg)


def patch_pair(scale: float = 1.0, seed_sub: int = 0) -> Catalogues:
    """Small patch cross-match: 100k x 100k in RA 150-160, Dec 0-10, r = 1 arcsec.

    B is 30% counterparts of distinct A sources (Gaussian sigma = 0.3 arcsec)
    and 70% uniform in the same patch. ``scale`` shrinks both sides (tests).
    """
    g = rng(0, seed_sub)
    na = max(1, int(round(100_000 * scale)))
    nb = na
    a_ra, a_dec = uniform_patch(g, na, 150.0, 160.0, 0.0, 10.0)
    nc = int(round(0.3 * nb))
    c_ra, c_dec = _counterparts(g, a_ra, a_dec, nc, 0.3 * ARCSEC)
    u_ra, u_dec = uniform_patch(g, nb - nc, 150.0, 160.0, 0.0, 10.0)
    b_ra, b_dec = _shuffle(g, np.concatenate([c_ra, u_ra]), np.concatenate([c_dec, u_dec]))
    return Catalogues("patch_100k", a_ra, a_dec, b_ra, b_dec, 1.0,
                      dict(na=na, nb=nb, counterparts=nc, sigma_arcsec=0.3))


def _fullsky_mix(g, n, cap_deg=1.0, strip_arcsec=1.0):
    n_cap = int(round(0.01 * n))
    n_strip = int(round(0.01 * n))
    n_bg = n - n_cap - n_strip
    r1, d1 = band_sphere(g, n_bg)
    r2, d2 = polar_caps(g, n_cap, cap_deg)
    r3, d3 = ra_seam_strip(g, n_strip, strip_arcsec * ARCSEC)
    return np.concatenate([r1, r2, r3]), np.concatenate([d1, d2, d3])


def fullsky_pair(n: int = 10_000_000, seed_sub: int = 0) -> Catalogues:
    """Full-sky 10M x 10M, r = 2 arcsec (the headline workload).

    A: 98% uniform on the sphere thinned to give a 5:1 dense band within 10 deg
    of a great circle tilted 60 deg to the equator (pole at ra 270, dec +30),
    1% in the two 1-deg polar caps, 1% within 1 arcsec of RA 0/360.
    B: 40% counterparts of distinct A sources (sigma = 0.5 arcsec), 60% drawn
    like A. Both sides are shuffled.
    """
    g = rng(1, seed_sub)
    a_ra, a_dec = _shuffle(g, *_fullsky_mix(g, n))
    nc = int(round(0.4 * n))
    c_ra, c_dec = _counterparts(g, a_ra, a_dec, nc, 0.5 * ARCSEC)
    o_ra, o_dec = _fullsky_mix(g, n - nc)
    b_ra, b_dec = _shuffle(g, np.concatenate([c_ra, o_ra]), np.concatenate([c_dec, o_dec]))
    return Catalogues(f"fullsky_{n}", a_ra, a_dec, b_ra, b_dec, 2.0,
                      dict(na=n, nb=n, counterparts=nc, sigma_arcsec=0.5))


def stress_pair(r_arcsec: float, n: int = 20_000_000, n_clumps: int = 10_000,
                seed_sub: int | None = None) -> Catalogues:
    """Precision stress: A = B = n, counterparts at separation U[0.99 r, 1.01 r].

    Each side: 50% in clumps (centres uniform on the sphere and shared by A and
    B; sigma = 30 arcsec), 25% uniform on the sphere, 12.5% with |dec| > 89 deg,
    12.5% within 2 arcsec of RA 0/360. B: n/2 counterparts of distinct A sources
    placed on the ring [0.99 r, 1.01 r], n/2 drawn like A.
    """
    sub = {0.5: 0, 1.0: 1, 5.0: 2}.get(float(r_arcsec), 3) if seed_sub is None else seed_sub
    g = rng(3, sub)
    centres = uniform_sphere(g, n_clumps)

    def side(m):
        n_cl = m // 2
        n_un = m // 4
        n_cap = m // 8
        n_st = m - n_cl - n_un - n_cap
        k = g.integers(0, n_clumps, n_cl)
        cr, cd = gaussian_offset(g, centres[0][k], centres[1][k], 30.0 * ARCSEC)
        ur, ud = uniform_sphere(g, n_un)
        pr, pd = polar_caps(g, n_cap, 1.0)
        sr, sd = ra_seam_strip(g, n_st, 2.0 * ARCSEC)
        return np.concatenate([cr, ur, pr, sr]), np.concatenate([cd, ud, pd, sd])

    a_ra, a_dec = _shuffle(g, *side(n))
    nc = n // 2
    idx = g.choice(n, size=nc, replace=False)
    c_ra, c_dec = ring_offset(g, a_ra[idx], a_dec[idx], 0.99 * r_arcsec * ARCSEC,
                              1.01 * r_arcsec * ARCSEC)
    o_ra, o_dec = side(n - nc)
    b_ra, b_dec = _shuffle(g, np.concatenate([c_ra, o_ra]), np.concatenate([c_dec, o_dec]))
    return Catalogues(f"stress_{n}_r{r_arcsec:g}", a_ra, a_dec, b_ra, b_dec, float(r_arcsec),
                      dict(na=n, nb=n, counterparts=nc))


def large_pair(na: int = 400_000_000, nb: int = 100_000_000, seed_sub: int = 0) -> Catalogues:
    """Large streamed join: A = 400M, B = 100M in the small-patch density model.

    Area-uniform in RA 150-160, Dec 0-10; 20% of B are counterparts of distinct
    A sources at sigma = 0.3 arcsec; r = 1 arcsec.
    """
    g = rng(2, seed_sub)
    a_ra, a_dec = uniform_patch(g, na, 150.0, 160.0, 0.0, 10.0)
    nc = int(round(0.2 * nb))
    c_ra, c_dec = _counterparts(g, a_ra, a_dec, nc, 0.3 * ARCSEC)
    u_ra, u_dec = uniform_patch(g, nb - nc, 150.0, 160.0, 0.0, 10.0)
    b_ra, b_dec = _shuffle(g, np.concatenate([c_ra, u_ra]), np.concatenate([c_dec, u_dec]))
    return Catalogues(f"large_{na}x{nb}", a_ra, a_dec, b_ra, b_dec, 1.0,
                      dict(na=na, nb=nb, counterparts=nc))


@dataclass
class Batch:
    """Many independent jobs packed into four flat arrays.

    Job j owns a_ra[a_off[j]:a_off[j]+na[j]] (likewise for B) and radius r[j].
    """
    a_ra: np.ndarray
    a_dec: np.ndarray
    b_ra: np.ndarray
    b_dec: np.ndarray
    a_off: np.ndarray
    na: np.ndarray
    b_off: np.ndarray
    nb: np.ndarray
    r_arcsec: np.ndarray

    @property
    def njobs(self):
        return len(self.na)


def batch_jobs(njobs: int = 10_000, median: float = 2000.0, sigma_ln: float = 1.0,
               nmin: int = 100, nmax: int = 1_000_000, seed_sub: int = 0) -> Batch:
    """Batched workload: njobs cones with lognormal per-side sizes.

    Per job: sizes nA, nB ~ lognormal(median, sigma_ln) clipped to [nmin, nmax];
    a cone of radius U[0.1, 2] deg centred uniformly on the sphere; A uniform in
    the cone; B = min(round(0.3 nB), nA) counterparts (sigma 0.3 arcsec) plus
    uniform-in-cone sources; r ~ U[0.5, 3] arcsec.
    """
    g = rng(4, seed_sub)
    na = np.clip(np.round(np.exp(g.normal(math.log(median), sigma_ln, njobs))), nmin, nmax).astype(np.int64)
    nb = np.clip(np.round(np.exp(g.normal(math.log(median), sigma_ln, njobs))), nmin, nmax).astype(np.int64)
    radius = g.uniform(0.1, 2.0, njobs)
    cra, cdec = uniform_sphere(g, njobs)
    r = g.uniform(0.5, 3.0, njobs)
    A_ra, A_dec, B_ra, B_dec = [], [], [], []
    for j in range(njobs):
        ar, ad = cone(g, int(na[j]), cra[j], cdec[j], radius[j])
        nc = int(min(round(0.3 * nb[j]), na[j]))
        idx = g.choice(int(na[j]), size=nc, replace=False)
        cr, cd = gaussian_offset(g, ar[idx], ad[idx], 0.3 * ARCSEC)
        ur, ud = cone(g, int(nb[j]) - nc, cra[j], cdec[j], radius[j])
        br, bd = _shuffle(g, np.concatenate([cr, ur]), np.concatenate([cd, ud]))
        A_ra.append(ar); A_dec.append(ad); B_ra.append(br); B_dec.append(bd)
    a_off = np.concatenate([[0], np.cumsum(na)[:-1]]).astype(np.int64)
    b_off = np.concatenate([[0], np.cumsum(nb)[:-1]]).astype(np.int64)
    return Batch(np.concatenate(A_ra), np.concatenate(A_dec), np.concatenate(B_ra),
                 np.concatenate(B_dec), a_off, na, b_off, nb, r)


# ---------------------------------------------------------------------------
# small adversarial sets (brute-force completeness tests)
# ---------------------------------------------------------------------------

def adversarial(kind: str, n: int, seed: int, r_arcsec: float = 2.0):
    """Tiny inputs aimed at the places a spatial index can lose pairs.

    kinds: 'random' (whole sphere), 'pole' (within 3 r of a pole), 'seam'
    (within 3 r of RA 0/360, in a Dec strip 30 r high), 'grid' (positions on a coarse lattice of
    multiples of r/2, so many sit exactly on cell and zone edges), 'dup'
    (heavy duplication), 'same' (all points identical), 'dense' (one tight
    clump a few r across).
    Returns (a_ra, a_dec, b_ra, b_dec).
    """
    g = rng(100, seed)
    r = r_arcsec * ARCSEC
    seam_dec0 = float(g.uniform(-60.0, 60.0))
    grid_ra0, grid_dec0 = float(g.uniform(0, 360)), float(g.uniform(-80, 80))

    def one(m):
        if kind == "random":
            return uniform_sphere(g, m)
        if kind == "pole":
            ra = g.uniform(0.0, 360.0, m)
            s = g.choice([-1.0, 1.0], m)
            return ra, s * (90.0 - g.uniform(0.0, 3.0 * r, m))
        if kind == "seam":
            d0 = seam_dec0
            return _wrap_ra(g.uniform(-3.0 * r, 3.0 * r, m)), g.uniform(d0, d0 + 30.0 * r, m)
        if kind == "grid":
            base_ra, base_dec = grid_ra0, grid_dec0
            ra = _wrap_ra(base_ra + 0.5 * r * g.integers(-8, 9, m))
            dec = base_dec + 0.5 * r * g.integers(-8, 9, m)
            return ra, dec
        if kind == "dup":
            ra, dec = uniform_patch(g, max(1, m // 10), 10.0, 10.0 + 20 * r, 5.0, 5.0 + 20 * r)
            k = g.integers(0, len(ra), m)
            return ra[k], dec[k]
        if kind == "same":
            return np.full(m, 123.456), np.full(m, -33.3)
        if kind == "dense":
            return gaussian_offset(g, np.full(m, 359.9999), np.full(m, 45.0), r)
        raise ValueError(kind)

    a = one(n)
    b = one(n)
    return (np.ascontiguousarray(a[0], dtype=np.float64), np.ascontiguousarray(a[1], dtype=np.float64),
            np.ascontiguousarray(b[0], dtype=np.float64), np.ascontiguousarray(b[1], dtype=np.float64))
