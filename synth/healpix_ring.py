"""HEALPix pixelisation in RING order, written from the geometry of the scheme.

The paper pixelises its maps with HEALPix (Algorithm section, data model,
and the simulation section's N_side 512 maps) but does not fix the ordering;
this module uses RING order.  Geometry (Gorski et al. 2005):

* ``npix = 12 N^2`` equal-area pixels on ``4N - 1`` iso-latitude rings.
* Polar caps (``|z| > 2/3``): ring ``i = 1..N-1`` counted from the pole holds
  ``4 i`` pixels centred at ``z = +-(1 - i^2 / (3 N^2))`` and
  ``phi = (j - 1/2) * pi / (2 i)``, ``j = 1..4i``.
* Equatorial belt (``|z| <= 2/3``): rings ``i = N..3N`` hold ``4N`` pixels each,
  centred at ``z = 4/3 - 2 i / (3 N)`` and ``phi = (j - 1 + s/2) * pi / (2N)``, ``j = 1..4N``, with
  ``s = (i - N + 1) mod 2`` (rings with ``s = 0`` start at ``phi = 0``).
* Pixels are numbered ring by ring from the north pole, west to east.

Inside the belt the pixel edges are the straight lines ``tt -+ 3 z / 4 =
const`` in the ``(tt = 2 phi / pi, z)`` plane; in the caps they are the curves
``tp * N * sqrt(3 (1 - |z|)) = const`` and ``(1 - tp) * N * sqrt(3 (1 - |z|))
= const``, with ``tp`` the position inside the base-pixel quadrant.  Both maps
below invert exactly those relations.

This module is input synthesis, shared by both sides of every comparison.  It
holds no step of the destriping method.
"""
from __future__ import annotations

import numpy as np


def nside2npix(nside: int) -> int:
    return 12 * int(nside) * int(nside)


def ring_of_pixel_counts(nside: int) -> np.ndarray:
    """Number of pixels on each of the ``4 nside - 1`` rings, north to south."""
    n = int(nside)
    i = np.arange(1, 4 * n)
    north = np.minimum(i, 4 * n - i)
    return np.where(north < n, 4 * north, 4 * n).astype(np.int64)


def ang2pix_ring(nside: int, theta, phi) -> np.ndarray:
    """Pixel index (int64, RING order) containing the direction (theta, phi).

    ``theta`` is the colatitude in [0, pi] and ``phi`` the longitude (any real
    value, taken modulo 2 pi), both in radians, float64 arrays of one shape.
    """
    return ang2pix_ring_z(nside, np.cos(np.asarray(theta, dtype=np.float64)), phi)


def ang2pix_ring_z(nside: int, z, phi) -> np.ndarray:
    """``ang2pix_ring`` from ``z = cos(theta)`` directly."""
    n = int(nside)
    z = np.asarray(z, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    za = np.abs(z)
    twopi = 2.0 * np.pi
    ph = np.mod(phi, twopi)
    # guard: mod can return exactly 2 pi for tiny negative inputs
    ph = np.where(ph >= twopi, 0.0, ph)
    tt = ph / (0.5 * np.pi)  # in [0, 4)

    out = np.empty(z.shape, dtype=np.int64)

    # ---- equatorial belt -------------------------------------------------
    eq = za <= 2.0 / 3.0
    if np.any(eq):
        zt, t = z[eq], tt[eq]
        a = n * (0.5 + t)
        b = 0.75 * n * zt
        jp = np.floor(a - b).astype(np.int64)  # index of the ascending edge line
        jm = np.floor(a + b).astype(np.int64)  # index of the descending edge line
        ir = n + 1 + jp - jm  # ring number counted from z = 2/3, 1..2n+1
        kshift = 1 - (ir & 1)
        ip = (jp + jm - n + kshift + 1) // 2
        ip = np.mod(ip, 4 * n)
        out[eq] = 2 * n * (n - 1) + (ir - 1) * 4 * n + ip

    # ---- polar caps ------------------------------------------------------
    po = ~eq
    if np.any(po):
        zt, t = z[po], tt[po]
        tp = t - np.floor(t)
        tmp = n * np.sqrt(3.0 * (1.0 - np.abs(zt)))
        jp = np.floor(tp * tmp).astype(np.int64)
        jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
        ir = jp + jm + 1  # ring counted from the nearer pole, 1..n
        ip = np.floor(t * ir).astype(np.int64)
        ip = np.mod(ip, 4 * ir)
        north = zt > 0
        out[po] = np.where(north, 2 * ir * (ir - 1) + ip, 12 * n * n - 2 * ir * (ir + 1) + ip)
    return out


def pix2ang_ring(nside: int, pix) -> tuple[np.ndarray, np.ndarray]:
    """Centre (theta, phi) in radians of RING pixels ``pix`` (int array)."""
    n = int(nside)
    p = np.asarray(pix, dtype=np.int64)
    npix = 12 * n * n
    ncap = 2 * n * (n - 1)
    z = np.empty(p.shape, dtype=np.float64)
    phi = np.empty(p.shape, dtype=np.float64)

    north = p < ncap
    south = p >= npix - ncap
    belt = ~(north | south)

    if np.any(north):
        q = p[north]
        # ring i holds pixels 2 i (i-1) .. 2 i (i+1) - 1
        i = np.floor(0.5 * (1.0 + np.sqrt(1.0 + 2.0 * q))).astype(np.int64)
        i = np.where(2 * i * (i - 1) > q, i - 1, i)
        i = np.where(2 * (i + 1) * i <= q, i + 1, i)
        j = q - 2 * i * (i - 1) + 1
        z[north] = 1.0 - (i * i) / (3.0 * n * n)
        phi[north] = (j - 0.5) * np.pi / (2.0 * i)
    if np.any(south):
        q = npix - 1 - p[south]  # mirror index counted from the south pole
        i = np.floor(0.5 * (1.0 + np.sqrt(1.0 + 2.0 * q))).astype(np.int64)
        i = np.where(2 * i * (i - 1) > q, i - 1, i)
        i = np.where(2 * (i + 1) * i <= q, i + 1, i)
        # position inside the ring, west to east
        j = 4 * i - (q - 2 * i * (i - 1))
        z[south] = -(1.0 - (i * i) / (3.0 * n * n))
        phi[south] = (j - 0.5) * np.pi / (2.0 * i)
    if np.any(belt):
        q = p[belt] - ncap
        i = q // (4 * n) + n  # ring number from the north pole, n..3n
        j = q % (4 * n) + 1
        s = (i - n + 1) % 2
        z[belt] = 4.0 / 3.0 - 2.0 * i / (3.0 * n)
        phi[belt] = (j - 1.0 + 0.5 * s) * np.pi / (2.0 * n)
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    return theta, phi
