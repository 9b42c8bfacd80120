"""HEALPix RING-scheme geometry in plain numpy (FP64).

The paper builds its maps on HEALPix (Sect. 3, first paragraphs; it cites
Gorski et al. 2005 for the scheme) and uses the RING ordering for disc
queries (Sect. 3.2). This module restates the published RING construction:

* 12 N^2 equal-area pixels on 4N-1 iso-latitude rings;
* north polar cap, rings i = 1..N-1: 4i pixels, z = 1 - i^2/(3N^2),
  azimuths (j + 1/2) * pi / (2i);
* equatorial belt, rings i = N..3N: 4N pixels, z = 4/3 - 2i/(3N),
  azimuths (j + 1/2) * pi/(2N) when i - N is even, j * pi/(2N) otherwise;
* south cap mirrors the north one.

Pins (tests/test_oracle_healpix.py): ring counts sum to 12 N^2; the NSIDE-1
and NSIDE-2 centres the construction fixes by hand; point->pixel of every
pixel centre returns that pixel; uniform random points fill pixels equally
(chi-square); points are assigned to the pixel whose boundary contains them
(checked against a brute-force point-in-cell test built from the boundary
curves); disc membership equals a brute-force scan.
"""
from __future__ import annotations

import math

import numpy as np


def check_nside(nside: int) -> None:
    if nside < 1 or (nside & (nside - 1)) != 0 or nside > (1 << 14):
        raise ValueError(f"NSIDE must be a power of two <= 16384, got {nside}")


def npix(nside: int) -> int:
    return 12 * nside * nside


def ring_table(nside: int):
    """Arrays over rings i = 1..4N-1 (index i-1): z, one_minus_absz, sin_theta,
    pixels per ring, first pixel, azimuth offset in units of the pixel step."""
    N = nside
    rows = []
    for i in range(1, 4 * N):
        if i < N:
            n = 4 * i
            first = 2 * i * (i - 1)
            omz = i * i / (3.0 * N * N)
            z = 1.0 - omz
            off = 0.5
        elif i <= 3 * N:
            n = 4 * N
            first = 2 * N * (N - 1) + 4 * N * (i - N)
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * N)
            omz = 1.0 - abs(z)
            off = 0.5 if (i - N) % 2 == 0 else 0.0
        else:
            k = 4 * N - i
            n = 4 * k
            first = 12 * N * N - 2 * k * (k + 1)
            omz = k * k / (3.0 * N * N)
            z = -(1.0 - omz)
            off = 0.5
        sin_t = math.sqrt(omz * (2.0 - omz))
        rows.append((z, omz, sin_t, n, first, off))
    a = np.array(rows, dtype=np.float64)
    return {
        "z": a[:, 0],
        "omz": a[:, 1],
        "sin": a[:, 2],
        "n": a[:, 3].astype(np.int64),
        "first": a[:, 4].astype(np.int64),
        "off": a[:, 5],
    }


def pix2ring(nside: int, pix):
    """(ring i in 1..4N-1, index j within the ring) for RING pixel numbers."""
    N = nside
    p = np.asarray(pix, dtype=np.int64)
    if np.any(p < 0) or np.any(p >= npix(N)):
        raise ValueError("pixel out of range")
    ncap = 2 * N * (N - 1)
    ring = np.empty_like(p)
    j = np.empty_like(p)
    north = p < ncap
    south = p >= npix(N) - ncap
    belt = ~(north | south)
    if north.any():
        pn = p[north]
        i = ((1 + np.sqrt(1.0 + 2.0 * pn)) // 2).astype(np.int64)
        # integer correction: ring i holds [2i(i-1), 2i(i+1))
        i = np.where(2 * i * (i - 1) > pn, i - 1, i)
        i = np.where(2 * i * (i + 1) <= pn, i + 1, i)
        ring[north] = i
        j[north] = pn - 2 * i * (i - 1)
    if belt.any():
        pb = p[belt] - ncap
        ring[belt] = pb // (4 * N) + N
        j[belt] = pb % (4 * N)
    if south.any():
        q = npix(N) - p[south]  # 1 .. ncap
        k = ((1 + np.sqrt(2.0 * q - 1.0)) // 2).astype(np.int64)
        # ring k (from the south pole) holds q in (2k(k-1), 2k(k+1)]
        k = np.where(2 * k * (k - 1) >= q, k - 1, k)
        k = np.where(2 * k * (k + 1) < q, k + 1, k)
        ring[south] = 4 * N - k
        j[south] = p[south] - (npix(N) - 2 * k * (k + 1))
    return ring, j


def pix2zphi(nside: int, pix):
    """(z, sin_theta, phi) of pixel centres."""
    rt = ring_table(nside)
    ring, j = pix2ring(nside, pix)
    r = ring - 1
    phi = (j + rt["off"][r]) * (2.0 * math.pi / rt["n"][r])
    return rt["z"][r], rt["sin"][r], phi


def pix2vec(nside: int, pix):
    z, s, phi = pix2zphi(nside, pix)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=-1)


def pix2radec(nside: int, pix):
    z, s, phi = pix2zphi(nside, pix)
    return phi, np.arctan2(z, s)


def radec2pix(nside: int, ra, dec):
    """RING pixel containing each point (ra, dec in radians).

    Follows the published point->pixel construction: in the belt the pixel
    boundaries are the lines phi/(pi/2) +- (3/4) z * ... of slope +-1 in the
    (phi, z) plane; in the caps they are the curves of constant
    (phi mod pi/2) * sqrt(3 (1-|z|)) etc.
    """
    N = nside
    ra = np.asarray(ra, dtype=np.float64)
    dec = np.asarray(dec, dtype=np.float64)
    z = np.sin(dec)
    za = np.abs(z)
    # 1 - |z| computed without cancellation near the poles
    omz = 2.0 * np.sin(0.5 * (0.5 * math.pi - np.abs(dec))) ** 2
    tt = np.mod(ra, 2 * math.pi) / (0.5 * math.pi)
    tt = np.where(tt >= 4.0, 0.0, tt)
    out = np.empty(ra.shape, dtype=np.int64)

    belt = za <= 2.0 / 3.0
    if belt.any():
        t = tt[belt]
        zb = z[belt]
        a = N * (0.5 + t)
        b = N * zb * 0.75
        jp = np.floor(a - b).astype(np.int64)   # ascending edge index
        jm = np.floor(a + b).astype(np.int64)   # descending edge index
        ir = N + 1 + jp - jm                    # ring counted from z = 2/3: 1..2N+1
        kshift = 1 - (ir & 1)
        ip = (jp + jm - N + kshift + 1) // 2
        ip = np.mod(ip, 4 * N)
        out[belt] = 2 * N * (N - 1) + (ir - 1) * 4 * N + ip
    cap = ~belt
    if cap.any():
        t = tt[cap]
        tp = t - np.floor(t)
        tmp = N * np.sqrt(3.0 * omz[cap])
        jp = np.floor(tp * tmp).astype(np.int64)
        jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
        ir = jp + jm + 1                        # ring counted from the nearest pole
        ip = np.floor(t * ir).astype(np.int64)
        ip = np.mod(ip, 4 * ir)
        north = z[cap] > 0
        out[cap] = np.where(north, 2 * ir * (ir - 1) + ip, npix(N) - 2 * ir * (ir + 1) + ip)
    return out


def disc_brute(nside: int, vec, radius: float):
    """All pixels whose centre is strictly within ``radius`` (great-circle) of
    the unit vector ``vec``, by scanning every pixel (small NSIDE only)."""
    v = pix2vec(nside, np.arange(npix(nside)))
    d = v - np.asarray(vec)[None, :]
    c2 = (d * d).sum(1)
    return np.nonzero(c2 < 4.0 * math.sin(0.5 * radius) ** 2)[0]


# ---------------------------------------------------------------------------
# Face coordinates and pixel neighbours (for the detection step, Sect. 6.1)
# ---------------------------------------------------------------------------
#
# The 12 base pixels (faces) of the construction are curvilinear squares,
# each cut into N x N cells. Face f gets continuous coordinates (alpha,
# beta) in [0, N)^2, (0, 0) at its northern corner, alpha growing to the
# south-east and beta to the south-west; cell (floor alpha, floor beta) is
# one pixel. In the belt these are the two edge-line coordinates of the
# point->pixel construction, Jp = N (1/2 + tt - 3z/4) and
# Jm = N (1/2 + tt + 3z/4) (tt = 2 phi / pi), shifted per face; in the caps
# they are tp * t and (1 - tp) * t (t = N sqrt(3 (1 - |z|)), tp = tt mod 1),
# measured from the pole for the north faces and turned round for the south
# ones. Both forms agree on |z| = 2/3.

def face_coords(nside: int, z, tt, omz):
    """(face, alpha, beta) of points given by z, tt = 2 phi / pi in [0, 4)
    and omz = 1 - |z|."""
    N = float(nside)
    z = np.asarray(z, np.float64)
    tt = np.asarray(tt, np.float64)
    omz = np.asarray(omz, np.float64)
    face = np.empty(z.shape, np.int64)
    al = np.empty(z.shape)
    be = np.empty(z.shape)
    belt = np.abs(z) <= 2.0 / 3.0
    jp = N * (0.5 + tt - 0.75 * z)
    jm = N * (0.5 + tt + 0.75 * z)
    ifp = np.floor(jp / N).astype(np.int64)
    ifm = np.floor(jm / N).astype(np.int64)
    fb = np.where(ifp == ifm, 4 + ifp % 4, np.where(ifp < ifm, ifp % 4, 8 + ifm % 4))
    face[belt] = fb[belt]
    al[belt] = (jp - ifp * N)[belt]
    be[belt] = ((ifm + 1) * N - jm)[belt]
    t = N * np.sqrt(3.0 * omz)
    fl = np.floor(tt)
    tp = tt - fl
    north = ~belt & (z > 0)
    south = ~belt & (z < 0)
    face[north] = fl[north].astype(np.int64)
    al[north] = (tp * t)[north]
    be[north] = ((1.0 - tp) * t)[north]
    face[south] = 8 + fl[south].astype(np.int64)
    al[south] = (N - (1.0 - tp) * t)[south]
    be[south] = (N - tp * t)[south]
    return face, al, be


def face_point(nside: int, face, al, be):
    """Inverse of face_coords, continued a little beyond the face: (z, omz,
    phi) of face coordinates (alpha, beta)."""
    N = float(nside)
    face = np.asarray(face, np.int64)
    al = np.asarray(al, np.float64)
    be = np.asarray(be, np.float64)
    g = face % 4
    row = face // 4  # 0 north, 1 equatorial, 2 south
    # belt form (every face, where it applies): Jp, Jm of the point
    off_p = np.where(row == 0, g, np.where(row == 1, g, g + 1)) * N
    off_m = np.where(row == 0, g + 2, np.where(row == 1, g + 1, g + 1)) * N
    jp = al + off_p
    jm = off_m - be
    zb = (jm - jp) / (1.5 * N)
    ttb = (jp + jm) / (2.0 * N) - 0.5
    z = zb.copy()
    tt = ttb.copy()
    omz = 1.0 - np.abs(zb)
    s_n = al + be            # north faces: distance from the pole in cells
    s_s = 2.0 * N - al - be  # south faces: from the south pole
    capn = (row == 0) & (s_n < N)
    caps = (row == 2) & (s_s < N)
    if capn.any():
        s = s_n[capn]
        tt[capn] = g[capn] + np.divide(al[capn], s, out=np.zeros_like(s), where=s > 0)  # the pole: any azimuth
        omz[capn] = s * s / (3.0 * N * N)
        z[capn] = 1.0 - omz[capn]
    if caps.any():
        s = s_s[caps]
        tt[caps] = g[caps] + np.divide(N - be[caps], s, out=np.zeros_like(s), where=s > 0)
        omz[caps] = s * s / (3.0 * N * N)
        z[caps] = -(1.0 - omz[caps])
    return z, omz, np.mod(tt, 4.0) * (0.5 * math.pi)


def pix2face(nside: int, pix):
    """(face, cell alpha index, cell beta index) of RING pixels."""
    z, s, phi = pix2zphi(nside, pix)
    rt = ring_table(nside)
    ring, _ = pix2ring(nside, pix)
    f, al, be = face_coords(nside, z, np.mod(phi / (0.5 * math.pi), 4.0), rt["omz"][ring - 1])
    return f, np.floor(al).astype(np.int64), np.floor(be).astype(np.int64)


def _point_pix(nside, z, omz, phi):
    dec = np.where(z >= 0, 0.5 * math.pi - 2.0 * np.arcsin(np.sqrt(0.5 * omz)),
                   -(0.5 * math.pi - 2.0 * np.arcsin(np.sqrt(0.5 * omz))))
    return radec2pix(nside, phi, dec)


# edge probes: just across the middle of the cell's four edges, in the order
# alpha-, beta-, alpha+, beta+ (consecutive edges meet at a vertex)
_EDGE_PROBE = [(-1e-6, 0.5), (0.5, -1e-6), (1.0 + 1e-6, 0.5), (0.5, 1.0 + 1e-6)]


def edge_neighbours(nside: int, pix):
    """[n, 4] pixels across the four edges of each pixel (every edge of the
    grid is shared by exactly two pixels)."""
    f, ia, ib = pix2face(nside, pix)
    out = []
    for da, db in _EDGE_PROBE:
        z, omz, phi = face_point(nside, f, ia + da, ib + db)
        out.append(_point_pix(nside, z, omz, phi))
    return np.stack(out, axis=1)


def neighbours(nside: int, pix):
    """[n, 8] neighbours of each pixel: the four across its edges, then the
    one diagonally across each vertex (between edges k and k+1), -1 where
    the vertex is shared by only three pixels (the corners where three faces
    meet). The pixel across a vertex is the common edge neighbour, other
    than the pixel itself, of the two pixels across the vertex's edges;
    when those two share an edge, the vertex has three pixels and there is
    none."""
    pix = np.asarray(pix, np.int64)
    e = edge_neighbours(nside, pix)
    ee = edge_neighbours(nside, e.ravel()).reshape(pix.size, 4, 4)
    out = np.full((pix.size, 8), -1, np.int64)
    out[:, :4] = e
    for k in range(4):
        a, b = k, (k + 1) % 4
        A, B = ee[:, a, :], ee[:, b, :]
        three = np.any(A == e[:, b:b + 1], axis=1)  # the two share an edge: three pixels at this vertex
        match = (A[:, :, None] == B[:, None, :]).any(axis=2) & (A != pix[:, None])
        n_common = np.array([np.unique(A[i][match[i]]).size for i in range(pix.size)])
        bad = ~three & (n_common != 1)
        if bad.any():
            raise RuntimeError(f"vertex neighbour not unique for pixels {pix[bad][:5]}")
        first = np.argmax(match, axis=1)
        out[:, 4 + k] = np.where(three, -1, A[np.arange(pix.size), first])
    return out
