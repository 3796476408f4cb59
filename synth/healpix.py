"""HEALPix RING-scheme pixelisation used only to *generate* synthetic pointing.

Written from the HEALPix definition (Gorski et al. 2005, ApJ 622, 759): the
sphere is split into 12*nside^2 equal-area pixels laid out on 4*nside-1 iso-
latitude rings; the two polar caps (|z| > 2/3) hold rings of 4*i pixels, the
equatorial belt rings of 4*nside pixels, alternately shifted by half a pixel.
RING numbering runs along each ring from phi = 0, rings from north to south.

The paper pre-computes one HEALPix pixel per sample (section 4.1), so the
decoded pixel stream is the only pointing the hot path ever sees; this module
is preprocessing, never part of the GPU path.
"""
import numpy as np

HALFPI = 0.5 * np.pi
TWOTHIRD = 2.0 / 3.0


def npix_of(nside):
    return 12 * int(nside) * int(nside)


def ang2pix_ring(nside, theta, phi):
    """Pixel index (RING) of points at colatitude theta, longitude phi (radians)."""
    nside = int(nside)
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    z = np.cos(theta)
    za = np.abs(z)
    tt = np.mod(phi, 2.0 * np.pi) / HALFPI          # in [0, 4)
    tt = np.where(tt >= 4.0, 0.0, tt)
    ncap = 2 * nside * (nside - 1)
    npix = 12 * nside * nside
    out = np.empty(z.shape, dtype=np.int64)

    eq = za <= TWOTHIRD
    if np.any(eq):
        zq, tq = z[eq], tt[eq]
        t1 = nside * (0.5 + tq)
        t2 = nside * zq * 0.75
        jp = np.floor(t1 - t2).astype(np.int64)      # ascending edge line
        jm = np.floor(t1 + t2).astype(np.int64)      # descending edge line
        ir = nside + 1 + jp - jm                     # ring in {1..2nside+1}
        kshift = 1 - (ir & 1)
        ip = (jp + jm - nside + kshift + 1) // 2
        ip = np.mod(ip, 4 * nside)
        out[eq] = ncap + (ir - 1) * 4 * nside + ip

    po = ~eq
    if np.any(po):
        zp, tp_full = z[po], tt[po]
        tp = tp_full - np.floor(tp_full)
        tmp = nside * np.sqrt(3.0 * (1.0 - np.abs(zp)))
        jp = np.floor(tp * tmp).astype(np.int64)
        jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
        ir = jp + jm + 1                             # ring counted from the pole
        ip = np.floor(tp_full * ir).astype(np.int64)
        ip = np.mod(ip, 4 * ir)
        north = zp > 0
        out[po] = np.where(north, 2 * ir * (ir - 1) + ip,
                           npix - 2 * ir * (ir + 1) + ip)
    return out


def pix2ang_ring(nside, pix):
    """Centre (theta, phi) of RING pixels; inverse of ang2pix_ring on centres."""
    nside = int(nside)
    pix = np.asarray(pix, dtype=np.int64)
    ncap = 2 * nside * (nside - 1)
    npix = 12 * nside * nside
    theta = np.empty(pix.shape)
    phi = np.empty(pix.shape)

    north = pix < ncap
    if np.any(north):
        p = pix[north]
        ir = ((1 + np.floor(np.sqrt(1 + 2 * p)).astype(np.int64)) >> 1)
        # guard against rounding of sqrt
        ir = np.where(2 * ir * (ir - 1) > p, ir - 1, ir)
        ir = np.where(2 * (ir + 1) * ir <= p, ir + 1, ir)
        ip = p - 2 * ir * (ir - 1)
        z = 1.0 - ir * ir / (3.0 * nside * nside)
        theta[north] = np.arccos(z)
        phi[north] = (ip + 0.5) * HALFPI / ir

    south = pix >= npix - ncap
    if np.any(south):
        p = npix - pix[south]                        # 1..ncap
        ir = ((1 + np.floor(np.sqrt(2 * p - 1)).astype(np.int64)) >> 1)
        ir = np.where(2 * ir * (ir - 1) >= p, ir - 1, ir)
        ir = np.where(2 * (ir + 1) * ir < p, ir + 1, ir)
        ip = 4 * ir + 1 - (p - 2 * ir * (ir - 1))    # 1..4ir
        z = -(1.0 - ir * ir / (3.0 * nside * nside))
        theta[south] = np.arccos(z)
        phi[south] = (ip - 0.5) * HALFPI / ir

    eq = ~(north | south)
    if np.any(eq):
        p = pix[eq] - ncap
        iring = p // (4 * nside) + nside             # ring number from north pole
        iphi = p % (4 * nside) + 1
        fodd = np.where(((iring + nside) & 1) == 1, 1.0, 0.5)
        z = (2 * nside - iring) * 2.0 / (3.0 * nside)
        theta[eq] = np.arccos(z)
        phi[eq] = (iphi - fodd) * HALFPI / nside
    return theta, phi


def ring_of_pix(nside, pix):
    """Ring number (1..4nside-1, north to south) of RING pixels."""
    th, _ = pix2ang_ring(nside, pix)
    z = np.cos(th)
    nside = int(nside)
    out = np.empty(np.shape(pix), dtype=np.int64)
    za = np.abs(z)
    cap = za > TWOTHIRD
    irc = np.rint(nside * np.sqrt(3.0 * (1.0 - za))).astype(np.int64)
    ire = np.rint(nside * (2.0 - 1.5 * z)).astype(np.int64)
    out = np.where(cap, np.where(z > 0, irc, 4 * nside - irc), ire)
    return out
