"""Error scales of the chi^2 and its adjoint for the GPU parity tests (a test
helper, not a test module): sums of the magnitudes of the summed terms and
bounds of the transforms' rounding in the Whittle terms, computed with the
oracle's functions."""
import numpy as np

from oracle import tod as ot


def magnitudes(ts, m_r, nc_r, eps):
    """Per segment: error scales of J, dJ/dg, dJ/dsigma0, dJ/df_knee,
    dJ/dalpha (sums of the terms' magnitudes, times tol in the test) and the
    transform-error bounds of their Whittle parts (absolute); per pixel: the
    sum of the map gradient's terms' magnitudes."""
    gp = ot.global_pix(ts, ts.pix)
    out = np.zeros((5, ts.nseg))
    fft = np.zeros((5, ts.nseg))
    gmag = np.zeros((3, ts.npix_total))
    for q in range(ts.nseg):
        a, b = ts.seg_off[q], ts.seg_off[q + 1]
        p, cc, ss = ot.pointing_rows(gp[a:b], ts.psi[a:b])
        Pm = m_r[0, p] + m_r[1, p] * cc + m_r[2, p] * ss
        r = ts.d[a:b] - ts.gain[q] * Pm - nc_r[a:b]
        s0, fk, al = ts.sigma0[q], ts.fknee[q], ts.alpha[q]
        I, P, f = ot.whittle_parts(nc_r[a:b], ts.band_fsamp[ts.seg_band[q]], s0, fk, al)
        u = np.abs(1.0 - I / P) + I / P + 1.0
        N = ot.fft_length(b - a)
        e = ot.extend(nc_r[a:b], N)
        delta = 4.0 * eps * np.log2(N) * np.sqrt(np.mean(e * e))
        dIP = (2.0 * np.sqrt(I) * delta + delta ** 2) / P
        fft[0, q] = np.sum(dIP)
        fft[2, q] = 2.0 / s0 * np.sum(dIP)
        fft[3, q] = abs(al / fk) * np.sum(dIP)
        fft[4, q] = np.sum(dIP * np.abs(np.log(f / fk)))
        out[0, q] = np.sum(r * r) / s0 ** 2 + np.sum(I / P) + np.sum(np.abs(np.log(P)))
        out[1, q] = 2.0 * np.sum(np.abs(Pm * r)) / s0 ** 2
        out[2, q] = 2.0 * np.sum(r * r) / s0 ** 3 + 2.0 / s0 * np.sum(u)
        out[3, q] = abs(al / fk) * np.sum(u)
        out[4, q] = np.sum(u * np.abs(np.log(f / fk)))
        w = np.abs(2.0 * ts.gain[q] * r / s0 ** 2)
        np.add.at(gmag[0], p, w)
        np.add.at(gmag[1], p, w * np.abs(cc))
        np.add.at(gmag[2], p, w * np.abs(ss))
    return out, fft, gmag
