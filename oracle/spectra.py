"""Structure factor and lamellar orientation of a 2D order-parameter field (numpy, FP64).

TEST INFRASTRUCTURE (part of the oracle).  The paper judges lamellar order by eye from snapshots
(Section 3: lamellae parallel or perpendicular to the thermal fronts); these two observables make
that judgement quantitative.

Structure factor.  phi_hat = DFT of (phi - mean phi) over the whole lattice (the wall axis is
wrapped as well, so the transform is the plain periodic DFT).  Each mode k = 2 pi (m_x/n_x,
m_y/n_y) with signed integer m falls in shell b = floor(|k| / dk), dk = 2 pi / min(n_x, n_y); the
shell index is computed exactly in integers: b = isqrt(floor((m_x^2 n_y^2 + m_y^2 n_x^2) /
max(n_x, n_y)^2)).  S[b] is the mean of |phi_hat|^2 / N over the modes of shell b (k = 0 left
out; 0 for an empty shell).  The peak is refined by the vertex of the parabola through the
largest shell and its two neighbours, shell centres at (b + 1/2) dk.  <k> is the |phi_hat|^2
weighted mean of |k| over all modes k != 0.

Orientation.  Gradients by central differences (periodic in x; even reflection at the walls, so
the normal derivative on a wall layer is half the difference to the next layer; periodic in y if
there are no walls).  Each site adds its weight |grad phi|^2 to the bin of its gradient angle
theta = atan2(g_y, g_x) mod pi in nbins equal bins of [0, pi).  Q = sum (g_y^2 - g_x^2) / sum
|grad phi|^2: +1 when every gradient is normal to the walls (lamellae parallel to the walls), -1
when lamellae are perpendicular to them.  Q_row is the same ratio per row y.
"""
from __future__ import annotations

import math

import numpy as np


def shell_index(nx: int, ny: int) -> np.ndarray:
    """Exact integer shell index of every DFT mode, shape (ny, nx), numpy FFT ordering."""
    mx = np.fft.fftfreq(nx, 1.0 / nx).round().astype(np.int64)
    my = np.fft.fftfreq(ny, 1.0 / ny).round().astype(np.int64)
    num = (mx[None, :] ** 2) * (ny * ny) + (my[:, None] ** 2) * (nx * nx)
    den = max(nx, ny) ** 2
    q = num // den
    b = np.floor(np.sqrt(q.astype(np.float64))).astype(np.int64)
    # exact integer square root: correct the float estimate by at most one either way
    b = np.where(b * b > q, b - 1, b)
    b = np.where((b + 1) * (b + 1) <= q, b + 1, b)
    return b


def structure_factor(phi: np.ndarray, nbins: int) -> dict:
    phi = np.asarray(phi, dtype=np.float64)
    assert phi.ndim == 2
    ny, nx = phi.shape
    N = nx * ny
    ph = np.fft.fft2(phi - phi.mean())
    power = (ph.real ** 2 + ph.imag ** 2) / N
    b = shell_index(nx, ny)
    zero = np.zeros_like(b, dtype=bool)
    zero[0, 0] = True
    S = np.zeros(nbins)
    cnt = np.zeros(nbins, np.int64)
    sel = (~zero) & (b < nbins)
    np.add.at(S, b[sel], power[sel])
    np.add.at(cnt, b[sel], 1)
    S = np.where(cnt > 0, S / np.maximum(cnt, 1), 0.0)
    dk = 2.0 * math.pi / min(nx, ny)
    kx = 2.0 * math.pi * np.fft.fftfreq(nx)
    ky = 2.0 * math.pi * np.fft.fftfreq(ny)
    kmag = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    tot = power[~zero].sum()
    k_mean = float((kmag[~zero] * power[~zero]).sum() / tot) if tot > 0 else 0.0
    m = int(np.argmax(S))
    k_peak, S_peak = (m + 0.5) * dk, float(S[m])
    if 0 < m < nbins - 1:
        den = S[m - 1] - 2.0 * S[m] + S[m + 1]
        if den != 0.0:
            d = 0.5 * (S[m - 1] - S[m + 1]) / den
            k_peak = (m + 0.5 + d) * dk
            S_peak = float(S[m] - 0.25 * (S[m - 1] - S[m + 1]) * d)
    return dict(S=S, counts=cnt, k_peak=float(k_peak), S_peak=S_peak, k_mean=k_mean, dk=dk,
                peak_bin=m)


def gradients(phi: np.ndarray, walls: bool):
    phi = np.asarray(phi, dtype=np.float64)
    gx = 0.5 * (np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1))
    if walls:
        ext = np.concatenate([phi[:1], phi, phi[-1:]], axis=0)  # even reflection
        gy = 0.5 * (ext[2:] - ext[:-2])
    else:
        gy = 0.5 * (np.roll(phi, -1, axis=0) - np.roll(phi, 1, axis=0))
    return gx, gy


def gradients3(phi: np.ndarray, walls: bool):
    """Central differences of a 3D field [z][y][x]: x and y periodic, z reflected evenly across
    the wall planes (or periodic)."""
    phi = np.asarray(phi, dtype=np.float64)
    gx = 0.5 * (np.roll(phi, -1, axis=2) - np.roll(phi, 1, axis=2))
    gy = 0.5 * (np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1))
    if walls:
        ext = np.concatenate([phi[:1], phi, phi[-1:]], axis=0)
        gz = 0.5 * (ext[2:] - ext[:-2])
    else:
        gz = 0.5 * (np.roll(phi, -1, axis=0) - np.roll(phi, 1, axis=0))
    return gx, gy, gz


def orientation3(phi: np.ndarray, nbins: int, walls: bool = True) -> dict:
    """Orientation of grad phi in 3D relative to the wall normal z: theta = arccos(|g_z| / |g|) in
    [0, pi/2], histogram of nbins equal bins weighted by |g|^2 (fractions of the total);
    Q = sum(g_z^2 - (g_x^2 + g_y^2)/2) / sum |g|^2, the weighted second Legendre polynomial of
    cos theta: +1 for lamellae parallel to the walls, -1/2 perpendicular, 0 isotropic; Q per layer
    along z."""
    gx, gy, gz = gradients3(phi, walls)
    w = gx * gx + gy * gy + gz * gz
    num = gz * gz - 0.5 * (gx * gx + gy * gy)
    c = np.where(w > 0, np.abs(gz) / np.sqrt(np.where(w > 0, w, 1.0)), 1.0)
    theta = np.arccos(np.clip(c, 0.0, 1.0))
    b = np.minimum((theta / (0.5 * math.pi / nbins)).astype(np.int64), nbins - 1)
    hist = np.zeros(nbins)
    np.add.at(hist, b.ravel(), w.ravel())
    tot = w.sum()
    Q = float(num.sum() / tot) if tot > 0 else 0.0
    lw = w.sum(axis=(1, 2))
    Qrow = np.where(lw > 0, num.sum(axis=(1, 2)) / np.where(lw > 0, lw, 1.0), 0.0)
    return dict(hist=hist / tot if tot > 0 else hist, Q=Q, Q_row=Qrow, theta=theta, weight=w,
                total_weight=float(tot))


def orientation(phi: np.ndarray, nbins: int, walls: bool = True) -> dict:
    if np.ndim(phi) == 3:
        return orientation3(phi, nbins, walls)
    gx, gy = gradients(phi, walls)
    w = gx * gx + gy * gy
    theta = np.mod(np.arctan2(gy, gx), math.pi)
    b = np.minimum((theta / (math.pi / nbins)).astype(np.int64), nbins - 1)
    hist = np.zeros(nbins)
    np.add.at(hist, b.ravel(), w.ravel())
    tot = w.sum()
    Q = float((gy * gy - gx * gx).sum() / tot) if tot > 0 else 0.0
    rw = w.sum(axis=1)
    Qrow = np.where(rw > 0, (gy * gy - gx * gx).sum(axis=1) / np.where(rw > 0, rw, 1.0), 0.0)
    return dict(hist=hist / tot if tot > 0 else hist, Q=Q, Q_row=Qrow, theta=theta, weight=w,
                total_weight=float(tot))
